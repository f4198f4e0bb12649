"""The algorithmic VALU counts behind the roofline fractions (bench.alg_valu_per_event)
against the event loops the compiler actually emits: the kernels are compiled
for gfx950 to assembly here (no GPU needed) and the VALU instructions of each
kernel's event loop (the longest path from the header of an innermost loop
whose body holds the LDS histogram atomics back to it) are counted. Each loop may issue at most a few instructions more
than the count (loop and scheduling overhead), and never fewer."""
import os
import re
import subprocess

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2010_09341_amd", "csrc")


def _event_loops(asm: str):
    """{kernel symbol: VALU instructions of its event loop}."""
    out = {}
    for m in re.finditer(r"^(_ZN5vegas9k_iterate\S+):[^\n]*\n(.*?)^\.Lfunc_end", asm, re.S | re.M):
        name, body = m.group(1), m.group(2).split("\n")
        labels = {}
        for i, line in enumerate(body):
            lm = re.match(r"^(\.LBB\S+):", line)
            if lm:
                labels[lm.group(1)] = i
        latches = []  # (label line, branch line) of every backward branch
        for i, line in enumerate(body):
            bm = re.match(r"\s+s_c?branch\w*\s+(\.LBB\S+)", line)
            if bm and bm.group(1) in labels and labels[bm.group(1)] < i:
                latches.append((labels[bm.group(1)], i))
        best = None
        for lo, hi in latches:
            # innermost loops only: no loop with another header lies inside
            # [lo, hi] (a second latch back to the same header is another
            # path through the same loop: the RAMBO phase-space-only mode)
            if any(lo <= a and b <= hi and a != lo for a, b in latches):
                continue
            ins = [x.split()[0] for x in body[lo:hi + 1] if x.strip() and
                   not x.strip().startswith((";", ".")) and not x.strip().endswith(":")]
            if any(x.startswith("ds_add") for x in ins):
                valu = sum(1 for x in ins if x.startswith("v_"))
                if best is None or valu > best:
                    best = valu
        out[name] = best
    return out


@pytest.fixture(scope="module")
def loops(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("asm") / "count_kernels.s")
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-munsafe-fp-atomics",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "--cuda-device-only", "-S",
           os.path.join(ROOT, "tests", "helpers", "count_kernels.hip"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return _event_loops(open(out).read())


# (template arguments in the mangled name, dim, precision, integrand id)
CASES = [("ILi8ELi2ELi1ELb0", 8, 1, 2), ("ILi8ELi2ELi0ELb0", 8, 0, 2),
         ("ILi4ELi3ELi1ELb0", 4, 1, 3), ("ILi16ELi4ELi1ELb0", 16, 1, 4)]


@pytest.mark.parametrize("key,dim,prec,fid", CASES, ids=["gauss8d_fp32", "gauss8d_fp64", "lo_toy_fp32",
                                                         "rambo24_fp32"])
def test_event_loop_matches_count(loops, key, dim, prec, fid):
    issued = [v for k, v in loops.items() if key in k]
    assert len(issued) == 1 and issued[0] is not None, loops
    counted = bench.alg_valu_per_event(dim, prec, fid)
    assert counted <= issued[0] <= counted + 6, (issued[0], counted)
