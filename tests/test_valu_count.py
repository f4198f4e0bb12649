"""The algorithmic VALU counts behind the roofline fractions (bench.alg_valu_per_event)
against the event loops the compiler actually emits: the kernels are compiled
for gfx950 to assembly here (no GPU needed) and the VALU instructions of each
kernel's event loop (the longest path once around the innermost loop, by the
compiler's loop annotations, whose blocks hold the LDS histogram atomics) are
counted. Each loop may issue at most a few instructions more
than the count (loop and scheduling overhead), and never fewer."""
import os
import re
import subprocess

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2010_09341_amd", "csrc")


def _blocks(lines):
    """Basic blocks in layout order: [name, instruction lines, label comments]."""
    blocks = []
    cur = None
    for line in lines:
        lm = re.match(r"^\.L(BB\S+):(.*)$", line)
        um = re.match(r"^; %bb\.(\d+):(.*)$", line)
        if lm or um:
            cur = [lm.group(1) if lm else f"bb.{um.group(1)}", [], (lm or um).group(2)]
            blocks.append(cur)
            continue
        if cur is None:
            cur = ["entry", [], ""]
            blocks.append(cur)
        if line.strip().startswith(";") and not cur[1]:
            cur[2] += " " + line.strip()  # a header's comment can follow its label line
            continue
        cur[1].append(line)
    return blocks


def _insts(lines):
    return [x.strip() for x in lines if x.strip() and not x.strip().startswith((";", "."))]


def _event_loop(lines):
    """VALU instructions on the longest path once around the kernel's event
    loop: the innermost loop (by the compiler's loop annotations) whose blocks
    hold the LDS histogram atomics, its blocks' control-flow graph with the
    edges back to the header removed, the path from the header to a latch."""
    blocks = _blocks(lines)
    names = [b[0] for b in blocks]
    at = {n: i for i, n in enumerate(names)}
    loop_of, headers = {}, set()
    for n, _, ann in blocks:
        if re.search(r"This (Inner )?Loop Header: Depth=\d+", ann):
            headers.add(n)
            loop_of[n] = n
        m = re.search(r"in Loop: Header=(BB\S+) Depth=\d+", ann)
        if m and n not in loop_of:
            loop_of[n] = m.group(1)
    succ = {}
    for i, (n, body, _) in enumerate(blocks):
        ins = _insts(body)
        out = [m.group(1) for x in ins for m in [re.match(r"s_c?branch\w*\s+\.L(BB\S+)", x)] if m]
        last = ins[-1] if ins else ""
        if not (last.startswith("s_branch") or last.startswith("s_endpgm")) and i + 1 < len(blocks):
            out.append(names[i + 1])
        succ[n] = out
    best = None
    for h in headers:
        members = {n for n in names if loop_of.get(n) == h}
        bodies = {n: _insts(blocks[at[n]][1]) for n in members}
        if not any(x.startswith("ds_add") for b in bodies.values() for x in b):
            continue
        if any(n in headers and n != h for n in members):
            continue  # not innermost
        valu = {n: sum(1 for x in b if x.startswith("v_")) for n, b in bodies.items()}
        memo = {}

        def longest(n, h=h, members=members, valu=valu, memo=memo):
            if n not in memo:
                memo[n] = valu[n] + max([longest(s) for s in succ[n] if s != h and s in members],
                                        default=0)
            return memo[n]

        v = longest(h)
        best = v if best is None else max(best, v)
    return best


def _event_loops(asm: str):
    """{kernel symbol: VALU instructions once around its event loop}."""
    return {m.group(1): _event_loop(m.group(2).split("\n"))
            for m in re.finditer(r"^(_ZN5vegas9k_iterate\S+):[^\n]*\n(.*?)^\.Lfunc_end", asm,
                                 re.S | re.M)}


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
         ("ILi4ELi3ELi1ELb0", 4, 1, 3), ("ILi4ELi3ELi0ELb0", 4, 0, 3),
         ("ILi16ELi4ELi1ELb0", 16, 1, 4)]


@pytest.mark.parametrize("key,dim,prec,fid", CASES, ids=["gauss8d_fp32", "gauss8d_fp64", "lo_toy_fp32",
                                                         "lo_toy_fp64", "rambo24_fp32"])
def test_event_loop_matches_count(loops, key, dim, prec, fid):
    issued = [v for k, v in loops.items() if key in k]
    assert len(issued) == 1 and issued[0] is not None, loops
    counted = bench.alg_valu_per_event(dim, prec, fid)
    assert counted <= issued[0] <= counted + 6, (issued[0], counted)
