"""The C interface without a GPU: the library loads, exports every function
include/vegas.h declares, and rejects invalid arguments before any device
call. Also the serving scheduler's host logic (arena, admission, chunking),
compiled on its own with g++."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vegas.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vegas_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2010_09341_amd import vegas
    return vegas.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 28
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(
        ROOT, "paper_2010_09341_amd", "libvegas.so")], capture_output=True, text=True,
        check=True).stdout
    exported = set(re.findall(r"\bT (vegas_[a-z_0-9]+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(L, n)


def test_binding_names_match_header():
    from paper_2010_09341_amd import vegas
    for n in _declared():
        if n == "vegas_strerror":
            continue
        assert hasattr(vegas, n), n


def test_status_names(L):
    L.vegas_strerror.restype = ctypes.c_char_p
    assert L.vegas_strerror(0) == b"ok"
    assert L.vegas_strerror(-1) == b"invalid argument"
    assert L.vegas_strerror(-5) == b"non-finite weights"
    assert L.vegas_strerror(42) == b"unknown status"


def test_validation_before_device(L):
    h = ctypes.c_void_p()
    EINVAL = -1
    for dim, nb in ((0, 10), (33, 10), (4, 1), (4, 513), (32, 300), (17, 512), (-1, 5)):
        assert L.vegas_create(dim, nb, ctypes.byref(h)) == EINVAL
    assert L.vegas_create(4, 10, None) == EINVAL
    n = ctypes.c_size_t()
    assert L.vegas_workspace_bytes(8, 50, ctypes.byref(n)) == 0
    assert n.value > 8 * 51 * 8 and n.value % 256 == 0
    assert L.vegas_workspace_bytes(64, 50, ctypes.byref(n)) == EINVAL
    I = ctypes.c_double()
    s = ctypes.c_double()
    assert L.vegas_iterate(None, 2, 100, 0, ctypes.byref(I), ctypes.byref(s)) == EINVAL
    assert L.vegas_refine(None, ctypes.c_double(1.5)) == EINVAL
    assert L.vegas_destroy(None) == 0
    srv = ctypes.c_void_p()
    assert L.vegas_server_create(ctypes.c_size_t(1 << 20), 0, ctypes.c_int64(0),
                                 ctypes.byref(srv)) == EINVAL
    assert L.vegas_server_create(ctypes.c_size_t(1 << 20), 5000, ctypes.c_int64(0),
                                 ctypes.byref(srv)) == EINVAL
    assert L.vegas_server_submit(None, None, None) == EINVAL
    assert L.vegas_server_destroy(None) == 0


def test_scheduler_host_logic(tmp_path):
    exe = str(tmp_path / "sched_test")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I" + os.path.join(ROOT, "paper_2010_09341_amd", "csrc"),
                    os.path.join(ROOT, "tests", "helpers", "sched_test.cpp"), "-o", exe],
                   check=True)
    res = subprocess.run([exe], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    assert res.stdout.strip() == "ok"


def test_integrand_compile_without_gpu():
    """Run-time integrands compile with hiprtc on a machine without a GPU:
    consecutive ids from VEGAS_F_USER, the compiler's log on an error, and
    argument checks."""
    from paper_2010_09341_amd import vegas as vg
    src = ("__device__ double vegas_user_f64(const double* x, int dim, const double* p)"
           " { return x[0] * p[0]; }\n"
           "__device__ float vegas_user_f32(const float* x, int dim, const float* p)"
           " { return x[0] * p[0]; }\n")
    a = vg.vegas_integrand_compile(src)
    b = vg.vegas_integrand_compile(src, 3)
    assert vg.VEGAS_F_USER <= a < vg.VEGAS_F_USER + vg.VEGAS_MAX_USER and b == a + 1
    with pytest.raises(vg.VegasError) as e:
        vg.vegas_integrand_compile(src.replace("x[0] * p[0]; }\n__device__ float",
                                               "y; }\n__device__ float"))
    assert e.value.code == vg.VEGAS_ECOMPILE
    assert "integrand.hip:1" in e.value.log and "undeclared identifier 'y'" in e.value.log
    with pytest.raises(vg.VegasError) as e:  # vegas_user_f32 missing
        vg.vegas_integrand_compile(src.split("\n")[0])
    assert e.value.code == vg.VEGAS_ECOMPILE and "vegas_user_f32" in e.value.log
    L = vg.lib()
    fid = ctypes.c_int(-1)
    assert L.vegas_integrand_compile(None, 0, ctypes.byref(fid), None, 0) == -1
    assert L.vegas_integrand_compile(src.encode(), 33, ctypes.byref(fid), None, 0) == -1
    assert L.vegas_integrand_compile(src.encode(), -1, ctypes.byref(fid), None, 0) == -1
    assert L.vegas_integrand_compile(src.encode(), 0, None, None, 0) == -1
    assert fid.value == -1


def test_integrand_compile_from_threads():
    """vegas_integrand_compile from four threads at once (the library call
    releases the interpreter lock): four distinct ids, each within the
    run-time range."""
    import threading
    from paper_2010_09341_amd import vegas as vg
    ids, errors = [], []

    def compile_one(k):
        src = (f"__device__ double vegas_user_f64(const double* x, int dim, const double* p)"
               f" {{ return x[0] + {k}.0; }}\n"
               f"__device__ float vegas_user_f32(const float* x, int dim, const float* p)"
               f" {{ return x[0] + {k}.0f; }}\n")
        try:
            ids.append(vg.vegas_integrand_compile(src, 2))
        except Exception as e:  # noqa: BLE001 - reported by the assertion below
            errors.append(repr(e))

    threads = [threading.Thread(target=compile_one, args=(k,)) for k in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=300.0)
    assert not errors, errors
    assert len(set(ids)) == 4
    assert all(vg.VEGAS_F_USER <= i < vg.VEGAS_F_USER + vg.VEGAS_MAX_USER for i in ids)
