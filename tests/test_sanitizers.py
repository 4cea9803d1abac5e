"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU side:
the oracle's C library (gcc) running the oracle pin tests, and the host
side of libfusedir (hipcc with the sanitizers for the host pass only)
running its argument validation and error paths, which need no GPU.  Each
runs in a child process with the sanitizer runtime preloaded; any report
aborts it."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _run(cmd, env, timeout):
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=timeout)
    out = res.stdout + res.stderr
    assert "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert res.returncode == 0, out[-4000:]
    return out


def _gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not available")
    return path


# oracle pin tests that cover every oracle module in a few seconds each
ORACLE_TESTS = [
    "tests/test_oracle_pins.py",
    "tests/test_oracle_numpy_objective.py",
    "tests/test_oracle_visibility_pins.py",
    "tests/test_oracle_learned_pins.py",
    "tests/test_oracle_fpmvo_pins.py",
    "tests/test_oracle_gabor_pins.py",
    "tests/test_oracle_volume_pins.py",
    "tests/test_oracle_phg_pins.py",
]


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    import oracle
    with tempfile.TemporaryDirectory() as tmp:
        lib = oracle.build(out=os.path.join(tmp, "liboracle_san.so"), sanitize=True)
        env = dict(os.environ)
        env.update(FD_ORACLE_LIB=lib, LD_PRELOAD=_gcc_runtime("libasan.so"),
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
                   OMP_NUM_THREADS="4")
        out = _run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                    "-p", "no:cacheprovider", "-k", "not brute_force"] + ORACLE_TESTS,
                   env, timeout=1200)
        assert " passed" in out, out[-2000:]


HOST_SCRIPT = r"""
import ctypes, sys
sys.path.insert(0, sys.argv[2])
from paper_2604_05794_amd import native
native.LIB_PATH = sys.argv[1]
L = native.lib()
P = native.Params()
L.fd_params_init(ctypes.byref(P))
assert P.top_k == 5
err = lambda: L.fd_last_error().decode()
null = None
buf = (ctypes.c_float * 64)()
cams = (ctypes.c_float * 16 * 4)()

def expect_fail(r, what):
    assert r != 0, what
    msg = err()
    assert msg, what
    return msg

# plain entry: each check fails before anything touches a device
bad = native.Params(); L.fd_params_init(ctypes.byref(bad))
bad.width, bad.height = 64, 64
expect_fail(L.fd_fuse_directions(buf, -1, cams, 4, buf, buf, ctypes.byref(bad), buf, buf), "n < 0")
expect_fail(L.fd_fuse_directions(buf, 10, cams, 0, buf, buf, ctypes.byref(bad), buf, buf), "V = 0")
expect_fail(L.fd_fuse_directions(null, 10, cams, 4, buf, buf, ctypes.byref(bad), buf, buf), "null points")
expect_fail(L.fd_fuse_directions(buf, 10, cams, 4, buf, buf, None, buf, buf), "null params")
for field, value in (("patch", 4), ("patch", 0), ("n_candidates", 0), ("n_candidates", 1 << 20),
                     ("refine_iters", -1), ("refine_iters", 1000), ("top_k", 0), ("top_k", 99),
                     ("width", 0), ("height", 1 << 20), ("map_dtype", 7), ("mode", 9),
                     ("learned_iters", -3), ("z_near", -1.0), ("vis_tau", -1.0)):
    q = native.Params(); L.fd_params_init(ctypes.byref(q)); q.width = q.height = 64
    setattr(q, field, value)
    expect_fail(L.fd_fuse_directions(buf, 10, cams, 4, buf, buf, ctypes.byref(q), buf, buf), field)
    expect_fail(L.fd_fuse_directions_noalloc(buf, 10, cams, 4, buf, buf, ctypes.byref(q), buf, buf), field)
q = native.Params(); L.fd_params_init(ctypes.byref(q)); q.width = q.height = 64
expect_fail(L.fd_fuse_directions_noalloc(buf, 1 << 40, cams, 4, buf, buf, ctypes.byref(q), buf, buf), "too many points")
# batched entry
scenes = (native.Scene * 2)()
expect_fail(L.fd_fuse_directions_batched(scenes, 0, ctypes.byref(q), None), "no scenes")
expect_fail(L.fd_fuse_directions_batched(scenes, 10000, ctypes.byref(q), None), "too many scenes")
expect_fail(L.fd_fuse_directions_batched(None, 2, ctypes.byref(q), None), "null scenes")
expect_fail(L.fd_fuse_directions_batched(scenes, 2, ctypes.byref(q), None), "no context")
# the stages around the path
g = native.GaborParams(); L.fd_gabor_params_init(ctypes.byref(g))
expect_fail(L.fd_orientation_maps(buf, 0, 64, 64, ctypes.byref(g), buf, buf), "no frames")
g.radius = -2
expect_fail(L.fd_orientation_maps(buf, 1, 64, 64, ctypes.byref(g), buf, buf), "radius")
# a message longer than any buffer, and a device-side call without a device
long_path = ("x" * 5000).encode()
m = ctypes.c_void_p()
r = L.fd_mlp_create(ctypes.byref(m), 1)
if r == 0:
    expect_fail(L.fd_mlp_load(m, long_path), "missing checkpoint")
    L.fd_mlp_destroy(m)
else:
    assert err()
c = ctypes.c_void_p()
r = L.fd_context_create(ctypes.byref(c))
if r == 0:
    L.fd_context_destroy(c)
else:
    assert err()
print("host checks done")
"""


def test_host_library_under_address_and_undefined_behaviour_sanitizers():
    from paper_2604_05794_amd import build as fdbuild
    rt = None
    for d in sorted(os.listdir("/opt/rocm/llvm/lib/clang")) if os.path.isdir(
            "/opt/rocm/llvm/lib/clang") else []:
        cand = f"/opt/rocm/llvm/lib/clang/{d}/lib/linux/libclang_rt.asan-x86_64.so"
        if os.path.exists(cand):
            rt = cand
    if rt is None:
        pytest.skip("clang AddressSanitizer runtime not available")
    with tempfile.TemporaryDirectory() as tmp:
        lib = os.path.join(tmp, "libfusedir_san.so")
        # sanitizers for the host pass only (each flag behind -Xarch_host);
        # the device code is the same as the product's
        fdbuild.build(out=lib, extra=["-Xarch_host", "-fsanitize=address",
                                      "-Xarch_host", "-fsanitize=undefined",
                                      "-Xarch_host", "-fno-sanitize-recover=all",
                                      "-Xarch_host", "-fno-omit-frame-pointer",
                                      "-shared-libsan"])
        env = dict(os.environ)
        env.update(LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
        out = _run([sys.executable, "-c", HOST_SCRIPT, lib, ROOT], env, timeout=600)
        assert "host checks done" in out, out[-2000:]
