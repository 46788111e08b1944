"""Host hygiene: the FP64 C oracle and the HIP library's host code built with
AddressSanitizer and UndefinedBehaviorSanitizer and run on the CPU.

The oracle is rebuilt with gcc's sanitizers and driven through every code path
the tests use (each problem family, every cycle shape, the adaptive test, the
lagged Algorithm 1, the variants, loads, checkpoints, the inspection calls and
the argument errors).  The library's host code (validation, layout, schedule
and batch sizing in biotlbm.cpp) is rebuilt with clang's sanitizers on the host
side only, linked with the normally built kernel object, and driven through
the calls that need no GPU.  Either run fails on any sanitizer report."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2409_11382_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG_ASAN = "/opt/rocm/llvm/lib/clang/22/lib/linux/libclang_rt.asan-x86_64.so"


def _gcc_runtime(name):
    try:
        path = subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _run(script, preload, env_extra=None):
    env = dict(os.environ)
    env.update({"LD_PRELOAD": preload, "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=86",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1:exitcode=87",
                "PYTHONPATH": ROOT, "OMP_NUM_THREADS": "2"})
    env.update(env_extra or {})
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, env=env, timeout=600)
    report = r.stderr[-4000:]
    assert r.returncode == 0, report
    for marker in ("AddressSanitizer", "runtime error:", "LeakSanitizer"):
        assert marker not in r.stderr, report
    return r.stdout


ORACLE_SCRIPT = r'''
import sys
import numpy as np
import oracle.oracle as O
from paper_2409_11382_amd import problem as P
O._LIB = __import__("os").environ["SAN_ORACLE_LIB"]

def run(p, n, loads=None, threads=1):
    o = O.Oracle(p, threads=threads, history=8)
    if loads is not None:
        f, s = loads
        o.set_loads(f, s)
    o.step(n)
    F = o.fields()
    assert all(np.isfinite(F[k]).all() for k in ("eta", "p", "sigma"))
    return o

strip = P.loaded_strip(n=16, alpha=1.0, ne_fixed=2, K=2, levels=3)
o = run(strip, 3, threads=2)
o.get_history()
st = o.get_state()
o.set_state(st["f"], st["g"], st["D1"], st["D2"], step=st["step"])
o.step(1)
o.explicit_force()
for l in range(1, o.levels + 1):
    nx, ny = o.level_shape(l)
    g = np.random.default_rng(l).standard_normal((8, ny, nx)) * 1e-3
    o.apply_elastic(l, g)
    o.mg_cycle(l, g)
o.flow_step(np.zeros((strip.ny, strip.nx)))
o.coarsest_visits()
for cyc in (P.CYCLE_W, P.CYCLE_F, P.CYCLE_FMG):
    run(strip.replace(cycle=cyc), 2)
    run(strip.replace(cycle=cyc, ne_fixed=0, ne_tol=1e-6, ne_max=12), 2)
run(strip.replace(ne_fixed=0, ne_tol=1e-6, ne_max=20), 3)
o = O.Oracle(strip.replace(ne_fixed=0, ne_tol=1e-6, ne_max=20))
o.set_ne_schedule([1, 2, 3])
o.step(3)
run(strip.replace(fstar_literal=1, coarse_sweeps=16, pressure_gradient=P.GRAD_CENTRAL), 2)
run(strip.replace(levels=1, ne_fixed=4, lag=1, gamma=1.0), 2)
run(strip.replace(levels=1, ne_fixed=4, lag=0, gamma=1.0), 2)
M = P.Manufactured(8, alpha=0.5, r=0.0, K=2, ne_fixed=2)
run(M.problem, 2, loads=M.loads(M.problem.dt))
run(P.terzaghi(nx=8, ny=32, levels=2, ne_fixed=0, ne_tol=1e-8, ne_max=10), 2)
run(P.layered_column(n=16, nx=4), 2)
run(P.with_random_boundary_data(P.loaded_strip(n=16, levels=2, ne_fixed=1, K=2), seed=1), 2)
run(P.heterogeneous_strip(n=32, levels=2, ne_fixed=1, K=2), 2)
for bad in (dict(nx=0), dict(levels=9), dict(cycle=7), dict(coarse_sweeps=3), dict(lag=1)):
    try:
        O.Oracle(strip.replace(**bad))
    except O.OracleError:
        pass
    else:
        raise AssertionError(bad)
print("oracle ok")
'''


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc's sanitizer runtimes are not installed")
    lib = str(tmp_path / "libbiot_oracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-Wall", "-Wno-unused-variable", "-o", lib,
                           os.path.join(ROOT, "oracle", "biot_oracle.c"), "-lm"])
    out = _run(ORACLE_SCRIPT, f"{asan}:{ubsan}", {"SAN_ORACLE_LIB": lib})
    assert "oracle ok" in out


LIB_SCRIPT = r'''
import ctypes as C
import os
import sys
import types
sys.modules["torch"] = types.ModuleType("torch")  # host-only calls: no PyTorch, no device
from paper_2409_11382_amd import lbm as L, problem as P
L.LIB_PATH = os.environ["SAN_LIB"]
lib = L.load_library()
probs = [P.loaded_strip(n=64), P.loaded_strip(n=16384), P.terzaghi(nx=8, ny=128, levels=3),
         P.heterogeneous_strip(n=256, levels=4), P.loading_2d(n=64),
         P.Manufactured(16).problem, P.layered_column(n=32, nx=4),
         P.loaded_strip(n=64).replace(cycle=P.CYCLE_W), P.loaded_strip(n=64).replace(cycle=P.CYCLE_FMG),
         P.loaded_strip(n=64).replace(ne_fixed=0, ne_tol=1e-6, ne_max=20),
         P.loaded_strip(n=64).replace(levels=1, ne_fixed=4, lag=1, gamma=1.0),
         P.loaded_strip(n=64).replace(fstar_literal=1, coarse_sweeps=16)]
for p in probs:
    for prec in ("fp64", "fp32_shifted", "fp32"):
        assert L.workspace_bytes(p, prec) > 0
base = P.loaded_strip(n=64)
for kw in (dict(nx=0), dict(levels=7), dict(nx=63, levels=2), dict(alpha=float("nan")), dict(cycle=4),
           dict(coarse_sweeps=3), dict(lag=1), dict(ne_fixed=0, ne_tol=0.0), dict(gamma=1.5)):
    try:
        L.workspace_bytes(base.replace(**kw), "fp64")
    except L.BiotError:
        pass
    else:
        raise AssertionError(kw)
n = C.c_size_t(0)
arr = (L._Problem * 3)()
keep = []
for i, p in enumerate(P.batch_problems(count=3, seed=1)):
    arr[i], k = L.marshal_problem(p, "fp32_shifted")
    keep.append(k)
assert lib.bp_batch_workspace_bytes(arr, 3, C.byref(n)) == L.BP_OK and n.value > 0
assert lib.bp_batch_workspace_bytes(None, 0, C.byref(n)) == L.BP_ERR_ARG
pb, keep1 = L.marshal_problem(base, "fp32_shifted")
h = C.c_void_p()
assert lib.bp_create(C.byref(pb), None, 0, None, C.byref(h)) != L.BP_OK
assert lib.bp_create_static(C.byref(pb), None, C.byref(h)) != L.BP_OK
assert lib.bp_create(None, None, 0, None, C.byref(h)) != L.BP_OK
assert len(lib.bp_last_error()) > 0
print("library ok")
'''


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG_ASAN)),
                    reason="hipcc or clang's sanitizer runtime is not installed")
def test_library_host_code_under_address_and_undefined_sanitizers(tmp_path):
    kernels = os.path.join(CSRC, "_build", "lbm_kernels.o")
    if not os.path.exists(kernels):
        pytest.skip("the library has not been built (paper_2409_11382_amd/build.py)")
    obj = str(tmp_path / "biotlbm_san.o")
    lib = str(tmp_path / "libbiotlbm_san.so")
    # sanitizers on the host side of the compilation only
    subprocess.check_call([HIPCC, "-x", "hip", "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-function",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-sanitize-recover=undefined",
                           "-Xarch_host", "-fno-omit-frame-pointer",
                           "-c", os.path.join(CSRC, "biotlbm.cpp"), "-o", obj],
                          stderr=subprocess.DEVNULL)
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, obj, kernels,
                           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"])
    out = _run(LIB_SCRIPT, CLANG_ASAN, {"SAN_LIB": lib})
    assert "library ok" in out
