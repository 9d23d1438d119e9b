"""Host C++ under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle's core (g++) and the library's host sources (the symbolic pass,
layout maps and boundary in symbolic.cpp and api.cpp, built by hipcc with the
sanitizers on the host side only, linked with the normally built device
objects) are compiled with -fsanitize=address,undefined and driven from a
child Python process with the sanitizer runtime preloaded.  The child runs
the host paths the CPU suite covers (patterns of periodic, mixed and open
systems, plans in every transpose form, the chain's symbolic pass, the
oracle's products and chain); any sanitizer report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
       "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run_child(script, preload, tmp_path):
    env = dict(os.environ, LD_PRELOAD=preload, PYTHONPATH=ROOT, **ENV)
    env.pop("OMP_NUM_THREADS", None)
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=600,
                       cwd=str(tmp_path))
    log = r.stdout + r.stderr
    assert r.returncode == 0 and "SANITIZED RUN OK" in r.stdout, log[-4000:]
    assert "runtime error" not in log and "Sanitizer" not in log, log[-4000:]


def _instrumented(so):
    """the library calls into the sanitizer runtime (its code is instrumented)"""
    syms = subprocess.run(["nm", "-D", "--undefined-only", so], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms, so


def _runtime(cmd, name):
    out = subprocess.run(cmd + [f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not out or not os.path.isabs(out) or not os.path.exists(out):
        pytest.skip(f"{name} not available")
    return out



def test_oracle_core_under_asan_ubsan(tmp_path):
    so = str(tmp_path / "libref_core_san.so")
    subprocess.check_call(["g++", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                           "-ffp-contract=off", os.path.join(ROOT, "oracle", "ref_core.cpp"), "-o", so])
    _instrumented(so)
    script = f"""
import ctypes, numpy as np, oracle, workloads
assert hasattr(ctypes.CDLL(None), "__asan_init")
oracle._SO = {so!r}
for s, (rS, rH, rL) in ((workloads.diamond(1), (8.0, 12.0, 12.0)),
                        (workloads.random_box(40, 9.0, 30, 13, 5, seed=2), (4.0, 5.0, 5.0)),
                        (workloads.random_cluster(30, 9.0, nfn=np.arange(30) % 7 + 1, seed=4), (4.0, 5.0, 5.5))):
    inp = oracle.make_inputs(s, rS, rH, rL)
    E = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], rS, rH, rL)["E"]
    G = oracle.lnv_gradient(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    A, B = inp["L"], inp["S"]
    pC = oracle.pattern(s, rL + rS)
    for tA in (0, 1):
        for tB in (0, 1):
            oracle.multiply_op(A, tA, B, tB, pC)
    oracle.multiply_adjoint(A, 0, B, 0, oracle.Matrix(pC, np.ones(pC.nval)))
    oracle.mcweeny(inp["L"], inp["S"], rS, rL)
    assert np.isfinite(E) and np.all(np.isfinite(G.val))
print("SANITIZED RUN OK")
"""
    _run_child(script, _runtime(["g++"], "libasan.so"), tmp_path)


def test_library_host_code_under_asan_ubsan(tmp_path):
    build = os.path.join(ROOT, "paper_0911_3584_amd", "_build")
    dev_objs = [os.path.join(build, f) for f in ("kernels.hip.o", "pattern.hip.o")]
    if not all(os.path.exists(o) for o in dev_objs):
        pytest.skip("build the library first (its device objects are linked as they are)")
    from paper_0911_3584_amd import build as B
    csrc = os.path.join(ROOT, "paper_0911_3584_amd", "csrc")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    procs = []
    for src in ("symbolic.cpp", "api.cpp"):
        o = str(tmp_path / (src + ".o"))
        procs.append(subprocess.Popen([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC"] + B.DEVFLAGS + san
                                      + ["-c", os.path.join(csrc, src), "-o", o],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        objs.append(o)
    for p in procs:
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, out[-3000:]
    so = str(tmp_path / "liblsdm_san.so")
    subprocess.check_call([HIPCC] + B.DEVFLAGS + ["-shared", "-fPIC", "-o", so] + objs + dev_objs + ["-lpthread"])
    _instrumented(so)
    script = f"""
import ctypes, numpy as np, workloads
assert hasattr(ctypes.CDLL(None), "__asan_init")
from paper_0911_3584_amd import _lib
_lib.SO = {so!r}
import paper_0911_3584_amd as lsdm
cases = ((workloads.diamond(1), (8.0, 12.0, 12.0)),
         (workloads.diamond(2, jitter=0.1, seed=1), (8.0, 12.0, 16.0)),
         (workloads.random_box(60, 10.0, 48, 13, 5, seed=2), (4.0, 5.0, 5.0)),
         (workloads.random_cluster(40, 10.0, nfn=np.arange(40) % 7 + 1, seed=4), (4.0, 5.0, 5.5)),
         (workloads.si_slab((2, 1, 1)), (6.0, 8.0, 8.0)))
for s, (rS, rH, rL) in cases:
    gs = lsdm.System.from_workload(s)
    pa, pb, pc = lsdm.Pattern(gs, rL), lsdm.Pattern(gs, rS), lsdm.Pattern(gs, rL + rS)
    for tA in (0, 1):
        for tB in (0, 1):
            assert lsdm.Plan(pa, tA, pb, tB, pc).n_triples >= 0
    for sym in (False, True):
        lnv = lsdm.LNV(gs, rS, rH, rL, symmetric=sym)
        assert lnv.info(True)[0] > 0
        for w in lnv.patterns:
            lnv.patterns[w].keys()
        del lnv
for bad in (-1.0, float("nan"), 1e300):
    try:
        lsdm.Pattern(lsdm.System.from_workload(workloads.diamond(1)), bad)
    except lsdm.LsdmError:
        pass
print("SANITIZED RUN OK")
"""
    _run_child(script, _runtime([os.path.join(os.path.dirname(HIPCC), "..", "llvm", "bin", "clang")],
                                "libclang_rt.asan-x86_64.so"), tmp_path)
