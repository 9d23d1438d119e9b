"""Host-side checks of the HIP library: it loads, exports every declared
symbol, builds the same range patterns as the oracle, counts the same useful
block triples, and reports errors with the documented codes.  No kernel runs
here (the container has no GPU); compute calls are exercised in the gpu tests."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import workloads
import paper_0911_3584_amd as lsdm
from tests._sides import same_pattern

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "lsdm.h")).read()
    names = set(re.findall(r"\b(lsdm_[a-z0-9_]+)\s*\(", hdr))
    assert len(names) >= 18
    L = ctypes.CDLL(lsdm._lib.SO)
    for n in sorted(names):
        assert hasattr(L, n), n
    assert names == set(lsdm._lib.SIGNATURES), names ^ set(lsdm._lib.SIGNATURES)


SYSTEMS = {
    "si64": lambda: workloads.diamond(2),
    "si64_jitter": lambda: workloads.diamond(2, jitter=0.1, seed=2),
    "si8_cell": lambda: workloads.diamond(1),
    "mixed_box": lambda: workloads.random_box(120, 14.0, 96, 13, 5, seed=3),
    "open_mixed": lambda: workloads.random_cluster(50, 12.0, nfn=np.arange(50) % 7 + 1, seed=4),
    "si_slab_h": lambda: workloads.si_slab((2, 1, 1)),
}


@pytest.mark.parametrize("name", list(SYSTEMS))
@pytest.mark.parametrize("R", [0.0, 4.5, 8.0, 12.0, 20.0, 36.0])
def test_pattern_equals_oracle(name, R):
    s = SYSTEMS[name]()
    gs = lsdm.System.from_workload(s)
    gp = lsdm.Pattern(gs, R)
    op = oracle.pattern(s, R)
    assert gp.n_blocks == op.nblocks and gp.n_values == op.nval
    assert same_pattern(gp, op)


@pytest.mark.parametrize("name", ["si64", "mixed_box", "open_mixed", "si_slab_h"])
@pytest.mark.parametrize("tA,tB", [(0, 0), (1, 0), (0, 1)])
def test_plan_triples_equal_oracle(name, tA, tB):
    s = SYSTEMS[name]()
    rA, rB, rC = 7.0, 6.0, 9.0
    gs = lsdm.System.from_workload(s)
    plan = lsdm.Plan(lsdm.Pattern(gs, rA), tA, lsdm.Pattern(gs, rB), tB, lsdm.Pattern(gs, rC))
    pA, pB, pC = oracle.pattern(s, rA), oracle.pattern(s, rB), oracle.pattern(s, rC)
    A = oracle.Matrix(pA, np.ones(pA.nval))
    B = oracle.Matrix(pB, np.ones(pB.nval))
    if tA:
        A = oracle.transpose(A, pA)
    if tB:
        B = oracle.transpose(B, pB)
    _, nt = oracle.multiply(A, B, pC, count=True)
    assert plan.n_triples == nt
    # flops: sum over triples of 2 nfn_i nfn_k nfn_j, by brute force on the oracle patterns
    nfn = s.nfn.astype(np.int64)
    fl = 0
    bi, bk, bim = pA.keys()
    cset = set(zip(*[a.tolist() for a in pC.keys()[:2]], map(tuple, pC.img.tolist())))
    for i, k, m in zip(bi, bk, map(tuple, bim.tolist())):
        for b in range(pB.row_ptr[k], pB.row_ptr[k + 1]):
            j = int(pB.col[b]); n = tuple(int(x) + y for x, y in zip(pB.img[b], m))
            if (int(i), j, n) in cset:
                fl += 2 * nfn[i] * nfn[k] * nfn[j]
    assert plan.flops == fl


def test_lnv_work_counts_si64():
    """Useful triples per atom of the chain on perfect diamond Si, RL = 12:
    forward X, LSL, LSLSL and the five adjoint products."""
    s = workloads.diamond(2)
    lnv = lsdm.LNV(lsdm.System.from_workload(s), 8.0, 12.0, 12.0)
    nf, ff = lnv.info(False)
    ng, fg = lnv.info(True)
    from tests.test_oracle_pins import diamond_triples
    R = oracle.chain_ranges(8.0, 12.0, 12.0)
    fwd = diamond_triples(12, 8, R["X"]) + diamond_triples(R["X"], 12, R["M"]) + diamond_triples(R["X"], R["M"], 12)
    assert nf == s.n * fwd
    assert ff == 128.0 * nf
    adj = (diamond_triples(R["X"], 12, R["M"]) + diamond_triples(12, R["M"], R["X"]) + diamond_triples(R["M"], 12, R["X"])
           + diamond_triples(R["X"], R["M"], 12) + diamond_triples(R["X"], 8, 12))
    assert ng == s.n * (fwd + adj)


def test_errors():
    s = workloads.diamond(1)
    xyz = s.xyz.copy(); xyz[3, 1] = np.nan
    with pytest.raises(lsdm.LsdmError) as e:
        lsdm.System(xyz, s.nfn, s.lattice)
    assert e.value.code == lsdm._lib.EINVAL
    nfn = s.nfn.copy(); nfn[0] = 17
    with pytest.raises(lsdm.LsdmError) as e:
        lsdm.System(s.xyz, nfn, s.lattice)
    assert e.value.code == lsdm._lib.EINVAL
    gs = lsdm.System.from_workload(s)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(lsdm.LsdmError) as e:
            lsdm.Pattern(gs, bad)
        assert e.value.code == lsdm._lib.EINVAL
    other = lsdm.System.from_workload(workloads.diamond(1))
    with pytest.raises(lsdm.LsdmError) as e:
        lsdm.Plan(lsdm.Pattern(gs, 5.0), 0, lsdm.Pattern(other, 5.0), 0, lsdm.Pattern(gs, 5.0))
    assert e.value.code == lsdm._lib.EPATTERN
    sing = np.zeros((3, 3))
    with pytest.raises(lsdm.LsdmError) as e:
        lsdm.System(s.xyz, s.nfn, sing)
    assert e.value.code == lsdm._lib.EINVAL
    # ranges far beyond what the image encoding can hold fail cleanly, however large
    for huge in (3000.0, 1e5, 1e12, 1e300):
        with pytest.raises(lsdm.LsdmError) as e:
            lsdm.Pattern(gs, huge)
        assert e.value.code == lsdm._lib.EUNSUPPORTED
    h = ctypes.c_void_p()
    rc = lsdm.lib().lsdm_lnv_create_ex(gs._h, 4.0, 5.0, 5.0, 2, ctypes.byref(h))
    assert rc == lsdm._lib.EINVAL and not h.value
    # symmetric-mode plans: fewer triples than the full chain, same patterns
    full, sym = lsdm.LNV(gs, 4.0, 6.0, 6.0), lsdm.LNV(gs, 4.0, 6.0, 6.0, symmetric=True)
    assert sym.info(True)[0] < full.info(True)[0] and sym.info(False)[0] < full.info(False)[0]
    for w in full.patterns:
        assert full.patterns[w].n_values == sym.patterns[w].n_values


def test_pattern_beyond_the_block_limit_is_enomem():
    """A finite range whose pattern would exceed the library's size limit
    (2^31 blocks, whose values alone would fill the device) is refused with
    LSDM_ENOMEM before any row is stored, and the system stays usable."""
    import time
    s = workloads.diamond(4)                     # 512 atoms, 41 bohr cell
    gs = lsdm.System.from_workload(s)
    t0 = time.perf_counter()
    with pytest.raises(lsdm.LsdmError) as e:
        lsdm.Pattern(gs, 600.0)                  # about 3.4e9 pairs
    assert e.value.code == lsdm._lib.ENOMEM
    assert "2^31" in str(e.value)
    assert time.perf_counter() - t0 < 60.0
    assert lsdm.Pattern(gs, 8.0).n_blocks == 512 * 17


def test_compute_without_device_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    s = workloads.diamond(1)
    gs = lsdm.System.from_workload(s)
    p = lsdm.Pattern(gs, 5.0)
    rc = lsdm.lib().lsdm_dot(p._h, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8), None)
    assert rc == lsdm._lib.EDEVICE


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr and r.stdout == ""


def test_degenerate_systems():
    """One atom (open): every pattern holds its on-site block only, and each of
    the chain's eight products has exactly one block triple in either mode;
    zero atoms are refused."""
    s1 = workloads.System(xyz=np.zeros((1, 3)), nfn=np.array([4], np.int32), lattice=None)
    g = lsdm.System.from_workload(s1)
    for R in (0.0, 5.0, 100.0):
        p = lsdm.Pattern(g, R)
        assert (p.n_blocks, p.n_values) == (1, 16)
        assert oracle.pattern(s1, R).nblocks == 1
    for sym in (False, True):
        lnv = lsdm.LNV(g, 4.0, 5.0, 5.0, symmetric=sym)
        assert lnv.info(False) == (3, 3 * 128.0) and lnv.info(True) == (8, 8 * 128.0)
    with pytest.raises(lsdm.LsdmError) as e:
        lsdm.System(np.zeros((0, 3)), np.zeros(0, np.int32))
    assert e.value.code == lsdm._lib.EINVAL
