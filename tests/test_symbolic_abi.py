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


def _reach_pattern(s, rL, rS):
    """X's structural pattern through the oracle: the blocks of the rL + rS
    sphere where the product of all-ones L and S (or S and L) is nonzero."""
    pS, pL, pX = oracle.pattern(s, rS), oracle.pattern(s, rL), oracle.pattern(s, rL + rS)
    one = lambda p: oracle.Matrix(p, np.ones(p.nval))
    nz = (oracle.multiply(one(pL), one(pS), pX).val != 0) | (oracle.multiply(one(pS), one(pL), pX).val != 0)
    keep = np.add.reduceat(nz.astype(np.int64), pX.off) > 0
    rows = pX.rows_of_blocks()[keep]
    row_ptr = np.zeros(s.n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=s.n), out=row_ptr[1:])
    nfn = np.asarray(s.nfn, np.int64)
    sz = nfn[rows] * nfn[pX.col[keep]]
    off = np.zeros(sz.size, np.int64)
    off[1:] = np.cumsum(sz)[:-1]
    sub = oracle.Pattern(s, pX.R, row_ptr, pX.col[keep].copy(), pX.img[keep].copy(), off, int(sz.sum()),
                         np.ones(s.n, np.uint8))
    return sub, pX, keep


def _diamond_reach_count(rL, rS, a=10.26):
    """Sites k within rL + rS of a site where some site l has |l| <= rL and
    |k - l| <= rS, or |l| <= rS and |k - l| <= rL (integer a/4 coordinates)."""
    m = int(np.ceil(4 * (rL + rS) / a)) + 2
    g = np.arange(-m, m + 1)
    x, y, z = (v.ravel() for v in np.meshgrid(g, g, g, indexing="ij"))
    sm = x + y + z
    even = (x % 2 == 0) & (y % 2 == 0) & (z % 2 == 0) & (sm % 4 == 0)
    odd = (x % 2 != 0) & (y % 2 != 0) & (z % 2 != 0) & (sm % 4 == 3)
    pts = np.stack([x, y, z], 1)[even | odd]
    u2 = (a / 4.0) ** 2
    r2 = (pts ** 2).sum(1) * u2
    K = pts[r2 <= (rL + rS) ** 2]
    hit = np.zeros(len(K), bool)
    for r1, r2_ in ((rL, rS), (rS, rL)):
        Lp = pts[r2 <= r1 * r1]
        d = ((K[:, None, :] - Lp[None, :, :]) ** 2).sum(2) * u2
        hit |= np.any(d <= r2_ * r2_, axis=1)
    return int(hit.sum()), int(len(K))


def test_structural_x_pattern():
    """X = LS on the blocks of the rL + rS sphere that L S or S L reaches: the
    library's pattern equals the oracle's reach set (all-ones products), its
    rows hold the integer-enumerated count on perfect diamond, the dropped
    blocks of the oracle's X on seeded values are exactly zero, and the
    pattern is symmetric."""
    for s, rS, rH, rL, perfect in ((workloads.diamond(2), 8.0, 12.0, 16.0, True),
                                   (workloads.diamond(2), 8.0, 12.0, 12.0, True),
                                   (workloads.diamond(2, jitter=0.1, seed=7), 8.0, 12.0, 16.0, False),
                                   (workloads.random_cluster(60, 12.0, nfn=np.arange(60) % 5 + 1, seed=9), 5.0, 6.0, 6.5,
                                    False)):
        lnv = lsdm.LNV(lsdm.System.from_workload(s), rS, rH, rL)
        sub, sphere, keep = _reach_pattern(s, rL, rS)
        assert same_pattern(lnv.patterns["X"], sub)
        if perfect:
            reach, ball = _diamond_reach_count(rL, rS)
            assert np.all(np.diff(sub.row_ptr) == reach) and reach < ball
        inp = oracle.make_inputs(s, rS, rH, rL)
        X = oracle.multiply(inp["L"], inp["S"], sphere)
        dropped = np.repeat(~keep, np.diff(np.append(sphere.off, sphere.nval)))
        assert np.all(X.val[dropped] == 0.0)
        assert np.count_nonzero(X.val[~dropped]) > 0
        T = oracle.transpose(oracle.Matrix(sub, np.arange(sub.nval, dtype=np.float64) + 1.0), sub)
        assert np.all(T.val != 0.0)        # every mirror block is in the pattern


def test_lnv_work_counts_si64():
    """Useful triples of the chain on perfect diamond Si, RL = 12: forward X,
    LSL, LSLSL and the five adjoint products, against the oracle's own counts
    on the same patterns (X on its structural pattern)."""
    s = workloads.diamond(2)
    rS, rH, rL = 8.0, 12.0, 12.0
    lnv = lsdm.LNV(lsdm.System.from_workload(s), rS, rH, rL)
    nf, ff = lnv.info(False)
    ng, fg = lnv.info(True)
    R = oracle.chain_ranges(rS, rH, rL)
    pS, pH, pL, pM = (oracle.pattern(s, R[w]) for w in "SHLM")
    pX = _reach_pattern(s, rL, rS)[0]
    one = lambda p: oracle.Matrix(p, np.ones(p.nval))
    T = lambda p: oracle.transpose(one(p), p)

    def cnt(A, B, pC):
        return oracle.multiply(A, B, pC, count=True)[1]
    fwd = cnt(one(pL), one(pS), pX) + cnt(one(pX), one(pL), pM) + cnt(one(pX), one(pM), pH)
    assert nf == fwd
    assert ff == 128.0 * nf
    adj = (cnt(T(pX), one(pH), pM) + cnt(one(pH), one(pM), pX) + cnt(one(pM), one(pL), pX)
           + cnt(T(pX), one(pM), pL) + cnt(one(pX), one(pS), pL))
    assert ng == fwd + adj
    # on the sphere X the chain would do more: the structural pattern saves work
    from tests.test_oracle_pins import diamond_triples
    full_fwd = s.n * (diamond_triples(12, 8, R["X"]) + diamond_triples(R["X"], 12, R["M"])
                      + diamond_triples(R["X"], R["M"], 12))
    assert nf < full_fwd


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


def test_allocator_arguments():
    """lsdm_set_allocator takes both functions or neither; without a device
    no workspace is allocated, so the caller's allocator is never called."""
    L = lsdm.lib()
    a = lsdm._ALLOC_FN(lambda n, ctx: None)
    f = lsdm._FREE_FN(lambda ptr, ctx: None)
    assert L.lsdm_set_allocator(ctypes.cast(a, ctypes.c_void_p), None, None) == lsdm._lib.EINVAL
    assert L.lsdm_set_allocator(None, ctypes.cast(f, ctypes.c_void_p), None) == lsdm._lib.EINVAL
    assert L.lsdm_set_allocator(None, None, None) == lsdm._lib.OK
    with pytest.raises(ValueError):
        lsdm.set_allocator(lambda n: 0, None)
    import torch
    if torch.cuda.is_available():
        return
    calls = []
    lsdm.set_allocator(lambda n: calls.append(n), lambda ptr: None)
    try:
        gs = lsdm.System.from_workload(workloads.diamond(1))
        lnv = lsdm.LNV(gs, 4.0, 6.0, 6.0, symmetric=True)
        assert lnv.info(True)[0] > 0
        del lnv, gs
    finally:
        lsdm.set_allocator()
    assert calls == []


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
    the chain's products has exactly one block triple (eight in the full
    chain, seven in symmetric mode, where dE/dL's 6 HX term is a projection of
    B1's HX); zero atoms are refused."""
    s1 = workloads.System(xyz=np.zeros((1, 3)), nfn=np.array([4], np.int32), lattice=None)
    g = lsdm.System.from_workload(s1)
    for R in (0.0, 5.0, 100.0):
        p = lsdm.Pattern(g, R)
        assert (p.n_blocks, p.n_values) == (1, 16)
        assert oracle.pattern(s1, R).nblocks == 1
    for sym, n_adj in ((False, 5), (True, 4)):
        lnv = lsdm.LNV(g, 4.0, 5.0, 5.0, symmetric=sym)
        assert lnv.info(False) == (3, 3 * 128.0) and lnv.info(True) == (3 + n_adj, (3 + n_adj) * 128.0)
    with pytest.raises(lsdm.LsdmError) as e:
        lsdm.System(np.zeros((0, 3)), np.zeros(0, np.int32))
    assert e.value.code == lsdm._lib.EINVAL
