"""Work counts of the GPU symbolic pass against the oracle.

With a device present, a plan's useful block triples and flops come from the
counters of the step generator on the GPU (the host path that the CPU suite
checks does not run).  These tests hold those GPU counts to the oracle's own
triple counts and to a brute-force flop sum on the same patterns, for single
products (all transpose forms, mixed function counts, periodic and open
systems) and for the whole chain."""
import numpy as np
import pytest

import oracle
import workloads
import paper_0911_3584_amd as lsdm
from tests.test_symbolic_abi import SYSTEMS, _reach_pattern

pytestmark = pytest.mark.gpu


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def _brute_flops(s, pA, pB, pC):
    """2 nfn_i nfn_k nfn_j summed over the triples (i, k, j) with (i, k) in A,
    (k, j) in B and (i, j) in C, images composed."""
    nfn = s.nfn.astype(np.int64)
    cset = set(zip(*[a.tolist() for a in pC.keys()[:2]], map(tuple, pC.img.tolist())))
    fl = 0
    bi, bk, bim = pA.keys()
    for i, k, m in zip(bi, bk, map(tuple, bim.tolist())):
        for b in range(pB.row_ptr[k], pB.row_ptr[k + 1]):
            j = int(pB.col[b])
            n = tuple(int(x) + y for x, y in zip(pB.img[b], m))
            if (int(i), j, n) in cset:
                fl += 2 * nfn[i] * nfn[k] * nfn[j]
    return fl


@pytest.mark.parametrize("name", ["si64", "mixed_box", "open_mixed", "si_slab_h"])
@pytest.mark.parametrize("tA,tB", [(0, 0), (1, 0), (0, 1)])
def test_gpu_plan_counts_equal_oracle(name, tA, tB):
    _need_gpu()
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
    assert plan.flops == _brute_flops(s, pA, pB, pC)


def test_gpu_lnv_work_counts_si64():
    """The chain's useful triples on perfect diamond Si (R_L = 12) with the GPU
    step generator: forward X, LSL, LSLSL and the five adjoint products of the
    full chain, against the oracle's counts on the same patterns."""
    _need_gpu()
    s = workloads.diamond(2)
    rS, rH, rL = 8.0, 12.0, 12.0
    lnv = lsdm.LNV(lsdm.System.from_workload(s), rS, rH, rL)
    nf, ff = lnv.info(False)
    ng, _ = lnv.info(True)
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
