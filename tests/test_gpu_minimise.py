"""GPU parity of the ground-state search: the exact line search, the
conjugate-gradient minimiser, the chemical-potential shift H - mu S and the
electron number N_e = 2 Tr(KS), against the FP64 oracle on the same seeded
inputs (section 2: the minimisation over L and constraint 2).

Bars: shift exact up to one rounding of mu S (fused or not); N_e and dN_e/dL
1e-12 relative (the FP64 bar of the chain); line coefficients within 1e-11 of
sum |c_k| h^k (four energies combined by interpolation, each good to about
1e-14 relative); minimiser histories 1e-9 relative in E and 1e-6 in |dE/dL|
over eight steps (the GPU line uses energy differences, whose rounding moves
each step length by about 1e-12 relative and accumulates over the steps).
"""
import sys

import numpy as np
import pytest

import oracle
import workloads
from tests._sides import gpu_values, onsite_values, rel, same_pattern

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_0911_3584_amd as lsdm  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).to(DEV)


def _si64():
    c = workloads.workload("si64_rl12")
    s, rS, rH, rL = c["system"], c["rS"], c["rH"], c["rL"]
    lnv = lsdm.LNV(lsdm.System.from_workload(s), rS, rH, rL)
    v = {w: gpu_values(lnv.patterns[w], s, w, rS=rS) for w in "LSH"}
    inp = oracle.make_inputs(s, rS, rH, rL)
    for w in "LSH":
        assert same_pattern(lnv.patterns[w], inp[w].pattern)
        np.testing.assert_array_equal(v[w], inp[w].val)
    return s, (rS, rH, rL), lnv, v, inp


def test_shift_and_electron_number():
    s, (rS, rH, rL), lnv, v, inp = _si64()
    say(f"[shift/electrons] si64 atoms={s.n}")
    Hm_ref = oracle.shift(inp["H"], inp["S"], 1.0)
    Hm = lnv.shift(T(v["S"]), T(v["H"]), mu=1.0).cpu().numpy()
    np.testing.assert_allclose(Hm, Hm_ref.val, rtol=0, atol=2.3e-16 * np.abs(v["S"]).max())
    only_s = lnv.shift(T(v["S"]), mu=-1.0).cpu().numpy()
    np.testing.assert_array_equal(only_s, oracle.shift(oracle.zeros(inp["H"].pattern), inp["S"], -1.0).val)
    N_ref = oracle.electron_number(inp["L"], inp["S"], rS, rH, rL)
    Sh = oracle.shift(oracle.zeros(inp["H"].pattern), inp["S"], -1.0)
    G_ref = oracle.lnv_gradient(inp["L"], inp["S"], Sh, rS, rH, rL)
    N, G = lnv.electrons(T(v["L"]), T(v["S"]), grad=True)
    assert abs(N.item() - N_ref) <= 1e-12 * abs(N_ref), (N.item(), N_ref)
    assert rel(G.cpu().numpy(), G_ref.val) <= 1e-12
    assert lnv.electrons(T(v["L"]), T(v["S"])).item() == N.item()


@pytest.mark.parametrize("h", [1.0, 0.25])
def test_line_coefficients(h):
    s, (rS, rH, rL), lnv, v, inp = _si64()
    say(f"[line] si64 h={h}")
    pL = inp["L"].pattern
    D = 0.05 * workloads.fd_direction(pL.nval, seed=3)          # no symmetry imposed
    c_ref = oracle.lnv_line_coeffs(inp["L"], oracle.Matrix(pL, D), inp["S"], inp["H"], rS, rH, rL)
    c = lnv.line(T(v["L"]), T(D), T(v["S"]), T(v["H"]), h=h)
    scale = np.sum(np.abs(c_ref) * h ** np.arange(4))
    for k in range(4):
        assert abs(c[k] - c_ref[k]) * h ** k <= 1e-11 * scale, (k, c, c_ref)


def test_minimise_grand_potential_si64():
    s, (rS, rH, rL), lnv, v, inp = _si64()
    say(f"[minimise fp64] si64 mu=1")
    Hm = lnv.shift(T(v["S"]), T(v["H"]), mu=1.0)
    L = T(v["L"]).clone()
    Es, gs = lnv.minimise(L, T(v["S"]), Hm, max_iter=8, gtol=0.0)
    Lf, Er, gr = oracle.lnv_minimise(inp["L"], inp["S"], oracle.shift(inp["H"], inp["S"], 1.0), rS, rH, rL,
                                     max_iter=8)
    say("E gpu", Es, "\nE ref", Er, "\n|g| gpu", gs, "\n|g| ref", gr)
    assert Es.size == Er.size == 9
    np.testing.assert_allclose(Es, Er, rtol=1e-9)
    np.testing.assert_allclose(gs, gr, rtol=1e-6)
    assert rel(L.cpu().numpy(), Lf.val) <= 1e-7
    assert np.all(np.diff(Es) < 0)


@pytest.mark.parametrize("prec", ["fp32", "fp32_rc"])
def test_minimise_reduced_precision_tracks_fp64(prec):
    """Other precision modes run the same search; their energies stay within the
    modes' own error of the FP64 path (energy errors near 1e-7 relative on
    this cell)."""
    s, (rS, rH, rL), lnv, v, inp = _si64()
    Hm = lnv.shift(T(v["S"]), T(v["H"]), mu=1.0)
    E64, _ = lnv.minimise(T(v["L"]).clone(), T(v["S"]), Hm, max_iter=6, gtol=0.0)
    E, _ = lnv.minimise(T(v["L"]).clone(), T(v["S"]), Hm, max_iter=6, gtol=0.0, prec=prec)
    say(prec, E, E64)
    np.testing.assert_allclose(E, E64, rtol=1e-6)


def test_minimise_onsite_closed_form():
    """On-site blocks only (ranges below the nearest-neighbour distance), S = I,
    levels (-1, -0.5, 0.3, 1) per atom, mu = 0.5: the minimum fills the three
    levels below mu, E - mu N_e = -5.4 and N_e = 6 per atom."""
    s = workloads.diamond(2, jitter=0.05, seed=2)
    lnv = lsdm.LNV(lsdm.System.from_workload(s), 4.0, 4.0, 4.0)
    for w in "LSH":
        rp, col, img, off = lnv.patterns[w].export()
        assert np.array_equal(col, np.arange(s.n)) and np.array_equal(rp, np.arange(s.n + 1))
    v = onsite_values(s.n)
    say(f"[minimise fp64] on-site closed form atoms={s.n}")
    S = T(v["S"])
    Hm = lnv.shift(S, T(v["H"]), mu=0.5)
    L = T(v["L"]).clone()
    Es, gs = lnv.minimise(L, S, Hm, max_iter=80, gtol=1e-6)
    say("E", Es[-3:], "|g|", gs[-3:])
    assert gs[-1] <= 1e-6
    assert abs(Es[-1] + 5.4 * s.n) <= 1e-10 * 5.4 * s.n
    assert np.all(np.diff(Es) <= 1e-12 * 5.4 * s.n)
    assert abs(lnv.electrons(L, S).item() - 6.0 * s.n) <= 1e-5 * s.n


def test_minimise_symmetric_mode_matches():
    s, (rS, rH, rL), lnv, v, inp = _si64()
    sym = lsdm.LNV(lsdm.System.from_workload(s), rS, rH, rL, symmetric=True)
    Hm = lnv.shift(T(v["S"]), T(v["H"]), mu=1.0)
    E1, g1 = lnv.minimise(T(v["L"]).clone(), T(v["S"]), Hm, max_iter=6, gtol=0.0)
    E2, g2 = sym.minimise(T(v["L"]).clone(), T(v["S"]), sym.shift(T(v["S"]), T(v["H"]), mu=1.0), max_iter=6, gtol=0.0)
    np.testing.assert_allclose(E2, E1, rtol=1e-10)
    np.testing.assert_allclose(g2, g1, rtol=1e-6)


# ---------------------------------------------------------------------------
# McWeeny purification step
# ---------------------------------------------------------------------------
PURIFY_CASES = {
    "si64_rl12": lambda: (workloads.workload("si64_rl12")["system"], 8.0, 12.0, 12.0),     # the chain's LSL serves
    "si64_jitter_rl16": lambda: (workloads.diamond(2, jitter=0.1, seed=7), 8.0, 12.0, 16.0),  # own LSL pattern (rH < rL)
    "mixed_box_13_5": lambda: (workloads.random_box(300, 17.5, 240, 13, 5, seed=2), 6.0, 8.0, 8.0),
    "si_slab_h_2x2x2": lambda: (workloads.si_slab((2, 2, 2)), 8.0, 12.0, 16.0),
}


@pytest.mark.parametrize("symmetric", [False, True], ids=["full", "sym"])
@pytest.mark.parametrize("name", list(PURIFY_CASES))
def test_purify_parity(name, symmetric):
    s, rS, rH, rL = PURIFY_CASES[name]()
    say(f"[purify] {name} atoms={s.n} symmetric={symmetric}")
    lnv = lsdm.LNV(lsdm.System.from_workload(s), rS, rH, rL, symmetric=symmetric)
    v = {w: gpu_values(lnv.patterns[w], s, w, rS=rS) for w in "LS"}
    inp = oracle.make_inputs(s, rS, rH, rL)
    ref = oracle.mcweeny(inp["L"], inp["S"], rS, rL)
    out = lnv.purify(T(v["L"]), T(v["S"])).cpu().numpy()
    assert rel(out, ref.val) <= 1e-12, rel(out, ref.val)
    out32 = lnv.purify(T(v["L"]), T(v["S"]), prec="fp32").cpu().numpy()
    assert rel(out32, ref.val) <= 1e-5, rel(out32, ref.val)


def test_purify_iterates_and_electron_count():
    """Three McWeeny steps on the 64-atom cell against the oracle's, with the
    electron number of each iterate."""
    s, (rS, rH, rL), lnv, v, inp = _si64()
    L = T(v["L"])
    Lr = inp["L"]
    for it in range(3):
        L = lnv.purify(L, T(v["S"]))
        Lr = oracle.mcweeny(Lr, inp["S"], rS, rL)
        assert rel(L.cpu().numpy(), Lr.val) <= 1e-11, it
        N = lnv.electrons(L, T(v["S"])).item()
        Nr = oracle.electron_number(Lr, inp["S"], rS, rH, rL)
        assert abs(N - Nr) <= 1e-11 * abs(Nr), (it, N, Nr)
        say(f"    step {it}: N_e = {N:.10f}")
    with pytest.raises(lsdm.LsdmError):
        lnv.purify(L, T(v["S"]), prec="bf16")
