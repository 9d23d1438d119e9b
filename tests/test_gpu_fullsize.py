"""GPU checks at the full workload sizes and in reduced precision.

At full size the oracle computes sampled rows one by one through their
dependency cones (K rows and dE/dL rows); the energy of a perfect crystal is
checked through extensivity against the oracle's 64-atom cell; dE/dL is checked
against exact Richardson differences of the GPU's own energy (E is a cubic
polynomial of L).  Reduced-precision chains state their energy error per atom
against FP64.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads
from tests._sides import gpu_values, rel, same_pattern

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


def setup(s, rS, rH, rL, symmetric=False):
    lnv = lsdm.LNV(lsdm.System.from_workload(s), rS, rH, rL, symmetric=symmetric)
    v = {w: T(gpu_values(lnv.patterns[w], s, w, rS=rS)) for w in "LSH"}
    return lnv, v


def row_block(pattern_gpu, vec, i):
    rp, col, img, off = pattern_gpu.export()
    nfn = pattern_gpu.system.nfn
    lo = off[rp[i]]
    last = rp[i + 1] - 1
    hi = off[last] + nfn[i] * nfn[col[last]]
    return vec[lo:hi]


def check_rows(lnv, s, v, rS, rH, rL, rows, grad_rows=None, K=None, G=None):
    """K rows (and dE/dL rows) against the oracle's dependency cones."""
    ec = oracle.energy_cone(s, rS, rH, rL, rows)
    lrows = ec["L"] if grad_rows is None else np.union1d(ec["L"], oracle.gradient_cone(s, rS, rH, rL, grad_rows)["L"])
    srows = ec["S"] if grad_rows is None else np.union1d(ec["S"], oracle.gradient_cone(s, rS, rH, rL, grad_rows)["S"])
    hrows = np.union1d(ec["H"], rows) if grad_rows is None else np.union1d(
        np.union1d(ec["H"], rows), oracle.gradient_cone(s, rS, rH, rL, grad_rows)["H"])
    inp = oracle.make_inputs(s, rS, rH, rL, rows_L=lrows, rows_S=srows, rows_H=hrows)
    ref = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], rS, rH, rL, rows=rows)
    Kh = K.cpu().numpy()
    for i in rows:
        got = row_block(lnv.patterns["H"], Kh, i)
        assert rel(got, oracle.row_slice(ref["K"], i)) <= 1e-12, i
    if grad_rows is not None:
        Gr = oracle.lnv_gradient(inp["L"], inp["S"], inp["H"], rS, rH, rL, rows=grad_rows)
        Gh = G.cpu().numpy()
        for i in grad_rows:
            assert rel(row_block(lnv.patterns["L"], Gh, i), oracle.row_slice(Gr, i)) <= 1e-12, i
    return ref


def fd_check(lnv, v, G, n_blocks=20, h=0.25, prec="fp64", seed=0, tol=1e-7):
    """Richardson-extrapolated central differences of E along single stored L
    blocks (exact for a cubic up to rounding) against <dE/dL, direction>."""
    p = lnv.patterns["L"]
    rp, col, img, off = p.export()
    nfn = p.system.nfn
    rows = np.repeat(np.arange(p.system.n), np.diff(rp))
    blocks = workloads.fd_blocks(p.n_blocks, n_blocks, seed=seed)
    dirs = workloads.fd_direction(p.n_values, seed=seed)
    Lh = v["L"].clone()
    g = G.cpu().numpy()
    worst = 0.0
    for b in blocks:
        sz = int(nfn[rows[b]] * nfn[col[b]])
        d = np.zeros(p.n_values)
        d[off[b]:off[b] + sz] = dirs[off[b]:off[b] + sz]
        dt = T(d)

        def E(t):
            Lh.copy_(v["L"]).add_(dt, alpha=t)
            return lnv.energy(Lh, v["S"], v["H"], prec=prec).item()
        d1 = (E(h) - E(-h)) / (2 * h)
        d2 = (E(h / 2) - E(-h / 2)) / h
        fd = (4 * d2 - d1) / 3
        an = float(np.dot(g, d))
        err = abs(fd - an) / max(1.0, abs(an))
        worst = max(worst, err)
        assert err <= tol, (int(b), fd, an)
    return worst


# ---------------------------------------------------------------------------
# reduced precision on small chains
# ---------------------------------------------------------------------------
SMALL = {
    "si64_rl12": lambda: (workloads.workload("si64_rl12")["system"], 8.0, 12.0, 12.0),
    "mixed_box_13_5": lambda: (workloads.random_box(300, 17.5, 240, 13, 5, seed=2), 6.0, 8.0, 8.0),
    "si_slab_h_2x2x2": lambda: (workloads.si_slab((2, 2, 2)), 8.0, 12.0, 16.0),
}
# regression guard: about ten times the relative error observed when these
# chains were first measured (the correctness criterion is the a-priori bound
# below; this keeps the errors where they were measured)
CHAIN_TOL = {"fp32": (1e-5, 1e-4), "bf16": (3e-2, 1.5e-1), "fp32_rc": (1e-8, 1e-6)}
BOUND_CASES = ("si64_rl12", "si_slab_h_2x2x2")


@pytest.mark.parametrize("symmetric", [False, True], ids=["full", "sym"])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp32_rc"])
@pytest.mark.parametrize("name", list(SMALL))
def test_lnv_reduced_precision(prec, name, symmetric):
    """E and dE/dL against the oracle, within the first-order a-priori bound of
    the chain as the mode computes it (tests/_bounds.py: operands rounded with
    the mode's unit roundoff, n-term FP32 sums, errors carried from product to
    product), E as a whole and dE/dL element by element; a factor 2 covers the
    second-order terms the bound drops.  The bound needs a dozen oracle
    products of absolute values; for the 300-atom box with 13-function atoms
    they take minutes, so that case keeps the regression guard alone."""
    from tests._bounds import chain_error_bounds
    s, rS, rH, rL = SMALL[name]()
    say(f"[reduced] {name} {prec} symmetric={symmetric}")
    lnv, v = setup(s, rS, rH, rL, symmetric=symmetric)
    inp = oracle.make_inputs(s, rS, rH, rL)
    ref = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    Gref = oracle.lnv_gradient(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    E, G = lnv.energy_grad(v["L"], v["S"], v["H"], prec=prec)
    G = G.cpu().numpy()
    dE = abs(E.item() - ref["E"])
    eE = dE / abs(ref["E"])
    eG = rel(G, Gref.val)
    say(f"    E rel err {eE:.3e} ({1e6 * dE / s.n:.4f} uHa/atom), dE/dL rel err {eG:.3e}")
    if name in BOUND_CASES:
        bE, bG = chain_error_bounds(inp, rS, rH, rL, "bf16" if prec == "bf16" else "fp32", symmetric)
        dG = np.abs(G - Gref.val)
        say(f"    E error {dE / bE:.2e} of its bound, worst dE/dL element {np.max(dG / (bG + 1e-300)):.2e} of its bound")
        assert dE <= 2 * bE
        assert np.all(dG <= 2 * bG + 1e-12 * np.abs(Gref.val) + 1e-300)
    assert eE <= CHAIN_TOL[prec][0] and eG <= CHAIN_TOL[prec][1]


# ---------------------------------------------------------------------------
# full sizes
# ---------------------------------------------------------------------------
def test_si13824_jitter_fp64_rows_and_fd():
    c = workloads.workload("si13824_jitter_rl16")
    s = c["system"]
    rS, rH, rL = c["rS"], c["rH"], c["rL"]
    say(f"[si13824] {s.n} atoms, jittered, RL16: setup")
    lnv, v = setup(s, rS, rH, rL)
    E, K = lnv.energy(v["L"], v["S"], v["H"], want_K=True)
    _, G = lnv.energy_grad(v["L"], v["S"], v["H"])
    say("[si13824] oracle rows")
    rows = np.array([0, 6911, 13823])
    check_rows(lnv, s, v, rS, rH, rL, rows, grad_rows=np.array([5000]), K=K, G=G)
    # E equals the sum of the per-row contributions 2 <K_i, H_i> (FP64 on the host)
    Hh = v["H"].cpu().numpy()
    assert abs(float(np.sum(K.cpu().numpy() * Hh)) * 2 - E.item()) <= 1e-12 * abs(E.item())
    say("[si13824] finite differences on 20 L blocks")
    worst = fd_check(lnv, v, G, n_blocks=20)
    say(f"    worst FD relative deviation {worst:.2e}")


def _fd_exact(lnv, v, blocks, dirs, h=0.25):
    """Richardson-extrapolated central differences of the FP64 energy along
    single stored L blocks: exact derivatives up to rounding (E is a cubic
    polynomial of L)."""
    p = lnv.patterns["L"]
    rp, col, img, off = p.export()
    nfn = p.system.nfn
    rows = np.repeat(np.arange(p.system.n), np.diff(rp))
    Lh = v["L"].clone()
    out = []
    for b in blocks:
        sz = int(nfn[rows[b]] * nfn[col[b]])
        d = np.zeros(p.n_values)
        d[off[b]:off[b] + sz] = dirs[off[b]:off[b] + sz]
        dt = T(d)

        def E(t):
            Lh.copy_(v["L"]).add_(dt, alpha=t)
            return lnv.energy(Lh, v["S"], v["H"], prec="fp64").item()
        d1 = (E(h) - E(-h)) / (2 * h)
        d2 = (E(h / 2) - E(-h / 2)) / h
        out.append((d, (4 * d2 - d1) / 3))
    return out


def test_si13824_autograd_fp64_fp32_fd():
    """The 13,824-atom jittered cell through the autograd.Function in FP64 and
    FP32: dE/dL from backward() against exact finite differences on 20 seeded L
    blocks.  FP64 is held to 1e-7 of max(1, |<G, d>|) (the differences'
    own rounding).  FP32: every product rounds its inputs to FP32 and sums n
    terms in FP32; with random rounding the error of such a sum stays below
    lambda sqrt(n) u |a||b| with high probability (Higham & Mary, SIAM J. Sci.
    Comput. 41, 2019: lambda = 6 gives a failure probability below 1e-15),
    and the gradient passes through at most `levels` products, so the
    projection of the FP32 gradient on a direction is allowed
    levels * lambda sqrt(n) u32 of max(1, |<G, d>|), n the longest inner sum."""
    c = workloads.workload("si13824_jitter_rl16")
    s = c["system"]
    rS, rH, rL = c["rS"], c["rH"], c["rL"]
    say(f"[si13824 autograd] {s.n} atoms: setup")
    lnv, v = setup(s, rS, rH, rL)
    p = lnv.patterns["L"]
    blocks = workloads.fd_blocks(p.n_blocks, 20, seed=0)
    dirs = workloads.fd_direction(p.n_values, seed=0)
    say("[si13824 autograd] exact finite differences (FP64 energies)")
    fds = _fd_exact(lnv, v, blocks, dirs)
    # longest inner sum of the chain: 4 functions x the most blocks in a row of M
    n_inner = 4 * int(np.diff(lnv.patterns["M"].export()[0]).max())
    levels, lam, u32 = 5, 6.0, 2.0 ** -24
    tol = {"fp64": 1e-7, "fp32": levels * lam * np.sqrt(n_inner) * u32}
    for prec in ("fp64", "fp32"):
        L = v["L"].clone().requires_grad_(True)
        E = lsdm.LNVEnergy.apply(L, v["S"], v["H"], lnv, prec)
        E.backward()
        g = L.grad.cpu().numpy()
        worst = 0.0
        for d, fd in fds:
            an = float(np.dot(g, d))
            err = abs(fd - an) / max(1.0, abs(an))
            worst = max(worst, err)
            assert err <= tol[prec], (prec, fd, an, err, tol[prec])
        say(f"    {prec}: E = {E.item():.10f}, worst |FD - <dE/dL, d>| / max(1, |.|) = {worst:.2e} "
            f"(allowed {tol[prec]:.1e})")


@pytest.mark.parametrize("symmetric", [False, True], ids=["full", "sym"])
def test_si32768_extensive_energy_rows_and_modes(symmetric):
    c = workloads.workload("si32768_rl16")
    s = c["system"]
    rS, rH, rL = c["rS"], c["rH"], c["rL"]
    say(f"[si32768] {s.n} atoms, RL16, symmetric={symmetric}: setup")
    lnv, v = setup(s, rS, rH, rL, symmetric=symmetric)
    E, K = lnv.energy(v["L"], v["S"], v["H"], want_K=True)
    _, G = lnv.energy_grad(v["L"], v["S"], v["H"])
    # translation-class values make E extensive: the 64-atom cell fixes E/N
    small = workloads.diamond(2)
    inp = oracle.make_inputs(small, rS, rH, rL)
    e_small = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], rS, rH, rL)["E"] / small.n
    assert abs(E.item() / s.n - e_small) <= 1e-12 * abs(e_small), (E.item() / s.n, e_small)
    say("[si32768] oracle rows")
    check_rows(lnv, s, v, rS, rH, rL, np.array([0, 12345, 32767]), grad_rows=np.array([20000]), K=K, G=G)
    for prec in ("fp32", "bf16", "fp32_rc"):
        Em, Gm = lnv.energy_grad(v["L"], v["S"], v["H"], prec=prec)
        eE = abs(Em.item() - E.item()) / abs(E.item())
        eG = rel(Gm.cpu().numpy(), G.cpu().numpy())
        say(f"    {prec}: E rel err {eE:.3e} = {1e6 * abs(Em.item() - E.item()) / s.n:.4f} uHa/atom; dE/dL rel {eG:.3e}")
        assert eE <= CHAIN_TOL[prec][0] and eG <= CHAIN_TOL[prec][1]


def test_si32768_pair_keys_rows():
    """The 32,768-atom cell with per-pair value keys (no translation symmetry in
    the values): K and dE/dL rows against the oracle's dependency cones, in
    symmetric mode (the bench's default)."""
    c = workloads.workload("si32768_rl16")
    s = workloads.diamond(16, key_mode="pair")
    rS, rH, rL = c["rS"], c["rH"], c["rL"]
    say(f"[si32768 pair keys] {s.n} atoms: setup")
    lnv, v = setup(s, rS, rH, rL, symmetric=True)
    E, K = lnv.energy(v["L"], v["S"], v["H"], want_K=True)
    _, G = lnv.energy_grad(v["L"], v["S"], v["H"])
    say("[si32768 pair keys] oracle rows")
    check_rows(lnv, s, v, rS, rH, rL, np.array([1, 16383, 32766]), grad_rows=np.array([777, 31000]), K=K, G=G)


def test_mixed8000_blocks_rows_and_fd():
    c = workloads.workload("mixed8000_rl14")
    s = c["system"]
    rS, rH, rL = c["rS"], c["rH"], c["rL"]
    say(f"[mixed8000] {s.n} atoms, 13/5 functions: setup")
    lnv, v = setup(s, rS, rH, rL)
    E, K = lnv.energy(v["L"], v["S"], v["H"], want_K=True)
    _, G = lnv.energy_grad(v["L"], v["S"], v["H"])
    say("[mixed8000] oracle rows")
    check_rows(lnv, s, v, rS, rH, rL, np.array([0, 4000, 7999]), K=K)
    say("[mixed8000] finite differences on 8 L blocks")
    fd_check(lnv, v, G, n_blocks=8, seed=5)
    Em, Gm = lnv.energy_grad(v["L"], v["S"], v["H"], prec="fp32")
    eE = abs(Em.item() - E.item()) / abs(E.item())
    eG = rel(Gm.cpu().numpy(), G.cpu().numpy())
    say(f"    fp32: E rel err {eE:.3e} = {1e6 * abs(Em.item() - E.item()) / s.n:.4f} uHa/atom; dE/dL rel {eG:.3e}")
    assert eE <= CHAIN_TOL["fp32"][0] and eG <= CHAIN_TOL["fp32"][1]


def test_slab18432_rows_and_fd():
    """H-terminated (001) slab: surface and hydrogen rows have fewer neighbours
    than bulk rows; K and dE/dL rows against the oracle at full size."""
    c = workloads.workload("si001slab18432_h_rl16")
    s = c["system"]
    rS, rH, rL = c["rS"], c["rH"], c["rL"]
    say(f"[slab18432] {s.n} atoms, slab with H: setup")
    lnv, v = setup(s, rS, rH, rL)
    E, K = lnv.energy(v["L"], v["S"], v["H"], want_K=True)
    _, G = lnv.energy_grad(v["L"], v["S"], v["H"])
    si = np.where(s.nfn == 4)[0]
    h = np.where(s.nfn == 1)[0]
    z = s.xyz[:, 2]
    mid = si[np.argmin(np.abs(z[si] - np.median(z[si])))]
    rows = np.array(sorted({int(si[np.argmax(z[si])]), int(mid), int(h[0]), int(h[-1])}))
    grad_rows = np.array(sorted({int(si[np.argmin(z[si])]), int(h[7])}))
    say(f"[slab18432] oracle rows {rows.tolist()} grad rows {grad_rows.tolist()}")
    check_rows(lnv, s, v, rS, rH, rL, rows, grad_rows=grad_rows, K=K, G=G)
    say("[slab18432] finite differences on 10 L blocks")
    fd_check(lnv, v, G, n_blocks=10, seed=6)
    Em, _ = lnv.energy_grad(v["L"], v["S"], v["H"], prec="fp32")
    eE = abs(Em.item() - E.item()) / abs(E.item())
    say(f"    fp32: E rel err {eE:.3e} = {1e6 * abs(Em.item() - E.item()) / s.n:.4f} uHa/atom")
    assert eE <= CHAIN_TOL["fp32"][0]
