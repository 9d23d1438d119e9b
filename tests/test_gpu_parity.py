"""GPU parity: the HIP path against the FP64 oracle on the same seeded inputs.

FP64 bar (stated target): relative error <= 1e-12 for E, and in Frobenius norm
for every product, K and dE/dL.  FP32, BF16 and FP32-residual products are
held to the a-priori bound of the rounding of inputs and accumulation
(test_product_parity); whole chains in those modes are in test_gpu_fullsize.py.
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
TOL64 = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).to(DEV)


# ---------------------------------------------------------------------------
# single truncated products
# ---------------------------------------------------------------------------
PRODUCT_CASES = [
    # name, system factory, (rA, rB, rC), transA, transB, alpha, beta
    ("si64_lossless", lambda: workloads.diamond(2), (12.0, 8.0, 20.0), 0, 0, 1.0, 0.0),
    ("si64_lossy", lambda: workloads.diamond(2), (20.0, 12.0, 24.0), 0, 0, 1.0, 0.0),
    ("si64_small_out", lambda: workloads.diamond(2), (24.0, 32.0, 12.0), 0, 0, 1.0, 0.0),
    ("si64_transA", lambda: workloads.diamond(2), (20.0, 12.0, 24.0), 1, 0, -4.0, 0.0),
    ("si64_transB", lambda: workloads.diamond(2), (12.0, 20.0, 16.0), 0, 1, 1.0, 0.0),
    ("si64_beta", lambda: workloads.diamond(2), (12.0, 12.0, 16.0), 0, 0, 0.5, 2.0),
    ("si8_images", lambda: workloads.diamond(1), (12.0, 8.0, 14.0), 0, 0, 1.0, 0.0),
    ("jitter_rl16", lambda: workloads.diamond(2, jitter=0.1, seed=5), (16.0, 8.0, 24.0), 0, 0, 1.0, 0.0),
    ("mixed_box", lambda: workloads.random_box(150, 15.0, 120, 13, 5, seed=3), (7.0, 6.0, 10.0), 0, 0, 1.0, 0.0),
    ("mixed_box_tA", lambda: workloads.random_box(150, 15.0, 120, 13, 5, seed=3), (7.0, 6.0, 10.0), 1, 0, 1.0, 1.0),
    ("open_ragged", lambda: workloads.random_cluster(61, 12.0, nfn=np.arange(61) % 7 + 1, seed=4), (6.0, 5.0, 7.0), 0, 0, 1.0, 0.0),
    ("empty_output", lambda: workloads.diamond(1), (4.0, 4.0, 0.0), 0, 0, 1.0, 0.0),
]


def _rand(p, seed):
    return np.random.default_rng(seed).normal(size=p.nval)


def _offsite(p, v):
    """Values with the on-site blocks (i, i, image 0) set to zero."""
    v = v.copy()
    bi, bj, bim = p.keys()
    nfn = np.asarray(p.system.nfn, np.int64)
    for b in np.where((bi == bj) & np.all(bim == 0, axis=1))[0]:
        v[p.off[b]:p.off[b] + nfn[bi[b]] * nfn[bj[b]]] = 0.0
    return v


@pytest.mark.parametrize("case", PRODUCT_CASES, ids=[c[0] for c in PRODUCT_CASES])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "fp32_rc"])
def test_product_parity(case, prec):
    name, mk, (rA, rB, rC), tA, tB, alpha, beta = case
    say(f"[product] {name} prec={prec} ranges={rA},{rB},{rC} tA={tA} tB={tB}")
    s = mk()
    gs = lsdm.System.from_workload(s)
    gA, gB, gC = lsdm.Pattern(gs, rA), lsdm.Pattern(gs, rB), lsdm.Pattern(gs, rC)
    oA, oB, oC = oracle.pattern(s, rA), oracle.pattern(s, rB), oracle.pattern(s, rC)
    assert same_pattern(gA, oA) and same_pattern(gB, oB) and same_pattern(gC, oC)
    a, b, c0 = _rand(oA, 1), _rand(oB, 2), _rand(oC, 3)
    ref = oracle.multiply_op(oracle.Matrix(oA, a), tA, oracle.Matrix(oB, b), tB, oC).val * alpha + beta * c0
    plan = lsdm.Plan(gA, tA, gB, tB, gC)
    C = T(c0)
    lsdm.multiply(plan, T(a), T(b), C, alpha=alpha, beta=beta, prec=prec)
    got = C.cpu().numpy()
    if prec == "fp64":
        assert rel(got, ref) <= TOL64, rel(got, ref)
    else:
        # a-priori bound (Higham, Accuracy and Stability of Numerical Algorithms,
        # sec. 3.1): inputs rounded with unit roundoff ui (relative error of a
        # product of two rounded inputs <= 2 ui + ui^2), then n-term FP32
        # accumulation, |fl(sum ab) - sum ab| <= (2 ui + ui^2 + gamma_n) sum |a||b|
        if prec == "fp32_rc":
            # only the off-site parts are multiplied in FP32; the on-site (atom
            # diagonal, image 0) terms are exact FP64 scalings
            a, b = _offsite(oA, a), _offsite(oB, b)
        absref = oracle.multiply_op(oracle.Matrix(oA, np.abs(a)), tA, oracle.Matrix(oB, np.abs(b)), tB, oC).val
        n = 4 * int(np.diff(oA.row_ptr).max()) * 4 + 8   # summands per output element, generously
        u = 2.0 ** -24
        ui = 2.0 ** -8 if prec == "bf16" else u
        gam = (n + 2) * u / (1 - (n + 2) * u)
        bound = abs(alpha) * (2 * ui + ui * ui + gam) * absref + 4 * u * np.abs(beta * c0) + 4 * u * np.abs(ref) + 1e-30
        assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / (bound + 1e-300))


def test_product_adjoint_and_dot():
    s = workloads.random_box(150, 15.0, 120, 13, 5, seed=8)
    say("[adjoint] mixed_box")
    gs = lsdm.System.from_workload(s)
    rA, rB, rC = 7.0, 6.0, 9.0
    gA, gB, gC = lsdm.Pattern(gs, rA), lsdm.Pattern(gs, rB), lsdm.Pattern(gs, rC)
    oA, oB, oC = oracle.pattern(s, rA), oracle.pattern(s, rB), oracle.pattern(s, rC)
    for tA, tB in ((0, 0), (1, 0), (0, 1), (1, 1)):
        a, b, cb = _rand(oA, 1), _rand(oB, 2), _rand(oC, 3)
        ab0, bb0 = _rand(oA, 4), _rand(oB, 5)
        Ab, Bb = oracle.multiply_adjoint(oracle.Matrix(oA, a), tA, oracle.Matrix(oB, b), tB, oracle.Matrix(oC, cb))
        plan = lsdm.Plan(gA, tA, gB, tB, gC)
        gAb, gBb = T(ab0), T(bb0)
        lsdm.multiply_adjoint(plan, T(cb), T(a), T(b), gAb, gBb)
        assert rel(gAb.cpu().numpy(), Ab.val + ab0) <= TOL64
        assert rel(gBb.cpu().numpy(), Bb.val + bb0) <= TOL64
    a, b = _rand(oA, 6), _rand(oA, 7)
    d = lsdm.dot(gA, T(a), T(b)).item()
    assert abs(d - oracle.dot(a, b)) <= 1e-13 * np.sum(np.abs(a * b))


def test_dot_calls_queued_back_to_back():
    """lsdm_dot returns without waiting and reuses the pattern's partial
    sums: dots queued one after another on a stream each give their own
    oracle value."""
    s = workloads.diamond(2, jitter=0.1, seed=4)
    gs = lsdm.System.from_workload(s)
    gp, op = lsdm.Pattern(gs, 12.0), oracle.pattern(s, 12.0)
    pairs = [(_rand(op, 10 + 2 * k), _rand(op, 11 + 2 * k)) for k in range(4)]
    outs = [lsdm.dot(gp, T(a), T(b)) for a, b in pairs]
    for (a, b), o in zip(pairs, outs):
        assert abs(o.item() - oracle.dot(a, b)) <= 1e-13 * np.sum(np.abs(a * b))


# ---------------------------------------------------------------------------
# the LNV chain
# ---------------------------------------------------------------------------
def _chain_setup(s, rS, rH, rL, seed=0, symmetric=False):
    gs = lsdm.System.from_workload(s)
    lnv = lsdm.LNV(gs, rS, rH, rL, symmetric=symmetric)
    p = lnv.patterns
    vals = {w: gpu_values(p[w], s, w, seed=seed, rS=rS) for w in "LSH"}
    return lnv, vals


CHAIN_CASES = {
    "si64_rl12": lambda: (workloads.workload("si64_rl12")["system"], 8.0, 12.0, 12.0),
    "si8_cell_images": lambda: (workloads.diamond(1), 8.0, 12.0, 12.0),
    "si64_jitter_rl16": lambda: (workloads.diamond(2, jitter=0.1, seed=7), 8.0, 12.0, 16.0),
    "mixed_box_13_5": lambda: (workloads.random_box(300, 17.5, 240, 13, 5, seed=2), 6.0, 8.0, 8.0),
    "open_cluster_ragged": lambda: (workloads.random_cluster(90, 14.0, nfn=np.arange(90) % 5 + 1, seed=9), 5.0, 6.0, 6.5),
    "si_slab_h_2x2x2": lambda: (workloads.si_slab((2, 2, 2)), 8.0, 12.0, 16.0),
    # H's range beyond that of LSL (rH > 2 rL + rS): K = -2P on the far H blocks
    "si64_h_beyond_lsl": lambda: (workloads.diamond(2, jitter=0.1, seed=3), 4.5, 14.0, 4.6),
}


@pytest.mark.parametrize("symmetric", [False, True], ids=["full", "sym"])
@pytest.mark.parametrize("name", list(CHAIN_CASES))
def test_lnv_energy_grad_fp64(name, symmetric):
    s, rS, rH, rL = CHAIN_CASES[name]()
    say(f"[lnv fp64] {name} atoms={s.n} symmetric={symmetric}")
    lnv, v = _chain_setup(s, rS, rH, rL, symmetric=symmetric)
    inp = oracle.make_inputs(s, rS, rH, rL)
    for w in "LSH":
        assert same_pattern(lnv.patterns[w], inp[w].pattern)
        np.testing.assert_array_equal(v[w], inp[w].val)
    ref = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    G_ref = oracle.lnv_gradient(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    E, K = lnv.energy(T(v["L"]), T(v["S"]), T(v["H"]), want_K=True)
    assert abs(E.item() - ref["E"]) <= TOL64 * abs(ref["E"]), (E.item(), ref["E"])
    assert rel(K.cpu().numpy(), ref["K"].val) <= TOL64
    E2, G = lnv.energy_grad(T(v["L"]), T(v["S"]), T(v["H"]))
    if symmetric:
        # the energy-and-gradient call forms E without P in symmetric FP64 mode
        # (2 <3 M|_H, H> + <X, Xbar>, the same value): held to the oracle, not
        # to the bits of the energy call
        assert abs(E2.item() - ref["E"]) <= TOL64 * abs(ref["E"]), (E2.item(), ref["E"])
    else:
        assert E2.item() == E.item()
    assert rel(G.cpu().numpy(), G_ref.val) <= TOL64, rel(G.cpu().numpy(), G_ref.val)


@pytest.mark.parametrize("key_mode", ["class", "pair"])
def test_lnv_si4096_fp64(key_mode):
    """4,096 atoms; with per-pair value keys as well, so that no translation
    symmetry of the values can hide a block read from the wrong place."""
    c = workloads.workload("si4096_rl12")
    s = c["system"] if key_mode == "class" else workloads.diamond(8, key_mode="pair")
    say(f"[lnv fp64] si4096 atoms={s.n} keys={key_mode}")
    lnv, v = _chain_setup(s, c["rS"], c["rH"], c["rL"])
    inp = oracle.make_inputs(s, c["rS"], c["rH"], c["rL"])
    for w in "LSH":
        assert same_pattern(lnv.patterns[w], inp[w].pattern)
    ref = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], c["rS"], c["rH"], c["rL"])
    E, K = lnv.energy(T(v["L"]), T(v["S"]), T(v["H"]), want_K=True)
    assert abs(E.item() - ref["E"]) <= TOL64 * abs(ref["E"])
    assert rel(K.cpu().numpy(), ref["K"].val) <= TOL64
    # gradient on sampled rows through the oracle's dependency cone
    rows = np.array([0, 1, 777, 2048, 4095])
    Gr = oracle.lnv_gradient(inp["L"], inp["S"], inp["H"], c["rS"], c["rH"], c["rL"], rows=rows)
    _, G = lnv.energy_grad(T(v["L"]), T(v["S"]), T(v["H"]))
    G = G.cpu().numpy()
    p = inp["L"].pattern
    for i in rows:
        lo, hi = p.off[p.row_ptr[i]], p.off[p.row_ptr[i + 1] - 1] + 16
        assert rel(G[lo:hi], oracle.row_slice(Gr, i)) <= TOL64


def test_lnv_deterministic():
    s, rS, rH, rL = CHAIN_CASES["mixed_box_13_5"]()
    lnv, v = _chain_setup(s, rS, rH, rL)
    out = []
    for _ in range(2):
        E, G = lnv.energy_grad(T(v["L"]), T(v["S"]), T(v["H"]))
        out.append((E.cpu().numpy().copy(), G.cpu().numpy().copy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_symmetric_handle_mode_sequence():
    """One symmetric handle runs every precision mode, the energy-only chain
    and the McWeeny step (whose LSL shares M's workspace here, rH = rL), in
    turn, twice over: each call's second result equals its first bit for
    bit, whatever ran on the shared workspaces in between.  The FP32 and FP64
    chains write M's dropped half from F2's epilogue and rely on the absent
    blocks of its dropped strips holding zeros in their own element type."""
    s, rS, rH, rL = CHAIN_CASES["si64_rl12"]()
    lnv, v = _chain_setup(s, rS, rH, rL, symmetric=True)
    L, S, H = T(v["L"]), T(v["S"]), T(v["H"])
    calls = {
        "fp32": lambda: lnv.energy_grad(L, S, H, prec="fp32"),
        "fp64": lambda: lnv.energy_grad(L, S, H, prec="fp64"),
        "energy64": lambda: lnv.energy(L, S, H, prec="fp64", want_K=True),
        "purify64": lambda: (lnv.purify(L, S, prec="fp64"),),
        "bf16": lambda: lnv.energy_grad(L, S, H, prec="bf16"),
        "energy32": lambda: lnv.energy(L, S, H, prec="fp32", want_K=True),
        "fp32_rc": lambda: lnv.energy_grad(L, S, H, prec="fp32_rc"),
        "purify32": lambda: (lnv.purify(L, S, prec="fp32"),),
    }
    first = {}
    for rep in range(2):
        for name, call in calls.items():
            r = [x.cpu().numpy().copy() for x in call()]
            if rep == 0:
                first[name] = r
            else:
                assert all(np.array_equal(a, b) for a, b in zip(first[name], r)), name
    ref = oracle.lnv_energy(*(oracle.make_inputs(s, rS, rH, rL)[w] for w in "LSH"), rS, rH, rL)["E"]
    assert abs(first["fp64"][0].item() - ref) <= TOL64 * abs(ref)
    assert abs(first["energy64"][0].item() - ref) <= TOL64 * abs(ref)


def test_caller_allocator_serves_every_workspace():
    """With torch's caching allocator set through lsdm_set_allocator, a
    symmetric handle's workspaces (patterns, plans, chain buffers, lazy maps)
    come from it and all go back to it when the handle is destroyed; the
    results equal those of a handle on hipMalloc bit for bit."""
    import gc
    s, rS, rH, rL = CHAIN_CASES["si64_jitter_rl16"]()
    ref, v = _chain_setup(s, rS, rH, rL, symmetric=True)
    L, S, H = T(v["L"]), T(v["S"]), T(v["H"])
    want = {p: [x.cpu().numpy().copy() for x in ref.energy_grad(L, S, H, prec=p)] for p in ("fp64", "fp32", "bf16")}
    live, made = {}, [0]

    def alloc(n):
        ptr = torch.cuda.caching_allocator_alloc(n)
        live[ptr] = n
        made[0] += 1
        return ptr

    def release(ptr):
        assert ptr in live, ptr
        del live[ptr]
        torch.cuda.caching_allocator_delete(ptr)

    lsdm.set_allocator(alloc, release)
    try:
        lnv, _ = _chain_setup(s, rS, rH, rL, symmetric=True)
        for p, w in want.items():
            got = [x.cpu().numpy() for x in lnv.energy_grad(L, S, H, prec=p)]
            assert all(np.array_equal(a, b) for a, b in zip(w, got)), p
        assert made[0] > 0 and live
        torch.cuda.synchronize()
        del lnv
        gc.collect()
        assert not live, f"{len(live)} workspaces not given back"
    finally:
        lsdm.set_allocator()


def test_checkpoint_resume_on_the_device(tmp_path):
    """A handle and values loaded from a checkpoint onto the GPU give the
    saved handle's energy and dE/dL bit for bit."""
    s, rS, rH, rL = CHAIN_CASES["si_slab_h_2x2x2"]()
    lnv, v = _chain_setup(s, rS, rH, rL, symmetric=True)
    L, S, H = T(v["L"]), T(v["S"]), T(v["H"])
    E0, G0 = lnv.energy_grad(L, S, H, prec="fp32")
    path = tmp_path / "run.npz"
    lsdm.save_checkpoint(path, lnv, {"L": L, "S": S, "H": H})
    lnv2, vals = lsdm.load_checkpoint(path, device=DEV)
    E1, G1 = lnv2.energy_grad(vals["L"], vals["S"], vals["H"], prec="fp32")
    assert torch.equal(E0, E1) and torch.equal(G0, G1)


def test_autograd_function():
    s, rS, rH, rL = CHAIN_CASES["si64_jitter_rl16"]()
    lnv, v = _chain_setup(s, rS, rH, rL)
    L = T(v["L"]).requires_grad_(True)
    E = lsdm.LNVEnergy.apply(L, T(v["S"]), T(v["H"]), lnv, "fp64")
    (3.0 * E).backward()
    _, G = lnv.energy_grad(T(v["L"]), T(v["S"]), T(v["H"]))
    assert torch.equal(L.grad, 3.0 * G)


def test_symmetric_mode_flops_and_agreement():
    """The symmetric handle does fewer flops and agrees with the full one; its
    K and dE/dL are exactly symmetric (mirrored halves)."""
    s, rS, rH, rL = CHAIN_CASES["si64_jitter_rl16"]()
    full, v = _chain_setup(s, rS, rH, rL)
    sym, _ = _chain_setup(s, rS, rH, rL, symmetric=True)
    assert sym.info(True)[1] < 0.8 * full.info(True)[1]
    inp = oracle.make_inputs(s, rS, rH, rL)
    for prec in ("fp64", "fp32", "bf16", "fp32_rc"):
        E1, G1 = full.energy_grad(T(v["L"]), T(v["S"]), T(v["H"]), prec=prec)
        E2, G2 = sym.energy_grad(T(v["L"]), T(v["S"]), T(v["H"]), prec=prec)
        # the two handles differ by the rounding of each mode (the mirrored
        # half is computed as the transposed product)
        tE, tG = {"fp64": (1e-13, 1e-12), "fp32": (1e-6, 1e-5), "bf16": (1e-2, 1e-1),
                  "fp32_rc": (1e-11, 1e-7)}[prec]
        assert abs(E1.item() - E2.item()) <= tE * abs(E1.item()), (prec, E1.item(), E2.item())
        assert rel(G2.cpu().numpy(), G1.cpu().numpy()) <= tG, prec
        _assert_mirrored(G2.cpu().numpy(), inp["L"].pattern, tG)
    _, K = sym.energy(T(v["L"]), T(v["S"]), T(v["H"]), want_K=True)
    _assert_mirrored(K.cpu().numpy(), inp["H"].pattern)


def _assert_mirrored(vals, pat, tol=1e-12):
    """Off-site blocks equal their mirrors' transposes exactly; on-site blocks,
    computed whole, are symmetric up to rounding."""
    t = oracle.transpose(oracle.Matrix(pat, vals), pat).val
    rows = pat.rows_of_blocks()
    onsite = np.zeros(vals.size, bool)
    for b in np.where((pat.col == rows) & np.all(np.asarray(pat.img).reshape(-1, 3) == 0, axis=1))[0]:
        n = int(np.sqrt(pat.off[b + 1] - pat.off[b])) if b + 1 < pat.nblocks else int(np.sqrt(pat.nval - pat.off[b]))
        onsite[pat.off[b]:pat.off[b] + n * n] = True
    np.testing.assert_array_equal(vals[~onsite], t[~onsite])
    np.testing.assert_allclose(vals[onsite], t[onsite], rtol=0, atol=tol * np.abs(vals).max())
