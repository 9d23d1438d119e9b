"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test ties one part of the oracle to mathematics or to an independent
computation: integer lattice enumeration, dense numpy algebra on small open
clusters (library matmul), an untruncated scipy.sparse computation on an
unfolded crystal, eigen-decompositions (the McWeeny spectral identity and a
purified density matrix), closed forms, and exact Richardson-extrapolated
finite differences of a cubic.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

import oracle
import workloads
from tests import _dense
from tests._sides import onsite_values, sym_random


# ---------------------------------------------------------------------------
# range patterns: integer enumeration of the diamond lattice
# ---------------------------------------------------------------------------
def diamond_neighbour_count(R, a=10.26, sub_is_odd=False):
    """Atoms of the infinite diamond lattice within R of a site, counted on
    integer coordinates in units of a/4: fcc sites are all-even triples with
    x+y+z = 0 mod 4, the second fcc lattice is all-odd with x+y+z = 3 mod 4
    relative to an fcc site (and x+y+z = 1 mod 4 seen from a second-lattice site)."""
    m = int(np.ceil(4 * R / a)) + 2
    g = np.arange(-m, m + 1)
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    s = x + y + z
    even = (x % 2 == 0) & (y % 2 == 0) & (z % 2 == 0) & (s % 4 == 0)
    odd = (x % 2 != 0) & (y % 2 != 0) & (z % 2 != 0) & (s % 4 == (1 if sub_is_odd else 3))
    site = even | odd
    r2 = (x * x + y * y + z * z) * (a / 4.0) ** 2
    return int(np.sum(site & (r2 <= R * R)))


@pytest.mark.parametrize("R", [4.0, 8.0, 10.0, 12.0, 16.0, 20.0, 24.0, 32.0, 36.0])
def test_pattern_counts_diamond(R):
    s = workloads.diamond(4)
    p = oracle.pattern(s, R, rows=[0, 5, 100])
    cnt = np.diff(p.row_ptr)[[0, 5, 100]]
    assert cnt[0] == diamond_neighbour_count(R)
    assert cnt[1] == diamond_neighbour_count(R, sub_is_odd=True)     # sublattice 5 is on the shifted fcc
    assert cnt[2] == diamond_neighbour_count(R, sub_is_odd=True)


def test_pattern_images_small_cell():
    """A 1x1x1 cell with a range larger than the cell: every lattice site within
    R appears once as (j, n), including self images (i, i, n != 0)."""
    s = workloads.diamond(1)
    for R in (6.0, 12.0, 20.0):
        p = oracle.pattern(s, R)
        assert np.all(np.diff(p.row_ptr)[[0]] == diamond_neighbour_count(R))
        # brute force over images and atoms
        i = 0
        found = []
        for j in range(8):
            for n in itertools.product(range(-4, 5), repeat=3):
                d = s.xyz[j] + np.array(n) @ s.lattice - s.xyz[i]
                if d @ d <= R * R:
                    found.append((j,) + n)
        got = [(int(c),) + tuple(int(v) for v in im) for c, im in
               zip(p.col[p.row_ptr[0]:p.row_ptr[1]], p.img[p.row_ptr[0]:p.row_ptr[1]])]
        assert got == sorted(found)


def test_pattern_inclusive_boundary():
    """A pair at exactly the range is kept (the cutoff removes only pairs beyond it)."""
    s = workloads.System(xyz=np.array([[0.0, 0, 0], [3.0, 0, 0], [0, 4.0, 0]]),
                         nfn=np.array([1, 1, 1], np.int32), lattice=None)
    p = oracle.pattern(s, 3.0)
    assert list(p.col[p.row_ptr[0]:p.row_ptr[1]]) == [0, 1]
    p = oracle.pattern(s, 5.0)
    assert list(p.col[p.row_ptr[1]:p.row_ptr[2]]) == [0, 1, 2]


# ---------------------------------------------------------------------------
# truncated products: brute force with dense numpy
# ---------------------------------------------------------------------------
def _cluster(n=40, edge=14.0, mixed=True, seed=3):
    nfn = np.where(np.arange(n) % 3 == 0, 5, np.where(np.arange(n) % 3 == 1, 3, 1)) if mixed else 4
    return workloads.random_cluster(n, edge, nfn=nfn, seed=seed)


def _random_matrix(p, seed):
    rng = np.random.default_rng(seed)
    return oracle.Matrix(p, rng.normal(size=p.nval))


@pytest.mark.parametrize("ranges", [(5.0, 6.0, 11.0), (5.0, 6.0, 7.0), (8.0, 4.0, 3.0), (30.0, 30.0, 30.0)])
def test_multiply_vs_dense(ranges):
    rA, rB, rC = ranges
    s = _cluster()
    A = _random_matrix(oracle.pattern(s, rA), 1)
    B = _random_matrix(oracle.pattern(s, rB), 2)
    pC = oracle.pattern(s, rC)
    C = oracle.multiply(A, B, pC)
    ref = _dense.mask_dense(pC) * (_dense.to_dense(A) @ _dense.to_dense(B))
    np.testing.assert_allclose(_dense.to_dense(C), ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    # A B^T form
    Bt = _random_matrix(oracle.pattern(s, rB), 5)
    C2 = oracle.multiply_nt(A, Bt, pC)
    ref2 = _dense.mask_dense(pC) * (_dense.to_dense(A) @ _dense.to_dense(Bt).T)
    np.testing.assert_allclose(_dense.to_dense(C2), ref2, rtol=0, atol=1e-13 * np.abs(ref2).max())


def test_transpose_project_dot():
    s = _cluster(mixed=True)
    A = _random_matrix(oracle.pattern(s, 6.0), 7)
    T = oracle.transpose(A, oracle.pattern(s, 6.0))
    np.testing.assert_array_equal(_dense.to_dense(T), _dense.to_dense(A).T)
    Q = oracle.project(A, oracle.pattern(s, 4.0))
    np.testing.assert_array_equal(_dense.to_dense(Q), _dense.to_dense(A) * _dense.mask_dense(oracle.pattern(s, 4.0)))
    x = np.random.default_rng(0).normal(size=1000)
    y = np.random.default_rng(1).normal(size=1000)
    assert abs(oracle.dot(x, y) - float(np.dot(x.astype(np.longdouble), y.astype(np.longdouble)))) < 1e-13


def test_dot_compensated():
    """Neumaier summation recovers a sum that naive FP64 summation loses."""
    a = np.array([1.0, 1e100, 1.0, -1e100])
    assert oracle.dot(a, np.ones(4)) == 2.0


def test_adjoint_identity():
    """<Cbar, P_C(op(dA) op(B))> = <Abar, dA> and likewise for B (bilinearity)."""
    s = _cluster(n=30, mixed=True)
    pA, pB, pC = oracle.pattern(s, 6.0), oracle.pattern(s, 5.0), oracle.pattern(s, 7.0)
    for tA, tB in itertools.product([False, True], repeat=2):
        A, B = _random_matrix(pA, 1), _random_matrix(pB, 2)
        Cb = _random_matrix(pC, 3)
        Ab, Bb = oracle.multiply_adjoint(A, tA, B, tB, Cb)
        dA, dB = _random_matrix(pA, 4), _random_matrix(pB, 5)
        lhsA = float(np.dot(Cb.val, oracle.multiply_op(dA, tA, B, tB, pC).val))
        lhsB = float(np.dot(Cb.val, oracle.multiply_op(A, tA, dB, tB, pC).val))
        assert abs(lhsA - np.dot(Ab.val, dA.val)) < 1e-12 * max(1, abs(lhsA))
        assert abs(lhsB - np.dot(Bb.val, dB.val)) < 1e-12 * max(1, abs(lhsB))
        # and against the dense definition
        opA = _dense.to_dense(A).T if tA else _dense.to_dense(A)
        opB = _dense.to_dense(B).T if tB else _dense.to_dense(B)
        Cbd = _dense.to_dense(Cb)
        refA = (opB @ Cbd.T) if tA else (Cbd @ opB.T)
        refB = (Cbd.T @ opA) if tB else (opA.T @ Cbd)
        np.testing.assert_allclose(_dense.to_dense(Ab), _dense.mask_dense(pA) * refA, atol=1e-12)
        np.testing.assert_allclose(_dense.to_dense(Bb), _dense.mask_dense(pB) * refB, atol=1e-12)


# ---------------------------------------------------------------------------
# the LNV chain on open clusters: dense untruncated algebra
# ---------------------------------------------------------------------------
def _inputs(s, rS, rH, rL, seed=0):
    return oracle.make_inputs(s, rS, rH, rL, seed=seed)


@pytest.mark.parametrize("mixed", [False, True])
def test_chain_vs_dense(mixed):
    s = _cluster(n=36, edge=13.0, mixed=mixed, seed=11)
    rS, rH, rL = 4.0, 5.0, 5.5
    inp = _inputs(s, rS, rH, rL)
    r = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    L, S, H = (_dense.to_dense(inp[k]) for k in "LSH")
    Kd = 3 * L @ S @ L - 2 * L @ S @ L @ S @ L       # eq. 3 with no truncation at all
    Ed = 2 * np.trace(Kd @ H)
    assert abs(r["E"] - Ed) <= 1e-13 * abs(Ed)
    np.testing.assert_allclose(_dense.to_dense(r["K"]), Kd * _dense.mask_dense(inp["H"].pattern),
                               atol=1e-13 * np.abs(Kd).max())
    # per-row energies add up to E
    assert abs(r["e_rows"].sum() - r["E"]) < 1e-12 * abs(r["E"])


def test_k_symmetry_and_associativity():
    c = workloads.workload("si64_rl12")
    s = c["system"]
    inp = _inputs(s, c["rS"], c["rH"], c["rL"])
    r = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], c["rS"], c["rH"], c["rL"])
    K = r["K"]
    KT = oracle.transpose(K, K.pattern)
    assert np.abs(K.val - KT.val).max() < 1e-13 * np.abs(K.val).max()
    R = oracle.chain_ranges(c["rS"], c["rH"], c["rL"])
    pM = oracle.pattern(s, R["M"])
    LSL1 = oracle.multiply(oracle.multiply(inp["L"], inp["S"], oracle.pattern(s, R["X"])), inp["L"], pM)
    SL = oracle.multiply(inp["S"], inp["L"], oracle.pattern(s, R["X"]))
    LSL2 = oracle.multiply(inp["L"], SL, pM)
    assert np.abs(LSL1.val - LSL2.val).max() < 1e-13 * np.abs(LSL1.val).max()


# ---------------------------------------------------------------------------
# periodic images: the image-resolved chain equals the central rows of an
# untruncated computation on an unfolded open cluster
# ---------------------------------------------------------------------------
def test_unfold_periodic_images():
    rS, rH, rL = 4.5, 6.0, 6.0
    cellsys = workloads.diamond(1)
    inp = _inputs(cellsys, rS, rH, rL)
    r = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    # open replica: 7x7x7 cells, values keyed by translation class as in the cell
    m = 7
    big = workloads.diamond((m, m, m), periodic=False, key_mode="class")
    binp = _inputs(big, rS, rH, rL)
    Ls, Ss, Hs = (_dense.to_sparse(binp[k]) for k in "LSH")
    X = Ls @ Ss                                     # every product untruncated
    center = np.where(np.all(big.cell == m // 2, axis=1))[0]
    assert center.size == 8
    oo = _dense.orbital_offsets(big.nfn)
    crow = np.concatenate([np.arange(oo[a], oo[a + 1]) for a in center])
    Mc = X[crow] @ Ls
    Pc = Mc @ X.T
    Kc = (3 * Mc - 2 * Pc).toarray()
    Hc = Hs[crow].toarray()
    E_open = 2 * np.sum(Kc * Hc)                   # 2 Tr(KH) over the central cell's rows
    assert abs(E_open - r["E"]) <= 1e-12 * abs(r["E"])
    # block by block: K_{i,(j,n)} of the cell equals K of the replica at (i_center, j at cell center+n)
    K = r["K"]
    bi, bj, bim = K.pattern.keys()
    cidx = {tuple(c) + (int(sb),): a for a, (c, sb) in enumerate(zip(big.cell, big.sub))}
    for b in range(K.pattern.nblocks):
        i, j, n = int(bi[b]), int(bj[b]), bim[b]
        ia = cidx[(m // 2,) * 3 + (i,)]
        ja = cidx[tuple(m // 2 + n) + (j,)]
        ri = np.where(center == ia)[0][0]
        blk = Kc[4 * ri:4 * ri + 4, oo[ja]:oo[ja] + 4]
        np.testing.assert_allclose(K.block(b), blk, atol=1e-13)


def test_extensivity_energy_per_atom():
    """Translation-class values make E an extensive quantity: E/N of 1x1x1 and
    2x2x2 periodic cells agree (cf. the constant energy per atom across the
    4,096 ... 2,097,152-atom cells of Table 1)."""
    rS, rH, rL = 8.0, 12.0, 12.0
    e = []
    for nc in (1, 2):
        s = workloads.diamond(nc)
        inp = _inputs(s, rS, rH, rL)
        e.append(oracle.lnv_energy(inp["L"], inp["S"], inp["H"], rS, rH, rL)["E"] / s.n)
    assert abs(e[0] - e[1]) <= 1e-13 * abs(e[0])


# ---------------------------------------------------------------------------
# McWeeny / LNV properties (the eigenvalue argument around eq. 3)
# ---------------------------------------------------------------------------
def _full_range_cluster(n=12, seed=5):
    s = workloads.random_cluster(n, 6.0, nfn=4, seed=seed)
    return s, 20.0          # range beyond the cluster diameter: nothing is truncated


def test_spectral_identity():
    """KS = f(LS) with f(x) = 3x^2 - 2x^3, so Tr(KS) = sum f(lambda_i(LS))."""
    s, R = _full_range_cluster()
    inp = _inputs(s, R, R, R)
    r = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], R, R, R)
    S = _dense.to_dense(inp["S"])
    lam = np.linalg.eigvals(_dense.to_dense(inp["L"]) @ S).real
    f = 3 * lam ** 2 - 2 * lam ** 3
    trKS = oracle.dot(r["K"].val, oracle.project(inp["S"], r["K"].pattern).val)   # <K, S> = Tr(K S), S symmetric
    assert abs(trKS - f.sum()) < 1e-12 * abs(f.sum())
    # eigenvalues of LS inside [-1/2, 3/2] map into [0, 1]
    assert np.all((lam > -0.5) & (lam < 1.5))
    kev = np.linalg.eigvals(_dense.to_dense(r["K"]) @ S).real
    assert kev.min() >= -1e-12 and kev.max() <= 1 + 1e-12


def test_purified_density_matrix():
    """At an idempotent L = C_occ C_occ^T (generalised eigenvectors of H, S):
    LSL = L, so K = L, Tr(KS) = N_occ (N_e = 2 Tr(KS)) and E = 2 sum of the
    occupied eigenvalues."""
    s, R = _full_range_cluster(n=10, seed=8)
    inp = _inputs(s, R, R, R)
    S, H = _dense.to_dense(inp["S"]), _dense.to_dense(inp["H"])
    w, C = scipy.linalg.eigh(H, S)
    nocc = 2 * s.n                      # two doubly occupied states per 4-function atom
    Lp = C[:, :nocc] @ C[:, :nocc].T
    L = _dense.from_dense(inp["L"].pattern, Lp)
    r = oracle.lnv_energy(L, inp["S"], inp["H"], R, R, R)
    np.testing.assert_allclose(_dense.to_dense(r["K"]), Lp, atol=1e-11)
    trKS = oracle.dot(r["K"].val, oracle.project(inp["S"], r["K"].pattern).val)
    assert abs(trKS - nocc) < 1e-10
    assert abs(r["E"] - 2 * w[:nocc].sum()) < 1e-10 * abs(r["E"])


def test_closed_form_scalar():
    """S = I and L = lam I give K = (3 lam^2 - 2 lam^3) I and E = 2 (3 lam^2 - 2 lam^3) Tr H."""
    s = workloads.diamond(1)
    rS, rH, rL = 8.0, 12.0, 12.0
    inp = _inputs(s, rS, rH, rL)
    lam = 0.37
    for name, scale in (("S", 1.0), ("L", lam)):
        p = inp[name].pattern
        bi, bj, bim = p.keys()
        v = np.zeros(p.nval)
        for b in np.where((bi == bj) & np.all(bim == 0, axis=1))[0]:
            v[p.off[b]:p.off[b] + 16] = scale * np.eye(4).ravel()
        inp[name] = oracle.Matrix(p, v)
    r = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    f = 3 * lam ** 2 - 2 * lam ** 3
    trH = 4.0 * s.n                     # H's on-site blocks are the identity
    assert abs(r["E"] - 2 * f * trH) < 1e-13 * abs(r["E"])


def test_closed_form_block_diagonal():
    """Ranges below the nearest-neighbour distance (4.443 bohr) leave only on-site
    blocks: K_ii = 3 L_ii S_ii L_ii - 2 L_ii S_ii L_ii S_ii L_ii atom by atom."""
    s = workloads.diamond(2, jitter=0.05, seed=2)
    rS = rH = rL = 4.0
    inp = _inputs(s, rS, rH, rL)
    rng = np.random.default_rng(1)
    for name in "LSH":               # random symmetric on-site blocks so that the test is not trivial
        blk = rng.normal(size=(s.n, 4, 4))
        blk = 0.5 * (blk + blk.transpose(0, 2, 1))
        assert inp[name].pattern.nblocks == s.n
        inp[name] = oracle.Matrix(inp[name].pattern, blk.ravel().copy())
    r = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    E = 0.0
    for i in range(s.n):
        Li, Si, Hi = (inp[k].val[16 * i:16 * i + 16].reshape(4, 4) for k in "LSH")
        Ki = 3 * Li @ Si @ Li - 2 * Li @ Si @ Li @ Si @ Li
        np.testing.assert_allclose(r["K"].block(i), Ki, atol=1e-12)
        E += 2 * np.sum(Ki * Hi)
    assert abs(E - r["E"]) < 1e-12 * abs(E)


# ---------------------------------------------------------------------------
# gradient: E is a cubic polynomial of L, so a Richardson-extrapolated central
# difference is exact up to rounding
# ---------------------------------------------------------------------------
def _richardson(Efun, h):
    d1 = (Efun(h) - Efun(-h)) / (2 * h)
    d2 = (Efun(h / 2) - Efun(-h / 2)) / h
    return (4 * d2 - d1) / 3


@pytest.mark.parametrize("case", ["periodic_cell", "open_mixed"])
def test_gradient_vs_richardson(case):
    if case == "periodic_cell":
        s = workloads.diamond(1)
        rS, rH, rL = 8.0, 12.0, 12.0
    else:
        s = _cluster(n=30, edge=12.0, mixed=True, seed=4)
        rS, rH, rL = 4.0, 5.0, 5.5
    inp = _inputs(s, rS, rH, rL)
    G = oracle.lnv_gradient(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    rng = np.random.default_rng(9)
    pL = inp["L"].pattern
    for trial in range(4):
        if trial < 2:
            d = rng.normal(size=pL.nval)          # every stored block, no symmetry imposed
        else:
            d = np.zeros(pL.nval)                 # a single off-site block
            b = int(np.where(pL.col != pL.rows_of_blocks())[0][5 + trial])
            sz = int(s.nfn[pL.rows_of_blocks()[b]] * s.nfn[pL.col[b]])
            d[pL.off[b]:pL.off[b] + sz] = rng.normal(size=sz)
        dsym = 0.5 * (d + oracle.transpose(oracle.Matrix(pL, d), pL).val)

        def Efun(h, lit, dd):
            Lh = oracle.Matrix(pL, inp["L"].val + h * dd)
            return oracle.lnv_energy(Lh, inp["S"], inp["H"], rS, rH, rL, literal=lit)["E"]
        # eq. 3 taken literally, along any direction
        fd = _richardson(lambda h: Efun(h, True, d), 1e-2)
        an = float(np.dot(G.val, d))
        assert abs(fd - an) <= 1e-9 * max(1.0, abs(an)), (fd, an)
        # the M X^T chain along symmetric directions (where it is eq. 3)
        fds = _richardson(lambda h: Efun(h, False, dsym), 1e-2)
        ans = float(np.dot(G.val, dsym))
        assert abs(fds - ans) <= 1e-9 * max(1.0, abs(ans)), (fds, ans)
    assert np.abs(G.val - oracle.transpose(G, pL).val).max() < 1e-12 * np.abs(G.val).max()


def test_gradient_vs_dense_formula_open():
    """Independent check of the gradient chain's truncations on an open cluster."""
    s = _cluster(n=30, edge=12.0, mixed=False, seed=6)
    rS, rH, rL = 4.0, 5.0, 5.5
    inp = _inputs(s, rS, rH, rL)
    G = oracle.lnv_gradient(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    L, S, H = (_dense.to_dense(inp[k]) for k in "LSH")
    Gd = 6 * (H @ L @ S + S @ L @ H) - 4 * (H @ L @ S @ L @ S + S @ L @ H @ L @ S + S @ L @ S @ L @ H)
    np.testing.assert_allclose(_dense.to_dense(G), Gd * _dense.mask_dense(inp["L"].pattern), atol=1e-12)


# ---------------------------------------------------------------------------
# row cones: single rows of a large system match the full computation
# ---------------------------------------------------------------------------
def test_row_cones_match_full():
    c = workloads.workload("si64_rl12")
    s = workloads.diamond(2, jitter=0.1, seed=1)
    rS, rH, rL = c["rS"], c["rH"], c["rL"]
    inp = _inputs(s, rS, rH, rL)
    full = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    Gf = oracle.lnv_gradient(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    rows = np.array([3, 17, 40])
    part = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], rS, rH, rL, rows=rows)
    np.testing.assert_allclose(part["e_rows"], full["e_rows"][rows], rtol=1e-13)
    Gp = oracle.lnv_gradient(inp["L"], inp["S"], inp["H"], rS, rH, rL, rows=rows)
    for i in rows:
        np.testing.assert_allclose(oracle.row_slice(Gp, i), oracle.row_slice(Gf, i), atol=1e-12)


def test_row_cone_missing_input_raises():
    s = workloads.diamond(2)
    inp = oracle.make_inputs(s, 8.0, 12.0, 12.0, rows_L=[0], rows_S=[0], rows_H=[0])
    with pytest.raises(ValueError):
        oracle.lnv_energy(inp["L"], inp["S"], inp["H"], 8.0, 12.0, 12.0, rows=[0])


# ---------------------------------------------------------------------------
# triple counts (the unit of work) against integer enumeration
# ---------------------------------------------------------------------------
def diamond_triples(rA, rB, rC, a=10.26):
    """Triples (k, j) around a site i = 0: |k| <= rA, |j - k| <= rB, |j| <= rC,
    enumerated on integer a/4 coordinates (site 0 on the even lattice)."""
    m = int(np.ceil(4 * max(rA, rC) / a)) + 2
    g = np.arange(-m, m + 1)
    x, y, z = (v.ravel() for v in np.meshgrid(g, g, g, indexing="ij"))
    s = x + y + z
    even = (x % 2 == 0) & (y % 2 == 0) & (z % 2 == 0) & (s % 4 == 0)
    odd = (x % 2 != 0) & (y % 2 != 0) & (z % 2 != 0) & (s % 4 == 3)
    pts = np.stack([x, y, z], 1)[even | odd]
    u2 = (a / 4.0) ** 2
    r2 = (pts ** 2).sum(1) * u2
    K = pts[r2 <= rA * rA]
    J = pts[r2 <= rC * rC]
    d = ((J[None, :, :] - K[:, None, :]) ** 2).sum(2) * u2
    return int(np.sum(d <= rB * rB))


def test_triple_counts_per_atom():
    s = workloads.diamond(4)
    rS, rH, rL = 8.0, 12.0, 12.0
    R = oracle.chain_ranges(rS, rH, rL)
    inp = _inputs(s, rS, rH, rL)
    X, n1 = oracle.multiply(inp["L"], inp["S"], oracle.pattern(s, R["X"]), count=True)
    assert n1 == s.n * diamond_triples(rL, rS, R["X"])
    _, n2 = oracle.multiply(X, inp["L"], oracle.pattern(s, R["M"], rows=np.arange(8)), count=True)
    assert n2 == 8 * diamond_triples(R["X"], rL, R["M"])


# ---------------------------------------------------------------------------
# the seeded generator: symmetry, determinism, order independence
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["S", "H", "L"])
@pytest.mark.parametrize("sysname", ["class", "pair", "mixed"])
def test_generator_symmetric_and_order_free(which, sysname):
    if sysname == "class":
        s = workloads.diamond(1)
    elif sysname == "pair":
        s = workloads.diamond(1, jitter=0.1, seed=3)
    else:
        s = workloads.random_box(30, 9.0, 20, 13, 5, seed=1)
    p = oracle.pattern(s, 9.0)
    i, j, img = p.keys()
    v = workloads.block_values(s, which, i, j, img, seed=4, rS=8.0)
    M = oracle.Matrix(p, v)
    T = oracle.transpose(M, p)
    np.testing.assert_array_equal(M.val, T.val)
    perm = np.random.default_rng(0).permutation(i.size)
    v2 = workloads.block_values(s, which, i[perm], j[perm], img[perm], seed=4, rS=8.0)
    for k, b in enumerate(perm[:50]):
        np.testing.assert_array_equal(M.block(b).ravel(),
                                      v2[np.sum((s.nfn[i[perm[:k]]] * s.nfn[j[perm[:k]]])):][:M.block(b).size])
    on = np.where((i == j) & np.all(img == 0, axis=1))[0]
    for b in on[:5]:
        expect = np.eye(s.nfn[i[b]]) * (0.5 if which == "L" else 1.0)
        np.testing.assert_array_equal(M.block(b), expect)


def test_slab_geometry():
    """H-terminated (001) slab: 8 Si per cell, two H per surface Si on each face,
    every Si four-fold bonded (Si at the bulk distance or H at 2.8 bohr), every
    H bonded to one Si, and the vacuum wider than the longest range in use."""
    nx, ny, nz = 2, 3, 2
    s = workloads.si_slab((nx, ny, nz))
    si, h = s.nfn == 4, s.nfn == 1
    assert si.sum() == 8 * nx * ny * nz and h.sum() == 8 * nx * ny
    a = 10.26
    L = np.diag(s.lattice)
    d = s.xyz[:, None, :] - s.xyz[None, :, :]
    d[..., :2] -= np.round(d[..., :2] / L[:2]) * L[:2]          # periodic in x and y only
    r = np.sqrt((d * d).sum(-1))
    bulk = np.sqrt(3.0) * a / 4
    nsi = ((np.abs(r - bulk) < 1e-9) & si[None, :]).sum(1)
    nh = ((np.abs(r - 2.8) < 1e-9) & h[None, :]).sum(1)
    assert np.all(nsi[si] + nh[si] == 4)
    assert np.all(((np.abs(r - 2.8) < 1e-9) & si[None, :]).sum(1)[h] == 1)
    gap = L[2] - np.ptp(s.xyz[:, 2])
    assert gap >= 2 * 16.0 + 8.0                                  # 2 R_L + R_S of the slab workload


def test_generator_translation_invariance():
    s = workloads.diamond(2)
    p = oracle.pattern(s, 12.0)
    i, j, img = p.keys()
    v = workloads.block_values(s, "H", i, j, img, seed=0)
    M = oracle.Matrix(p, v)
    # atom 0 and atom 8 are the same sublattice one cell apart: their rows hold
    # the same blocks once matched by (sublattice of j, cell offset)
    rows = []
    for a in (0, 8):
        bs = np.arange(p.row_ptr[a], p.row_ptr[a + 1])
        d = s.cell[j[bs]] + img[bs] * 2 - s.cell[a]
        key = s.sub[j[bs]] * 10**6 + (d[:, 0] + 50) * 10**4 + (d[:, 1] + 50) * 100 + d[:, 2] + 50
        rows.append(np.concatenate([M.block(b).ravel() for b in bs[np.argsort(key)]]))
    np.testing.assert_array_equal(rows[0], rows[1])


# ---------------------------------------------------------------------------
# minimisation of E over L: exact cubic line search and conjugate gradients
# ---------------------------------------------------------------------------
def test_line_coeffs_reproduce_energy_and_gradient():
    """The expanded coefficients of E(L + tD) reproduce the literal energy at
    arbitrary t (E is exactly cubic in t), for a non-symmetric direction too,
    and c1 equals <dE/dL, D> from the independent gradient chain."""
    s = workloads.workload("si64_rl12")["system"]
    rS, rH, rL = 8.0, 12.0, 12.0
    inp = _inputs(s, rS, rH, rL)
    G = oracle.lnv_gradient(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    rng = np.random.default_rng(7)
    for D in (oracle.Matrix(G.pattern, -G.val), oracle.Matrix(G.pattern, 0.05 * rng.normal(size=G.val.size))):
        c = oracle.lnv_line_coeffs(inp["L"], D, inp["S"], inp["H"], rS, rH, rL)
        for t in (0.37, -0.8, 1.3):
            Lt = oracle.Matrix(inp["L"].pattern, inp["L"].val + t * D.val)
            E = oracle.lnv_energy(Lt, inp["S"], inp["H"], rS, rH, rL, literal=True)["E"]
            assert abs(E - (c[0] + c[1] * t + c[2] * t * t + c[3] * t ** 3)) <= 1e-12 * max(abs(E), 1.0)
    Dsym = oracle.Matrix(G.pattern, -G.val)      # symmetric direction: the gradient formula applies
    c = oracle.lnv_line_coeffs(inp["L"], Dsym, inp["S"], inp["H"], rS, rH, rL)
    assert abs(c[1] - oracle.dot(G.val, Dsym.val)) <= 1e-12 * abs(c[1])


def test_cubic_step_is_local_minimum():
    for c in ([0.0, -3.0, 2.0, 0.5], [1.0, -1.0, 0.0, 1.0], [0.0, -2.0, 1.0, 0.0]):
        t = oracle.cubic_step(c, 0.1)
        assert t > 0
        assert abs(c[1] + 2 * c[2] * t + 3 * c[3] * t * t) < 1e-12
        assert 2 * c[2] + 6 * c[3] * t > 0
    # a cubic with no local minimum along the line takes the trial step
    assert oracle.cubic_step([0.0, -1.0, -1.0, -1.0], 0.25) == 0.25


def onsite_minimiser_case():
    """On-site-only system (ranges below the nearest-neighbour distance), S = I,
    H_ii = Q_i diag(-1, -0.5, 0.3, 1) Q_i^T, L = I/2: the minimum of
    2 Tr[(3L^2 - 2L^3) H] is the projector on H's negative eigenvectors,
    E = 2 (-1.5) per atom."""
    s = workloads.diamond(2, jitter=0.05, seed=2)
    rS = rH = rL = 4.0
    v = onsite_values(s.n)
    pat = {k: oracle.pattern(s, r) for k, r in (("S", rS), ("H", rH), ("L", rL))}
    for p in pat.values():
        assert p.nblocks == s.n and np.all(p.col == np.arange(s.n))
    S, H, L0 = (oracle.Matrix(pat[k], v[k].copy()) for k in "SHL")
    return s, (rS, rH, rL), L0, S, H, v["P"], -3.0 * s.n


def test_minimiser_closed_form_projector():
    s, (rS, rH, rL), L0, S, H, P, Emin = onsite_minimiser_case()
    Lf, Es, gs = oracle.lnv_minimise(L0, S, H, rS, rH, rL, max_iter=80, gtol=1e-11)
    assert np.all(np.diff(Es) <= 1e-12 * abs(Emin))          # monotone descent
    assert gs[-1] <= 1e-11
    assert abs(Es[-1] - Emin) <= 1e-12 * abs(Emin)
    np.testing.assert_allclose(Lf.val, P, atol=1e-9)


def test_minimiser_gradients_mutually_orthogonal():
    """Near L = 0 the energy is the convex quadratic 6 Tr(L S L H) (S and H
    positive definite; the cubic term is smaller by a factor |L|).  On a
    convex quadratic, conjugate gradients with exact line searches make each
    new gradient orthogonal to all earlier ones, not only to the last one;
    steepest descent (a Polak-Ribiere beta dropped, of the wrong sign, or with
    the old gradient in place of the new one, all of which fall back to it)
    leaves G_2 . G_0 of the order of |G_2| |G_0| (0.6 here).  On a quadratic
    the Polak-Ribiere and Fletcher-Reeves betas agree, so this does not tell
    them apart.  Gradients come from lnv_gradient, pinned on its own."""
    s = _cluster(n=12, edge=9.0, mixed=False, seed=21)
    r = 5.0
    inp = _inputs(s, r, r, r)
    S = inp["S"]
    H = oracle.Matrix(S.pattern, S.val.copy())                  # H = S: positive definite
    assert np.linalg.eigvalsh(_dense.to_dense(S)).min() > 0.5
    L0 = sym_random(inp["L"].pattern, np.random.default_rng(5))
    L0 = oracle.Matrix(L0.pattern, 1e-4 * L0.val)
    G = [oracle.lnv_gradient(L0, S, H, r, r, r).val]
    for k in (1, 2, 3):
        Lk, _, _ = oracle.lnv_minimise(L0, S, H, r, r, r, max_iter=k)
        G.append(oracle.lnv_gradient(Lk, S, H, r, r, r).val)
    for i in range(4):
        for j in range(i):
            c = np.dot(G[i], G[j]) / np.sqrt(np.dot(G[i], G[i]) * np.dot(G[j], G[j]))
            assert abs(c) <= 5e-3, (i, j, c)


# ---------------------------------------------------------------------------
# electron number and chemical potential (constraint 2 of the ground-state search)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mixed", [False, True])
def test_electron_number_vs_dense(mixed):
    """N_e = 2 Tr(KS) with K = 3LSL - 2LSLSL untruncated (dense), and H - mu S
    equals the dense H - mu S on H's pattern."""
    s = _cluster(n=36, edge=13.0, mixed=mixed, seed=11)
    rS, rH, rL = 4.0, 5.0, 5.5
    inp = _inputs(s, rS, rH, rL)
    L, S, H = (_dense.to_dense(inp[k]) for k in "LSH")
    Kd = 3 * L @ S @ L - 2 * L @ S @ L @ S @ L
    Nd = 2 * np.trace(Kd @ S)
    N = oracle.electron_number(inp["L"], inp["S"], rS, rH, rL)
    assert abs(N - Nd) <= 1e-13 * abs(Nd)
    Hm = oracle.shift(inp["H"], inp["S"], 0.37)
    np.testing.assert_array_equal(_dense.to_dense(Hm), (H - 0.37 * S) * _dense.mask_dense(inp["H"].pattern))
    Ed = 2 * np.trace(Kd @ (H - 0.37 * S))
    E = oracle.lnv_energy(inp["L"], inp["S"], Hm, rS, rH, rL)["E"]
    assert abs(E - Ed) <= 1e-13 * max(abs(Ed), abs(Nd))


def test_electron_number_closed_form():
    """On-site blocks only, S = I, L = l I: K = (3 l^2 - 2 l^3) I, N_e = 2 (3 l^2 - 2 l^3) n_orb."""
    s, (rS, rH, rL), _, S, H, P, _ = onsite_minimiser_case()
    for l in (0.3, 0.5, 1.1):
        L = oracle.Matrix(oracle.pattern(s, rL), np.tile(l * np.eye(4).ravel(), s.n))
        N = oracle.electron_number(L, S, rS, rH, rL)
        assert abs(N - 2 * (3 * l * l - 2 * l ** 3) * 4 * s.n) <= 1e-13 * 4 * s.n
    # the projector on two of four functions per atom holds 4 electrons per atom
    Lp = oracle.Matrix(oracle.pattern(s, rL), P)
    assert abs(oracle.electron_number(Lp, S, rS, rH, rL) - 4.0 * s.n) <= 1e-12 * s.n


def test_minimiser_grand_potential_closed_form():
    """Minimising 2 Tr[K(H - mu S)] on the on-site case fills every level below
    mu: with levels (-1, -0.5, 0.3, 1) and mu = 0.5, three per atom, so
    E - mu N_e = 2 (-1.5 - 1.0 - 0.2) per atom and N_e = 6 per atom."""
    s, (rS, rH, rL), L0, S, H, _, _ = onsite_minimiser_case()
    Hm = oracle.shift(H, S, 0.5)
    Lf, Es, gs = oracle.lnv_minimise(L0, S, Hm, rS, rH, rL, max_iter=80, gtol=1e-11)
    assert abs(Es[-1] - (-5.4 * s.n)) <= 1e-12 * 5.4 * s.n
    assert abs(oracle.electron_number(Lf, S, rS, rH, rL) - 6.0 * s.n) <= 1e-9 * s.n


# ---------------------------------------------------------------------------
# McWeeny purification step (eq. 3 as a map of L)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mixed", [False, True])
def test_mcweeny_vs_dense(mixed):
    """One step equals the untruncated 3LSL - 2LSLSL restricted to L's pattern."""
    s = _cluster(n=36, edge=13.0, mixed=mixed, seed=12)
    rS, rH, rL = 4.0, 5.0, 5.5
    inp = _inputs(s, rS, rH, rL)
    L, S = _dense.to_dense(inp["L"]), _dense.to_dense(inp["S"])
    ref = (3 * L @ S @ L - 2 * L @ S @ L @ S @ L) * _dense.mask_dense(inp["L"].pattern)
    got = _dense.to_dense(oracle.mcweeny(inp["L"], inp["S"], rS, rL))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_mcweeny_closed_forms():
    """On-site blocks, S = I: L = l I maps to (3 l^2 - 2 l^3) I, and a projector
    is a fixed point."""
    s, (rS, rH, rL), _, S, H, P, _ = onsite_minimiser_case()
    pL = oracle.pattern(s, rL)
    for l in (0.2, 0.5, 0.9, 1.2):
        L = oracle.Matrix(pL, np.tile(l * np.eye(4).ravel(), s.n))
        out = oracle.mcweeny(L, S, rS, rL)
        np.testing.assert_allclose(out.val, np.tile((3 * l * l - 2 * l ** 3) * np.eye(4).ravel(), s.n), atol=1e-15)
    Lp = oracle.Matrix(pL, P)
    np.testing.assert_allclose(oracle.mcweeny(Lp, S, rS, rL).val, P, atol=1e-14)


def test_mcweeny_iteration_reaches_projector():
    """With every pair in range, iterating the step maps each eigenvalue of LS
    in (-1/2, 3/2) through 3x^2 - 2x^3 towards 0 (below 1/2) or 1 (above): LS
    becomes idempotent and Tr(LS) counts the eigenvalues above 1/2."""
    s, R = _full_range_cluster(n=10, seed=8)
    inp = _inputs(s, R, R, R)
    S = _dense.to_dense(inp["S"])
    lam = np.linalg.eigvals(_dense.to_dense(inp["L"]) @ S).real
    assert lam.min() > -0.5 and lam.max() < 1.5 and np.all(np.abs(lam - 0.5) > 1e-3)
    L = inp["L"]
    for _ in range(40):
        L = oracle.mcweeny(L, inp["S"], R, R)
    LS = _dense.to_dense(L) @ S
    np.testing.assert_allclose(LS @ LS, LS, atol=1e-9)
    assert abs(np.trace(LS) - np.sum(lam > 0.5)) < 1e-9


# ---------------------------------------------------------------------------
# stored oracle results (tests/golden, written by tests/golden/make_golden.py)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["si64_rl12", "mixed_cluster_40"])
def test_oracle_matches_stored_results(name):
    import json
    import os
    import importlib.util
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(here, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    ref = json.load(open(os.path.join(here, f"oracle_{name}.json")))
    case = next(c for c in mg.cases() if c[0] == name)
    got = mg.record(*case)
    for key in ("E", "N_e", "grad_norm"):
        assert abs(got[key] - ref[key]) <= 1e-13 * abs(ref[key]), key
    for key in ("grad_samples", "K_samples"):
        for i, v in ref[key].items():
            assert abs(got[key][i] - v) <= 1e-13 * max(abs(v), 1e-3), (key, i)
