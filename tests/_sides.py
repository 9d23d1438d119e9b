"""Builds the same synthetic problem on the GPU library and on the oracle.

Values come from the seeded generator (workloads) keyed by block, so each side
fills its own pattern independently; nothing computed by the GPU path is fed
to the oracle.
"""
import numpy as np

import oracle
import workloads


def gpu_values(pattern, sysm, which, seed=0, rS=None):
    i, j, img = pattern.keys()
    return workloads.block_values(sysm, which, i, j, img, seed=seed, rS=rS)


def same_pattern(gp, op):
    """GPU-exported pattern equals the oracle pattern (rows, columns, images)."""
    rp, col, img, off = gp.export()
    return (np.array_equal(rp, op.row_ptr) and np.array_equal(col, op.col) and np.array_equal(img, op.img)
            and np.array_equal(off, op.off))


def rel(a, b):
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


ONSITE_LEVELS = (-1.0, -0.5, 0.3, 1.0)


def onsite_values(n_atoms, seed=11):
    """Values of an on-site-only problem (one 4x4 block per atom, rows in atom
    order): S = I, H_ii = Q_i diag(ONSITE_LEVELS) Q_i^T with random orthogonal
    Q_i, L = I/2, and the projector on the two lowest levels per atom."""
    rng = np.random.default_rng(seed)
    e = np.array(ONSITE_LEVELS)
    Hb, Pb = [], []
    for _ in range(n_atoms):
        Q, _ = np.linalg.qr(rng.normal(size=(4, 4)))
        Hb.append((Q * e) @ Q.T)
        Pb.append(Q[:, :2] @ Q[:, :2].T)
    S = np.tile(np.eye(4).ravel(), n_atoms)
    L = 0.5 * S
    return dict(S=S, H=np.concatenate([b.ravel() for b in Hb]), L=L, P=np.concatenate([b.ravel() for b in Pb]))


# ---------------------------------------------------------------------------
# block-wise comparison on inputs that do not decay with distance
# ---------------------------------------------------------------------------
FLOOR = 0.05     # blocks are compared against max(own norm, FLOOR x RMS block norm)


def sym_random(p, rng):
    """Symmetric unit-size normal values on an oracle pattern p (mirror pairs
    averaged, so block (j,i,-n) is exactly the transpose of block (i,j,n))."""
    A = oracle.Matrix(p, rng.standard_normal(p.nval))
    return oracle.Matrix(p, 0.5 * (A.val + oracle.transpose(A, p).val))


def block_sizes(p):
    nfn = np.asarray(p.system.nfn, np.int64)
    return nfn[p.rows_of_blocks()] * nfn[p.col]


def blockwise_rel(got, ref, p):
    """Largest per-block error ||got_b - ref_b|| / max(||ref_b||, FLOOR rms)
    over the blocks of oracle pattern p."""
    if p.nblocks == 0:
        return 0.0
    d2 = np.add.reduceat((np.asarray(got) - ref) ** 2, p.off)
    r2 = np.add.reduceat(np.asarray(ref) ** 2, p.off)
    rms = np.sqrt(np.mean(r2))
    den = np.maximum(np.sqrt(r2), FLOOR * rms)
    return float(np.max(np.sqrt(d2) / den))


def assert_mirrored(vals, p):
    """Off-site blocks equal the transposes of their mirrors bit for bit."""
    t = oracle.transpose(oracle.Matrix(p, vals), p).val
    rows = p.rows_of_blocks()
    onsite_b = (p.col == rows) & np.all(np.asarray(p.img).reshape(-1, 3) == 0, axis=1)
    onsite = np.repeat(onsite_b, block_sizes(p))
    np.testing.assert_array_equal(vals[~onsite], t[~onsite])
