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
