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
