"""The block-wise comparison used by the GPU parity tests on non-decaying
inputs (CPU): it must see a single wrong far block that a norm-wise comparison
misses, and a mirror that is not an exact transpose."""
import numpy as np
import pytest

import oracle
import workloads
from tests._sides import assert_mirrored, block_sizes, blockwise_rel, sym_random


def _setup():
    s, rS, rH, rL = workloads.diamond(2, jitter=0.1, seed=7), 8.0, 12.0, 16.0
    rng = np.random.default_rng(17)
    pL, pS, pH = (oracle.pattern(s, r) for r in (rL, rS, rH))
    L, S, H = sym_random(pL, rng), sym_random(pS, rng), sym_random(pH, rng)
    return s, pL, oracle.lnv_gradient(L, S, H, rS, rH, rL).val


def test_sees_one_wrong_far_block():
    s, pL, G = _setup()
    rows = pL.rows_of_blocks()
    vec = s.xyz[pL.col] - s.xyz[rows] + np.asarray(pL.img, np.float64) @ s.lattice
    b = int(np.argmax(np.einsum("ij,ij->i", vec, vec)))      # the farthest block of the range
    bad = G.copy()
    n = int(block_sizes(pL)[b])
    bad[pL.off[b]:pL.off[b] + n] *= 1.0 + 1e-9
    assert blockwise_rel(G, G, pL) == 0.0
    assert blockwise_rel(bad, G, pL) > 1e-12
    assert np.linalg.norm(bad - G) / np.linalg.norm(G) < 1e-9


def test_mirror_check():
    s, pL, G = _setup()
    G = 0.5 * (G + oracle.transpose(oracle.Matrix(pL, G), pL).val)    # exactly symmetric
    assert_mirrored(G, pL)
    bad = G.copy()
    rows = pL.rows_of_blocks()
    b = int(np.where(rows != pL.col)[0][3])
    bad[pL.off[b]] += 1e-14 * abs(bad[pL.off[b]]) + 1e-300
    with pytest.raises(AssertionError):
        assert_mirrored(bad, pL)    # one changed off-site element breaks it
