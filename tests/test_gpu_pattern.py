"""Range patterns built by the GPU neighbour search.

With a device present the library searches pairs on the GPU (count, fill,
per-row sort); the CPU suite checks the host search.  These tests hold the
GPU-built patterns to the oracle's brute-force patterns, on the same systems
and ranges as the host tests, and check the GPU path's error cases."""
import pytest

import oracle
import workloads
import paper_0911_3584_amd as lsdm
from tests._sides import same_pattern
from tests.test_symbolic_abi import SYSTEMS

pytestmark = pytest.mark.gpu


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


@pytest.mark.parametrize("name", list(SYSTEMS))
@pytest.mark.parametrize("R", [0.0, 4.5, 8.0, 12.0, 20.0, 36.0])
def test_gpu_pattern_equals_oracle(name, R):
    _need_gpu()
    s = SYSTEMS[name]()
    gs = lsdm.System.from_workload(s)
    gp = lsdm.Pattern(gs, R)
    op = oracle.pattern(s, R)
    assert gp.n_blocks == op.nblocks and gp.n_values == op.nval
    assert same_pattern(gp, op)


def test_gpu_pattern_32768_counts():
    """The 32,768-atom cell at M's range (40 bohr): every row of the perfect
    crystal holds the same number of blocks, the oracle's count per row on a
    216-atom cell of the same crystal (every row sees the same shells)."""
    _need_gpu()
    s = workloads.diamond(16)
    gs = lsdm.System.from_workload(s)
    op = oracle.pattern(workloads.diamond(3), 40.0)     # 216 atoms: every row sees the same shells
    per_row = op.nblocks // 216
    assert op.nblocks == 216 * per_row
    gp = lsdm.Pattern(gs, 40.0)
    assert gp.n_blocks == s.n * per_row


def test_gpu_pattern_beyond_block_limit_is_enomem():
    _need_gpu()
    s = workloads.diamond(4)
    gs = lsdm.System.from_workload(s)
    with pytest.raises(lsdm.LsdmError) as e:
        lsdm.Pattern(gs, 600.0)
    assert e.value.code == lsdm._lib.ENOMEM
    assert "2^31" in str(e.value)
    assert lsdm.Pattern(gs, 8.0).n_blocks == 512 * 17
