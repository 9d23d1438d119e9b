"""Argument checks of the Python binding (CPU): tensors that are not
contiguous float64 device tensors of the pattern's size are refused before any
library call, so no host pointer can reach a device entry point."""
import numpy as np
import pytest
import torch

import workloads
import paper_0911_3584_amd as lsdm
from paper_0911_3584_amd import _dev, _prec


def test_dev_refuses_host_and_wrong_tensors():
    with pytest.raises(TypeError):
        _dev(torch.zeros(4, dtype=torch.float64), what="L")          # host tensor
    with pytest.raises(TypeError):
        _dev(np.zeros(4), what="L")                                    # not a tensor
    assert _dev(None) is None


def test_precision_names():
    assert [_prec(n) for n in ("fp64", "fp32", "bf16", "fp32_rc")] == [lsdm.FP64, lsdm.FP32, lsdm.BF16,
                                                                       lsdm.FP32_RC]
    with pytest.raises(KeyError):
        _prec("fp16")


def test_lnv_calls_refuse_host_tensors():
    s = workloads.diamond(1)
    lnv = lsdm.LNV(lsdm.System.from_workload(s), 4.0, 5.0, 5.0, symmetric=True)
    v = {w: torch.zeros(lnv.patterns[w].n_values, dtype=torch.float64) for w in "LSH"}
    with pytest.raises(TypeError):
        lnv.energy(v["L"], v["S"], v["H"])
    with pytest.raises(TypeError):
        lnv.energy_grad(v["L"], v["S"], v["H"], prec="fp32")


def test_system_shape_checks():
    with pytest.raises(ValueError):
        lsdm.System(np.zeros((4, 2)), np.full(4, 4))
    with pytest.raises(ValueError):
        lsdm.System(np.zeros((4, 3)), np.full(3, 4))
