"""Checkpoint and resume (CPU): the saved system, ranges, mode and values come
back exactly, and a file whose block layout no longer matches is refused."""
import numpy as np
import pytest

import workloads
import paper_0911_3584_amd as lsdm


def _setup(s, rS, rH, rL, symmetric):
    lnv = lsdm.LNV(lsdm.System.from_workload(s), rS, rH, rL, symmetric=symmetric)
    vals = {w: workloads.block_values(s, w, *lnv.patterns[w].keys(), seed=5, rS=rS) for w in "LSH"}
    return lnv, vals


@pytest.mark.parametrize("name,symmetric", [("periodic", True), ("open", False)])
def test_checkpoint_round_trip(tmp_path, name, symmetric):
    s = (workloads.diamond(2, jitter=0.05, seed=3) if name == "periodic"
         else workloads.random_cluster(40, 10.0, nfn=np.arange(40) % 5 + 1, seed=6))
    rS, rH, rL = (8.0, 12.0, 12.0) if name == "periodic" else (5.0, 6.0, 6.5)
    lnv, vals = _setup(s, rS, rH, rL, symmetric)
    path = tmp_path / "lnv.npz"
    lsdm.save_checkpoint(path, lnv, vals)
    lnv2, v2 = lsdm.load_checkpoint(path)
    assert lnv2.symmetric == symmetric and (lnv2.rS, lnv2.rH, lnv2.rL) == (rS, rH, rL)
    assert np.array_equal(lnv2.system.xyz, s.xyz) and np.array_equal(lnv2.system.nfn, s.nfn)
    assert (lnv2.system.lattice is None) == (s.lattice is None)
    assert lnv2.info(True) == lnv.info(True) and lnv2.info(False) == lnv.info(False)
    for w in "LSH":
        assert np.array_equal(v2[w], vals[w])
        for a, b in zip(lnv2.patterns[w].export(), lnv.patterns[w].export()):
            assert np.array_equal(a, b)
    # a subset of the matrices is fine
    lsdm.save_checkpoint(tmp_path / "l_only.npz", lnv, {"L": vals["L"]})
    _, v3 = lsdm.load_checkpoint(tmp_path / "l_only.npz")
    assert set(v3) == {"L"} and np.array_equal(v3["L"], vals["L"])


def test_checkpoint_refuses_wrong_values_and_layouts(tmp_path):
    s = workloads.diamond(1)
    lnv, vals = _setup(s, 6.0, 8.0, 8.0, False)
    with pytest.raises(ValueError):
        lsdm.save_checkpoint(tmp_path / "bad.npz", lnv, {"L": vals["L"][:-1]})
    with pytest.raises(ValueError):
        lsdm.save_checkpoint(tmp_path / "bad.npz", lnv, {"X": vals["L"]})
    path = tmp_path / "lnv.npz"
    lsdm.save_checkpoint(path, lnv, vals)
    with np.load(path, allow_pickle=False) as f:
        data = {k: f[k] for k in f.files}
    data["col_L"] = data["col_L"][::-1].copy()      # a block layout this system does not produce
    np.savez(tmp_path / "tampered.npz", **data)
    with pytest.raises(ValueError):
        lsdm.load_checkpoint(tmp_path / "tampered.npz")
    data = dict(data, format=np.int64(99))
    np.savez(tmp_path / "future.npz", **data)
    with pytest.raises(ValueError):
        lsdm.load_checkpoint(tmp_path / "future.npz")
