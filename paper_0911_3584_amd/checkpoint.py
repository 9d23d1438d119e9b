"""Checkpoint and resume of an LNV calculation: the system (positions,
functions per atom, lattice), the ranges and mode of the handle, the block
keys of its S, H and L patterns and the value arrays (L, and S, H if given),
in one NPZ file read back without pickling.  Loading rebuilds the handle from
the system and ranges and checks that the rebuilt patterns have the saved
keys, so values are never paired with a different block layout."""
import numpy as np

FORMAT = 1
_WHICH = ("S", "H", "L")


def _host(x):
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    return np.ascontiguousarray(x, np.float64)


def save_checkpoint(path, lnv, values):
    """Write `lnv`'s system, ranges and mode and `values` ({"L": ..., "S": ...,
    "H": ...}, any subset; torch tensors or arrays in block layout) to `path`."""
    sysm = lnv.system
    out = {"format": np.int64(FORMAT), "xyz": sysm.xyz, "nfn": sysm.nfn,
           "lattice": np.zeros((0, 3)) if sysm.lattice is None else sysm.lattice,
           "ranges": np.array([lnv.rS, lnv.rH, lnv.rL], np.float64), "symmetric": np.int64(lnv.symmetric)}
    for w in _WHICH:
        rp, col, img, off = lnv.patterns[w].export()
        out[f"rp_{w}"], out[f"col_{w}"], out[f"img_{w}"] = rp, col, img
    for w, v in values.items():
        if w not in _WHICH:
            raise ValueError(f"unknown matrix {w!r}: checkpoints hold S, H and L")
        v = _host(v)
        if v.shape != (lnv.patterns[w].n_values,):
            raise ValueError(f"{w} has {v.size} values, its pattern {lnv.patterns[w].n_values}")
        out[f"val_{w}"] = v
    np.savez(path, **out)


def load_checkpoint(path, device=None):
    """(lnv, values) from `path`: the handle rebuilt from the saved system and
    ranges, and the saved value arrays (torch tensors on `device`, or numpy
    arrays when device is None)."""
    from . import LNV, System
    with np.load(path, allow_pickle=False) as f:
        if int(f["format"]) != FORMAT:
            raise ValueError(f"checkpoint format {int(f['format'])}, this library reads {FORMAT}")
        lat = f["lattice"]
        sysm = System(f["xyz"], f["nfn"], None if lat.size == 0 else lat)
        rS, rH, rL = (float(x) for x in f["ranges"])
        lnv = LNV(sysm, rS, rH, rL, symmetric=bool(int(f["symmetric"])))
        for w in _WHICH:
            rp, col, img, _ = lnv.patterns[w].export()
            if not (np.array_equal(rp, f[f"rp_{w}"]) and np.array_equal(col, f[f"col_{w}"])
                    and np.array_equal(img, f[f"img_{w}"])):
                raise ValueError(f"the rebuilt {w} pattern differs from the saved one")
        vals = {w: f[f"val_{w}"].copy() for w in _WHICH if f"val_{w}" in f.files}
    if device is not None:
        import torch
        vals = {w: torch.from_numpy(v).to(device) for w, v in vals.items()}
    return lnv, vals
