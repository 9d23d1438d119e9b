"""Seeded synthetic inputs for the LNV block-sparse path.

This module makes geometries (diamond-silicon supercells, jittered copies of
them, random mixed-species boxes) and the seeded value laws of the overlap S,
Hamiltonian H and auxiliary density matrix L.  It is shared by the oracle side
and the GPU side as their only common code, so it holds none of the method's
arithmetic: no products, no truncation, no energies.

Value laws (the paper's workloads are bulk Si in cubic supercells, Results
section and Table 1; the per-block laws are a synthetic stand-in for the
CONQUEST Hamiltonian, which is not available):

* S and H: on-site blocks are the identity; every other block is
  exp(-r/2) * G with G an i.i.d. normal matrix of standard deviation 0.1.
  One member of each mirror pair {(i,j,n), (j,i,-n)} is drawn and the other is
  its transpose, so S and H are symmetric.
* L (a "0.5 S^-1"-like start): 0.5 * (2 I - S) on the S range (first Neumann
  term of S^-1, halved) plus an independent symmetric 0.5 * exp(-r/2) * G term
  on every off-site pair inside the L range.

Random numbers come from a counter-based hash (SplitMix64, Steele, Lea & Flood,
OOPSLA 2014) of (seed, matrix tag, canonical block key, element index) and the
Box-Muller transform, so a value does not depend on the order in which blocks
are enumerated or on who enumerated them.  Perfect crystals key blocks by
translation class (sublattice pair and integer cell offset), so the matrices are
translation invariant; jittered and random systems key blocks by atom pair and
image.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

BOHR_PER_ANGSTROM = 1.8897261

TAG_S, TAG_H, TAG_L, TAG_JITTER, TAG_POS, TAG_SPECIES, TAG_FD, TAG_DIR = 1, 2, 3, 4, 5, 6, 7, 8

# conventional diamond cell: fcc sites plus the same shifted by (1/4,1/4,1/4)
_FCC = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], dtype=np.float64)
DIAMOND_BASIS = np.concatenate([_FCC, _FCC + 0.25])


@dataclasses.dataclass
class System:
    """Atoms with orbital blocks.  Positions in bohr; lattice rows are the
    periodic translation vectors (None for an open cluster)."""
    xyz: np.ndarray                  # (n, 3) float64
    nfn: np.ndarray                  # (n,) int32, orbitals per atom
    lattice: Optional[np.ndarray]    # (3, 3) float64 rows, or None
    key_mode: str = "pair"           # "class" (perfect crystal) or "pair"
    cell: Optional[np.ndarray] = None     # (n, 3) int64 conventional cell of each atom
    sub: Optional[np.ndarray] = None      # (n,) int64 sublattice 0..7
    ncell: Optional[tuple] = None
    a: float = 0.0
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])


def diamond(ncell, a: float = 10.26, nfn: int = 4, jitter: float = 0.0, seed: int = 0,
            periodic: bool = True, key_mode: Optional[str] = None) -> System:
    """Diamond-structure supercell of ncell = (nx, ny, nz) conventional cells."""
    if np.isscalar(ncell):
        ncell = (int(ncell),) * 3
    nx, ny, nz = (int(v) for v in ncell)
    c = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1).reshape(-1, 3)
    cell = np.repeat(c, 8, axis=0).astype(np.int64)
    sub = np.tile(np.arange(8), c.shape[0]).astype(np.int64)
    xyz = (cell + DIAMOND_BASIS[sub]) * a
    lattice = np.diag([nx * a, ny * a, nz * a]).astype(np.float64) if periodic else None
    if jitter > 0.0:
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, TAG_JITTER])))
        xyz = xyz + rng.normal(0.0, jitter, size=xyz.shape)
        if periodic:
            xyz = np.mod(xyz, np.diag(lattice)[None, :])
    if key_mode is None:
        key_mode = "class" if jitter == 0.0 else "pair"
    return System(xyz=np.ascontiguousarray(xyz), nfn=np.full(xyz.shape[0], nfn, np.int32),
                  lattice=lattice, key_mode=key_mode, cell=cell, sub=sub, ncell=(nx, ny, nz), a=a,
                  name=f"diamond{nx}x{ny}x{nz}")


def random_box(n_atoms: int, edge: float, n_heavy: int, nfn_heavy: int = 13, nfn_light: int = 5,
               seed: int = 0) -> System:
    """Periodic cubic box with i.i.d. uniform positions and a random species
    assignment (exactly n_heavy atoms with nfn_heavy orbitals, the rest with
    nfn_light)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, TAG_POS])))
    xyz = rng.uniform(0.0, edge, size=(n_atoms, 3))
    rs = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, TAG_SPECIES])))
    nfn = np.full(n_atoms, nfn_light, np.int32)
    nfn[rs.permutation(n_atoms)[:n_heavy]] = nfn_heavy
    return System(xyz=np.ascontiguousarray(xyz), nfn=nfn, lattice=np.diag([edge] * 3).astype(np.float64),
                  key_mode="pair", name=f"random{n_atoms}")


def random_cluster(n_atoms: int, edge: float, nfn=4, seed: int = 0) -> System:
    """Open (non-periodic) cluster with uniform positions; nfn is an int or an
    array of per-atom orbital counts."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, TAG_POS])))
    xyz = rng.uniform(0.0, edge, size=(n_atoms, 3))
    nf = np.full(n_atoms, nfn, np.int32) if np.isscalar(nfn) else np.asarray(nfn, np.int32)
    return System(xyz=np.ascontiguousarray(xyz), nfn=nf, lattice=None, key_mode="pair",
                  name=f"cluster{n_atoms}")


def si_slab(ncell, a: float = 10.26, vacuum: float = 45.0, bond_h: float = 2.8, nfn_si: int = 4,
            nfn_h: int = 1) -> System:
    """Hydrogen-terminated (001) slab of diamond silicon: ncell = (nx, ny, nz)
    conventional cells, periodic in x and y, `vacuum` bohr of empty space along
    z, and one H atom (nfn_h functions) on every broken bond, `bond_h` bohr from
    its Si along the bulk bond direction.  Atoms near the surfaces have fewer
    neighbours within a range than bulk atoms."""
    nx, ny, nz = (int(v) for v in ncell)
    c = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1).reshape(-1, 3)
    cell = np.repeat(c, 8, axis=0).astype(np.int64)
    sub = np.tile(np.arange(8), c.shape[0]).astype(np.int64)
    si = (cell + DIAMOND_BASIS[sub]) * a
    # bulk bonds: from an fcc site along (1,1,1) and the vectors with two signs
    # flipped; from a shifted site along their negatives
    bonds = 0.25 * a * np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    top = nz * a
    hs = []
    for k in range(4):
        v = np.where((sub < 4)[:, None], bonds[k][None, :], -bonds[k][None, :])
        zn = si[:, 2] + v[:, 2]
        broken = (zn < -1e-9) | (zn > top - 0.25 * a + 1e-9)
        hs.append(si[broken] + (bond_h / np.sqrt(3.0) / (0.25 * a)) * v[broken])
    h = np.concatenate(hs)
    xyz = np.concatenate([si, h])
    xyz[:, 2] += 0.5 * vacuum                     # slab in the middle of the cell along z
    xyz[:, 0] = np.mod(xyz[:, 0], nx * a)
    xyz[:, 1] = np.mod(xyz[:, 1], ny * a)
    nfn = np.concatenate([np.full(si.shape[0], nfn_si, np.int32), np.full(h.shape[0], nfn_h, np.int32)])
    lattice = np.diag([nx * a, ny * a, nz * a + vacuum]).astype(np.float64)
    return System(xyz=np.ascontiguousarray(xyz), nfn=nfn, lattice=lattice, key_mode="pair",
                  name=f"si001slab{nx}x{ny}x{nz}_h")


# ---------------------------------------------------------------------------
# workloads: the five synthetic configurations (sizes from the paper's Table 1
# rows where they match: 4,096 and 32,768 atoms)
# ---------------------------------------------------------------------------
def _mixed_box_edge(n=8000, density_per_A3=0.05):
    return (n / density_per_A3) ** (1.0 / 3.0) * BOHR_PER_ANGSTROM


WORKLOADS = {
    "si64_rl12": dict(atoms=64, rS=8.0, rH=12.0, rL=12.0,
         make=lambda seed=0: diamond(2, seed=seed)),
    "si4096_rl12": dict(atoms=4096, rS=8.0, rH=12.0, rL=12.0,
         make=lambda seed=0: diamond(8, seed=seed)),
    "si13824_jitter_rl16": dict(atoms=13824, rS=8.0, rH=12.0, rL=16.0,
         make=lambda seed=0: diamond(12, jitter=0.1, seed=seed)),
    "si32768_rl16": dict(atoms=32768, rS=8.0, rH=12.0, rL=16.0,
         make=lambda seed=0: diamond(16, seed=seed)),
    "mixed8000_rl14": dict(atoms=8000, rS=10.0, rH=14.0, rL=14.0,
         make=lambda seed=0: random_box(8000, _mixed_box_edge(), 6400, 13, 5, seed=seed)),
    # surface-terminated, non-cubic cell: 16 x 16 x 8 conventional cells of Si
    # (16,384 atoms) with 2,048 H on the two (001) faces and 45 bohr of vacuum
    "si001slab18432_h_rl16": dict(atoms=18432, rS=8.0, rH=12.0, rL=16.0,
         make=lambda seed=0: si_slab((16, 16, 8))),
}


def workload(name: str, seed: int = 0):
    """The named workload: its system, ranges and size, as a dict."""
    c = dict(WORKLOADS[name])
    c["name"] = name
    c["system"] = c.pop("make")(seed)
    return c


# ---------------------------------------------------------------------------
# counter-based normal numbers
# ---------------------------------------------------------------------------
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    """SplitMix64 output function (Steele, Lea & Flood 2014)."""
    z = (z + _GOLDEN)
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _hash(*parts):
    with np.errstate(over="ignore"):
        h = np.uint64(0x243F6A8885A308D3)
        for p in parts:
            p = np.asarray(p).astype(np.int64).astype(np.uint64)
            h = _mix(h ^ p)
        return h


def _unit(h):
    """(0, 1) uniform from the top 53 bits."""
    return ((h >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def keyed_normal(seed, tag, *key):
    """Standard normal deviates, one per element of the broadcast key arrays."""
    with np.errstate(over="ignore"):
        h = _hash(seed, tag, *key)
        u1 = _unit(_mix(h ^ np.uint64(1)))
        u2 = _unit(_mix(h ^ np.uint64(2)))
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


# ---------------------------------------------------------------------------
# block keys
# ---------------------------------------------------------------------------
def _block_geometry(sysm: System, i, j, img):
    """Per block: distance r, canonical flag, canonical key tuple, self flag."""
    i = np.asarray(i, np.int64); j = np.asarray(j, np.int64); img = np.asarray(img, np.int64).reshape(-1, 3)
    if sysm.key_mode == "class":
        nc = np.asarray(sysm.ncell, np.int64)
        d = sysm.cell[j] + img * nc[None, :] - sysm.cell[i]
        sa, sb = sysm.sub[i], sysm.sub[j]
        vec = (d + DIAMOND_BASIS[sb] - DIAMOND_BASIS[sa]) * sysm.a
        r = np.sqrt((vec * vec).sum(1))
        D = 1 << 12
        fwd = ((sa * 8 + sb) * (2 * D + 1) + (d[:, 0] + D)) * (2 * D + 1)
        fwd = ((fwd + d[:, 1] + D) * (2 * D + 1)) + d[:, 2] + D
        bwd = ((sb * 8 + sa) * (2 * D + 1) + (-d[:, 0] + D)) * (2 * D + 1)
        bwd = ((bwd + -d[:, 1] + D) * (2 * D + 1)) - d[:, 2] + D
        is_self = fwd == bwd
        canon = fwd <= bwd
        k0 = np.where(canon, sa, sb); k1 = np.where(canon, sb, sa)
        kd = np.where(canon[:, None], d, -d)
        key = (k0, k1, kd[:, 0], kd[:, 1], kd[:, 2])
    else:
        if sysm.lattice is None and np.any(img != 0):
            raise ValueError("open system has only the zero image")
        K = 257
        fwd = ((i * (1 << 20) + j) * K + img[:, 0] + 128) * K * K + (img[:, 1] + 128) * K + img[:, 2] + 128
        bwd = ((j * (1 << 20) + i) * K - img[:, 0] + 128) * K * K + (-img[:, 1] + 128) * K - img[:, 2] + 128
        is_self = fwd == bwd
        canon = fwd <= bwd
        k0 = np.where(canon, i, j); k1 = np.where(canon, j, i)
        kn = np.where(canon[:, None], img, -img)
        key = (k0, k1, kn[:, 0], kn[:, 1], kn[:, 2])
        # distance from the canonical orientation, so a block and its mirror agree bit for bit
        shift = np.zeros((i.size, 3)) if sysm.lattice is None else kn.astype(np.float64) @ sysm.lattice
        vec = sysm.xyz[k1] + shift - sysm.xyz[k0]
        r = np.sqrt((vec * vec).sum(1))
    return r, canon, key, is_self


def _expand(nfn, i, j):
    """Flat element arrays for blocks (i,j) laid out block after block, each
    block row-major nfn[i] x nfn[j]."""
    ni = nfn[i].astype(np.int64); nj = nfn[j].astype(np.int64)
    sz = ni * nj
    blk = np.repeat(np.arange(i.size, dtype=np.int64), sz)
    start = np.concatenate([[0], np.cumsum(sz)[:-1]]) if i.size else np.zeros(0, np.int64)
    e = np.arange(int(sz.sum()), dtype=np.int64) - np.repeat(start, sz)
    alpha = e // nj[blk]; beta = e % nj[blk]
    return blk, alpha, beta, ni[blk], nj[blk]


def _law_sh(sysm, seed, tag, i, j, img):
    r, canon, key, is_self = _block_geometry(sysm, i, j, img)
    blk, al, be, ni, nj = _expand(sysm.nfn, np.asarray(i, np.int64), np.asarray(j, np.int64))
    c = canon[blk]
    # element index inside the canonical block (the mirror block is its transpose)
    ecan = np.where(c, al * nj + be, be * ni + al)
    z = keyed_normal(seed, tag, *(k[blk] for k in key), ecan)
    v = np.exp(-0.5 * r[blk]) * 0.1 * z
    selfb = is_self[blk]
    return np.where(selfb, (al == be).astype(np.float64), v), r, blk, al, be, selfb


def block_values(sysm: System, which: str, i, j, img, seed: int = 0, rS: float = None,
                 chunk: int = 1 << 20) -> np.ndarray:
    """Values of matrix `which` in {"S","H","L"} for the blocks (i[b], j[b], img[b]),
    laid out block after block (row-major nfn_i x nfn_j).  rS is required for L."""
    i = np.asarray(i, np.int64); j = np.asarray(j, np.int64); img = np.asarray(img, np.int64).reshape(-1, 3)
    out = []
    for s in range(0, max(i.size, 1), chunk):
        sl = slice(s, min(s + chunk, i.size))
        if i[sl].size == 0:
            break
        if which in ("S", "H"):
            v, *_ = _law_sh(sysm, seed, TAG_S if which == "S" else TAG_H, i[sl], j[sl], img[sl])
        elif which == "L":
            if rS is None:
                raise ValueError("the L law needs the S range")
            sv, r, blk, al, be, selfb = _law_sh(sysm, seed, TAG_S, i[sl], j[sl], img[sl])
            in_s = (r * r <= rS * rS)[blk]
            delta = (selfb & (al == be)).astype(np.float64)
            base = np.where(in_s, 0.5 * (2.0 * delta - sv), 0.0)
            nv, *_ = _law_sh(sysm, seed, TAG_L, i[sl], j[sl], img[sl])
            noise = np.where(selfb, 0.0, 0.5 * nv)
            v = base + noise
        else:
            raise ValueError(which)
        out.append(v)
    return np.concatenate(out) if out else np.zeros(0)


def fd_blocks(n_blocks_total: int, count: int = 20, seed: int = 0) -> np.ndarray:
    """Indices of `count` distinct blocks chosen for finite-difference checks."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, TAG_FD])))
    return np.sort(rng.choice(n_blocks_total, size=min(count, n_blocks_total), replace=False))


def fd_direction(n_values: int, seed: int = 0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, TAG_DIR])))
    return rng.normal(0.0, 1.0, size=n_values)
