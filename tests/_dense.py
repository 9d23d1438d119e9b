"""Dense and scipy.sparse views of block matrices, for brute-force checks.

Open systems only (every block has image 0): the orbital index of atom i,
function a is off[i] + a with off the prefix sum of the orbital counts.
"""
import numpy as np
import scipy.sparse as sp


def orbital_offsets(nfn):
    off = np.zeros(len(nfn) + 1, np.int64)
    np.cumsum(np.asarray(nfn, np.int64), out=off[1:])
    return off


def block_coo(M, sysm=None):
    """(rows, cols, vals) of every stored element, in orbital indices."""
    p = M.pattern
    sysm = sysm or p.system
    nfn = np.asarray(sysm.nfn, np.int64)
    oo = orbital_offsets(nfn)
    bi, bj, _ = p.keys()
    ni, nj = nfn[bi], nfn[bj]
    sz = ni * nj
    blk = np.repeat(np.arange(bi.size), sz)
    # element e of block b sits at p.off[b] + e
    e = np.arange(int(sz.sum())) - np.repeat(np.concatenate([[0], np.cumsum(sz)[:-1]]), sz)
    r = oo[bi[blk]] + e // nj[blk]
    c = oo[bj[blk]] + e % nj[blk]
    vals = M.val[np.repeat(p.off, sz) + e]
    return r, c, vals


def to_dense(M):
    p = M.pattern
    if np.any(p.img != 0):
        raise ValueError("dense view needs an open system")
    n_orb = int(np.sum(p.system.nfn))
    D = np.zeros((n_orb, n_orb))
    r, c, v = block_coo(M)
    D[r, c] = v
    return D


def to_sparse(M):
    p = M.pattern
    if np.any(p.img != 0):
        raise ValueError("sparse view needs an open system")
    n_orb = int(np.sum(p.system.nfn))
    r, c, v = block_coo(M)
    return sp.csr_matrix((v, (r, c)), shape=(n_orb, n_orb))


def mask_dense(p):
    """Boolean orbital mask of a pattern (open system)."""
    n_orb = int(np.sum(p.system.nfn))
    D = np.zeros((n_orb, n_orb), bool)
    nfn = np.asarray(p.system.nfn, np.int64)
    oo = orbital_offsets(nfn)
    bi, bj, _ = p.keys()
    for a, b in zip(bi, bj):
        D[oo[a]:oo[a + 1], oo[b]:oo[b + 1]] = True
    return D


def from_dense(p, D):
    """Matrix values on pattern p taken from the dense array D."""
    import oracle
    nfn = np.asarray(p.system.nfn, np.int64)
    oo = orbital_offsets(nfn)
    bi, bj, _ = p.keys()
    v = np.zeros(p.nval)
    for b, (a, c) in enumerate(zip(bi, bj)):
        blk = D[oo[a]:oo[a + 1], oo[c]:oo[c + 1]]
        v[p.off[b]:p.off[b] + blk.size] = blk.ravel()
    return oracle.Matrix(p, v)
