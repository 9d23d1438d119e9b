"""FP64 CPU oracle for the LNV block-sparse hot path.

TEST INFRASTRUCTURE.  Only `tests/`, `__graft_entry__.smoke()` and the
`cpu_baseline` leg of `bench.py` may import this package.  It shares no code
with the GPU library (`paper_0911_3584_amd`); the only common code is the
seeded input generator `workloads`, which holds none of the method's
arithmetic.

What it computes (Bowler & Miyazaki, section 2 "Methodology"):

* range patterns: atom-pair blocks kept when the interatomic distance is at most
  the range (the cutoff on L stated after eq. 3; eq. 1 and eq. 2 give the
  (atom, support function) indexing that makes matrices atom-blocked);
* truncated products C = P_C(op(A) op(B)): the exact product projected on C's
  range pattern (matrix multiplication, item 1 of the list of operations);
* the LNV (McWeeny) density matrix of eq. 3, K = 3 LSL - 2 LSLSL, on H's range;
* the energy E = 2 Tr(KH) with the spin factor of the electron count
  N_e = 2 Tr(KS) (constraint 2 of the ground-state search), N_e itself, the
  shifted Hamiltonian H - mu S of a chemical potential, and one McWeeny step
  L -> 3 LSL - 2 LSLSL on L's range;
* dE/dL on L's range, by the analytic formula
  6 (HLS + SLH) - 4 (HLSLS + SLHLS + SLSLH) evaluated through an evaluation
  order different from the forward chain;
* the minimisation of E over L (the ground-state search of section 2): the
  coefficients of the cubic E(L + tD), expanded term by term from eq. 3, and a
  conjugate-gradient loop whose steps go to the cubic's local minimum.

Readings where the paper is silent are listed in the design notes; the ones that
shape this code: intermediate ranges follow the "needed range" rule
(X = LS on R_L + R_S, LSL on min(2 R_L + R_S, R_H + R_L + R_S), LSLSL on R_H), so
no truncation changes E or dE/dL; periodic systems are image-resolved infinite
crystals; the gradient is taken with respect to each stored block.

Every function works on a subset of rows ("present" rows), so single rows of a
32,768-atom system can be computed through their dependency cone.  A product
whose needed input row is absent raises instead of returning a wrong value.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libref_core.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle's C++ core with g++ (OpenMP, FP64, -O2, no fast-math)."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "ref_core.cpp")
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                               src, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.ref_pairs.argtypes = [i64, P, P, ctypes.c_double, i64, P, P, P, P, P]
        lib.ref_pairs.restype = ctypes.c_int
        pat = [P] * 6
        lib.ref_multiply.argtypes = [i64, P] + pat * 3 + [P]
        lib.ref_multiply.restype = ctypes.c_int
        lib.ref_multiply_nt.argtypes = [i64, P] + pat * 3 + [P]
        lib.ref_multiply_nt.restype = ctypes.c_int
        lib.ref_transpose.argtypes = [i64, P] + pat * 2
        lib.ref_transpose.restype = ctypes.c_int
        lib.ref_project.argtypes = [i64, P] + pat * 2
        lib.ref_project.restype = ctypes.c_int
        lib.ref_dot.argtypes = [i64, P, P]
        lib.ref_dot.restype = ctypes.c_double
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# patterns and matrices
# ---------------------------------------------------------------------------
@dataclass
class Pattern:
    """Block-CSR pattern of one range over the atoms of a system: row i holds
    the blocks (i, col, img) sorted by (col, img); block b's values start at
    off[b] and are nfn[i] x nfn[col] row-major."""
    system: object
    R: float
    row_ptr: np.ndarray   # (n+1,) int64
    col: np.ndarray       # (nb,) int32
    img: np.ndarray       # (nb, 3) int32
    off: np.ndarray       # (nb,) int64
    nval: int
    present: np.ndarray   # (n,) uint8

    @property
    def nblocks(self) -> int:
        return int(self.col.size)

    def rows_of_blocks(self) -> np.ndarray:
        return np.repeat(np.arange(self.row_ptr.size - 1, dtype=np.int64), np.diff(self.row_ptr))

    def keys(self):
        return self.rows_of_blocks(), self.col.astype(np.int64), self.img.astype(np.int64)

    def _args(self):
        return [_p(self.row_ptr), _p(self.col), _p(self.img), _p(self.off), _p(self.present)]


@dataclass
class Matrix:
    pattern: Pattern
    val: np.ndarray       # (nval,) float64

    def block(self, b: int) -> np.ndarray:
        p = self.pattern
        i = int(np.searchsorted(p.row_ptr, b, side="right") - 1)
        ni, nj = int(p.system.nfn[i]), int(p.system.nfn[p.col[b]])
        return self.val[p.off[b]:p.off[b] + ni * nj].reshape(ni, nj)

    def _args(self):
        return self.pattern._args() + [_p(self.val)]


def pattern(sysm, R: float, rows=None) -> Pattern:
    """Range pattern: all (i, j, n) with |x_j + n T - x_i| <= R, for the given
    rows (all rows if None).  Rows not listed are empty and not present."""
    if not (R >= 0.0) or not np.isfinite(R):
        raise ValueError("range must be finite and non-negative")
    n = sysm.n
    xyz = np.ascontiguousarray(sysm.xyz, np.float64)
    if not np.all(np.isfinite(xyz)):
        raise ValueError("non-finite positions")
    lat = None if sysm.lattice is None else np.ascontiguousarray(sysm.lattice, np.float64)
    rows = np.arange(n, dtype=np.int64) if rows is None else np.unique(np.asarray(rows, np.int64))
    counts = np.zeros(rows.size, np.int64)
    lib = _L()
    lib.ref_pairs(n, _p(xyz), _p(lat), float(R), rows.size, _p(rows), None, _p(counts), None, None)
    rp_rows = np.zeros(rows.size + 1, np.int64)
    np.cumsum(counts, out=rp_rows[1:])
    col = np.zeros(int(rp_rows[-1]), np.int32)
    img = np.zeros((int(rp_rows[-1]), 3), np.int32)
    lib.ref_pairs(n, _p(xyz), _p(lat), float(R), rows.size, _p(rows), _p(rp_rows[:-1].copy()), _p(counts),
                  _p(col), _p(img))
    full_counts = np.zeros(n, np.int64)
    full_counts[rows] = counts
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(full_counts, out=row_ptr[1:])
    # rows were filled in increasing row order, which is the CSR order
    present = np.zeros(n, np.uint8)
    present[rows] = 1
    nfn = np.asarray(sysm.nfn, np.int64)
    bi = np.repeat(np.arange(n, dtype=np.int64), full_counts)
    sz = nfn[bi] * nfn[col]
    off = np.zeros(col.size, np.int64)
    if col.size:
        np.cumsum(sz[:-1], out=off[1:])
    return Pattern(sysm, float(R), row_ptr, col, img, off, int(sz.sum()), present)


def zeros(p: Pattern) -> Matrix:
    return Matrix(p, np.zeros(p.nval, np.float64))


def ball(sysm, rows, R: float) -> np.ndarray:
    """Atoms within R of any listed atom (through any lattice image)."""
    p = pattern(sysm, R, rows)
    return np.unique(np.concatenate([np.unique(p.col).astype(np.int64), np.asarray(rows, np.int64)]))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"{what}: input row {-rc - 1} is not present (dependency cone too small)")


def multiply(A: Matrix, B: Matrix, pC: Pattern, out: Optional[Matrix] = None, count: bool = False):
    """P_C(A B) on the present rows of pC (accumulated into `out` if given)."""
    C = zeros(pC) if out is None else out
    nt = np.zeros(1, np.int64)
    sysm = pC.system
    nfn = np.ascontiguousarray(sysm.nfn, np.int32)
    rc = _L().ref_multiply(sysm.n, _p(nfn), *A._args(), *B._args(), *C._args(), _p(nt))
    _check(rc, "multiply")
    return (C, int(nt[0])) if count else C


def multiply_nt(A: Matrix, B: Matrix, pC: Pattern, out: Optional[Matrix] = None, count: bool = False):
    """P_C(A B^T) on the present rows of pC: needs rows i of A and rows j of B
    for the blocks (i, j, n) of pC only."""
    C = zeros(pC) if out is None else out
    nt = np.zeros(1, np.int64)
    sysm = pC.system
    nfn = np.ascontiguousarray(sysm.nfn, np.int32)
    rc = _L().ref_multiply_nt(sysm.n, _p(nfn), *A._args(), *B._args(), *C._args(), _p(nt))
    _check(rc, "multiply_nt")
    return (C, int(nt[0])) if count else C


def transpose(A: Matrix, pT: Pattern) -> Matrix:
    """A^T on the present rows of pT: block (i,j,n) = block (j,i,-n) of A, transposed."""
    T = zeros(pT)
    sysm = pT.system
    nfn = np.ascontiguousarray(sysm.nfn, np.int32)
    _check(_L().ref_transpose(sysm.n, _p(nfn), *A._args(), *T._args()), "transpose")
    return T


def project(A: Matrix, pQ: Pattern) -> Matrix:
    """P_Q(A): A's blocks that lie in Q's pattern (zero where A has none)."""
    Q = zeros(pQ)
    sysm = pQ.system
    nfn = np.ascontiguousarray(sysm.nfn, np.int32)
    _check(_L().ref_project(sysm.n, _p(nfn), *A._args(), *Q._args()), "project")
    return Q


def dot(a: np.ndarray, b: np.ndarray) -> float:
    """Compensated (Neumaier) sum of a[k] b[k], sequential."""
    a = np.ascontiguousarray(a, np.float64); b = np.ascontiguousarray(b, np.float64)
    assert a.shape == b.shape
    return float(_L().ref_dot(a.size, _p(a), _p(b)))


def row_slice(M: Matrix, i: int) -> np.ndarray:
    p = M.pattern
    s = p.off[p.row_ptr[i]] if p.row_ptr[i] < p.nblocks else p.nval
    e = p.off[p.row_ptr[i + 1]] if p.row_ptr[i + 1] < p.nblocks else p.nval
    return M.val[s:e]


# ---------------------------------------------------------------------------
# ranges used by the chain ("needed range" reading)
# ---------------------------------------------------------------------------
def chain_ranges(rS: float, rH: float, rL: float) -> dict:
    rX = rL + rS
    rM = min(2.0 * rL + rS, rH + rL + rS)
    return dict(S=rS, H=rH, L=rL, X=rX, M=rM, P=rH,
                A2=rL + rH, Y=min(rL + rX, rX + rH))


# ---------------------------------------------------------------------------
# inputs on the oracle's own patterns
# ---------------------------------------------------------------------------
def make_inputs(sysm, rS, rH, rL, seed=0, rows_L=None, rows_S=None, rows_H=None):
    """S, H, L from the seeded value laws on the oracle's own patterns."""
    import workloads
    out = {}
    for name, R, rows in (("S", rS, rows_S), ("H", rH, rows_H), ("L", rL, rows_L)):
        p = pattern(sysm, R, rows)
        i, j, img = p.keys()
        v = workloads.block_values(sysm, name, i, j, img, seed=seed, rS=rS)
        out[name] = Matrix(p, np.ascontiguousarray(v))
    return out


# ---------------------------------------------------------------------------
# the LNV chain: eq. 3 and E = 2 Tr(KH)
# ---------------------------------------------------------------------------
def energy_cone(sysm, rS, rH, rL, rows):
    """Rows of L, S, H needed for K on `rows`."""
    R = chain_ranges(rS, rH, rL)
    xr = ball(sysm, rows, rH)                 # X rows: the K rows and their H neighbours
    lr = np.union1d(xr, ball(sysm, rows, R["X"]))
    sr = ball(sysm, xr, rL)
    return dict(X=xr, L=lr, S=sr, H=np.asarray(rows, np.int64))


def lnv_energy(L: Matrix, S: Matrix, H: Matrix, rS, rH, rL, rows=None, literal: bool = False) -> dict:
    """Forward chain X = LS, M = LSL, P = LSLSL (on H's range), K = 3M - 2P on
    H's range and E = 2 <K, H>.  With `rows`, K and the row energies are
    computed for those rows only and E is their sum.

    P is taken as M X^T, which is LSLSL when L and S are symmetric.  With
    literal=True it is taken as M (S L) instead, which is eq. 3 for any L
    (used to differentiate eq. 3 along non-symmetric directions)."""
    sysm = L.pattern.system
    R = chain_ranges(rS, rH, rL)
    rows = np.arange(sysm.n) if rows is None else np.unique(np.asarray(rows, np.int64))
    xr = ball(sysm, rows, rH) if rows.size < sysm.n else rows
    X = multiply(L, S, pattern(sysm, R["X"], xr))                 # X = L S
    M = multiply(X, L, pattern(sysm, R["M"], rows))               # M = X L = LSL
    pH = pattern(sysm, rH, rows)
    if literal:
        SL = multiply(S, L, pattern(sysm, R["X"], ball(sysm, rows, R["M"]) if rows.size < sysm.n else None))
        P = multiply(M, SL, pH)                                   # P = (LSL)(SL)
    else:
        P = multiply_nt(M, X, pH)                                 # P = M X^T = LSLSL on H's range
    MH = project(M, pH)
    K = Matrix(pH, 3.0 * MH.val - 2.0 * P.val)                   # eq. 3
    Hr = project(H, pH)
    E = 2.0 * dot(K.val, Hr.val)                                  # E = 2 Tr(KH), H symmetric
    prod = K.val * Hr.val
    starts = pH.off[pH.row_ptr[rows]] if pH.nblocks else np.zeros(rows.size, np.int64)
    e_rows = 2.0 * np.add.reduceat(prod, starts) if prod.size else np.zeros(rows.size)
    return dict(E=E, K=K, X=X, M=M, P=P, rows=rows, e_rows=e_rows)


def gradient_cone(sysm, rS, rH, rL, rows):
    R = chain_ranges(rS, rH, rL)
    rows = np.asarray(rows, np.int64)
    J1 = ball(sysm, rows, rL)
    J2 = ball(sysm, J1, rH)
    xr = np.union1d(np.union1d(J2, ball(sysm, J2, R["X"])), ball(sysm, rows, R["Y"]))
    return dict(J1=J1, J2=J2, X=xr, L=xr, S=ball(sysm, xr, rL),
                H=np.union1d(np.union1d(J1, J2), ball(sysm, rows, R["X"])))


def lnv_gradient(L: Matrix, S: Matrix, H: Matrix, rS, rH, rL, rows=None) -> Matrix:
    """dE/dL on L's range: G = 6 (HLS + SLH) - 4 (HLSLS + SLHLS + SLSLH),
    for symmetric L, S, H.  Evaluation order, independent of the forward chain:
    X = LS, A1 = HX, A2 = XX, A3 = H A2, Y = X^T H, A4 = Y X,
    G = 6 (A1 + A1^T) - 4 (A3 + A3^T + A4)."""
    sysm = L.pattern.system
    R = chain_ranges(rS, rH, rL)
    allrows = rows is None
    rows = np.arange(sysm.n) if allrows else np.unique(np.asarray(rows, np.int64))
    if allrows:
        J1 = J2 = xr = rows
    else:
        c = gradient_cone(sysm, rS, rH, rL, rows)
        J1, J2, xr = c["J1"], c["J2"], c["X"]
    pL_rows = pattern(sysm, rL, rows)
    X = multiply(L, S, pattern(sysm, R["X"], xr))                          # LS
    A1 = multiply(H, X, pattern(sysm, rL, J1))                             # HLS on L's range
    A2 = multiply(X, X, pattern(sysm, R["A2"], J2))                        # LSLS on R_L + R_H
    A3 = multiply(H, A2, pattern(sysm, rL, J1))                            # HLSLS on L's range
    XT = transpose(X, pattern(sysm, R["X"], rows))                         # SL
    Y = multiply(XT, H, pattern(sysm, R["Y"], rows))                       # SLH
    A4 = multiply(Y, X, pL_rows)                                           # SLHLS on L's range
    A1T = transpose(A1, pL_rows)
    A3T = transpose(A3, pL_rows)
    A1r = project(A1, pL_rows)
    A3r = project(A3, pL_rows)
    G = 6.0 * (A1r.val + A1T.val) - 4.0 * (A3r.val + A3T.val + A4.val)
    return Matrix(pL_rows, G)


# ---------------------------------------------------------------------------
# adjoint of one truncated product (plain definition)
# ---------------------------------------------------------------------------
def multiply_op(A: Matrix, transA: bool, B: Matrix, transB: bool, pC: Pattern) -> Matrix:
    """P_C(op(A) op(B)) with op = transpose when the flag is set (transposes
    materialised on patterns of the operand's own range)."""
    sysm = pC.system
    if transA:
        A = transpose(A, pattern(sysm, A.pattern.R))
    if transB:
        return multiply_nt(A, B, pC)
    return multiply(A, B, pC)


def multiply_adjoint(A: Matrix, transA: bool, B: Matrix, transB: bool, Cbar: Matrix):
    """For C = P_C(op(A) op(B)) and an upstream gradient Cbar on C's pattern:
    Abar = P_A(Cbar op(B)^T) (or P_A(op(B) Cbar^T) when A enters transposed) and
    Bbar = P_B(op(A)^T Cbar) (or P_B(Cbar^T op(A)) when B enters transposed)."""
    sysm = A.pattern.system
    pA, pB = pattern(sysm, A.pattern.R), pattern(sysm, B.pattern.R)
    CbT = transpose(Cbar, pattern(sysm, Cbar.pattern.R))
    opA = transpose(A, pattern(sysm, A.pattern.R)) if transA else A
    opB = transpose(B, pattern(sysm, B.pattern.R)) if transB else B
    opAT = A if transA else transpose(A, pattern(sysm, A.pattern.R))
    # op(B)^T is B itself when B enters transposed, else B^T (taken in the A B^T form)
    Abar = multiply(opB, CbT, pA) if transA else (multiply(Cbar, B, pA) if transB else multiply_nt(Cbar, B, pA))
    Bbar = multiply(CbT, opA, pB) if transB else multiply(opAT, Cbar, pB)
    return Abar, Bbar


# ---------------------------------------------------------------------------
# minimisation of E over L (section 2, the ground-state search)
# ---------------------------------------------------------------------------
def shift(H: Matrix, S: Matrix, mu: float) -> Matrix:
    """H - mu S on H's range: with it the energy 2 Tr[K(H - mu S)] = E - mu N_e
    is the grand potential at chemical potential mu (constraint 2 of section 2
    imposed through mu)."""
    return Matrix(H.pattern, H.val - mu * project(S, H.pattern).val)


def electron_number(L: Matrix, S: Matrix, rS, rH, rL) -> float:
    """N_e = 2 Tr(KS) (constraint 2 of section 2) with K of eq. 3 on H's range;
    Tr(KS) = sum over stored blocks of K_ij . S_ij for symmetric S."""
    pH = pattern(L.pattern.system, rH)
    K = lnv_energy(L, S, zeros(pH), rS, rH, rL)["K"]
    return 2.0 * dot(K.val, project(S, pH).val)


def mcweeny(L: Matrix, S: Matrix, rS, rL) -> Matrix:
    """One McWeeny step on L's range (eq. 3 as a map of L, section 2):
    P_L(3 LSL - 2 LSLSL), with X = LS on rL + rS and LSL on 2 rL + rS, the
    ranges an exact result on L's range needs."""
    sysm = L.pattern.system
    pL = pattern(sysm, rL)
    X = multiply(L, S, pattern(sysm, rL + rS))                   # X = LS
    M = multiply(X, L, pattern(sysm, 2 * rL + rS))               # LSL
    P = multiply(X, M, pL)                                       # LSLSL on L's range
    return Matrix(pL, 3.0 * project(M, pL).val - 2.0 * P.val)


def lnv_line_coeffs(L: Matrix, D: Matrix, S: Matrix, H: Matrix, rS, rH, rL) -> np.ndarray:
    """c0..c3 of E(L + tD) = c0 + c1 t + c2 t^2 + c3 t^3, expanded from eq. 3
    with L_t = L + tD (literal products, valid for any L and D on L's range):
      L_t S L_t       = LSL + t (LSD + DSL) + t^2 DSD
      L_t S L_t S L_t = LSLSL + t (LSLSD + LSDSL + DSLSL)
                        + t^2 (LSDSD + DSLSD + DSDSL) + t^3 DSDSD
    and E(t) = 2 <3 L_t S L_t - 2 L_t S L_t S L_t, H> on H's range."""
    sysm = L.pattern.system
    R = chain_ranges(rS, rH, rL)
    pX, pM, pH = pattern(sysm, R["X"]), pattern(sysm, R["M"]), pattern(sysm, rH)
    LS, DS = multiply(L, S, pX), multiply(D, S, pX)
    SL, SD = multiply(S, L, pX), multiply(S, D, pX)
    LSL, LSD, DSL, DSD = (multiply(LS, L, pM), multiply(LS, D, pM), multiply(DS, L, pM), multiply(DS, D, pM))

    def h(m):            # <m, H> on H's range, m on M's or H's range
        return dot(project(m, pH).val, project(H, pH).val)

    def five(a, b):      # <a b, H>, a on M's range, b on X's range
        return dot(multiply(a, b, pH).val, project(H, pH).val)

    c0 = 2.0 * (3.0 * h(LSL) - 2.0 * five(LSL, SL))
    c1 = 2.0 * (3.0 * (h(LSD) + h(DSL)) - 2.0 * (five(LSL, SD) + five(LSD, SL) + five(DSL, SL)))
    c2 = 2.0 * (3.0 * h(DSD) - 2.0 * (five(LSD, SD) + five(DSL, SD) + five(DSD, SL)))
    c3 = 2.0 * (-2.0 * five(DSD, SD))
    return np.array([c0, c1, c2, c3])


def cubic_step(c, h: float) -> float:
    """Step t > 0 to the local minimum of c1 t + c2 t^2 + c3 t^3 along a descent
    direction: the root of c1 + 2 c2 t + 3 c3 t^2 = 0 where the second
    derivative 2 c2 + 6 c3 t is positive; t = h when there is none."""
    c1, c2, c3 = float(c[1]), float(c[2]), float(c[3])
    disc = c2 * c2 - 3.0 * c1 * c3
    t = -1.0
    if disc >= 0.0 and c2 + np.sqrt(disc) > 0.0:
        t = -c1 / (c2 + np.sqrt(disc))
    if not (t > 0.0) or not np.isfinite(t):
        t = h
    return t


def lnv_minimise(L: Matrix, S: Matrix, H: Matrix, rS, rH, rL, max_iter: int, gtol: float = 0.0, h0: float = 1.0):
    """Polak-Ribiere conjugate gradients on E(L) (beta clipped at 0, restart on
    a non-descent direction), each step exact along its line (the cubic's
    local minimum, first trial scale h0, then the previous step).
    Returns (L_final, energies, gradient norms), the first entries at the start.
    For symmetric L, S, H the gradient stays symmetric."""
    L = Matrix(L.pattern, L.val.copy())
    G = lnv_gradient(L, S, H, rS, rH, rL)
    Es = [lnv_energy(L, S, H, rS, rH, rL)["E"]]
    gs = [np.sqrt(dot(G.val, G.val))]
    D = -G.val
    h = h0
    for _ in range(max_iter):
        if gs[-1] <= gtol:
            break
        c = lnv_line_coeffs(L, Matrix(L.pattern, D), S, H, rS, rH, rL)
        t = cubic_step(c, h)
        L = Matrix(L.pattern, L.val + t * D)
        Gn = lnv_gradient(L, S, H, rS, rH, rL)
        Es.append(lnv_energy(L, S, H, rS, rH, rL)["E"])
        beta = max(0.0, (dot(Gn.val, Gn.val) - dot(Gn.val, G.val)) / dot(G.val, G.val))
        D = -Gn.val + beta * D
        if dot(D, Gn.val) >= 0.0:
            D = -Gn.val
        G = Gn
        gs.append(np.sqrt(dot(G.val, G.val)))
        h = t
    return L, np.array(Es), np.array(gs)
