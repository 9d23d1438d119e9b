"""A-priori error bounds of the reduced-precision LNV chain, element by element.

Every GPU product C = alpha op(A) op(B) reads its operands rounded to the
input precision (unit roundoff ui: 2^-24 for FP32, 2^-8 for BF16) and sums n
terms in FP32.  With |A - A~| <= eA and |B - B~| <= eB already carried by its
operands, first-order error analysis (Higham, Accuracy and Stability of
Numerical Algorithms, sec. 3.1 and 3.5) gives, element by element on C's
pattern,

    |C~ - C| <= |alpha| (eA |B| + |A| eB + eA eB
                          + (2 ui + ui^2 + gamma_n (1 + ui)^2 + 2 u) (|A| + eA)(|B| + eB)),

gamma_n = n u / (1 - n u), u = 2^-24; the last 2u covers the scaling by alpha
and the rounding of the stored result.  The bounds are carried through the
chain exactly as each mode computes it (F1-F3, K and E in FP64; the adjoint
written out term by term, or in symmetric mode regrouped with Y = HX and the
halves mirrored), with the oracle's own products of absolute values.  FP32_RC
multiplies only off-site parts in FP32 and adds FP64 corrections, so the FP32
bound holds for it as well.
"""
import numpy as np

import oracle

U = 2.0 ** -24


def _m(p, v):
    return oracle.Matrix(p, v)


def chain_error_bounds(inp, rS, rH, rL, prec, symmetric):
    """(bound on |E~ - E|, element-wise bound on |dE/dL~ - dE/dL| on L's pattern)."""
    L, S, H = inp["L"], inp["S"], inp["H"]
    s = L.pattern.system
    R = oracle.chain_ranges(rS, rH, rL)
    pX, pM, pL, pH = oracle.pattern(s, R["X"]), oracle.pattern(s, R["M"]), L.pattern, H.pattern
    ui = 2.0 ** -8 if prec == "bf16" else U
    nfn_max = int(np.max(s.nfn))

    def mul(A, tA, B, tB, pC):
        return oracle.multiply_op(A, tA, B, tB, pC).val

    def prod(A, eA, tA, B, eB, tB, pC, alpha=1.0):
        """exact value and error bound of alpha op(A) op(B) on pC"""
        n = int(np.diff(A.pattern.row_ptr).max()) * nfn_max + 2
        gam = n * U / (1.0 - n * U)
        c = 2 * ui + ui * ui + gam * (1 + ui) ** 2 + 2 * U
        aA, aB = _m(A.pattern, np.abs(A.val)), _m(B.pattern, np.abs(B.val))
        EA, EB = _m(A.pattern, eA), _m(B.pattern, eB)
        AA, BB = _m(A.pattern, np.abs(A.val) + eA), _m(B.pattern, np.abs(B.val) + eB)
        e = abs(alpha) * (mul(EA, tA, aB, tB, pC) + mul(aA, tA, EB, tB, pC) + mul(EA, tA, EB, tB, pC)
                          + c * mul(AA, tA, BB, tB, pC))
        return _m(pC, alpha * mul(A, tA, B, tB, pC)), e

    def sym(p, e):
        """a result kept on one half and mirrored: each block carries the larger bound"""
        return np.maximum(e, oracle.transpose(_m(p, e), p).val)

    def onto(e, p_from, p_to):
        return oracle.project(_m(p_from, e), p_to).val

    z = lambda M: np.zeros_like(M.val)
    X, eX = prod(L, z(L), False, S, z(S), False, pX)
    M, eM = prod(X, eX, False, L, z(L), False, pM)
    if symmetric:
        eM = sym(pM, eM)
    P, eP = prod(X, eX, False, M, eM, False, pH)
    if symmetric:
        eP = sym(pH, eP)
    eK = 3 * onto(eM, pM, pH) + 2 * eP
    E = 2 * float(np.dot(3 * onto(M.val, pM, pH) - 2 * P.val, H.val))
    bE = 2 * float(np.dot(eK, np.abs(H.val))) + 1e-13 * abs(E)

    if not symmetric:
        Mb, eMb = prod(X, eX, True, H, z(H), False, pM, alpha=-4.0)
        Mb = _m(pM, Mb.val + 6.0 * onto(H.val, pH, pM))
        eMb = eMb + 6.0 * U * onto(np.abs(H.val), pH, pM) + 2 * U * np.abs(Mb.val)
        Xb, eXb = prod(H, z(H), False, M, eM, False, pX, alpha=-4.0)
        Xb2, eXb2 = prod(Mb, eMb, False, L, z(L), False, pX)
        Xb = _m(pX, Xb.val + Xb2.val)
        eXb = eXb + eXb2 + 2 * U * np.abs(Xb.val)
        Lb, eLb = prod(X, eX, True, Mb, eMb, False, pL)
        Lb2, eLb2 = prod(Xb, eXb, False, S, z(S), False, pL)
        G = Lb.val + Lb2.val
        eG = eLb + eLb2 + 2 * U * np.abs(G)
    else:
        Y, eY = prod(H, z(H), False, X, eX, False, pM)
        Xb, eXb = prod(H, z(H), False, M, eM, False, pX, alpha=-4.0)
        Lb, eLb = prod(X, eX, True, Y, eY, False, pL, alpha=-4.0)
        eLb = sym(pL, eLb)
        V1, eV1 = prod(Xb, eXb, False, S, z(S), False, pL)
        V = V1.val + 6.0 * onto(Y.val, pM, pL)
        eV = eV1 + 6.0 * onto(eY, pM, pL) + 2 * U * np.abs(V)
        Vt, eVt = oracle.transpose(_m(pL, V), pL).val, oracle.transpose(_m(pL, eV), pL).val
        G = Lb.val + V + Vt
        eG = eLb + eV + eVt + 2 * U * np.abs(G)
    return bE, eG
