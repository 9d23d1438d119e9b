"""MI355X-native hot path of the LNV linear-scaling density-matrix method.

A thin binding of the HIP library liblsdm.so (C ABI in include/lsdm.h):
range patterns, truncated atom-blocked products, the LNV density matrix
K = 3LSL - 2LSLSL, the energy E = 2 Tr(KH) and dE/dL.  Arguments are
marshalled here; every step of the computation runs in the library's kernels.
PyTorch tensors supply device memory and the current stream.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import BF16, FP32, FP32_RC, FP64, LsdmError, check, lib

__all__ = ["System", "Pattern", "Plan", "LNV", "multiply", "multiply_adjoint", "dot",
           "FP64", "FP32", "BF16", "FP32_RC", "LsdmError", "LNVEnergy"]

PREC = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "fp32_rc": FP32_RC}


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if isinstance(a, np.ndarray) else ctypes.c_void_p(a)


def _dev(t, n=None, what="tensor"):
    """Device pointer of a contiguous float64 CUDA tensor (optionally of n elements)."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous float64 tensor on the GPU")
    if n is not None and t.numel() != n:
        raise ValueError(f"{what} has {t.numel()} values, the pattern has {n}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _prec(p):
    return PREC[p] if isinstance(p, str) else int(p)


class System:
    """Atoms with orbital blocks: positions (n, 3) in bohr, orbitals per atom,
    optional lattice (3, 3) whose rows are the periodic translations."""

    def __init__(self, xyz, nfn, lattice=None):
        xyz = np.ascontiguousarray(xyz, np.float64)
        nfn = np.ascontiguousarray(nfn, np.int32)
        if xyz.ndim != 2 or xyz.shape[1] != 3 or nfn.shape != (xyz.shape[0],):
            raise ValueError("xyz must be (n, 3) and nfn (n,)")
        lat = None if lattice is None else np.ascontiguousarray(lattice, np.float64).reshape(9)
        h = ctypes.c_void_p()
        check(lib().lsdm_system_create(xyz.shape[0], _ptr(xyz), _ptr(nfn), None if lat is None else _ptr(lat),
                                       ctypes.byref(h)))
        self._h = h
        self._destroy = lib().lsdm_system_destroy
        self.n = xyz.shape[0]
        self.nfn = nfn.copy()
        self.xyz = xyz.copy()
        self.lattice = None if lat is None else lat.reshape(3, 3).copy()

    @classmethod
    def from_workload(cls, sysm):
        return cls(sysm.xyz, sysm.nfn, sysm.lattice)

    def __del__(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None


class Pattern:
    """Range pattern (blocks within a distance); owned, or borrowed from an LNV."""

    def __init__(self, system, R=None, _borrowed=None, _owner=None):
        self.system = system
        if _borrowed is not None:
            self._h, self._own, self._owner = _borrowed, False, _owner
        else:
            h = ctypes.c_void_p()
            check(lib().lsdm_pattern_create(system._h, float(R), ctypes.byref(h)))
            self._h, self._own = h, True
            self._destroy = lib().lsdm_pattern_destroy
        nb, nv = ctypes.c_int64(), ctypes.c_int64()
        check(lib().lsdm_pattern_info(self._h, ctypes.byref(nb), ctypes.byref(nv)))
        self.n_blocks, self.n_values = nb.value, nv.value
        self._exp = None

    def export(self):
        """(row_ptr, col, img (nb, 3), val_off) on the host."""
        if self._exp is None:
            rp = np.zeros(self.system.n + 1, np.int64)
            col = np.zeros(self.n_blocks, np.int32)
            img = np.zeros((self.n_blocks, 3), np.int8)
            off = np.zeros(self.n_blocks, np.int64)
            check(lib().lsdm_pattern_export(self._h, _ptr(rp), _ptr(col), _ptr(img), _ptr(off)))
            self._exp = (rp, col, img, off)
        return self._exp

    def keys(self):
        """(i, j, img) of every block, in value-layout order."""
        rp, col, img, _ = self.export()
        return np.repeat(np.arange(self.system.n, dtype=np.int64), np.diff(rp)), col.astype(np.int64), img.astype(np.int64)

    def __del__(self):
        if getattr(self, "_own", False) and getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None


class Plan:
    """Task list of C = P_C(op(A) op(B))."""

    def __init__(self, A, transA, B, transB, C):
        h = ctypes.c_void_p()
        check(lib().lsdm_plan_create(A._h, int(transA), B._h, int(transB), C._h, ctypes.byref(h)))
        self._h = h
        self._destroy = lib().lsdm_plan_destroy
        self.A, self.B, self.C = A, B, C
        nt, fl, nb = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
        check(lib().lsdm_plan_info(h, ctypes.byref(nt), ctypes.byref(fl), ctypes.byref(nb)))
        self.n_triples, self.flops, self.plan_bytes = nt.value, fl.value, nb.value

    def __del__(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocators = []   # every pair ever set stays alive: buffers keep the allocator that made them


def set_allocator(alloc=None, release=None):
    """Route the library's device workspaces through alloc(nbytes) -> device
    pointer (int; None or 0 for failure) and release(ptr) (lsdm_set_allocator);
    no arguments restores hipMalloc.  Handles made while a pair is set give
    their workspaces back through it when destroyed, so destroy them before
    the interpreter shuts down (the pair's Python functions may be gone by
    then)."""
    if (alloc is None) != (release is None):
        raise ValueError("set_allocator needs both alloc and release, or neither")
    if alloc is None:
        check(lib().lsdm_set_allocator(None, None, None))
        return
    a = _ALLOC_FN(lambda n, ctx: alloc(int(n)) or None)
    f = _FREE_FN(lambda ptr, ctx: release(int(ptr)))
    _allocators.append((a, f))
    check(lib().lsdm_set_allocator(ctypes.cast(a, ctypes.c_void_p), ctypes.cast(f, ctypes.c_void_p), None))


def use_torch_allocator():
    """set_allocator with torch's caching allocator (current device and stream)."""
    import torch
    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n), torch.cuda.caching_allocator_delete)


def multiply(plan, A, B, C, alpha=1.0, beta=0.0, prec="fp64", stream=None):
    """C = alpha P_C(op(A) op(B)) + beta C (device tensors in block layout)."""
    check(lib().lsdm_multiply(plan._h, _prec(prec), float(alpha), _dev(A, plan.A.n_values, "A"),
                              _dev(B, plan.B.n_values, "B"), float(beta), _dev(C, plan.C.n_values, "C"),
                              _stream(stream)))
    return C


def multiply_adjoint(plan, Cbar, A, B, Abar=None, Bbar=None, prec="fp64", stream=None):
    """Abar += P_A(Cbar op(B)^T), Bbar += P_B(op(A)^T Cbar) (either may be None)."""
    check(lib().lsdm_multiply_adjoint(plan._h, _prec(prec), _dev(Cbar, plan.C.n_values, "Cbar"),
                                      _dev(A, plan.A.n_values, "A"), _dev(B, plan.B.n_values, "B"),
                                      _dev(Abar, plan.A.n_values, "Abar"), _dev(Bbar, plan.B.n_values, "Bbar"),
                                      _stream(stream)))
    return Abar, Bbar


def dot(pattern, A, B, out=None, stream=None, noalloc=False):
    """sum over pattern blocks of <A_b, B_b> as a one-element device tensor.
    Asynchronous; its partial sums live on the pattern (allocated on the
    first call).  noalloc=True: the variant that allocates nothing, not even on
    its first call (its partial sums sit in the library's static scratch;
    concurrent calls on one device race), for graph capture and serving loops."""
    import torch
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=A.device)
    fn = lib().lsdm_dot_noalloc if noalloc else lib().lsdm_dot
    check(fn(pattern._h, _dev(A, pattern.n_values, "A"), _dev(B, pattern.n_values, "B"),
             _dev(out, 1, "out"), _stream(stream)))
    return out


class LNV:
    """Patterns and plans of the LNV chain for ranges rS, rH, rL."""

    NAMES = ("S", "H", "L", "X", "M")

    SYMMETRIC = 1

    def __init__(self, system, rS, rH, rL, symmetric=False):
        """symmetric=True: L, S and H are symmetric (every L passed later too);
        M, P and the X^T H X term of dE/dL are then computed on one half and
        mirrored, and dE/dL is assembled as V + V^T - 4 X^T H X with
        V = 6 HX - 4 HMS (the gradient's terms, regrouped)."""
        h = ctypes.c_void_p()
        check(lib().lsdm_lnv_create_ex(system._h, float(rS), float(rH), float(rL),
                                       self.SYMMETRIC if symmetric else 0, ctypes.byref(h)))
        self.symmetric = bool(symmetric)
        self._h = h
        self._destroy = lib().lsdm_lnv_destroy
        self.system = system
        self.rS, self.rH, self.rL = rS, rH, rL
        self.patterns = {}
        for w, name in enumerate(self.NAMES):
            ph = ctypes.c_void_p()
            check(lib().lsdm_lnv_pattern(h, w, ctypes.byref(ph)))
            self.patterns[name] = Pattern(system, _borrowed=ph, _owner=self)

    def info(self, grad=True):
        nt, fl = ctypes.c_int64(), ctypes.c_double()
        check(lib().lsdm_lnv_info(self._h, int(grad), ctypes.byref(nt), ctypes.byref(fl)))
        return nt.value, fl.value

    def energy(self, L, S, H, prec="fp64", want_K=False, E=None, stream=None):
        import torch
        p = self.patterns
        E = torch.empty(1, dtype=torch.float64, device=L.device) if E is None else E
        K = torch.empty(p["H"].n_values, dtype=torch.float64, device=L.device) if want_K else None
        check(lib().lsdm_lnv_energy(self._h, _prec(prec), _dev(L, p["L"].n_values, "L"), _dev(S, p["S"].n_values, "S"),
                                    _dev(H, p["H"].n_values, "H"), _dev(K), _dev(E, 1, "E"), _stream(stream)))
        return (E, K) if want_K else E

    def energy_grad(self, L, S, H, prec="fp64", E=None, G=None, stream=None):
        import torch
        p = self.patterns
        E = torch.empty(1, dtype=torch.float64, device=L.device) if E is None else E
        G = torch.empty(p["L"].n_values, dtype=torch.float64, device=L.device) if G is None else G
        check(lib().lsdm_lnv_energy_grad(self._h, _prec(prec), _dev(L, p["L"].n_values, "L"),
                                         _dev(S, p["S"].n_values, "S"), _dev(H, p["H"].n_values, "H"),
                                         _dev(E, 1, "E"), _dev(G, p["L"].n_values, "G"), _stream(stream)))
        return E, G

    def line(self, L, D, S, H, h=1.0, prec="fp64", stream=None):
        """Coefficients c0..c3 of E(L + tD) (numpy array, exact cubic)."""
        p = self.patterns
        c = np.zeros(4)
        check(lib().lsdm_lnv_line(self._h, _prec(prec), _dev(L, p["L"].n_values, "L"), _dev(D, p["L"].n_values, "D"),
                                  _dev(S, p["S"].n_values, "S"), _dev(H, p["H"].n_values, "H"), float(h), _ptr(c),
                                  _stream(stream)))
        return c

    def minimise(self, L, S, H, max_iter=20, gtol=1e-8, h0=1.0, prec="fp64", stream=None):
        """Conjugate-gradient minimisation of E over L in place; returns
        (energies, gradient norms) per step, the first entry for the start."""
        p = self.patterns
        Eh = np.zeros(max_iter + 1); gh = np.zeros(max_iter + 1); it = ctypes.c_int(0)
        check(lib().lsdm_lnv_minimise(self._h, _prec(prec), _dev(L, p["L"].n_values, "L"),
                                      _dev(S, p["S"].n_values, "S"), _dev(H, p["H"].n_values, "H"), int(max_iter),
                                      float(gtol), float(h0), _ptr(Eh), _ptr(gh), ctypes.byref(it), _stream(stream)))
        return Eh[:it.value + 1], gh[:it.value + 1]

    def shift(self, S, H=None, mu=0.0, out=None, stream=None):
        """H - mu S on H's pattern (a new tensor unless `out` is given; H=None
        gives -mu S).  The chain's energy with it is 2 Tr[K(H - mu S)]."""
        import torch
        p = self.patterns
        out = torch.empty(p["H"].n_values, dtype=torch.float64, device=S.device) if out is None else out
        check(lib().lsdm_lnv_shift(self._h, -float(mu), _dev(S, p["S"].n_values, "S"), 1.0 if H is not None else 0.0,
                                   _dev(H, p["H"].n_values, "H") if H is not None else None,
                                   _dev(out, p["H"].n_values, "out"), _stream(stream)))
        return out

    def electrons(self, L, S, prec="fp64", grad=False, stream=None):
        """N_e = 2 Tr(KS) (tensor of one double), and dN_e/dL when grad=True."""
        import torch
        p = self.patterns
        N = torch.empty(1, dtype=torch.float64, device=L.device)
        G = torch.empty(p["L"].n_values, dtype=torch.float64, device=L.device) if grad else None
        check(lib().lsdm_lnv_electrons(self._h, _prec(prec), _dev(L, p["L"].n_values, "L"),
                                       _dev(S, p["S"].n_values, "S"), _dev(N, 1, "N"),
                                       _dev(G, p["L"].n_values, "G") if grad else None, _stream(stream)))
        return (N, G) if grad else N

    def purify(self, L, S, prec="fp64", out=None, stream=None):
        """One McWeeny step: 3 LSL - 2 LSLSL on L's pattern (a new tensor unless
        `out` is given)."""
        import torch
        p = self.patterns
        out = torch.empty(p["L"].n_values, dtype=torch.float64, device=L.device) if out is None else out
        check(lib().lsdm_lnv_purify(self._h, _prec(prec), _dev(L, p["L"].n_values, "L"), _dev(S, p["S"].n_values, "S"),
                                    _dev(out, p["L"].n_values, "out"), _stream(stream)))
        return out

    PRODUCTS = ("F1", "F2", "F3", "B1", "B2", "B3", "B4", "B5")

    def profile(self, enable=True):
        """Bracket every product launch with HIP events (see profile_read)."""
        check(lib().lsdm_lnv_profile(self._h, int(enable)))

    def profile_read(self):
        """{product: (summed ms, launches, useful flops per launch)} since the last read."""
        ms = np.zeros(8); n = np.zeros(8, np.int64); fl = np.zeros(8)
        check(lib().lsdm_lnv_profile_read(self._h, _ptr(ms), _ptr(n), _ptr(fl)))
        return {p: (float(ms[k]), int(n[k]), float(fl[k])) for k, p in enumerate(self.PRODUCTS)}

    def __del__(self):
        if getattr(self, "_h", None):
            self.patterns = {}
            self._destroy(self._h)
            self._h = None


from .autograd import LNVEnergy  # noqa: E402
from .checkpoint import load_checkpoint, save_checkpoint  # noqa: E402
