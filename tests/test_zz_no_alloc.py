"""The dot that allocates nothing (lsdm_dot_noalloc, for callers that cannot
call hipMalloc: graph capture, serving loops) against lsdm_dot through the C
ABI: two calls in a row, the second on a smaller pattern, each equal to
lsdm_dot's result bit for bit (the same kernels and the same fixed grid), which
is held to the oracle's compensated sum."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_0911_3584_amd as lsdm  # noqa: E402

DEV = "cuda:0"


def _abi_dot(fn, pattern, a, b, out):
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    lsdm.check(fn(pattern._h, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                  ctypes.c_void_p(out.data_ptr()), stream))


def test_dot_noalloc_equals_dot_twice():
    L = lsdm.lib()
    for step, (s, R) in enumerate(((workloads.diamond(3), 16.0), (workloads.diamond(2), 8.0))):
        print(f"[no-alloc dot] call {step}: {s.n} atoms, range {R}", flush=True)
        gs = lsdm.System.from_workload(s)
        p = lsdm.Pattern(gs, R)
        rng = np.random.default_rng(40 + step)
        a, b = rng.standard_normal(p.n_values), rng.standard_normal(p.n_values)
        da, db = torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV)
        ref = torch.zeros(1, dtype=torch.float64, device=DEV)
        got = torch.full((1,), np.nan, dtype=torch.float64, device=DEV)
        _abi_dot(L.lsdm_dot, p, da, db, ref)
        _abi_dot(L.lsdm_dot_noalloc, p, da, db, got)
        torch.cuda.synchronize()
        assert got.item() == ref.item(), (got.item(), ref.item())
        exact = oracle.dot(a, b)
        assert abs(got.item() - exact) <= 1e-13 * np.sum(np.abs(a * b))
