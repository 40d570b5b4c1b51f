"""GPU: rtsvd_solve_noalloc (the library's fixed scratch array, no device allocation) against
rtsvd_solve on the same factor and data, on two calls in a row, the second with a smaller input,
and its size limit."""
import ctypes

import numpy as np
import pytest

from paper_2110_02485_amd import workloads as wl
from tests.problems import blur_problem

pytestmark = pytest.mark.gpu


def _t(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=getattr(torch, dtype))


@pytest.mark.parametrize("precision,dtype", [("fp64", "float64"), ("fp32", "float32"), ("mixed", "float32")])
def test_noalloc_solve_matches_solve(precision, dtype):
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    size, n, k_max, rho = 96, 32, 24, 8
    print(f"[no-alloc] {precision} l=m={size} n={n}", flush=True)
    A, X, B, Om, delta = blur_problem(size, n, 2.5, 8, 8, 1e-2, k_max, rho, seed=3, video=True)
    f = rt.factor(_t(A, dtype), k_max, rho, 1, precision, _t(Om, dtype))
    deltas = [delta / np.sqrt(8.0)] * 8
    for p, k_start in ((8, 1), (3, 0)):                 # second call: fewer slices, the experiments' rule
        Bp = _t(B[:, :p, :], dtype)
        dl = deltas[:p]
        ref = f.solve(Bp, dl, 1.01, k_start)
        got = f.solve(Bp, dl, 1.01, k_start, no_alloc=True)
        torch.cuda.synchronize()
        assert torch.equal(got.X, ref.X)
        assert torch.equal(got.k, ref.k) and torch.equal(got.resid, ref.resid)
        assert torch.equal(got.status, ref.status)
        assert torch.isfinite(got.X).all()
    # joint bound (n_delta = 1) through the raw C ABI with caller-owned outputs
    lib = rt.load()
    Bp = _t(B[:, :2, :], dtype)
    ref = f.solve(Bp, delta, 1.01)
    Xo = torch.empty_like(ref.X)
    k = torch.empty(1, dtype=torch.int32, device="cuda")
    res = torch.empty_like(ref.resid)
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    arr = (ctypes.c_double * 1)(delta)
    rc = lib.rtsvd_solve_noalloc(f._h, Bp.data_ptr(), 2, rt._dtype_code(Bp), arr, 1, 1.01, 1, Xo.data_ptr(),
                                 k.data_ptr(), res.data_ptr(), st.data_ptr(), rt._stream())
    torch.cuda.synchronize()
    assert rc >= 0
    assert torch.equal(Xo, ref.X) and torch.equal(k, ref.k) and torch.equal(res, ref.resid)


def test_noalloc_solve_rejects_sizes_beyond_its_scratch():
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    size, n, k_max, rho = 64, 16, 10, 4
    A, X, B, Om, delta = blur_problem(size, n, 2.0, 6, 1, 1e-2, k_max, rho, seed=1)
    f = rt.factor(_t(A, "float64"), k_max, rho, 0, "fp64", _t(Om, "float64"))
    p = 4096                                           # B-hat alone: 9 x 64 x 4096 x 16 B = 37.7 MB, X-hat as much
    Bbig = torch.zeros((n, p, size), dtype=torch.float64, device="cuda")
    with pytest.raises(rt.RtsvdError) as e:
        f.solve(Bbig, delta, 1.01, no_alloc=True)
    assert e.value.code == rt.E_UNSUPPORTED and "maximum" in str(e.value)
    # the ordinary solve takes it
    res = f.solve(Bbig, delta, 1.01)
    torch.cuda.synchronize()
    assert torch.isfinite(res.X).all()
