"""GPU: the Tikhonov variants (tGKT_p on the tGKB space, t-LanczosTik_p on the t-Lanczos space,
nested_tGKT_p on the nested space of nested_tGKB_p, mu by bisection for the discrepancy equation)
against the FP64 oracle: k, mu, X, the residual at mu and the status, including intervals that
cannot meet the bound."""
import numpy as np
import pytest

from oracle import tikhonov as tk
from oracle import tproduct as tp
from paper_2110_02485_amd import workloads as wl
from tests.problems import blur_problem

pytestmark = pytest.mark.gpu


def _t(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=getattr(torch, dtype))


def _np(t):
    return t.detach().double().cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _check(out, orc, Xtol, mutol):
    import torch
    X, k, mu, res, status = out
    torch.cuda.synchronize()
    kg = [int(v) for v in k.cpu()]
    mug = mu.cpu().numpy()
    x_err = _rel(_np(X), wl.to_storage(orc["X"]))
    mu_err = float(np.max(np.abs(mug - orc["mu"]) / np.asarray(orc["mu"])))
    r_err = float(np.max(np.abs(res.cpu().numpy() - orc["res"]) / np.asarray(orc["res"])))
    print(f"[tikhonov] k {kg} vs {orc['k']}, mu {mug} vs {orc['mu']} (rel {mu_err:.2e}), X rel {x_err:.2e}, "
          f"residual rel {r_err:.2e}, status {int(status[0])} vs {orc['status']}", flush=True)
    assert kg == orc["k"] and int(status[0]) == orc["status"]
    assert mu_err <= mutol and x_err <= Xtol and r_err <= Xtol


@pytest.mark.parametrize("dtype,Xtol,mutol", [("float64", 1e-10, 1e-8), ("float32", 1e-5, 1e-4)])
def test_tgkt_blur_two_slices(dtype, Xtol, mutol):
    from paper_2110_02485_amd import rtsvd as rt
    A, X, B, Om, delta = blur_problem(48, 16, 2.0, 6, 2, 1e-2, 20, 0, seed=31, video=True)
    Am, Bm, Xm = wl.to_math(A), wl.to_math(B), wl.to_math(X)
    E = Bm - tp.tprod(Am, Xm)
    deltas = [float(np.linalg.norm(E[:, j, :])) for j in range(2)]
    orc = tk.tgkt_restore(Am, Bm, deltas, 1.1, 20, 1e-2, 1e7)
    _check(rt.tgkt_solve(_t(A, dtype), _t(B, dtype), deltas, 1.1, 20, 1e-2, 1e7), orc, Xtol, mutol)


@pytest.mark.parametrize("dtype,Xtol,mutol", [("float64", 1e-10, 1e-8), ("float32", 1e-5, 1e-4)])
def test_tlanczos_tik_symmetric_blur(dtype, Xtol, mutol):
    from paper_2110_02485_amd import rtsvd as rt
    A, X, B, Om, delta = blur_problem(48, 16, 2.0, 6, 2, 1e-2, 20, 0, seed=33, video=True, symmetric=True)
    Am, Bm, Xm = wl.to_math(A), wl.to_math(B), wl.to_math(X)
    E = Bm - tp.tprod(Am, Xm)
    deltas = [float(np.linalg.norm(E[:, j, :])) for j in range(2)]
    orc = tk.tlanczos_tik_restore(Am, Bm, deltas, 1.1, 20, 1e-2, 1e7)
    _check(rt.tlanczos_tik_solve(_t(A, dtype), _t(B, dtype), deltas, 1.1, 20, 1e-2, 1e7), orc, Xtol, mutol)


def test_tikhonov_interval_that_cannot_meet_the_bound():
    from paper_2110_02485_amd import rtsvd as rt
    A, X, B, Om, delta = blur_problem(32, 8, 2.0, 5, 1, 1e-2, 10, 0, seed=35)
    Am, Bm = wl.to_math(A), wl.to_math(B)
    orc = tk.tgkt_restore(Am, Bm, delta, 1.1, 10, 1e-6, 1e-4)
    assert orc["status"] == tk.DP_NOT_MET and orc["mu"] == [1e-4]
    _check(rt.tgkt_solve(_t(A, "float64"), _t(B, "float64"), delta, 1.1, 10, 1e-6, 1e-4), orc, 1e-10, 1e-12)


def test_tgkt_256_fp32():
    # the 256 x 256 x 256 blur at relative noise 1e-2 (k = 7), mu on the paper's [1e1, 1e7]
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    w = wl.WORKLOADS["blur256n2"]
    A, X, E0, Om = wl.make_inputs(w)
    Am, Xm = wl.to_math(A), wl.to_math(X)
    Bt = tp.tprod(Am, Xm)
    E = wl.scale_noise(wl.to_math(E0), Bt, w.noise)
    Bm = Bt + E
    delta = float(np.linalg.norm(E))
    orc = tk.tgkt_restore(Am, Bm, delta, w.eta, w.k_max, 1e1, 1e7)
    _check(rt.tgkt_solve(_t(A, "float32"), _t(wl.to_storage(Bm), "float32"), delta, w.eta, w.k_max, 1e1, 1e7),
           orc, 1e-5, 1e-4)


# nested_tGKT_p: Tikhonov on the nested space of nested_tGKB_p (one basis from B_1)
@pytest.mark.parametrize("dtype,Xtol,mutol", [("float64", 1e-10, 1e-8), ("float32", 1e-5, 1e-4)])
def test_nested_tgkt_video_slices(dtype, Xtol, mutol):
    from paper_2110_02485_amd import rtsvd as rt
    A, X, B, Om, delta = blur_problem(48, 16, 2.0, 6, 4, 1e-2, 20, 0, seed=37, video=True)
    Am, Bm, Xm = wl.to_math(A), wl.to_math(B), wl.to_math(X)
    E = Bm - tp.tprod(Am, Xm)
    deltas = [float(np.linalg.norm(E[:, j, :])) for j in range(4)]
    orc = tk.nested_tgkt_restore(Am, Bm, deltas, 1.1, 20, 1e-2, 1e7)
    _check(rt.nested_tgkt_solve(_t(A, dtype), _t(B, dtype), deltas, 1.1, 20, 2, 1e-2, 1e7), orc, Xtol, mutol)


def test_nested_tgkt_ragged_k_init_and_unmet_interval():
    # 5 slices of a random problem with odd n and k_init = 1, then an interval of tiny mu: slice 1
    # (which started the basis) cannot reach its bound (mu_hi, DP_NOT_MET); for some of the others
    # even y = 0 leaves a projected residual ||Q_{k+1}^T * B_j|| below the bound (mu_lo)
    from paper_2110_02485_amd import rtsvd as rt
    rng = np.random.default_rng(39)
    l, m, n, p = 21, 17, 7, 5
    A = rng.standard_normal((n, m, l))
    B = rng.standard_normal((n, p, l))
    Am, Bm = wl.to_math(A), wl.to_math(B)
    deltas = [fr * float(np.linalg.norm(Bm[:, j, :])) for j, fr in enumerate([0.45, 0.6, 0.5, 0.55, 0.65])]
    orc = tk.nested_tgkt_restore(Am, Bm, deltas, 1.05, 12, 1e-3, 1e5, k_init=1)
    _check(rt.nested_tgkt_solve(_t(A, "float64"), _t(B, "float64"), deltas, 1.05, 12, 1, 1e-3, 1e5), orc, 1e-10,
           1e-8)
    orc2 = tk.nested_tgkt_restore(Am, Bm, deltas, 1.05, 12, 1e-9, 1e-7, k_init=1)
    assert orc2["status"] == tk.DP_NOT_MET and orc2["mu"][0] == 1e-7 and set(orc2["mu"]) == {1e-7, 1e-9}
    _check(rt.nested_tgkt_solve(_t(A, "float64"), _t(B, "float64"), deltas, 1.05, 12, 1, 1e-9, 1e-7), orc2, 1e-10,
           1e-12)
