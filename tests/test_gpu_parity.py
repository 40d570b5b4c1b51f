"""GPU parity: the HIP path through the C ABI against the FP64 oracle on identical seeded inputs.

Tolerances: FP64 path 1e-12 (relative, Frobenius), FP32 path 1e-5, truncation indices equal.
"""
import numpy as np
import pytest

from oracle import tproduct as tp
from oracle import factor as fa
from oracle import solve as so
from paper_2110_02485_amd import workloads as wl
from tests.problems import blur_problem, random_problem

pytestmark = pytest.mark.gpu


def _t(a, dtype="float64"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=getattr(torch, dtype))


def _np(t):
    return t.detach().double().cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ---------------------------------------------------------------------------------------------
# t-products
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("l,m,p,n", [(5, 3, 2, 8), (37, 29, 3, 16), (64, 64, 1, 1), (33, 17, 4, 7),
                                     (130, 70, 5, 12), (300, 260, 2, 64), (8, 8, 1, 2)])
@pytest.mark.parametrize("dtype,tol", [("float64", 1e-12), ("float32", 2e-5)])
def test_tprod_and_adjoint(l, m, p, n, dtype, tol):
    from paper_2110_02485_amd import rtsvd as rt
    rng = np.random.default_rng(l * 1000 + m * 10 + n)
    A = rng.standard_normal((n, m, l))
    X = rng.standard_normal((n, p, m))
    Y = rng.standard_normal((n, p, l))
    C = _np(rt.tprod(_t(A, dtype), _t(X, dtype)))
    ref = wl.to_storage(tp.tprod(wl.to_math(A), wl.to_math(X)))
    assert _rel(C, ref) <= tol
    Bt = _np(rt.tprod_adjoint(_t(A, dtype), _t(Y, dtype)))
    ref = wl.to_storage(tp.tprod(tp.ttranspose(wl.to_math(A)), wl.to_math(Y)))
    assert _rel(Bt, ref) <= tol


# ---------------------------------------------------------------------------------------------
# R-tSVD restorations
# ---------------------------------------------------------------------------------------------
def _oracle_rtsvd(A, B, Om, delta, eta, k_max, q, k_start=1, per_slice=False, rho=None):
    return so.rtsvd_restore(wl.to_math(A), wl.to_math(B), wl.to_math(Om), delta, eta, k_max, q, k_start,
                            per_slice, rho)


def _gpu_rtsvd(A, B, Om, delta, eta, k_max, rho, q, precision, dtype, k_start=1):
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    f = rt.factor(_t(A, dtype), k_max, rho, q, precision, _t(Om, dtype))
    res = f.solve(_t(B, dtype), delta, eta, k_start)
    torch.cuda.synchronize()
    return f, res


def test_rtsvd_fp64_blur64():
    # the 64 x 64 x 16 FP64 workload: sigma 2, band 6, 5 blobs, noise 1e-2, k <= 20, rho = 10
    w = wl.WORKLOADS["blur64"]
    A, X, B, Om, delta = blur_problem(w.size, w.n, w.sigma, w.band, 1, w.noise, w.k_max, w.oversample)
    orc = _oracle_rtsvd(A, B, Om, delta, w.eta, w.k_max, 0)
    f, res = _gpu_rtsvd(A, B, Om, delta, w.eta, w.k_max, w.oversample, 0, "fp64", "float64")
    assert int(res.k[0]) == orc["k"] and int(res.status[0]) == orc["status"]
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-12
    np.testing.assert_allclose(_np(res.resid)[0], orc["res"][:, 0], rtol=1e-12)
    r, faces, eta, r_eps, sig, flags = f.info()
    np.testing.assert_allclose(sig, orc["factor"]["s"][:, :faces].T, rtol=1e-12, atol=1e-14 * sig.max())
    np.testing.assert_allclose(eta, fa.eta_prefix(wl.to_math(A), orc["factor"]["C"]), rtol=0,
                               atol=1e-12 * eta[0])
    assert flags == 0


@pytest.mark.parametrize("q", [0, 1, 2])
def test_rtsvd_fp64_random_ragged(q):
    # ragged sizes (not multiples of any tile), non-power-of-two tube length, several RHS
    l, m, n, p, k_max, rho = 45, 38, 6, 3, 9, 4
    A, B, Om = random_problem(l, m, n, p, k_max + rho, seed=q)
    delta = 0.6 * np.linalg.norm(B)
    orc = _oracle_rtsvd(A, B, Om, delta, 1.05, k_max, q)
    f, res = _gpu_rtsvd(A, B, Om, delta, 1.05, k_max, rho, q, "fp64", "float64")
    assert int(res.k[0]) == orc["k"]
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-11
    np.testing.assert_allclose(_np(res.resid)[0], orc["res"][:, 0], rtol=1e-11)


@pytest.mark.parametrize("r_cols,precision,tol", [(200, "fp64", 1e-10), (256, "fp64", 1e-10), (200, "fp32", 2e-5)])
def test_rtsvd_wide_sketch(r_cols, precision, tol):
    # sketch widths above 128: the Cholesky factor and its block-row inverse run from global
    # scratch (up to three tiles of an L^{-1} block row per wave; r = 256 is the largest r), and
    # the eigensolver takes its one-kernel path; q = 1, ragged l, several RHS
    l, m, n, p, rho = 271, 256, 4, 2, 10
    k_max = r_cols - rho
    A, B, Om = random_problem(l, m, n, p, r_cols, seed=r_cols)
    delta = 0.5 * np.linalg.norm(B)
    orc = _oracle_rtsvd(A, B, Om, delta, 1.05, k_max, 1)
    dt = "float64" if precision == "fp64" else "float32"
    f, res = _gpu_rtsvd(A, B, Om, delta, 1.05, k_max, rho, 1, precision, dt)
    r, faces, eta, r_eps, sig, flags = f.info()
    assert r == r_cols and flags == 0
    assert int(res.k[0]) == orc["k"]
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= tol
    kk = orc["k"]
    np.testing.assert_allclose(_np(res.resid)[0][:kk], orc["res"][:kk, 0], rtol=tol)


def test_rtsvd_per_slice_and_paper_mode():
    w = wl.WORKLOADS["blur64"]
    A, X, B, Om, delta = blur_problem(48, 10, 2.0, 6, 3, 1e-2, 12, 6, seed=3, video=True)
    Bm = wl.to_math(B)
    deltas = [0.01 * np.linalg.norm(Bm[:, j]) for j in range(3)]
    orc = _oracle_rtsvd(A, B, Om, deltas, 1.01, 12, 0, per_slice=True)
    f, res = _gpu_rtsvd(A, B, Om, deltas, 1.01, 12, 6, 0, "fp64", "float64")
    assert [int(v) for v in res.k.cpu()] == orc["k"]
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-11
    # experiments' rule: start at r - rho, search up to r
    orc = _oracle_rtsvd(A, B, Om, delta, 1.01, 12, 0, k_start=0, rho=6)
    res = f.solve(_t(B), delta, 1.01, 0)
    assert int(res.k[0]) == orc["k"] and int(res.k[0]) >= 12
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-11


@pytest.mark.parametrize("p", [16, 17, 24])
def test_rtsvd_per_slice_many_slices(p):
    # one discrepancy bound per lateral slice: up to 16 bounds ride in the selection kernel's
    # arguments, more come from device memory.  Slice-dependent levels (some met at small k, slice
    # 5 never met), search from k = 3; k per slice, status, X and residuals against the oracle
    A, X, B, Om, delta = blur_problem(48, 10, 2.0, 6, p, 1e-2, 14, 6, seed=p, video=True)
    Bm = wl.to_math(B)
    fac = [0.005 + 0.03 * ((7 * j) % 11) / 10.0 for j in range(p)]
    fac[5] = 1e-14
    deltas = [fac[j] * float(np.linalg.norm(Bm[:, j])) for j in range(p)]
    orc = _oracle_rtsvd(A, B, Om, deltas, 1.01, 14, 0, k_start=3, per_slice=True)
    f, res = _gpu_rtsvd(A, B, Om, deltas, 1.01, 14, 6, 0, "fp64", "float64", k_start=3)
    assert [int(v) for v in res.k.cpu()] == orc["k"]
    assert int(res.status[0]) == orc["status"] == 1
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-11
    got = _np(res.resid)
    for j in range(p):
        np.testing.assert_allclose(got[j][:14], orc["res"][:14, j], rtol=1e-10)


@pytest.mark.parametrize("q", [0, 1])
def test_rtsvd_fixed_precision_adaptive(q):
    # Alg. 6's fixed-precision rank: the factor keeps r_eps = first j with eta^[j] < eps^2 sketch
    # columns; the solve then searches k from r_eps - rho (experiments' rule).  eps is placed
    # midway (geometrically) between eta^[j0] and eta^[j0 - 1] of the oracle, far from a tie.
    A, X, B, Om, delta = blur_problem(56, 12, 2.0, 6, 1, 1e-2, 16, 8, seed=11)
    k_max, rho = 16, 8
    Am = wl.to_math(A)
    full = fa.rtsvd_block(Am, wl.to_math(Om), q)
    eta_o = fa.eta_prefix(Am, full["C"])
    j0 = 14
    eps = float(np.sqrt(np.sqrt(eta_o[j0] * eta_o[j0 - 1])))
    if q == 0:
        lit = fa.rtsvd_literal(Am, wl.to_math(Om), eps=eps)
        assert lit["Q"].shape[1] == j0
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    f = rt.factor(_t(A), k_max, rho, q, "fp64", _t(Om), eps=eps, adaptive=True)
    r, faces, eta, r_eps, sig, flags = f.info()
    assert r == j0 and r_eps == j0 and f.r == j0
    np.testing.assert_allclose(eta, eta_o[:j0 + 1], rtol=0, atol=1e-12 * eta_o[0])
    Om_j0 = np.ascontiguousarray(Om[:, :j0, :])
    orc = _oracle_rtsvd(A, B, Om_j0, delta, 1.01, k_max, q, k_start=0, rho=rho)
    np.testing.assert_allclose(sig, orc["factor"]["s"][:, :faces].T, rtol=1e-12, atol=1e-14 * sig.max())
    res = f.solve(_t(B), delta, 1.01, 0)
    torch.cuda.synchronize()
    assert int(res.k[0]) == orc["k"] and int(res.k[0]) >= j0 - rho
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-11
    # eps above eta^[1] everywhere: r_eps = 1; eps below every eta: the full r_max columns
    f1 = rt.factor(_t(A), k_max, rho, q, "fp64", _t(Om), eps=float(np.sqrt(eta_o[0])), adaptive=True)
    assert f1.info()[0] == 1
    f2 = rt.factor(_t(A), k_max, rho, q, "fp64", _t(Om), eps=float(np.sqrt(eta_o[-1]) * 0.5), adaptive=True)
    assert f2.info()[0] == k_max + rho


def test_rtsvd_dp_not_met_status():
    A, X, B, Om, delta = blur_problem(40, 8, 2.0, 6, 1, 1e-2, 8, 4, seed=4)
    f, res = _gpu_rtsvd(A, B, Om, 1e-12, 1.01, 8, 4, 0, "fp64", "float64")
    assert int(res.k[0]) == 8 and int(res.status[0]) == 1


def test_rtsvd_fp32_blur():
    A, X, B, Om, delta = blur_problem(96, 32, 3.0, 10, 2, 1e-2, 24, 8, seed=5, video=True)
    orc = _oracle_rtsvd(A, B, Om, delta, 1.01, 24, 0)
    f, res = _gpu_rtsvd(A, B, Om, delta, 1.01, 24, 8, 0, "fp32", "float32")
    assert int(res.k[0]) == orc["k"]
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-5


def test_ttsvd_fp64():
    A, X, B, Om, delta = blur_problem(40, 12, 2.0, 6, 1, 1e-2, 20, 0, seed=6)
    orc = so.tsvd_restore(wl.to_math(A), wl.to_math(B), delta, 1.01, 20)
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    f = rt.ttsvd_factor(_t(A), 20, "fp64")
    res = f.solve(_t(B), delta, 1.01, 1)
    torch.cuda.synchronize()
    assert int(res.k[0]) == orc["k"]
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-10


def _structured(l, m, n, svals, seed):
    """A with every Fourier face U_f diag(svals) V_f^H (conjugate-symmetric, so A is real)."""
    rng = np.random.default_rng(seed)
    ah = np.zeros((l, m, n), dtype=complex)
    for i in range(n // 2 + 1):
        cplx = 0 if i in (0, n // 2) or n == 1 else 1
        u, _ = np.linalg.qr(rng.standard_normal((l, m)) + 1j * cplx * rng.standard_normal((l, m)))
        v, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * cplx * rng.standard_normal((m, m)))
        face = (u * np.asarray(svals)[None, :]) @ v.conj().T
        ah[:, :, i] = face
        ah[:, :, (n - i) % n] = np.conj(face)
    return wl.to_storage(tp.ifft_tubes(ah))


def test_rtsvd_clustered_singular_values():
    # repeated singular values (clusters of 3, 2, 4, ...): the small eigensolver must return an
    # orthonormal basis inside each cluster; X_k is unique at cluster boundaries (k = 3, 5, 9)
    l, m, n = 40, 24, 6
    sv = np.array([9.0] * 3 + [5.0] * 2 + [2.0] * 4 + list(np.linspace(1.0, 0.05, m - 9)))
    A = _structured(l, m, n, sv, 11)
    rng = np.random.default_rng(12)
    B = rng.standard_normal((n, 2, l))
    Om = rng.standard_normal((n, m, m))  # r = m: the sketch spans everything
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    f = rt.factor(_t(A), 20, 4, 0, "fp64", _t(Om))
    r, faces, eta, r_eps, sig, flags = f.info()
    np.testing.assert_allclose(sig[:, :len(sv)], np.tile(sv, (faces, 1)), rtol=1e-12, atol=1e-12)
    ts = fa.tsvd(wl.to_math(A))
    T = so.coefficients_tsvd(ts, wl.to_math(B))
    for k in (3, 5, 9):
        ff = rt.factor(_t(A), k, m - k, 0, "fp64", _t(Om))
        res = ff.solve(_t(B), 1e30, 1.01, k)   # huge delta: k = k_start
        torch.cuda.synchronize()
        assert int(res.k[0]) == k
        ref = wl.to_storage(so.x_of_k(ts["V"], T, k))
        assert _rel(_np(res.X), ref) <= 1e-11


def test_ttsvd_fp32_256():
    # the T-tSVD comparator at l = m = 256 (packed eigenproblem larger than LDS -> global path)
    A, X, B, Om, delta = blur_problem(256, 8, 3.0, 10, 1, 1e-2, 60, 0, seed=7)
    orc = so.tsvd_restore(wl.to_math(A), wl.to_math(B), delta, 1.01, 60)
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    f = rt.ttsvd_factor(_t(A, "float32"), 60, "fp32")
    res = f.solve(_t(B, "float32"), delta, 1.01, 1)
    torch.cuda.synchronize()
    assert int(res.k[0]) == orc["k"]
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-5


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_face_groups_give_identical_factors(precision):
    # the per-face work split into 1, 2 or 3 concurrently issued face groups: every per-face
    # computation is the same, so factor and solution agree bit for bit
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    A, X, B, Om, delta = blur_problem(128, 32, 2.0, 8, 1, 1e-2, 20, 10, seed=61)
    dt = "float64" if precision == "fp64" else "float32"
    At, Bt, Omt = _t(A, dt), _t(B, dt), _t(Om, dt)
    outs = []
    for g in (1, 2, 3):
        f = rt.factor(At, 20, 10, 1, precision, Omt, face_groups=g)
        res = f.solve(Bt, delta, 1.01, 1)
        torch.cuda.synchronize()
        info = f.info()
        outs.append((_np(res.X), int(res.k[0]), info[2], info[4]))
        f.close()
    for X_, k_, eta_, sig_ in outs[1:]:
        assert k_ == outs[0][1]
        assert np.array_equal(X_, outs[0][0])
        assert np.array_equal(eta_, outs[0][2]) and np.array_equal(sig_, outs[0][3])


@pytest.mark.parametrize("precision", ["mixed"])
@pytest.mark.parametrize("size,n,r_cols,q", [(256, 16, 120, 1), (128, 32, 40, 1), (256, 8, 30, 0), (384, 4, 72, 2),
                                             (192, 8, 30, 1)])
def test_fused_packing_matches_separate_packing(precision, size, n, r_cols, q, monkeypatch):
    # mixed precision: Q = Y R^{-1} also writes Q (and Z) as the packed bf16 operand of the next
    # pass over A-hat; with RTSVD_PACK_FUSION=0 every pass packs its operand itself.  The packed
    # values are the same bf16 roundings, so factor and solution agree bit for bit (192 rows: not a
    # multiple of 128, every pass packs).
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    k_max = r_cols - 10
    A, X, B, Om, delta = blur_problem(size, n, 2.0, 8, 1, 1e-2, k_max, 10, seed=73)
    At, Bt, Omt = _t(A, "float32"), _t(B, "float32"), _t(Om, "float32")
    outs = []
    # fused first, each factor after releasing the library's buffer cache: a packed operand that a
    # fused product failed to write cannot be masked by a stale copy from an unfused run
    for mode in ("1", "0"):
        print(f"[pack fusion] {mode} {precision} size={size} n={n} r={r_cols} q={q}", flush=True)
        monkeypatch.setenv("RTSVD_PACK_FUSION", mode)
        for groups in (1, 3):
            torch.cuda.synchronize()
            rt.trim()
            f = rt.factor(At, k_max, 10, q, precision, Omt, face_groups=groups)
            res = f.solve(Bt, delta, 1.01, 1)
            torch.cuda.synchronize()
            info = f.info()
            outs.append((_np(res.X), int(res.k[0]), info[2], info[4]))
            f.close()
    for X_, k_, eta_, sig_ in outs[1:]:
        assert k_ == outs[0][1]
        assert np.array_equal(X_, outs[0][0])
        assert np.array_equal(eta_, outs[0][2]) and np.array_equal(sig_, outs[0][3])


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_restorations_in_flight_on_several_streams_match_sequential(precision):
    # independent restorations (three different problems, twice each) issued round robin on three
    # caller streams, one face group each, give the bits of the same restorations issued one after
    # another on one stream: a call's work and scratch stay on its own stream
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    from paper_2110_02485_amd import tune
    dt = "float64" if precision == "fp64" else "float32"
    probs = []
    for seed, noise in ((81, 1e-2), (82, 1e-3), (83, 3e-2)):
        A, X, B, Om, delta = blur_problem(128, 16, 2.0, 8, 1, noise, 20, 10, seed=seed)
        probs.append((_t(A, dt), _t(B, dt), _t(Om, dt), delta))
    torch.cuda.synchronize()

    def run(nstreams):
        streams = [torch.cuda.current_stream()] if nstreams == 1 else tune.caller_streams(nstreams)
        fs, outs = [], []
        for rep in range(2):
            for i, (At, Bt, Omt, delta) in enumerate(probs):
                with torch.cuda.stream(streams[(3 * rep + i) % nstreams]):
                    f = rt.factor(At, 20, 10, 1, precision, Omt, face_groups=1)
                    outs.append(f.solve(Bt, delta, 1.01, 1))
                fs.append(f)
        torch.cuda.synchronize()
        got = [(_np(o.X), int(o.k[0]), _np(o.resid)) for o in outs]
        for f in fs:
            f.close()
        return got

    print(f"[in flight] {precision}", flush=True)
    seq = run(1)
    par = run(3)
    for (X0, k0, r0), (X1, k1, r1) in zip(seq, par):
        assert k0 == k1
        assert np.array_equal(X0, X1) and np.array_equal(r0, r1)
    # the two repetitions of a problem agree as well
    for i in range(3):
        assert np.array_equal(seq[i][0], seq[i + 3][0])


@pytest.mark.parametrize("precision,r_cols", [("mixed", 30), ("mixed", 120), ("fp32", 120), ("fp64", 30)])
def test_sketch_tiles_give_identical_factors(precision, r_cols):
    # 1, 2, 4 or 8 sixteen-column MFMA tiles per workgroup in the factor's A-hat products: only the
    # work split changes (no sum changes order), so factor and solution agree bit for bit
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    k_max = r_cols - 10
    A, X, B, Om, delta = blur_problem(256, 16, 2.0, 8, 1, 1e-2, k_max, 10, seed=67)
    dt = "float64" if precision == "fp64" else "float32"
    At, Bt, Omt = _t(A, dt), _t(B, dt), _t(Om, dt)
    outs = []
    for tile in (0, 1, 2, 4, 8):
        print(f"[sketch_tile] {precision} r={r_cols} tile={tile}", flush=True)
        f = rt.factor(At, k_max, 10, 1, precision, Omt, sketch_tile=tile)
        res = f.solve(Bt, delta, 1.01, 1)
        torch.cuda.synchronize()
        info = f.info()
        outs.append((_np(res.X), int(res.k[0]), info[2], info[4]))
        f.close()
    for X_, k_, eta_, sig_ in outs[1:]:
        assert k_ == outs[0][1]
        assert np.array_equal(X_, outs[0][0])
        assert np.array_equal(eta_, outs[0][2]) and np.array_equal(sig_, outs[0][3])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_captured_in_a_graph_replays_like_eager(precision):
    # rtsvd_solve keeps k, residuals and status on the device and launches kernels only, so after a
    # warm-up on the capturing stream (the workspace cache is per stream) it can be captured once and
    # replayed for new data in the same input buffer; every replay equals an eager solve bit for bit
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    A, X, B, Om, delta = blur_problem(64, 16, 2.0, 6, 2, 1e-2, 20, 10, seed=71, video=True)
    dt = "float64" if precision == "fp64" else "float32"
    f = rt.factor(_t(A, dt), 20, 10, 1, precision, _t(Om, dt))
    rng = np.random.default_rng(72)
    inputs = [B + 0.01 * np.abs(B).max() * rng.standard_normal(B.shape) for _ in range(3)]
    deltas = [0.02 * float(np.linalg.norm(B[:, j])) for j in range(2)]
    eager = []
    for Bi in inputs:
        r = f.solve(_t(Bi, dt), deltas, 1.01, 1)
        torch.cuda.synchronize()
        eager.append((_np(r.X), r.k.cpu().numpy().copy(), _np(r.resid), int(r.status[0])))
    s = torch.cuda.Stream()
    Bbuf = _t(inputs[0], dt).clone()
    with torch.cuda.stream(s):
        out = f.solve(Bbuf, deltas, 1.01, 1)
        f.solve(Bbuf, deltas, 1.01, 1, out=out)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        f.solve(Bbuf, deltas, 1.01, 1, out=out)
    torch.cuda.synchronize()
    for rep in range(2):
        for i, Bi in enumerate(inputs):
            Bbuf.copy_(_t(Bi, dt))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            Xe, ke, re, se = eager[i]
            assert np.array_equal(out.k.cpu().numpy(), ke), (rep, i)
            assert int(out.status[0]) == se
            assert np.array_equal(_np(out.X), Xe), (rep, i)
            assert np.array_equal(_np(out.resid), re), (rep, i)
            # eager work between replays
            r = f.solve(_t(inputs[(i + 1) % 3], dt), deltas, 1.01, 1)
            torch.cuda.synchronize()
            assert np.array_equal(_np(r.X), eager[(i + 1) % 3][0])
    f.close()


# ---------------------------------------------------------------------------------------------
# symmetric A: T-tEVD and t-Lanczos_p
# ---------------------------------------------------------------------------------------------
def _sym_storage(m, n, seed, shift=0.0):
    """Storage-order random t-symmetric tensor S + S^T (+ shift I on the first frontal slice)."""
    s = np.random.default_rng(seed).standard_normal((m, m, n))
    a = s + tp.ttranspose(s)
    a[:, :, 0] += shift * np.eye(m)
    return wl.to_storage(a)


def _check_eigs(f, orc_factor, faces, tol):
    # stored sigma = |eigenvalues| by decreasing magnitude, face by face
    sig = f.info()[4]
    d = np.abs(orc_factor["d"])
    for i in range(faces):
        np.testing.assert_allclose(sig[i], d[:, i], rtol=tol, atol=tol * d[0, i])


def test_ttevd_symmetric_blur_fp64():
    from oracle import symmetric as sy
    A, X, B, Om, delta = blur_problem(40, 12, 2.0, 6, 1, 1e-2, 20, 0, seed=21, symmetric=True)
    orc = sy.tevd_restore(wl.to_math(A), wl.to_math(B), delta, 1.01, 20)
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    f = rt.ttevd_factor(_t(A), 20, "fp64")
    res = f.solve(_t(B), delta, 1.01, 1)
    torch.cuda.synchronize()
    assert int(res.k[0]) == orc["k"]
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-10
    np.testing.assert_allclose(_np(res.resid)[0, :orc["k"]], orc["res"][:orc["k"], 0], rtol=1e-9)
    _check_eigs(f, orc["factor"], 7, 1e-10)


def test_ttevd_nearly_singular_faces_fp64():
    # the symmetric blur with the wide tube (sigma_c = 2): its DFT falls to 4e-5 of the largest
    # face, so 85 of the 640 face eigenvalues (times the blur's own small ones) lie below the
    # pseudo-inverse tolerance sqrt(4 r eps) max |d| (r = m here, every eigenvalue kept on both
    # sides); the GPU's k, X and residuals must follow the oracle's reading of diag(d)^{-1}
    from oracle import symmetric as sy
    m, n = 40, 16
    A = wl.blur_operator(m, n, 2.0, 6, sigma_c=2.0, symmetric=True)
    Am = wl.to_math(A)
    fo = sy.tevd(Am)
    ad = np.abs(fo["d"])
    assert (ad <= so.pinv_cut(ad)).sum() > 50     # many eigenvalues below the tolerance
    rx = wl.rng_for("parity", "xtrue", 41)
    X = wl.lateral_slices(wl.blob_image(m, n, rx)[None])
    Bt = tp.tprod(Am, wl.to_math(X))
    E = wl.scale_noise(wl.noise_direction(Bt.shape, wl.rng_for("parity", "noise", 41)), Bt, 1e-3)
    Bm = Bt + E
    delta = float(np.linalg.norm(E))
    orc = sy.tevd_restore(Am, Bm, delta, 1.01, m)
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    f = rt.ttevd_factor(_t(A), m, "fp64")
    res = f.solve(_t(wl.to_storage(Bm)), delta, 1.01, 1)
    torch.cuda.synchronize()
    assert int(res.k[0]) == orc["k"]
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-9
    kk = orc["k"]
    np.testing.assert_allclose(_np(res.resid)[0, :kk], orc["res"][:kk, 0], rtol=1e-9)


def test_ttevd_indefinite_per_slice_odd_n():
    # random t-symmetric A with eigenvalues of both signs, odd n, two slices with their own k
    from oracle import symmetric as sy
    A = _sym_storage(24, 7, 22)
    B = np.random.default_rng(23).standard_normal((7, 2, 24))
    Bm = wl.to_math(B)
    deltas = [0.5 * np.linalg.norm(Bm[:, 0]), 0.2 * np.linalg.norm(Bm[:, 1])]
    orc = sy.tevd_restore(wl.to_math(A), Bm, deltas, 1.01, 24, per_slice=True)
    assert orc["k"][0] != orc["k"][1]
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    f = rt.ttevd_factor(_t(A), 24, "fp64")
    res = f.solve(_t(B), deltas, 1.01, 1)
    torch.cuda.synchronize()
    assert [int(v) for v in res.k.cpu()] == orc["k"]
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-10
    _check_eigs(f, orc["factor"], 4, 1e-10)


def test_ttevd_fp32_256():
    # m = 256: the eigenproblem takes the eigensolver's global-memory path
    from oracle import symmetric as sy
    A, X, B, Om, delta = blur_problem(256, 8, 3.0, 9, 1, 1e-2, 60, 0, seed=24, symmetric=True)
    orc = sy.tevd_restore(wl.to_math(A), wl.to_math(B), delta, 1.01, 60)
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    f = rt.ttevd_factor(_t(A, "float32"), 60, "fp32")
    res = f.solve(_t(B, "float32"), delta, 1.01, 1)
    torch.cuda.synchronize()
    assert int(res.k[0]) == orc["k"]
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-5


def _gpu_tlanczos(A, B, delta, eta, k_max, dtype):
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    X, k, resid, status = rt.tlanczos_solve(_t(A, dtype), _t(B, dtype), delta, eta, k_max)
    torch.cuda.synchronize()
    return X, k, resid, status


@pytest.mark.parametrize("dtype,tol", [("float64", 1e-10), ("float32", 1e-4)])
def test_tlanczos_symmetric_blur(dtype, tol):
    from oracle import symmetric as sy
    A, X, B, Om, delta = blur_problem(64, 16, 2.0, 6, 1, 1e-2, 20, 0, seed=25, symmetric=True)
    orc = sy.tlanczos_restore(wl.to_math(A), wl.to_math(B), delta, 1.01, 30)
    Xg, k, resid, status = _gpu_tlanczos(A, B, delta, 1.01, 30, dtype)
    assert [int(v) for v in k.cpu()] == orc["k"] and int(status[0]) == orc["status"]
    assert _rel(_np(Xg), wl.to_storage(orc["X"])) <= tol
    kk = orc["k"][0]
    np.testing.assert_allclose(_np(resid)[0, :kk], orc["res"][:kk, 0], rtol=max(tol, 1e-9))


def test_tlanczos_indefinite_slices_ragged():
    # indefinite t-symmetric A, odd n, 5 slices (more than the 4 per product launch), a never-met
    # bound: k per slice, X, residuals and status vs the oracle
    from oracle import symmetric as sy
    A = _sym_storage(33, 7, 26, shift=2.0)
    B = np.random.default_rng(27).standard_normal((7, 5, 33))
    Am, Bm = wl.to_math(A), wl.to_math(B)
    deltas = [f * np.linalg.norm(Bm[:, j]) for j, f in enumerate([0.9, 0.5, 0.3, 1e-13, 0.7])]
    orc = sy.tlanczos_restore(Am, Bm, deltas, 1.01, 12)
    assert orc["status"] == sy.DP_NOT_MET
    Xg, k, resid, status = _gpu_tlanczos(A, B, deltas, 1.01, 12, "float64")
    assert [int(v) for v in k.cpu()] == orc["k"] and int(status[0]) == orc["status"]
    assert _rel(_np(Xg), wl.to_storage(orc["X"])) <= 1e-10
    for j, kj in enumerate(orc["k"]):
        np.testing.assert_allclose(_np(resid)[j, :kj], orc["res"][:kj, j], rtol=1e-9)


@pytest.mark.parametrize("n", [1, 2])
def test_krylov_and_symmetric_methods_one_and_two_faces(n):
    # tubes of length 1 and 2 (one and two Fourier faces, both weighted 1): nested_tGKB_p,
    # t-Lanczos_p and T-tEVD against the oracle, every slice run to k = m (tiny bounds)
    import torch
    from oracle import tgkb as tg, symmetric as sy
    from paper_2110_02485_amd import rtsvd as rt
    rng = np.random.default_rng(40 + n)
    A = rng.standard_normal((n, 5, 7))
    B = rng.standard_normal((n, 2, 7))
    orc = tg.nested_tgkb_restore(wl.to_math(A), wl.to_math(B), 1e-13, 1.01, 5)
    Xg, k, resid, status = _gpu_nested(A, B, 1e-13, 1.01, 5, "float64")
    _check_nested(orc, Xg, k, resid, status, 1e-9)
    As = _sym_storage(6, n, 50 + n, shift=3.0)
    Bs = rng.standard_normal((n, 2, 6))
    orc = sy.tlanczos_restore(wl.to_math(As), wl.to_math(Bs), 1e-13, 1.01, 6)
    Xg, k, resid, status = _gpu_tlanczos(As, Bs, 1e-13, 1.01, 6, "float64")
    assert [int(v) for v in k.cpu()] == orc["k"]
    assert _rel(_np(Xg), wl.to_storage(orc["X"])) <= 1e-9
    delta = 0.3 * float(np.linalg.norm(Bs))
    orc = sy.tevd_restore(wl.to_math(As), wl.to_math(Bs), delta, 1.01, 6)
    f = rt.ttevd_factor(_t(As), 6, "fp64")
    res = f.solve(_t(Bs), delta, 1.01, 1)
    torch.cuda.synchronize()
    assert int(res.k[0]) == orc["k"]
    assert _rel(_np(res.X), wl.to_storage(orc["X"])) <= 1e-10


# ---------------------------------------------------------------------------------------------
# tGKB baseline
# ---------------------------------------------------------------------------------------------
def _gpu_tgkb(A, B, delta, eta, k_max, dtype):
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    X, k, resid, status = rt.tgkb_solve(_t(A, dtype), _t(B, dtype), delta, eta, k_max)
    torch.cuda.synchronize()
    return X, k, resid, status


@pytest.mark.parametrize("dtype,tol", [("float64", 1e-10), ("float32", 1e-4)])
def test_tgkb_blur_single_rhs(dtype, tol):
    from oracle import tgkb as tg
    A, X, B, Om, delta = blur_problem(64, 16, 2.0, 6, 1, 1e-2, 20, 0, seed=8)
    orc = tg.tgkb_restore(wl.to_math(A), wl.to_math(B), delta, 1.01, 30)
    Xg, k, resid, status = _gpu_tgkb(A, B, delta, 1.01, 30, dtype)
    assert [int(v) for v in k.cpu()] == orc["k"]
    assert _rel(_np(Xg), wl.to_storage(orc["X"])) <= tol
    kk = orc["k"][0]
    np.testing.assert_allclose(_np(resid)[0, :kk], orc["res"][:kk, 0], rtol=max(tol, 1e-9))


def test_tgkb_multi_rhs_per_slice_ragged():
    from oracle import tgkb as tg
    A, X, B, Om, delta = blur_problem(40, 6, 2.0, 6, 5, 1e-2, 20, 0, seed=9, video=True)
    Bm = wl.to_math(B)
    deltas = [0.02 * np.linalg.norm(Bm[:, j]) for j in range(5)]
    orc = tg.tgkb_restore(wl.to_math(A), wl.to_math(B), deltas, 1.05, 25)
    Xg, k, resid, status = _gpu_tgkb(A, B, deltas, 1.05, 25, "float64")
    assert [int(v) for v in k.cpu()] == orc["k"]
    assert _rel(_np(Xg), wl.to_storage(orc["X"])) <= 1e-10


def test_tgkb_dp_not_met_and_random():
    from oracle import tgkb as tg
    l, m, n, p = 33, 21, 5, 2
    rng = np.random.default_rng(10)
    A = rng.standard_normal((n, m, l))
    B = rng.standard_normal((n, p, l))
    orc = tg.tgkb_restore(wl.to_math(A), wl.to_math(B), 1e-12, 1.01, 6)
    Xg, k, resid, status = _gpu_tgkb(A, B, 1e-12, 1.01, 6, "float64")
    assert [int(v) for v in k.cpu()] == [6, 6] and int(status[0]) == 1
    assert _rel(_np(Xg), wl.to_storage(orc["X"])) <= 1e-10


# ---------------------------------------------------------------------------------------------
# nested_tGKB_p: one recycled t-Krylov space for every lateral slice
# ---------------------------------------------------------------------------------------------
def _gpu_nested(A, B, delta, eta, k_max, dtype, k_init=2):
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    X, k, resid, status = rt.nested_tgkb_solve(_t(A, dtype), _t(B, dtype), delta, eta, k_max, k_init)
    torch.cuda.synchronize()
    return X, k, resid, status


def _check_nested(orc, Xg, k, resid, status, tol):
    ks = [int(v) for v in k.cpu()]
    assert ks == orc["k"]
    assert int(status[0]) == orc["status"]
    assert _rel(_np(Xg), wl.to_storage(orc["X"])) <= tol
    top = max(ks)          # every slice's projected residual is known up to the largest k reached
    np.testing.assert_allclose(_np(resid)[:, :top], orc["res"][:top, :].T, rtol=max(tol, 1e-9), atol=0)


@pytest.mark.parametrize("dtype,tol", [("float64", 1e-10), ("float32", 1e-4)])
def test_nested_tgkb_video_slices(dtype, tol):
    # moving-blob video: later frames need a larger space than the one B_1 alone would stop at
    from oracle import tgkb as tg
    A, X, B, Om, delta = blur_problem(48, 8, 2.0, 6, 6, 1e-2, 20, 0, seed=31, video=True)
    Bm = wl.to_math(B)
    fac = [2.0, 1.5, 1.2, 1.0, 0.8, 0.7]                     # tighter bounds for later frames
    deltas = [0.01 * fac[j] * np.linalg.norm(Bm[:, j]) for j in range(6)]
    orc = tg.nested_tgkb_restore(wl.to_math(A), Bm, deltas, 1.05, 30)
    assert orc["k"][-1] > orc["k"][0]
    top = max(orc["k"])                                        # no decision within 0.1% of its bound
    assert np.abs(np.log(orc["res"][:top] / (1.05 * np.array(deltas)))).min() > 1e-3
    Xg, k, resid, status = _gpu_nested(A, B, deltas, 1.05, 30, dtype)
    _check_nested(orc, Xg, k, resid, status, tol)


def test_nested_tgkb_many_slices_ragged_and_k_init():
    # p = 9 slices (more than one block of slices), odd n, deltas mixing met at once / late / never
    from oracle import tgkb as tg
    l, m, n, p = 37, 29, 7, 9
    rng = np.random.default_rng(32)
    A = rng.standard_normal((n, m, l))
    B = rng.standard_normal((n, p, l))
    Am, Bm = wl.to_math(A), wl.to_math(B)
    # bounds relative to each slice's projected residual at k = 1: met at once, after a few
    # steps, or never (slice 8), with every decision at least 1% away from its bound
    r1 = tg.nested_tgkb_restore(Am, Bm, 1e-300, 1.01, 1, k_init=1)["res"][0]
    deltas = list(r1 * np.array([1.3, 0.9, 0.95, 2.0, 0.8, 0.8, 0.75, 1e-13, 2.0]) / 1.01)
    for k_init in (1, 2, 5):
        orc = tg.nested_tgkb_restore(Am, Bm, deltas, 1.01, 12, k_init=k_init)
        assert orc["status"] == tg.DP_NOT_MET and orc["k"][-1] == 12
        assert np.abs(np.log(orc["res"] / (1.01 * np.array(deltas)))).min() > 1e-2
        Xg, k, resid, status = _gpu_nested(A, B, deltas, 1.01, 12, "float64", k_init=k_init)
        _check_nested(orc, Xg, k, resid, status, 1e-10)


def test_nested_tgkb_identical_slices_and_single_slice():
    # identical slices share k and X; one slice reduces to tGKB from k_init = 2
    from oracle import tgkb as tg
    A, X, B, Om, delta = blur_problem(40, 6, 2.0, 6, 1, 1e-2, 20, 0, seed=33)
    B3 = np.concatenate([B] * 3, axis=1)
    orc = tg.nested_tgkb_restore(wl.to_math(A), wl.to_math(B3), delta, 1.01, 25)
    Xg, k, resid, status = _gpu_nested(A, B3, delta, 1.01, 25, "float64")
    _check_nested(orc, Xg, k, resid, status, 1e-10)
    assert len(set(int(v) for v in k.cpu())) == 1
    Xs, ks, _, _ = _gpu_nested(A, B, delta, 1.01, 25, "float64")
    ref = tg.tgkb_restore(wl.to_math(A), wl.to_math(B), delta, 1.01, 25)
    assert int(ks[0]) == max(2, ref["k"][0])
    if ref["k"][0] >= 2:
        assert _rel(_np(Xs), wl.to_storage(ref["X"])) <= 1e-10


# ---------------------------------------------------------------------------------------------
# differentiable restoration: hand-written adjoint vs the FP64 oracle gradient and finite differences
# ---------------------------------------------------------------------------------------------
def _grad_problem(size, n, sigma, band, p, k, rho, seed):
    A = wl.blur_operator(size, n, sigma, band)
    dA = wl.blur_operator_dsigma(size, n, sigma, band)
    rng = np.random.default_rng(seed)
    Xt = wl.lateral_slices(wl.moving_blob_video(size, n, p, rng))
    B = wl.to_storage(tp.tprod(wl.to_math(A), wl.to_math(Xt)) + 1e-2 * rng.standard_normal((size, p, n)))
    Om = rng.standard_normal((n, k + rho, size))
    return A, dA, B, Om, Xt


@pytest.mark.parametrize("dtype,tol", [("float64", 1e-8), ("float32", 2e-3)])
def test_vjp_matches_oracle_gradient(dtype, tol):
    import torch
    from oracle import adjoint as ad
    from paper_2110_02485_amd import autograd as ag
    size, n, sigma, band, p, k, rho = 48, 8, 3.0, 10, 3, 12, 6
    A, dA, B, Om, Xt = _grad_problem(size, n, sigma, band, p, k, rho, 21)
    loss, gb, gs = ad.grads(wl.to_math(A), wl.to_math(dA), wl.to_math(B), wl.to_math(Om), k, wl.to_math(Xt))
    Bt = _t(B, dtype).requires_grad_(True)
    s = torch.tensor(sigma, dtype=getattr(torch, dtype), device="cuda", requires_grad=True)
    X = ag.restore(Bt, s, _t(A, dtype), _t(dA, dtype), _t(Om, dtype), k, rho)
    L = 0.5 * ((X - _t(Xt, dtype)) ** 2).sum()
    L.backward()
    torch.cuda.synchronize()
    assert abs(float(L) - loss) <= tol * loss
    assert _rel(_np(Bt.grad), wl.to_storage(gb)) <= tol
    assert abs(float(s.grad) - gs) <= tol * abs(gs) + 1e-12


def test_vjp_sigma_vs_central_difference_gpu():
    # h = 1e-3 central difference of the GPU forward itself (FP64)
    import torch
    from paper_2110_02485_amd import autograd as ag
    size, n, sigma, band, p, k, rho = 64, 8, 3.0, 10, 2, 16, 8
    A, dA, B, Om, Xt = _grad_problem(size, n, sigma, band, p, k, rho, 22)
    s = torch.tensor(sigma, dtype=torch.float64, device="cuda", requires_grad=True)
    X = ag.restore(_t(B), s, _t(A), _t(dA), _t(Om), k, rho)
    L = 0.5 * ((X - _t(Xt)) ** 2).sum()
    L.backward()
    def Lval(sg):
        As = wl.blur_operator(size, n, sg, band)
        Xs = ag.restore(_t(B), torch.tensor(sg, device="cuda"), _t(As), None, _t(Om), k, rho)
        return float(0.5 * ((Xs - _t(Xt)) ** 2).sum())
    h = 1e-3
    fd = (Lval(sigma + h) - Lval(sigma - h)) / (2 * h)
    assert abs(fd - float(s.grad)) <= 1e-4 * abs(fd) + 1e-10
