"""Pins of the oracle's t-product algebra against definitions and identities (Section 2)."""
import numpy as np
import pytest

from oracle import tproduct as tp

pytestmark = pytest.mark.filterwarnings("ignore")


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("l,p,m,n", [(3, 4, 2, 5), (5, 3, 3, 7), (2, 2, 2, 1), (4, 3, 5, 6)])
def test_tprod_equals_bcirc_and_tube_convolution(l, p, m, n):
    # Definition 2.1: tube-wise circular convolution; bcirc(A) unfold(B) is the same product.
    a, b = _rand((l, p, n), 1), _rand((p, m, n), 2)
    c_fft = tp.tprod(a, b)
    c_conv = tp.tprod_conv(a, b)
    c_bcirc = tp.fold(tp.bcirc(a) @ tp.unfold(b), l, n)
    np.testing.assert_allclose(c_fft, c_conv, rtol=0, atol=1e-12)
    np.testing.assert_allclose(c_fft, c_bcirc, rtol=0, atol=1e-12)


def test_bcirc_block_layout():
    # first block column of bcirc(A) is unfold(A); block (s, u) holds slice (s - u) mod n
    a = _rand((2, 3, 4), 3)
    bc = tp.bcirc(a)
    np.testing.assert_array_equal(bc[:, :3], tp.unfold(a))
    np.testing.assert_array_equal(bc[0:2, 3:6], a[:, :, 3])


def test_transpose_of_product():
    a, b = _rand((3, 4, 5), 4), _rand((4, 2, 5), 5)
    np.testing.assert_allclose(tp.ttranspose(tp.tprod(a, b)),
                               tp.tprod(tp.ttranspose(b), tp.ttranspose(a)), atol=1e-12)


def test_transpose_is_bcirc_transpose():
    a = _rand((3, 4, 6), 6)
    np.testing.assert_allclose(tp.bcirc(tp.ttranspose(a)), tp.bcirc(a).T, atol=0)


def test_identity_tensor():
    a = _rand((3, 4, 5), 7)
    np.testing.assert_allclose(tp.tprod(tp.identity(3, 5), a), a, atol=1e-13)
    np.testing.assert_allclose(tp.tprod(a, tp.identity(4, 5)), a, atol=1e-13)


def test_adjoint_dot_product():
    # <A * X, Y> = <X, A^T * Y>: the transpose is the adjoint of the t-product
    a, x, y = _rand((5, 3, 6), 8), _rand((3, 2, 6), 9), _rand((5, 2, 6), 10)
    lhs = np.sum(tp.tprod(a, x) * y)
    rhs = np.sum(x * tp.tprod(tp.ttranspose(a), y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_conjugate_symmetry_and_parseval():
    a = _rand((4, 3, 8), 11)
    ah = tp.fft_tubes(a)
    for i in range(8):
        np.testing.assert_allclose(ah[:, :, (8 - i) % 8], np.conj(ah[:, :, i]), atol=1e-13)
    assert abs(np.sum(np.abs(ah) ** 2) / 8 - tp.fro(a) ** 2) <= 1e-12 * tp.fro(a) ** 2


def test_frobenius_from_tube_inner():
    # ||X||_F^2 is the first entry of the tube X^T * X (eq. (tfrobX))
    x = _rand((5, 1, 7), 12)
    t = tp.tube_inner(x, x)
    assert abs(t[0] - tp.fro(x) ** 2) <= 1e-12 * tp.fro(x) ** 2


def test_orthogonal_tensor_preserves_norm():
    # eq. (normF): an orthogonal tensor Q (facewise unitary, conjugate-symmetric) keeps ||Q*A||_F
    n, m = 6, 4
    qh = np.empty((m, m, n), dtype=complex)
    rng = np.random.default_rng(13)
    for i in range(n // 2 + 1):
        z = rng.standard_normal((m, m)) + (0 if i in (0, n // 2) else 1j) * rng.standard_normal((m, m))
        q, _ = np.linalg.qr(z)
        qh[:, :, i] = q
        qh[:, :, (n - i) % n] = np.conj(q)
    Q = tp.ifft_tubes(qh)
    np.testing.assert_allclose(tp.tprod(tp.ttranspose(Q), Q), tp.identity(m, n), atol=1e-12)
    a = _rand((m, 3, n), 14)
    assert abs(tp.fro(tp.tprod(Q, a)) - tp.fro(a)) <= 1e-12 * tp.fro(a)
