"""GPU: the first use of a tube length on the device happens inside a factor split over the
library's face-group streams (the twiddle table of that length is filled on one stream and read by
others): the result must equal the one-group factor bit for bit.  This file sorts first among the
GPU tests so that n = 512 in FP32 has not been used before in the process."""
import numpy as np
import pytest

from paper_2110_02485_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_first_use_of_a_length_in_a_grouped_factor():
    import torch
    from paper_2110_02485_amd import rtsvd as rt
    n, size, k_max, rho = 512, 40, 8, 4                  # 257 faces: three face groups
    print(f"[first-use] FP32 n={n} l=m={size} r={k_max + rho}", flush=True)
    A = wl.blur_operator(size, n, 2.0, 5)
    rng = np.random.default_rng(5)
    B = rng.standard_normal((n, 2, size))
    Om = rng.standard_normal((n, k_max + rho, size))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", torch.float32)
    f3 = rt.factor(t(A), k_max, rho, 0, "fp32", t(Om), face_groups=3)
    r3 = f3.solve(t(B), 1e-3, 1.01)
    f1 = rt.factor(t(A), k_max, rho, 0, "fp32", t(Om), face_groups=1)
    r1 = f1.solve(t(B), 1e-3, 1.01)
    torch.cuda.synchronize()
    s3, s1 = f3.info()[4], f1.info()[4]
    assert np.array_equal(s3, s1)
    assert torch.equal(r3.X, r1.X) and torch.equal(r3.resid, r1.resid) and torch.equal(r3.k, r1.k)
    assert torch.isfinite(r3.X).all()
