"""Hand-derived fixtures (tests/golden/*.json, each citing its passage) against the oracle's t-product
and the input generator's blur of eq. (za)."""
import json
import os

import numpy as np

from oracle import tproduct as tp
from paper_2110_02485_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def _tube(v):
    return np.asarray(v, dtype=np.float64)[None, None, :]


def test_tproduct_hand_examples():
    g = _load("tproduct_hand_examples.json")
    e = g["tube_product_n3"]
    c = tp.tprod(_tube(e["a"]), _tube(e["b"]))
    np.testing.assert_allclose(c[0, 0], e["c"], atol=1e-12)
    np.testing.assert_allclose(tp.tprod_conv(_tube(e["a"]), _tube(e["b"]))[0, 0], e["c"], atol=1e-12)
    e = g["tensor_product_n2"]
    A = np.stack([np.asarray(s, dtype=np.float64) for s in e["A_slices"]], axis=2)
    B = np.stack([np.asarray(s, dtype=np.float64) for s in e["B_slices"]], axis=2)
    C = np.stack([np.asarray(s, dtype=np.float64) for s in e["C_slices"]], axis=2)
    np.testing.assert_allclose(tp.tprod(A, B), C, atol=1e-12)
    e = g["transpose_n3"]
    np.testing.assert_array_equal(tp.ttranspose(_tube(e["a"]))[0, 0], e["aT"])
    e = g["tube_norm_n3"]
    x = _tube(e["x"])
    np.testing.assert_allclose(tp.tprod(tp.ttranspose(x), x)[0, 0, 0], e["first_entry_of_xT_x"], atol=1e-12)


def test_blur_generator_follows_eq_za():
    g = _load("blur_za_sigma1_band3.json")
    T = wl.blur_toeplitz(g["size"], g["sigma"], g["band"])
    np.testing.assert_allclose(T[0], g["first_row"], rtol=1e-15, atol=1e-17)
    np.testing.assert_allclose(T, T.T)
    np.testing.assert_allclose(T[2], [g["first_row"][2], g["first_row"][1], g["first_row"][0], g["first_row"][1],
                                      g["first_row"][2]], rtol=1e-15)
