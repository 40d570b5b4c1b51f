"""Autotuner: the candidate set (host logic) and, on the GPU, a small tuning run."""
import numpy as np
import pytest

from tests.problems import blur_problem


def test_candidates_cover_group_counts_and_tile_widths():
    from paper_2110_02485_amd import tune
    # r = 120 over 65 faces: 1..3 groups, 1, 2, 4, 8 tiles (8 tiles = 128 columns is the first to cover r),
    # and 2 or 3 restorations in flight with one group
    c = tune.candidates(120, 65)
    assert c[:12] == [(g, t, 1) for g in (1, 2, 3) for t in (1, 2, 4, 8)]
    assert c[12:] == [(1, t, s) for t in (1, 2, 4, 8) for s in (2, 3)]
    # r = 30: two tiles already cover it; 9 faces allow two groups of at least four faces
    assert tune.candidates(30, 9) == [(1, 1, 1), (1, 2, 1), (2, 1, 1), (2, 2, 1), (1, 1, 2), (1, 1, 3), (1, 2, 2),
                                      (1, 2, 3)]
    # one face: one group; r = 16: one tile
    assert tune.candidates(16, 1) == [(1, 1, 1), (1, 1, 2), (1, 1, 3)]
    # more than one restoration in flight only with a single face group (the group streams are shared)
    assert all(g == 1 for g, t, s in c if s > 1)


@pytest.mark.gpu
def test_tune_picks_a_candidate_and_results_agree():
    import torch
    from paper_2110_02485_amd import tune
    A, X, B, Om, delta = blur_problem(128, 32, 2.0, 8, 1, 1e-2, 20, 10, seed=71)
    t32 = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", torch.float32)
    out = tune.tune(t32(A), t32(B), t32(Om), 20, 10, 1, "mixed", delta, 1.01, steps=2, rounds=1)
    assert out["identical"]
    assert (out["face_groups"], out["sketch_tile"], out["in_flight"]) in tune.candidates(30, 17)
    assert len(out["table"]) == len(tune.candidates(30, 17)) and out["ms_per_step"] > 0
