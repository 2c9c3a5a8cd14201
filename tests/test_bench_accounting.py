"""The bench's algorithmic-byte accounting (CPU): the window lags a step
applies, sum over pairs of min(W_ij, n + 1), averaged over the timed steps,
against a brute-force sum."""
import numpy as np

import bench


def test_near_lags_mean_equals_brute_force():
    rng = np.random.Generator(np.random.PCG64(11))
    W = rng.integers(1, 600, size=2000)
    for n0, n1 in ((0, 0), (0, 50), (100, 700), (599, 620), (1000, 1010)):
        ref = np.mean([np.minimum(W, n + 1).sum() for n in range(n0, n1 + 1)])
        assert bench.near_lags_mean(W, n0, n1) == ref


def test_near_lags_mean_at_full_history_is_the_window_sum():
    W = np.array([5, 17, 64, 128, 3])
    assert bench.near_lags_mean(W, 200, 300) == W.sum()
