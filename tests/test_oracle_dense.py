"""Pins of the oracle's Tier-A dense convolution (Eq. 4), CPU only."""
from fractions import Fraction

import numpy as np

from oracle.dense import convolve_dense, convolve_rows, convolve_rows_at
from oracle.kernel2d import Problem
from synth import impulse_slip_rate, straight_fault, uniform_slip_rate


def test_impulse_response_returns_kernel_columns():
    """D = delta_{j0} delta_{n0}  =>  T_{i,n} = K_{i j0, n-n0} exactly."""
    N, M = 24, 18
    xa, xb = straight_fault(N)
    K = Problem(xa, xb).kernel_tensor(M)
    for j0, n0 in [(0, 0), (11, 3), (23, 7)]:
        D = impulse_slip_rate(N, M, j0, n0)
        T = convolve_dense(K, D)
        for n in range(M):
            ref = K[n - n0][:, j0] if n >= n0 else np.zeros(N)
            assert np.array_equal(T[n], ref)


def test_exact_rational_triple_loop():
    """A tiny case with exact rationals: the definition summed exactly."""
    rng = np.random.Generator(np.random.PCG64(7))
    N, M, S = 3, 5, 7
    Kq = [[[Fraction(int(rng.integers(-50, 50)), int(rng.integers(1, 9))) for _ in range(N)] for _ in range(N)] for _ in range(M)]
    Dq = [[Fraction(int(rng.integers(-50, 50)), int(rng.integers(1, 9))) for _ in range(N)] for _ in range(S)]
    ref = [[sum((Kq[m][i][j] * Dq[n - m][j] for m in range(min(n, M - 1) + 1) for j in range(N)), Fraction(0)) for i in range(N)] for n in range(S)]
    T = convolve_dense(np.array(Kq, dtype=float), np.array(Dq, dtype=float))
    for n in range(S):
        for i in range(N):
            assert abs(T[n][i] - float(ref[n][i])) <= 1e-12 * max(1.0, abs(float(ref[n][i])))


def test_row_forms_agree_with_full_form():
    N, M = 20, 16
    xa, xb = straight_fault(N)
    K = Problem(xa, xb).kernel_tensor(M)
    D = uniform_slip_rate(N, M, 1)
    T = convolve_dense(K, D)
    rows = np.transpose(K, (1, 2, 0))[[0, 7, 19]]  # [R][N][M]
    Tr = convolve_rows(rows, D)
    assert np.allclose(Tr, T[:, [0, 7, 19]].T, rtol=1e-13, atol=1e-13)
    Ta = convolve_rows_at(rows, D, [0, 5, 15])
    assert np.allclose(Ta, T[[0, 5, 15]][:, [0, 7, 19]].T, rtol=1e-13, atol=1e-13)


def test_fft_rows_match_direct_rows():
    N, M = 40, 64
    xa, xb = straight_fault(N)
    K = Problem(xa, xb).kernel_tensor(M)
    D = uniform_slip_rate(N, 80, 3)
    rows = np.transpose(K, (1, 2, 0))[[1, 20, 39]]
    from oracle.dense import convolve_rows_fft
    a = convolve_rows(rows, D)
    b = convolve_rows_fft(rows, D)
    assert np.allclose(a, b, rtol=0, atol=1e-12 * np.abs(a).max())
