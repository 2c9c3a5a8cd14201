"""Tier-A: the exact dense time-marching convolution (Eq. 4).

Test infrastructure only (see the package docstring).

T_{i,n} = sum_{m=0}^{min(n, M-1)} sum_j K_{ij,m} D_{j,n-m}, with D at negative
steps equal to zero (quiescent past, Sec. 2.1).  Written as the definition:
a loop over the lag m with a matrix-vector product per lag.

Parity: pinned by the impulse response (a unit slip rate at (j0, n0) must
return the kernel column K_{:,j0,n-n0} exactly) and by a tiny case summed
with exact rational arithmetic (tests/test_oracle_dense.py).
"""
from __future__ import annotations

import numpy as np


def convolve_dense(K, D):
    """T[n][i] for n < D.shape[0], given K[M][N][N] and D[steps][N]: the sum of
    Eq. 4 over lags m <= min(n, M - 1), the past before step 0 quiescent."""
    K = np.asarray(K, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    M = K.shape[0]
    steps, N = D.shape
    T = np.zeros((steps, N))
    for n in range(steps):
        for m in range(min(n, M - 1) + 1):
            T[n] += K[m] @ D[n - m]
    return T


def convolve_rows(Krows, D, steps=None):
    """T[i][n] of Eq. 4 for sampled receivers, from their kernel rows.

    Krows: [R][N][M] rows K_{i,:,m} of the sampled receivers.  D: [S][N].
    Uses, per lag, the definition T_{i,n} += sum_j K_{ij,m} D_{j,n-m}.
    """
    Krows = np.asarray(Krows, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    R, N, M = Krows.shape
    S = D.shape[0] if steps is None else steps
    T = np.zeros((R, S))
    for m in range(min(M, S)):
        # T[:, n] for n >= m receives K[:, :, m] @ D[n - m]
        T[:, m:] += Krows[:, :, m] @ D[: S - m].T
    return T


def convolve_rows_at(Krows, D, n_list):
    """T[i][k] of Eq. 4 at selected steps n_list[k] only (direct dot products)."""
    Krows = np.asarray(Krows, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    R, N, M = Krows.shape
    out = np.zeros((R, len(n_list)))
    for k, n in enumerate(n_list):
        L = min(n, M - 1) + 1
        # D[n - m] for m = 0..L-1
        hist = D[n - np.arange(L)]  # [L][N]
        out[:, k] = np.einsum("rjm,mj->r", Krows[:, :, :L], hist)
    return out


def convolve_rows_fft(Krows, D, steps=None):
    """T[i][n] of Eq. 4 for sampled receivers via FFT convolution along time.

    Same definition as convolve_rows (zero history before step 0, lags
    limited to the rows' length M); the time convolution of every
    (receiver, source) pair is evaluated with a real FFT of length >= M + S.
    """
    Krows = np.asarray(Krows, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    R, N, M = Krows.shape
    S = D.shape[0] if steps is None else steps
    L = 1
    while L < M + S:
        L *= 2
    Df = np.fft.rfft(D[:S].T, n=L, axis=1)  # [N][L/2+1]
    T = np.zeros((R, S))
    for r in range(R):
        Kf = np.fft.rfft(Krows[r], n=L, axis=1)
        T[r] = np.fft.irfft((Kf * Df).sum(axis=0), n=L)[:S]
    return T
