"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module holds only input generation: fault geometries (segment end
points) and slip-rate histories.  It contains none of the boundary-integral
arithmetic, so that both sides of every parity test consume identical inputs
while computing everything else independently.

Geometries follow the 2D settings of the paper's numerical experiments
(Sec. 6: elements of constant length covering x in (i dx, (i+1) dx) on the
x-axis) and a smooth nonplanar variant (a sinusoidal trace).  Slip-rate
histories are i.i.d. uniform draws, or a Gaussian-smoothed random field in
space and time, standardized to zero mean and unit variance.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "straight_fault",
    "curved_fault",
    "uniform_slip_rate",
    "smooth_slip_rate",
    "impulse_slip_rate",
    "ensemble_sizes",
]


def straight_fault(n: int, dx: float = 1.0):
    """Planar fault on y=0: element j covers x in (j dx, (j+1) dx).

    Returns (xa, xb), each float64 [n][2]: the two end points of every element.
    """
    j = np.arange(n, dtype=np.float64)
    xa = np.stack([j * dx, np.zeros(n)], axis=1)
    xb = np.stack([(j + 1.0) * dx, np.zeros(n)], axis=1)
    return np.ascontiguousarray(xa), np.ascontiguousarray(xb)


def _curve_len(L, amp_frac, wl_frac, npts=200001):
    x = np.linspace(0.0, L, npts)
    A, lam = amp_frac * L, wl_frac * L
    dy = A * (2 * math.pi / lam) * np.cos(2 * math.pi * x / lam)
    f = np.sqrt(1.0 + dy * dy)
    return float(np.sum(0.5 * (f[1:] + f[:-1]) * np.diff(x)))


def curved_fault(n: int, dx: float = 1.0, amp_frac: float = 0.05, wl_frac: float = 0.25):
    """Sinusoidal trace y = a L sin(2 pi x / (w L)) cut into n straight chords.

    L (the x-extent) is chosen so that the arc length of the trace equals
    n*dx; consecutive chord end points lie on the trace at Euclidean distance
    dx from each other.  Returns (xa, xb) as float64 [n][2].
    """
    target = n * dx
    lo, hi = 0.1 * target, target
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if _curve_len(mid, amp_frac, wl_frac) < target:
            lo = mid
        else:
            hi = mid
    L = 0.5 * (lo + hi)
    A, lam = amp_frac * L, wl_frac * L

    def y(x):
        return A * math.sin(2 * math.pi * x / lam)

    pts = np.empty((n + 1, 2))
    px, py = 0.0, 0.0
    pts[0] = (px, py)
    for k in range(1, n + 1):
        a, b = px, px + dx  # the chord end lies within one dx in x
        for _ in range(60):
            m = 0.5 * (a + b)
            d = math.hypot(m - px, y(m) - py)
            if d < dx:
                a = m
            else:
                b = m
        px = 0.5 * (a + b)
        py = y(px)
        pts[k] = (px, py)
    xa = np.ascontiguousarray(pts[:-1])
    xb = np.ascontiguousarray(pts[1:])
    return xa, xb


def uniform_slip_rate(n: int, m: int, seed: int):
    """D[m][n], i.i.d. U(0,1) per element and step (PCG64 stream `seed`)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.random((m, n)))


def _gauss_taps(sigma: float):
    r = max(1, int(math.ceil(4.0 * sigma)))
    x = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-0.5 * (x / sigma) ** 2)
    return w / w.sum()


def _smooth_axis(a, sigma, axis):
    """Circular convolution with a truncated Gaussian along one axis."""
    w = _gauss_taps(sigma)
    r = (len(w) - 1) // 2
    L = a.shape[axis]
    kern = np.zeros(L)
    for k, wk in enumerate(w):
        kern[(k - r) % L] += wk
    kf = np.fft.rfft(kern)
    shape = [1] * a.ndim
    shape[axis] = kf.shape[0]
    af = np.fft.rfft(a, axis=axis)
    af *= kf.reshape(shape)
    return np.fft.irfft(af, n=L, axis=axis)


def smooth_slip_rate(n: int, m: int, ell: float, ell_t: float, seed: int):
    """D[m][n]: Gaussian-smoothed random field, zero mean, unit variance.

    Z ~ N(0,1) i.i.d. over (step, element) from PCG64 stream `seed`, smoothed
    by Gaussians of standard deviation `ell` elements (space) and `ell_t`
    steps (time), each truncated at four standard deviations, then shifted
    and scaled to zero mean and unit variance over the whole array.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((m, n))
    if ell > 0:
        z = _smooth_axis(z, ell, axis=1)
    if ell_t > 0:
        z = _smooth_axis(z, ell_t, axis=0)
    z -= z.mean()
    z /= z.std()
    return np.ascontiguousarray(z)


def impulse_slip_rate(n: int, m: int, j0: int, n0: int = 0):
    """D[m][n] that is 1 at (step n0, element j0) and 0 elsewhere."""
    d = np.zeros((m, n))
    d[n0, j0] = 1.0
    return d


def ensemble_sizes(count: int, n_lo: int, n_hi: int, seed: int):
    """Element counts of an ensemble of independent faults.

    N_k = round(exp(U(ln n_lo, ln n_hi))) for k < count (log-uniform, PCG64
    stream `seed`), returned as an int64 array.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(math.log(n_lo), math.log(n_hi), size=count)
    return np.rint(np.exp(u)).astype(np.int64)
