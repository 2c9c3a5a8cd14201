"""Closed-form discrete kernel of the 2D in-plane (P-SV) ST-BIEM on a straight fault.

Test infrastructure only (see the package docstring).

Problem statement followed (paper Sec. 2.1, with the in-plane medium of the
paper's Quantization experiments, App. A: P and S waves of speeds alpha and
beta, alpha dt / dx = 1/2): slip and opening rates piecewise constant in
space and time on the elements of a straight fault, tractions (shear,
normal) collocated at the element midpoints at t_n = (n + eps_t) dt, and
T_n = sum_m K_m D_{n-m} (Eq. 4) with K_m the integral of the continuous
kernel over (t_{m-1}, t_m).  On a straight fault the shear traction depends
on the slip rate only and the normal traction on the opening rate only
(mirror symmetry about the fault plane), so the 2 x 2 kernel is diagonal.

Step response of the source segment [-h, h] x {0} (unit rate switched on at
t = 0) at the receiver (x, 0), written with the front terms of each wave
speed c in {alpha, beta}:

    A_c = asin(clip((x+h)/(c t))) - asin(clip((x-h)/(c t)))
    B_c = R_c(x+h)/(x+h) - R_c(x-h)/(x-h),   R_c(z) = sqrt(max(c^2 t^2 - z^2, 0))
    Q_c(z) = sqrt(max(t^2 - z^2/c^2, 0))
    F(z) = [Q_beta(z)(t^2 + 2 z^2/beta^2) - Q_alpha(z)(t^2 + 2 z^2/alpha^2)] / z^3

    S_shear  = -(mu/(2 pi beta)) A_beta - (2 mu/(pi beta)) B_beta
               + (2 mu beta^2/(pi alpha^3)) B_alpha + (2 mu beta^2/(3 pi)) [F(x+h) - F(x-h)]
    S_normal = -(mu alpha/(2 pi beta^2)) A_alpha - (2 mu/(pi alpha)) B_alpha
               + (2 mu/(pi beta)) B_beta - (2 mu beta^2/(3 pi)) [F(x+h) - F(x-h)]

F is the near-field term between the P and S fronts.  Once both fronts have
passed z, the difference in F cancels to leading order; it is evaluated as
F(z) = [t^2 (1/alpha^2 - 1/beta^2)/(Q_beta + Q_alpha) + 2 (Q_beta/beta^2 -
Q_alpha/alpha^2)] / z, the same quantity without the cancellation.

Parity: pinned in tests/test_oracle_inplane.py against (i) the radiation-
damping self terms -mu/(2 beta) (shear) and -mu alpha/(2 beta^2) (normal),
(ii) the plane-strain elastostatic dislocation field (the anti-plane one
times 2 (1 - beta^2/alpha^2) = 1/(1 - nu)) as the late-time limit, (iii) the
k = 0 and k^2 moments of the Fourier-Laplace symbols of the in-plane
traction-slip relations (principal-value sum rules, derived symbolically in
the test), (iv) exact zeros before the P wave arrives, (v) symmetry in x.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def _front(z, ct):
    """R_c(z)/z: sqrt(max(c^2 t^2 - z^2, 0)) / z."""
    return np.sqrt(np.maximum(ct * ct - z * z, 0.0)) / z


def _near_field(z, t, alpha, beta):
    """F(z) of the module docstring (0 before the P wave reaches z)."""
    z = np.asarray(z, dtype=np.float64)
    az = np.abs(z)
    qa = np.sqrt(np.maximum(t * t - (z / alpha) ** 2, 0.0))
    qb = np.sqrt(np.maximum(t * t - (z / beta) ** 2, 0.0))
    both = t > az / beta
    only_p = (t > az / alpha) & ~both
    with np.errstate(divide="ignore", invalid="ignore"):
        f_both = (t * t * (1.0 / alpha**2 - 1.0 / beta**2) / (qb + qa) + 2.0 * (qb / beta**2 - qa / alpha**2)) / z
        f_p = -qa * (t * t + 2.0 * z * z / alpha**2) / z**3
    return np.where(both, f_both, np.where(only_p, f_p, 0.0))


def step_inplane(x, t, h, mu, alpha, beta):
    """(S_shear, S_normal) at (x, 0) at time t after a unit slip rate (resp.
    opening rate) starts on [-h, h] x {0}: the in-plane step responses whose
    differences over a step are the kernel of Eq. 4 for the medium of App. A
    (closed forms of the module docstring).  Broadcasts; S(t <= 0) = 0."""
    x, t, h = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (x, t, h)))
    tp = np.where(t > 0.0, t, 0.0)
    up, um = x + h, x - h

    def A(c):
        """Arcsine front term of speed c (A_c of the module docstring)."""
        ct = c * tp
        with np.errstate(divide="ignore", invalid="ignore"):
            a = np.arcsin(np.clip(np.where(ct > 0, up / ct, 0.0), -1, 1)) - np.arcsin(
                np.clip(np.where(ct > 0, um / ct, 0.0), -1, 1))
        return np.where(ct > 0, a, 0.0)

    def B(c):
        """Root front term of speed c (B_c of the module docstring)."""
        ct = c * tp
        return _front(up, ct) - _front(um, ct)

    Fd = _near_field(up, tp, alpha, beta) - _near_field(um, tp, alpha, beta)
    Aa, Ab, Ba, Bb = A(alpha), A(beta), B(alpha), B(beta)
    pi = np.pi
    s_sh = (-(mu / (2 * pi * beta)) * Ab - (2 * mu / (pi * beta)) * Bb
            + (2 * mu * beta**2 / (pi * alpha**3)) * Ba + (2 * mu * beta**2 / (3 * pi)) * Fd)
    s_no = (-(mu * alpha / (2 * pi * beta**2)) * Aa - (2 * mu / (pi * alpha)) * Ba
            + (2 * mu / (pi * beta)) * Bb - (2 * mu * beta**2 / (3 * pi)) * Fd)
    live = tp > 0
    return np.where(live, s_sh, 0.0), np.where(live, s_no, 0.0)


def static_rate_inplane(x, h, mu, alpha, beta):
    """Late-time slope dS/dt of both components (the static limit, App. B.1,
    of the App. A medium): the plane-strain static
    traction per unit slip (opening) of the segment, 2 (1 - beta^2/alpha^2)
    times the anti-plane one, mu h / (pi (x^2 - h^2))."""
    x = np.asarray(x, dtype=np.float64)
    return 2.0 * (1.0 - beta**2 / alpha**2) * mu * h / (np.pi * (x * x - h * h))


@dataclass
class InplaneProblem:
    """In-plane problem (App. A medium, Sec. 2.1 discretization) on a straight
    fault along x: element j covers (xa_j, xb_j) on y = 0."""

    xa: np.ndarray  # [N] left end points (x)
    xb: np.ndarray  # [N] right end points (x)
    mu: float = 1.0
    alpha: float = float(np.sqrt(3.0))
    beta: float = 1.0
    dt: float = 0.5 / float(np.sqrt(3.0))
    eps_t: float = 1.0

    def __post_init__(self):
        self.xa = np.asarray(self.xa, dtype=np.float64)
        self.xb = np.asarray(self.xb, dtype=np.float64)
        self.center = 0.5 * (self.xa + self.xb)
        self.half = 0.5 * (self.xb - self.xa)

    @property
    def n(self):
        """Number of elements N."""
        return len(self.xa)

    def step(self, i, j, t):
        """(shear, normal) step responses at receiver i from source j (Sec. 2.1)."""
        x = self.center[i] - self.center[j]
        return step_inplane(x, t, self.half[j], self.mu, self.alpha, self.beta)

    def kernel(self, i, j, m):
        """(K_shear, K_normal)[i, j, m] = S((m + eps_t) dt) - S((m + eps_t - 1) dt)
        (the definition under Eq. 4)."""
        m = np.asarray(m, dtype=np.float64)
        hi = self.step(i, j, (m + self.eps_t) * self.dt)
        lo = self.step(i, j, (m + self.eps_t - 1.0) * self.dt)
        return hi[0] - lo[0], hi[1] - lo[1]

    def kernel_tensor(self, M):
        """Dense (K_shear, K_normal), each [M][N][N]: the tensors of Eq. 4."""
        i = np.arange(self.n)[:, None]
        j = np.arange(self.n)[None, :]
        Ks = np.empty((M, self.n, self.n))
        Kn = np.empty((M, self.n, self.n))
        prev = self.step(i, j, (self.eps_t - 1.0) * self.dt)
        for m in range(M):
            cur = self.step(i, j, (m + self.eps_t) * self.dt)
            Ks[m] = cur[0] - prev[0]
            Kn[m] = cur[1] - prev[1]
            prev = cur
        return Ks, Kn
