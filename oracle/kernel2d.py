"""Closed-form discrete kernel of the 2D anti-plane (mode III) ST-BIEM.

Test infrastructure only (see the package docstring).

Problem statement followed (paper Sec. 2.1): slip rate piecewise constant in
space (Eq. 2.5 area: D_i(t) on element Gamma_i) and in time (piecewise
constant over (m dt, (m+1) dt)), traction collocated at x_i and at
t_n = (n + eps_t) dt, and the fully discrete law T_n = sum_m K_m D_{n-m}
(Eq. 4) with K_m the integral of the continuous kernel over
(t_{m-1}, t_m).  The paper cites the closed forms of the 2D kernel without
printing them; the expressions below are the double-layer representation of
a uniformly slipping segment integrated in closed form:

  source element: the segment [-h, h] x {0} in its own frame, unit slip
  rate switched on at tau = 0 (slip = t), receiver at (X, Y):

    q   = sqrt(b^2 t^2 - Y^2)                      (only if b t > |Y|)
    r+- = sqrt((X +- h)^2 + Y^2),  R+- = sqrt(max(b^2 t^2 - r+-^2, 0))
    I   = asin(clip((X+h)/q)) - asin(clip((X-h)/q))
    s_yz = -(mu / (2 pi b)) [ I + (X+h) R+/r+^2 - (X-h) R-/r-^2 ]
    s_xz = +(mu / (2 pi b)) Y [ R+/r+^2 - R-/r-^2 ]

  (these equal -mu^2 d_yy Phi and -mu^2 d_xy Phi, where Phi is the time-and-
  element integral of the 2D scalar Green's function; the antiderivatives in
  the source coordinate give the end-point forms above).  The slip sense is
  Delta u = u(+nu) - u(-nu) with nu the element normal (Sec. 2.1), so that
  slip relieves stress: the self term is -mu/(2 b), the radiation damping.

The step response S(t) is the stress at time t; the discrete kernel is
K_m = S((m + eps_t) dt) - S((m + eps_t - 1) dt), with S(t <= 0) = 0.

Parity: pinned in tests/test_oracle_kernel.py against (i) brute-force
quadrature of the Green's-function representation off the fault, (ii) the
radiation-damping self term, (iii) the elastostatic dislocation field as
the late-time limit, (iv) the k=0 and k^2 moments of the Fourier-Laplace
symbol (principal-value sum rules), (v) exact zeros outside the causal cone.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

TWO_PI = 2.0 * np.pi


def step_stress_local(X, Y, t, h, mu, beta):
    """Stress vector (s_xz, s_yz) in the source frame, unit slip rate from t=0.

    X, Y: receiver offset in the source element's frame (tangent, normal);
    t: elapsed time; h: half length of the element.  Broadcasts.  Returns a
    pair of float64 arrays.  S(t <= 0) = 0 (quiescent past, Sec. 2.1).
    """
    X, Y, t, h = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (X, Y, t, h)))
    bt = beta * np.where(t > 0.0, t, 0.0)
    bt2 = bt * bt
    Y2 = Y * Y
    up = X + h
    um = X - h
    rp2 = up * up + Y2
    rm2 = um * um + Y2
    Rp = np.sqrt(np.maximum(bt2 - rp2, 0.0))
    Rm = np.sqrt(np.maximum(bt2 - rm2, 0.0))
    inside = bt > np.abs(Y)
    q = np.sqrt(np.where(inside, bt2 - Y2, 1.0))
    I = np.where(
        inside,
        np.arcsin(np.clip(up / q, -1.0, 1.0)) - np.arcsin(np.clip(um / q, -1.0, 1.0)),
        0.0,
    )
    with np.errstate(divide="ignore", invalid="ignore"):
        ap = np.where(Rp > 0.0, Rp / rp2, 0.0)
        am = np.where(Rm > 0.0, Rm / rm2, 0.0)
    c = mu / (TWO_PI * beta)
    s_yz = -c * (I + up * ap - um * am)
    s_xz = c * Y * (ap - am)
    return s_xz, s_yz


def static_rate_local(X, Y, h, mu):
    """Late-time slope dS/dt of the step response, in the source frame.

    Equals the elastostatic stress of a unit uniform slip on [-h, h]
    (a screw-dislocation dipole): the Domain-S time-invariant kernel
    rate (Eq. 2.3 area, K^S = K-hat^S H(m - m^{beta+})).
    """
    X, Y, h = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (X, Y, h)))
    up = X + h
    um = X - h
    rp2 = up * up + Y * Y
    rm2 = um * um + Y * Y
    c = mu / TWO_PI
    s_yz = -c * (up / rp2 - um / rm2)
    s_xz = c * Y * (1.0 / rp2 - 1.0 / rm2)
    return s_xz, s_yz


@dataclass
class Problem:
    """Geometry, medium and time step of a 2D anti-plane problem (Sec. 2.1).

    xa, xb: [N][2] element end points.  Collocation at midpoints; element
    normal nu = rot90(xb - xa)/|xb - xa| (counter-clockwise), which is +y on
    a fault traced in the +x direction.  eps_t = 1 (Sec. 4.3).
    """

    xa: np.ndarray
    xb: np.ndarray
    mu: float = 1.0
    beta: float = 1.0
    dt: float = 0.5
    eps_t: float = 1.0

    def __post_init__(self):
        self.xa = np.asarray(self.xa, dtype=np.float64)
        self.xb = np.asarray(self.xb, dtype=np.float64)
        d = self.xb - self.xa
        self.length = np.hypot(d[:, 0], d[:, 1])
        self.tangent = d / self.length[:, None]
        self.normal = np.stack([-self.tangent[:, 1], self.tangent[:, 0]], axis=1)
        self.center = 0.5 * (self.xa + self.xb)
        self.half = 0.5 * self.length

    @property
    def n(self):
        """Number of elements N."""
        return self.xa.shape[0]

    # -- geometry helpers -------------------------------------------------
    def local_coords(self, P, j):
        """Offsets of points P (broadcast [..., 2]) in the frame of sources j (the
        frame the closed form of the Sec. 2.1 kernel is written in)."""
        P = np.asarray(P, dtype=np.float64)
        d = P - self.center[j]
        X = d[..., 0] * self.tangent[j, 0] + d[..., 1] * self.tangent[j, 1]
        Y = d[..., 0] * self.normal[j, 0] + d[..., 1] * self.normal[j, 1]
        return X, Y

    def stress_step(self, P, j, t):
        """Global stress vector (s_xz, s_yz) at points P due to sources j: the
        step response of Sec. 2.1 in closed form, rotated to global axes."""
        X, Y = self.local_coords(P, j)
        sX, sY = step_stress_local(X, Y, t, self.half[j], self.mu, self.beta)
        tx, ty = self.tangent[j, 0], self.tangent[j, 1]
        nx, ny = self.normal[j, 0], self.normal[j, 1]
        return sX * tx + sY * nx, sX * ty + sY * ny

    def stress_static(self, P, j):
        """Global static stress rate (late-time slope of stress_step) at points P
        due to sources j: the elastostatic dislocation-dipole field that
        Domain S keeps (App. B.1)."""
        X, Y = self.local_coords(P, j)
        sX, sY = static_rate_local(X, Y, self.half[j], self.mu)
        tx, ty = self.tangent[j, 0], self.tangent[j, 1]
        nx, ny = self.normal[j, 0], self.normal[j, 1]
        return sX * tx + sY * nx, sX * ty + sY * ny

    def traction_step(self, i, j, t):
        """Traction step response S_ij(t) = nu_i . sigma at x_i due to j (Sec. 2.1)."""
        sx, sy = self.stress_step(self.center[i], j, t)
        return sx * self.normal[i, 0] + sy * self.normal[i, 1]

    def traction_static(self, i, j):
        """Static traction rate K^S_ij: nu_i . the static stress rate (App. B.1, App. E)."""
        sx, sy = self.stress_static(self.center[i], j)
        return sx * self.normal[i, 0] + sy * self.normal[i, 1]

    def kernel(self, i, j, m):
        """Discrete kernel K_{ij,m} = S_ij(t_m) - S_ij(t_{m-1}) (Eq. 4)."""
        m = np.asarray(m, dtype=np.float64)
        t1 = (m + self.eps_t) * self.dt
        t0 = (m + self.eps_t - 1.0) * self.dt
        return self.traction_step(i, j, t1) - self.traction_step(i, j, t0)

    def kernel_tensor(self, M):
        """Dense K[m][i][j] for m < M (float64 [M][N][N]), the tensor of Eq. 4."""
        N = self.n
        i = np.arange(N)[:, None]
        j = np.arange(N)[None, :]
        K = np.empty((M, N, N))
        prev = self.traction_step(i, j, (self.eps_t - 1.0) * self.dt)
        for m in range(M):
            cur = self.traction_step(i, j, (m + self.eps_t) * self.dt)
            K[m] = cur - prev
            prev = cur
        return K

    def self_term(self):
        """|K_{jj,0}| of the radiation-damping limit, mu/(2 beta): the unit the
        paper normalizes stresses by (Sec. 6)."""
        return self.mu / (2.0 * self.beta)
