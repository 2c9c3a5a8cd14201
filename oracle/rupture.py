"""Dynamic rupture: the time-marching convolution coupled to a friction law.

Test infrastructure only (see the package docstring).

Problem (paper Sec. 6.2, its boundary conditions; App. A.2.3, the initial
stress of the single-asperity model):
  * the shear traction on element i at step n is T0_i + T_{i,n}, with T_n the
    convolution of Eq. 4 over the slip-rate history (any kernel tensor: the
    exact one, or the FDP=H-approximated one);
  * an element that has not ruptured keeps a zero slip rate until its
    traction reaches the yield value T_th; from then on it is ruptured and its
    traction equals the frictional strength of the law at its current slip
    (it sticks, D = 0, whenever that would take a negative slip rate);
  * laws: exponential slip weakening, strength (T_th - T_dy) exp(-slip/D_c)
    + T_dy (Sec. 6.2); static-dynamic, strength T_dy once ruptured
    (App. A.2.3);
  * the slip rate is constant over a step, so slip_{i,n} = slip_{i,n-1} +
    dt D_{i,n}.

Reading (the paper does not spell out the discrete solve; this is the
standard implicit treatment of the first lag):
  T_{i,n} = sum_{m >= 1} (K_m D_{n-m})_i + K_{ii,0} D_{i,n}, valid when the
  first lag couples each element only to itself (no other element within
  beta eps_t dt of its collocation point: the wave of a neighbour has not
  reached it by the first collocation time).  A neighbour at that distance up
  to rounding (a curved trace cut into chords at beta dt = dx/2) is grazed by
  the front and has a tiny first-lag entry (4.5e-10 on the sinusoidal fault);
  such entries, below 1e-7 |K_ii,0|, are left out.  Per element and step:
    tau* = T0_i + sum_{m >= 1} (K_m D_{n-m})_i      (traction with D_n = 0)
    not ruptured and tau* < T_th:  D = 0
    otherwise ruptured;  g(D) = tau* + K_{ii,0} D - strength(slip_{n-1} + dt D)
      g(0) <= 0:  D = 0 (stick)
      else:       D is the root of g in (0, (tau* - T_dy) / |K_ii,0|]
  (g is positive at 0 and not positive at the upper end, because the
  strength never falls below T_dy; with K_ii,0 < 0 and any D_c, g rises at
  most once before it falls, so the root is unique).  The static-dynamic law
  has the root in closed form; the exponential law's is found by Brent's
  method to full double precision.

Parity: pinned in tests/test_oracle_rupture.py against the radiation-damped
slider that the interior of a uniformly ruptured fault must follow before
waves from the fault ends arrive (a scalar recursion solved there by its own
bisection), the rupture-free case, discrete causality of the rupture front,
mirror symmetry, and the reduction of the exponential law to the
static-dynamic one as D_c -> 0.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.optimize import brentq

LAWS = ("exp", "static_dynamic")


@dataclass
class Friction:
    """Friction law of the rupture problem: exponential slip weakening (Sec. 6.2)
    or static-dynamic (App. A.2.3), and the time step of the slip update."""

    law: str          # "exp" (Sec. 6.2) or "static_dynamic" (App. A.2.3)
    t_th: float       # yield traction
    t_dy: float       # dynamic (fully weakened) traction
    d_c: float = 0.0  # slip-weakening distance (exponential law)
    dt: float = 0.5

    def __post_init__(self):
        if self.law not in LAWS:
            raise ValueError(self.law)

    def strength(self, slip):
        """Frictional strength of a ruptured element at the given slip (Sec. 6.2
        exponential weakening; App. A.2.3 static-dynamic)."""
        if self.law == "static_dynamic":
            return self.t_dy
        return (self.t_th - self.t_dy) * np.exp(-slip / self.d_c) + self.t_dy


def single_asperity_stress(center_x, t_bg, t_th, x_lo, x_hi):
    """Initial traction of the single-asperity model (App. A.2.3): T_bg
    outside (x_lo, x_hi), T_th inside it."""
    x = np.asarray(center_x, dtype=np.float64)
    return np.where((x > x_lo) & (x < x_hi), t_th, t_bg).astype(np.float64)


def solve_element(fr: Friction, tau_star, k0, slip_prev):
    """Slip rate of a ruptured element (the per-element solve of the module
    docstring).  k0 = K_ii,0 < 0."""
    if k0 >= 0.0:
        raise ValueError("the first-lag self term must be negative (radiation damping)")

    def g(D):
        """Traction minus strength at slip rate D (the implicit first-lag equation)."""
        return tau_star + k0 * D - fr.strength(slip_prev + fr.dt * D)

    if g(0.0) <= 0.0:
        return 0.0
    hi = (tau_star - fr.t_dy) / (-k0)
    if fr.law == "static_dynamic":
        return hi
    if g(hi) >= 0.0:  # strength already at T_dy to rounding: the bound is the root
        return hi
    return brentq(g, 0.0, hi, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=400)


def simulate(Krows, T0, fr: Friction, steps, ruptured=None):
    """Coupled time marching (Sec. 6.2 boundary conditions, first lag implicit).

    Krows: [N][N][M] kernel K_{ij,m} (receiver i, source j, lag m).  T0: [N]
    initial traction.  Returns (D [steps][N], T [steps][N] total traction,
    slip [N], ruptured [N] bool) at the end of the run.
    """
    Krows = np.asarray(Krows, dtype=np.float64)
    N, N2, M = Krows.shape
    assert N == N2
    k0 = np.diagonal(Krows[:, :, 0]).copy()
    off = Krows[:, :, 0] - np.diag(k0)
    if np.abs(off).max(initial=0.0) > 1e-7 * np.abs(k0).max():
        raise ValueError("the first lag couples different elements: the per-element solve does not apply")
    T0 = np.asarray(T0, dtype=np.float64)
    D = np.zeros((steps, N))
    T = np.zeros((steps, N))
    slip = np.zeros(N)
    rup = np.zeros(N, dtype=bool) if ruptured is None else np.asarray(ruptured, dtype=bool).copy()
    Km = np.ascontiguousarray(np.moveaxis(Krows, 2, 0))  # [M][N][N]
    for n in range(steps):
        L = min(n, M - 1)  # lags m = 1..L: the history only
        hist = np.einsum("mij,mj->i", Km[1:L + 1], D[n - L:n][::-1]) if L > 0 else np.zeros(N)
        tau_star = T0 + hist
        for i in range(N):
            if not rup[i] and tau_star[i] < fr.t_th:
                d = 0.0
            else:
                rup[i] = True
                d = solve_element(fr, tau_star[i], k0[i], slip[i])
            D[n, i] = d
            T[n, i] = tau_star[i] + k0[i] * d
            slip[i] += fr.dt * d
    return D, T, slip, rup
