"""Pins of the oracle's closed-form anti-plane kernel (CPU only).

Each check comes from a route that does not use the closed form itself:
brute-force quadrature of the Green's-function representation, the plane-
wave (radiation damping) limit, the elastostatic dislocation field, moments
of the Fourier-Laplace symbol, and the causal cone.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle.kernel2d import Problem, static_rate_local, step_stress_local
from greens_quadrature import brute_stress as _brute_stress
from synth import curved_fault, straight_fault


@pytest.mark.parametrize(
    "X,Y,t",
    [
        (0.3, 0.05, 0.4),
        (0.3, 0.05, 2.0),
        (2.0, 0.5, 1.7),
        (2.0, 0.5, 9.0),
        (-1.2, 1.0, 3.0),
        (5.0, -2.0, 6.0),
        (0.0, 0.3, 0.45),
        (-7.5, 0.8, 8.1),
    ],
)
@pytest.mark.parametrize("mu,beta,h", [(1.0, 1.0, 0.5), (2.5, 1.7, 0.8)])
def test_closed_form_matches_green_quadrature(X, Y, t, mu, beta, h):
    sx, sy = step_stress_local(X, Y, t, h, mu, beta)
    bx, by = _brute_stress(X, Y, t, h, mu, beta)
    scale = mu / beta
    assert abs(float(sy) - by) <= 1e-9 * scale
    assert abs(float(sx) - bx) <= 1e-9 * scale


@pytest.mark.parametrize("mu,beta,dt,h", [(1.0, 1.0, 0.5, 0.5), (3.0, 2.0, 0.1, 0.5), (1.0, 0.7, 0.3, 0.6)])
def test_self_term_is_radiation_damping(mu, beta, dt, h):
    """While no edge wave has reached the centre (beta dt <= h) the self
    response is the plane-wave impedance: K_ii0 = -mu/(2 beta)."""
    sx, sy = step_stress_local(0.0, 0.0, dt, h, mu, beta)
    assert float(sy) == pytest.approx(-mu / (2 * beta), rel=1e-15, abs=0)
    assert float(sx) == 0.0


@pytest.mark.parametrize("X,Y", [(0.0, 0.0), (3.0, 0.0), (-10.0, 0.0), (2.0, 1.5), (0.1, -0.4)])
def test_late_time_slope_is_elastostatic(X, Y):
    """dS/dt -> stress of a unit screw-dislocation dipole (elastostatics):
    s_yz = -(mu/2pi)[(X+h)/r+^2 - (X-h)/r-^2], s_xz = (mu/2pi) Y [1/r+^2 - 1/r-^2].
    The approach is O(1/t^2)."""
    mu, beta, h = 1.3, 0.9, 0.5
    rp2 = (X + h) ** 2 + Y * Y
    rm2 = (X - h) ** 2 + Y * Y
    ref_y = -(mu / (2 * math.pi)) * ((X + h) / rp2 - (X - h) / rm2)
    ref_x = (mu / (2 * math.pi)) * Y * (1 / rp2 - 1 / rm2)
    errs = []
    for t in (2e2, 4e2, 8e2):
        d = 1e-3
        a = step_stress_local(X, Y, t + d, h, mu, beta)
        b = step_stress_local(X, Y, t - d, h, mu, beta)
        slope_y = (float(a[1]) - float(b[1])) / (2 * d)
        slope_x = (float(a[0]) - float(b[0])) / (2 * d)
        errs.append(abs(slope_y - ref_y) + abs(slope_x - ref_x))
    assert errs[-1] < 1e-5
    assert errs[1] / errs[0] < 0.3 and errs[2] / errs[1] < 0.3  # ~1/4 per doubling
    # the oracle's own static-rate function is the same elastostatic field
    sx, sy = static_rate_local(X, Y, h, mu)
    assert float(sy) == pytest.approx(ref_y, rel=1e-14, abs=1e-16)
    assert float(sx) == pytest.approx(ref_x, rel=1e-14, abs=1e-16)


def _pv_moment(t, power, mu=1.0, beta=1.0, h=0.5):
    """Principal-value integral of x^power S(x, t) over the fault line."""
    L = h + beta * t  # S vanishes for |x| >= L
    A = mu * t / (2 * math.pi)  # S ~ A/(x-h) near x=h, ~ -A/(x+h) near x=-h
    B = -A

    def f(x):
        s = float(step_stress_local(x, 0.0, t, h, mu, beta)[1])
        return x**power * s - A * h**power / (x - h) - B * (-h) ** power / (x + h)

    brk = sorted({-L, -h, h, L, -h - beta * t + 1e-300, h - beta * t, -h + beta * t})
    brk = [b for b in brk if -L <= b <= L]
    total = 0.0
    for a, b in zip(brk[:-1], brk[1:]):
        if b - a < 1e-14:
            continue
        v, _ = integrate.quad(f, a, b, epsabs=1e-12, epsrel=1e-12, limit=400)
        total += v
    log_term = math.log((L - h) / (L + h))  # PV int dx/(x-h) over (-L, L)
    total += A * h**power * log_term + B * (-h) ** power * (-log_term)
    return total


@pytest.mark.parametrize("t", [0.25, 1.0, 3.7, 12.0])
def test_sum_rules_of_the_symbol(t):
    """Moments in x of the on-fault response follow from the symbol
    sigma^ = -(mu/(2 b)) sqrt(s^2 + b^2 k^2)/s V^ at k = 0:
    int S dx = -mu h / b  and  int x^2 S dx = (mu/b)(b^2 h t^2/2 - h^3/3)."""
    mu, beta, h = 1.0, 1.0, 0.5
    m0 = _pv_moment(t, 0)
    m2 = _pv_moment(t, 2)
    assert m0 == pytest.approx(-mu * h / beta, rel=1e-8)
    assert m2 == pytest.approx((mu / beta) * (beta**2 * h * t * t / 2 - h**3 / 3), rel=1e-8)


def test_causal_cone_exact_zeros():
    xa, xb = straight_fault(64)
    pr = Problem(xa, xb, dt=0.5)
    K = pr.kernel_tensor(40)
    d = np.abs(np.arange(64)[:, None] - np.arange(64)[None, :])
    for m in range(40):
        # nearest source point at distance d - 1/2; reachable by time (m+1) dt
        outside = (d - 0.5) >= pr.beta * (m + 1) * pr.dt
        assert np.all(K[m][outside] == 0.0)
        inside_front = (d - 0.5) < pr.beta * (m + 1) * pr.dt - 1e-9
        assert np.all(K[m][inside_front & (d > 0)] != 0.0)


def test_straight_fault_symmetry_and_self_term():
    xa, xb = straight_fault(48)
    pr = Problem(xa, xb, dt=0.5)
    K = pr.kernel_tensor(30)
    assert np.allclose(K, np.transpose(K, (0, 2, 1)), rtol=0, atol=1e-15)
    assert np.all(np.diag(K[0]) == -0.5)


def test_traction_projection_rotation_invariance():
    """Rotating the whole geometry leaves tractions unchanged."""
    xa, xb = curved_fault(40)
    pr = Problem(xa, xb, dt=0.5)
    a = 0.7
    Rm = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
    pr2 = Problem(xa @ Rm.T + 3.0, xb @ Rm.T + 3.0, dt=0.5)
    K1 = pr.kernel_tensor(12)
    K2 = pr2.kernel_tensor(12)
    # Entries whose source end point lies on the wavefront at a collocation
    # time behave like sqrt(b t - r) there: a 1e-15 change of r from rounding
    # moves them by ~1e-9.  Every other entry agrees to rounding.
    d = np.abs(K1 - K2)
    N = pr.n
    i = np.arange(N)[:, None]
    j = np.arange(N)[None, :]
    X, Y = pr.local_coords(pr.center[i], j)
    re = np.stack([np.hypot(X + pr.half[j], Y), np.hypot(X - pr.half[j], Y)])
    for m in range(12):
        fronts = np.array([m * pr.dt, (m + 1) * pr.dt]) * pr.beta
        graze = np.any(np.abs(re[:, None] - fronts[None, :, None, None]) < 1e-9, axis=(0, 1))
        assert np.all(d[m][~graze] <= 1e-12)
        assert np.all(d[m][graze] <= 1e-7)


@pytest.mark.parametrize("mu,beta", [(1.0, 1.0), (2.5, 1.7)])
def test_second_lag_self_term_special_value(mu, beta):
    """With beta dt = dx/2 the second-lag self term has a value worked out by
    hand from the step response at t = dt (front at the element edges: the
    radiation damping) and t = 2 dt (front one element half-width beyond the
    edges: arcsine terms pi/3, root terms 2 sqrt(3)):
    K_ii,1 = -(mu / (pi beta)) (sqrt(3) - pi/3), -0.2179955620884587 at
    mu = beta = 1."""
    pr = Problem(*straight_fault(8), mu=mu, beta=beta, dt=0.5 / beta)
    K = pr.kernel_tensor(3)
    ref = -(mu / (math.pi * beta)) * (math.sqrt(3.0) - math.pi / 3.0)
    for i in range(8):
        assert K[1][i][i] == pytest.approx(ref, rel=1e-14, abs=0)
    if mu == 1.0 and beta == 1.0:
        assert ref == pytest.approx(-0.2179955620884587, rel=1e-15)
