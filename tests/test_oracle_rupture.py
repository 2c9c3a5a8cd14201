"""Pins of the dynamic-rupture oracle against what the mechanics fixes.

  * a fault ruptured everywhere at once: away from its ends, the tractions of
    the other elements cancel (a uniform slip rate on a line radiates a plane
    wave), so each element is a slider with radiation damping mu/(2 beta),
    T0 - (mu/(2 beta)) D_n = strength(slip_{n-1} + dt D_n).  The test solves
    that scalar recursion by its own bisection.  The end effects travel one
    element per step (a source element is felt once the wave from its near
    edge arrives, and the next element's near edge is half an element
    further), so element i keeps the slider's slip rate while n <= i;
  * a fault loaded below the yield traction everywhere never slips;
  * causality: an element cannot slip before the first step at which some
    chain of nonzero kernel entries (source j reaches receiver i at lag m)
    connects it to the nucleation patch;
  * mirror symmetry of a symmetric problem;
  * the exponential law tends to the static-dynamic one as D_c -> 0.
Planted mistakes in the oracle (half the radiation damping, the first lag
counted again in the history, the slip update without dt, a strict yield
test) each break one of these.
"""
import numpy as np
import pytest

import oracle.rupture as rp
from oracle.kernel2d import Problem
from synth import straight_fault

MU, BETA, DT = 1.0, 1.0, 0.5


def _krows(N, M):
    xa, xb = straight_fault(N)
    K = Problem(xa, xb, mu=MU, beta=BETA, dt=DT).kernel_tensor(M)
    return np.ascontiguousarray(np.transpose(K, (1, 2, 0))), 0.5 * (xa[:, 0] + xb[:, 0])


def _strength(fr, slip):
    """The two laws as the paper states them (written here, not taken from the oracle)."""
    if fr.law == "static_dynamic":
        return fr.t_dy
    return (fr.t_th - fr.t_dy) * np.exp(-slip / fr.d_c) + fr.t_dy


def _slider(fr, t0, steps):
    """Radiation-damped slider: D_n from T0 - (mu/2beta) D = strength(u + dt D)."""
    eta = MU / (2 * BETA)
    u, out = 0.0, []
    for _ in range(steps):
        lo, hi = 0.0, (t0 - fr.t_dy) / eta
        f = lambda D: t0 - eta * D - float(_strength(fr, u + DT * D))  # noqa: E731
        if f(0.0) <= 0.0:
            d = 0.0
        else:
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if f(mid) > 0.0:
                    lo = mid
                else:
                    hi = mid
            d = 0.5 * (lo + hi)
        out.append(d)
        u += DT * d
    return np.array(out)


def _uniform_case(fr, N=48, steps=40):
    """Uniform initial traction at the yield value (static-dynamic law: it
    ruptures and drops to T_dy) or 10% above it (exponential law: at the
    yield value and zero slip the strength equals the traction, so it would
    stay stuck)."""
    Kr, _ = _krows(N, steps)
    t0 = fr.t_th * (1.0 if fr.law == "static_dynamic" else 1.1)
    D, T, slip, rup = rp.simulate(Kr, np.full(N, t0), fr, steps)
    ref = _slider(fr, t0, steps)
    if not ref.all():
        return False
    i = np.arange(N)
    for n in range(steps):
        interior = np.minimum(i, N - 1 - i) >= n
        if not np.allclose(D[n, interior], ref[n], rtol=1e-11, atol=1e-13):
            return False
    return bool(rup.all())


@pytest.mark.parametrize("law", ["static_dynamic", "exp"])
def test_uniform_rupture_is_the_radiation_damped_slider(law):
    fr = rp.Friction(law, t_th=1.0, t_dy=0.2, d_c=2.0, dt=DT)
    assert _uniform_case(fr)


def test_below_yield_nothing_slips():
    N, steps = 32, 30
    Kr, x = _krows(N, steps)
    fr = rp.Friction("exp", t_th=1.0, t_dy=0.0, d_c=0.1, dt=DT)
    T0 = np.linspace(0.2, 0.99, N)
    D, T, slip, rup = rp.simulate(Kr, T0, fr, steps)
    assert not D.any() and not rup.any()
    assert np.array_equal(T, np.broadcast_to(T0, T.shape))


def _asperity_case(fr, N=48, steps=60, over=0.1):
    Kr, x = _krows(N, steps)
    T0 = rp.single_asperity_stress(x, 0.3, fr.t_th * (1 + over), 20.0, 28.0)
    return x, rp.simulate(Kr, T0, fr, steps)


def _earliest_slip(x, steps, patch):
    """Earliest step at which element i can carry load from the patch: the
    shortest path over 'source j reaches receiver i at its first lag m', with
    m the first lag whose collocation time (m + 1) dt puts the S front past
    the source's near edge (the kernel's support, from the geometry alone)."""
    N = len(x)
    e = np.full(N, np.inf)
    e[patch] = 0.0
    gap = np.maximum(np.abs(x[:, None] - x[None, :]) - 0.5, 0.0)  # collocation point to source edge
    first = np.floor(gap / (BETA * DT)).astype(float)  # (m + 1) dt beta > gap
    np.fill_diagonal(first, 0.0)
    for _ in range(N):
        e = np.minimum(e, (e[None, :] + np.maximum(first, 1.0)).min(axis=1))
    return e


def test_rupture_front_is_causal_and_symmetric():
    fr = rp.Friction("static_dynamic", t_th=1.0, t_dy=0.0, dt=DT)
    x, (D, T, slip, rup) = _asperity_case(fr)
    N, steps = len(x), D.shape[0]
    e = _earliest_slip(x, steps, (x > 20.0) & (x < 28.0))
    n = np.arange(steps)[:, None]
    assert not D[n < e[None, :]].any()
    assert rup.sum() > 8  # the rupture leaves the patch
    assert np.allclose(D, D[:, ::-1], rtol=1e-10, atol=1e-12 * np.abs(D).max())


def test_exponential_law_tends_to_static_dynamic():
    sd = rp.Friction("static_dynamic", t_th=1.0, t_dy=0.1, dt=DT)
    ex = rp.Friction("exp", t_th=1.0, t_dy=0.1, d_c=1e-10, dt=DT)
    _, (D1, T1, _, r1) = _asperity_case(sd, steps=40)
    _, (D2, T2, _, r2) = _asperity_case(ex, steps=40)
    assert np.array_equal(r1, r2)
    assert np.allclose(D2, D1, rtol=1e-8, atol=1e-12)


def _pins_hold():
    try:
        for law in ("static_dynamic", "exp"):
            if not _uniform_case(rp.Friction(law, t_th=1.0, t_dy=0.2, d_c=2.0, dt=DT), N=24, steps=20):
                return False
    except (AssertionError, ValueError):
        return False
    return True


@pytest.mark.parametrize("mutant", ["damping_halved", "first_lag_in_history", "slip_without_dt", "strict_yield"])
def test_planted_mistakes_fail_a_pin(monkeypatch, mutant):
    solve, strength = rp.solve_element, rp.Friction.strength
    if mutant == "damping_halved":
        monkeypatch.setattr(rp, "solve_element", lambda fr, ts, k0, s: solve(fr, ts, k0 / 2, s))
    elif mutant == "first_lag_in_history":
        orig = rp.simulate

        def sim(Kr, T0, fr, steps, ruptured=None):
            Kr2 = Kr.copy()
            Kr2[:, :, 1] += Kr[:, :, 0]  # the self term once more, one step late
            return orig(Kr2, T0, fr, steps, ruptured)

        monkeypatch.setattr(rp, "simulate", sim)
    elif mutant == "slip_without_dt":
        monkeypatch.setattr(rp.Friction, "strength", lambda self, s: strength(self, s / self.dt))
    else:
        orig_solve = rp.solve_element

        def strict(fr, ts, k0, s):
            return 0.0 if ts <= fr.t_th and s == 0.0 else orig_solve(fr, ts, k0, s)

        monkeypatch.setattr(rp, "solve_element", strict)
    assert not _pins_hold()


def test_pins_hold_for_the_oracle():
    assert _pins_hold()
