"""Brute-force quadrature of the anti-plane Green's-function representation.

Test infrastructure: an independent route to the step response of a
uniformly slipping segment (the stress at time t due to unit slip rate
switched on at tau = 0 on [-h, h] x {0}), used to pin the oracle's closed
form and quantities built from it.
"""
import math

from scipy import integrate


# ---------------------------------------------------------------------------
# Brute-force route: the double-layer representation of a slipping segment.
#
# With g the 2D scalar Green's function of rho w_tt = mu lap w, a slip
# Delta w(xi, tau) = tau H(tau) on [-h, h] gives w = -mu d_y Phi with
# Phi = int dxi int dtau tau g = (1/(2 pi mu b)) int dxi F(r, b t),
# F(r, T) = T acosh(T/r) - sqrt(T^2 - r^2).  Differentiating under the
# integral and substituting u = x - xi = q sin(theta), q^2 = T^2 - y^2
# (so that du / sqrt(q^2 - u^2) = d theta) leaves smooth integrands that we
# integrate numerically.
# ---------------------------------------------------------------------------
def brute_stress(X, Y, t, h, mu, beta):
    T = beta * t
    if T <= abs(Y):
        return 0.0, 0.0
    q = math.sqrt(T * T - Y * Y)
    lo = max(-1.0, (X - h) / q)
    hi = min(1.0, (X + h) / q)
    if lo >= hi:
        return 0.0, 0.0
    th_lo, th_hi = math.asin(lo), math.asin(hi)

    def g_yz(th):
        u = q * math.sin(th)
        R = q * math.cos(th)
        r2 = u * u + Y * Y
        return Y * Y / r2 - R * R * (r2 - 2 * Y * Y) / (r2 * r2)

    def g_xz(th):
        u = q * math.sin(th)
        R = q * math.cos(th)
        r2 = u * u + Y * Y
        return Y * u * (1.0 / r2 + 2 * R * R / (r2 * r2))

    pts = None
    if th_lo < 0.0 < th_hi:
        pts = [0.0]
    iy, _ = integrate.quad(g_yz, th_lo, th_hi, points=pts, epsabs=1e-13, epsrel=1e-12, limit=400)
    ix, _ = integrate.quad(g_xz, th_lo, th_hi, points=pts, epsabs=1e-13, epsrel=1e-12, limit=400)
    c = mu / (2 * math.pi * beta)
    return -c * ix, -c * iy
