// Closed-form step response of the 2D anti-plane problem (host and device).
//
// A source element is the segment [-h, h] x {0} in its own frame (tangent X,
// normal Y).  With a unit slip rate switched on at t = 0 (slip = t), the
// stress vector at a receiver (X, Y) follows from the double-layer
// representation with the 2D scalar Green's function, integrated in closed
// form over the element:
//   q = sqrt(b^2 t^2 - Y^2),  R+- = sqrt(max(b^2 t^2 - (X +- h)^2 - Y^2, 0))
//   s_yz = -(mu/(2 pi b)) [asin(clip((X+h)/q)) - asin(clip((X-h)/q))
//                          + (X+h) R+/r+^2 - (X-h) R-/r-^2]
//   s_xz = +(mu/(2 pi b)) Y [R+/r+^2 - R-/r-^2]
// and S(t <= 0) = 0.  The late-time slope is the elastostatic field of a
// unit slip (Domain S, Sec. 2.2).  The discrete kernel with eps_t is
//   K_m = S((m + eps_t) dt) - S((m + eps_t - 1) dt)      (Eq. 4).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace bie {

struct Frame {
    double cx, cy;   // element midpoint
    double tx, ty;   // unit tangent
    double nx, ny;   // unit normal = tangent rotated by +90 degrees
    double h;        // half length
};

__host__ __device__ inline double clip1(double v) { return v > 1.0 ? 1.0 : (v < -1.0 ? -1.0 : v); }

// Stress vector (s_xz, s_yz) in the source frame.
__host__ __device__ inline void step_local(double X, double Y, double t, double h, double mu,
                                           double beta, double *sX, double *sY) {
    if (!(t > 0.0)) {
        *sX = 0.0;
        *sY = 0.0;
        return;
    }
    const double bt = beta * t;
    const double bt2 = bt * bt;
    const double Y2 = Y * Y;
    const double up = X + h, um = X - h;
    const double rp2 = up * up + Y2, rm2 = um * um + Y2;
    const double dp = bt2 - rp2, dm = bt2 - rm2;
    const double ap = dp > 0.0 ? sqrt(dp) / rp2 : 0.0;
    const double am = dm > 0.0 ? sqrt(dm) / rm2 : 0.0;
    double I = 0.0;
    if (bt > fabs(Y)) {
        const double q = sqrt(bt2 - Y2);
        I = asin(clip1(up / q)) - asin(clip1(um / q));
    }
    const double c = mu / (2.0 * M_PI * beta);
    *sY = -c * (I + up * ap - um * am);
    *sX = c * Y * (ap - am);
}

// Elastostatic stress of a unit slip (late-time slope), source frame.
__host__ __device__ inline void static_local(double X, double Y, double h, double mu, double *sX,
                                             double *sY) {
    const double up = X + h, um = X - h;
    const double rp2 = up * up + Y * Y, rm2 = um * um + Y * Y;
    const double c = mu / (2.0 * M_PI);
    *sY = -c * (up / rp2 - um / rm2);
    *sX = c * Y * (1.0 / rp2 - 1.0 / rm2);
}

// Global stress vector at point (px, py) due to the source of frame f.
__host__ __device__ inline void stress_step(const Frame &f, double px, double py, double t,
                                            double mu, double beta, double *sx, double *sy) {
    const double dx = px - f.cx, dy = py - f.cy;
    const double X = dx * f.tx + dy * f.ty;
    const double Y = dx * f.nx + dy * f.ny;
    double sX, sY;
    step_local(X, Y, t, f.h, mu, beta, &sX, &sY);
    *sx = sX * f.tx + sY * f.nx;
    *sy = sX * f.ty + sY * f.ny;
}

__host__ __device__ inline void stress_static(const Frame &f, double px, double py, double mu,
                                              double *sx, double *sy) {
    const double dx = px - f.cx, dy = py - f.cy;
    const double X = dx * f.tx + dy * f.ty;
    const double Y = dx * f.nx + dy * f.ny;
    double sX, sY;
    static_local(X, Y, f.h, mu, &sX, &sY);
    *sx = sX * f.tx + sY * f.nx;
    *sy = sX * f.ty + sY * f.ny;
}

// Projection of the step response on direction (ex, ey): traction on a
// receiver whose normal is (ex, ey), or one stress component.
__host__ __device__ inline double proj_step(const Frame &f, double px, double py, double ex,
                                            double ey, double t, double mu, double beta) {
    double sx, sy;
    stress_step(f, px, py, t, mu, beta, &sx, &sy);
    return sx * ex + sy * ey;
}

__host__ __device__ inline double proj_static(const Frame &f, double px, double py, double ex,
                                              double ey, double mu) {
    double sx, sy;
    stress_static(f, px, py, mu, &sx, &sy);
    return sx * ex + sy * ey;
}

// Discrete kernel value for lag m (eps_t folded into t0 = (m + eps_t - 1) dt).
__host__ __device__ inline double proj_kernel(const Frame &f, double px, double py, double ex,
                                              double ey, int64_t m, double dt, double eps_t,
                                              double mu, double beta) {
    const double t1 = ((double)m + eps_t) * dt;
    const double t0 = ((double)m + eps_t - 1.0) * dt;
    return proj_step(f, px, py, ex, ey, t1, mu, beta) - proj_step(f, px, py, ex, ey, t0, mu, beta);
}

// ------------------------------------------------------------ in-plane --
// Straight fault, plane strain, P and S speeds alpha > beta.  Step response
// of the segment [-h, h] x {0} (unit slip rate, resp. opening rate, from
// t = 0) at the on-fault receiver (x, 0); by mirror symmetry the shear
// traction depends on the slip only and the normal traction on the opening
// only.  With, for c in {alpha, beta},
//   A_c = asin(clip((x+h)/(c t))) - asin(clip((x-h)/(c t)))
//   B_c = R_c(x+h)/(x+h) - R_c(x-h)/(x-h),  R_c(z) = sqrt(max(c^2 t^2 - z^2, 0))
//   F(z) = [Q_b (t^2 + 2 z^2/b^2) - Q_a (t^2 + 2 z^2/a^2)] / z^3,  Q_c = sqrt(max(t^2 - z^2/c^2, 0))
// (F, the near-field term between the fronts, in a cancellation-free form
// once both fronts have passed z):
//   shear  = -(mu/(2 pi b)) A_b - (2 mu/(pi b)) B_b + (2 mu b^2/(pi a^3)) B_a + (2 mu b^2/(3 pi)) dF
//   normal = -(mu a/(2 pi b^2)) A_a - (2 mu/(pi a)) B_a + (2 mu/(pi b)) B_b - (2 mu b^2/(3 pi)) dF
// with dF = F(x+h) - F(x-h).  Radiation damping -mu/(2b) and -mu a/(2 b^2);
// late-time slope 2 (1 - b^2/a^2) times the anti-plane static field.
__host__ __device__ inline double inplane_front(double z, double ct) {
    const double d = ct * ct - z * z;
    return d > 0.0 ? sqrt(d) / z : 0.0;
}

__host__ __device__ inline double inplane_near(double z, double t, double a, double b) {
    const double az = fabs(z);
    if (!(t > az / a)) return 0.0;
    const double qa2 = t * t - z * z / (a * a);
    const double qa = qa2 > 0.0 ? sqrt(qa2) : 0.0;
    if (t > az / b) {
        const double qb = sqrt(t * t - z * z / (b * b));
        return (t * t * (1.0 / (a * a) - 1.0 / (b * b)) / (qb + qa) + 2.0 * (qb / (b * b) - qa / (a * a))) / z;
    }
    return -qa * (t * t + 2.0 * z * z / (a * a)) / (z * z * z);
}

// comp 0: shear traction from slip; comp 1: normal traction from opening.
__host__ __device__ inline double inplane_step(double x, double t, double h, double mu, double a, double b,
                                               int comp) {
    if (!(t > 0.0)) return 0.0;
    const double up = x + h, um = x - h;
    const double at = a * t, bt = b * t;
    const double Aa = asin(clip1(up / at)) - asin(clip1(um / at));
    const double Ab = asin(clip1(up / bt)) - asin(clip1(um / bt));
    const double Ba = inplane_front(up, at) - inplane_front(um, at);
    const double Bb = inplane_front(up, bt) - inplane_front(um, bt);
    const double dF = inplane_near(up, t, a, b) - inplane_near(um, t, a, b);
    if (comp == 0)
        return -(mu / (2.0 * M_PI * b)) * Ab - (2.0 * mu / (M_PI * b)) * Bb + (2.0 * mu * b * b / (M_PI * a * a * a)) * Ba +
               (2.0 * mu * b * b / (3.0 * M_PI)) * dF;
    return -(mu * a / (2.0 * M_PI * b * b)) * Aa - (2.0 * mu / (M_PI * a)) * Ba + (2.0 * mu / (M_PI * b)) * Bb -
           (2.0 * mu * b * b / (3.0 * M_PI)) * dF;
}

}  // namespace bie
