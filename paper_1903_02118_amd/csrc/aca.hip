// ACA+ (partially pivoted adaptive cross approximation with random reference
// row and column, Sec. 6.1.1) of the admissible blocks on the device, in
// FP64.  One workgroup of 256 lanes factors one block: entries are evaluated
// from the closed-form kernel on the fly (never stored), residual rows and
// columns are spread over the lanes, pivots come from workgroup-wide argmax
// reductions and the Frobenius-norm estimate from workgroup sums.
//
// Per block, with residual S_k = A - sum_{l<k} u_l v_l^T:
//   * a random unused reference row i_r and column j_r hold residual rows /
//     columns; the next pivot row (or column) is the argmax of the larger
//     reference, the pivot column (row) the argmax of that residual row;
//   * u_k = S_k(:, j_p), v_k = S_k(i_p, :) / S_k(i_p, j_p);
//   * ||S||^2 estimate: ||A_k||^2 = ||A_{k-1}||^2 + 2 sum_l (u_k.u_l)(v_k.v_l)
//     + |u_k|^2 |v_k|^2;
//   * stop when |u_k||v_k| and the reference residuals (scaled to the block)
//     are within eps ||A_k||, confirmed on two fresh random rows and columns;
//     when both references vanish, fresh ones are drawn three times, then
//     every unused row is swept: stop if the whole residual is within
//     eps ||A_k||, else pivot on its largest entry.
// A block that reaches its stored rank cap without converging is reported
// (ACA_CAPPED) and factored again on the host.  The random draws use
// SplitMix64 (Steele, Lea and Flood, 2014) on a per-block counter.
#include "bie_internal.hpp"

namespace bie {

namespace {

constexpr int AT = 256;  // lanes per block
constexpr int AW = AT / 64;

__device__ inline uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Red {
    double d[AW][4];
    int i[AW];
    double v[AW];
};

__device__ inline double wave_sum(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Sums of n <= 4 values over the workgroup; every lane gets the same result.
__device__ inline void block_sum(double (&x)[4], int n, Red &R) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = 0; k < n; ++k) x[k] = wave_sum(x[k]);
    __syncthreads();
    if (lane == 0)
        for (int k = 0; k < n; ++k) R.d[w][k] = x[k];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        double t = 0.0;
        for (int q = 0; q < AW; ++q) t += R.d[q][k];
        x[k] = t;
    }
}

// Index of the largest |v[j]| over unused j (the smallest such index on
// ties), -1 when every index is used; *absmax gets |v| there (0 if none).
__device__ inline int block_argmax(const double *v, const uint8_t *used, int n, double *absmax, Red &R) {
    double bv = -1.0;
    int bi = -1;
    for (int j = threadIdx.x; j < n; j += AT)
        if (!used[j]) {
            const double a = fabs(v[j]);
            if (a > bv) {
                bv = a;
                bi = j;
            }
        }
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ov > bv || (ov == bv && oi >= 0 && (bi < 0 || oi < bi))) {
            bv = ov;
            bi = oi;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        R.v[w] = bv;
        R.i[w] = bi;
    }
    __syncthreads();
    bv = -1.0;
    bi = -1;
    for (int q = 0; q < AW; ++q) {
        const double ov = R.v[q];
        const int oi = R.i[q];
        if (ov > bv || (ov == bv && oi >= 0 && (bi < 0 || oi < bi))) {
            bv = ov;
            bi = oi;
        }
    }
    *absmax = bi >= 0 ? bv : 0.0;
    return bi;
}

// A random unused index: the first unused one at or after a uniformly drawn
// start, cyclically; -1 when every index is used.
__device__ inline int pick_unused(const uint8_t *used, int n, uint64_t draw, Red &R) {
    const int start = (int)(draw % (uint64_t)n);
    int best = n;
    for (int j = threadIdx.x; j < n; j += AT)
        if (!used[j]) best = min(best, j >= start ? j - start : j - start + n);
    for (int o = 32; o > 0; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) R.i[w] = best;
    __syncthreads();
    best = n;
    for (int q = 0; q < AW; ++q) best = min(best, R.i[q]);
    if (best >= n) return -1;
    const int k = start + best;
    return k >= n ? k - n : k;
}

struct Blk {
    const Frame *fr;
    const int32_t *ri, *si;
    const int64_t *mbar, *dmj;
    int nr, ns, kind;
    double ex, ey, sx, sy, dt, mu, beta;
    double *U, *V;  // U[l * nr + i], V[l * ns + j]
};

__device__ inline double entry(const Blk &B, const Frame &fi, const Frame &fj, int j) {
    return far_entry(fi, fj, B.kind, B.ex, B.ey, B.sx, B.sy, B.mbar[j], B.dmj[j], B.dt, B.mu, B.beta);
}

// Residual row i of the first `rank` terms into out[ns] (all lanes).
__device__ void resid_row(const Blk &B, int rank, int i, double *out, double *w) {
    __syncthreads();
    for (int l = threadIdx.x; l < rank; l += AT) w[l] = B.U[(size_t)l * B.nr + i];
    __syncthreads();
    const Frame fi = B.fr[B.ri[i]];
    for (int j = threadIdx.x; j < B.ns; j += AT) {
        double e = entry(B, fi, B.fr[B.si[j]], j);
        for (int l = 0; l < rank; ++l) e -= w[l] * B.V[(size_t)l * B.ns + j];
        out[j] = e;
    }
    __syncthreads();
}

// Residual column j into out[nr] (all lanes).
__device__ void resid_col(const Blk &B, int rank, int j, double *out, double *w) {
    __syncthreads();
    for (int l = threadIdx.x; l < rank; l += AT) w[l] = B.V[(size_t)l * B.ns + j];
    __syncthreads();
    const Frame fj = B.fr[B.si[j]];
    for (int i = threadIdx.x; i < B.nr; i += AT) {
        double e = entry(B, B.fr[B.ri[i]], fj, j);
        for (int l = 0; l < rank; ++l) e -= B.U[(size_t)l * B.nr + i] * w[l];
        out[i] = e;
    }
    __syncthreads();
}

__device__ inline void sumsq2(const double *a, int na, const double *b, int nb, double (&x)[4], Red &R) {
    x[0] = x[1] = x[2] = x[3] = 0.0;
    for (int k = threadIdx.x; k < na; k += AT) x[0] += a[k] * a[k];
    for (int k = threadIdx.x; k < nb; k += AT) x[1] += b[k] * b[k];
    block_sum(x, 2, R);
}

__device__ inline void set_flag(uint8_t *f, int k) {
    __syncthreads();
    if (threadIdx.x == 0) f[k] = 1;
    __syncthreads();
}

__global__ __launch_bounds__(AT) void k_aca(const Frame *fr, const AcaLeafDev *leaves, const int32_t *ridx,
                                            const int32_t *sidx, const int64_t *mbar, const int64_t *dmj,
                                            const AcaBlockDev *blocks, double *fac, double *work, uint8_t *flags,
                                            AcaOutDev *out, double dt, double mu, double beta, double eps) {
    __shared__ Red R;
    __shared__ double wl[ACA_KCAP];
    const AcaBlockDev D = blocks[blockIdx.x];
    const AcaLeafDev L = leaves[D.leaf];
    const int nr = L.nr, ns = L.ns, cap = D.cap;
    if (nr <= 0 || ns <= 0 || cap <= 0 || cap > ACA_KCAP) {  // never built so; nothing to factor
        if (threadIdx.x == 0) out[blockIdx.x] = AcaOutDev{0, nr > 0 && ns > 0 ? ACA_CAPPED : ACA_CONVERGED, 0, 0};
        return;
    }
    Blk B;
    B.fr = fr;
    B.ri = ridx + L.r_off;
    B.si = sidx + L.s_off;
    B.mbar = mbar + L.s_off;
    B.dmj = dmj + L.s_off;
    B.nr = nr;
    B.ns = ns;
    B.kind = D.kind;
    B.ex = D.ex;
    B.ey = D.ey;
    B.sx = L.sx;
    B.sy = L.sy;
    B.dt = dt;
    B.mu = mu;
    B.beta = beta;
    B.U = fac + D.fac_off;
    B.V = B.U + (size_t)cap * nr;
    double *r = work + D.work_off, *c = r + ns, *rref = c + nr, *cref = rref + ns;
    uint8_t *urow = flags + D.flag_off, *ucol = urow + nr;
    for (int k = threadIdx.x; k < nr + ns; k += AT) urow[k] = 0;
    __syncthreads();

    uint64_t ctr = 0;
    auto draw = [&]() { return splitmix64(D.seed + 0x9E3779B97F4A7C15ull * (++ctr)); };
    int rank = 0, sweeps = 0, status = ACA_CONVERGED, stall = 0;
    // every pass adds a term, retires a row or column, or draws fresh
    // references (at most three times between the other two): this bound
    // is never reached; it only guarantees the loop ends
    const int64_t max_iters = 5ll * (cap + nr + ns + 1);
    int64_t iters = 0;
    double norm2 = 0.0, x[4];
    int iref = pick_unused(urow, nr, draw(), R);
    int jref = pick_unused(ucol, ns, draw(), R);
    resid_row(B, 0, iref, rref, wl);
    resid_col(B, 0, jref, cref, wl);
    while (true) {
        if (rank >= cap || ++iters > max_iters) {
            status = ACA_CAPPED;
            break;
        }
        double vc, vr;
        const int ic = block_argmax(cref, urow, nr, &vc, R);
        const int jr = block_argmax(rref, ucol, ns, &vr, R);
        int ip = -1, jp = -1;
        if (vc == 0.0 && vr == 0.0) {
            // both references vanish: fresh ones, then a sweep of the residual
            if (++stall <= 3) {
                iref = pick_unused(urow, nr, draw(), R);
                jref = pick_unused(ucol, ns, draw(), R);
                if (iref >= 0 && jref >= 0) {
                    resid_row(B, rank, iref, rref, wl);
                    resid_col(B, rank, jref, cref, wl);
                    continue;
                }
            }
            ++sweeps;
            double rest2 = 0.0, best = 0.0;
            for (int i = 0; i < nr; ++i) {
                if (urow[i]) continue;
                resid_row(B, rank, i, r, wl);
                sumsq2(r, ns, r, 0, x, R);
                rest2 += x[0];
                double bv;
                const int jb = block_argmax(r, ucol, ns, &bv, R);
                if (jb >= 0 && bv > best) {
                    best = bv;
                    ip = i;
                    jp = jb;
                }
            }
            if (ip < 0 || sqrt(rest2) <= eps * sqrt(fmax(norm2, 0.0))) break;
            stall = 0;
            resid_row(B, rank, ip, r, wl);
            resid_col(B, rank, jp, c, wl);
        } else if (vc >= vr) {
            stall = 0;
            ip = ic;
            resid_row(B, rank, ip, r, wl);
            double bv;
            jp = block_argmax(r, ucol, ns, &bv, R);
            if (jp < 0 || r[jp] == 0.0) {
                set_flag(urow, ip);
                continue;
            }
            resid_col(B, rank, jp, c, wl);
        } else {
            stall = 0;
            jp = jr;
            resid_col(B, rank, jp, c, wl);
            double bv;
            ip = block_argmax(c, urow, nr, &bv, R);
            if (ip < 0 || c[ip] == 0.0) {
                set_flag(ucol, jp);
                continue;
            }
            resid_row(B, rank, ip, r, wl);
        }
        // new cross term
        const double piv = r[jp];
        double *Uk = B.U + (size_t)rank * nr, *Vk = B.V + (size_t)rank * ns;
        for (int i = threadIdx.x; i < nr; i += AT) Uk[i] = c[i];
        for (int j = threadIdx.x; j < ns; j += AT) Vk[j] = r[j] / piv;
        __syncthreads();
        double cross = 0.0;
        for (int l0 = 0; l0 < rank; l0 += 2) {
            const bool two = l0 + 1 < rank;
            const double *U0 = B.U + (size_t)l0 * nr, *V0 = B.V + (size_t)l0 * ns;
            x[0] = x[1] = x[2] = x[3] = 0.0;
            for (int i = threadIdx.x; i < nr; i += AT) {
                x[0] += Uk[i] * U0[i];
                if (two) x[2] += Uk[i] * U0[nr + i];
            }
            for (int j = threadIdx.x; j < ns; j += AT) {
                x[1] += Vk[j] * V0[j];
                if (two) x[3] += Vk[j] * V0[ns + j];
            }
            block_sum(x, 4, R);
            cross += x[0] * x[1] + (two ? x[2] * x[3] : 0.0);
        }
        sumsq2(Uk, nr, Vk, ns, x, R);
        const double nu = sqrt(x[0]), nv = sqrt(x[1]);
        norm2 += 2.0 * cross + x[0] * x[1];
        ++rank;
        // the references lose the new term
        const double uref = iref >= 0 ? Uk[iref] : 0.0, vref = jref >= 0 ? Vk[jref] : 0.0;
        for (int j = threadIdx.x; j < ns; j += AT) rref[j] -= uref * Vk[j];
        for (int i = threadIdx.x; i < nr; i += AT) cref[i] -= Uk[i] * vref;
        __syncthreads();
        if (threadIdx.x == 0) {
            urow[ip] = 1;
            ucol[jp] = 1;
        }
        __syncthreads();
        if (iref >= 0 && urow[iref]) {
            const int k = pick_unused(urow, nr, draw(), R);
            if (k >= 0) {
                iref = k;
                resid_row(B, rank, iref, rref, wl);
            }
        }
        if (jref >= 0 && ucol[jref]) {
            const int k = pick_unused(ucol, ns, draw(), R);
            if (k >= 0) {
                jref = k;
                resid_col(B, rank, jref, cref, wl);
            }
        }
        sumsq2(cref, nr, rref, ns, x, R);
        const double snorm = sqrt(fmax(norm2, 0.0));
        const double rest = fmax(sqrt(x[0]) * sqrt((double)ns), sqrt(x[1]) * sqrt((double)nr));
        if (nu * nv <= eps * snorm && rest <= eps * snorm) {
            // confirm on fresh random rows and columns; a probe above the
            // bound becomes the new reference pair
            bool pass = true;
            for (int probe = 0; probe < 2 && pass; ++probe) {
                const int ip2 = pick_unused(urow, nr, draw(), R);
                const int jp2 = pick_unused(ucol, ns, draw(), R);
                if (ip2 < 0 || jp2 < 0) break;
                resid_row(B, rank, ip2, r, wl);
                resid_col(B, rank, jp2, c, wl);
                sumsq2(c, nr, r, ns, x, R);
                if (fmax(sqrt(x[0]) * sqrt((double)ns), sqrt(x[1]) * sqrt((double)nr)) > eps * snorm) {
                    pass = false;
                    iref = ip2;
                    jref = jp2;
                    for (int j = threadIdx.x; j < ns; j += AT) rref[j] = r[j];
                    for (int i = threadIdx.x; i < nr; i += AT) cref[i] = c[i];
                    __syncthreads();
                }
            }
            if (pass) break;
        }
    }
    if (threadIdx.x == 0) {
        AcaOutDev o;
        o.rank = rank;
        o.status = status;
        o.sweeps = sweeps;
        o.reserved = 0;
        out[blockIdx.x] = o;
    }
}

}  // namespace

int launch_aca(const Frame *fr, const AcaLeafDev *leaves, const int32_t *ridx, const int32_t *sidx,
               const int64_t *mbar, const int64_t *dmj, const AcaBlockDev *blocks, int64_t n_blocks, double *fac,
               double *work, uint8_t *flags, AcaOutDev *out, double dt, double mu, double beta, double eps,
               hipStream_t s) {
    if (n_blocks <= 0) return BIE_OK;
    if (n_blocks > 0x7fffffff) {
        set_error("too many admissible blocks for one ACA+ dispatch");
        return BIE_EINVAL;
    }
    hipLaunchKernelGGL(k_aca, dim3((unsigned)n_blocks), dim3(AT), 0, s, fr, leaves, ridx, sidx, mbar, dmj, blocks, fac,
                       work, flags, out, dt, mu, beta, eps);
    BIE_HIP_TRY(hipGetLastError());
    return BIE_OK;
}

}  // namespace bie
