// Device kernels of the BIEM convolution library (gfx950, wave64).
//
// Setup kernels: dense kernel tensor (Eq. 4), near-field windows and their
// static cut-off (App. E with the eps_Q / eps_st rule of Apps. A.1, H.1).
// Per-step kernels of the plain form: history update and the dense sum.
// Per-step kernels of the FDP=H form (Sec. 5 and App. B):
//   update   D_n into the near history (time-reversed rings), the running
//            sum U_n (for the static part of the near pairs, App. E) and the
//            time-major recent history read by the far-field FIR;
//   near     windowed convolution of every inadmissible pair, one work item
//            per (32 x 32 tile, 128-lag chunk), source history staged in LDS;
//            the windows hold K_ij,m - K^S_ij dt, the deviation from the
//            static rate, so that K^S_ij dt U_n adds the static part of every
//            lag, inside the window and past it;
//   far_src  D -> D^ (Eq. 52) and the scatter G D^ into the representative-
//            stress rings (Eq. 56; the shift M is a moving base index);
//   tr_fir   2D Domain-S transient: temporal FIR of the transient rings
//            (App. B.3);
//   recv     per receiver: near partial sums, K^S_ij dt U_n of its near pairs, the gather
//            F T' (Eqs. 57/59) for Domain F and the transient, and the
//            Domain-S increment into the FP64 running stress (App. B.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "bie_internal.hpp"

namespace bie {

// Per-step scratch of bie_run_static (the partial sums of the dense lag
// chunks or of the near-field work items), for callers that cannot allocate:
// one copy per GPU, held until the process ends.  Host code never uses the
// array's name: its device address comes from hipGetSymbolAddress, once per
// device, with that device current.
static __device__ __align__(256) double scratch[BIE_STATIC_SCRATCH_BYTES / sizeof(double)];

int static_scratch_ptr(double **out) {
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static double *ptr[MAX_DEVICES] = {};
    int dev = -1;
    BIE_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_error("bie_run_static: device index " + std::to_string(dev) + " beyond the supported 64");
        return BIE_EINVAL;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        BIE_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("bie_run_static: hipGetSymbolAddress returned a null address");
            return BIE_EHIP;
        }
        ptr[dev] = static_cast<double *>(p);
    }
    *out = ptr[dev];
    return BIE_OK;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Low-rank factors are stored as FP64, FP32 or BF16 (bit patterns); a BF16
// value is the upper half of the FP32 with the same bits.
struct bf16_t {
    uint16_t bits;
};
__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ double widen(float v) { return (double)v; }
__device__ __forceinline__ double widen(bf16_t v) { return (double)__uint_as_float((uint32_t)v.bits << 16); }

// ============================================================ setup kernels
// First lag at which source j is inside receiver i's causal band (the bands
// grow with the lag), or M if never.
__device__ inline int band_entry_lag(const int64_t *__restrict__ off, const int32_t *__restrict__ blo, int N, int M,
                                     int i, int j) {
    int lo = 0, hi = M;  // the answer is in [lo, hi]
    while (lo < hi) {
        const int m = (lo + hi) >> 1;
        const int64_t r = (int64_t)m * N + i;
        const int a = blo[r];
        const int64_t w = off[r + 1] - off[r];
        if (j >= a && j < a + w) hi = m; else lo = m + 1;
    }
    return lo;
}

// K_ij,m inside the causal band, one thread per (i, j): the step response
// differenced over each step from the lag the pair enters the band.
// comp < 0: anti-plane (stress projected on the receiver normal); else the
// in-plane component comp (receivers at signed distance x along the source).
__global__ void k_dense_build(const Frame *__restrict__ fr, const int64_t *__restrict__ off,
                              const int32_t *__restrict__ blo, int N, int M, double dt, double eps_t, double mu,
                              double alpha, double beta, int comp, double *__restrict__ K) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)N * N) return;
    const int i = (int)(idx / N), j = (int)(idx % N);
    const int m_in = band_entry_lag(off, blo, N, M, i, j);
    if (m_in >= M) return;
    const Frame fi = fr[i], fj = fr[j];
    const double x = (fi.cx - fj.cx) * fj.tx + (fi.cy - fj.cy) * fj.ty;
    auto S = [&](double t) {
        return comp < 0 ? proj_step(fj, fi.cx, fi.cy, fi.nx, fi.ny, t, mu, beta)
                        : inplane_step(x, t, fj.h, mu, alpha, beta, comp);
    };
    double prev = S(((double)m_in + eps_t - 1.0) * dt);
    for (int m = m_in; m < M; ++m) {
        const double cur = S(((double)m + eps_t) * dt);
        const int64_t r = (int64_t)m * N + i;
        K[off[r] + (j - blo[r])] = cur - prev;
        prev = cur;
    }
}

int launch_dense_build(const Geometry &g, const DenseOp &d, hipStream_t s) {
    const int64_t n = (int64_t)d.N * d.N;
    const int bs = 256;
    BIE_HIP_TRY(hipMemsetAsync(d.K, 0, (size_t)d.ncomp * d.E * sizeof(double), s));  // band padding
    for (int c = 0; c < d.ncomp; ++c)
        hipLaunchKernelGGL(k_dense_build, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, d.dfr, d.off, d.blo,
                           d.N, d.M, g.dt, g.eps_t, g.mu, g.alpha, g.beta, d.ncomp == 1 ? -1 : c, d.K + (size_t)c * d.E);
    BIE_HIP_TRY(hipGetLastError());
    return BIE_OK;
}

// W_ij: one past the last lag m < M_k (the lag count of the pair's problem)
// where |K_ij,m - K^S_ij dt| exceeds min(eps_q |K^S_ij dt|, tol_abs);
// K^S_ij dt is kept per pair.  The scan runs down from the last lag and stops
// at the first violation: on a nonplanar fault the deviation can change sign
// after the fronts have passed, so no lag above W_ij may be skipped.
__global__ void k_near_windows(const Frame *__restrict__ fr, const int32_t *__restrict__ prec,
                               const int32_t *__restrict__ psrc, const int32_t *__restrict__ hz, int64_t np,
                               double dt, double mu, double beta, double eps_q, double tol_abs,
                               int32_t *__restrict__ W, double *__restrict__ ks) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    if (prec[p] < 0) {  // placeholder between packed sub-blocks: no window
        W[p] = 0;
        ks[p] = 0.0;
        return;
    }
    const Frame fi = fr[prec[p]], fj = fr[psrc[p]];
    const int M = hz[prec[p]];
    const double kst = proj_static(fj, fi.cx, fi.cy, fi.nx, fi.ny, mu) * dt;
    const double tol = fmin(eps_q * fabs(kst), tol_abs);
    double s_hi = proj_step(fj, fi.cx, fi.cy, fi.nx, fi.ny, (double)M * dt, mu, beta);
    int w = 0;
    for (int m = M - 1; m >= 0; --m) {
        const double s_lo = proj_step(fj, fi.cx, fi.cy, fi.nx, fi.ny, (double)m * dt, mu, beta);
        if (fabs((s_hi - s_lo) - kst) > tol) {
            w = m + 1;
            break;
        }
        s_hi = s_lo;
    }
    W[p] = w;
    ks[p] = kst;
}

int launch_near_windows(const Geometry &g, const Frame *dfr, const int32_t *d_prec, const int32_t *d_psrc,
                        const int32_t *d_hz, int64_t n_pairs, double eps_q, double tol_abs, int32_t *d_W,
                        double *d_ks, hipStream_t s) {
    const int bs = 128;
    hipLaunchKernelGGL(k_near_windows, dim3((unsigned)((n_pairs + bs - 1) / bs)), dim3(bs), 0, s, dfr, d_prec, d_psrc,
                       d_hz, n_pairs, g.dt, g.mu, g.beta, eps_q, tol_abs, d_W, d_ks);
    BIE_HIP_TRY(hipGetLastError());
    return BIE_OK;
}

// Windows in the chunk-major layout: lag m of pair p goes to item
// tile_item0[tile] + m / chunk, at item_base + item_rel[q] + m % chunk.
// One workgroup per pair, striding over the pairs: a dispatch counts its
// work-items in 32 bits, so the grid stays far below 2^32 / 256 workgroups.
template <class T>
__global__ void k_near_fill(const Frame *__restrict__ fr, const int32_t *__restrict__ prec,
                            const int32_t *__restrict__ psrc, const int32_t *__restrict__ W,
                            const int32_t *__restrict__ ptile, const int32_t *__restrict__ pq,
                            const int32_t *__restrict__ tile_item0, const int64_t *__restrict__ item_base,
                            const int32_t *__restrict__ item_rel, const double *__restrict__ ks, int64_t np,
                            int chunk, double dt, double mu, double beta, T *__restrict__ Kw) {
    for (int64_t p = blockIdx.x; p < np; p += gridDim.x) {
        if (prec[p] < 0) continue;  // placeholder pair
        const Frame fi = fr[prec[p]], fj = fr[psrc[p]];
        const int w = W[p];
        const double kst = ks[p];
        const int item0 = tile_item0[ptile[p]];
        const int q = pq[p];
        for (int m = threadIdx.x; m < w; m += blockDim.x) {
            const int item = item0 + m / chunk;
            const int64_t dst = item_base[item] + item_rel[(int64_t)item * (TILE * TILE) + q] + (m % chunk);
            const double k = proj_step(fj, fi.cx, fi.cy, fi.nx, fi.ny, (double)(m + 1) * dt, mu, beta) -
                             proj_step(fj, fi.cx, fi.cy, fi.nx, fi.ny, (double)m * dt, mu, beta);
            Kw[dst] = (T)(k - kst);
        }
    }
}

int launch_near_fill(const Geometry &g, const FdphOp &f, const int32_t *d_prec, const int32_t *d_ptile,
                     const int32_t *d_pq, const int32_t *d_tile_item0, const double *d_ks, hipStream_t s) {
    const unsigned grid = (unsigned)std::min<int64_t>(f.n_pairs, MAX_GRID_BLOCKS);
    if (f.precision == BIE_FP64)
        hipLaunchKernelGGL(k_near_fill<double>, dim3(grid), dim3(256), 0, s, f.dfr, d_prec, f.pSrc, f.pW, d_ptile,
                           d_pq, d_tile_item0, f.item_base, f.item_rel, d_ks, f.n_pairs, f.near_chunk, g.dt, g.mu,
                           g.beta, f.Kw);
    else
        hipLaunchKernelGGL(k_near_fill<float>, dim3(grid), dim3(256), 0, s, f.dfr, d_prec, f.pSrc, f.pW, d_ptile,
                           d_pq, d_tile_item0, f.item_base, f.item_rel, d_ks, f.n_pairs, f.near_chunk, g.dt, g.mu,
                           g.beta, f.Kw32);
    BIE_HIP_TRY(hipGetLastError());
    return BIE_OK;
}

// Mixed precision: the lag-0 self term K_ii,0 is applied in FP64 by the
// gather, so the FP32 window's lag-0 value of the self pair keeps only its
// static part, -K^S_ii dt.
__global__ void k_set_self(float *__restrict__ Kw32, const int64_t *__restrict__ off, const double *__restrict__ ks,
                           int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) Kw32[off[k]] = (float)(-ks[k]);
}

int launch_set_self(const FdphOp &f, const int64_t *d_self_off, const double *d_self_ks, int n_self, hipStream_t s) {
    if (n_self > 0 && f.Kw32) {
        hipLaunchKernelGGL(k_set_self, dim3((n_self + 255) / 256), dim3(256), 0, s, f.Kw32, d_self_off, d_self_ks,
                           n_self);
        BIE_HIP_TRY(hipGetLastError());
    }
    return BIE_OK;
}

// Plain clang vector types: operands of the non-temporal load builtin, for
// kernel values streamed once per step (far more than the caches hold).
typedef double nt_double2 __attribute__((ext_vector_type(2)));
typedef float nt_float2 __attribute__((ext_vector_type(2)));
typedef float nt_float4 __attribute__((ext_vector_type(4)));
typedef double lds_double2 __attribute__((ext_vector_type(2)));

// ============================================================== dense form
// D rows hold N x nc values (nc components per element, interleaved).
__global__ void k_dense_hist(const double *__restrict__ d, double *__restrict__ hist, int N, int L, StepIdx si,
                             int nc, int c) {
    const int64_t n = si.get();
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < N) hist[(int64_t)(n & (L - 1)) * N + j] = d[(n - si.n0) * N * nc + (int64_t)j * nc + c];
}

// One wave per receiver row and lag chunk: lanes stream the band row of K at
// (m, i) (coalesced) against the same sources of the history row D_{n-m}.
// V = 2: 16-byte loads (band rows on even sources); NT: non-temporal hint on
// K, for tensors far larger than the last-level cache (a cache-resident K is
// left to the cache).
template <int V, bool NT>
__global__ __launch_bounds__(256) void k_dense_step(const double *__restrict__ K, const int64_t *__restrict__ off,
                                                    const int32_t *__restrict__ blo,
                                                    const double *__restrict__ hist, int N, int M, int L,
                                                    int lag_chunk, StepIdx si, double *__restrict__ partial) {
    const int64_t n = si.get();
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int chunk = blockIdx.y;
    if (row >= N) return;
    const int64_t mlast = n < (int64_t)(M - 1) ? n : (int64_t)(M - 1);
    const int64_t m0 = (int64_t)chunk * lag_chunk;
    const int64_t m1 = m0 + lag_chunk - 1 < mlast ? m0 + lag_chunk - 1 : mlast;
    double acc0 = 0.0, acc1 = 0.0;
    for (int64_t m = m0; m <= m1; ++m) {
        const int64_t r = m * N + row;
        const int64_t o = off[r];
        const int w = (int)(off[r + 1] - o);
        const double *kr = K + o;
        const double *dv = hist + (int64_t)((n - m) & (L - 1)) * N + blo[r];
        if constexpr (V == 2) {
#pragma unroll 4
            for (int j = 2 * lane; j < w; j += 128) {
                const nt_double2 k = NT ? __builtin_nontemporal_load(reinterpret_cast<const nt_double2 *>(kr + j))
                                        : *reinterpret_cast<const nt_double2 *>(kr + j);
                const nt_double2 d = *reinterpret_cast<const nt_double2 *>(dv + j);
                acc0 = fma(k.x, d.x, acc0);
                acc1 = fma(k.y, d.y, acc1);
            }
        } else {
#pragma unroll 4
            for (int j = lane; j < w; j += 64) {
                const double k = NT ? __builtin_nontemporal_load(kr + j) : kr[j];
                acc0 = fma(k, dv[j], acc0);
            }
        }
    }
    const double acc = wave_sum(acc0 + acc1);
    if (lane == 0) partial[(int64_t)chunk * N + row] = acc;
}

__global__ void k_dense_reduce(const double *__restrict__ partial, int N, int n_chunks, StepIdx si,
                               double *__restrict__ t, int nc, int comp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double acc = 0.0;
    for (int c = 0; c < n_chunks; ++c) acc += partial[(int64_t)c * N + i];
    t[(si.get() - si.n0) * N * nc + (int64_t)i * nc + comp] = acc;
}

// Debug scan of one step's tractions: the smallest (step * row + index) of
// a non-finite value goes to *word (all ones while every value is finite).
__global__ void k_scan_finite(const double *__restrict__ t, int64_t row, StepIdx si, unsigned long long *word) {
    const int64_t n = si.get();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= row) return;
    const double v = t[(n - si.n0) * row + i];
    if (!isfinite(v)) atomicMin(word, (unsigned long long)(n * row + i));
}

int launch_scan_finite(const double *t, int64_t row, const StepIdx &si, int64_t *word, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_finite, dim3((unsigned)((row + 255) / 256)), dim3(256), 0, s, t, row, si,
                       reinterpret_cast<unsigned long long *>(word));
    BIE_HIP_TRY(hipGetLastError());
    return BIE_OK;
}

// Last node of a captured step: advances the device step counter.
__global__ void k_step_advance(int64_t *n_dev, int64_t by) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *n_dev += by;
}

int launch_step_advance(int64_t *n_dev, hipStream_t s, int64_t by) {
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, n_dev, by);
    BIE_HIP_TRY(hipGetLastError());
    return BIE_OK;
}

__global__ void k_step_set(int64_t *n_dev, int64_t value) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *n_dev = value;
}

int launch_step_set(int64_t *n_dev, int64_t value, hipStream_t s) {
    hipLaunchKernelGGL(k_step_set, dim3(1), dim3(64), 0, s, n_dev, value);
    BIE_HIP_TRY(hipGetLastError());
    return BIE_OK;
}

int dense_step(bie_op_impl *op, const double *d, double *t, hipStream_t s, const StepIdx &si, bool advance) {
    DenseOp &D = op->dense;
    const size_t kc = (size_t)D.E, hc = (size_t)D.L * D.N, pc = (size_t)D.n_chunks * D.N;
    for (int c = 0; c < D.ncomp; ++c)
        hipLaunchKernelGGL(k_dense_hist, dim3((D.N + 255) / 256), dim3(256), 0, s, d, D.hist + c * hc, D.N, D.L, si,
                           D.ncomp, c);
    const int tk = si.dev ? -1 : op->timer.begin(s);
    const bool even = D.V == 2;
    const bool stream = (double)kc * sizeof(double) > 1024.0 * 1024 * 1024;  // K of a component beyond 1 GiB
    const dim3 g((D.N + 3) / 4, D.n_chunks), b(256);
    for (int c = 0; c < D.ncomp; ++c) {
        const double *Kc = D.K + c * kc, *hc_ = D.hist + c * hc;
        double *pc_ = D.partial + c * pc;
#define BIE_DENSE_LAUNCH(VV, NTT)                                                                              \
    hipLaunchKernelGGL((k_dense_step<VV, NTT>), g, b, 0, s, Kc, D.off, D.blo, hc_, D.N, D.M, D.L, D.lag_chunk, si, \
                       pc_)
        if (even && stream)
            BIE_DENSE_LAUNCH(2, true);
        else if (even)
            BIE_DENSE_LAUNCH(2, false);
        else if (stream)
            BIE_DENSE_LAUNCH(1, true);
        else
            BIE_DENSE_LAUNCH(1, false);
#undef BIE_DENSE_LAUNCH
    }
    op->timer.end(tk, s);
    for (int c = 0; c < D.ncomp; ++c)
        hipLaunchKernelGGL(k_dense_reduce, dim3((D.N + 255) / 256), dim3(256), 0, s, D.partial + c * pc, D.N,
                           D.n_chunks, si, t, D.ncomp, c);
    BIE_HIP_TRY(hipGetLastError());
    if (op->scan_finite)
        if (int rc = launch_scan_finite(t, op->N, si, op->nonfinite, s)) return rc;
    if (si.dev)
        return launch_step_advance(const_cast<int64_t *>(si.dev), s);
    if (advance) op->step++;
    return BIE_OK;
}

// Commit of a predicted step (the prediction ran with D_n = 0): D_n into the
// history slot of step n, then the next step.
int dense_commit(bie_op_impl *op, const double *d, hipStream_t s) {
    DenseOp &D = op->dense;
    StepIdx si;
    si.n = si.n0 = op->step;
    hipLaunchKernelGGL(k_dense_hist, dim3((D.N + 255) / 256), dim3(256), 0, s, d, D.hist, D.N, D.L, si, 1, 0);
    BIE_HIP_TRY(hipGetLastError());
    op->step++;
    return BIE_OK;
}

// K_ii,0 from the lag-0 band rows (the receiver's own element is always in
// its band).
__global__ void k_first_lag_dense(const double *__restrict__ K, const int64_t *__restrict__ off,
                                  const int32_t *__restrict__ blo, int N, double *__restrict__ k0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) k0[i] = K[off[i] + (i - blo[i])];
}

int launch_first_lag(const bie_op_impl *op, double *k0, hipStream_t s) {
    if (op->kind == BIE_KIND_DENSE) {
        const DenseOp &D = op->dense;
        hipLaunchKernelGGL(k_first_lag_dense, dim3((D.N + 255) / 256), dim3(256), 0, s, D.K, D.off, D.blo, D.N, k0);
        BIE_HIP_TRY(hipGetLastError());
    } else {
        BIE_HIP_TRY(hipMemcpyAsync(k0, op->fdph.first_lag, (size_t)op->N * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    return BIE_OK;
}

// Friction solve of a coupled step, one thread per element: t holds the
// prediction P_n on entry and the shear traction t0 + T_n on exit.  A ruptured
// element (or one whose traction reaches t_th) solves
// g(D) = t* + k0 D - strength(slip + dt D) = 0 for D >= 0, g decreasing past
// its single rise; g(0) <= 0 means it sticks.  The exponential law's root is
// bracketed in (0, (t* - t_dy) / |k0|], where the strength cannot be below
// t_dy, and found by Newton steps kept inside the shrinking bracket (a
// bisection wherever a step would leave it or g' >= 0), until a step is
// within the rounding of g divided by |g'| or the bracket has closed (at most
// 13 iterations over a wide sweep of laws and loads).
__device__ inline double fr_strength(int law, double t_th, double t_dy, double d_c, double slip) {
    return law == BIE_LAW_EXP_WEAKENING ? (t_th - t_dy) * exp(-slip / d_c) + t_dy : t_dy;
}

__global__ void k_friction(int N, int law, double t_th, double t_dy, double d_c, double dt,
                           const double *__restrict__ t0, const double *__restrict__ k0,
                           double *__restrict__ slip, int32_t *__restrict__ state, double *__restrict__ t,
                           double *__restrict__ d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double ts = t0[i] + t[i];
    const double kk = k0[i];
    const double u = slip[i];
    int st = state[i];
    double D = 0.0;
    if (st || ts >= t_th) {
        st = 1;
        if (ts - fr_strength(law, t_th, t_dy, d_c, u) > 0.0) {
            double hi = (ts - t_dy) / (-kk);
            D = hi;
            if (law == BIE_LAW_EXP_WEAKENING) {
                // g(D) = ts + kk D - a exp(-b D) - t_dy, a = (t_th - t_dy) exp(-u / d_c), b = dt / d_c
                const double a = (t_th - t_dy) * exp(-u / d_c), b = dt / d_c;
                double e = exp(-b * hi);
                if (ts + kk * hi - a * e - t_dy < 0.0) {
                    double lo = 0.0, x = hi;
                    for (int it = 0; it < 200; ++it) {
                        const double gx = ts + kk * x - a * e - t_dy;
                        if (gx == 0.0) break;
                        if (gx > 0.0) lo = x; else hi = x;
                        const double gp = kk + a * b * e;  // g'(x)
                        constexpr double EPS = 2.220446049250313e-16;
                        double xn = 0.5 * (lo + hi);
                        bool done = false;
                        if (gp < 0.0) {
                            // stop once the step is within the rounding of g over |g'|
                            const double xs = x - gx / gp;
                            if (xs >= lo && xs <= hi) xn = xs;
                            done = fabs(xn - x) <= 8.0 * EPS * (fabs(xn) + (fabs(ts) + fabs(t_dy) + a) / -gp);
                        }
                        done = done || !(hi - lo > 8.0 * EPS * hi);
                        x = xn;
                        e = exp(-b * x);
                        if (done) break;
                    }
                    hi = x;
                }
                D = hi;
            }
        }
    }
    state[i] = st;
    d[i] = D;
    t[i] = ts + kk * D;
    slip[i] = u + dt * D;
}

int launch_friction(int N, const bie_friction &fr, double dt, const double *t0, const double *k0, double *slip,
                    int32_t *state, double *t, double *d, hipStream_t s) {
    hipLaunchKernelGGL(k_friction, dim3((N + 255) / 256), dim3(256), 0, s, N, fr.law, fr.t_th, fr.t_dy, fr.d_c, dt,
                       t0, k0, slip, state, t, d);
    BIE_HIP_TRY(hipGetLastError());
    return BIE_OK;
}

__global__ void k_dense_zero_hist(double *__restrict__ hist, int N, int L, int64_t n0, int64_t count) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count * N) return;
    const int64_t t = n0 + idx / N;
    hist[(t & (L - 1)) * N + idx % N] = 0.0;
}

int dense_advance(bie_op_impl *op, int64_t steps, hipStream_t s) {
    DenseOp &D = op->dense;
    const int64_t count = steps < D.L ? steps : D.L;  // older slots are overwritten anyway
    if (count > 0) {
        const int64_t n0 = op->step + steps - count;
        const int64_t tot = count * D.N;
        for (int c = 0; c < D.ncomp; ++c)
            hipLaunchKernelGGL(k_dense_zero_hist, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                               D.hist + (size_t)c * D.L * D.N, D.N, D.L, n0, count);
        BIE_HIP_TRY(hipGetLastError());
    }
    op->step += steps;
    return BIE_OK;
}

int dense_reset(bie_op_impl *op, hipStream_t s) {
    DenseOp &D = op->dense;
    BIE_HIP_TRY(hipMemsetAsync(D.hist, 0, (size_t)D.ncomp * D.L * D.N * sizeof(double), s));
    op->step = 0;
    return BIE_OK;
}

// ============================================================== FDP=H form
// One thread per (element, scenario blockIdx.y).  what: 1 the near history,
// 2 the running sum and the recent history of the far field, 3 both (a time
// block writes the near histories of all its steps first).
__global__ void k_fdph_update(const double *__restrict__ d, double *__restrict__ Dring, double *__restrict__ Uring,
                              double *__restrict__ Drec, int N, int L, int Lf, StepIdx si, Scn sc, int what,
                              int steps) {
    const int64_t n0 = si.get();
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int c = blockIdx.y;
    Dring += c * sc.D;
    Uring += c * sc.U;
    Drec += c * sc.Drec;
    // steps n0 .. n0 + steps - 1 in order (a time block's histories)
    for (int b = 0; b < steps; ++b) {
        const int64_t n = n0 + b;
        const double v = d[(n - si.n0) * sc.row + (int64_t)c * N + j];
        if (what & 1) Dring[(int64_t)j * L + ((-n) & (L - 1))] = v;
        if (what & 2) {
            // a ring of slots: writing U_n from U_{n-1} keeps a repeated update
            // of step n (the commit after a prediction) idempotent
            Uring[(n & (U_SLOTS - 1)) * N + j] = Uring[((n - 1) & (U_SLOTS - 1)) * N + j] + v;
            Drec[(int64_t)(n & (Lf - 1)) * N + j] = v;
        }
    }
}

// Near field: work item = (tile, lag chunk).  The chunk's 32 source histories
// (time-reversed rings make lag m contiguous) and the tile's pair windows and
// offsets are staged in LDS (38 KB for 128 lags in FP64, so four 8-wave
// workgroups fit a CU).  Each wave owns receivers of the tile; its lanes
// cover consecutive lags (PER per lane: 8- or 16-byte loads, 4 bytes for FP32
// in 64-lag chunks) and the loop over the tile's sources issues one coalesced
// window load per source (per two sources, each on half the wave, where a
// wave-wide load would span more than the chunk), so a wave keeps many
// independent HBM loads in flight.
template <class KT, int CHUNK, int UNR, int PER>
__global__ __launch_bounds__(NEAR_THREADS) void k_near(const NearTile *__restrict__ tiles,
                                                       const int32_t *__restrict__ items,
                                                       const int32_t *__restrict__ pW,
                                                       const int64_t *__restrict__ item_base,
                                                       const int32_t *__restrict__ item_rel,
                                                       const uint16_t *__restrict__ item_rng,
                                                       const KT *__restrict__ Kw, const double *__restrict__ Dring,
                                                       int L, StepIdx si,
                                                       const int32_t *__restrict__ perm,
                                                       const int32_t *__restrict__ pslot,
                                                       double *__restrict__ partial) {
    const int64_t n = si.get();
    constexpr int SP = (64 * PER > CHUNK) ? 64 * PER / CHUNK : 1;  // sources per wave-wide load
    constexpr int SPAN = 64 / SP * PER;                             // lags per source per load
    static_assert(PER * sizeof(KT) <= 16, "at most 16-byte loads");
    static_assert(SP <= 2 && CHUNK % SPAN == 0, "a chunk is a whole number of loads");
    __shared__ double Dt[TILE][CHUNK];
    __shared__ int32_t Ol[TILE * TILE];
    __shared__ uint16_t Wl[TILE * TILE];
    __shared__ uint16_t Rg[TILE];
    __shared__ int32_t Ps[TILE];
    // optional launch order: workgroup -> item (-1: padding slot)
    const int item = perm ? perm[blockIdx.x] : (int)blockIdx.x;
    if (item < 0) return;
    const int t = items[2 * item];
    const int ch = items[2 * item + 1];
    const NearTile &T = tiles[t];
    const int nr = T.nr, ns = T.ns;
    const int64_t m0 = (int64_t)ch * CHUNK;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    constexpr int NW = NEAR_THREADS / 64;
    if (n >= T.hz) return;  // the tile's problem has finished its run; its receivers read nothing
    if (m0 > n) {  // no history reaches this chunk yet
        for (int r = threadIdx.x; r < nr; r += blockDim.x) partial[pslot[(int64_t)item * TILE + r]] = 0.0;
        return;
    }
    const int np = nr * ns;
    for (int q = threadIdx.x; q < np; q += blockDim.x) {
        Wl[q] = (uint16_t)pW[T.pair_begin + q];
        Ol[q] = item_rel[(int64_t)item * (TILE * TILE) + q];
    }
    if (threadIdx.x < TILE) {
        Rg[threadIdx.x] = item_rng[(int64_t)item * TILE + threadIdx.x];
        Ps[threadIdx.x] = pslot[(int64_t)item * TILE + threadIdx.x];
    }
    for (int idx = threadIdx.x; idx < ns * CHUNK; idx += blockDim.x) {
        const int sl = idx / CHUNK, mm = idx % CHUNK;
        Dt[sl][mm] = Dring[(int64_t)T.src[sl] * L + ((m0 + mm - n) & (L - 1))];
    }
    __syncthreads();
    const int hist_len = (int)((n - m0 + 1) < CHUNK ? (n - m0 + 1) : CHUNK);  // lags with history
    const KT *__restrict__ Kt = Kw + item_base[item];
    const int subs = (hist_len + SPAN - 1) / SPAN;
    for (int r = wave; r < nr; r += NW) {
        double acc = 0.0;
        const int pb = r * ns;
        // sources whose windows reach this chunk (the tail chunks of a tile
        // hold only the pairs with the longest windows), widened to whole
        // unrolled blocks so that every block issues UNR loads back to back
        const int r_lo = Rg[r] & 0xFF, r_hi = Rg[r] >> 8;
        const int s_lo = r_lo & ~(UNR - 1);
        const int s_hi = r_hi > r_lo ? min(ns, s_lo + ((r_hi - s_lo + UNR - 1) & ~(UNR - 1))) : s_lo;
        const int half = lane / (64 / SP);  // which of the load's sources this lane serves
        for (int sub = 0; sub < subs; ++sub) {
            const int mm = sub * SPAN + lane % (64 / SP) * PER;  // first lag of this lane in the chunk
            // branch-free: lanes past a segment read its last aligned element(s)
            // (one cache line for the whole wave) and contribute zero, so the
            // unrolled loads are independent and issued back to back
#pragma unroll (UNR / SP)
            for (int s2 = s_lo; s2 < s_hi; s2 += SP) {
                // two sources per load: the range may end on its first (odd
                // count at the end of a tile); the second then reads the first's
                // metadata and contributes zero
                const bool live = SP == 1 || s2 + half < s_hi;
                const int sl = live ? s2 + half : s2;
                const int q = pb + sl;
                const int len = live ? (int)Wl[q] - (int)m0 : 0;  // lags of this pair in the chunk (may be <= 0 or > CHUNK)
                const int lim = len < hist_len ? len : hist_len;
                const int last = len > 0 ? (((len < CHUNK ? len : CHUNK) - 1) & ~(PER - 1)) : 0;
                const int mc = mm < last ? mm : last;
                // the mask goes on the history operand so that every load's
                // result is consumed (window values are finite), which keeps the
                // compiler from sinking the loads into branches
                if constexpr (PER == 1) {
                    const double kv = (double)__builtin_nontemporal_load(Kt + Ol[q] + mc);
                    const double dv = (mm < lim) ? Dt[sl][mm] : 0.0;
                    acc = fma(kv, dv, acc);
                } else if constexpr (PER == 2) {
                    using V2 = typename std::conditional<sizeof(KT) == 8, nt_double2, nt_float2>::type;
                    const V2 kv = __builtin_nontemporal_load(reinterpret_cast<const V2 *>(Kt + Ol[q] + mc));
                    const double da = (mm < lim) ? Dt[sl][mm] : 0.0;
                    const double db = (mm + 1 < lim) ? Dt[sl][mm + 1] : 0.0;
                    acc = fma((double)kv.x, da, acc);
                    acc = fma((double)kv.y, db, acc);
                } else {
                    const nt_float4 kv = __builtin_nontemporal_load(reinterpret_cast<const nt_float4 *>(Kt + Ol[q] + mc));
                    const double d0 = (mm < lim) ? Dt[sl][mm] : 0.0;
                    const double d1 = (mm + 1 < lim) ? Dt[sl][mm + 1] : 0.0;
                    const double d2 = (mm + 2 < lim) ? Dt[sl][mm + 2] : 0.0;
                    const double d3 = (mm + 3 < lim) ? Dt[sl][mm + 3] : 0.0;
                    acc = fma((double)kv.x, d0, acc);
                    acc = fma((double)kv.y, d1, acc);
                    acc = fma((double)kv.z, d2, acc);
                    acc = fma((double)kv.w, d3, acc);
                }
            }
        }
        acc = wave_sum(acc);
        if (lane == 0) partial[Ps[r]] = acc;
    }
}

// Time block: the near field of the B consecutive steps n .. n+B-1 of a
// prescribed-slip run in one pass over the windows.  The staged history
// covers the chunk's lags for all B steps (CHUNK + B - 1 times per source);
// each window value loaded once feeds B multiply-adds, one per step, in the
// order a single step's kernel uses (same sums, bit for bit, for finite slip
// rates).  Lags before a step's first history read ring slots of times before
// step 0, which hold zeros (the ring has B - 1 spare slots); the mask by
// window length goes on the window value, so a non-finite slip rate reaches
// every receiver of its tile from its own step on (the single-step kernel
// masks the history instead and keeps it to the windows that cover it).
template <class KT, int CHUNK, int UNR, int PER, int B>
__global__ __launch_bounds__(NEAR_THREADS) void k_near_tb(const NearTile *__restrict__ tiles,
                                                          const int32_t *__restrict__ items,
                                                          const int32_t *__restrict__ pW,
                                                          const int64_t *__restrict__ item_base,
                                                          const int32_t *__restrict__ item_rel,
                                                          const uint16_t *__restrict__ item_rng,
                                                          const KT *__restrict__ Kw, const double *__restrict__ Dring,
                                                          int L, StepIdx si,
                                                          const int32_t *__restrict__ perm,
                                                          const int32_t *__restrict__ pslot,
                                                          double *__restrict__ partial, int64_t part) {
    const int64_t n = si.get();  // first step of the block
    constexpr int SP = (64 * PER > CHUNK) ? 64 * PER / CHUNK : 1;
    constexpr int SPAN = 64 / SP * PER;
    constexpr int H = CHUNK + B - 1;  // staged times per source
    constexpr int HP = CHUNK + B;     // row length: 16-byte aligned rows for paired reads
    static_assert(PER * sizeof(KT) <= 16, "at most 16-byte loads");
    static_assert(SP <= 2 && CHUNK % SPAN == 0, "a chunk is a whole number of loads");
    static_assert(B % 2 == 0, "even blocks keep the rows 16-byte aligned");
    __shared__ __align__(16) double Dt[TILE][HP];
    __shared__ int32_t Ol[TILE * TILE];
    __shared__ uint16_t Wl[TILE * TILE];
    __shared__ uint16_t Rg[TILE];
    __shared__ int32_t Ps[TILE];
    const int item = perm ? perm[blockIdx.x] : (int)blockIdx.x;
    if (item < 0) return;
    const int t = items[2 * item];
    const int ch = items[2 * item + 1];
    const NearTile &T = tiles[t];
    const int nr = T.nr, ns = T.ns;
    const int64_t m0 = (int64_t)ch * CHUNK;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    constexpr int NW = NEAR_THREADS / 64;
    if (n >= T.hz) return;  // every step of the block is past the tile's run
    if (m0 > n + B - 1) {   // no step of the block reaches this chunk
        for (int r = threadIdx.x; r < nr; r += blockDim.x)
            for (int c = 0; c < B; ++c) partial[c * part + pslot[(int64_t)item * TILE + r]] = 0.0;
        return;
    }
    const int np = nr * ns;
    for (int q = threadIdx.x; q < np; q += blockDim.x) {
        Wl[q] = (uint16_t)pW[T.pair_begin + q];
        Ol[q] = item_rel[(int64_t)item * (TILE * TILE) + q];
    }
    if (threadIdx.x < TILE) {
        Rg[threadIdx.x] = item_rng[(int64_t)item * TILE + threadIdx.x];
        Ps[threadIdx.x] = pslot[(int64_t)item * TILE + threadIdx.x];
    }
    // Dt[s][u] = D of time n + B - 1 - m0 - u: step n + c reads lag mm at
    // u = mm + B - 1 - c.  Times older than the ring holds (m0 + u >= L: lags
    // past every window) are staged as zeros, not as the newer times whose
    // slots they would alias (a masked window value times a non-finite
    // slip rate would otherwise reach an earlier step).
    for (int idx = threadIdx.x; idx < ns * HP; idx += blockDim.x) {
        const int sl = idx / HP, u = idx % HP;
        Dt[sl][u] = (u < H && m0 + u < L) ? Dring[(int64_t)T.src[sl] * L + ((m0 + u - (B - 1) - n) & (L - 1))] : 0.0;
    }
    __syncthreads();
    // lags with history for the block's last step
    const int hist_len = (int)((n + B - m0) < CHUNK ? (n + B - m0) : CHUNK);
    const KT *__restrict__ Kt = Kw + item_base[item];
    const int subs = (hist_len + SPAN - 1) / SPAN;
    for (int r = wave; r < nr; r += NW) {
        double acc[B];
#pragma unroll
        for (int c = 0; c < B; ++c) acc[c] = 0.0;
        const int pb = r * ns;
        const int r_lo = Rg[r] & 0xFF, r_hi = Rg[r] >> 8;
        const int s_lo = r_lo & ~(UNR - 1);
        const int s_hi = r_hi > r_lo ? min(ns, s_lo + ((r_hi - s_lo + UNR - 1) & ~(UNR - 1))) : s_lo;
        const int half = lane / (64 / SP);
        for (int sub = 0; sub < subs; ++sub) {
            const int mm = sub * SPAN + lane % (64 / SP) * PER;
#pragma unroll (UNR / SP)
            for (int s2 = s_lo; s2 < s_hi; s2 += SP) {
                const bool live = SP == 1 || s2 + half < s_hi;
                const int sl = live ? s2 + half : s2;
                const int q = pb + sl;
                const int len = live ? (int)Wl[q] - (int)m0 : 0;
                const int last = len > 0 ? (((len < CHUNK ? len : CHUNK) - 1) & ~(PER - 1)) : 0;
                const int mc = mm < last ? mm : last;
                // window values, masked by the pair's window (in their own
                // precision, before widening)
                KT kk[PER];
                if constexpr (PER == 1) {
                    kk[0] = __builtin_nontemporal_load(Kt + Ol[q] + mc);
                } else if constexpr (PER == 2) {
                    using V2 = typename std::conditional<sizeof(KT) == 8, nt_double2, nt_float2>::type;
                    const V2 kv = __builtin_nontemporal_load(reinterpret_cast<const V2 *>(Kt + Ol[q] + mc));
                    kk[0] = kv.x;
                    kk[1] = kv.y;
                } else {
                    const nt_float4 kv =
                        __builtin_nontemporal_load(reinterpret_cast<const nt_float4 *>(Kt + Ol[q] + mc));
                    kk[0] = kv.x;
                    kk[1] = kv.y;
                    kk[2] = kv.z;
                    kk[3] = kv.w;
                }
                double k[PER];
#pragma unroll
                for (int p = 0; p < PER; ++p) k[p] = (double)((mm + p < len) ? kk[p] : (KT)0);
                // the lane's PER + B - 1 history values, in 16-byte reads where
                // its first lag is even
                constexpr int NH = PER + B - 1;
                double h[NH + 1];
                if constexpr (PER >= 2) {
#pragma unroll
                    for (int i = 0; i < (NH + 1) / 2; ++i) {
                        const lds_double2 v = *reinterpret_cast<const lds_double2 *>(&Dt[sl][mm + 2 * i]);
                        h[2 * i] = v.x;
                        h[2 * i + 1] = v.y;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < NH; ++j) h[j] = Dt[sl][mm + j];
                }
#pragma unroll
                for (int c = 0; c < B; ++c)
#pragma unroll
                    for (int p = 0; p < PER; ++p) acc[c] = fma(k[p], h[p + B - 1 - c], acc[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < B; ++c) {
            const double a = wave_sum(acc[c]);
            if (lane == 0) partial[c * part + Ps[r]] = a;
        }
    }
}

// Time block on the matrix cores.  With the B = 16 steps of a block as the
// columns, the near field of a tile is a matrix product: receiver r, step c
// collects the sum over sources s and lags m of W_rs[m] D_s(n + c - m), so
// the rows are the tile's receivers (two groups of 16), the columns the steps
// and the reduction runs over (source, lag) with a Hankel right operand built
// from the staged history.  One 16x16x4 MFMA takes 4 lags of 16 receivers'
// windows (the left operand, straight from HBM into registers) and the 4 x 16
// history values of those lags (from LDS); the windows keep their own
// precision (FP64 MFMA for FP64 windows; FP32 windows times the history
// rounded to FP32 with FP32 accumulation in the mixed modes).  A unit of work
// is 128 bytes of every window row of one source (16 FP64 or 32 FP32 lags):
// eight lanes load a whole 128-byte row of a unit (8 rows per instruction,
// two instructions per row group), a lane permutation (a DPP row shift and a
// ds_bpermute) puts the pieces in the MFMA layout, and one read of the Hankel
// operand serves both receiver groups.  The workgroup's waves take units in
// turn; their 32 x 16 results are summed in LDS in wave order (deterministic)
// and written as the work item's partial sums of the B steps.  A work item is
// one lag chunk of a tile, or (GR) up to NEAR_GROUP consecutive chunks of one
// tile taken in turn into the same accumulators, with one partial sum per
// receiver and step for the group.  Rows past the tile or past a window's
// padded segment read a zero block past the windows.
typedef double mfma_d4 __attribute__((ext_vector_type(4)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

template <class KT>
struct NearMfma;
// Both MFMAs take the left operand as lane l = A[l % 16][l / 16] and the right
// one as lane l = B[l / 16][l % 16]; their results differ in layout: element
// v of lane l is row (l / 16) + 4 v in the FP64 one, row 4 (l / 16) + v in
// the FP32 one, column l % 16 in both (checked on the device).
template <>
struct NearMfma<double> {
    using Acc = mfma_d4;
    using V = nt_double2;  // one 16-byte load
    static __device__ __forceinline__ Acc mma(double a, double b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int kq, int v) { return kq + 4 * v; }
};
template <>
struct NearMfma<float> {
    using Acc = mfma_f4;
    using V = nt_float4;
    static __device__ __forceinline__ Acc mma(float a, float b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int kq, int v) { return 4 * kq + v; }
};

template <class KT, int CHUNK, bool GR>
__global__ __launch_bounds__(NEAR_THREADS) __attribute__((amdgpu_waves_per_eu(
    sizeof(KT) == 8 ? (CHUNK > 128 ? 4 : 6) : (GR ? 6 : 8)))) void k_near_mfma(const NearTile *__restrict__ tiles,
                                                            const int32_t *__restrict__ items,
                                                            const int32_t *__restrict__ pW,
                                                            const int64_t *__restrict__ item_base,
                                                            const int32_t *__restrict__ item_rel,
                                                            const KT *__restrict__ Kw, int64_t zero_off,
                                                            const double *__restrict__ Dring, int L, StepIdx si,
                                                            const int32_t *__restrict__ perm,
                                                            const int32_t *__restrict__ grp,
                                                            const int32_t *__restrict__ pslot,
                                                            double *__restrict__ partial, int64_t part) {
    using MF = NearMfma<KT>;
    using Acc = typename MF::Acc;
    using V = typename MF::V;
    constexpr int B = TIME_BLOCK;
    constexpr int PL = 16 / (int)sizeof(KT);   // lags per 16-byte load
    constexpr int UL = 8 * PL;                 // lags per unit: 128 bytes of a window row
    constexpr int NU = CHUNK / UL;             // units per source and chunk
    constexpr int H = CHUNK + B - 1;           // staged times per source
    constexpr int HP = CHUNK + B;
    constexpr int NW = NEAR_THREADS / 64;
    static_assert(B == 16, "the steps of a block are the 16 columns of the MFMA");
    static_assert(TILE == 32 && TILE * B == NEAR_THREADS, "two receiver groups; one thread per (receiver, step)");
    static_assert(CHUNK % UL == 0 && NU < 32 && TILE * NU <= 65536, "whole units per chunk");
    constexpr size_t DT_BYTES = sizeof(KT) * TILE * HP;
    constexpr size_t RED_BYTES = sizeof(KT) * NW * TILE * B;
    __shared__ __align__(16) unsigned char smem[DT_BYTES > RED_BYTES ? DT_BYTES : RED_BYTES];
    __shared__ uint32_t Pm[TILE * TILE];  // per pair: segment offset << 5 | units its window reaches
    __shared__ int32_t Ps[TILE];
    __shared__ uint16_t Un[TILE * NU];    // units: source | unit << 8
    __shared__ uint16_t Gm[TILE];         // per source: units of rows 0-15 | those of rows 16-31 << 8
    __shared__ int n_units;
    KT(*Dt)[HP] = reinterpret_cast<KT(*)[HP]>(smem);
    KT(*red)[TILE][B] = reinterpret_cast<KT(*)[TILE][B]>(smem);
    // work item: one (tile, lag chunk) item, or with grp a group of
    // consecutive lag chunks of one tile summed into one partial per receiver
    const int wi = perm ? perm[blockIdx.x] : (int)blockIdx.x;
    if (wi < 0) return;
    const int item0 = GR ? grp[2 * wi] : wi;
    const int n_it = GR ? grp[2 * wi + 1] : 1;
    const int t = items[2 * item0];
    const NearTile &T = tiles[t];
    const int nr = T.nr, ns = T.ns;
    const int64_t n = si.get();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if (n >= T.hz) return;  // every step of the block is past the tile's run
    if (threadIdx.x < TILE) Ps[threadIdx.x] = pslot[(int64_t)wi * TILE + threadIdx.x];
    const int rho = lane & 15, kq = lane >> 4;  // MFMA layout: row rho, lag group kq
    Acc c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
    for (int gi = 0; gi < n_it; ++gi) {
        const int item = item0 + gi;
        const int ch = items[2 * item + 1];
        const int64_t m0 = (int64_t)ch * CHUNK;
        if (m0 > n + B - 1) break;  // no step of the block reaches this chunk (nor the group's later ones)
        // units of lags with history for the block's last step
        const int hist_len = (int)((n + B - m0) < CHUNK ? (n + B - m0) : CHUNK);
        const int hb = (hist_len + UL - 1) / UL;
        const int np = nr * ns;
        for (int q = threadIdx.x; q < np; q += blockDim.x) {
            const int len = min(max(pW[T.pair_begin + q] - (int)m0, 0), CHUNK);
            const int nb = min((len + UL - 1) / UL, hb);
            Pm[q] = ((uint32_t)item_rel[(int64_t)item * (TILE * TILE) + q] << 5) | (uint32_t)nb;
        }
        // Dt[s][u] = D of time n + B - 1 - m0 - u (zero past the ring's reach, as
        // in the kernel above); step n + c reads lag mm of the chunk at u = mm + B - 1 - c
        for (int idx = threadIdx.x; idx < ns * HP; idx += blockDim.x) {
            const int sl = idx / HP, u = idx % HP;
            Dt[sl][u] = (KT)((u < H && m0 + u < L) ? Dring[(int64_t)T.src[sl] * L + ((m0 + u - (B - 1) - n) & (L - 1))]
                                                   : 0.0);
        }
        __syncthreads();
        // the units: for each source, the 128-byte blocks of the chunk that some
        // receiver's window reaches and some step of the block has history for
        if (wave == 0) {
            int cnt = 0, n0u = 0, n1u = 0;
            if (lane < ns) {
                for (int r = 0; r < nr; ++r) {
                    const int u = (int)(Pm[r * ns + lane] & 31);
                    if (r < 16) n0u = max(n0u, u);
                    else n1u = max(n1u, u);
                }
                cnt = max(n0u, n1u);
                Gm[lane] = (uint16_t)(n0u | (n1u << 8));
            }
            int inc = cnt;
    #pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int v = __shfl_up(inc, d);
                if (lane >= d) inc += v;
            }
            for (int b = 0; b < cnt; ++b) Un[inc - cnt + b] = (uint16_t)(lane | (b << 8));
            if (lane == 63) n_units = inc;
        }
        __syncthreads();
        const KT *__restrict__ Kt = Kw + item_base[item];
        const int64_t zoff = zero_off - item_base[item];  // the zero block, relative to Kt
        // The loads: eight lanes read a whole 128-byte unit row (lane l: row
        // 8 t + l / 8 of load t, 16-byte piece l % 8), so that every request is a
        // full cache line; a permutation then hands piece 4 h + kq of row rho to
        // lane (rho, kq) of the MFMA layout of half h (from load rho / 8).
        const int lr = lane >> 3, lp = lane & 7;
        // the permutation in two moves: a row shift by 4 lanes (DPP) gathers half
        // h of both loads in one register (lane (r, x, kq): load x, lane (r, h, kq)),
        // then one ds_bpermute per dword moves it to the MFMA layout
        const bool hi4 = (lane & 4) != 0;
        const int src = ((rho & 7) * 8 + (rho >> 3) * 4 + kq) * 4;  // byte address
        const int nu = n_units;
        // element offset (from Kt) of this lane's load of row r for unit (s, b)
        auto row_off = [&](int r, int s, int b) -> int64_t {
            const bool rv = r < nr;
            const uint32_t v = Pm[rv ? r * ns + s : 0];
            const bool ok = rv && b < (int)(v & 31);
            return (ok ? (int64_t)(v >> 5) + b * UL : zoff) + lp * PL;
        };
        // both halves of the MFMA operands of a row group from its two loads
        auto to_mfma = [&](V v0, V v1, V &y0, V &y1) {
            typedef int i4 __attribute__((ext_vector_type(4)));
            const i4 w0 = __builtin_bit_cast(i4, v0), w1 = __builtin_bit_cast(i4, v1);
            i4 u0, u1;
    #pragma unroll
            for (int d = 0; d < 4; ++d) {
                // row_shr:4 brings lane i - 4, row_shl:4 lane i + 4 (within 16-lane rows)
                const int s1 = __builtin_amdgcn_update_dpp(0, w1[d], 0x114, 0xF, 0xF, false);
                const int s0 = __builtin_amdgcn_update_dpp(0, w0[d], 0x104, 0xF, 0xF, false);
                u0[d] = hi4 ? s1 : w0[d];
                u1[d] = hi4 ? w1[d] : s0;
            }
            i4 a, b;
    #pragma unroll
            for (int d = 0; d < 4; ++d) {
                a[d] = __builtin_amdgcn_ds_bpermute(src, u0[d]);
                b[d] = __builtin_amdgcn_ds_bpermute(src, u1[d]);
            }
            y0 = __builtin_bit_cast(V, a);
            y1 = __builtin_bit_cast(V, b);
        };
        // each wave: a contiguous run of the unit list (consecutive 128-byte
        // pieces of the same rows, source by source); the next unit's windows are
        // loaded before the current unit's products
        auto run = [&](auto two_c) {
            constexpr bool TWO = decltype(two_c)::value;
            V a0[2], a1[2];
            int s = 0, b = 0;
            auto load = [&](int u, V(&x0)[2], V(&x1)[2], int &su, int &bu) {
                su = Un[u] & 0xFF;
                bu = Un[u] >> 8;
    #pragma unroll
                for (int t = 0; t < 2; ++t)
                    x0[t] = __builtin_nontemporal_load(reinterpret_cast<const V *>(Kt + row_off(8 * t + lr, su, bu)));
                if constexpr (TWO)
    #pragma unroll
                    for (int t = 0; t < 2; ++t)
                        x1[t] = __builtin_nontemporal_load(
                            reinterpret_cast<const V *>(Kt + row_off(16 + 8 * t + lr, su, bu)));
            };
            const int per = (nu + NW - 1) / NW;  // units per wave
            const int u0 = wave * per;
            const int cnt = nu - u0 < per ? nu - u0 : per;  // units of this wave
            if (cnt <= 0) return;
            // right operand of the MFMA for (h, p): lane (kq, column rho) holds
            // the history of step n + rho at the lag of the left operand's column kq
            // the products of one row group (a group none of whose windows reaches
            // the unit is skipped: its rows read the zero block)
            auto group = [&](const V(&x)[2], Acc &c, const KT *dh) {
                V y[2];
                to_mfma(x[0], x[1], y[0], y[1]);
    #pragma unroll
                for (int h = 0; h < 2; ++h)
    #pragma unroll
                    for (int p = 0; p < PL; ++p) c = MF::mma(y[h][p], dh[h * (UL / 2) + p], c);
            };
            auto products = [&](const V(&x0)[2], const V(&x1)[2], int su, int bu) {
                const KT *dh = &Dt[su][bu * UL + kq * PL + B - 1 - rho];
                if constexpr (TWO) {
                    const int gm = Gm[su];
                    const bool act0 = bu < (gm & 0xFF), act1 = bu < (gm >> 8);
                    if (act0 && act1) {
                        // both groups, one read of the right operand for the two
                        V y0[2], y1[2];
                        to_mfma(x0[0], x0[1], y0[0], y0[1]);
                        to_mfma(x1[0], x1[1], y1[0], y1[1]);
    #pragma unroll
                        for (int h = 0; h < 2; ++h)
    #pragma unroll
                            for (int p = 0; p < PL; ++p) {
                                const KT bv = dh[h * (UL / 2) + p];
                                c0 = MF::mma(y0[h][p], bv, c0);
                                c1 = MF::mma(y1[h][p], bv, c1);
                            }
                    } else if (act0) {
                        group(x0, c0, dh);
                    } else {
                        group(x1, c1, dh);
                    }
                } else {
                    group(x0, c0, dh);
                }
            };
            // two register sets in turn: the next unit's loads stay in flight
            // during the current unit's products (a fixed trip count, with no
            // branch between a load and its use, keeps the compiler from sinking
            // them; past the wave's last unit the loads repeat that unit)
            auto unit = [&](int k) { return u0 + (k < cnt ? k : cnt - 1); };
            V e0[2], e1[2];
            int se, be;
            load(unit(0), a0, a1, s, b);
            int k = 0;
            for (; k + 2 <= cnt; k += 2) {
                load(unit(k + 1), e0, e1, se, be);
                __builtin_amdgcn_sched_barrier(0);
                products(a0, a1, s, b);
                load(unit(k + 2), a0, a1, s, b);
                __builtin_amdgcn_sched_barrier(0);
                products(e0, e1, se, be);
            }
            if (k < cnt) products(a0, a1, s, b);
        };
        if (nr > 16) run(std::true_type{});
        else run(std::false_type{});
        __syncthreads();  // every wave is done with the staged history and unit list
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        red[wave][MF::row(kq, v)][rho] = c0[v];
        red[wave][16 + MF::row(kq, v)][rho] = c1[v];
    }
    __syncthreads();
    const int r = threadIdx.x / B, c = threadIdx.x % B;
    if (r < nr) {
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) acc += (double)red[w][r][c];
        partial[c * part + Ps[r]] = acc;
    }
}

// Several scenarios (R = 2 or 4) sharing the windows: the kernel below with
// R histories staged and R accumulators per lane.  One scenario runs the
// separate kernel above: with the scenario loop in the same template the
// register allocator settles at 86 VGPRs for the FP32 variants (two
// workgroups per CU instead of three; 10-20% slower).
template <class KT, int CHUNK, int UNR, int PER, int R>
__global__ __launch_bounds__(NEAR_THREADS) void k_near_scn(const NearTile *__restrict__ tiles,
                                                       const int32_t *__restrict__ items,
                                                       const int32_t *__restrict__ pW,
                                                       const int64_t *__restrict__ item_base,
                                                       const int32_t *__restrict__ item_rel,
                                                       const uint16_t *__restrict__ item_rng,
                                                       const KT *__restrict__ Kw, const double *__restrict__ Dring,
                                                       int L, StepIdx si,
                                                       const int32_t *__restrict__ perm,
                                                       const int32_t *__restrict__ pslot,
                                                       double *__restrict__ partial, Scn sc) {
    const int64_t n = si.get();
    constexpr int SP = (64 * PER > CHUNK) ? 64 * PER / CHUNK : 1;  // sources per wave-wide load
    constexpr int SPAN = 64 / SP * PER;                             // lags per source per load
    static_assert(PER * sizeof(KT) <= 16, "at most 16-byte loads");
    static_assert(SP <= 2 && CHUNK % SPAN == 0, "a chunk is a whole number of loads");
    static_assert(R > 1, "one scenario runs k_near");
    // R scenarios share the windows: each window value loaded once is applied
    // to the R histories staged here
    __shared__ double Dt[R][TILE][CHUNK];
    __shared__ int32_t Ol[TILE * TILE];
    __shared__ uint16_t Wl[TILE * TILE];
    __shared__ uint16_t Rg[TILE];
    __shared__ int32_t Ps[TILE];
    // optional launch order: workgroup -> item (-1: padding slot)
    const int item = perm ? perm[blockIdx.x] : (int)blockIdx.x;
    if (item < 0) return;
    const int t = items[2 * item];
    const int ch = items[2 * item + 1];
    const NearTile &T = tiles[t];
    const int nr = T.nr, ns = T.ns;
    const int64_t m0 = (int64_t)ch * CHUNK;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    constexpr int NW = NEAR_THREADS / 64;
    if (n >= T.hz) return;  // the tile's problem has finished its run; its receivers read nothing
    if (m0 > n) {  // no history reaches this chunk yet
        for (int r = threadIdx.x; r < nr; r += blockDim.x)
            for (int c = 0; c < R; ++c) partial[c * sc.part + pslot[(int64_t)item * TILE + r]] = 0.0;
        return;
    }
    const int np = nr * ns;
    for (int q = threadIdx.x; q < np; q += blockDim.x) {
        Wl[q] = (uint16_t)pW[T.pair_begin + q];
        Ol[q] = item_rel[(int64_t)item * (TILE * TILE) + q];
    }
    if (threadIdx.x < TILE) {
        Rg[threadIdx.x] = item_rng[(int64_t)item * TILE + threadIdx.x];
        Ps[threadIdx.x] = pslot[(int64_t)item * TILE + threadIdx.x];
    }
#pragma unroll
    for (int c = 0; c < R; ++c)
        for (int idx = threadIdx.x; idx < ns * CHUNK; idx += blockDim.x) {
            const int sl = idx / CHUNK, mm = idx % CHUNK;
            Dt[c][sl][mm] = Dring[c * sc.D + (int64_t)T.src[sl] * L + ((m0 + mm - n) & (L - 1))];
        }
    __syncthreads();
    const int hist_len = (int)((n - m0 + 1) < CHUNK ? (n - m0 + 1) : CHUNK);  // lags with history
    const KT *__restrict__ Kt = Kw + item_base[item];
    const int subs = (hist_len + SPAN - 1) / SPAN;
    for (int r = wave; r < nr; r += NW) {
        double acc[R];
#pragma unroll
        for (int c = 0; c < R; ++c) acc[c] = 0.0;
        const int pb = r * ns;
        // sources whose windows reach this chunk (the tail chunks of a tile
        // hold only the pairs with the longest windows), widened to whole
        // unrolled blocks so that every block issues UNR loads back to back
        const int r_lo = Rg[r] & 0xFF, r_hi = Rg[r] >> 8;
        const int s_lo = r_lo & ~(UNR - 1);
        const int s_hi = r_hi > r_lo ? min(ns, s_lo + ((r_hi - s_lo + UNR - 1) & ~(UNR - 1))) : s_lo;
        const int half = lane / (64 / SP);  // which of the load's sources this lane serves
        for (int sub = 0; sub < subs; ++sub) {
            const int mm = sub * SPAN + lane % (64 / SP) * PER;  // first lag of this lane in the chunk
            // branch-free: lanes past a segment read its last aligned element(s)
            // (one cache line for the whole wave) and contribute zero, so the
            // unrolled loads are independent and issued back to back
#pragma unroll (UNR / SP)
            for (int s2 = s_lo; s2 < s_hi; s2 += SP) {
                // two sources per load: the range may end on its first (odd
                // count at the end of a tile); the second then reads the first's
                // metadata and contributes zero
                const bool live = SP == 1 || s2 + half < s_hi;
                const int sl = live ? s2 + half : s2;
                const int q = pb + sl;
                const int len = live ? (int)Wl[q] - (int)m0 : 0;  // lags of this pair in the chunk (may be <= 0 or > CHUNK)
                const int lim = len < hist_len ? len : hist_len;
                const int last = len > 0 ? (((len < CHUNK ? len : CHUNK) - 1) & ~(PER - 1)) : 0;
                const int mc = mm < last ? mm : last;
                // the mask goes on the history operand so that every load's
                // result is consumed (window values are finite), which keeps the
                // compiler from sinking the loads into branches
                if constexpr (PER == 1) {
                    const double kv = (double)__builtin_nontemporal_load(Kt + Ol[q] + mc);
#pragma unroll
                    for (int c = 0; c < R; ++c) {
                        const double dv = (mm < lim) ? Dt[c][sl][mm] : 0.0;
                        acc[c] = fma(kv, dv, acc[c]);
                    }
                } else if constexpr (PER == 2) {
                    using V2 = typename std::conditional<sizeof(KT) == 8, nt_double2, nt_float2>::type;
                    const V2 kv = __builtin_nontemporal_load(reinterpret_cast<const V2 *>(Kt + Ol[q] + mc));
                    // the mask goes on the window value, once for all scenarios
                    // (the staged histories are finite ring values)
                    const double ka = (mm < lim) ? (double)kv.x : 0.0;
                    const double kb = (mm + 1 < lim) ? (double)kv.y : 0.0;
#pragma unroll
                    for (int c = 0; c < R; ++c) {
                        acc[c] = fma(ka, Dt[c][sl][mm], acc[c]);
                        acc[c] = fma(kb, Dt[c][sl][mm + 1], acc[c]);
                    }
                } else {
                    const nt_float4 kv = __builtin_nontemporal_load(reinterpret_cast<const nt_float4 *>(Kt + Ol[q] + mc));
#pragma unroll
                    for (int c = 0; c < R; ++c) {
                        const double d0 = (mm < lim) ? Dt[c][sl][mm] : 0.0;
                        const double d1 = (mm + 1 < lim) ? Dt[c][sl][mm + 1] : 0.0;
                        const double d2 = (mm + 2 < lim) ? Dt[c][sl][mm + 2] : 0.0;
                        const double d3 = (mm + 3 < lim) ? Dt[c][sl][mm + 3] : 0.0;
                        acc[c] = fma((double)kv.x, d0, acc[c]);
                        acc[c] = fma((double)kv.y, d1, acc[c]);
                        acc[c] = fma((double)kv.z, d2, acc[c]);
                        acc[c] = fma((double)kv.w, d3, acc[c]);
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const double a = wave_sum(acc[c]);
            if (lane == 0) partial[c * sc.part + Ps[r]] = a;
        }
    }
}

// Far field, source side: one thread per group of sources sharing a delay.
// INJECT: commit of a step predicted with D_n = 0 (its history slot now holds
// D_n): each source adds only its D_n terms (the first FIR tap in Domain F,
// D_n itself in the Domain-S and transient pieces), without clearing (the
// prediction did).
// XS: step xb of a time block whose source inputs (the FIR outputs of Domain
// F, D itself elsewhere) k_far_fir_tb has already computed, xs[xb][source]
// (xn sources per row).
template <class FT, bool INJECT, bool XS = false>
__global__ void k_far_src(const SrcGroup *__restrict__ groups, int n_groups, const GroupSrc *__restrict__ gsrc,
                          const FarBlock *__restrict__ blocks, const FT *__restrict__ gdat,
                          const double *__restrict__ hdat, const double *__restrict__ Drec, int N, int Lf, StepIdx si,
                          double *__restrict__ rings, Scn sc, int tb, const double *__restrict__ xs = nullptr,
                          int xb = 0, int xn = 0) {
    const int64_t n = si.get();
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= n_groups) return;
    Drec += blockIdx.y * sc.Drec;  // scenario blockIdx.y
    rings += blockIdx.y * sc.ring;
    const SrcGroup G = groups[gi];
    const FarBlock B = blocks[G.block];
    if (n >= B.hz) return;
    const int64_t Lr = B.ring_len;
    double *ring = rings + B.ring_off;
    // F and S rings are [slot][rank]; transient u rings are [rank][slot]
    const bool tr = B.kind == PIECE_TR;
    const int64_t rs = tr ? Lr : 1;        // stride between ranks
    const int64_t ss = tr ? 1 : B.rank;    // stride between slots
    if (G.clear && !INJECT) {
        // F and S: the slot the oldest gather still to come (of this step's
        // time block) has read, tb - 1 steps before the single-step case
        const int64_t tc = tr ? n - B.dm_min - B.ntr - tb : n - tb - B.dm_max;
        for (int l = 0; l < B.rank; ++l) ring[l * rs + (tc & (Lr - 1)) * ss] = 0.0;
    }
    const int64_t slot = (n + G.delay) & (Lr - 1);
    constexpr int CH = 8;
    for (int q0 = 0; q0 < G.count; q0 += CH) {
        double x[CH];
        int jl[CH];
        const int cnt = G.count - q0 < CH ? G.count - q0 : CH;
        for (int q = 0; q < cnt; ++q) {
            const GroupSrc S = gsrc[G.first + q0 + q];
            jl[q] = S.jl;
            if (XS) {
                x[q] = xs[(int64_t)xb * xn + G.first + q0 + q];
            } else if (INJECT) {
                const double dn = Drec[(int64_t)(n & (Lf - 1)) * N + S.j];
                x[q] = B.kind != PIECE_F ? dn : (S.h_len > 0 ? hdat[S.h_off] * dn : 0.0);
            } else if (B.kind == PIECE_F) {
                // waveforms tap-major (stride N_s) and the time-major recent
                // history: lanes with neighbouring sources read neighbouring
                // addresses; four taps per pass keep eight loads in flight
                const double *h = hdat + S.h_off;
                const int64_t hs = B.ns;
                const double *dj = Drec + S.j;
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                int m = 0;
                for (; m + 4 <= S.h_len; m += 4) {
                    a0 += h[m * hs] * dj[(int64_t)((n - m) & (Lf - 1)) * N];
                    a1 += h[(m + 1) * hs] * dj[(int64_t)((n - m - 1) & (Lf - 1)) * N];
                    a2 += h[(m + 2) * hs] * dj[(int64_t)((n - m - 2) & (Lf - 1)) * N];
                    a3 += h[(m + 3) * hs] * dj[(int64_t)((n - m - 3) & (Lf - 1)) * N];
                }
                for (; m < S.h_len; ++m) a0 += h[m * hs] * dj[(int64_t)((n - m) & (Lf - 1)) * N];
                x[q] = (a0 + a1) + (a2 + a3);
            } else {
                x[q] = Drec[(int64_t)(n & (Lf - 1)) * N + S.j];
            }
        }
        const FT *g = gdat + B.g_off;
        double *rr = ring + slot * ss;
        if (cnt == 1) {
            // the usual case: one source per delay; four ranks per pass
            const FT *gj = g + (int64_t)jl[0] * B.rank;
            const double x0 = x[0];
            int l = 0;
            for (; l + 4 <= B.rank; l += 4) {
                const double g0 = widen(gj[l]), g1 = widen(gj[l + 1]), g2 = widen(gj[l + 2]), g3 = widen(gj[l + 3]);
                const double r0 = rr[l * rs], r1 = rr[(l + 1) * rs], r2 = rr[(l + 2) * rs], r3 = rr[(l + 3) * rs];
                rr[l * rs] = fma(g0, x0, r0);
                rr[(l + 1) * rs] = fma(g1, x0, r1);
                rr[(l + 2) * rs] = fma(g2, x0, r2);
                rr[(l + 3) * rs] = fma(g3, x0, r3);
            }
            for (; l < B.rank; ++l) rr[l * rs] = fma(widen(gj[l]), x0, rr[l * rs]);
        } else {
            for (int l = 0; l < B.rank; ++l) {
                double acc = 0.0;
                for (int q = 0; q < cnt; ++q) acc = fma(widen(g[(int64_t)jl[q] * B.rank + l]), x[q], acc);
                rr[l * rs] += acc;
            }
        }
    }
}

// 2D transient: y_{p*} = sum_k h^tr_k u_{p*-k}, p* = n - min dm (App. B.3).
__global__ __launch_bounds__(256) void k_tr_fir(const int32_t *__restrict__ tr_list, int n_tr,
                                                const FarBlock *__restrict__ blocks, const double *__restrict__ htr,
                                                const double *__restrict__ rings, double *__restrict__ yrings,
                                                StepIdx si, Scn sc) {
    const int64_t n = si.get();
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= n_tr) return;
    rings += blockIdx.y * sc.ring;  // scenario blockIdx.y
    yrings += blockIdx.y * sc.y;
    const int b = tr_list[2 * w], l = tr_list[2 * w + 1];
    const FarBlock B = blocks[b];
    if (n >= B.hz) return;
    const int64_t Lu = B.ring_len, Ly = B.y_len;
    const double *u = rings + B.ring_off + (int64_t)l * Lu;
    const double *h = htr + B.htr_off;
    const int64_t ps = n - B.dm_min;
    double a0 = 0.0, a1 = 0.0;
    int k = lane;
    for (; k + 64 < B.ntr; k += 128) {
        a0 += h[k] * u[(ps - k) & (Lu - 1)];
        a1 += h[k + 64] * u[(ps - k - 64) & (Lu - 1)];
    }
    if (k < B.ntr) a0 += h[k] * u[(ps - k) & (Lu - 1)];
    double acc = wave_sum(a0 + a1);
    if (lane == 0) yrings[B.y_off + (ps & (Ly - 1)) * B.rank + l] = acc;
}

// 2D transient with a staircase waveform (App. A.1, Eq. A.3): per run q the
// running sum S_q(p) = sum_{k in run q} u_{p-k} advances by one step as
// S_q += u_{p - b_q} - u_{p - b_{q+1}}, and y_p = sum_q h^_q S_q.
__global__ __launch_bounds__(256) void k_tr_quant(const int32_t *__restrict__ tr_list, int n_tr,
                                                  const FarBlock *__restrict__ blocks,
                                                  const int32_t *__restrict__ qbounds,
                                                  const double *__restrict__ qrep, double *__restrict__ qstate,
                                                  const double *__restrict__ rings, double *__restrict__ yrings,
                                                  StepIdx si, Scn sc) {
    const int64_t n = si.get();
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= n_tr) return;
    rings += blockIdx.y * sc.ring;  // scenario blockIdx.y
    yrings += blockIdx.y * sc.y;
    qstate += blockIdx.y * sc.q;
    const int b = tr_list[2 * w], l = tr_list[2 * w + 1];
    const FarBlock B = blocks[b];
    if (n >= B.hz) return;
    const int64_t Lu = B.ring_len, Ly = B.y_len;
    const double *u = rings + B.ring_off + (int64_t)l * Lu;
    const int32_t *qb = qbounds + B.qb_off;
    const double *rep = qrep + B.qr_off;
    double *S = qstate + B.qs_off + (int64_t)l * B.nq;
    const int64_t ps = n - B.dm_min;
    double acc = 0.0;
    for (int q = lane; q < B.nq; q += 64) {
        const double v = S[q] + u[(ps - qb[q]) & (Lu - 1)] - u[(ps - qb[q + 1]) & (Lu - 1)];
        S[q] = v;
        acc += rep[q] * v;
    }
    acc = wave_sum(acc);
    if (lane == 0) yrings[B.y_off + (ps & (Ly - 1)) * B.rank + l] = acc;
}

// Time block, far-field source side, first part: the source inputs of the
// B steps n .. n+B-1 of every group source, xs[xb0 + b][source] (step-major,
// xn group sources per row, so that each step's scatter reads a row; Domain F: the FIR
// of Eq. 52 over the degenerate waveform, each tap loaded once for the B
// steps, summed as the single-step kernel sums it; Domain S and transient:
// D itself).  The scatter of each step then reads them (k_far_src<.., XS>).
template <int B>
__global__ void k_far_fir_tb(const SrcGroup *__restrict__ groups, int n_groups, const GroupSrc *__restrict__ gsrc,
                             const FarBlock *__restrict__ blocks, const double *__restrict__ hdat,
                             const double *__restrict__ Drec, int N, int Lf, StepIdx si, double *__restrict__ xs,
                             int xn, int xb0) {
    const int64_t n = si.get();
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= n_groups) return;
    const SrcGroup G = groups[gi];
    const FarBlock Bk = blocks[G.block];
    if (n >= Bk.hz) return;
    for (int q = 0; q < G.count; ++q) {
        const GroupSrc S = gsrc[G.first + q];
        const double *dj = Drec + S.j;
        double x[B];
        if (Bk.kind == PIECE_F) {
            const double *h = hdat + S.h_off;
            const int64_t hs = Bk.ns;
            double a0[B], a1[B], a2[B], a3[B];
#pragma unroll
            for (int b = 0; b < B; ++b) a0[b] = a1[b] = a2[b] = a3[b] = 0.0;
            int m = 0;
            for (; m + 4 <= S.h_len; m += 4) {
                const double h0 = h[m * hs], h1 = h[(m + 1) * hs], h2 = h[(m + 2) * hs], h3 = h[(m + 3) * hs];
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    a0[b] += h0 * dj[(int64_t)((n + b - m) & (Lf - 1)) * N];
                    a1[b] += h1 * dj[(int64_t)((n + b - m - 1) & (Lf - 1)) * N];
                    a2[b] += h2 * dj[(int64_t)((n + b - m - 2) & (Lf - 1)) * N];
                    a3[b] += h3 * dj[(int64_t)((n + b - m - 3) & (Lf - 1)) * N];
                }
            }
            for (; m < S.h_len; ++m) {
                const double hm = h[m * hs];
#pragma unroll
                for (int b = 0; b < B; ++b) a0[b] += hm * dj[(int64_t)((n + b - m) & (Lf - 1)) * N];
            }
#pragma unroll
            for (int b = 0; b < B; ++b) x[b] = (a0[b] + a1[b]) + (a2[b] + a3[b]);
        } else {
#pragma unroll
            for (int b = 0; b < B; ++b) x[b] = dj[(int64_t)((n + b) & (Lf - 1)) * N];
        }
#pragma unroll
        for (int b = 0; b < B; ++b) xs[(int64_t)(xb0 + b) * xn + G.first + q] = x[b];
    }
}

// Time block, the scatter of all its steps in one launch.  The per-step
// kernel above run for the B steps in step order gives the same sums: every
// ring slot takes its contributions in step order, each added as that kernel
// adds it (one source: a fused multiply-add into the slot; several: their
// partial sum, eight sources at a time).  Work item: a tile of one far
// block's ring slots, one wave, a lane per (slot, rank); slot u of the block
// (the absolute slot n + dmin + u of the block's first step n) takes the
// group of delay dmin + u - k at step k.  The tile's groups are staged in LDS
// by delay; the loads of half a block's contributions to a slot are issued
// before the first of them is added.  The slots the block's steps clear (the oldest slot a gather still
// to come has read, one per step) start from zero where a tile owns them; the
// block's first tile clears the others.
template <class FT>
__global__ __launch_bounds__(64) void k_far_scat_tb(const ScatItem *__restrict__ items,
                                                    const SrcGroup *__restrict__ groups,
                                                    const GroupSrc *__restrict__ gsrc, const FT *__restrict__ gdat,
                                                    const double *__restrict__ xs, int xn,
                                                    double *__restrict__ rings, StepIdx si) {
    constexpr int B = TIME_BLOCK, H = B / 2;
    constexpr int W = SCAT_TILE + B - 1;
    __shared__ int32_t wf[W], wc[W], wj[W];  // per delay of the window: first source, count, first column
    const ScatItem it = items[blockIdx.x];
    const int64_t n = si.get();
    const int kmax = (int)(it.hz - n < B ? it.hz - n : B);  // steps of the block with work in this far block
    if (kmax <= 0) return;
    const int rank = it.rank;
    const int64_t mask = (int64_t)it.ring_len - 1;
    double *ring = rings + it.ring_off;
    // F and S rings are [slot][rank]; transient u rings are [rank][slot]
    const bool tr = it.kind == PIECE_TR;
    const int64_t rs = tr ? (int64_t)it.ring_len : 1, ss = tr ? 1 : rank;
    const int64_t cbase = n - it.cb;  // step k clears slot cbase + k
    const int64_t S0 = n + it.dmin;   // the absolute slot of u = 0
    const int U = it.D + kmax - 1;    // slots with contributions
    const int lane = threadIdx.x;
    if (it.first)
        for (int idx = lane; idx < kmax * rank; idx += 64) {
            const int k = idx % kmax, l = idx / kmax;
            const int64_t p = cbase + k;
            if (((p - S0) & mask) < U) continue;  // a tile owns it
            ring[l * rs + (p & mask) * ss] = 0.0;
        }
    const int u0 = it.u0;
    const int nu = it.nu < U - u0 ? it.nu : U - u0;
    if (nu <= 0) return;
    const int w0 = u0 - (B - 1);  // delay (relative to dmin) of window entry 0
    const int wn = nu + B - 1;
    for (int w = lane; w < wn; w += 64) wc[w] = 0;
    __syncthreads();
    // distinct increasing delays: group i has relative delay in [i, i + D - ng]
    const int i_lo = max(0, w0 - (it.D - it.ng)), i_hi = min(it.ng, w0 + wn);
    for (int i = i_lo + lane; i < i_hi; i += 64) {
        const SrcGroup G = groups[it.g0 + i];
        const int w = G.delay - it.dmin - w0;
        if (w >= 0 && w < wn) {
            wf[w] = G.first;
            wc[w] = G.count;
            wj[w] = G.jl0;
        }
    }
    __syncthreads();
    const FT *__restrict__ g = gdat + it.g_off;
    const int nout = nu * rank;
    for (int idx = lane; idx < nout; idx += 64) {
        int u, l;
        if (tr) {
            l = idx / nu;
            u = u0 + idx % nu;
        } else {
            u = u0 + idx / rank;
            l = idx % rank;
        }
        const int64_t sl = S0 + u;
        const bool clr = ((sl - cbase) & mask) < kmax;
        double *rp = ring + l * rs + (sl & mask) * ss;
        double r = clr ? 0.0 : *rp;
        bool any = clr;
        // half a block's steps at a time: their loads, then their sums in step order
#pragma unroll
        for (int k0 = 0; k0 < B; k0 += H) {
            int c[H], f[H];
            double gv[H], xv[H];
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const int k = k0 + h;
                const int w = u - u0 + B - 1 - k;
                c[h] = k < kmax ? wc[w] : 0;
                f[h] = c[h] > 0 ? wf[w] : 0;
                const int j = c[h] == 1 ? wj[w] : 0;
                gv[h] = widen(g[(int64_t)j * rank + l]);
                xv[h] = xs[(int64_t)k * xn + f[h]];
            }
#pragma unroll
            for (int h = 0; h < H; ++h) {
                if (c[h] == 1) {
                    r = fma(gv[h], xv[h], r);
                    any = true;
                } else if (c[h] > 1) {
                    const double *xk = xs + (int64_t)(k0 + h) * xn + f[h];
                    for (int q0 = 0; q0 < c[h]; q0 += 8) {
                        const int cc = c[h] - q0 < 8 ? c[h] - q0 : 8;
                        if (cc == 1) {
                            r = fma(widen(g[(int64_t)gsrc[f[h] + q0].jl * rank + l]), xk[q0], r);
                        } else {
                            double acc = 0.0;
                            for (int q = 0; q < cc; ++q)
                                acc = fma(widen(g[(int64_t)gsrc[f[h] + q0 + q].jl * rank + l]), xk[q0 + q], acc);
                            r += acc;
                        }
                    }
                    any = true;
                }
            }
        }
        if (any) *rp = r;
    }
}

// Time block, 2D transient FIR of the B steps (sums as in k_tr_fir: per lane
// the taps k = lane + 128 i in one accumulator, k + 64 in the other).  Each
// wave stages the u values of a pair of 64-tap chunks for all B steps in LDS
// (128 + B - 1 values, read from the ring once) and every lane reads its B
// values per tap from there.  The u rings are complete: every scatter of the
// block ran before (a transient source reaches its u ring no earlier than the
// next step).
template <int B>
__global__ __launch_bounds__(256) void k_tr_fir_tb(const int32_t *__restrict__ tr_list, int n_tr,
                                                   const FarBlock *__restrict__ blocks, const double *__restrict__ htr,
                                                   const double *__restrict__ rings, double *__restrict__ yrings,
                                                   StepIdx si) {
    constexpr int US = 128 + B;  // staged values per wave (128 + B - 1 used)
    __shared__ double ust[4][US];
    const int64_t n = si.get();
    const int wv = threadIdx.x >> 6;
    const int w = blockIdx.x * 4 + wv;
    const int lane = threadIdx.x & 63;
    if (w >= n_tr) return;
    const int b_ = tr_list[2 * w], l = tr_list[2 * w + 1];
    const FarBlock Bk = blocks[b_];
    if (n >= Bk.hz) return;
    const int64_t Lu = Bk.ring_len, Ly = Bk.y_len;
    const double *u = rings + Bk.ring_off + (int64_t)l * Lu;
    const double *h = htr + Bk.htr_off;
    const int64_t ps = n - Bk.dm_min;
    double *us = ust[wv];
    double a0[B], a1[B];
#pragma unroll
    for (int b = 0; b < B; ++b) a0[b] = a1[b] = 0.0;
    // taps k = k0 + lane (first chunk) and k + 64 (second) for step ps + b
    // read u at ps + b - k, staged at index b + 127 - (k - k0).  The chunk
    // pairs are wave-uniform; per lane, pairs with both taps below ntr, then
    // at most one with the first only, as in the single-step loop.  The
    // wave's LDS writes and reads stay in program order, and no other wave
    // touches its row.
    for (int k0 = 0; k0 < Bk.ntr; k0 += 128) {
        for (int i = lane; i < 127 + B; i += 64) us[i] = u[(ps - k0 - 127 + i) & (Lu - 1)];
        __builtin_amdgcn_wave_barrier();
        const int k = k0 + lane;
        if (k + 64 < Bk.ntr) {
            const double hk = h[k], hk64 = h[k + 64];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                a0[b] += hk * us[b + 127 - lane];
                a1[b] += hk64 * us[b + 63 - lane];
            }
        } else if (k < Bk.ntr) {
            const double hk = h[k];
#pragma unroll
            for (int b = 0; b < B; ++b) a0[b] += hk * us[b + 127 - lane];
        }
        __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const double acc = wave_sum(a0[b] + a1[b]);
        if (lane == 0 && n + b < Bk.hz) yrings[Bk.y_off + ((ps + b) & (Ly - 1)) * Bk.rank + l] = acc;
    }
}

// Time block, staircase transient: the B steps' running-sum updates in order.
template <int B>
__global__ __launch_bounds__(256) void k_tr_quant_tb(const int32_t *__restrict__ tr_list, int n_tr,
                                                     const FarBlock *__restrict__ blocks,
                                                     const int32_t *__restrict__ qbounds,
                                                     const double *__restrict__ qrep, double *__restrict__ qstate,
                                                     const double *__restrict__ rings, double *__restrict__ yrings,
                                                     StepIdx si) {
    const int64_t n = si.get();
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= n_tr) return;
    const int b_ = tr_list[2 * w], l = tr_list[2 * w + 1];
    const FarBlock Bk = blocks[b_];
    const int64_t Lu = Bk.ring_len, Ly = Bk.y_len;
    const double *u = rings + Bk.ring_off + (int64_t)l * Lu;
    const int32_t *qb = qbounds + Bk.qb_off;
    const double *rep = qrep + Bk.qr_off;
    double *S = qstate + Bk.qs_off + (int64_t)l * Bk.nq;
    for (int b = 0; b < B; ++b) {
        if (n + b >= Bk.hz) return;
        const int64_t ps = n + b - Bk.dm_min;
        double acc = 0.0;
        for (int q = lane; q < Bk.nq; q += 64) {
            const double v = S[q] + u[(ps - qb[q]) & (Lu - 1)] - u[(ps - qb[q + 1]) & (Lu - 1)];
            S[q] = v;
            acc += rep[q] * v;
        }
        acc = wave_sum(acc);
        if (lane == 0) yrings[Bk.y_off + (ps & (Ly - 1)) * Bk.rank + l] = acc;
    }
}

// Per receiver: one wave sums the near partials, the static tails of its
// near pairs (App. E: K^S_ij dt times the running slip sum U_{j, n - W_ij}),
// and its far-field gathers; lane 0 updates the Domain-S stress and writes T_n.
template <class FT>
__global__ __launch_bounds__(256) void k_recv(
    int N, StepIdx si, int L, const int32_t *__restrict__ rn_ptr, const double *__restrict__ partial,
    const int32_t *__restrict__ rp_ptr, const TailPair *__restrict__ tails, const double *__restrict__ Uring,
    const int32_t *__restrict__ re_ptr,
    const RecvEntry *__restrict__ re, const FT *__restrict__ fdat, const double *__restrict__ rings,
    const double *__restrict__ yrings, double *__restrict__ TS, const double *__restrict__ self0,
    const double *__restrict__ Dring, const int32_t *__restrict__ hz, double *__restrict__ t, Scn sc) {
    const int64_t n = si.get();
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= N) return;
    const int c = blockIdx.y;  // scenario
    partial += c * sc.part;
    Uring += c * sc.U;
    Dring += c * sc.D;
    rings += c * sc.ring;
    yrings += c * sc.y;
    TS += (int64_t)c * N;
    t += (n - si.n0) * sc.row + (int64_t)c * N;
    if (n >= hz[i]) {  // the receiver's problem has finished its run
        if (lane == 0) t[i] = 0.0;
        return;
    }
    double acc = 0.0, accS = 0.0;
    if (self0 && lane == 0) acc = self0[i] * Dring[(int64_t)i * L + ((-n) & (L - 1))];
    for (int k = rn_ptr[i] + lane; k < rn_ptr[i + 1]; k += 64) acc += partial[k];
    for (int k = rp_ptr[i] + lane; k < rp_ptr[i + 1]; k += 64) {
        const TailPair tp = tails[k];
        // the window holds K - K^S dt over its lags, so the static part of every
        // lag comes in through the running sum: sum_m K^S dt D_{n-m} = K^S dt U_n
        acc += tp.ks * Uring[(n & (U_SLOTS - 1)) * N + tp.src];
    }
    for (int k = re_ptr[i] + lane; k < re_ptr[i + 1]; k += 64) {
        const RecvEntry e = re[k];
        const int64_t slot = (n - e.dm) & e.mask;
        const FT *f = fdat + e.f_off;
        const double *r = (e.kind == PIECE_TR ? yrings : rings) + e.r_off + slot * e.rank;
        // four ranks per pass: eight independent loads in flight per lane
        double v = 0.0;
        int l = 0;
        for (; l + 4 <= e.cnt; l += 4) {
            const double a0 = widen(f[l]), a1 = widen(f[l + 1]), a2 = widen(f[l + 2]), a3 = widen(f[l + 3]);
            const double b0 = r[l], b1 = r[l + 1], b2 = r[l + 2], b3 = r[l + 3];
            v += (a0 * b0 + a1 * b1) + (a2 * b2 + a3 * b3);
        }
        for (; l < e.cnt; ++l) v += widen(f[l]) * r[l];
        if (e.kind == PIECE_S)
            accS += v;
        else
            acc += v;
    }
    acc = wave_sum(acc);
    accS = wave_sum(accS);
    if (lane == 0) {
        const double ts = TS[i] + accS;
        TS[i] = ts;
        t[i] = acc + ts;
    }
}

// Time block: the gathers of the B steps n .. n+B-1 (one scenario), each
// entry's metadata and factors loaded once for the B steps; every step's sums
// are added in the order k_recv adds them, and the Domain-S stress advances
// step by step.
template <class FT, int B>
__global__ __launch_bounds__(256) void k_recv_tb(
    int N, StepIdx si, int L, const int32_t *__restrict__ rn_ptr, const double *__restrict__ partial, int64_t part,
    const int32_t *__restrict__ rp_ptr, const TailPair *__restrict__ tails, const double *__restrict__ Uring,
    const int32_t *__restrict__ re_ptr, const RecvEntry *__restrict__ re, const FT *__restrict__ fdat,
    const double *__restrict__ rings, const double *__restrict__ yrings, double *__restrict__ TS,
    const double *__restrict__ self0, const double *__restrict__ Dring, const int32_t *__restrict__ hz,
    double *__restrict__ t, int64_t row) {
    const int64_t n = si.get();
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= N) return;
    t += (n - si.n0) * row;
    // steps of the block before the receiver's problem ends its run
    const int live = (int)(hz[i] - n < B ? (hz[i] - n > 0 ? hz[i] - n : 0) : B);
    double acc[B], accS[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        acc[b] = 0.0;
        accS[b] = 0.0;
    }
    if (self0 && lane == 0)
#pragma unroll
        for (int b = 0; b < B; ++b) acc[b] = self0[i] * Dring[(int64_t)i * L + ((-(n + b)) & (L - 1))];
    // two passes' loads in flight before their sums (added in the single-step
    // kernel's order)
    const int ke = rn_ptr[i + 1];
    for (int k = rn_ptr[i] + lane; k < ke; k += 128) {
        const bool two = k + 64 < ke;
        double p0[B], p1[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            p0[b] = partial[b * part + k];
            p1[b] = two ? partial[b * part + k + 64] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < B; ++b) acc[b] += p0[b];
        if (two)
#pragma unroll
            for (int b = 0; b < B; ++b) acc[b] += p1[b];
    }
    const int pe = rp_ptr[i + 1];
    for (int k = rp_ptr[i] + lane; k < pe; k += 128) {
        const bool two = k + 64 < pe;
        const TailPair tp0 = tails[k], tp1 = tails[two ? k + 64 : k];
        double u0[B], u1[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            u0[b] = Uring[((n + b) & (U_SLOTS - 1)) * N + tp0.src];
            u1[b] = Uring[((n + b) & (U_SLOTS - 1)) * N + tp1.src];
        }
#pragma unroll
        for (int b = 0; b < B; ++b) acc[b] += tp0.ks * u0[b];
        if (two)
#pragma unroll
            for (int b = 0; b < B; ++b) acc[b] += tp1.ks * u1[b];
    }
    for (int k = re_ptr[i] + lane; k < re_ptr[i + 1]; k += 64) {
        const RecvEntry e = re[k];
        const FT *f = fdat + e.f_off;
        const double *r0 = (e.kind == PIECE_TR ? yrings : rings) + e.r_off;
        double v[B];
#pragma unroll
        for (int b = 0; b < B; ++b) v[b] = 0.0;
        int l = 0;
        for (; l + 4 <= e.cnt; l += 4) {
            const double a0 = widen(f[l]), a1 = widen(f[l + 1]), a2 = widen(f[l + 2]), a3 = widen(f[l + 3]);
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const double *r = r0 + ((n + b - e.dm) & e.mask) * e.rank;
                const double b0 = r[l], b1 = r[l + 1], b2 = r[l + 2], b3 = r[l + 3];
                v[b] += (a0 * b0 + a1 * b1) + (a2 * b2 + a3 * b3);
            }
        }
        for (; l < e.cnt; ++l) {
            const double a = widen(f[l]);
#pragma unroll
            for (int b = 0; b < B; ++b) v[b] += a * r0[((n + b - e.dm) & e.mask) * e.rank + l];
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            if (e.kind == PIECE_S)
                accS[b] += v[b];
            else
                acc[b] += v[b];
        }
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
        acc[b] = wave_sum(acc[b]);
        accS[b] = wave_sum(accS[b]);
    }
    if (lane == 0) {
        double ts = TS[i];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            if (b < live) {
                ts += accS[b];
                t[b * row + i] = acc[b] + ts;
            } else {
                t[b * row + i] = 0.0;
            }
        }
        TS[i] = ts;
    }
}

// Window bytes each lane loads at once in a configuration (as launched below).
static int near_load_bytes(const FdphOp &F, const NearTune &c) {
    const int narrow = (F.precision != BIE_FP64 && F.near_chunk == 64) ? 4 : 8;
    return c.wide ? 2 * narrow : narrow;
}

// The near-field kernel in a given launch configuration (unroll, load width,
// occupancy cap through unused LDS, workgroup order).
int launch_near(const FdphOp &F, const NearTune &c, hipStream_t s, const StepIdx &si) {
    const dim3 g(c.perm ? c.grid : F.n_items), b(NEAR_THREADS);
    const size_t pad = (size_t)c.lds_pad;
    const bool deep = c.unroll >= 16;
    const bool wide = c.wide != 0;
#define BIE_NEAR_LAUNCH(KT, C, U, P, RR, KW)                                                                   \
    do {                                                                                                       \
        if constexpr (RR == 1)                                                                                 \
            hipLaunchKernelGGL((k_near<KT, C, U, P>), g, b, pad, s, F.tiles, F.items, F.pW, F.item_base,       \
                               F.item_rel, F.item_rng, KW, F.Dring, F.L, si, c.perm, F.pslot, F.partial);      \
        else                                                                                                   \
            hipLaunchKernelGGL((k_near_scn<KT, C, U, P, RR>), g, b, pad, s, F.tiles, F.items, F.pW,            \
                               F.item_base, F.item_rel, F.item_rng, KW, F.Dring, F.L, si, c.perm, F.pslot,     \
                               F.partial, F.scn);                                                              \
    } while (0)
#define BIE_NEAR_UNROLL(KT, C, P, RR, KW)                  \
    do {                                                   \
        if (deep) BIE_NEAR_LAUNCH(KT, C, 16, P, RR, KW);   \
        else BIE_NEAR_LAUNCH(KT, C, 8, P, RR, KW);         \
    } while (0)
    // narrow: 8-byte loads (4 for FP32 in 64-lag chunks); wide: twice that.
    // Several scenarios: 64- or 128-lag chunks (the staged histories fill the LDS).
#define BIE_NEAR_SCN(RR)                                                                                      \
    do {                                                                                                      \
        if (F.precision == BIE_FP64) {                                                                        \
            if (F.near_chunk == 64) {                                                                         \
                if (wide) BIE_NEAR_UNROLL(double, 64, 2, RR, F.Kw); else BIE_NEAR_UNROLL(double, 64, 1, RR, F.Kw); \
            } else {                                                                                          \
                if (wide) BIE_NEAR_UNROLL(double, 128, 2, RR, F.Kw); else BIE_NEAR_UNROLL(double, 128, 1, RR, F.Kw); \
            }                                                                                                 \
        } else {                                                                                              \
            if (F.near_chunk == 64) {                                                                         \
                if (wide) BIE_NEAR_UNROLL(float, 64, 2, RR, F.Kw32); else BIE_NEAR_UNROLL(float, 64, 1, RR, F.Kw32); \
            } else {                                                                                          \
                if (wide) BIE_NEAR_UNROLL(float, 128, 4, RR, F.Kw32); else BIE_NEAR_UNROLL(float, 128, 2, RR, F.Kw32); \
            }                                                                                                 \
        }                                                                                                     \
    } while (0)
    if (F.R == 2) {
        BIE_NEAR_SCN(2);
    } else if (F.R == 4) {
        BIE_NEAR_SCN(4);
    } else if (F.precision == BIE_FP64) {
        if (F.near_chunk == 64) {
            if (wide) BIE_NEAR_UNROLL(double, 64, 2, 1, F.Kw); else BIE_NEAR_UNROLL(double, 64, 1, 1, F.Kw);
        } else if (F.near_chunk == 128) {
            if (wide) BIE_NEAR_UNROLL(double, 128, 2, 1, F.Kw); else BIE_NEAR_UNROLL(double, 128, 1, 1, F.Kw);
        } else {
            if (wide) BIE_NEAR_UNROLL(double, 256, 2, 1, F.Kw); else BIE_NEAR_UNROLL(double, 256, 1, 1, F.Kw);
        }
    } else {
        if (F.near_chunk == 64) {
            if (wide) BIE_NEAR_UNROLL(float, 64, 2, 1, F.Kw32); else BIE_NEAR_UNROLL(float, 64, 1, 1, F.Kw32);
        } else if (F.near_chunk == 128) {
            if (wide) BIE_NEAR_UNROLL(float, 128, 4, 1, F.Kw32); else BIE_NEAR_UNROLL(float, 128, 2, 1, F.Kw32);
        } else {
            if (wide) BIE_NEAR_UNROLL(float, 256, 4, 1, F.Kw32); else BIE_NEAR_UNROLL(float, 256, 2, 1, F.Kw32);
        }
    }
#undef BIE_NEAR_SCN
#undef BIE_NEAR_UNROLL
#undef BIE_NEAR_LAUNCH
    BIE_HIP_TRY(hipGetLastError());
    return BIE_OK;
}

// The time-blocked near kernel in the launch configuration c (its load
// width, unroll, LDS pad and item order).
int launch_near_tb(const FdphOp &F, const NearTune &c, hipStream_t s, const StepIdx &si) {
    constexpr int B = TIME_BLOCK;
    const dim3 g(c.perm ? c.grid : F.n_items), b(NEAR_THREADS);
    const size_t pad = (size_t)c.lds_pad;
    if (c.mfma) {
        // chunk groups: one partial per (group, receiver, step), read by the
        // block gather through the groups' receiver lists
        const bool gr = c.mfma == 2 && F.n_grp > 0;
        const dim3 gm(c.perm ? c.grid : (gr ? F.n_grp : F.n_items));
        const int32_t *grp = gr ? F.grp : nullptr, *slots = gr ? F.gslot : F.pslot;
#define BIE_MFMA_LAUNCH_G(KT, C, KW, G)                                                                             \
    hipLaunchKernelGGL((k_near_mfma<KT, C, G>), gm, b, pad, s, F.tiles, F.items, F.pW, F.item_base, F.item_rel, KW, \
                       F.near_lags, F.Dring, F.L, si, c.perm, grp, slots, F.partial, F.scn.part)
#define BIE_MFMA_LAUNCH(KT, C, KW)                         \
    do {                                                   \
        if (gr) BIE_MFMA_LAUNCH_G(KT, C, KW, true);        \
        else BIE_MFMA_LAUNCH_G(KT, C, KW, false);          \
    } while (0)
        if (F.precision == BIE_FP64) {
            if (F.near_chunk == 64) BIE_MFMA_LAUNCH(double, 64, F.Kw);
            else if (F.near_chunk == 128) BIE_MFMA_LAUNCH(double, 128, F.Kw);
            else BIE_MFMA_LAUNCH(double, 256, F.Kw);
        } else {
            if (F.near_chunk == 64) BIE_MFMA_LAUNCH(float, 64, F.Kw32);
            else if (F.near_chunk == 128) BIE_MFMA_LAUNCH(float, 128, F.Kw32);
            else BIE_MFMA_LAUNCH(float, 256, F.Kw32);
        }
#undef BIE_MFMA_LAUNCH
#undef BIE_MFMA_LAUNCH_G
        BIE_HIP_TRY(hipGetLastError());
        return BIE_OK;
    }
    // the lane-per-lag kernel: SUB_BLOCK steps per launch
    const bool deep = c.unroll >= 16;
    const bool wide = c.wide != 0;
    constexpr int SB = SUB_BLOCK;
    for (int j = 0; j < B; j += SB) {
        StepIdx sj = si;
        if (sj.dev) sj.off += j;
        else sj.n += j;
        double *part = F.partial + (int64_t)j * F.scn.part;
#define BIE_TB_LAUNCH(KT, C, U, P, KW)                                                                         \
    hipLaunchKernelGGL((k_near_tb<KT, C, U, P, SB>), g, b, pad, s, F.tiles, F.items, F.pW, F.item_base,        \
                       F.item_rel, F.item_rng, KW, F.Dring, F.L, sj, c.perm, F.pslot, part, F.scn.part)
#define BIE_TB_UNROLL(KT, C, P, KW)                  \
    do {                                             \
        if (deep) BIE_TB_LAUNCH(KT, C, 16, P, KW);   \
        else BIE_TB_LAUNCH(KT, C, 8, P, KW);         \
    } while (0)
        if (F.precision == BIE_FP64) {
            if (F.near_chunk == 64) {
                if (wide) BIE_TB_UNROLL(double, 64, 2, F.Kw); else BIE_TB_UNROLL(double, 64, 1, F.Kw);
            } else if (F.near_chunk == 128) {
                if (wide) BIE_TB_UNROLL(double, 128, 2, F.Kw); else BIE_TB_UNROLL(double, 128, 1, F.Kw);
            } else {
                if (wide) BIE_TB_UNROLL(double, 256, 2, F.Kw); else BIE_TB_UNROLL(double, 256, 1, F.Kw);
            }
        } else {
            if (F.near_chunk == 64) {
                if (wide) BIE_TB_UNROLL(float, 64, 2, F.Kw32); else BIE_TB_UNROLL(float, 64, 1, F.Kw32);
            } else if (F.near_chunk == 128) {
                if (wide) BIE_TB_UNROLL(float, 128, 4, F.Kw32); else BIE_TB_UNROLL(float, 128, 2, F.Kw32);
            } else {
                if (wide) BIE_TB_UNROLL(float, 256, 4, F.Kw32); else BIE_TB_UNROLL(float, 256, 2, F.Kw32);
            }
        }
#undef BIE_TB_UNROLL
#undef BIE_TB_LAUNCH
    }
    BIE_HIP_TRY(hipGetLastError());
    return BIE_OK;
}

size_t near_lds_bytes(const FdphOp &F, bool mfma) {
    const size_t meta = TILE * TILE * (sizeof(int32_t) + sizeof(uint16_t)) + TILE * (sizeof(uint16_t) + sizeof(int32_t));
    if (mfma) {  // staged history in the windows' precision (or the wave results, if larger), unit list
        const size_t kb = F.precision == BIE_FP64 ? sizeof(double) : sizeof(float);
        const size_t dt = kb * TILE * (F.near_chunk + TIME_BLOCK), red = kb * (NEAR_THREADS / 64) * TILE * TIME_BLOCK;
        const size_t units = sizeof(uint16_t) * TILE * (F.near_chunk / (128 / kb));
        return std::max(dt, red) + meta + units + sizeof(int);
    }
    return (size_t)F.R * TILE * (F.near_chunk + (F.tb > 1 ? SUB_BLOCK : 0)) * sizeof(double) + meta;
}

// Times every near-kernel configuration (unroll 8/16, 4/3/2 workgroups per
// CU, build or XCD-grouped order; for time blocks also the matrix-core kernel
// under each occupancy cap and order) on the operator's own data and keeps
// the fastest.  An operator with time blocks has two configurations, tuned in
// turn: the time-block kernel's (bie_run, bie_run_graph; reported in out) and
// the single-step kernel's (bie_step, coupled steps).  The kernels only write
// the per-item partial sums, which the next step recomputes, so the
// operator's state is unchanged.
int fdph_autotune(bie_op_impl *op, int reps, hipStream_t s, bie_tune *out) {
    FdphOp &F = op->fdph;
    auto report = [&](const NearTune &c, bool blocks, bie_tune &r) {
        r.unroll = c.unroll;
        r.lds_pad = c.lds_pad;
        r.item_order = c.order;
        r.load_bytes = near_load_bytes(F, c);
        r.mfma = blocks ? c.mfma : 0;
    };
    bie_tune r{};
    report(F.tb > 1 ? F.tune_tb : F.tune, F.tb > 1, r);
    if (F.n_items == 0) {
        if (out) *out = r;
        return BIE_OK;
    }
    StepIdx si;
    si.n = si.n0 = F.tune_step;
    constexpr int LDS_CU = 160 * 1024;
    auto pads_of = [&](bool mfma) {
        const int base = (int)near_lds_bytes(F, mfma);
        std::vector<int> pads{0};
        for (int k : {3, 2}) {
            const int p = (LDS_CU / k - base + 1) / 256 * 256;
            if (p > 0 && p <= 64 * 1024 && LDS_CU / (base + p) == k) pads.push_back(p);
        }
        return pads;
    };
    // work-item orders: build order, grouped by source slice per XCD, largest first
    std::vector<int> orders{0};
    if (F.perm_grouped) orders.push_back(1);
    if (F.perm_size) orders.push_back(2);
    auto set_order = [&](NearTune &c, int o) {
        c.order = o;
        c.perm = o == 1 ? F.perm_grouped : o == 2 ? F.perm_size : nullptr;
        c.grid = o == 1 ? F.grid_grouped : o == 2 ? F.n_items : 0;
    };
    // the same orders of the chunk groups
    std::vector<int> gorders{0};
    if (F.gperm_grouped) gorders.push_back(1);
    if (F.gperm_size) gorders.push_back(2);
    auto set_gorder = [&](NearTune &c, int o) {
        c.order = o;
        c.perm = o == 1 ? F.gperm_grouped : o == 2 ? F.gperm_size : nullptr;
        c.grid = o == 1 ? F.ggrid_grouped : o == 2 ? F.n_grp : 0;
    };
    hipEvent_t e0, e1;
    BIE_HIP_TRY(hipEventCreate(&e0));
    BIE_HIP_TRY(hipEventCreate(&e1));
    auto tune = [&](bool blocks, NearTune &cur, bie_tune &res) -> int {
        std::vector<NearTune> cand;
        for (int w = 0; w < 2; ++w)
            for (int u : {8, 16})
                for (int p : pads_of(false))
                    for (int o : orders) {
                        NearTune c;
                        c.unroll = u;
                        c.wide = w;
                        c.lds_pad = p;
                        set_order(c, o);
                        c.mfma = 0;
                        cand.push_back(c);
                    }
        if (blocks)
            for (int p : pads_of(true)) {
                for (int o : orders) {
                    NearTune c;
                    c.lds_pad = p;
                    set_order(c, o);
                    c.mfma = 1;
                    cand.push_back(c);
                }
                if (F.n_grp > 0)
                    for (int o : gorders) {
                        NearTune c;
                        c.lds_pad = p;
                        set_gorder(c, o);
                        c.mfma = 2;
                        cand.push_back(c);
                    }
            }
        auto launch = [&](const NearTune &c) { return blocks ? launch_near_tb(F, c, s, si) : launch_near(F, c, s, si); };
        auto time = [&](const NearTune &c, double *ms) -> int {
            int rc = launch(c);  // warm-up
            if (rc) return rc;
            BIE_HIP_TRY(hipEventRecord(e0, s));
            for (int k = 0; k < reps; ++k)
                if ((rc = launch(c))) return rc;
            BIE_HIP_TRY(hipEventRecord(e1, s));
            BIE_HIP_TRY(hipEventSynchronize(e1));
            float t = 0.0f;
            BIE_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
            *ms = (double)t / reps;
            return BIE_OK;
        };
        res = bie_tune{};
        int rc = time(cur, &res.default_ms);
        res.best_ms = res.default_ms;
        NearTune best = cur;
        for (const NearTune &c : cand) {
            double ms = 0.0;
            if (rc || (rc = time(c, &ms))) break;
            res.candidates++;
            if (ms < res.best_ms) {
                res.best_ms = ms;
                best = c;
            }
        }
        if (rc) return rc;
        cur = best;
        report(best, blocks, res);
        return BIE_OK;
    };
    bie_tune r1{};
    int rc = tune(false, F.tune, r1);
    if (!rc) r = r1;
    if (!rc && F.tb > 1) rc = tune(true, F.tune_tb, r);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (out) *out = r;
    return BIE_OK;
}

namespace {

int launch_update(const FdphOp &F, const double *d, hipStream_t s, const StepIdx &si, int what, int steps = 1) {
    hipLaunchKernelGGL(k_fdph_update, dim3((F.N + 255) / 256, (unsigned)F.R), dim3(256), 0, s, d, F.Dring, F.Uring,
                       F.Drec, F.N, F.L, F.Lf, si, F.scn, what, steps);
    BIE_HIP_TRY(hipGetLastError());
    return BIE_OK;
}

// The far-field source side of one step (or only D_n's own terms of a
// committed step), then its transient FIR.
template <bool INJECT>
int launch_far_side(const FdphOp &F, hipStream_t sf, const StepIdx &si) {
    const int N = F.N;
    const unsigned R = INJECT ? 1u : (unsigned)F.R;
    if (F.n_groups > 0) {
        const dim3 g((F.n_groups + 127) / 128, R), b(128);
        if (F.precision == BIE_FP64)
            hipLaunchKernelGGL((k_far_src<double, INJECT>), g, b, 0, sf, F.groups, F.n_groups, F.gsrc, F.blocks,
                               F.gdat, F.hdat, F.Drec, N, F.Lf, si, F.rings, F.scn, F.tb);
        else if (F.precision == BIE_MIXED_FP32)
            hipLaunchKernelGGL((k_far_src<float, INJECT>), g, b, 0, sf, F.groups, F.n_groups, F.gsrc, F.blocks,
                               F.gdat32, F.hdat, F.Drec, N, F.Lf, si, F.rings, F.scn, F.tb);
        else
            hipLaunchKernelGGL((k_far_src<bf16_t, INJECT>), g, b, 0, sf, F.groups, F.n_groups, F.gsrc, F.blocks,
                               reinterpret_cast<const bf16_t *>(F.gdat16), F.hdat, F.Drec, N, F.Lf, si, F.rings,
                               F.scn, F.tb);
    }
    if (!INJECT && F.n_tr > 0) {
        const dim3 g((F.n_tr + 3) / 4, R), b(256);
        if (F.quantized)
            hipLaunchKernelGGL(k_tr_quant, g, b, 0, sf, F.tr_list, F.n_tr, F.blocks, F.qbounds, F.qrep, F.qstate,
                               F.rings, F.yrings, si, F.scn);
        else
            hipLaunchKernelGGL(k_tr_fir, g, b, 0, sf, F.tr_list, F.n_tr, F.blocks, F.htr, F.rings, F.yrings, si,
                               F.scn);
    }
    BIE_HIP_TRY(hipGetLastError());
    return BIE_OK;
}

// The far-field source side of a time block: the source inputs of all its
// steps in one pass over the waveforms, the scatter of all its steps (one
// launch, or one per step in step order), then the transient FIR (or
// staircase sums) of all its steps.
template <class StepOf>
int launch_far_side_tb(const FdphOp &F, hipStream_t sf, const StepIdx &si0, StepOf step) {
    constexpr int B = TIME_BLOCK;
    const int N = F.N;
    if (F.n_groups > 0) {
        const dim3 g((F.n_groups + 127) / 128), b(128);
        for (int j = 0; j < B; j += SUB_BLOCK)
            hipLaunchKernelGGL(k_far_fir_tb<SUB_BLOCK>, g, b, 0, sf, F.groups, F.n_groups, F.gsrc, F.blocks, F.hdat,
                               F.Drec, N, F.Lf, step(j), F.xs, F.n_gsrc, j);
        if (F.scat_tb) {
            const dim3 gs((unsigned)F.n_scat), bs(64);
            const StepIdx s0 = step(0);
            if (F.precision == BIE_FP64)
                hipLaunchKernelGGL(k_far_scat_tb<double>, gs, bs, 0, sf, F.scat, F.groups, F.gsrc, F.gdat, F.xs,
                                   F.n_gsrc, F.rings, s0);
            else if (F.precision == BIE_MIXED_FP32)
                hipLaunchKernelGGL(k_far_scat_tb<float>, gs, bs, 0, sf, F.scat, F.groups, F.gsrc, F.gdat32, F.xs,
                                   F.n_gsrc, F.rings, s0);
            else
                hipLaunchKernelGGL(k_far_scat_tb<bf16_t>, gs, bs, 0, sf, F.scat, F.groups, F.gsrc,
                                   reinterpret_cast<const bf16_t *>(F.gdat16), F.xs, F.n_gsrc, F.rings, s0);
        }
        for (int k = 0; k < B && !F.scat_tb; ++k) {
            const StepIdx sk = step(k);
            if (F.precision == BIE_FP64)
                hipLaunchKernelGGL((k_far_src<double, false, true>), g, b, 0, sf, F.groups, F.n_groups, F.gsrc,
                                   F.blocks, F.gdat, F.hdat, F.Drec, N, F.Lf, sk, F.rings, F.scn, F.tb, F.xs, k,
                                   F.n_gsrc);
            else if (F.precision == BIE_MIXED_FP32)
                hipLaunchKernelGGL((k_far_src<float, false, true>), g, b, 0, sf, F.groups, F.n_groups, F.gsrc,
                                   F.blocks, F.gdat32, F.hdat, F.Drec, N, F.Lf, sk, F.rings, F.scn, F.tb, F.xs, k,
                                   F.n_gsrc);
            else
                hipLaunchKernelGGL((k_far_src<bf16_t, false, true>), g, b, 0, sf, F.groups, F.n_groups, F.gsrc,
                                   F.blocks, reinterpret_cast<const bf16_t *>(F.gdat16), F.hdat, F.Drec, N, F.Lf, sk,
                                   F.rings, F.scn, F.tb, F.xs, k, F.n_gsrc);
        }
    }
    if (F.n_tr > 0) {
        const dim3 g((F.n_tr + 3) / 4), b(256);
        if (F.quantized)
            hipLaunchKernelGGL(k_tr_quant_tb<B>, g, b, 0, sf, F.tr_list, F.n_tr, F.blocks, F.qbounds, F.qrep,
                               F.qstate, F.rings, F.yrings, si0);
        else
            hipLaunchKernelGGL(k_tr_fir_tb<B>, g, b, 0, sf, F.tr_list, F.n_tr, F.blocks, F.htr, F.rings, F.yrings,
                               si0);
    }
    BIE_HIP_TRY(hipGetLastError());
    return BIE_OK;
}

int launch_recv(const FdphOp &F, double *t, hipStream_t s, const StepIdx &si, const double *partial) {
    const int N = F.N;
    const dim3 gr((N + 3) / 4, (unsigned)F.R), br(256);
    if (F.precision == BIE_FP64)
        hipLaunchKernelGGL(k_recv<double>, gr, br, 0, s, N, si, F.L, F.rn_ptr, partial, F.rp_ptr, F.tails, F.Uring,
                           F.re_ptr, F.re, F.fdat, F.rings, F.yrings, F.TS, F.self0, F.Dring, F.hz, t, F.scn);
    else if (F.precision == BIE_MIXED_FP32)
        hipLaunchKernelGGL(k_recv<float>, gr, br, 0, s, N, si, F.L, F.rn_ptr, partial, F.rp_ptr, F.tails, F.Uring,
                           F.re_ptr, F.re, F.fdat32, F.rings, F.yrings, F.TS, F.self0, F.Dring, F.hz, t, F.scn);
    else
        hipLaunchKernelGGL(k_recv<bf16_t>, gr, br, 0, s, N, si, F.L, F.rn_ptr, partial, F.rp_ptr, F.tails, F.Uring,
                           F.re_ptr, F.re, reinterpret_cast<const bf16_t *>(F.fdat16), F.rings, F.yrings, F.TS,
                           F.self0, F.Dring, F.hz, t, F.scn);
    BIE_HIP_TRY(hipGetLastError());
    return BIE_OK;
}

// The gathers of a time block, SUB_BLOCK steps per launch in step order (the
// Domain-S stress advances from one launch to the next).
template <class StepOf>
int launch_recv_tb(const FdphOp &F, double *t, hipStream_t s, StepOf step) {
    constexpr int B = TIME_BLOCK, SB = SUB_BLOCK;
    const int N = F.N;
    const dim3 gr((N + 3) / 4), br(256);
    // the partial sums of the near kernel's work items: chunk groups or single chunks
    const int32_t *rn = (F.tune_tb.mfma == 2 && F.n_grp > 0) ? F.rn_ptr_g : F.rn_ptr;
    for (int j = 0; j < B; j += SB) {
        const StepIdx si = step(j);
        const double *part = F.partial + (int64_t)j * F.scn.part;
        if (F.precision == BIE_FP64)
            hipLaunchKernelGGL((k_recv_tb<double, SB>), gr, br, 0, s, N, si, F.L, rn, part, F.scn.part,
                               F.rp_ptr, F.tails, F.Uring, F.re_ptr, F.re, F.fdat, F.rings, F.yrings, F.TS, F.self0,
                               F.Dring, F.hz, t, F.scn.row);
        else if (F.precision == BIE_MIXED_FP32)
            hipLaunchKernelGGL((k_recv_tb<float, SB>), gr, br, 0, s, N, si, F.L, rn, part, F.scn.part,
                               F.rp_ptr, F.tails, F.Uring, F.re_ptr, F.re, F.fdat32, F.rings, F.yrings, F.TS, F.self0,
                               F.Dring, F.hz, t, F.scn.row);
        else
            hipLaunchKernelGGL((k_recv_tb<bf16_t, SB>), gr, br, 0, s, N, si, F.L, rn, part, F.scn.part,
                               F.rp_ptr, F.tails, F.Uring, F.re_ptr, F.re, reinterpret_cast<const bf16_t *>(F.fdat16),
                               F.rings, F.yrings, F.TS, F.self0, F.Dring, F.hz, t, F.scn.row);
    }
    BIE_HIP_TRY(hipGetLastError());
    return BIE_OK;
}

}  // namespace

int fdph_step(bie_op_impl *op, const double *d, double *t, hipStream_t s, const StepIdx &si, bool advance) {
    FdphOp &F = op->fdph;
    int rc;
    if ((rc = launch_update(F, d, s, si, 3))) return rc;
    // The far-field source side and the transient FIR touch ring slots
    // disjoint from this step's gathers (discretized causality), so they run
    // on the side stream while the near field streams its windows.
    const bool side = F.side != nullptr && (F.n_groups > 0 || F.n_tr > 0);
    if (side) {
        BIE_HIP_TRY(hipEventRecord(F.ev_fork, s));
        BIE_HIP_TRY(hipStreamWaitEvent(F.side, F.ev_fork, 0));
    }
    hipStream_t sf = side ? F.side : s;
    if ((rc = launch_far_side<false>(F, sf, si))) return rc;
    if (side) BIE_HIP_TRY(hipEventRecord(F.ev_join, sf));
    if (F.n_items > 0) {
        const int tk = si.dev ? -1 : op->timer.begin(s);
        if ((rc = launch_near(F, F.tune, s, si))) return rc;
        op->timer.end(tk, s);
    }
    if (side) {
        BIE_HIP_TRY(hipStreamWaitEvent(s, F.ev_join, 0));
        F.side_pending = false;
    }
    if ((rc = launch_recv(F, t, s, si, F.partial))) return rc;
    if (op->scan_finite)
        if ((rc = launch_scan_finite(t, op->N, si, op->nonfinite, s))) return rc;
    if (si.dev) return launch_step_advance(const_cast<int64_t *>(si.dev), s);
    if (advance) op->step++;
    return BIE_OK;
}

// A time block of tb steps (prescribed slip, one scenario).  The near
// histories of all its steps are written first; the far-field source side and
// transient FIR of its steps run in step order on the caller's stream (their
// rings hold tb - 1 extra slots, so no gather of the block has been
// overwritten) while the near field of all tb steps streams the windows once
// on the second stream; then the gathers in step order.
int fdph_block(bie_op_impl *op, const double *d, double *t, hipStream_t s, const StepIdx &si0) {
    FdphOp &F = op->fdph;
    const int B = F.tb;
    auto step = [&](int b) {
        StepIdx sb = si0;
        if (sb.dev) sb.off = b;
        else sb.n = si0.n + b;
        return sb;
    };
    int rc;
    // the histories of every step of the block (the recent-history ring of the
    // far FIR and the running-sum ring hold the block's extra slots)
    if ((rc = launch_update(F, d, s, si0, 3, B))) return rc;
    const bool side = F.side != nullptr;
    // the near field of the block runs on the second stream, the far-field
    // source side on the caller's: so the near kernel's timing events are
    // followed on their stream by nothing that waits for the other
    if (side) {
        BIE_HIP_TRY(hipEventRecord(F.ev_fork, s));
        BIE_HIP_TRY(hipStreamWaitEvent(F.side, F.ev_fork, 0));
    }
    hipStream_t sn = side ? F.side : s;
    // the near field is submitted first, so that its workgroups reach the
    // compute units ahead of the far side's many small ones
    if (F.n_items > 0) {
        const int tk = si0.dev ? -1 : op->timer.begin(sn);
        if ((rc = launch_near_tb(F, F.tune_tb, sn, si0))) return rc;
        op->timer.end(tk, sn);
    }
    if (side) BIE_HIP_TRY(hipEventRecord(F.ev_join, sn));
    if ((rc = launch_far_side_tb(F, s, si0, step))) return rc;
    if (side) {
        BIE_HIP_TRY(hipStreamWaitEvent(s, F.ev_join, 0));
        F.side_pending = false;
    }
    if ((rc = launch_recv_tb(F, t, s, step))) return rc;
    if (op->scan_finite)
        for (int b = 0; b < B; ++b)
            if ((rc = launch_scan_finite(t, op->N, step(b), op->nonfinite, s))) return rc;
    if (si0.dev) return launch_step_advance(const_cast<int64_t *>(si0.dev), s, B);
    op->step += B;
    return BIE_OK;
}

// Commit of a predicted step (the prediction ran the whole step with D_n = 0):
// D_n overwrites the history slots of step n, and the far field adds D_n's
// terms to the ring slots step n scatters into (no gather of step n reads
// them: min dm_i + mbar_j >= 1 in every admissible leaf).  That scatter runs
// on the side stream, ahead of the next step's far-field work there and
// beside its near field; it reads D_n from the recent-history ring, which the
// next Lf - 1 steps leave alone.  Calls that touch the rings outside a step
// (reset, graph runs) first wait for it (fdph_join_side).
int fdph_commit(bie_op_impl *op, const double *d, hipStream_t s) {
    FdphOp &F = op->fdph;
    StepIdx si;
    si.n = si.n0 = op->step;
    int rc;
    if ((rc = launch_update(F, d, s, si, 3))) return rc;
    if (F.n_groups > 0) {
        hipStream_t sf = s;
        if (F.side) {
            BIE_HIP_TRY(hipEventRecord(F.ev_fork, s));
            BIE_HIP_TRY(hipStreamWaitEvent(F.side, F.ev_fork, 0));
            sf = F.side;
        }
        if ((rc = launch_far_side<true>(F, sf, si))) return rc;
        if (F.side) {
            BIE_HIP_TRY(hipEventRecord(F.ev_join, F.side));
            F.side_pending = true;
        }
    }
    op->step++;
    return BIE_OK;
}

// Orders stream s after side-stream work that no step has joined yet (a
// commit's far-field scatter).
int fdph_join_side(bie_op_impl *op, hipStream_t s) {
    FdphOp &F = op->fdph;
    if (F.side_pending) {
        BIE_HIP_TRY(hipStreamWaitEvent(s, F.ev_join, 0));
        F.side_pending = false;
    }
    return BIE_OK;
}

int fdph_reset(bie_op_impl *op, hipStream_t s) {
    FdphOp &F = op->fdph;
    if (int rc = fdph_join_side(op, s)) return rc;
    BIE_HIP_TRY(hipMemsetAsync(F.Dring, 0, (size_t)F.R * F.scn.D * sizeof(double), s));
    BIE_HIP_TRY(hipMemsetAsync(F.Uring, 0, (size_t)F.R * F.scn.U * sizeof(double), s));
    BIE_HIP_TRY(hipMemsetAsync(F.Drec, 0, (size_t)F.R * F.scn.Drec * sizeof(double), s));
    BIE_HIP_TRY(hipMemsetAsync(F.TS, 0, (size_t)F.R * F.N * sizeof(double), s));
    if (F.rings_bytes) BIE_HIP_TRY(hipMemsetAsync(F.rings, 0, F.rings_bytes, s));
    if (F.yrings_bytes) BIE_HIP_TRY(hipMemsetAsync(F.yrings, 0, F.yrings_bytes, s));
    if (F.qstate_bytes) BIE_HIP_TRY(hipMemsetAsync(F.qstate, 0, F.qstate_bytes, s));
    op->step = 0;
    return BIE_OK;
}

}  // namespace bie
