// C ABI of the BIEM convolution library (declarations in include/bie.h).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>

#include "bie_internal.hpp"

namespace bie {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

int KernelTimer::begin(hipStream_t s) {
    if (!enabled || used >= CAP) return -1;
    if ((int)start.size() <= used) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return -1;
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return -1;
        }
        start.push_back(a);
        stop.push_back(b);
    }
    if (hipEventRecord(start[used], s) != hipSuccess) return -1;
    return used++;
}

void KernelTimer::end(int k, hipStream_t s) {
    if (k >= 0) (void)hipEventRecord(stop[k], s);
}

void KernelTimer::release() {
    for (auto e : start) (void)hipEventDestroy(e);
    for (auto e : stop) (void)hipEventDestroy(e);
    start.clear();
    stop.clear();
    used = 0;
    enabled = false;
}

int plan_dense(const bie_problem *p, bie_plan_impl *pl) {
    DensePlan &D = pl->dense;
    int rc = D.g.build(p);
    if (rc) return rc;
    D.N = D.g.N;
    D.M = p->n_lags;
    D.ncomp = D.g.mode == BIE_MODE_INPLANE ? 2 : 1;
    D.L = 1;
    while (D.L < D.M) D.L <<= 1;
    // lag chunks: enough waves to fill the chip even for small N
    D.n_chunks = (int)std::min<int64_t>(D.M, std::max<int64_t>(1, (32768 + D.N - 1) / D.N));
    D.lag_chunk = (D.M + D.n_chunks - 1) / D.n_chunks;
    D.n_chunks = (D.M + D.lag_chunk - 1) / D.lag_chunk;
    if ((int64_t)D.N * D.N > MAX_DISPATCH_ITEMS || (int64_t)D.L * D.N > MAX_DISPATCH_ITEMS) {
        set_error("problem too large for the plain form (N^2 or the history exceeds one dispatch)");
        return BIE_EINVAL;
    }
    // Causal band (Eq. 4 skips nothing else): S_ij(t) is zero until the
    // fastest wave (beta anti-plane, alpha in-plane) has covered the distance
    // d_ij from x_i to the nearest point of element j, so K_ij,m = 0 unless
    // c (m + eps_t) dt > d_ij.  The first such lag, less one against rounding,
    // enters j into the bands of receiver i from that lag on; each band is
    // the hull of its sources (rounded out to even indices for 16-byte loads
    // when N is even).
    const Geometry &g = D.g;
    const double c = g.mode == BIE_MODE_INPLANE ? g.alpha : g.beta;
    const int N = D.N, M = D.M;
    D.V = N % 2 == 0 ? 2 : 1;
    D.blo.assign((size_t)M * N, 0);
    std::vector<int32_t> width((size_t)M * N, 0);
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < N; ++i) {
        std::vector<int32_t> alo(M, N), ahi(M, 0);
        for (int j = 0; j < N; ++j) {
            const Frame &f = g.fr[j];
            const double px = g.fr[i].cx - f.cx, py = g.fr[i].cy - f.cy;
            const double X = px * f.tx + py * f.ty, Y = px * f.nx + py * f.ny;
            const double ex = std::max(std::fabs(X) - f.h, 0.0);
            const double d = std::sqrt(ex * ex + Y * Y);
            const double v = d / (c * g.dt) - g.eps_t;
            int64_t m0 = v < 0.0 ? 0 : (int64_t)std::floor(v) + 1;
            m0 = std::max<int64_t>(0, m0 - 1);
            if (m0 >= M) continue;
            alo[m0] = std::min(alo[m0], j);
            ahi[m0] = std::max(ahi[m0], j + 1);
        }
        int lo = N, hi = 0;
        for (int m = 0; m < M; ++m) {
            lo = std::min(lo, alo[m]);
            hi = std::max(hi, ahi[m]);
            int a = lo, b = hi;
            if (b <= a) a = b = 0;
            if (D.V == 2) {
                a &= ~1;
                b = std::min(N, (b + 1) & ~1);
            }
            D.blo[(size_t)m * N + i] = a;
            width[(size_t)m * N + i] = b - a;
        }
    }
    D.off.assign((size_t)M * N + 1, 0);
    for (size_t k = 0; k < (size_t)M * N; ++k) D.off[k + 1] = D.off[k] + width[k];
    pl->kind = BIE_KIND_DENSE;
    return BIE_OK;
}

bie_stats dense_stats(const DensePlan &D) {
    bie_stats st{};
    st.kind = BIE_KIND_DENSE;
    st.n_elem = D.N;
    st.n_lags = D.M;
    st.precision = BIE_FP64;
    // steady state (n >= M-1): every band entry of every lag (read once per
    // step), the history row of every lag (N values, shared by the receivers
    // of that lag: cache-resident after its first read), and the band's row
    // offset and first source
    const double E = (double)D.off.back();
    st.bytes_per_step = D.ncomp * (E * 8.0 + (double)D.M * D.N * 8.0) + (double)D.M * D.N * 12.0;
    st.near_bytes_per_step = 0.0;
    st.flops_per_step = D.ncomp * 2.0 * E;
    st.scratch_bytes = (int64_t)D.ncomp * D.n_chunks * D.N * (int64_t)sizeof(double);
    st.time_block = 1;
    return st;
}

int materialize_dense(const DensePlan &P, DevArena &A, hipStream_t s, bie_op_impl *op) {
    const auto t0 = std::chrono::steady_clock::now();
    DenseOp &D = op->dense;
    D.N = P.N;
    D.M = P.M;
    D.ncomp = P.ncomp;
    D.L = P.L;
    D.n_chunks = P.n_chunks;
    D.lag_chunk = P.lag_chunk;
    D.V = P.V;
    D.E = P.off.back();
    const size_t row = (size_t)D.N * D.ncomp;
    int rc;
    if ((rc = A.upload(&D.dfr, P.g.fr, s))) return rc;
    if ((rc = A.upload(&D.off, P.off, s))) return rc;
    if ((rc = A.upload(&D.blo, P.blo, s))) return rc;
    if ((rc = A.alloc(&D.K, (size_t)D.ncomp * D.E))) return rc;
    if ((rc = A.alloc(&D.hist, (size_t)D.ncomp * D.L * D.N))) return rc;
    if ((rc = A.alloc(&D.partial, (size_t)D.ncomp * D.n_chunks * D.N))) return rc;
    if ((rc = A.alloc(&op->zero_in, row))) return rc;
    if ((rc = A.alloc(&op->scratch_out, row))) return rc;
    if ((rc = A.alloc(&op->step_dev, 1))) return rc;
    if ((rc = A.alloc(&op->k0, row))) return rc;
    if ((rc = A.alloc(&op->nonfinite, 1))) return rc;
    if (A.dry) return BIE_OK;
    if ((rc = launch_dense_build(P.g, D, s))) return rc;
    if ((rc = dense_reset(op, s))) return rc;
    BIE_HIP_TRY(hipMemsetAsync(op->zero_in, 0, row * sizeof(double), s));
    BIE_HIP_TRY(hipStreamSynchronize(s));
    op->kind = BIE_KIND_DENSE;
    op->N = (int)row;  // values per step row of D and T
    op->M = D.M;
    op->mode = P.g.mode;
    op->dt = P.g.dt;
    op->first_lag_diag = P.g.first_lag_diagonal();
    op->stats = dense_stats(P);
    op->stats.device_bytes = (int64_t)A.bytes();
    op->stats.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return BIE_OK;
}

// Bytes of the workspace of a plan's operator (a sizing pass of its build).
int workspace_bytes(const bie_plan_impl *pl, size_t *bytes) {
    DevArena A;  // dry
    bie_op_impl tmp;
    int rc = BIE_OK;
    if (pl->kind == BIE_KIND_DENSE) {
        rc = materialize_dense(pl->dense, A, nullptr, &tmp);
    } else if (pl->kind == BIE_KIND_FDPH) {
        if (!pl->fdph.windows) {
            set_error("the FDP=H plan's windows are not scanned yet (bie_plan_windows)");
            return BIE_ESTATE;
        }
        rc = materialize_fdph(pl->fdph, A, nullptr, &tmp);
    } else {
        set_error("plan not built");
        return BIE_ESTATE;
    }
    *bytes = A.bytes();
    return rc;
}

// An FDP=H operator's runs end at the largest lag count of its problems (a
// problem's tractions are zero from its own lag count on): later steps are
// refused rather than silently zero.
int fdph_steps_ok(const bie_op_impl *op, int64_t steps, const char *who) {
    if (steps > (int64_t)op->M - op->step) {
        set_error(std::string(who) + ": the FDP=H operator's runs end at step " + std::to_string(op->M) +
                  " (its lag count); it is at step " + std::to_string(op->step) + " and was asked for " +
                  std::to_string(steps) + " more (bie_reset starts over)");
        return BIE_EINVAL;
    }
    return BIE_OK;
}

// Preconditions of the coupled step (predict / commit / rupture runs).
static int coupled_ok(const bie_op_impl *op, const char *who) {
    if (op->kind != BIE_KIND_DENSE && op->kind != BIE_KIND_FDPH) {
        set_error(std::string(who) + ": operator not built");
        return BIE_ESTATE;
    }
    if (op->mode != BIE_MODE_ANTIPLANE) {
        set_error(std::string(who) + ": the coupled step is for the anti-plane mode");
        return BIE_EINVAL;
    }
    if (op->kind == BIE_KIND_FDPH && op->fdph.R > 1) {
        set_error(std::string(who) + ": the coupled step is for an operator of one scenario (n_rhs = 1)");
        return BIE_EINVAL;
    }
    if (!op->first_lag_diag) {
        set_error(std::string(who) + ": the first lag couples different elements (a collocation point lies within "
                                     "beta eps_t dt of another element); reduce dt");
        return BIE_EINVAL;
    }
    return BIE_OK;
}

// ---- saved state (checkpoint / resume) -------------------------------------
struct StateSeg {
    void *p;
    size_t bytes;
};

// The arrays a step reads that earlier steps wrote, in a fixed order.
static std::vector<StateSeg> state_segments(const bie_op_impl *op) {
    std::vector<StateSeg> v;
    if (op->kind == BIE_KIND_DENSE) {
        const DenseOp &D = op->dense;
        v.push_back({D.hist, (size_t)D.ncomp * D.L * D.N * sizeof(double)});
    } else if (op->kind == BIE_KIND_FDPH) {
        const FdphOp &F = op->fdph;
        const size_t hb = (size_t)F.R * F.scn.D * sizeof(double);
        v.push_back({F.Dring, hb});
        v.push_back({F.Uring, (size_t)F.R * F.scn.U * sizeof(double)});
        v.push_back({F.Drec, (size_t)F.R * F.scn.Drec * sizeof(double)});
        v.push_back({F.TS, (size_t)F.R * F.N * sizeof(double)});
        if (F.rings_bytes) v.push_back({F.rings, F.rings_bytes});
        if (F.yrings_bytes) v.push_back({F.yrings, F.yrings_bytes});
        if (F.qstate_bytes) v.push_back({F.qstate, F.qstate_bytes});
    }
    return v;
}

static constexpr size_t STATE_ALIGN = 256;
static constexpr uint64_t STATE_MAGIC = 0x3154415453454942ull;  // "BIESTAT1"

struct StateHeader {
    uint64_t magic;
    int32_t kind, n_seg;
    int64_t n_values, n_lags, step, total_bytes;
    uint64_t fingerprint;
};
static_assert(sizeof(StateHeader) <= STATE_ALIGN, "the header fits its slot");

static size_t state_align(size_t x) { return (x + STATE_ALIGN - 1) & ~(STATE_ALIGN - 1); }

static int64_t state_total(const std::vector<StateSeg> &segs) {
    size_t t = STATE_ALIGN;
    for (const StateSeg &g : segs) t += state_align(g.bytes);
    return (int64_t)t;
}

// FNV-1a over the operator's shape and setup statistics: a state saved from
// an operator built otherwise is refused.
static uint64_t state_fingerprint(const bie_op_impl *op, const std::vector<StateSeg> &segs) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](int64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (uint64_t)((v >> (8 * b)) & 0xFF);
            h *= 1099511628211ull;
        }
    };
    const bie_stats &st = op->stats;
    mix(op->kind);
    mix(op->N);
    mix(op->M);
    mix(op->mode);
    mix(op->kind == BIE_KIND_FDPH ? op->fdph.R : 1);
    mix(st.n_elem);
    mix(st.n_lags);
    mix(st.precision);
    mix(st.n_adm);
    mix(st.n_inadm);
    mix(st.near_pairs);
    mix(st.near_lags);
    for (int k = 0; k < 3; ++k) {
        mix(st.rank_sum[k]);
        mix(st.rank_max[k]);
    }
    for (const StateSeg &g : segs) mix((int64_t)g.bytes);
    return h;
}

static int state_call_ok(const bie_op_impl *op, const void *buf, int64_t capacity, const char *who,
                         std::vector<StateSeg> &segs, int64_t &total) {
    if (!op || !buf) {
        set_error(std::string(who) + ": null operator or buffer");
        return BIE_EINVAL;
    }
    if (op->kind != BIE_KIND_DENSE && op->kind != BIE_KIND_FDPH) {
        set_error(std::string(who) + ": operator not built");
        return BIE_ESTATE;
    }
    if (op->predicted) {
        set_error(std::string(who) + ": the current step was predicted; commit it first");
        return BIE_ESTATE;
    }
    if ((uintptr_t)buf % STATE_ALIGN) {
        set_error(std::string(who) + ": the state buffer must be 256-byte aligned");
        return BIE_EINVAL;
    }
    segs = state_segments(op);
    total = state_total(segs);
    if (capacity < total) {
        set_error(std::string(who) + ": buffer of " + std::to_string(capacity) + " bytes, the state needs " +
                  std::to_string(total));
        return BIE_EINVAL;
    }
    return BIE_OK;
}

}  // namespace bie

using bie::set_error;

#define BIE_GUARD(...)                                               \
    try {                                                            \
        __VA_ARGS__                                                  \
    } catch (const std::bad_alloc &) {                               \
        set_error("host allocation failed");                         \
        return BIE_ENOMEM;                                           \
    } catch (const std::exception &e) {                              \
        set_error(std::string("internal error: ") + e.what());      \
        return BIE_EINVAL;                                           \
    } catch (...) {                                                  \
        set_error("internal error");                                 \
        return BIE_EINVAL;                                           \
    }

extern "C" {

const char *bie_last_error(void) { return bie::g_err.c_str(); }

int bie_plan_dense(const bie_problem *prob, bie_plan **plan_out) {
    BIE_GUARD({
        if (!plan_out) {
            set_error("bie_plan_dense: null output pointer");
            return BIE_EINVAL;
        }
        *plan_out = nullptr;
        bie_plan *pl = new bie_plan();
        const int rc = bie::plan_dense(prob, pl);
        if (rc) {
            delete pl;
            return rc;
        }
        *plan_out = pl;
        bie::set_error("");
        return BIE_OK;
    })
}

int bie_plan_fdph(const bie_problem *probs, int32_t count, const bie_fdph_params *params, bie_plan **plan_out) {
    BIE_GUARD({
        if (!plan_out || count < 1) {
            set_error("bie_plan_fdph: null output pointer or count below 1");
            return BIE_EINVAL;
        }
        *plan_out = nullptr;
        bie_plan *pl = new bie_plan();
        const int rc = bie::plan_fdph(probs, count, params, pl);
        if (rc) {
            delete pl;
            return rc;
        }
        *plan_out = pl;
        bie::set_error("");
        return BIE_OK;
    })
}

int bie_plan_scratch_size(const bie_plan *plan, int64_t *bytes_out) {
    BIE_GUARD({
        if (!plan || !bytes_out) {
            set_error("bie_plan_scratch_size: null pointer");
            return BIE_EINVAL;
        }
        *bytes_out = plan->kind == BIE_KIND_FDPH ? (int64_t)bie::plan_scratch_bytes(plan->fdph) : 0;
        return BIE_OK;
    })
}

int bie_plan_windows(bie_plan *plan, void *scratch_dev, int64_t scratch_bytes, void *stream) {
    BIE_GUARD({
        if (!plan || scratch_bytes < 0) {
            set_error("bie_plan_windows: null plan or negative size");
            return BIE_EINVAL;
        }
        if (plan->kind != BIE_KIND_FDPH) return BIE_OK;  // the plain form has no windows
        return bie::plan_windows(plan->fdph, scratch_dev, (size_t)scratch_bytes, (hipStream_t)stream);
    })
}

int bie_workspace_size(const bie_plan *plan, int64_t *bytes_out) {
    BIE_GUARD({
        if (!plan || !bytes_out) {
            set_error("bie_workspace_size: null pointer");
            return BIE_EINVAL;
        }
        size_t b = 0;
        if (int rc = bie::workspace_bytes(plan, &b)) return rc;
        *bytes_out = (int64_t)b;
        return BIE_OK;
    })
}

int bie_plan_query(const bie_plan *plan, bie_stats *stats_out) {
    BIE_GUARD({
        if (!plan || !stats_out) {
            set_error("bie_plan_query: null pointer");
            return BIE_EINVAL;
        }
        size_t b = 0;
        if (int rc = bie::workspace_bytes(plan, &b)) return rc;
        *stats_out = plan->kind == BIE_KIND_DENSE ? bie::dense_stats(plan->dense) : plan->fdph.stats;
        stats_out->device_bytes = (int64_t)b;
        stats_out->steps_done = 0;
        if (plan->kind == BIE_KIND_FDPH) stats_out->setup_seconds = plan->fdph.plan_seconds;
        return BIE_OK;
    })
}

void bie_plan_free(bie_plan *plan) { delete plan; }

// Builds an operator of a plan inside the caller's workspace; on failure the
// partly built operator's host resources are released.
static int build_in_workspace(const bie_plan *plan, int kind, void *ws, int64_t ws_bytes, void *stream,
                              bie_op **op_out, const char *who) {
    if (!op_out || !plan) {
        set_error(std::string(who) + ": null plan or output pointer");
        return BIE_EINVAL;
    }
    *op_out = nullptr;
    if (plan->kind != kind) {
        set_error(std::string(who) + (kind == BIE_KIND_DENSE ? ": not a plain-form plan" : ": not an FDP=H plan"));
        return BIE_EINVAL;
    }
    if (kind == BIE_KIND_FDPH && !plan->fdph.windows) {
        set_error(std::string(who) + ": the plan's windows are not scanned yet (bie_plan_windows)");
        return BIE_ESTATE;
    }
    if (!ws || ws_bytes <= 0 || (uintptr_t)ws % bie::WS_ALIGN) {
        set_error(std::string(who) + ": the workspace must be a non-null, 256-byte aligned device pointer");
        return BIE_EWORKSPACE;
    }
    size_t need = 0;
    if (int rc = bie::workspace_bytes(plan, &need)) return rc;
    if ((size_t)ws_bytes < need) {
        set_error(std::string(who) + ": workspace of " + std::to_string(ws_bytes) + " bytes, the operator needs " +
                  std::to_string(need));
        return BIE_EWORKSPACE;
    }
    bie_op *op = new bie_op();
    op->arena = bie::DevArena(ws, (size_t)ws_bytes);
    const int rc = kind == BIE_KIND_DENSE ? bie::materialize_dense(plan->dense, op->arena, (hipStream_t)stream, op)
                                          : bie::materialize_fdph(plan->fdph, op->arena, (hipStream_t)stream, op);
    if (rc) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        if (op->fdph.side) (void)hipStreamDestroy(op->fdph.side);
        if (op->fdph.ev_fork) (void)hipEventDestroy(op->fdph.ev_fork);
        if (op->fdph.ev_join) (void)hipEventDestroy(op->fdph.ev_join);
        delete op;
        return rc;
    }
    *op_out = op;
    bie::set_error("");
    return BIE_OK;
}

int bie_build_kernel(const bie_plan *plan, void *ws_dev, int64_t ws_bytes, void *stream, bie_op **op_out) {
    BIE_GUARD({ return build_in_workspace(plan, BIE_KIND_DENSE, ws_dev, ws_bytes, stream, op_out, "bie_build_kernel"); })
}

int bie_compress_fdph(const bie_plan *plan, void *ws_dev, int64_t ws_bytes, void *stream, bie_op **op_out) {
    BIE_GUARD({ return build_in_workspace(plan, BIE_KIND_FDPH, ws_dev, ws_bytes, stream, op_out, "bie_compress_fdph"); })
}

int bie_step(bie_op *op, const double *d_n_dev, double *t_n_dev, void *stream) {
    BIE_GUARD({
        if (!op || !d_n_dev || !t_n_dev) {
            set_error("bie_step: null operator or buffer");
            return BIE_EINVAL;
        }
        if (op->predicted) {
            set_error("bie_step: the current step was predicted; commit it first");
            return BIE_ESTATE;
        }
        hipStream_t s = (hipStream_t)stream;
        bie::StepIdx si;
        si.n = si.n0 = op->step;
        if (op->kind == BIE_KIND_DENSE) return bie::dense_step(op, d_n_dev, t_n_dev, s, si);
        if (op->kind == BIE_KIND_FDPH) {
            if (int rc = bie::fdph_steps_ok(op, 1, "bie_step")) return rc;
            return bie::fdph_step(op, d_n_dev, t_n_dev, s, si);
        }
        set_error("bie_step: operator not built");
        return BIE_ESTATE;
    })
}

int bie_run(bie_op *op, const double *D_dev, double *T_dev, int64_t steps, void *stream) {
    BIE_GUARD({
        if (!op || (steps > 0 && (!D_dev || !T_dev)) || steps < 0) {
            set_error("bie_run: null operator or buffer, or negative step count");
            return BIE_EINVAL;
        }
        if (op->kind == BIE_KIND_FDPH)
            if (int rc = bie::fdph_steps_ok(op, steps, "bie_run")) return rc;
        const int64_t N = op->N;
        int64_t k = 0;
        if (op->kind == BIE_KIND_FDPH && op->fdph.tb > 1) {
            if (op->predicted) {
                set_error("bie_run: the current step was predicted; commit it first");
                return BIE_ESTATE;
            }
            // whole time blocks: the near field of tb steps per pass over the windows
            const int64_t B = op->fdph.tb;
            for (; k + B <= steps; k += B) {
                bie::StepIdx si;
                si.n = si.n0 = op->step;
                if (int rc = bie::fdph_block(op, D_dev + k * N, T_dev + k * N, (hipStream_t)stream, si)) return rc;
            }
        }
        for (; k < steps; ++k) {
            int rc = bie_step(op, D_dev + k * N, T_dev + k * N, stream);
            if (rc) return rc;
        }
        return BIE_OK;
    })
}

int bie_run_static(bie_op *op, const double *D_dev, double *T_dev, int64_t steps, void *stream) {
    BIE_GUARD({
        if (!op || (steps > 0 && (!D_dev || !T_dev)) || steps < 0) {
            set_error("bie_run_static: null operator or buffer, or negative step count");
            return BIE_EINVAL;
        }
        if (op->kind != BIE_KIND_DENSE && op->kind != BIE_KIND_FDPH) {
            set_error("bie_run_static: operator not built");
            return BIE_ESTATE;
        }
        if (op->predicted) {
            set_error("bie_run_static: the current step was predicted; commit it first");
            return BIE_ESTATE;
        }
        // the per-step partial sums the step kernels write and read back
        double **slot = op->kind == BIE_KIND_DENSE ? &op->dense.partial : &op->fdph.partial;
        const size_t need = op->kind == BIE_KIND_DENSE
                                ? (size_t)op->dense.ncomp * op->dense.n_chunks * op->dense.N * sizeof(double)
                                : (size_t)op->fdph.R * op->fdph.scn.part * sizeof(double);
        if (need > (size_t)BIE_STATIC_SCRATCH_BYTES) {
            set_error("bie_run_static: the operator's per-step partial sums need " + std::to_string(need) +
                      " bytes, above the static scratch of " + std::to_string((long long)BIE_STATIC_SCRATCH_BYTES) +
                      " bytes; use bie_run");
            return BIE_EINVAL;
        }
        if (op->kind == BIE_KIND_FDPH)
            if (int rc = bie::fdph_steps_ok(op, steps, "bie_run_static")) return rc;
        double *ptr = nullptr;
        if (int rc = bie::static_scratch_ptr(&ptr)) return rc;
        double *own = *slot;
        *slot = ptr;  // the step kernels take it as they take the workspace's buffer
        int rc = BIE_OK;
        const int64_t N = op->N;
        for (int64_t k = 0; k < steps && !rc; ++k) rc = bie_step(op, D_dev + k * N, T_dev + k * N, stream);
        *slot = own;
        return rc;
    })
}

// Steps per captured graph: one graph launch then covers several steps, so
// its launch cost is shared (a step of a small operator is a few microseconds).
static constexpr int64_t GRAPH_STEPS = 32;

int bie_run_graph(bie_op *op, const double *D_dev, double *T_dev, int64_t steps, void *stream) {
    BIE_GUARD({
        if (!op || (steps > 0 && (!D_dev || !T_dev)) || steps < 0) {
            set_error("bie_run_graph: null operator or buffer, or negative step count");
            return BIE_EINVAL;
        }
        if (op->kind != BIE_KIND_DENSE && op->kind != BIE_KIND_FDPH) {
            set_error("bie_run_graph: operator not built");
            return BIE_ESTATE;
        }
        if (op->predicted) {
            set_error("bie_run_graph: the current step was predicted; commit it first");
            return BIE_ESTATE;
        }
        if (steps == 0) return BIE_OK;
        hipStream_t s = (hipStream_t)stream;
        if (op->kind == BIE_KIND_FDPH) {
            if (int rc = bie::fdph_steps_ok(op, steps, "bie_run_graph")) return rc;
            // a graph's far-field nodes must follow a commit's pending scatter
            if (int rc = bie::fdph_join_side(op, s)) return rc;
        }
        const int64_t G = std::min<int64_t>(steps, GRAPH_STEPS);
        const int64_t launches = steps / G;
        const int64_t rest = steps % G;
        const int64_t n0 = op->step;
        int rc = bie::launch_step_set(op->step_dev, n0, s);
        if (rc) return rc;
        // the same buffers, first step and graph length as the cached graph: replay it
        const bool cached = op->graph_exec && op->graph_D == D_dev && op->graph_T == T_dev &&
                            op->graph_n0 == n0 && op->graph_steps == G;
        if (!cached) {
            // the previous call's graph may still run: wait for it before replacing it
            if (op->graph_exec) {
                BIE_HIP_TRY(hipStreamSynchronize(op->graph_stream));
                (void)hipGraphExecDestroy(op->graph_exec);
                op->graph_exec = nullptr;
            }
            bie::StepIdx si;
            si.dev = op->step_dev;
            si.n0 = n0;
            // capture on a stream of the operator's own (the caller's may be the
            // null stream, which cannot capture); the graph runs on the caller's
            if (!op->cap_stream) BIE_HIP_TRY(hipStreamCreateWithFlags(&op->cap_stream, hipStreamNonBlocking));
            hipStream_t c = op->cap_stream;
            BIE_HIP_TRY(hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal));
            // FDP=H with time blocks: whole blocks, then single steps
            const int64_t B = op->kind == BIE_KIND_FDPH ? op->fdph.tb : 1;
            int64_t k = 0;
            if (B > 1)
                for (; k + B <= G && !rc; k += B) rc = bie::fdph_block(op, D_dev, T_dev, c, si);
            for (; k < G && !rc; ++k)
                rc = op->kind == BIE_KIND_DENSE ? bie::dense_step(op, D_dev, T_dev, c, si)
                                                : bie::fdph_step(op, D_dev, T_dev, c, si);
            hipGraph_t graph = nullptr;
            const hipError_t ec = hipStreamEndCapture(c, &graph);
            if (rc) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (ec != hipSuccess) {
                set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
                return BIE_EHIP;
            }
            hipGraphExec_t exec = nullptr;
            const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess) {
                set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
                return BIE_EHIP;
            }
            op->graph_exec = exec;
            op->graph_D = D_dev;
            op->graph_T = T_dev;
            op->graph_n0 = n0;
            op->graph_steps = G;
        }
        op->graph_stream = s;
        for (int64_t k = 0; k < launches; ++k) BIE_HIP_TRY(hipGraphLaunch(op->graph_exec, s));
        op->step = n0 + launches * G;
        // the remaining steps (fewer than one graph's worth) run as eager
        // launches, in whole time blocks where they hold any (as bie_run)
        const int64_t r = launches * G, N = op->N;
        return rest ? bie_run(op, D_dev + r * N, T_dev + r * N, rest, stream) : BIE_OK;
    })
}

int bie_autotune(bie_op *op, int32_t reps, bie_tune *out, void *stream) {
    BIE_GUARD({
        if (!op || op->kind != BIE_KIND_FDPH || reps < 1) {
            set_error("bie_autotune: needs an FDP=H operator and reps >= 1");
            return BIE_EINVAL;
        }
        // a captured graph has the previous launch configuration baked in
        if (op->graph_exec) {
            BIE_HIP_TRY(hipStreamSynchronize(op->graph_stream));
            (void)hipGraphExecDestroy(op->graph_exec);
            op->graph_exec = nullptr;
        }
        return bie::fdph_autotune(op, reps, (hipStream_t)stream, out);
    })
}

int bie_advance(bie_op *op, int64_t steps, void *stream) {
    BIE_GUARD({
        if (!op || steps < 0) {
            set_error("bie_advance: null operator or negative step count");
            return BIE_EINVAL;
        }
        if (op->predicted) {
            set_error("bie_advance: the current step was predicted; commit it first");
            return BIE_ESTATE;
        }
        hipStream_t s = (hipStream_t)stream;
        if (op->kind == BIE_KIND_DENSE) return bie::dense_advance(op, steps, s);
        if (op->kind != BIE_KIND_FDPH) {
            set_error("bie_advance: operator not built");
            return BIE_ESTATE;
        }
        if (int rc = bie::fdph_steps_ok(op, steps, "bie_advance")) return rc;
        int64_t k = 0;
        if (op->fdph.tb > 1)  // whole time blocks of zero rows
            for (; k + op->fdph.tb <= steps; k += op->fdph.tb) {
                bie::StepIdx si;
                si.n = si.n0 = op->step;
                if (int rc = bie::fdph_block(op, op->zero_in, op->scratch_out, s, si)) return rc;
            }
        for (; k < steps; ++k) {
            bie::StepIdx si;
            si.n = si.n0 = op->step;
            int rc = bie::fdph_step(op, op->zero_in, op->scratch_out, s, si);
            if (rc) return rc;
        }
        return BIE_OK;
    })
}

int bie_reset(bie_op *op, void *stream) {
    BIE_GUARD({
        if (!op) {
            set_error("bie_reset: null operator");
            return BIE_EINVAL;
        }
        hipStream_t s = (hipStream_t)stream;
        op->predicted = false;
        if (op->kind == BIE_KIND_DENSE) return bie::dense_reset(op, s);
        if (op->kind == BIE_KIND_FDPH) return bie::fdph_reset(op, s);
        set_error("bie_reset: operator not built");
        return BIE_ESTATE;
    })
}

int bie_query(const bie_op *op, bie_stats *out) {
    BIE_GUARD({
        if (!op || !out) {
            set_error("bie_query: null pointer");
            return BIE_EINVAL;
        }
        *out = op->stats;
        out->steps_done = op->step;
        return BIE_OK;
    })
}

int bie_state_bytes(const bie_op *op, int64_t *bytes_out) {
    BIE_GUARD({
        if (!op || !bytes_out) {
            set_error("bie_state_bytes: null pointer");
            return BIE_EINVAL;
        }
        if (op->kind != BIE_KIND_DENSE && op->kind != BIE_KIND_FDPH) {
            set_error("bie_state_bytes: operator not built");
            return BIE_ESTATE;
        }
        *bytes_out = bie::state_total(bie::state_segments(op));
        return BIE_OK;
    })
}

int bie_save_state(bie_op *op, void *dst_dev, int64_t capacity, void *stream) {
    BIE_GUARD({
        std::vector<bie::StateSeg> segs;
        int64_t total = 0;
        if (int rc = bie::state_call_ok(op, dst_dev, capacity, "bie_save_state", segs, total)) return rc;
        hipStream_t s = (hipStream_t)stream;
        if (op->kind == BIE_KIND_FDPH) {
            // a commit's far-field scatter may still run on the side stream
            if (int rc = bie::fdph_join_side(op, s)) return rc;
        }
        bie::StateHeader h{};
        h.magic = bie::STATE_MAGIC;
        h.kind = op->kind;
        h.n_seg = (int32_t)segs.size();
        h.n_values = op->N;
        h.n_lags = op->M;
        h.step = op->step;
        h.total_bytes = total;
        h.fingerprint = bie::state_fingerprint(op, segs);
        char *dst = static_cast<char *>(dst_dev);
        BIE_HIP_TRY(hipMemcpyAsync(dst, &h, sizeof(h), hipMemcpyHostToDevice, s));
        size_t off = bie::STATE_ALIGN;
        for (const bie::StateSeg &g : segs) {
            BIE_HIP_TRY(hipMemcpyAsync(dst + off, g.p, g.bytes, hipMemcpyDeviceToDevice, s));
            off += bie::state_align(g.bytes);
        }
        BIE_HIP_TRY(hipStreamSynchronize(s));  // the header copy reads host memory of this frame
        return BIE_OK;
    })
}

int bie_load_state(bie_op *op, const void *src_dev, int64_t capacity, void *stream) {
    BIE_GUARD({
        std::vector<bie::StateSeg> segs;
        int64_t total = 0;
        if (int rc = bie::state_call_ok(op, src_dev, capacity, "bie_load_state", segs, total)) return rc;
        hipStream_t s = (hipStream_t)stream;
        if (op->kind == BIE_KIND_FDPH) {
            if (int rc = bie::fdph_join_side(op, s)) return rc;
        }
        bie::StateHeader h{};
        const char *src = static_cast<const char *>(src_dev);
        BIE_HIP_TRY(hipMemcpyAsync(&h, src, sizeof(h), hipMemcpyDeviceToHost, s));
        BIE_HIP_TRY(hipStreamSynchronize(s));
        if (h.magic != bie::STATE_MAGIC) {
            set_error("bie_load_state: the buffer holds no saved state");
            return BIE_EINVAL;
        }
        if (h.kind != op->kind || h.n_values != op->N || h.n_lags != op->M || h.n_seg != (int32_t)segs.size() ||
            h.total_bytes != total || h.fingerprint != bie::state_fingerprint(op, segs)) {
            set_error("bie_load_state: the state was saved from an operator of another shape or setup");
            return BIE_EINVAL;
        }
        if (h.step < 0) {
            set_error("bie_load_state: corrupt header (negative step)");
            return BIE_EINVAL;
        }
        size_t off = bie::STATE_ALIGN;
        for (const bie::StateSeg &g : segs) {
            BIE_HIP_TRY(hipMemcpyAsync(g.p, src + off, g.bytes, hipMemcpyDeviceToDevice, s));
            off += bie::state_align(g.bytes);
        }
        BIE_HIP_TRY(hipStreamSynchronize(s));
        op->step = h.step;
        op->predicted = false;
        return BIE_OK;
    })
}

int bie_fdph_export(const bie_op *op, int32_t what, int64_t *buf_host, int64_t capacity, int64_t *rows_out) {
    BIE_GUARD({
        if (!op || op->kind != BIE_KIND_FDPH) {
            set_error("bie_fdph_export: not an FDP=H operator");
            return BIE_EINVAL;
        }
        return bie::export_fdph(op, what, buf_host, capacity, rows_out);
    })
}

int bie_timing(bie_op *op, int32_t enable) {
    BIE_GUARD({
        if (!op) {
            set_error("bie_timing: null operator");
            return BIE_EINVAL;
        }
        op->timer.enabled = enable != 0;
        op->timer.used = 0;
        return BIE_OK;
    })
}

int bie_timing_read(const bie_op *op, double *ms_total_out, int64_t *launches_out) {
    BIE_GUARD({
        if (!op || !ms_total_out || !launches_out) {
            set_error("bie_timing_read: null pointer");
            return BIE_EINVAL;
        }
        const bie::KernelTimer &T = op->timer;
        double tot = 0.0;
        if (T.used > 0) BIE_HIP_TRY(hipEventSynchronize(T.stop[T.used - 1]));
        for (int k = 0; k < T.used; ++k) {
            float ms = 0.0f;
            BIE_HIP_TRY(hipEventElapsedTime(&ms, T.start[k], T.stop[k]));
            tot += ms;
        }
        *ms_total_out = tot;
        *launches_out = T.used;
        return BIE_OK;
    })
}

void bie_destroy(bie_op *op) {
    if (!op) return;
    (void)hipDeviceSynchronize();
    if (op->graph_exec) (void)hipGraphExecDestroy(op->graph_exec);
    if (op->cap_stream) (void)hipStreamDestroy(op->cap_stream);
    op->timer.release();
    if (op->fdph.side) (void)hipStreamDestroy(op->fdph.side);
    if (op->fdph.ev_fork) (void)hipEventDestroy(op->fdph.ev_fork);
    if (op->fdph.ev_join) (void)hipEventDestroy(op->fdph.ev_join);
    delete op;
}

int bie_step_predict(bie_op *op, double *p_n_dev, void *stream) {
    BIE_GUARD({
        if (!op || !p_n_dev) {
            set_error("bie_step_predict: null operator or buffer");
            return BIE_EINVAL;
        }
        if (int rc = bie::coupled_ok(op, "bie_step_predict")) return rc;
        if (op->step >= op->horizon) {
            set_error("bie_step_predict: step past the lag count of the operator's problems");
            return BIE_EINVAL;
        }
        hipStream_t s = (hipStream_t)stream;
        bie::StepIdx si;
        si.n = si.n0 = op->step;
        const int rc = op->kind == BIE_KIND_DENSE ? bie::dense_step(op, op->zero_in, p_n_dev, s, si, false)
                                                  : bie::fdph_step(op, op->zero_in, p_n_dev, s, si, false);
        if (rc) return rc;
        op->predicted = true;
        return BIE_OK;
    })
}

int bie_step_commit(bie_op *op, const double *d_n_dev, void *stream) {
    BIE_GUARD({
        if (!op || !d_n_dev) {
            set_error("bie_step_commit: null operator or buffer");
            return BIE_EINVAL;
        }
        if (!op->predicted) {
            set_error("bie_step_commit: no predicted step to commit");
            return BIE_EINVAL;
        }
        hipStream_t s = (hipStream_t)stream;
        const int rc = op->kind == BIE_KIND_DENSE ? bie::dense_commit(op, d_n_dev, s) : bie::fdph_commit(op, d_n_dev, s);
        if (rc) return rc;
        op->predicted = false;
        return BIE_OK;
    })
}

int bie_first_lag(const bie_op *op, double *k0_dev, void *stream) {
    BIE_GUARD({
        if (!op || !k0_dev) {
            set_error("bie_first_lag: null operator or buffer");
            return BIE_EINVAL;
        }
        if (int rc = bie::coupled_ok(op, "bie_first_lag")) return rc;
        return bie::launch_first_lag(op, k0_dev, (hipStream_t)stream);
    })
}

int bie_rupture_run(bie_op *op, const bie_friction *fr, const double *t0_dev, double *slip_dev, int32_t *state_dev,
                    double *D_dev, double *T_dev, int64_t steps, void *stream) {
    BIE_GUARD({
        if (!op || !fr || steps < 0 || (steps > 0 && (!t0_dev || !slip_dev || !state_dev || !D_dev || !T_dev))) {
            set_error("bie_rupture_run: null operator, law or buffer, or negative step count");
            return BIE_EINVAL;
        }
        if (fr->law != BIE_LAW_STATIC_DYNAMIC && fr->law != BIE_LAW_EXP_WEAKENING) {
            set_error("bie_rupture_run: unknown friction law");
            return BIE_EINVAL;
        }
        if (!(fr->t_dy <= fr->t_th) || (fr->law == BIE_LAW_EXP_WEAKENING && !(fr->d_c > 0.0))) {
            set_error("bie_rupture_run: need t_dy <= t_th and, for the exponential law, d_c > 0");
            return BIE_EINVAL;
        }
        if (int rc = bie::coupled_ok(op, "bie_rupture_run")) return rc;
        if (op->predicted) {
            set_error("bie_rupture_run: the current step was predicted; commit it first");
            return BIE_ESTATE;
        }
        if (steps > op->horizon - op->step) {
            set_error("bie_rupture_run: steps past the lag count of the operator's problems");
            return BIE_EINVAL;
        }
        hipStream_t s = (hipStream_t)stream;
        const int64_t N = op->N;
        if (!op->k0_ready) {
            if (int rc = bie::launch_first_lag(op, op->k0, s)) return rc;
            op->k0_ready = true;
        }
        for (int64_t k = 0; k < steps; ++k) {
            double *t = T_dev + k * N;
            double *d = D_dev + k * N;
            if (int rc = bie_step_predict(op, t, stream)) return rc;
            if (int rc = bie::launch_friction((int)N, *fr, op->dt, t0_dev, op->k0, slip_dev, state_dev, t, d, s))
                return rc;
            if (int rc = bie_step_commit(op, d, stream)) return rc;
        }
        return BIE_OK;
    })
}

int bie_set_debug(bie_op *op, int32_t flags, void *stream) {
    BIE_GUARD({
        if (!op) {
            set_error("bie_set_debug: null operator");
            return BIE_EINVAL;
        }
        if (op->kind != BIE_KIND_DENSE && op->kind != BIE_KIND_FDPH) {
            set_error("bie_set_debug: operator not built");
            return BIE_ESTATE;
        }
        op->scan_finite = (flags & BIE_DEBUG_SCAN_FINITE) != 0;
        if (op->scan_finite)
            BIE_HIP_TRY(hipMemsetAsync(op->nonfinite, 0xFF, sizeof(int64_t), (hipStream_t)stream));
        return BIE_OK;
    })
}

int bie_debug_status(const bie_op *op, int64_t *first_bad_out, void *stream) {
    BIE_GUARD({
        if (!op || !first_bad_out) {
            set_error("bie_debug_status: null pointer");
            return BIE_EINVAL;
        }
        if (op->kind != BIE_KIND_DENSE && op->kind != BIE_KIND_FDPH) {
            set_error("bie_debug_status: operator not built");
            return BIE_ESTATE;
        }
        uint64_t w = ~0ull;
        if (op->scan_finite) {
            BIE_HIP_TRY(hipMemcpyAsync(&w, op->nonfinite, sizeof(w), hipMemcpyDeviceToHost, (hipStream_t)stream));
            BIE_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
        }
        *first_bad_out = w == ~0ull ? -1 : (int64_t)w;
        return BIE_OK;
    })
}

int bie_diag_aca(int32_t nr, int32_t ns, const double *A_host, double eps, uint64_t seed, int32_t *rank_out,
                 int32_t *fallback_out, int32_t *sweeps_out, double *rel_err_out) {
    BIE_GUARD({
        if (nr < 1 || ns < 1 || !A_host || !(eps > 0) || !rank_out || !fallback_out || !sweeps_out || !rel_err_out) {
            set_error("bie_diag_aca: invalid argument");
            return BIE_EINVAL;
        }
        int r = 0, f = 0, w = 0;
        double e = 0.0;
        const int rc = bie::diag_aca(nr, ns, A_host, eps, seed, &r, &f, &w, &e);
        *rank_out = r;
        *fallback_out = f;
        *sweeps_out = w;
        *rel_err_out = e;
        return rc;
    })
}

int bie_plan_block_errors(const bie_plan *plan, double *buf_host, int64_t capacity, int64_t *rows_out) {
    BIE_GUARD({
        if (!plan || plan->kind != BIE_KIND_FDPH) {
            set_error("bie_plan_block_errors: not an FDP=H plan");
            return BIE_EINVAL;
        }
        return bie::plan_block_errors(plan->fdph, buf_host, capacity, rows_out);
    })
}

int bie_plan_dense_lag_entries(const bie_plan *plan, int64_t *buf_host, int64_t capacity) {
    BIE_GUARD({
        if (!plan || !buf_host || plan->kind != BIE_KIND_DENSE) {
            set_error("bie_plan_dense_lag_entries: null pointer or not a plain-form plan");
            return BIE_EINVAL;
        }
        const bie::DensePlan &D = plan->dense;
        const int64_t n = std::min<int64_t>(capacity, D.M);
        for (int64_t m = 0; m < n; ++m) buf_host[m] = D.off[(size_t)(m + 1) * D.N] - D.off[(size_t)m * D.N];
        return BIE_OK;
    })
}

}  // extern "C"
