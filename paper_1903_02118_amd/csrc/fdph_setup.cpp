// Host-side setup of the FDP=H operator: clustering, block cluster tree, ART
// integers, degenerate and transient waveforms, ACA+ compression, and the
// packing of every per-step data structure into device memory.
//
// Paper references: clustering and admissibility Sec. 2.3 and Sec. 4.2.2
// (Eq. 8, box diagonal + longest element as diam, box centres as i*, j*,
// dist = |i* - j*| - diam); ART Eqs. 42 and App. C.2 (+ n_c broadening,
// Sec. 4.3 / App. H); amplitude Eq. 51; degenerate waveform Eq. 50; ACA+
// Sec. 6.1.1 (stop when |K_l - K_{l+1}| < eps |K_{l+1}|, keep K_{l+1}; keep
// the block dense when the rank reaches the block's rank, Sec. 6.2);
// Domain S static App. B.1; 2D transient App. B.3 / App. H.1; inadmissible
// leaves App. E.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <random>

#include "bie_internal.hpp"

namespace bie {

// ---------------------------------------------------------------------------
bool Geometry::first_lag_diagonal() const {
    if (mode != BIE_MODE_ANTIPLANE) return false;
    // S-front radius at the first collocation time, less a relative 1e-9: an
    // element at that distance up to rounding (neighbours on a curved trace
    // with beta dt = dx/2) is grazed by the front, and its first-lag entry
    // (below 1e-7 |K_ii,0|) is left out of the coupled step
    const double c = beta * eps_t * dt * (1.0 - 1e-9);
    double hmax = 0.0;
    for (const Frame &f : fr) hmax = std::max(hmax, f.h);
    // an element within c of a point has its midpoint within hmax + c of it:
    // bin midpoints on cells of that size and search the 3 x 3 neighbourhood
    const double cell = hmax + c;
    auto cell_of = [&](double x, double y) {
        return std::make_pair((int64_t)std::floor(x / cell), (int64_t)std::floor(y / cell));
    };
    std::map<std::pair<int64_t, int64_t>, std::vector<int>> bins;
    for (int j = 0; j < N; ++j) bins[cell_of(fr[j].cx, fr[j].cy)].push_back(j);
    std::vector<int> prob(N, 0);
    for (size_t k = 0; k + 1 < off.size(); ++k)
        for (int j = off[k]; j < off[k + 1]; ++j) prob[j] = (int)k;
    for (int i = 0; i < N; ++i) {
        const auto ci = cell_of(fr[i].cx, fr[i].cy);
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy) {
                const auto it = bins.find({ci.first + dx, ci.second + dy});
                if (it == bins.end()) continue;
                for (int j : it->second) {
                    if (j == i || prob[j] != prob[i]) continue;
                    const Frame &f = fr[j];
                    const double px = fr[i].cx - f.cx, py = fr[i].cy - f.cy;
                    const double X = px * f.tx + py * f.ty, Y = px * f.nx + py * f.ny;
                    const double ex = std::max(std::fabs(X) - f.h, 0.0);
                    if (ex * ex + Y * Y < c * c) return false;
                }
            }
    }
    return true;
}

int Geometry::build(const bie_problem *probs, int count) {
    if (!probs || count < 1) {
        set_error("invalid problem: null pointer or empty batch");
        return BIE_EINVAL;
    }
    int64_t total = 0;
    for (int k = 0; k < count; ++k) {
        const bie_problem *p = &probs[k];
        if (!p->xa_host || !p->xb_host || p->n_elem <= 0 || p->n_lags <= 0) {
            set_error("invalid problem: null end points or non-positive sizes");
            return BIE_EINVAL;
        }
        if (!(p->mu > 0) || !(p->beta > 0) || !(p->dt > 0)) {
            set_error("invalid problem: mu, beta and dt must be positive");
            return BIE_EINVAL;
        }
        if (p->mode != BIE_MODE_ANTIPLANE && p->mode != BIE_MODE_INPLANE) {
            set_error("invalid problem: unknown mode");
            return BIE_EINVAL;
        }
        if (p->mode == BIE_MODE_INPLANE && !(p->alpha > p->beta)) {
            set_error("invalid problem: the in-plane mode needs alpha > beta");
            return BIE_EINVAL;
        }
        if (k > 0 && (p->mu != probs[0].mu || p->beta != probs[0].beta || p->dt != probs[0].dt ||
                      p->eps_t != probs[0].eps_t || p->mode != probs[0].mode || p->alpha != probs[0].alpha)) {
            set_error("invalid batch: every problem must share mu, beta, dt and eps_t");
            return BIE_EINVAL;
        }
        total += p->n_elem;
    }
    if (total > (int64_t)1 << 30) {
        set_error("invalid batch: more than 2^30 elements");
        return BIE_EINVAL;
    }
    N = (int)total;
    mode = probs[0].mode;
    alpha = probs[0].alpha;
    mu = probs[0].mu;
    beta = probs[0].beta;
    dt = probs[0].dt;
    eps_t = probs[0].eps_t;
    fr.resize(N);
    length.resize(N);
    hz.resize(N);
    off.assign(1, 0);
    int j = 0;
    for (int k = 0; k < count; ++k) {
        const bie_problem *p = &probs[k];
        for (int e = 0; e < p->n_elem; ++e, ++j) {
            const double ax = p->xa_host[2 * e], ay = p->xa_host[2 * e + 1];
            const double bx = p->xb_host[2 * e], by = p->xb_host[2 * e + 1];
            const double dx = bx - ax, dy = by - ay;
            const double len = std::hypot(dx, dy);
            if (!(len > 0) || !std::isfinite(len)) {
                set_error("invalid problem: element " + std::to_string(e) + " has zero or non-finite length");
                return BIE_EINVAL;
            }
            Frame &f = fr[j];
            f.cx = 0.5 * (ax + bx);
            f.cy = 0.5 * (ay + by);
            f.tx = dx / len;
            f.ty = dy / len;
            f.nx = -f.ty;
            f.ny = f.tx;
            f.h = 0.5 * len;
            length[j] = len;
            hz[j] = p->n_lags;
        }
        off.push_back(j);
    }
    if (mode == BIE_MODE_INPLANE) {
        // the diagonal 2 x 2 kernel holds on a straight fault only
        const Frame &f0 = fr[0];
        double scale = 0.0;
        for (int e = 0; e < N; ++e) scale = std::max(scale, std::hypot(fr[e].cx - f0.cx, fr[e].cy - f0.cy));
        for (int e = 0; e < N; ++e) {
            const double off_line = std::fabs((fr[e].cx - f0.cx) * f0.nx + (fr[e].cy - f0.cy) * f0.ny);
            if (std::fabs(fr[e].tx - f0.tx) > 1e-12 || std::fabs(fr[e].ty - f0.ty) > 1e-12 ||
                off_line > 1e-9 * std::max(1.0, scale)) {
                set_error("invalid problem: the in-plane mode needs a straight fault (collinear, equally oriented elements)");
                return BIE_EINVAL;
            }
        }
    }
    return BIE_OK;
}

// ------------------------------------------------------------- clustering --
namespace {

constexpr double SNAP = 1e-9;

inline double snapv(double v) {
    const double r = std::nearbyint(v);
    return (std::fabs(v - r) <= SNAP * std::max(1.0, std::fabs(v))) ? r : v;
}
inline int64_t ifloor(double v) { return (int64_t)std::floor(snapv(v)); }
inline int64_t iceil(double v) { return (int64_t)std::ceil(snapv(v)); }

struct Clu {
    double lo[2], hi[2];
    std::vector<int> idx;
    int level = 0;
    int child[2] = {-1, -1};
    int nchild = 0;
    double maxlen = 0;
    double cx() const { return 0.5 * (lo[0] + hi[0]); }
    double cy() const { return 0.5 * (lo[1] + hi[1]); }
    double diag() const { return std::hypot(hi[0] - lo[0], hi[1] - lo[1]); }
    bool leaf() const { return nchild == 0; }
};

struct LeafH {
    int tau, sigma;
    bool adm;
    double diam, dist;
    // admissible data
    double ist[2], jst[2];
    std::vector<int64_t> mbar, dmj;  // per source, order of sigma idx
    std::vector<int64_t> dmi;        // per receiver, order of tau idx
    int jpiv = -1;
    int64_t s0 = 0;
    std::vector<int> ntr;            // per component
    std::vector<std::vector<double>> htr;
    std::vector<std::vector<int32_t>> qb;  // per component: staircase run starts (+ end)
    std::vector<std::vector<double>> qr;   // per component: staircase run values
};

}  // namespace

struct FdphHost {
    std::vector<Clu> clu;
    std::vector<LeafH> leaves;
    std::vector<int64_t> near_rows;  // receiver, source, W
    int ncomp = 1;
};

void free_fdph_host(FdphHost *h) { delete h; }

namespace {

// Cluster tree of the elements [j0, j1), appended to clu; returns its root.
int build_tree(const Geometry &g, int j0, int j1, int leaf_size, std::vector<Clu> &clu) {
    Clu root;
    root.lo[0] = root.lo[1] = INFINITY;
    root.hi[0] = root.hi[1] = -INFINITY;
    for (int j = j0; j < j1; ++j) {
        root.lo[0] = std::min(root.lo[0], g.fr[j].cx);
        root.lo[1] = std::min(root.lo[1], g.fr[j].cy);
        root.hi[0] = std::max(root.hi[0], g.fr[j].cx);
        root.hi[1] = std::max(root.hi[1], g.fr[j].cy);
        root.idx.push_back(j);
    }
    const int root_id = (int)clu.size();
    clu.push_back(root);
    std::vector<int> stack{root_id};
    while (!stack.empty()) {
        const int ci = stack.back();
        stack.pop_back();
        double ml = 0;
        for (int j : clu[ci].idx) ml = std::max(ml, g.length[j]);
        clu[ci].maxlen = ml;
        if ((int)clu[ci].idx.size() <= leaf_size || clu[ci].level >= 60) continue;
        const Clu c = clu[ci];
        const double e0 = c.hi[0] - c.lo[0], e1 = c.hi[1] - c.lo[1];
        const int ax = (e0 >= e1) ? 0 : 1;
        const double mid = 0.5 * (c.lo[ax] + c.hi[ax]);
        Clu a, b;
        a.level = b.level = c.level + 1;
        std::memcpy(a.lo, c.lo, sizeof a.lo);
        std::memcpy(a.hi, c.hi, sizeof a.hi);
        std::memcpy(b.lo, c.lo, sizeof b.lo);
        std::memcpy(b.hi, c.hi, sizeof b.hi);
        a.hi[ax] = mid;
        b.lo[ax] = mid;
        for (int j : c.idx) {
            const double v = ax == 0 ? g.fr[j].cx : g.fr[j].cy;
            (v <= mid ? a.idx : b.idx).push_back(j);
        }
        int kids[2], nk = 0;
        if (!a.idx.empty()) {
            clu.push_back(a);
            kids[nk++] = (int)clu.size() - 1;
        }
        if (!b.idx.empty()) {
            clu.push_back(b);
            kids[nk++] = (int)clu.size() - 1;
        }
        clu[ci].nchild = nk;
        for (int k = 0; k < nk; ++k) clu[ci].child[k] = kids[k];
        for (int k = nk - 1; k >= 0; --k) stack.push_back(kids[k]);
    }
    return root_id;
}

// Block cluster tree below (root, root), leaves appended.
void build_blocks(const std::vector<Clu> &clu, int root, double eta, std::vector<LeafH> &leaves) {
    std::vector<std::pair<int, int>> stack{{root, root}};
    while (!stack.empty()) {
        auto [t, s] = stack.back();
        stack.pop_back();
        const Clu &a = clu[t], &b = clu[s];
        const double diam = std::max(a.diag(), b.diag()) + std::max(a.maxlen, b.maxlen);
        const double rbar = std::hypot(a.cx() - b.cx(), a.cy() - b.cy());
        const double dist = rbar - diam;
        if (diam < eta * dist) {
            LeafH L;
            L.tau = t;
            L.sigma = s;
            L.adm = true;
            L.diam = diam;
            L.dist = dist;
            leaves.push_back(std::move(L));
        } else if (a.leaf() || b.leaf()) {
            LeafH L;
            L.tau = t;
            L.sigma = s;
            L.adm = false;
            L.diam = diam;
            L.dist = dist;
            leaves.push_back(std::move(L));
        } else {
            for (int x = a.nchild - 1; x >= 0; --x)
                for (int y = b.nchild - 1; y >= 0; --y) stack.push_back({a.child[x], b.child[y]});
        }
    }
}

// Quantization (App. A.1) of a waveform: greedy runs [b_q, b_{q+1}) whose
// representative, the mean of the run's first and last values, is within
// min(eps_rel |h^|, eps_abs) of every value of the run.
void staircase(const std::vector<double> &h, double eps_rel, double eps_abs, std::vector<int32_t> &b,
               std::vector<double> &rep) {
    const int64_t n = (int64_t)h.size();
    b.assign(1, 0);
    rep.clear();
    int64_t start = 0;
    while (start < n) {
        int64_t end = start + 1;
        double lo = h[start], hi = h[start], best = h[start];
        while (end < n) {
            const double lo2 = std::min(lo, h[end]);
            const double hi2 = std::max(hi, h[end]);
            const double r = 0.5 * (h[start] + h[end]);
            const double tol = std::min(eps_rel * std::fabs(r), eps_abs);
            if (std::max(hi2 - r, r - lo2) > tol) break;
            lo = lo2;
            hi = hi2;
            best = r;
            ++end;
        }
        rep.push_back(best);
        b.push_back((int32_t)end);
        start = end;
    }
}

// ------------------------------------------------------------------ ACA+ --
// Partially pivoted adaptive cross approximation with random reference row
// and column (ACA+).  Produces A ~= U V^T with U [nr][k] and V [ns][k]
// (stored column-wise: U[l*nr + i], V[l*ns + j]).
struct AcaResult {
    int rank = 0;
    bool fallback = false;
    std::vector<double> U, V;
};

template <class RowF, class ColF>
AcaResult aca_plus(int nr, int ns, double eps, uint64_t seed, RowF row, ColF col) {
    AcaResult res;
    const int kmax = std::min(nr, ns);
    std::mt19937_64 rng(seed);
    std::vector<char> urow(nr, 0), ucol(ns, 0);
    std::vector<double> r(ns), c(nr), rref(ns), cref(nr);
    double norm2 = 0.0;

    auto resid_row = [&](int i, std::vector<double> &out) {
        row(i, out.data());
        for (int l = 0; l < res.rank; ++l) {
            const double ui = res.U[(size_t)l * nr + i];
            if (ui == 0.0) continue;
            const double *v = &res.V[(size_t)l * ns];
            for (int j = 0; j < ns; ++j) out[j] -= ui * v[j];
        }
    };
    auto resid_col = [&](int j, std::vector<double> &out) {
        col(j, out.data());
        for (int l = 0; l < res.rank; ++l) {
            const double vj = res.V[(size_t)l * ns + j];
            if (vj == 0.0) continue;
            const double *u = &res.U[(size_t)l * nr];
            for (int i = 0; i < nr; ++i) out[i] -= u[i] * vj;
        }
    };
    auto pick_unused = [&](const std::vector<char> &used, int n) -> int {
        int cnt = 0;
        for (int k = 0; k < n; ++k) cnt += !used[k];
        if (cnt == 0) return -1;
        int pick = (int)(rng() % (uint64_t)cnt);
        for (int k = 0; k < n; ++k)
            if (!used[k] && pick-- == 0) return k;
        return -1;
    };
    auto argmax_unused = [](const std::vector<double> &v, const std::vector<char> &used) {
        int best = -1;
        double bv = -1.0;
        for (size_t k = 0; k < v.size(); ++k)
            if (!used[k] && std::fabs(v[k]) > bv) {
                bv = std::fabs(v[k]);
                best = (int)k;
            }
        return best;
    };
    auto nrm = [](const std::vector<double> &v) {
        double s = 0;
        for (double x : v) s += x * x;
        return std::sqrt(s);
    };

    int iref = pick_unused(urow, nr), jref = pick_unused(ucol, ns);
    resid_row(iref, rref);
    resid_col(jref, cref);
    int stall = 0;
    while (res.rank < kmax) {
        // pivot from the larger of the reference residuals (ACA+)
        int ic = argmax_unused(cref, urow);
        int jr = argmax_unused(rref, ucol);
        const double vc = ic >= 0 ? std::fabs(cref[ic]) : 0.0;
        const double vr = jr >= 0 ? std::fabs(rref[jr]) : 0.0;
        if (vc == 0.0 && vr == 0.0) {
            // both references exhausted: the residual vanishes on them; try fresh ones
            if (++stall > 3) break;
            iref = pick_unused(urow, nr);
            jref = pick_unused(ucol, ns);
            if (iref < 0 || jref < 0) break;
            resid_row(iref, rref);
            resid_col(jref, cref);
            continue;
        }
        int ip, jp;
        if (vc >= vr) {
            ip = ic;
            resid_row(ip, r);
            jp = argmax_unused(r, ucol);
            if (jp < 0 || r[jp] == 0.0) {
                urow[ip] = 1;
                continue;
            }
            resid_col(jp, c);
        } else {
            jp = jr;
            resid_col(jp, c);
            ip = argmax_unused(c, urow);
            if (ip < 0 || c[ip] == 0.0) {
                ucol[jp] = 1;
                continue;
            }
            resid_row(ip, r);
        }
        const double piv = r[jp];
        std::vector<double> u(c), v(ns);
        for (int j = 0; j < ns; ++j) v[j] = r[j] / piv;
        // ||S_{k+1}||^2 = ||S_k||^2 + 2 sum_l (u.U_l)(v.V_l) + |u|^2 |v|^2
        double cross = 0.0;
        for (int l = 0; l < res.rank; ++l) {
            double a = 0, b = 0;
            const double *Ul = &res.U[(size_t)l * nr];
            const double *Vl = &res.V[(size_t)l * ns];
            for (int i = 0; i < nr; ++i) a += u[i] * Ul[i];
            for (int j = 0; j < ns; ++j) b += v[j] * Vl[j];
            cross += a * b;
        }
        const double nu = nrm(u), nv = nrm(v);
        norm2 += 2.0 * cross + nu * nu * nv * nv;
        res.U.insert(res.U.end(), u.begin(), u.end());
        res.V.insert(res.V.end(), v.begin(), v.end());
        res.rank++;
        urow[ip] = 1;
        ucol[jp] = 1;
        // update the reference residuals; renew an exhausted reference
        for (int j = 0; j < ns; ++j) rref[j] -= u[iref] * v[j];
        for (int i = 0; i < nr; ++i) cref[i] -= u[i] * v[jref];
        if (urow[iref]) {
            int k = pick_unused(urow, nr);
            if (k >= 0) {
                iref = k;
                resid_row(iref, rref);
            }
        }
        if (ucol[jref]) {
            int k = pick_unused(ucol, ns);
            if (k >= 0) {
                jref = k;
                resid_col(jref, cref);
            }
        }
        const double snorm = std::sqrt(std::max(norm2, 0.0));
        const double rest = std::max(nrm(cref) * std::sqrt((double)ns), nrm(rref) * std::sqrt((double)nr));
        if (nu * nv <= eps * snorm && rest <= eps * snorm) break;
    }
    if (res.rank >= kmax && kmax > 0) {
        // not compressible at this tolerance: keep the block exactly
        res.fallback = true;
        res.U.assign((size_t)kmax * nr, 0.0);
        res.V.assign((size_t)kmax * ns, 0.0);
        if (nr <= ns) {
            std::vector<double> rr(ns);
            for (int i = 0; i < nr; ++i) {
                row(i, rr.data());
                res.U[(size_t)i * nr + i] = 1.0;
                for (int j = 0; j < ns; ++j) res.V[(size_t)i * ns + j] = rr[j];
            }
        } else {
            std::vector<double> cc(nr);
            for (int j = 0; j < ns; ++j) {
                col(j, cc.data());
                res.V[(size_t)j * ns + j] = 1.0;
                for (int i = 0; i < nr; ++i) res.U[(size_t)j * nr + i] = cc[i];
            }
        }
        res.rank = kmax;
    }
    return res;
}

inline int64_t pow2ceil(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Last k < len with |dev(k)| > tol, or -1 (scan down from the end; on a
// nonplanar fault the deviation can change sign after the fronts have
// passed, so no lag may be skipped).
template <class F>
int64_t last_exceeding(int64_t len, double tol, F dev) {
    for (int64_t k = len - 1; k >= 0; --k)
        if (std::fabs(dev(k)) > tol) return k;
    return -1;
}

// BF16 bit pattern of v: rounded to FP32, then to the nearest BF16 (ties to even).
inline uint16_t bf16_bits(double v) {
    const float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

}  // namespace

// ---------------------------------------------------------------------------
int build_fdph(const bie_problem *prob, int count, const bie_fdph_params *par, hipStream_t s, bie_op_impl *op) {
    const auto t_start = std::chrono::steady_clock::now();
    Geometry g;
    int rc = g.build(prob, count);
    if (rc) return rc;
    if (!par) {
        set_error("null FDP=H parameters");
        return BIE_EINVAL;
    }
    if (g.mode != BIE_MODE_ANTIPLANE) {
        set_error("the FDP=H form is built for the anti-plane problem only (in-plane: plain form)");
        return BIE_EINVAL;
    }
    int M = 0;
    for (int k = 0; k < count; ++k) M = std::max(M, (int)prob[k].n_lags);
    if (M > 65535) {
        set_error("n_lags above 65535 is not supported (near windows are kept as 16-bit lengths)");
        return BIE_EINVAL;
    }
    if (g.eps_t != 1.0) {
        set_error("the FDP=H form requires eps_t = 1 (time discretization of Sec. 4.3)");
        return BIE_EINVAL;
    }
    if (!(par->eta >= 0) || par->leaf_size < 1 || par->n_c < 0 || !(par->eps_aca > 0) ||
        !(par->eps_q >= 0) || !(par->eps_st >= 0)) {
        set_error("invalid FDP=H parameters");
        return BIE_EINVAL;
    }
    const bool quant = (par->flags & BIE_FLAG_QUANTIZE_TRANSIENT) != 0;
    if (quant && !(par->eps_qtr >= 0)) {
        set_error("invalid eps_qtr");
        return BIE_EINVAL;
    }
    if (par->precision != BIE_FP64 && par->precision != BIE_MIXED_FP32 && par->precision != BIE_MIXED_BF16) {
        set_error("unknown precision mode");
        return BIE_EINVAL;
    }
    const int R = par->n_rhs == 0 ? 1 : par->n_rhs;
    if (R != 1 && R != 2 && R != 4) {
        set_error("n_rhs must be 1, 2 or 4");
        return BIE_EINVAL;
    }
    const int N = g.N;
    const double dt = g.dt, cdt = g.beta * g.dt, c = g.beta;
    const double tol_abs = par->eps_st * g.mu / (2.0 * g.beta);
    FdphOp &F = op->fdph;
    F.N = N;
    F.M = M;
    F.dt = dt;
    F.precision = par->precision;
    // several scenarios stage R histories per work item: 64-lag chunks keep
    // two or more workgroups per compute unit (measured: 128 lags for one
    // scenario, 64 for two or four)
    F.near_chunk = R > 1 ? 64 : NEAR_CHUNK_DEFAULT;
    F.R = R;
    if (const char *e = std::getenv("BIE_NEAR_CHUNK")) {  // tuning knob: 64, 128 or 256 (64 or 128 for scenarios)
        const int v = std::atoi(e);
        if (v == 64 || v == 128 || (R == 1 && v == 256)) F.near_chunk = v;
    }
    const int NEAR_CHUNK = F.near_chunk;
    F.tune.unroll = (F.precision == BIE_FP64) ? 16 : 8;
    if (const char *e = std::getenv("BIE_NEAR_UNROLL")) F.tune.unroll = std::atoi(e) >= 16 ? 16 : 8;
    if (const char *e = std::getenv("BIE_NEAR_LDS_PAD")) F.tune.lds_pad = std::max(0, std::min(65536, std::atoi(e)));
    if (const char *e = std::getenv("BIE_NEAR_WIDE")) F.tune.wide = std::atoi(e) != 0;
    auto *H = new FdphHost();
    F.host = H;

    // components: a planar fault uses the traction itself; otherwise the
    // global stress components, projected on each receiver normal afterwards
    bool planar = true;
    for (int j = 1; j < N && planar; ++j)
        planar = std::fabs(g.fr[j].nx - g.fr[0].nx) <= 1e-12 && std::fabs(g.fr[j].ny - g.fr[0].ny) <= 1e-12;
    std::vector<std::array<double, 2>> comp;
    if (planar)
        comp.push_back({g.fr[0].nx, g.fr[0].ny});
    else {
        comp.push_back({1.0, 0.0});
        comp.push_back({0.0, 1.0});
    }
    H->ncomp = (int)comp.size();
    const int NC = (int)comp.size();

    for (int k = 0; k < count; ++k) {
        const int root = build_tree(g, g.off[k], g.off[k + 1], par->leaf_size, H->clu);
        build_blocks(H->clu, root, par->eta, H->leaves);
    }
    auto &clu = H->clu;
    auto &leaves = H->leaves;

    // ---- ART integers and causality ---------------------------------------
    int64_t n_adm = 0, n_inadm = 0;
    for (auto &L : leaves) {
        if (!L.adm) {
            n_inadm++;
            continue;
        }
        n_adm++;
        const Clu &a = clu[L.tau], &b = clu[L.sigma];
        L.ist[0] = a.cx();
        L.ist[1] = a.cy();
        L.jst[0] = b.cx();
        L.jst[1] = b.cy();
        const double rbar = std::hypot(L.ist[0] - L.jst[0], L.ist[1] - L.jst[1]);
        L.dmi.resize(a.idx.size());
        for (size_t k = 0; k < a.idx.size(); ++k) {
            const Frame &f = g.fr[a.idx[k]];
            const double rij = std::hypot(f.cx - L.jst[0], f.cy - L.jst[1]);
            L.dmi[k] = ifloor((rij - rbar) / cdt);
        }
        L.mbar.resize(b.idx.size());
        L.dmj.resize(b.idx.size());
        for (size_t k = 0; k < b.idx.size(); ++k) {
            const Frame &f = g.fr[b.idx[k]];
            const double r = std::hypot(f.cx - L.ist[0], f.cy - L.ist[1]);
            L.mbar[k] = ifloor((r - f.h) / cdt);
            const int64_t mend = iceil((r + f.h) / cdt);
            L.dmj[k] = mend - L.mbar[k] + par->n_c;
        }
        const int64_t mn = *std::min_element(L.dmi.begin(), L.dmi.end()) +
                           *std::min_element(L.mbar.begin(), L.mbar.end());
        if (mn < 1) {
            set_error("discretized causality violated in an admissible leaf (min dm_i + mbar_j = " +
                      std::to_string(mn) + " < 1); reduce eta or enlarge the leaves");
            return BIE_ECAUSALITY;
        }
    }

    // ---- transient pivots and waveforms ----------------------------------------
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t la = 0; la < (int64_t)leaves.size(); ++la) {
        LeafH &L = leaves[la];
        if (!L.adm) continue;
        const Clu &b = clu[L.sigma];
        int kbest = 0;
        double dbest = INFINITY;
        for (size_t k = 0; k < b.idx.size(); ++k) {
            const Frame &f = g.fr[b.idx[k]];
            const double d = std::hypot(f.cx - L.jst[0], f.cy - L.jst[1]);
            if (d < dbest) {
                dbest = d;
                kbest = (int)k;
            }
        }
        L.jpiv = b.idx[kbest];
        L.s0 = L.mbar[kbest] + L.dmj[kbest];
        const int64_t Mk = g.hz[L.jpiv];
        L.ntr.assign(NC, 0);
        L.htr.assign(NC, {});
        L.qb.assign(NC, {});
        L.qr.assign(NC, {});
        const Frame &fp = g.fr[L.jpiv];
        for (int cc = 0; cc < NC; ++cc) {
            if (L.s0 >= Mk) continue;
            const double ks = proj_static(fp, L.ist[0], L.ist[1], comp[cc][0], comp[cc][1], g.mu) * dt;
            const int64_t len = Mk - L.s0;
            auto dev = [&](int64_t k) {
                return proj_kernel(fp, L.ist[0], L.ist[1], comp[cc][0], comp[cc][1], L.s0 + k, dt, 1.0, g.mu,
                                   g.beta) - ks;
            };
            const double tol = std::min(par->eps_q * std::fabs(ks), tol_abs);
            const int64_t n = last_exceeding(len, tol, dev) + 1;
            if (n == 0) continue;
            std::vector<double> ser(n);
            for (int64_t k = 0; k < n; ++k) ser[k] = dev(k);
            if (ser[0] == 0.0) continue;
            L.ntr[cc] = (int)n;
            L.htr[cc].resize(n);
            for (int64_t k = 0; k < n; ++k) L.htr[cc][k] = ser[k] / ser[0];
            if (quant) staircase(L.htr[cc], par->eps_qtr, tol_abs / std::fabs(ser[0]), L.qb[cc], L.qr[cc]);
        }
    }

    // ---- ACA+ of the F, S and transient matrices (per component) -------------
    struct BlockH {
        int leaf, kind, comp, rank;
        bool fallback;
        std::vector<double> U, V;  // U [rank][nr] (receiver weights folded), V [rank][ns]
    };
    std::vector<int> adm_ids;
    for (size_t a = 0; a < leaves.size(); ++a)
        if (leaves[a].adm) adm_ids.push_back((int)a);
    const int n_pieces = 3 * NC;
    std::vector<BlockH> blk(adm_ids.size() * n_pieces);

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t w = 0; w < (int64_t)blk.size(); ++w) {
        const int la = adm_ids[w / n_pieces];
        const int piece = (int)(w % n_pieces);
        const int kind = piece / NC, cc = piece % NC;
        const LeafH &L = leaves[la];
        const Clu &a = clu[L.tau], &b = clu[L.sigma];
        const int nr = (int)a.idx.size(), ns = (int)b.idx.size();
        const double ex = comp[cc][0], ey = comp[cc][1];
        BlockH &B = blk[w];
        B.leaf = la;
        B.kind = kind;
        B.comp = cc;
        B.rank = 0;
        B.fallback = false;
        if (kind == PIECE_TR && L.ntr[cc] == 0) continue;
        auto entry = [&](int il, int jl) -> double {
            const Frame &fi = g.fr[a.idx[il]];
            const Frame &fj = g.fr[b.idx[jl]];
            if (kind == PIECE_F) {
                const double rij = std::hypot(fi.cx - fj.cx, fi.cy - fj.cy);
                const double rsj = std::hypot(fj.cx - L.ist[0], fj.cy - L.ist[1]);
                const double tm = rij / c - (rsj / c - (double)L.mbar[jl] * dt);
                const double tp = rij / c + ((double)(L.mbar[jl] + L.dmj[jl]) * dt - rsj / c);
                return proj_step(fj, fi.cx, fi.cy, ex, ey, tp, g.mu, g.beta) -
                       proj_step(fj, fi.cx, fi.cy, ex, ey, tm, g.mu, g.beta);
            } else if (kind == PIECE_S) {
                return proj_static(fj, fi.cx, fi.cy, ex, ey, g.mu);
            } else {
                const int64_t sij = L.dmi[il] + L.mbar[jl] + L.dmj[jl];
                if (sij >= g.hz[a.idx[il]]) return 0.0;
                return proj_kernel(fj, fi.cx, fi.cy, ex, ey, sij, dt, 1.0, g.mu, g.beta) -
                       proj_static(fj, fi.cx, fi.cy, ex, ey, g.mu) * dt;
            }
        };
        auto rowf = [&](int il, double *out) {
            for (int jl = 0; jl < ns; ++jl) out[jl] = entry(il, jl);
        };
        auto colf = [&](int jl, double *out) {
            for (int il = 0; il < nr; ++il) out[il] = entry(il, jl);
        };
        AcaResult R = aca_plus(nr, ns, par->eps_aca, par->seed * 0x9E3779B97F4A7C15ull + (uint64_t)w * 7919u + 1u,
                               rowf, colf);
        B.rank = R.rank;
        B.fallback = R.fallback;
        B.U = std::move(R.U);
        B.V = std::move(R.V);
        // receiver weights (projection of the component on each receiver normal)
        for (int l = 0; l < B.rank; ++l)
            for (int il = 0; il < nr; ++il) {
                const Frame &fi = g.fr[a.idx[il]];
                B.U[(size_t)l * nr + il] *= (fi.nx * ex + fi.ny * ey);
            }
        if (kind == PIECE_S)
            for (auto &v : B.V) v *= dt;
    }

    // ---- pack the far field ------------------------------------------------------
    std::vector<FarBlock> fb;
    std::vector<double> fdat, gdat, hdat, htrdat;
    std::vector<SrcGroup> groups;
    std::vector<GroupSrc> gsrc;
    std::vector<int32_t> trl;
    std::vector<std::vector<RecvEntry>> recv_entries(N);
    int64_t ring_total = 0, y_total = 0, qstate_total = 0;
    std::vector<int32_t> qbounds;
    std::vector<double> qreps;
    int64_t rank_sum[3] = {0, 0, 0}, rank_max[3] = {0, 0, 0}, fallbacks = 0;
    int64_t max_dmj = 1;
    // degenerate waveforms h_{a,j,m} per (leaf, component), tap-major: tap m of
    // source k at base + m * N_s + k, so that threads of neighbouring sources
    // read neighbouring addresses
    std::vector<std::vector<int64_t>> h_off_of(leaves.size());
    int64_t h_total = 0;
    for (int la : adm_ids) {
        const LeafH &L = leaves[la];
        const Clu &b = clu[L.sigma];
        const int64_t ns = (int64_t)b.idx.size();
        const int64_t taps = *std::max_element(L.dmj.begin(), L.dmj.end());
        max_dmj = std::max(max_dmj, taps);
        h_off_of[la].assign(ns * NC, 0);
        for (int cc = 0; cc < NC; ++cc) {
            for (int64_t k = 0; k < ns; ++k) h_off_of[la][cc * ns + k] = h_total + k;
            h_total += taps * ns;
        }
    }
    hdat.assign(h_total, 0.0);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t ai = 0; ai < (int64_t)adm_ids.size(); ++ai) {
        const int la = adm_ids[ai];
        const LeafH &L = leaves[la];
        const Clu &b = clu[L.sigma];
        std::vector<double> w;
        for (int cc = 0; cc < NC; ++cc)
            for (size_t k = 0; k < b.idx.size(); ++k) {
                const Frame &fj = g.fr[b.idx[k]];
                const int64_t n = L.dmj[k];
                w.assign(n, 0.0);
                double amp = 0.0;
                for (int64_t m = 0; m < n; ++m) {
                    w[m] = proj_kernel(fj, L.ist[0], L.ist[1], comp[cc][0], comp[cc][1], L.mbar[k] + m, dt, 1.0,
                                       g.mu, g.beta);
                    amp += w[m];
                }
                double *h = &hdat[h_off_of[la][cc * b.idx.size() + k]];
                for (int64_t m = 0; m < n; ++m) h[m * (int64_t)b.idx.size()] = std::fabs(amp) > 0 ? w[m] / amp : 0.0;
            }
    }
    for (const BlockH &B : blk) {
        if (B.rank == 0) continue;
        const LeafH &L = leaves[B.leaf];
        const Clu &a = clu[L.tau], &b = clu[L.sigma];
        const int nr = (int)a.idx.size(), ns = (int)b.idx.size();
        FarBlock f{};
        f.kind = B.kind;
        f.rank = B.rank;
        f.nr = nr;
        f.ns = ns;
        // factors element-major, ranks contiguous: f[il][l], g[jl][l]
        f.f_off = (int64_t)fdat.size();
        for (int il = 0; il < nr; ++il)
            for (int l = 0; l < B.rank; ++l) fdat.push_back(B.U[(size_t)l * nr + il]);
        f.g_off = (int64_t)gdat.size();
        for (int jl = 0; jl < ns; ++jl)
            for (int l = 0; l < B.rank; ++l) gdat.push_back(B.V[(size_t)l * ns + jl]);
        const int64_t dmax = *std::max_element(L.dmi.begin(), L.dmi.end());
        const int64_t dmin = *std::min_element(L.dmi.begin(), L.dmi.end());
        f.dm_max = (int32_t)dmax;
        f.dm_min = (int32_t)dmin;
        f.hz = g.hz[a.idx[0]];
        std::vector<int64_t> delay(ns);
        for (int k = 0; k < ns; ++k) delay[k] = (B.kind == PIECE_F) ? L.mbar[k] : L.mbar[k] + L.dmj[k];
        const int64_t maxd = *std::max_element(delay.begin(), delay.end());
        if (B.kind == PIECE_TR) {
            f.ntr = L.ntr[B.comp];
            // live times: the slot cleared at a step (n - dm_min - ntr - 1) up to the newest write
            f.ring_len = (int32_t)pow2ceil(maxd + dmin + f.ntr + 2);
            f.y_len = (int32_t)pow2ceil(dmax - dmin + 1);
            f.y_off = y_total;
            y_total += (int64_t)f.rank * f.y_len;
            f.htr_off = (int64_t)htrdat.size();
            htrdat.insert(htrdat.end(), L.htr[B.comp].begin(), L.htr[B.comp].end());
            if (quant) {
                const std::vector<int32_t> &qb = L.qb[B.comp];
                const std::vector<double> &qr = L.qr[B.comp];
                f.nq = (int32_t)qr.size();
                f.qb_off = (int64_t)qbounds.size();
                qbounds.insert(qbounds.end(), qb.begin(), qb.end());
                f.qr_off = (int64_t)qreps.size();
                qreps.insert(qreps.end(), qr.begin(), qr.end());
                f.qs_off = qstate_total;
                qstate_total += (int64_t)f.rank * f.nq;
            }
        } else {
            f.ring_len = (int32_t)pow2ceil(maxd + dmax + 2);
        }
        f.ring_off = ring_total;
        ring_total += (int64_t)f.rank * f.ring_len;
        const int bid = (int)fb.size();
        fb.push_back(f);
        rank_sum[B.kind] += B.rank;
        rank_max[B.kind] = std::max<int64_t>(rank_max[B.kind], B.rank);
        fallbacks += B.fallback;
        if (B.kind == PIECE_TR)
            for (int l = 0; l < B.rank; ++l) {
                trl.push_back(bid);
                trl.push_back(l);
            }
        // source groups by delay
        std::vector<int> order(ns);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return delay[x] < delay[y]; });
        bool first = true;
        for (int p = 0; p < ns;) {
            int q = p;
            while (q < ns && delay[order[q]] == delay[order[p]]) ++q;
            SrcGroup G{};
            G.block = bid;
            G.delay = (int32_t)delay[order[p]];
            G.first = (int32_t)gsrc.size();
            G.count = q - p;
            G.clear = first ? 1 : 0;
            first = false;
            for (int z = p; z < q; ++z) {
                const int k = order[z];
                GroupSrc S{};
                S.j = b.idx[k];
                S.jl = k;
                if (B.kind == PIECE_F) {
                    S.h_len = (int32_t)L.dmj[k];
                    S.h_off = h_off_of[B.leaf][B.comp * ns + k];
                }
                gsrc.push_back(S);
            }
            groups.push_back(G);
            p = q;
        }
        // one gather entry per RECV_SPLIT ranks, so that the lanes sharing a
        // receiver's list get comparable work (transient ranks reach hundreds)
        for (int il = 0; il < nr; ++il)
            for (int l0 = 0; l0 < f.rank; l0 += RECV_SPLIT) {
                RecvEntry e{};
                e.kind = f.kind;
                e.rank = f.rank;
                e.cnt = std::min(RECV_SPLIT, f.rank - l0);
                e.dm = (int32_t)L.dmi[il];
                e.f_off = f.f_off + (int64_t)il * f.rank + l0;
                if (f.kind == PIECE_TR) {
                    e.mask = f.y_len - 1;
                    e.r_off = f.y_off + l0;
                } else {
                    e.mask = f.ring_len - 1;
                    e.r_off = f.ring_off + l0;
                }
                recv_entries[a.idx[il]].push_back(e);
            }
    }

    // ---- near field: tiles and pairs -----------------------------------------------
    // Sub-blocks of at most 32 x 32 of the inadmissible leaves.  Small ones
    // (nonplanar faults have many) are packed together into one tile when
    // their receiver and source counts both fit: the tile's pairs between
    // different sub-blocks are placeholders (no window, prec = -1), which the
    // near kernel skips through its per-receiver source ranges.
    struct Sub {
        int nr, ns, hz;
        int32_t recv[TILE], src[TILE];
    };
    std::vector<Sub> subs;
    for (auto &L : leaves) {
        if (L.adm) continue;
        const Clu &a = clu[L.tau], &b = clu[L.sigma];
        for (size_t r0 = 0; r0 < a.idx.size(); r0 += TILE)
            for (size_t s0 = 0; s0 < b.idx.size(); s0 += TILE) {
                Sub u{};
                u.nr = (int)std::min<size_t>(TILE, a.idx.size() - r0);
                u.ns = (int)std::min<size_t>(TILE, b.idx.size() - s0);
                for (int k = 0; k < u.nr; ++k) u.recv[k] = a.idx[r0 + k];
                for (int k = 0; k < u.ns; ++k) u.src[k] = b.idx[s0 + k];
                u.hz = g.hz[u.recv[0]];
                subs.push_back(u);
            }
    }
    bool merge = true;
    if (const char *e = std::getenv("BIE_NEAR_MERGE")) merge = std::atoi(e) != 0;  // tuning knob
    std::vector<std::vector<int>> packs;  // sub-blocks of each tile
    {
        std::vector<int> ord(subs.size());
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int x, int y) { return subs[x].nr * subs[x].ns > subs[y].nr * subs[y].ns; });
        std::vector<int> fr_, fs_;  // receivers / sources used by each open tile
        for (int u : ord) {
            int put = -1;
            if (merge && subs[u].nr * subs[u].ns < TILE * TILE) {
                // first fit among the most recent tiles
                const int lo = std::max(0, (int)packs.size() - 64);
                for (int k = (int)packs.size() - 1; k >= lo; --k)
                    if (fr_[k] + subs[u].nr <= TILE && fs_[k] + subs[u].ns <= TILE &&
                        subs[packs[k][0]].hz == subs[u].hz) {
                        put = k;
                        break;
                    }
            }
            if (put < 0) {
                packs.push_back({});
                fr_.push_back(0);
                fs_.push_back(0);
                put = (int)packs.size() - 1;
            }
            packs[put].push_back(u);
            fr_[put] += subs[u].nr;
            fs_[put] += subs[u].ns;
        }
    }
    std::vector<NearTile> tiles;
    std::vector<int32_t> prec, psrc;
    int64_t near_pairs = 0;  // real pairs (placeholders excluded)
    for (const auto &pk : packs) {
        NearTile t{};
        std::vector<int> row_of, col_of;  // sub-block of each row / column
        for (size_t z = 0; z < pk.size(); ++z) {
            const Sub &u = subs[pk[z]];
            for (int k = 0; k < u.nr; ++k) {
                t.recv[t.nr++] = u.recv[k];
                row_of.push_back((int)z);
            }
            for (int k = 0; k < u.ns; ++k) {
                t.src[t.ns++] = u.src[k];
                col_of.push_back((int)z);
            }
            near_pairs += (int64_t)u.nr * u.ns;
        }
        t.pair_begin = (int64_t)prec.size();
        t.hz = subs[pk[0]].hz;
        for (int r = 0; r < t.nr; ++r)
            for (int q = 0; q < t.ns; ++q) {
                const bool real = row_of[r] == col_of[q];
                prec.push_back(real ? t.recv[r] : -1);
                psrc.push_back(real ? t.src[q] : -1);
            }
        tiles.push_back(t);
    }
    const int64_t pair_slots = (int64_t)prec.size();
    F.n_tiles = (int)tiles.size();
    F.n_pairs = pair_slots;
    if (pair_slots > MAX_DISPATCH_ITEMS) {
        set_error("too many near-field pairs for one dispatch");
        return BIE_EINVAL;
    }

    DevArena &A = op->arena;
    if ((rc = A.upload(&F.dfr, g.fr, s))) return rc;
    if ((rc = A.upload(&F.hz, g.hz, s))) return rc;
    int32_t *d_prec = nullptr;
    if ((rc = A.upload(&d_prec, prec, s))) return rc;
    if ((rc = A.upload(&F.pSrc, psrc, s))) return rc;
    if ((rc = A.alloc(&F.pW, pair_slots))) return rc;
    if ((rc = A.alloc(&F.pKs, pair_slots))) return rc;
    if (pair_slots > 0) {
        if ((rc = launch_near_windows(g, F, d_prec, par->eps_q, tol_abs, s))) return rc;
    }
    std::vector<int32_t> W(pair_slots);
    if (pair_slots > 0) {
        BIE_HIP_TRY(hipMemcpyAsync(W.data(), F.pW, pair_slots * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        BIE_HIP_TRY(hipStreamSynchronize(s));
    }
    // Chunk-major window layout: a work item is (tile, lag chunk); the chunk
    // segments of all the tile's pairs are stored back to back, each on a
    // 128-byte boundary, so that a work item streams one contiguous region.
    const int64_t align = (F.precision == BIE_FP64) ? 16 : 32;
    std::vector<int32_t> items;          // (tile, chunk)
    std::vector<int64_t> item_base;      // element offset of each item's region
    std::vector<int32_t> item_rel;       // [item][TILE*TILE]: segment offset in the region
    std::vector<uint16_t> item_rng;      // [item][TILE]: sources [lo, hi) of each receiver with lags in the chunk
    std::vector<int32_t> tile_item0(tiles.size(), 0);
    std::vector<int32_t> pTile(pair_slots), pQ(pair_slots);
    std::vector<std::vector<int32_t>> rn(N);
    std::vector<std::vector<int64_t>> rp(N);
    int64_t near_lags = 0, maxW = 1;
    for (int t = 0; t < F.n_tiles; ++t) {
        const NearTile &T = tiles[t];
        const int np = T.nr * T.ns;
        int64_t tw = 0;
        for (int q = 0; q < np; ++q) {
            tw = std::max<int64_t>(tw, W[T.pair_begin + q]);
            pTile[T.pair_begin + q] = t;
            pQ[T.pair_begin + q] = q;
        }
        maxW = std::max(maxW, tw);
        const int nch = (int)((tw + NEAR_CHUNK - 1) / NEAR_CHUNK);
        tile_item0[t] = (int32_t)(items.size() / 2);
        for (int ch = 0; ch < nch; ++ch) {
            const int item = (int)(items.size() / 2);
            items.push_back(t);
            items.push_back(ch);
            item_base.push_back(near_lags);
            const size_t r0 = item_rel.size();
            item_rel.resize(r0 + TILE * TILE, 0);
            int64_t cur = 0;
            for (int q = 0; q < np; ++q) {
                const int64_t len = std::clamp<int64_t>((int64_t)W[T.pair_begin + q] - (int64_t)ch * NEAR_CHUNK, 0, NEAR_CHUNK);
                item_rel[r0 + q] = (int32_t)cur;
                cur += (len + align - 1) / align * align;
            }
            for (int r = 0; r < TILE; ++r) {
                int lo = 0, hi = 0;
                if (r < T.nr) {
                    lo = T.ns;
                    for (int q = 0; q < T.ns; ++q)
                        if ((int64_t)W[T.pair_begin + (int64_t)r * T.ns + q] > (int64_t)ch * NEAR_CHUNK) {
                            lo = std::min(lo, q);
                            hi = q + 1;
                        }
                    if (hi == 0) lo = 0;
                }
                item_rng.push_back((uint16_t)(lo | (hi << 8)));
            }
            near_lags += cur;
            for (int r = 0; r < T.nr; ++r) rn[T.recv[r]].push_back(item * TILE + r);
        }
        for (int r = 0; r < T.nr; ++r)
            for (int q = 0; q < T.ns; ++q) {
                const int64_t p = T.pair_begin + (int64_t)r * T.ns + q;
                if (prec[p] >= 0 && W[p] < T.hz) rp[T.recv[r]].push_back(p);  // pairs with a static tail
            }
    }
    if ((int64_t)(items.size() / 2) * NEAR_THREADS > MAX_DISPATCH_ITEMS || (int64_t)N * 64 > MAX_DISPATCH_ITEMS) {
        set_error("operator too large for one dispatch per step (near-field work items, pairs or receivers)");
        return BIE_EINVAL;
    }
    F.n_items = (int)(items.size() / 2);
    {
        // an alternative workgroup order for the autotuner: items that stage
        // the same source histories (same first source, same lag chunk) go to
        // one XCD (workgroup w runs on XCD w mod 8), groups balanced over XCDs
        constexpr int XCD = 8;
        std::vector<int> ord(F.n_items);
        std::iota(ord.begin(), ord.end(), 0);
        auto key = [&](int it) { return std::make_pair(tiles[items[2 * it]].src[0], items[2 * it + 1]); };
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return key(x) < key(y); });
        std::vector<std::vector<int32_t>> q(XCD);
        for (size_t a0 = 0; a0 < ord.size();) {
            size_t a1 = a0;
            while (a1 < ord.size() && key(ord[a1]) == key(ord[a0])) ++a1;
            int best = 0;
            for (int x = 1; x < XCD; ++x)
                if (q[x].size() < q[best].size()) best = x;
            for (size_t z = a0; z < a1; ++z) q[best].push_back(ord[z]);
            a0 = a1;
        }
        size_t len = 0;
        for (auto &v : q) len = std::max(len, v.size());
        std::vector<int32_t> perm(len * XCD, -1);
        for (int x = 0; x < XCD; ++x)
            for (size_t k = 0; k < q[x].size(); ++k) perm[k * XCD + x] = q[x][k];
        if ((int64_t)perm.size() * NEAR_THREADS > MAX_DISPATCH_ITEMS) perm.clear();
        if (!perm.empty()) {
            if ((rc = A.upload(&F.perm_grouped, perm, s))) return rc;
            F.grid_grouped = (int)perm.size();
        }
        // step index at which the autotuner times the near kernel: every lag
        // chunk active, every problem still running
        int64_t min_hz = M;
        for (int k = 0; k < count; ++k) min_hz = std::min<int64_t>(min_hz, prob[k].n_lags);
        F.tune_step = std::max<int64_t>(0, std::min<int64_t>(maxW, min_hz - 1));
    }
    if ((rc = A.upload(&F.item_base, item_base, s))) return rc;
    if ((rc = A.upload(&F.item_rel, item_rel, s))) return rc;
    if ((rc = A.upload(&F.item_rng, item_rng, s))) return rc;
    // +64 elements of padding: an empty segment at the very end is read (and
    // ignored) at its offset by the branch-free near kernel
    if (F.precision == BIE_FP64) {
        if ((rc = A.alloc(&F.Kw, near_lags + 64))) return rc;
        BIE_HIP_TRY(hipMemsetAsync(F.Kw, 0, (near_lags + 64) * sizeof(double), s));
    } else {
        if ((rc = A.alloc(&F.Kw32, near_lags + 64))) return rc;
        BIE_HIP_TRY(hipMemsetAsync(F.Kw32, 0, (near_lags + 64) * sizeof(float), s));
    }
    if (near_pairs > 0) {
        int32_t *d_ptile = nullptr, *d_pq = nullptr, *d_ti0 = nullptr;
        if ((rc = A.upload(&d_ptile, pTile, s))) return rc;
        if ((rc = A.upload(&d_pq, pQ, s))) return rc;
        if ((rc = A.upload(&d_ti0, tile_item0, s))) return rc;
        if ((rc = launch_near_fill(g, F, d_prec, d_ptile, d_pq, d_ti0, s))) return rc;
    }
    {
        // K_ii,0 per receiver: kept for the coupled step's first-lag solve;
        // in the mixed modes also applied by the gather in FP64 (the FP32
        // window's own lag-0 value of the self pair is zeroed)
        std::vector<double> self0(N, 0.0);
        std::vector<int64_t> self_off;
        for (int64_t p = 0; p < pair_slots; ++p)
            if (prec[p] >= 0 && prec[p] == psrc[p] && W[p] > 0) {
                const Frame &f = g.fr[prec[p]];
                self0[prec[p]] = proj_kernel(f, f.cx, f.cy, f.nx, f.ny, 0, dt, 1.0, g.mu, g.beta);
                const int item0 = tile_item0[pTile[p]];
                self_off.push_back(item_base[item0] + item_rel[(size_t)item0 * TILE * TILE + pQ[p]]);
            }
        if ((rc = A.upload(&F.first_lag, self0, s))) return rc;
        if (F.precision != BIE_FP64) {
            if ((rc = A.upload(&F.self0, self0, s))) return rc;
            int64_t *d_so = nullptr;
            if ((rc = A.upload(&d_so, self_off, s))) return rc;
            if ((rc = launch_zero_self(F, d_so, (int)self_off.size(), s))) return rc;
        }
        BIE_HIP_TRY(hipStreamSynchronize(s));
    }
    BIE_HIP_TRY(hipStreamSynchronize(s));
    H->near_rows.clear();
    H->near_rows.reserve(3 * near_pairs);
    for (int64_t p = 0; p < pair_slots; ++p) {
        if (prec[p] < 0) continue;
        H->near_rows.push_back(prec[p]);
        H->near_rows.push_back(psrc[p]);
        H->near_rows.push_back(W[p]);
    }
    auto csr32 = [&](const std::vector<std::vector<int32_t>> &v, std::vector<int32_t> &ptr, std::vector<int32_t> &idx) {
        ptr.assign(N + 1, 0);
        for (int i = 0; i < N; ++i) ptr[i + 1] = ptr[i] + (int32_t)v[i].size();
        idx.clear();
        for (int i = 0; i < N; ++i) idx.insert(idx.end(), v[i].begin(), v[i].end());
    };
    std::vector<int32_t> rn_ptr, rn_idx, rp_ptr;
    std::vector<int64_t> rp_idx;
    csr32(rn, rn_ptr, rn_idx);
    // receiver-major partial slots: the near kernel writes (item, r) to the
    // position of that slot in its receiver's list
    std::vector<int32_t> pslot((size_t)std::max(F.n_items, 1) * TILE, -1);
    for (size_t k = 0; k < rn_idx.size(); ++k) pslot[rn_idx[k]] = (int32_t)k;
    rp_ptr.assign(N + 1, 0);
    for (int i = 0; i < N; ++i) rp_ptr[i + 1] = rp_ptr[i] + (int32_t)rp[i].size();
    for (int i = 0; i < N; ++i) rp_idx.insert(rp_idx.end(), rp[i].begin(), rp[i].end());
    std::vector<double> ks_host(pair_slots);
    if (pair_slots > 0) {
        BIE_HIP_TRY(hipMemcpyAsync(ks_host.data(), F.pKs, pair_slots * sizeof(double), hipMemcpyDeviceToHost, s));
        BIE_HIP_TRY(hipStreamSynchronize(s));
    }
    std::vector<TailPair> tails(rp_idx.size());
    for (size_t k = 0; k < rp_idx.size(); ++k) {
        const int64_t p = rp_idx[k];
        tails[k].src = psrc[p];
        tails[k].w = W[p];
        tails[k].ks = ks_host[p];
    }
    std::vector<int32_t> re_ptr(N + 1, 0);
    std::vector<RecvEntry> re;
    for (int i = 0; i < N; ++i) {
        re_ptr[i + 1] = re_ptr[i] + (int32_t)recv_entries[i].size();
        re.insert(re.end(), recv_entries[i].begin(), recv_entries[i].end());
    }

    // ---- histories and device upload -------------------------------------------------
    F.L = (int)pow2ceil(std::max<int64_t>(maxW + 1, 2));
    F.Lf = (int)pow2ceil(max_dmj + 1);
    // per-scenario state: R copies, scenario r at r strides
    F.scn.D = (int64_t)N * F.L;
    F.scn.Drec = (int64_t)N * F.Lf;
    F.scn.part = (int64_t)std::max<size_t>(rn_idx.size(), 1);
    F.scn.ring = std::max<int64_t>(ring_total, 1);
    F.scn.y = std::max<int64_t>(y_total, 1);
    F.scn.q = std::max<int64_t>(qstate_total, 1);
    F.scn.row = (int64_t)R * N;
    if ((rc = A.alloc(&F.Dring, (size_t)R * F.scn.D))) return rc;
    if ((rc = A.alloc(&F.Uring, (size_t)R * F.scn.D))) return rc;
    if ((rc = A.alloc(&F.Drec, (size_t)R * F.scn.Drec))) return rc;
    if ((rc = A.alloc(&F.TS, (size_t)R * N))) return rc;
    if ((rc = A.upload(&F.tiles, tiles, s))) return rc;
    if ((rc = A.upload(&F.items, items, s))) return rc;
    if ((rc = A.alloc(&F.partial, (size_t)R * F.scn.part))) return rc;
    if ((rc = A.upload(&F.rn_ptr, rn_ptr, s))) return rc;
    if ((rc = A.upload(&F.pslot, pslot, s))) return rc;
    if ((rc = A.upload(&F.rp_ptr, rp_ptr, s))) return rc;
    if ((rc = A.upload(&F.tails, tails, s))) return rc;
    F.n_blocks = (int)fb.size();
    F.n_groups = (int)groups.size();
    F.n_tr = (int)(trl.size() / 2);
    if ((rc = A.upload(&F.blocks, fb, s))) return rc;
    if (F.precision == BIE_FP64) {
        if ((rc = A.upload(&F.fdat, fdat, s))) return rc;
        if ((rc = A.upload(&F.gdat, gdat, s))) return rc;
    } else if (F.precision == BIE_MIXED_FP32) {
        std::vector<float> f32(fdat.begin(), fdat.end()), g32(gdat.begin(), gdat.end());
        if ((rc = A.upload(&F.fdat32, f32, s))) return rc;
        if ((rc = A.upload(&F.gdat32, g32, s))) return rc;
        BIE_HIP_TRY(hipStreamSynchronize(s));
    } else {
        std::vector<uint16_t> f16(fdat.size()), g16(gdat.size());
        for (size_t k = 0; k < fdat.size(); ++k) f16[k] = bf16_bits(fdat[k]);
        for (size_t k = 0; k < gdat.size(); ++k) g16[k] = bf16_bits(gdat[k]);
        if ((rc = A.upload(&F.fdat16, f16, s))) return rc;
        if ((rc = A.upload(&F.gdat16, g16, s))) return rc;
        BIE_HIP_TRY(hipStreamSynchronize(s));
    }
    if ((rc = A.alloc(&F.rings, (size_t)R * F.scn.ring))) return rc;
    if ((rc = A.alloc(&F.yrings, (size_t)R * F.scn.y))) return rc;
    F.rings_bytes = (size_t)R * F.scn.ring * sizeof(double);
    F.yrings_bytes = (size_t)R * F.scn.y * sizeof(double);
    F.quantized = quant;
    if (quant) {
        if ((rc = A.upload(&F.qbounds, qbounds, s))) return rc;
        if ((rc = A.upload(&F.qrep, qreps, s))) return rc;
        if ((rc = A.alloc(&F.qstate, (size_t)R * F.scn.q))) return rc;
        F.qstate_bytes = (size_t)R * F.scn.q * sizeof(double);
    }
    if ((rc = A.upload(&F.hdat, hdat, s))) return rc;
    if ((rc = A.upload(&F.htr, htrdat, s))) return rc;
    if ((rc = A.upload(&F.groups, groups, s))) return rc;
    if ((rc = A.upload(&F.gsrc, gsrc, s))) return rc;
    if ((rc = A.upload(&F.tr_list, trl, s))) return rc;
    if ((rc = A.upload(&F.re_ptr, re_ptr, s))) return rc;
    if ((rc = A.upload(&F.re, re, s))) return rc;
    F.n_groups = (int)groups.size();
    if (!std::getenv("BIE_NO_SIDE_STREAM")) {  // tuning knob: run everything on one stream
        BIE_HIP_TRY(hipStreamCreateWithFlags(&F.side, hipStreamNonBlocking));
        BIE_HIP_TRY(hipEventCreateWithFlags(&F.ev_fork, hipEventDisableTiming));
        BIE_HIP_TRY(hipEventCreateWithFlags(&F.ev_join, hipEventDisableTiming));
    }
    if ((rc = fdph_reset(op, s))) return rc;
    BIE_HIP_TRY(hipStreamSynchronize(s));

    // ---- statistics ---------------------------------------------------------------------
    bie_stats &st = op->stats;
    st.kind = BIE_KIND_FDPH;
    st.n_elem = N;
    st.n_lags = M;
    st.precision = F.precision;
    st.n_adm = n_adm;
    st.n_inadm = n_inadm;
    st.near_pairs = near_pairs;
    int64_t sumW = 0;
    for (int64_t p = 0; p < pair_slots; ++p) sumW += W[p];
    st.near_lags = sumW;
    for (int k = 0; k < 3; ++k) {
        st.rank_sum[k] = rank_sum[k];
        st.rank_max[k] = rank_max[k];
    }
    st.aca_fallbacks = fallbacks;
    st.device_bytes = A.bytes;
    const double kb = (F.precision == BIE_FP64) ? 8.0 : 4.0;
    const double fb_bytes = (F.precision == BIE_FP64) ? 8.0 : (F.precision == BIE_MIXED_FP32 ? 4.0 : 2.0);
    // near field: the windows, plus one history read per (tile, chunk) source row
    double tile_hist = 0;
    for (int it = 0; it < F.n_items; ++it) tile_hist += (double)tiles[items[2 * it]].ns * NEAR_CHUNK * 8.0;
    st.near_bytes_per_step = (double)sumW * kb;
    double far = 0;
    for (const FarBlock &f : fb) {
        far += (double)f.rank * (f.nr + f.ns) * fb_bytes;    // factors
        far += (double)f.rank * (f.nr + f.ns) * 8.0;         // ring reads and updates
        if (f.kind == PIECE_TR) far += (double)f.rank * (f.nq > 0 ? 3.0 * f.nq : (double)f.ntr) * 16.0;  // transient FIR
    }
    for (const GroupSrc &q : gsrc) far += (double)q.h_len * 16.0;  // FIR of D
    // the windows are read once for all scenarios; histories and far field per scenario
    st.bytes_per_step = st.near_bytes_per_step + R * (tile_hist + far) + (double)near_pairs * 20.0;
    double fl = 2.0 * (double)sumW;
    for (const FarBlock &f : fb)
        fl += 2.0 * f.rank * (f.nr + f.ns) + (f.kind == PIECE_TR ? 2.0 * f.rank * (f.nq > 0 ? 2.0 * f.nq : (double)f.ntr) : 0);
    for (const GroupSrc &q : gsrc) fl += 2.0 * q.h_len;
    st.flops_per_step = R * fl;
    st.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    op->kind = BIE_KIND_FDPH;
    op->N = R * N;  // values per step row of D and T
    op->M = M;
    op->mode = g.mode;
    op->dt = g.dt;
    op->first_lag_diag = g.first_lag_diagonal();
    op->horizon = M;
    for (int k = 0; k < count; ++k) op->horizon = std::min<int64_t>(op->horizon, prob[k].n_lags);
    (void)hipFree(nullptr);
    return BIE_OK;
}

// ---------------------------------------------------------------------------
int export_fdph(const bie_op_impl *op, int what, int64_t *buf, int64_t cap, int64_t *rows) {
    const FdphHost *H = op->fdph.host;
    if (!H) {
        set_error("operator has no FDP=H setup data");
        return BIE_ESTATE;
    }
    std::vector<int64_t> out;
    int width = 0;
    if (what == BIE_EXPORT_NEAR) {
        width = 3;
        out = H->near_rows;
    } else if (what == BIE_EXPORT_LEAVES) {
        width = 5;
        for (const auto &L : H->leaves) {
            const auto &a = H->clu[L.tau], &b = H->clu[L.sigma];
            out.push_back(L.adm ? 1 : 0);
            out.push_back((int64_t)a.idx.size());
            out.push_back((int64_t)b.idx.size());
            out.push_back(*std::min_element(a.idx.begin(), a.idx.end()));
            out.push_back(*std::min_element(b.idx.begin(), b.idx.end()));
        }
    } else if (what == BIE_EXPORT_ART) {
        width = 6;
        for (size_t la = 0; la < H->leaves.size(); ++la) {
            const auto &L = H->leaves[la];
            if (!L.adm) continue;
            const auto &a = H->clu[L.tau], &b = H->clu[L.sigma];
            for (size_t k = 0; k < b.idx.size(); ++k) {
                int64_t r[6] = {(int64_t)la, b.idx[k], L.mbar[k], L.dmj[k], -1, 0};
                out.insert(out.end(), r, r + 6);
            }
            for (size_t k = 0; k < a.idx.size(); ++k) {
                int64_t r[6] = {(int64_t)la, -1, 0, 0, a.idx[k], L.dmi[k]};
                out.insert(out.end(), r, r + 6);
            }
        }
    } else if (what == BIE_EXPORT_TRANS) {
        width = 4;
        for (size_t la = 0; la < H->leaves.size(); ++la) {
            const auto &L = H->leaves[la];
            if (!L.adm) continue;
            out.push_back((int64_t)la);
            out.push_back(L.jpiv);
            out.push_back(L.ntr.empty() ? 0 : L.ntr[0]);
            out.push_back(L.qr.empty() ? 0 : (int64_t)L.qr[0].size());
        }
    } else {
        set_error("unknown export selector");
        return BIE_EINVAL;
    }
    const int64_t n = width ? (int64_t)out.size() / width : 0;
    if (rows) *rows = n;
    if (buf && cap > 0) {
        const int64_t m = std::min(cap, n);
        std::memcpy(buf, out.data(), (size_t)m * width * sizeof(int64_t));
    }
    return BIE_OK;
}

}  // namespace bie
