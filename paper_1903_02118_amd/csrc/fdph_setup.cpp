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

// One ACA+ block: piece `kind` (F, S, transient) and stress component
// `comp` of admissible leaf `leaf`, and its factors U [rank][nr], V [rank][ns].
struct AcaBlockH {
    int leaf = 0, kind = 0, comp = 0, rank = 0, sweeps = 0;
    bool fallback = false;
    std::vector<double> U, V;
};

struct FdphHost {
    std::vector<Clu> clu;
    std::vector<LeafH> leaves;
    std::vector<int64_t> near_rows;  // receiver, source, W
    int ncomp = 1;
    std::vector<int> adm_ids;        // admissible leaves
    std::vector<AcaBlockH> blk;      // ACA+ blocks: 3 * ncomp per admissible leaf
};


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
    int sweeps = 0;         // full residual sweeps after the random references stalled
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
        int ip = -1, jp = -1;
        if (vc == 0.0 && vr == 0.0) {
            // both references exhausted: the residual vanishes on them; try fresh ones
            if (++stall <= 3) {
                iref = pick_unused(urow, nr);
                jref = pick_unused(ucol, ns);
                if (iref >= 0 && jref >= 0) {
                    resid_row(iref, rref);
                    resid_col(jref, cref);
                    continue;
                }
            }
            // the random references keep missing the residual (a block whose
            // nonzeros sit in few rows or columns): sweep every unused row,
            // stop if the whole residual meets the tolerance, else pivot on
            // its largest entry
            res.sweeps++;
            double rest2 = 0.0, best = 0.0;
            for (int i = 0; i < nr; ++i) {
                if (urow[i]) continue;
                resid_row(i, r);
                for (int j = 0; j < ns; ++j) {
                    rest2 += r[j] * r[j];
                    if (!ucol[j] && std::fabs(r[j]) > best) {
                        best = std::fabs(r[j]);
                        ip = i;
                        jp = j;
                    }
                }
            }
            if (ip < 0 || std::sqrt(rest2) <= eps * std::sqrt(std::max(norm2, 0.0))) break;
            stall = 0;
            resid_row(ip, r);
            resid_col(jp, c);
        } else if (vc >= vr) {
            stall = 0;
            ip = ic;
            resid_row(ip, r);
            jp = argmax_unused(r, ucol);
            if (jp < 0 || r[jp] == 0.0) {
                urow[ip] = 1;
                continue;
            }
            resid_col(jp, c);
        } else {
            stall = 0;
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
        if (nu * nv <= eps * snorm && rest <= eps * snorm) {
            // before accepting, probe the residual on fresh random rows and
            // columns: partial pivoting can stop on a block whose remaining
            // residual its references miss (a probe above the bound becomes
            // the new reference and the iteration goes on)
            bool pass = true;
            for (int probe = 0; probe < 2 && pass; ++probe) {
                const int ip2 = pick_unused(urow, nr), jp2 = pick_unused(ucol, ns);
                if (ip2 < 0 || jp2 < 0) break;
                resid_row(ip2, r);
                resid_col(jp2, c);
                if (std::max(nrm(c) * std::sqrt((double)ns), nrm(r) * std::sqrt((double)nr)) > eps * snorm) {
                    pass = false;
                    iref = ip2;
                    jref = jp2;
                    rref = r;
                    cref = c;
                }
            }
            if (pass) break;
        }
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

// The FP64 value of the BF16 nearest to v (as bf16_bits rounds).
inline double bf16_round(double v) {
    const uint32_t u = (uint32_t)bf16_bits(v) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
}

// Leading ACA cross terms to store as hi + lo BF16 pairs: the fewest k such
// that the BF16 rounding bound of the terms l >= k, 2^-8 |u_l| |v_l| each
// (two factors of relative error 2^-9), summed in quadrature, is below
// 2^-12 of the block's Frobenius norm (U [rank][nr], V [rank][ns] column-wise).
inline int bf16_split_terms(const std::vector<double> &U, const std::vector<double> &V, int rank, int nr, int ns) {
    if (rank == 0) return 0;
    std::vector<double> t(rank);
    double a2 = 0.0;
    for (int l = 0; l < rank; ++l) {
        double su = 0.0, sv = 0.0;
        for (int i = 0; i < nr; ++i) su += U[(size_t)l * nr + i] * U[(size_t)l * nr + i];
        for (int j = 0; j < ns; ++j) sv += V[(size_t)l * ns + j] * V[(size_t)l * ns + j];
        t[l] = std::sqrt(su * sv);
        for (int m = 0; m < rank; ++m) {
            double cu = 0.0, cv = 0.0;
            for (int i = 0; i < nr; ++i) cu += U[(size_t)l * nr + i] * U[(size_t)m * nr + i];
            for (int j = 0; j < ns; ++j) cv += V[(size_t)l * ns + j] * V[(size_t)m * ns + j];
            a2 += cu * cv;  // |U V^T|_F^2 = sum_lm (U_l . U_m)(V_l . V_m)
        }
    }
    const double bound = std::ldexp(std::sqrt(std::max(a2, 0.0)), -12);
    int k = 0;
    for (; k < rank; ++k) {
        double tail = 0.0;
        for (int l = k; l < rank; ++l) tail += t[l] * t[l];
        if (std::ldexp(std::sqrt(tail), -8) <= bound) break;
    }
    return k;
}

// Entry (il, jl) of the matrix that ACA+ compresses for one piece of an
// admissible leaf, stress component (ex, ey): the Domain-F amplitude over the
// pair's own window (t-, t+) (Eq. 51), the static rate (App. B.1), or the
// transient amplitude (App. H.1): the deviation from the static rate over the
// first step of the pair's Domain S in the same continuous frame, (t+, t+ + dt).
double block_entry(const Geometry &g, const LeafH &L, const Clu &a, const Clu &b, int kind, double ex, double ey,
                   int il, int jl) {
    return far_entry(g.fr[a.idx[il]], g.fr[b.idx[jl]], kind, ex, ey, L.ist[0], L.ist[1], L.mbar[jl], L.dmj[jl], g.dt,
                     g.mu, g.beta);
}

// Seed of the random reference pivots of ACA+ block w.
inline uint64_t aca_seed(const bie_fdph_params &par, int64_t w) {
    return par.seed * 0x9E3779B97F4A7C15ull + (uint64_t)w * 7919u + 1u;
}

}  // namespace

// ---------------------------------------------------------------------------
namespace {

// ACA+ of the listed blocks on the host (OpenMP over blocks), FP64: the
// reference path, and the path of blocks the device could not finish.
void aca_host(FdphPlan &P, const std::vector<int64_t> &which) {
    FdphHost *H = P.host.get();
    const Geometry &g = P.g;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < (int64_t)which.size(); ++q) {
        const int64_t w = which[q];
        AcaBlockH &B = H->blk[w];
        const LeafH &L = H->leaves[B.leaf];
        const Clu &a = H->clu[L.tau], &b = H->clu[L.sigma];
        const int nr = (int)a.idx.size(), ns = (int)b.idx.size();
        const double ex = P.comp[B.comp][0], ey = P.comp[B.comp][1];
        const int kind = B.kind;
        B.rank = 0;
        B.sweeps = 0;
        B.fallback = false;
        B.U.clear();
        B.V.clear();
        if (kind == PIECE_TR && L.ntr[B.comp] == 0) continue;
        auto entry = [&](int il, int jl) -> double { return block_entry(g, L, a, b, kind, ex, ey, il, jl); };
        auto rowf = [&](int il, double *out) {
            for (int jl = 0; jl < ns; ++jl) out[jl] = entry(il, jl);
        };
        auto colf = [&](int jl, double *out) {
            for (int il = 0; il < nr; ++il) out[il] = entry(il, jl);
        };
        AcaResult R = aca_plus(nr, ns, P.par.eps_aca, aca_seed(P.par, w), rowf, colf);
        B.rank = R.rank;
        B.sweeps = R.sweeps;
        B.fallback = R.fallback;
        B.U = std::move(R.U);
        B.V = std::move(R.V);
    }
}

// Far-field layout from the ACA+ factors of every block: receiver weights
// (the projection of the stress component on each receiver normal) folded
// into U and dt into V of the static piece, the storage-precision factors,
// the degenerate waveforms, the rings, the source groups by delay and the
// receiver gather lists.  Fails with BIE_ENOTCONV when a block fell back to
// exact storage and BIE_FLAG_NO_ACA_FALLBACK forbids it.
int pack_far(FdphPlan &P) {
    FdphHost *H = P.host.get();
    const Geometry &g = P.g;
    const auto &clu = H->clu;
    const auto &leaves = H->leaves;
    const auto &comp = P.comp;
    const int NC = P.NC, N = P.N;
    const bool quant = P.quant;
    const double dt = g.dt;
    const bie_fdph_params *par = &P.par;
    const std::vector<int> &adm_ids = H->adm_ids;
    std::vector<AcaBlockH> &blk = H->blk;
    P.aca_sweeps = 0;
    P.bf16_split = 0;
    P.fb_src.clear();
    for (const AcaBlockH &B : blk) {
        P.aca_sweeps += B.sweeps;
        if (B.fallback && (par->flags & BIE_FLAG_NO_ACA_FALLBACK)) {
            set_error("ACA+ did not reach eps_aca before the full rank of a " +
                      std::string(B.kind == PIECE_F ? "Domain-F" : B.kind == PIECE_S ? "Domain-S" : "transient") +
                      " block and the exact fallback is disabled (BIE_FLAG_NO_ACA_FALLBACK)");
            return BIE_ENOTCONV;
        }
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t w = 0; w < (int64_t)blk.size(); ++w) {
        AcaBlockH &B = blk[w];
        if (B.rank == 0) continue;
        const Clu &a = clu[leaves[B.leaf].tau];
        const int nr = (int)a.idx.size();
        const double ex = comp[B.comp][0], ey = comp[B.comp][1];
        for (int l = 0; l < B.rank; ++l)
            for (int il = 0; il < nr; ++il) {
                const Frame &fi = g.fr[a.idx[il]];
                B.U[(size_t)l * nr + il] *= (fi.nx * ex + fi.ny * ey);
            }
        if (B.kind == PIECE_S)
            for (auto &v : B.V) v *= dt;
    }
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
    for (const AcaBlockH &B : blk) {
        if (B.rank == 0) continue;
        const LeafH &L = leaves[B.leaf];
        const Clu &a = clu[L.tau], &b = clu[L.sigma];
        const int nr = (int)a.idx.size(), ns = (int)b.idx.size();
        FarBlock f{};
        f.kind = B.kind;
        f.nr = nr;
        f.ns = ns;
        // BF16 storage: the leading cross terms go as hi + lo BF16 pairs, each
        // term u v^T as uh vh^T + uh vl^T + ul vh^T (three stored columns), so
        // that the rounding bound of the terms left in plain BF16 is 16 times
        // below that of plain BF16 factors
        const int ks = P.precision == BIE_MIXED_BF16 ? bf16_split_terms(B.U, B.V, B.rank, nr, ns) : 0;
        f.rank = B.rank + 2 * ks;
        // factors element-major, ranks contiguous: f[il][l], g[jl][l]
        f.f_off = (int64_t)fdat.size();
        for (int il = 0; il < nr; ++il) {
            for (int l = 0; l < ks; ++l) fdat.push_back(bf16_round(B.U[(size_t)l * nr + il]));
            for (int l = 0; l < ks; ++l) fdat.push_back(bf16_round(B.U[(size_t)l * nr + il]));
            for (int l = 0; l < ks; ++l) {
                const double u = B.U[(size_t)l * nr + il];
                fdat.push_back(bf16_round(u - bf16_round(u)));
            }
            for (int l = ks; l < B.rank; ++l) fdat.push_back(B.U[(size_t)l * nr + il]);
        }
        f.g_off = (int64_t)gdat.size();
        for (int jl = 0; jl < ns; ++jl) {
            for (int l = 0; l < ks; ++l) gdat.push_back(bf16_round(B.V[(size_t)l * ns + jl]));
            for (int l = 0; l < ks; ++l) {
                const double v = B.V[(size_t)l * ns + jl];
                gdat.push_back(bf16_round(v - bf16_round(v)));
            }
            for (int l = 0; l < ks; ++l) gdat.push_back(bf16_round(B.V[(size_t)l * ns + jl]));
            for (int l = ks; l < B.rank; ++l) gdat.push_back(B.V[(size_t)l * ns + jl]);
        }
        P.bf16_split += ks;
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
            // the transient FIRs of a time block run after all its scatters
            f.ring_len = (int32_t)pow2ceil(maxd + dmin + f.ntr + 1 + P.tb);
            // a time block's transient FIRs all run before its gathers
            f.y_len = (int32_t)pow2ceil(dmax - dmin + P.tb);
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
            // live slots: a time block scatters all its steps before its gathers
            f.ring_len = (int32_t)pow2ceil(maxd + dmax + 1 + P.tb);
        }
        f.ring_off = ring_total;
        ring_total += (int64_t)f.rank * f.ring_len;
        const int bid = (int)fb.size();
        fb.push_back(f);
        P.fb_src.push_back({B.leaf, B.comp});
        rank_sum[B.kind] += B.rank;
        rank_max[B.kind] = std::max<int64_t>(rank_max[B.kind], B.rank);
        fallbacks += B.fallback;
        if (B.kind == PIECE_TR)
            for (int l = 0; l < f.rank; ++l) {
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
            G.jl0 = order[p];
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

    // time blocks: the scatter's work items, tiles of each block's slots
    // (delays dmin .. dmax collect at the block's steps 0 .. tb - 1)
    P.scat.clear();
    if (P.tb > 1) {
        size_t gi = 0;
        for (int bid = 0; bid < (int)fb.size(); ++bid) {
            const size_t g0 = gi;
            while (gi < groups.size() && groups[gi].block == bid) ++gi;
            if (gi == g0) continue;
            const int dmin = groups[g0].delay, D = groups[gi - 1].delay - dmin + 1;
            const int U = D + P.tb - 1;
            const int nu = std::max(1, std::min(SCAT_TILE, SCAT_OUT / std::max(1, (int)fb[bid].rank)));
            for (int u0 = 0; u0 < U; u0 += nu) {
                const FarBlock &f = fb[bid];
                ScatItem it{};
                it.kind = f.kind;
                it.rank = f.rank;
                it.ring_len = f.ring_len;
                it.hz = f.hz;
                it.cb = f.kind == PIECE_TR ? f.dm_min + f.ntr + P.tb : P.tb + f.dm_max;
                it.ring_off = f.ring_off;
                it.g_off = f.g_off;
                it.g0 = (int32_t)g0;
                it.ng = (int32_t)(gi - g0);
                it.dmin = dmin;
                it.D = D;
                it.u0 = u0;
                it.nu = std::min(nu, U - u0);
                it.first = u0 == 0 ? 1 : 0;
                P.scat.push_back(it);
            }
        }
    }

    P.fb = std::move(fb);
    P.fdat = std::move(fdat);
    P.gdat = std::move(gdat);
    P.hdat = std::move(hdat);
    P.htrdat = std::move(htrdat);
    P.groups = std::move(groups);
    P.gsrc = std::move(gsrc);
    P.trl = std::move(trl);
    P.qbounds = std::move(qbounds);
    P.qreps = std::move(qreps);
    P.ring_total = ring_total;
    P.y_total = y_total;
    P.qstate_total = qstate_total;
    P.max_dmj = max_dmj;
    for (int k = 0; k < 3; ++k) {
        P.rank_sum[k] = rank_sum[k];
        P.rank_max[k] = rank_max[k];
    }
    P.fallbacks = fallbacks;
    P.re_ptr.assign(N + 1, 0);
    P.re.clear();
    for (int i = 0; i < N; ++i) {
        P.re_ptr[i + 1] = P.re_ptr[i] + (int32_t)recv_entries[i].size();
        P.re.insert(P.re.end(), recv_entries[i].begin(), recv_entries[i].end());
    }
    P.aca_pending = false;
    return BIE_OK;
}

}  // namespace

int plan_fdph(const bie_problem *prob, int count, const bie_fdph_params *par, bie_plan_impl *pl) {
    const auto t_start = std::chrono::steady_clock::now();
    FdphPlan &P = pl->fdph;
    Geometry &g = P.g;
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
    const int tb = par->time_block <= 1 ? 1 : par->time_block;
    if (tb != 1 && tb != TIME_BLOCK) {
        set_error("time_block must be 0, 1 or " + std::to_string(TIME_BLOCK));
        return BIE_EINVAL;
    }
    if (tb > 1 && R > 1) {
        set_error("time blocks need one scenario (n_rhs = 1): several scenarios already share each window pass");
        return BIE_EINVAL;
    }
    P.tb = tb;
    const int N = g.N;
    const double dt = g.dt, cdt = g.beta * g.dt;
    const double tol_abs = par->eps_st * g.mu / (2.0 * g.beta);
    P.par = *par;
    P.count = count;
    P.N = N;
    P.M = M;
    P.quant = quant;
    P.precision = par->precision;
    // several scenarios stage R histories per work item: 64-lag chunks keep
    // two or more workgroups per compute unit (measured: 128 lags for one
    // scenario, 64 for two or four)
    P.near_chunk = R > 1 ? 64 : NEAR_CHUNK_DEFAULT;
    P.R = R;
    if (const char *e = std::getenv("BIE_NEAR_CHUNK")) {  // tuning knob: 64, 128 or 256 (64 or 128 for scenarios)
        const int v = std::atoi(e);
        if (v == 64 || v == 128 || (R == 1 && v == 256)) P.near_chunk = v;
    }
    P.tune.unroll = (P.precision == BIE_FP64) ? 16 : 8;
    if (const char *e = std::getenv("BIE_NEAR_UNROLL")) P.tune.unroll = std::atoi(e) >= 16 ? 16 : 8;
    if (const char *e = std::getenv("BIE_NEAR_LDS_PAD")) P.tune.lds_pad = std::max(0, std::min(65536, std::atoi(e)));
    if (const char *e = std::getenv("BIE_NEAR_WIDE")) P.tune.wide = std::atoi(e) != 0;
    if (const char *e = std::getenv("BIE_NEAR_MFMA")) P.tune.mfma = std::clamp(std::atoi(e), 0, 2);  // time blocks' kernel
    if (const char *e = std::getenv("BIE_FAR_SCATTER_TB")) P.scat_tb = std::atoi(e) != 0;  // tuning knob
    P.host = std::make_shared<FdphHost>();
    FdphHost *H = P.host.get();

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
    P.comp = comp;
    P.fb_src.clear();
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

    // ---- ACA+ blocks: the F, S and transient matrices (per component) ----------
    std::vector<int> &adm_ids = H->adm_ids;
    adm_ids.clear();
    for (size_t a = 0; a < leaves.size(); ++a)
        if (leaves[a].adm) adm_ids.push_back((int)a);
    const int n_pieces = 3 * NC;
    H->blk.assign(adm_ids.size() * n_pieces, AcaBlockH{});
    for (size_t w = 0; w < H->blk.size(); ++w) {
        AcaBlockH &B = H->blk[w];
        B.leaf = adm_ids[w / n_pieces];
        B.kind = (int)(w % n_pieces) / NC;
        B.comp = (int)(w % n_pieces) % NC;
    }
    P.NC = NC;
    P.n_adm = n_adm;
    P.n_inadm = n_inadm;
    P.aca_pending = true;
    if (par->flags & BIE_FLAG_HOST_ACA) {
        std::vector<int64_t> all(H->blk.size());
        std::iota(all.begin(), all.end(), 0);
        const auto t_aca = std::chrono::steady_clock::now();
        aca_host(P, all);
        P.aca_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_aca).count();
        if ((rc = pack_far(P))) return rc;
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
    if (pair_slots > MAX_DISPATCH_ITEMS) {
        set_error("too many near-field pairs for one dispatch");
        return BIE_EINVAL;
    }

    // ---- hand the near-field products to the plan -----------------------------------
    P.tiles = std::move(tiles);
    P.prec = std::move(prec);
    P.psrc = std::move(psrc);
    P.near_pairs = near_pairs;
    P.pair_slots = pair_slots;
    P.horizon = M;
    for (int k = 0; k < count; ++k) P.horizon = std::min<int64_t>(P.horizon, prob[k].n_lags);
    P.windows = false;
    P.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    pl->kind = BIE_KIND_FDPH;
    return BIE_OK;
}

namespace {

// Descriptors of the device ACA+: the leaves' receiver and source indices and
// ART integers, one descriptor per block with work to do (largest first, so
// that the longest blocks start first), and the element counts of the
// factor, residual and flag regions.
struct AcaDevPlan {
    std::vector<AcaLeafDev> leaves;
    std::vector<int32_t> ridx, sidx;
    std::vector<int64_t> mbar, dmj;
    std::vector<AcaBlockDev> blocks;
    std::vector<int64_t> bid;  // host block of each descriptor
    int64_t fac = 0, work = 0, flags = 0;
};

AcaDevPlan aca_dev_plan(const FdphPlan &P) {
    AcaDevPlan A;
    const FdphHost *H = P.host.get();
    std::vector<int> leaf_slot(H->leaves.size(), -1);
    for (int la : H->adm_ids) {
        const LeafH &L = H->leaves[la];
        const Clu &a = H->clu[L.tau], &b = H->clu[L.sigma];
        AcaLeafDev d{};
        d.r_off = (int32_t)A.ridx.size();
        d.nr = (int32_t)a.idx.size();
        d.s_off = (int32_t)A.sidx.size();
        d.ns = (int32_t)b.idx.size();
        d.sx = L.ist[0];
        d.sy = L.ist[1];
        A.ridx.insert(A.ridx.end(), a.idx.begin(), a.idx.end());
        A.sidx.insert(A.sidx.end(), b.idx.begin(), b.idx.end());
        A.mbar.insert(A.mbar.end(), L.mbar.begin(), L.mbar.end());
        A.dmj.insert(A.dmj.end(), L.dmj.begin(), L.dmj.end());
        leaf_slot[la] = (int)A.leaves.size();
        A.leaves.push_back(d);
    }
    for (int64_t w = 0; w < (int64_t)H->blk.size(); ++w) {
        const AcaBlockH &B = H->blk[w];
        const LeafH &L = H->leaves[B.leaf];
        if (B.kind == PIECE_TR && L.ntr[B.comp] == 0) continue;
        A.bid.push_back(w);
    }
    std::stable_sort(A.bid.begin(), A.bid.end(), [&](int64_t x, int64_t y) {
        const AcaLeafDev &lx = A.leaves[leaf_slot[H->blk[x].leaf]], &ly = A.leaves[leaf_slot[H->blk[y].leaf]];
        return (int64_t)lx.nr * lx.ns > (int64_t)ly.nr * ly.ns;
    });
    for (int64_t w : A.bid) {
        const AcaBlockH &B = H->blk[w];
        const AcaLeafDev &lv = A.leaves[leaf_slot[B.leaf]];
        AcaBlockDev d{};
        d.leaf = leaf_slot[B.leaf];
        d.kind = B.kind;
        d.cap = std::min({lv.nr, lv.ns, ACA_KCAP});
        d.ex = P.comp[B.comp][0];
        d.ey = P.comp[B.comp][1];
        d.fac_off = A.fac;
        d.work_off = A.work;
        d.flag_off = A.flags;
        d.seed = aca_seed(P.par, w);
        A.fac += (int64_t)d.cap * (lv.nr + lv.ns);
        A.work += 2ll * (lv.nr + lv.ns);
        A.flags += lv.nr + lv.ns;
        A.blocks.push_back(d);
    }
    return A;
}

// Device arrays of the device stage, carved in a fixed order from one arena
// (a dry arena only sizes them).
struct StageDev {
    Frame *fr = nullptr;
    int32_t *hz = nullptr, *prec = nullptr, *psrc = nullptr, *W = nullptr;
    double *ks = nullptr;
    AcaLeafDev *leaves = nullptr;
    int32_t *ridx = nullptr, *sidx = nullptr;
    int64_t *mbar = nullptr, *dmj = nullptr;
    AcaBlockDev *blocks = nullptr;
    AcaOutDev *out = nullptr;
    double *fac = nullptr, *work = nullptr;
    uint8_t *flags = nullptr;
};

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

int stage_layout(const FdphPlan &P, const AcaDevPlan *A, DevArena &D, StageDev &S, hipStream_t s) {
    int rc;
    if ((rc = D.upload(&S.fr, P.g.fr, s))) return rc;
    if (P.pair_slots > 0) {
        if ((rc = D.upload(&S.hz, P.g.hz, s))) return rc;
        if ((rc = D.upload(&S.prec, P.prec, s))) return rc;
        if ((rc = D.upload(&S.psrc, P.psrc, s))) return rc;
        if ((rc = D.alloc(&S.W, (size_t)P.pair_slots))) return rc;
        if ((rc = D.alloc(&S.ks, (size_t)P.pair_slots))) return rc;
    }
    if (A && !A->blocks.empty()) {
        if ((rc = D.upload(&S.leaves, A->leaves, s))) return rc;
        if ((rc = D.upload(&S.ridx, A->ridx, s))) return rc;
        if ((rc = D.upload(&S.sidx, A->sidx, s))) return rc;
        if ((rc = D.upload(&S.mbar, A->mbar, s))) return rc;
        if ((rc = D.upload(&S.dmj, A->dmj, s))) return rc;
        if ((rc = D.upload(&S.blocks, A->blocks, s))) return rc;
        if ((rc = D.alloc(&S.out, A->blocks.size()))) return rc;
        if ((rc = D.alloc(&S.fac, (size_t)A->fac))) return rc;
        if ((rc = D.alloc(&S.work, (size_t)A->work))) return rc;
        if ((rc = D.alloc(&S.flags, (size_t)A->flags))) return rc;
    }
    return BIE_OK;
}

}  // namespace

// Device scratch of the plan's device stage: the window scan's frames, lag
// counts, pair lists, windows and static rates, and (unless ACA+ ran on the
// host) the ACA+ descriptors, factors, residual vectors and flags.
size_t plan_scratch_bytes(const FdphPlan &P) {
    const bool aca = P.aca_pending;
    if (P.pair_slots == 0 && !aca) return 0;
    AcaDevPlan A;
    if (aca) A = aca_dev_plan(P);
    if (P.pair_slots == 0 && A.blocks.empty()) return 0;
    DevArena D;  // sizing pass
    StageDev S;
    (void)stage_layout(P, aca ? &A : nullptr, D, S, nullptr);
    return D.bytes();
}

namespace {

// Host layout of everything that depends on the windows: the chunk-major
// window regions and work items, the receiver lists of the gather, the
// static tails, the self terms, the ring lengths and the statistics.
void finish_layout(FdphPlan &P) {
    const Geometry &g = P.g;
    const int N = P.N, R = P.R;
    const int NEAR_CHUNK = P.near_chunk;
    const std::vector<NearTile> &tiles = P.tiles;
    const std::vector<int32_t> &W = P.W, &prec = P.prec, &psrc = P.psrc;
    const int64_t pair_slots = P.pair_slots;
    // Chunk-major window layout: a work item is (tile, lag chunk); the chunk
    // segments of all the tile's pairs are stored back to back, each on a
    // 128-byte boundary, so that a work item streams one contiguous region.
    const int64_t align = (P.precision == BIE_FP64) ? 16 : 32;
    std::vector<int32_t> &items = P.items;          // (tile, chunk)
    std::vector<int64_t> &item_base = P.item_base;  // element offset of each item's region
    std::vector<int32_t> &item_rel = P.item_rel;    // [item][TILE*TILE]: segment offset in the region
    std::vector<uint16_t> &item_rng = P.item_rng;   // [item][TILE]: sources [lo, hi) of each receiver with lags in the chunk
    items.clear();
    item_base.clear();
    item_rel.clear();
    item_rng.clear();
    P.tile_item0.assign(tiles.size(), 0);
    P.pTile.assign(pair_slots, 0);
    P.pQ.assign(pair_slots, 0);
    std::vector<std::vector<int32_t>> rn(N);
    std::vector<std::vector<int64_t>> rp(N);
    int64_t near_lags = 0, maxW = 1;
    for (int t = 0; t < (int)tiles.size(); ++t) {
        const NearTile &T = tiles[t];
        const int np = T.nr * T.ns;
        int64_t tw = 0;
        for (int q = 0; q < np; ++q) {
            tw = std::max<int64_t>(tw, W[T.pair_begin + q]);
            P.pTile[T.pair_begin + q] = t;
            P.pQ[T.pair_begin + q] = q;
        }
        maxW = std::max(maxW, tw);
        const int nch = (int)((tw + NEAR_CHUNK - 1) / NEAR_CHUNK);
        P.tile_item0[t] = (int32_t)(items.size() / 2);
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
                // every pair: its window holds the deviation from the static
                // rate, whose static part K^S dt U_n the gather adds
                if (prec[p] >= 0) rp[T.recv[r]].push_back(p);
            }
    }
    P.near_lags = near_lags;
    P.maxW = maxW;
    P.n_items = (int)(items.size() / 2);
    {
        // an alternative workgroup order for the autotuner: items that stage
        // the same source histories (same first source, same lag chunk) go to
        // one XCD (workgroup w runs on XCD w mod 8), groups balanced over XCDs
        constexpr int XCD = 8;
        std::vector<int> ord(P.n_items);
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
        P.perm.assign(len * XCD, -1);
        for (int x = 0; x < XCD; ++x)
            for (size_t k = 0; k < q[x].size(); ++k) P.perm[k * XCD + x] = q[x][k];
        if ((int64_t)P.perm.size() * NEAR_THREADS > MAX_DISPATCH_ITEMS) P.perm.clear();
        P.grid_grouped = (int)P.perm.size();
        // another: the largest work items first (the dispatch runs them in
        // order, so the last wave of workgroups holds the smallest)
        P.perm_size.resize(P.n_items);
        std::iota(P.perm_size.begin(), P.perm_size.end(), 0);
        auto size_of = [&](int it) { return (it + 1 < P.n_items ? item_base[it + 1] : near_lags) - item_base[it]; };
        std::stable_sort(P.perm_size.begin(), P.perm_size.end(),
                         [&](int x, int y) { return size_of(x) > size_of(y); });
        // step index at which the autotuner times the near kernel: every lag
        // chunk active, every problem still running (for every step of a time
        // block, so that each candidate does a block's work)
        P.tune_step = std::max<int64_t>(0, std::min<int64_t>(maxW, P.horizon - P.tb));
    }
    // K_ii,0 per receiver: kept for the coupled step's first-lag solve; in
    // the mixed modes also applied by the gather in FP64 (the FP32 window's
    // own lag-0 value of the self pair keeps only its static part)
    P.self0.assign(N, 0.0);
    P.self_off.clear();
    P.self_ks.clear();
    for (int64_t p = 0; p < pair_slots; ++p)
        if (prec[p] >= 0 && prec[p] == psrc[p] && W[p] > 0) {
            const Frame &f = g.fr[prec[p]];
            P.self0[prec[p]] = proj_kernel(f, f.cx, f.cy, f.nx, f.ny, 0, g.dt, 1.0, g.mu, g.beta);
            const int item0 = P.tile_item0[P.pTile[p]];
            P.self_off.push_back(item_base[item0] + item_rel[(size_t)item0 * TILE * TILE + P.pQ[p]]);
            P.self_ks.push_back(P.ks[p]);
        }
    FdphHost *H = P.host.get();
    H->near_rows.clear();
    H->near_rows.reserve(3 * P.near_pairs);
    for (int64_t p = 0; p < pair_slots; ++p) {
        if (prec[p] < 0) continue;
        H->near_rows.push_back(prec[p]);
        H->near_rows.push_back(psrc[p]);
        H->near_rows.push_back(W[p]);
    }
    // receiver-major partial slots: the near kernel writes (item, r) to the
    // position of that slot in its receiver's list
    P.rn_ptr.assign(N + 1, 0);
    for (int i = 0; i < N; ++i) P.rn_ptr[i + 1] = P.rn_ptr[i] + (int32_t)rn[i].size();
    P.pslot.assign((size_t)std::max(P.n_items, 1) * TILE, -1);
    {
        int32_t k = 0;
        for (int i = 0; i < N; ++i)
            for (int32_t slot : rn[i]) P.pslot[slot] = k++;
    }
    P.n_partial = std::max<int64_t>(P.rn_ptr[N], 1);
    // time blocks: chunk groups for the matrix-core kernel (up to NEAR_GROUP
    // consecutive lag chunks of one tile per work item, one partial sum per
    // receiver and step for the group), their orders and receiver-major slots
    P.grp.clear();
    P.gperm.clear();
    P.gperm_size.clear();
    P.gslot.clear();
    P.rn_ptr_g.clear();
    P.n_grp = P.ggrid_grouped = 0;
    if (P.tb > 1 && P.n_items > 0) {
        std::vector<std::vector<int32_t>> rg(N);
        for (int t = 0; t < (int)tiles.size(); ++t) {
            const int i0 = P.tile_item0[t];
            const int i1 = t + 1 < (int)tiles.size() ? P.tile_item0[t + 1] : P.n_items;
            for (int c = i0; c < i1; c += NEAR_GROUP) {
                const int gi = (int)(P.grp.size() / 2);
                P.grp.push_back(c);
                P.grp.push_back(std::min(NEAR_GROUP, i1 - c));
                for (int r = 0; r < tiles[t].nr; ++r) rg[tiles[t].recv[r]].push_back(gi * TILE + r);
            }
        }
        P.n_grp = (int)(P.grp.size() / 2);
        P.rn_ptr_g.assign(N + 1, 0);
        for (int i = 0; i < N; ++i) P.rn_ptr_g[i + 1] = P.rn_ptr_g[i] + (int32_t)rg[i].size();
        P.gslot.assign((size_t)P.n_grp * TILE, -1);
        int32_t k = 0;
        for (int i = 0; i < N; ++i)
            for (int32_t slot : rg[i]) P.gslot[slot] = k++;
        // the orders of the items, for groups: by (first source, first chunk)
        // onto XCDs, and largest first
        constexpr int XCD = 8;
        std::vector<int> ord(P.n_grp);
        std::iota(ord.begin(), ord.end(), 0);
        auto key = [&](int g) {
            const int it = P.grp[2 * g];
            return std::make_pair(tiles[items[2 * it]].src[0], items[2 * it + 1]);
        };
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
        P.gperm.assign(len * XCD, -1);
        for (int x = 0; x < XCD; ++x)
            for (size_t z = 0; z < q[x].size(); ++z) P.gperm[z * XCD + x] = q[x][z];
        if ((int64_t)P.gperm.size() * NEAR_THREADS > MAX_DISPATCH_ITEMS) P.gperm.clear();
        P.ggrid_grouped = (int)P.gperm.size();
        P.gperm_size.resize(P.n_grp);
        std::iota(P.gperm_size.begin(), P.gperm_size.end(), 0);
        auto gsize = [&](int g) {
            const int a = P.grp[2 * g], e = a + P.grp[2 * g + 1];
            return (e < P.n_items ? item_base[e] : near_lags) - item_base[a];
        };
        std::stable_sort(P.gperm_size.begin(), P.gperm_size.end(), [&](int x, int y) { return gsize(x) > gsize(y); });
    }
    P.rp_ptr.assign(N + 1, 0);
    for (int i = 0; i < N; ++i) P.rp_ptr[i + 1] = P.rp_ptr[i] + (int32_t)rp[i].size();
    P.tails.clear();
    P.tails.reserve(P.rp_ptr[N]);
    for (int i = 0; i < N; ++i)
        for (int64_t p : rp[i]) {
            // with FP32 windows the static rate is rounded as the windows'
            // -K^S dt is, so that lags where K is exactly zero (before the
            // wave, and lag 0 off the diagonal) stay exactly zero
            const double ks = P.precision == BIE_FP64 ? P.ks[p] : (double)(float)P.ks[p];
            P.tails.push_back(TailPair{psrc[p], W[p], ks});
        }

    // ---- histories: ring lengths and scenario strides --------------------------------
    // one slot per lag of the longest window, plus the newer steps of a time
    // block: slots of times before step 0 then still hold zeros
    P.L = (int)pow2ceil(std::max<int64_t>(maxW + P.tb, 2));
    // a time block writes the recent history of all its steps before its FIRs
    P.Lf = (int)pow2ceil(P.max_dmj + P.tb);
    P.scn.D = (int64_t)N * P.L;
    P.scn.U = (int64_t)U_SLOTS * N;
    P.scn.Drec = (int64_t)N * P.Lf;
    P.scn.part = P.n_partial;
    P.scn.ring = std::max<int64_t>(P.ring_total, 1);
    P.scn.y = std::max<int64_t>(P.y_total, 1);
    P.scn.q = std::max<int64_t>(P.qstate_total, 1);
    P.scn.row = (int64_t)R * N;

    // ---- statistics ---------------------------------------------------------------------
    bie_stats &st = P.stats;
    st = bie_stats{};
    st.kind = BIE_KIND_FDPH;
    st.n_elem = N;
    st.n_lags = P.M;
    st.precision = P.precision;
    st.n_adm = P.n_adm;
    st.n_inadm = P.n_inadm;
    st.near_pairs = P.near_pairs;
    int64_t sumW = 0;
    for (int64_t p = 0; p < pair_slots; ++p) sumW += W[p];
    st.near_lags = sumW;
    for (int k = 0; k < 3; ++k) {
        st.rank_sum[k] = P.rank_sum[k];
        st.rank_max[k] = P.rank_max[k];
    }
    st.aca_fallbacks = P.fallbacks;
    st.aca_sweeps = P.aca_sweeps;
    st.aca_host_blocks = P.aca_host_blocks;
    st.time_block = P.tb;
    st.aca_seconds = P.aca_seconds;
    st.scratch_bytes = (int64_t)R * P.n_partial * (int64_t)sizeof(double);
    const double kb = (P.precision == BIE_FP64) ? 8.0 : 4.0;
    const double fb_bytes = (P.precision == BIE_FP64) ? 8.0 : (P.precision == BIE_MIXED_FP32 ? 4.0 : 2.0);
    // near field: the windows, plus one history read per (tile, chunk) source row
    double tile_hist = 0;
    for (int it = 0; it < P.n_items; ++it) tile_hist += (double)tiles[items[2 * it]].ns * NEAR_CHUNK * 8.0;
    st.near_bytes_per_step = (double)sumW * kb;
    double far = 0;
    for (const FarBlock &f : P.fb) {
        far += (double)f.rank * (f.nr + f.ns) * fb_bytes;    // factors
        far += (double)f.rank * (f.nr + f.ns) * 8.0;         // ring reads and updates
        if (f.kind == PIECE_TR) far += (double)f.rank * (f.nq > 0 ? 3.0 * f.nq : (double)f.ntr) * 16.0;  // transient FIR
    }
    for (const GroupSrc &q : P.gsrc) far += (double)q.h_len * 16.0;  // FIR of D
    // the windows are read once for all scenarios; histories and far field per scenario
    st.bytes_per_step = st.near_bytes_per_step + R * (tile_hist + far) + (double)P.near_pairs * 20.0;
    double fl = 2.0 * (double)sumW;
    for (const FarBlock &f : P.fb)
        fl += 2.0 * f.rank * (f.nr + f.ns) + (f.kind == PIECE_TR ? 2.0 * f.rank * (f.nq > 0 ? 2.0 * f.nq : (double)f.ntr) : 0);
    for (const GroupSrc &q : P.gsrc) fl += 2.0 * q.h_len;
    st.flops_per_step = R * fl;
}

}  // namespace

// The plan's device stage, in the caller's scratch: the near-field windows
// W_ij and static rates K^S_ij dt, and (unless ACA+ ran on the host) ACA+ of
// every admissible block, whose factors come back to the host; blocks that
// reached the device rank cap are factored again on the host.  Then the
// far-field layout and the host layout that depends on the windows.
int plan_windows(FdphPlan &P, void *scratch, size_t bytes, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    P.W.assign(P.pair_slots, 0);
    P.ks.assign(P.pair_slots, 0.0);
    const bool aca = P.aca_pending;
    AcaDevPlan A;
    if (aca) A = aca_dev_plan(P);
    int rc;
    if (P.pair_slots > 0 || !A.blocks.empty()) {
        if (!scratch || (uintptr_t)scratch % WS_ALIGN) {
            set_error("bie_plan_windows: the scratch buffer must be a non-null, 256-byte aligned device pointer");
            return BIE_EWORKSPACE;
        }
        DevArena D(scratch, bytes);
        StageDev S;
        if ((rc = stage_layout(P, aca ? &A : nullptr, D, S, s))) return rc;
        EventPair ev;  // device time of the ACA+ kernel
        if (!A.blocks.empty()) {
            BIE_HIP_TRY(hipEventCreate(&ev.a));
            BIE_HIP_TRY(hipEventCreate(&ev.b));
            BIE_HIP_TRY(hipEventRecord(ev.a, s));
            if ((rc = launch_aca(S.fr, S.leaves, S.ridx, S.sidx, S.mbar, S.dmj, S.blocks, (int64_t)A.blocks.size(),
                                 S.fac, S.work, S.flags, S.out, P.g.dt, P.g.mu, P.g.beta, P.par.eps_aca, s)))
                return rc;
            BIE_HIP_TRY(hipEventRecord(ev.b, s));
        }
        if (P.pair_slots > 0) {
            const double tol_abs = P.par.eps_st * P.g.mu / (2.0 * P.g.beta);
            if ((rc = launch_near_windows(P.g, S.fr, S.prec, S.psrc, S.hz, P.pair_slots, P.par.eps_q, tol_abs, S.W,
                                          S.ks, s)))
                return rc;
            BIE_HIP_TRY(hipMemcpyAsync(P.W.data(), S.W, P.pair_slots * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            BIE_HIP_TRY(hipMemcpyAsync(P.ks.data(), S.ks, P.pair_slots * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        std::vector<AcaOutDev> out(A.blocks.size());
        std::unique_ptr<double[]> fac(A.fac > 0 ? new double[(size_t)A.fac] : nullptr);  // left uninitialized
        if (!A.blocks.empty()) {
            BIE_HIP_TRY(hipMemcpyAsync(out.data(), S.out, out.size() * sizeof(AcaOutDev), hipMemcpyDeviceToHost, s));
            BIE_HIP_TRY(hipMemcpyAsync(fac.get(), S.fac, (size_t)A.fac * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        BIE_HIP_TRY(hipStreamSynchronize(s));
        if (aca) {
            const auto t_aca = std::chrono::steady_clock::now();
            float kernel_ms = 0.0f;
            if (ev.a) BIE_HIP_TRY(hipEventElapsedTime(&kernel_ms, ev.a, ev.b));
            FdphHost *H = P.host.get();
            std::vector<int64_t> redo;
            for (size_t q = 0; q < A.blocks.size(); ++q) {
                const AcaBlockDev &d = A.blocks[q];
                const AcaLeafDev &lv = A.leaves[d.leaf];
                AcaBlockH &B = H->blk[A.bid[q]];
                if (out[q].status != ACA_CONVERGED || out[q].rank < 0 || out[q].rank > d.cap) {
                    redo.push_back(A.bid[q]);
                    continue;
                }
                B.rank = out[q].rank;
                B.sweeps = out[q].sweeps;
                B.fallback = false;
                const double *u = fac.get() + d.fac_off, *v = u + (size_t)d.cap * lv.nr;
                B.U.assign(u, u + (size_t)B.rank * lv.nr);
                B.V.assign(v, v + (size_t)B.rank * lv.ns);
            }
            fac.reset();
            aca_host(P, redo);
            P.aca_host_blocks = (int64_t)redo.size();
            // the kernel, then the unpacking of its factors and the host refactoring
            P.aca_seconds = 1e-3 * kernel_ms +
                            std::chrono::duration<double>(std::chrono::steady_clock::now() - t_aca).count();
            if ((rc = pack_far(P))) return rc;
        }
    } else if (aca) {
        if ((rc = pack_far(P))) return rc;
    }
    finish_layout(P);
    if ((int64_t)P.n_items * NEAR_THREADS > MAX_DISPATCH_ITEMS || (int64_t)P.N * 64 > MAX_DISPATCH_ITEMS) {
        set_error("operator too large for one dispatch per step (near-field work items, pairs or receivers)");
        return BIE_EINVAL;
    }
    P.windows = true;
    P.plan_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return BIE_OK;
}

// The operator's device arrays, carved from the arena in a fixed order and
// filled from the plan (a dry arena only sizes them).
int materialize_fdph(const FdphPlan &P, DevArena &A, hipStream_t s, bie_op_impl *op) {
    const auto t0 = std::chrono::steady_clock::now();
    const Geometry &g = P.g;
    const int N = P.N, R = P.R, M = P.M;
    FdphOp &F = op->fdph;
    F.N = N;
    F.M = M;
    F.dt = g.dt;
    F.precision = P.precision;
    F.near_chunk = P.near_chunk;
    F.R = R;
    F.tb = P.tb;
    F.scn = P.scn;
    F.L = P.L;
    F.Lf = P.Lf;
    F.tune = P.tune;
    F.tune.perm = nullptr;
    F.tune_tb = F.tune;
    F.n_tiles = (int)P.tiles.size();
    F.n_pairs = P.pair_slots;
    F.n_items = P.n_items;
    F.near_lags = P.near_lags;
    F.tune_step = P.tune_step;
    F.host = P.host;
    F.quantized = P.quant;
    int rc;
    if ((rc = A.upload(&F.dfr, g.fr, s))) return rc;
    if ((rc = A.upload(&F.hz, g.hz, s))) return rc;
    int32_t *d_prec = nullptr;
    if ((rc = A.upload(&d_prec, P.prec, s))) return rc;
    if ((rc = A.upload(&F.pSrc, P.psrc, s))) return rc;
    if ((rc = A.upload(&F.pW, P.W, s))) return rc;
    if (!P.perm_size.empty())
        if ((rc = A.upload(&F.perm_size, P.perm_size, s))) return rc;
    if (!P.perm.empty()) {
        if ((rc = A.upload(&F.perm_grouped, P.perm, s))) return rc;
        F.grid_grouped = P.grid_grouped;
    }
    if ((rc = A.upload(&F.item_base, P.item_base, s))) return rc;
    if ((rc = A.upload(&F.item_rel, P.item_rel, s))) return rc;
    if ((rc = A.upload(&F.item_rng, P.item_rng, s))) return rc;
    // +64 elements of padding: an empty segment at the very end is read (and
    // ignored) at its offset by the branch-free near kernel
    if (P.precision == BIE_FP64) {
        if ((rc = A.alloc(&F.Kw, P.near_lags + 64))) return rc;
        if (!A.dry) BIE_HIP_TRY(hipMemsetAsync(F.Kw, 0, (P.near_lags + 64) * sizeof(double), s));
    } else {
        if ((rc = A.alloc(&F.Kw32, P.near_lags + 64))) return rc;
        if (!A.dry) BIE_HIP_TRY(hipMemsetAsync(F.Kw32, 0, (P.near_lags + 64) * sizeof(float), s));
    }
    if (P.near_pairs > 0) {
        int32_t *d_ptile = nullptr, *d_pq = nullptr, *d_ti0 = nullptr;
        if ((rc = A.upload(&d_ptile, P.pTile, s))) return rc;
        if ((rc = A.upload(&d_pq, P.pQ, s))) return rc;
        if ((rc = A.upload(&d_ti0, P.tile_item0, s))) return rc;
        double *d_ks = nullptr;  // K^S_ij dt per pair slot: the windows hold K_ij,m - K^S_ij dt
        if ((rc = A.upload(&d_ks, P.ks, s))) return rc;
        if (!A.dry && (rc = launch_near_fill(g, F, d_prec, d_ptile, d_pq, d_ti0, d_ks, s))) return rc;
    }
    if ((rc = A.upload(&F.first_lag, P.self0, s))) return rc;
    if (P.precision != BIE_FP64) {
        if ((rc = A.upload(&F.self0, P.self0, s))) return rc;
        int64_t *d_so = nullptr;
        double *d_sk = nullptr;
        if ((rc = A.upload(&d_so, P.self_off, s))) return rc;
        if ((rc = A.upload(&d_sk, P.self_ks, s))) return rc;
        if (!A.dry && (rc = launch_set_self(F, d_so, d_sk, (int)P.self_off.size(), s))) return rc;
    }
    // per-scenario state: R copies, scenario r at r strides
    if ((rc = A.alloc(&F.Dring, (size_t)R * P.scn.D))) return rc;
    if ((rc = A.alloc(&F.Uring, (size_t)R * P.scn.U))) return rc;
    if ((rc = A.alloc(&F.Drec, (size_t)R * P.scn.Drec))) return rc;
    if ((rc = A.alloc(&F.TS, (size_t)R * N))) return rc;
    if ((rc = A.upload(&F.tiles, P.tiles, s))) return rc;
    if ((rc = A.upload(&F.items, P.items, s))) return rc;
    if ((rc = A.alloc(&F.partial, (size_t)std::max(R, P.tb) * P.scn.part))) return rc;
    if ((rc = A.upload(&F.rn_ptr, P.rn_ptr, s))) return rc;
    if ((rc = A.upload(&F.pslot, P.pslot, s))) return rc;
    F.n_grp = P.n_grp;
    if (F.tune_tb.mfma == 2 && P.n_grp == 0) F.tune_tb.mfma = 1;
    F.grp = F.gperm_grouped = F.gperm_size = F.gslot = F.rn_ptr_g = nullptr;
    F.ggrid_grouped = 0;
    if (P.n_grp > 0) {
        if ((rc = A.upload(&F.grp, P.grp, s))) return rc;
        if ((rc = A.upload(&F.gslot, P.gslot, s))) return rc;
        if ((rc = A.upload(&F.rn_ptr_g, P.rn_ptr_g, s))) return rc;
        if ((rc = A.upload(&F.gperm_size, P.gperm_size, s))) return rc;
        if (!P.gperm.empty()) {
            if ((rc = A.upload(&F.gperm_grouped, P.gperm, s))) return rc;
            F.ggrid_grouped = P.ggrid_grouped;
        }
    }
    if ((rc = A.upload(&F.rp_ptr, P.rp_ptr, s))) return rc;
    if ((rc = A.upload(&F.tails, P.tails, s))) return rc;
    F.n_blocks = (int)P.fb.size();
    F.n_groups = (int)P.groups.size();
    F.n_tr = (int)(P.trl.size() / 2);
    if ((rc = A.upload(&F.blocks, P.fb, s))) return rc;
    if (P.precision == BIE_FP64) {
        if ((rc = A.upload(&F.fdat, P.fdat, s))) return rc;
        if ((rc = A.upload(&F.gdat, P.gdat, s))) return rc;
    } else if (P.precision == BIE_MIXED_FP32) {
        std::vector<float> f32, g32;
        if (!A.dry) {
            f32.assign(P.fdat.begin(), P.fdat.end());
            g32.assign(P.gdat.begin(), P.gdat.end());
            if ((rc = A.upload(&F.fdat32, f32, s))) return rc;
            if ((rc = A.upload(&F.gdat32, g32, s))) return rc;
            BIE_HIP_TRY(hipStreamSynchronize(s));
        } else {
            if ((rc = A.alloc(&F.fdat32, P.fdat.size()))) return rc;
            if ((rc = A.alloc(&F.gdat32, P.gdat.size()))) return rc;
        }
    } else {
        std::vector<uint16_t> f16, g16;
        if (!A.dry) {
            f16.resize(P.fdat.size());
            g16.resize(P.gdat.size());
            for (size_t k = 0; k < P.fdat.size(); ++k) f16[k] = bf16_bits(P.fdat[k]);
            for (size_t k = 0; k < P.gdat.size(); ++k) g16[k] = bf16_bits(P.gdat[k]);
            if ((rc = A.upload(&F.fdat16, f16, s))) return rc;
            if ((rc = A.upload(&F.gdat16, g16, s))) return rc;
            BIE_HIP_TRY(hipStreamSynchronize(s));
        } else {
            if ((rc = A.alloc(&F.fdat16, P.fdat.size()))) return rc;
            if ((rc = A.alloc(&F.gdat16, P.gdat.size()))) return rc;
        }
    }
    if ((rc = A.alloc(&F.rings, (size_t)R * P.scn.ring))) return rc;
    if ((rc = A.alloc(&F.yrings, (size_t)R * P.scn.y))) return rc;
    F.rings_bytes = (size_t)R * P.scn.ring * sizeof(double);
    F.yrings_bytes = (size_t)R * P.scn.y * sizeof(double);
    if (P.quant) {
        if ((rc = A.upload(&F.qbounds, P.qbounds, s))) return rc;
        if ((rc = A.upload(&F.qrep, P.qreps, s))) return rc;
        if ((rc = A.alloc(&F.qstate, (size_t)R * P.scn.q))) return rc;
        F.qstate_bytes = (size_t)R * P.scn.q * sizeof(double);
    }
    if ((rc = A.upload(&F.hdat, P.hdat, s))) return rc;
    if ((rc = A.upload(&F.htr, P.htrdat, s))) return rc;
    if ((rc = A.upload(&F.groups, P.groups, s))) return rc;
    if ((rc = A.upload(&F.gsrc, P.gsrc, s))) return rc;
    F.xs = nullptr;
    F.n_gsrc = (int)P.gsrc.size();
    if (P.tb > 1 && (rc = A.alloc(&F.xs, std::max<size_t>(P.gsrc.size(), 1) * P.tb))) return rc;
    F.n_scat = (int)P.scat.size();
    // one work item per wave: the dispatch's work-item count must fit 32 bits
    F.scat_tb = P.scat_tb && F.n_scat > 0 && (int64_t)P.scat.size() * 64 < ((int64_t)1 << 32);
    if ((rc = A.upload(&F.scat, P.scat, s))) return rc;
    if ((rc = A.upload(&F.tr_list, P.trl, s))) return rc;
    if ((rc = A.upload(&F.re_ptr, P.re_ptr, s))) return rc;
    if ((rc = A.upload(&F.re, P.re, s))) return rc;
    // operator-level buffers: zero input and discarded output of quiescent and
    // predicted steps, the graph step counter, the first-lag terms of coupled
    // runs and the word of the non-finite scan
    // (as many rows as a time block, which quiescent steps also run in)
    const size_t qrows = (size_t)std::max(1, P.tb);
    if ((rc = A.alloc(&op->zero_in, qrows * R * N))) return rc;
    if ((rc = A.alloc(&op->scratch_out, qrows * R * N))) return rc;
    if ((rc = A.alloc(&op->step_dev, 1))) return rc;
    if ((rc = A.alloc(&op->k0, (size_t)R * N))) return rc;
    if ((rc = A.alloc(&op->nonfinite, 1))) return rc;
    if (A.dry) return BIE_OK;
    BIE_HIP_TRY(hipMemsetAsync(op->zero_in, 0, qrows * R * N * sizeof(double), s));
    if (!std::getenv("BIE_NO_SIDE_STREAM")) {  // tuning knob: run everything on one stream
        BIE_HIP_TRY(hipStreamCreateWithFlags(&F.side, hipStreamNonBlocking));
        BIE_HIP_TRY(hipEventCreateWithFlags(&F.ev_fork, hipEventDisableTiming));
        BIE_HIP_TRY(hipEventCreateWithFlags(&F.ev_join, hipEventDisableTiming));
    }
    if ((rc = fdph_reset(op, s))) return rc;
    BIE_HIP_TRY(hipStreamSynchronize(s));
    op->stats = P.stats;
    op->stats.device_bytes = (int64_t)A.bytes();
    op->stats.setup_seconds =
        P.plan_seconds + std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    op->kind = BIE_KIND_FDPH;
    op->N = R * N;  // values per step row of D and T
    op->M = M;
    op->mode = g.mode;
    op->dt = g.dt;
    op->first_lag_diag = g.first_lag_diagonal();
    op->horizon = P.horizon;
    return BIE_OK;
}

// ---------------------------------------------------------------------------
// ACA+ on a caller matrix (diagnostics): rank, exact fallback, residual
// sweeps and the relative Frobenius error of the factorization.
int diag_aca(int nr, int ns, const double *A, double eps, uint64_t seed, int *rank, int *fallback, int *sweeps,
             double *rel_err) {
    auto rowf = [&](int i, double *out) {
        for (int j = 0; j < ns; ++j) out[j] = A[(size_t)i * ns + j];
    };
    auto colf = [&](int j, double *out) {
        for (int i = 0; i < nr; ++i) out[i] = A[(size_t)i * ns + j];
    };
    AcaResult R = aca_plus(nr, ns, eps, seed, rowf, colf);
    double e2 = 0.0, a2 = 0.0;
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < ns; ++j) {
            double v = 0.0;
            for (int l = 0; l < R.rank; ++l) v += R.U[(size_t)l * nr + i] * R.V[(size_t)l * ns + j];
            const double a = A[(size_t)i * ns + j];
            e2 += (a - v) * (a - v);
            a2 += a * a;
        }
    *rank = R.rank;
    *fallback = R.fallback ? 1 : 0;
    *sweeps = R.sweeps;
    *rel_err = a2 > 0.0 ? std::sqrt(e2 / a2) : std::sqrt(e2);
    return BIE_OK;
}

// Exact errors of every low-rank block of a plan (diagnostics): the packed
// factors (receiver projection folded into f, dt into g of the static piece)
// against every entry of the block they approximate, in FP64 and with the
// factors rounded to BF16.
int plan_block_errors(const FdphPlan &P, double *buf, int64_t cap, int64_t *rows) {
    const int64_t nb = (int64_t)P.fb.size();
    if (rows) *rows = nb;
    if (!buf || cap <= 0) return BIE_OK;
    const FdphHost *H = P.host.get();
    const Geometry &g = P.g;
    const int64_t n = std::min(cap, nb);
    auto bf = [](double v) {
        const uint32_t u = (uint32_t)bf16_bits(v) << 16;
        float f;
        std::memcpy(&f, &u, 4);
        return (double)f;
    };
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < n; ++k) {
        const FarBlock &B = P.fb[k];
        const int leaf = P.fb_src[k][0], cc = P.fb_src[k][1];
        const LeafH &L = H->leaves[leaf];
        const Clu &a = H->clu[L.tau], &b = H->clu[L.sigma];
        const double ex = P.comp[cc][0], ey = P.comp[cc][1];
        const double *f = &P.fdat[B.f_off], *gg = &P.gdat[B.g_off];
        double e2 = 0.0, e2b = 0.0, a2 = 0.0;
        std::vector<double> fb16((size_t)B.nr * B.rank), gb16((size_t)B.ns * B.rank);
        for (size_t q = 0; q < fb16.size(); ++q) fb16[q] = bf(f[q]);
        for (size_t q = 0; q < gb16.size(); ++q) gb16[q] = bf(gg[q]);
        for (int il = 0; il < B.nr; ++il) {
            const Frame &fi = g.fr[a.idx[il]];
            const double w = (fi.nx * ex + fi.ny * ey) * (B.kind == PIECE_S ? g.dt : 1.0);
            for (int jl = 0; jl < B.ns; ++jl) {
                const double ent = w * block_entry(g, L, a, b, B.kind, ex, ey, il, jl);
                double v = 0.0, vb = 0.0;
                for (int l = 0; l < B.rank; ++l) {
                    v += f[(size_t)il * B.rank + l] * gg[(size_t)jl * B.rank + l];
                    vb += fb16[(size_t)il * B.rank + l] * gb16[(size_t)jl * B.rank + l];
                }
                e2 += (ent - v) * (ent - v);
                e2b += (ent - vb) * (ent - vb);
                a2 += ent * ent;
            }
        }
        double *r = buf + 8 * k;
        r[0] = leaf;
        r[1] = B.kind;
        r[2] = cc;
        r[3] = B.nr;
        r[4] = B.ns;
        r[5] = B.rank;
        r[6] = a2 > 0 ? std::sqrt(e2 / a2) : std::sqrt(e2);
        r[7] = a2 > 0 ? std::sqrt(e2b / a2) : std::sqrt(e2b);
    }
    return BIE_OK;
}

// ---------------------------------------------------------------------------
int export_fdph(const bie_op_impl *op, int what, int64_t *buf, int64_t cap, int64_t *rows) {
    const FdphHost *H = op->fdph.host.get();
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
