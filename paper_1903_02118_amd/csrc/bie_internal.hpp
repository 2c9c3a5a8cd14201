// Internal declarations of the BIEM convolution library.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/bie.h"
#include "../../include/bie_diag.h"
#include "kernel2d.hpp"

namespace bie {

// ---------------------------------------------------------------- errors --
void set_error(const std::string &msg);

struct Status {
    int code;
    std::string msg;
};

#define BIE_HIP_TRY(expr)                                                                      \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess) {                                                                \
            ::bie::set_error(std::string("HIP error in " #expr ": ") + hipGetErrorString(_e)); \
            return BIE_EHIP;                                                                   \
        }                                                                                      \
    } while (0)

// Device memory of an operator or of the window scan: consecutive 256-byte
// aligned pieces of one caller-owned region.  The library allocates no
// device memory itself.  A sizing pass (dry) only counts the bytes: its
// pointers stay null and nothing is copied.
constexpr size_t WS_ALIGN = 256;
struct DevArena {
    char *base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    bool dry = true;
    DevArena() = default;
    DevArena(void *b, size_t c) : base(static_cast<char *>(b)), cap(c), dry(false) {}
    template <class T>
    int alloc(T **p, size_t count) {
        *p = nullptr;
        if (count == 0) return BIE_OK;
        const size_t off = (used + WS_ALIGN - 1) & ~(WS_ALIGN - 1);
        const size_t bytes = count * sizeof(T);
        if (!dry && (off > cap || bytes > cap - off)) {
            set_error("workspace of " + std::to_string(cap) + " bytes is too small (needs more than " +
                      std::to_string(off + bytes) + ")");
            return BIE_EWORKSPACE;
        }
        used = off + bytes;
        if (!dry) *p = reinterpret_cast<T *>(base + off);
        return BIE_OK;
    }
    template <class T>
    int upload(T **p, const std::vector<T> &v, hipStream_t s) {
        int rc = alloc(p, v.size());
        if (rc) return rc;
        if (!dry && !v.empty()) BIE_HIP_TRY(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
        return BIE_OK;
    }
    size_t bytes() const { return (used + WS_ALIGN - 1) & ~(WS_ALIGN - 1); }
};

// ------------------------------------------------------------- geometry --
struct Geometry {
    int N = 0;
    std::vector<Frame> fr;          // per element frame
    std::vector<double> length;     // element length
    double mu = 1, beta = 1, dt = 0.5, eps_t = 1;
    // independent problems laid end to end (one for a single fault)
    std::vector<int> off;           // [count + 1] first element of each problem
    std::vector<int32_t> hz;        // per element: lag count (horizon) of its problem
    int mode = BIE_MODE_ANTIPLANE;
    double alpha = 0.0;             // P-wave speed (in-plane)
    int build(const bie_problem *p, int count = 1);
    // true when the first lag couples each element only to itself: no
    // collocation point within beta eps_t dt of another element of its
    // problem (anti-plane; the S front has not reached it at the first
    // collocation time)
    bool first_lag_diagonal() const;
};

// ------------------------------------------------------------ dense form --
// The plain form keeps, per lag m and receiver i, only the causal band of
// sources: the contiguous range [lo, lo + w) of element indices that holds
// every source whose nearest point the fastest wave has reached by
// t_m = (m + eps_t) dt (K_ij,m is exactly zero outside it).  Band rows are
// stored back to back, lag-major: row (m, i) at off[m * N + i].
struct DenseOp {
    Frame *dfr = nullptr;           // device copy of the element frames
    int N = 0, M = 0, L = 0;        // L: history ring length (power of two >= M)
    int ncomp = 1;                  // 1 (anti-plane) or 2 (in-plane: shear, normal)
    int lag_chunk = 0, n_chunks = 0;
    int V = 1;                      // 2: band rows start and end on even sources (16-byte loads)
    int64_t E = 0;                  // band entries per component
    double *K = nullptr;            // [ncomp][E]
    int64_t *off = nullptr;         // [M * N + 1] start of each band row
    int32_t *blo = nullptr;         // [M * N] first source of each band row
    double *hist = nullptr;         // [ncomp][L][N], slot = t & (L-1)
    double *partial = nullptr;      // [ncomp][n_chunks][N]
};

// Step index of a per-step launch.  Eager launches carry it by value; a
// captured step (HIP graph, replayed once per step) reads it from a device
// counter that the step's last node advances.  Inputs and outputs of step n
// sit at (n - n0) rows past the base pointers handed to the launch.
struct StepIdx {
    int64_t n = 0;                  // eager: the step
    const int64_t *dev = nullptr;   // replayed graph: device step counter
    int64_t n0 = 0;                 // step of the base pointers' first row
    int64_t off = 0;                // replayed graph: this step's offset from the counter (time blocks)
    __host__ __device__ int64_t get() const {
#if defined(__HIP_DEVICE_COMPILE__)
        return dev ? *dev + off : n;
#else
        return n;
#endif
    }
};

// Steps of a time block (prescribed-slip runs: the near field of TIME_BLOCK
// consecutive steps in one pass over the windows, the 16 columns of the
// matrix-core products).  The block kernels that keep registers per step
// (lane-per-lag near field, far-field inputs, gathers) take it in launches of
// SUB_BLOCK steps.
constexpr int TIME_BLOCK = BIE_TIME_BLOCK;
constexpr int SUB_BLOCK = 8;
static_assert(TIME_BLOCK % SUB_BLOCK == 0, "whole sub-blocks");
// Slots of the running slip sum U (a ring of its last values): a time block
// updates U for all its steps before the gathers read them.
constexpr int U_SLOTS = 2 * TIME_BLOCK;
static_assert((U_SLOTS & (U_SLOTS - 1)) == 0 && U_SLOTS > TIME_BLOCK, "power of two beyond a block");

// Entry of the matrix that ACA+ compresses for one piece of an admissible
// leaf (host and device), receiver frame fi, source frame fj, stress
// component (ex, ey), representative receiver point (sx, sy), the source's
// receiver-averaged travel-time step mbar and Domain-F duration dm:
//   Domain F: the amplitude over the pair's own window (t-, t+) (Eq. 51);
//   Domain S: the static rate (App. B.1);
//   transient: the deviation from the static rate over the first step after
//   the window, (t+, t+ + dt), in the pair's own time frame (App. H.1).
__host__ __device__ inline double far_entry(const Frame &fi, const Frame &fj, int kind, double ex, double ey,
                                            double sx, double sy, int64_t mbar, int64_t dm, double dt, double mu,
                                            double beta) {
    if (kind == 1) return proj_static(fj, fi.cx, fi.cy, ex, ey, mu);
    const double rij = sqrt((fi.cx - fj.cx) * (fi.cx - fj.cx) + (fi.cy - fj.cy) * (fi.cy - fj.cy));
    const double rsj = sqrt((fj.cx - sx) * (fj.cx - sx) + (fj.cy - sy) * (fj.cy - sy));
    const double tp = rij / beta + ((double)(mbar + dm) * dt - rsj / beta);
    if (kind == 0) {
        const double tm = rij / beta - (rsj / beta - (double)mbar * dt);
        return proj_step(fj, fi.cx, fi.cy, ex, ey, tp, mu, beta) - proj_step(fj, fi.cx, fi.cy, ex, ey, tm, mu, beta);
    }
    return proj_step(fj, fi.cx, fi.cy, ex, ey, tp + dt, mu, beta) - proj_step(fj, fi.cx, fi.cy, ex, ey, tp, mu, beta) -
           proj_static(fj, fi.cx, fi.cy, ex, ey, mu) * dt;
}

// ACA+ of the admissible blocks on the device, one workgroup per block
// (Sec. 6.1.1, FP64).  A leaf's receivers and sources are frame indices; a
// block is one piece (F, S or transient) and stress component of a leaf.
struct AcaLeafDev {
    int32_t r_off, nr;  // receivers: ridx[r_off, r_off + nr)
    int32_t s_off, ns;  // sources: sidx, mbar, dmj at [s_off, s_off + ns)
    double sx, sy;      // representative receiver point of the leaf
};
struct AcaBlockDev {
    int32_t leaf, kind;
    int32_t cap;        // rank columns stored (at most min(nr, ns))
    int32_t reserved;
    double ex, ey;      // stress component
    int64_t fac_off;    // U [cap][nr] then V [cap][ns], doubles
    int64_t work_off;   // residual vectors r [ns], c [nr], reference r [ns], c [nr], doubles
    int64_t flag_off;   // used rows [nr] then used columns [ns], bytes
    uint64_t seed;      // of the random reference pivots
};
struct AcaOutDev {
    int32_t rank, status, sweeps, reserved;
};
enum { ACA_CONVERGED = 0, ACA_CAPPED = 1 };
constexpr int ACA_KCAP = 32;  // rank columns a block stores on the device
int launch_aca(const Frame *fr, const AcaLeafDev *leaves, const int32_t *ridx, const int32_t *sidx,
               const int64_t *mbar, const int64_t *dmj, const AcaBlockDev *blocks, int64_t n_blocks, double *fac,
               double *work, uint8_t *flags, AcaOutDev *out, double dt, double mu, double beta, double eps,
               hipStream_t s);

// A dispatch counts its work-items in 32 bits: grids whose size is data
// dependent either stride (at most this many workgroups) or are checked
// against MAX_DISPATCH_ITEMS at setup.
constexpr int64_t MAX_GRID_BLOCKS = 1 << 20;
constexpr int64_t MAX_DISPATCH_ITEMS = (int64_t(1) << 32) - 1;

// -------------------------------------------------------------- FDP=H ----
constexpr int TILE = 32;            // receivers / sources per near-field tile
constexpr int NEAR_CHUNK_DEFAULT = 128;  // lags per near-field work item (64, 128 or 256)
constexpr int NEAR_THREADS = 512;        // work-items per near-field workgroup
constexpr int NEAR_GROUP = 4;            // time blocks: lag chunks per work item of the grouped matrix-core kernel

enum Piece { PIECE_F = 0, PIECE_S = 1, PIECE_TR = 2 };

// One low-rank block of an admissible leaf for one piece and component.
struct FarBlock {
    int32_t kind;       // Piece
    int32_t rank;
    int32_t nr, ns;
    int64_t f_off;      // f factors [nr][rank] (receiver weight folded in)
    int64_t g_off;      // g factors [ns][rank] (dt folded in for PIECE_S)
    int64_t ring_off;   // F, S: rings [ring_len][rank]; PIECE_TR: u rings [rank][ring_len]
    int32_t ring_len;   // power of two
    int32_t dm_max;     // max receiver shift dm_i of the leaf
    int32_t dm_min;
    int32_t ntr;        // PIECE_TR: transient length
    int64_t y_off;      // PIECE_TR: y rings [y_len][rank]
    int32_t y_len;      // power of two
    int32_t hz;         // lag count of the block's problem: no work at steps >= hz
    int64_t htr_off;    // PIECE_TR: transient waveform (ntr values)
    int32_t nq;         // PIECE_TR, staircase: number of runs (0 = plain FIR)
    int32_t pad1;
    int64_t qb_off;     // staircase run starts (nq + 1 ints) in qbounds
    int64_t qr_off;     // staircase run values (nq doubles) in qrep
    int64_t qs_off;     // running sums [rank][nq] in qstate
};

// Source-side work item: sources of one block sharing one delay.
struct SrcGroup {
    int32_t block;
    int32_t delay;      // mbar_j (F) or mbar_j + dm_j (S, transient)
    int32_t first;      // into the group-source list
    int32_t count;
    int32_t clear;      // 1: this item clears the stale ring slot of its block
    int32_t jl0;        // local index of its first source (column of g)
};

// Scatter of a time block: one work item per (far block, tile of ring slots).
// Slot u of the block (absolute slot n + dmin + u of the block's first step n)
// collects the groups of delay dmin + u - k at step k of the block.
struct ScatItem {
    int32_t g0, ng;     // the block's groups (contiguous, by increasing delay)
    int32_t dmin, D;    // smallest group delay; delays span [dmin, dmin + D)
    int32_t u0, nu;     // the tile: slots u0 .. u0 + nu - 1
    int32_t first;      // 1: the block's first tile (clears the ring slots no tile owns)
    // the block's own fields (no read of its record)
    int32_t kind, rank, ring_len, hz;
    int32_t cb;         // step n clears slot n - cb: tb + dm_max (F, S), dm_min + ntr + tb (transient)
    int64_t ring_off, g_off;
};
constexpr int SCAT_TILE = 256;    // slots per tile at most
constexpr int SCAT_OUT = 512;     // (slot, rank) outputs per tile at most

struct GroupSrc {
    int32_t j;          // global source index
    int32_t jl;         // local index in the block (column of g)
    int32_t h_len;      // PIECE_F: FIR length dm_j; else 0
    int32_t pad;
    int64_t h_off;      // PIECE_F: offset of h_{a,j,0..}
};

// Receiver-side entry: one block seen by one receiver, with everything the
// gather needs (no access to the block record).
struct RecvEntry {
    int32_t kind;       // Piece
    int32_t rank;       // the block's rank: ring slot stride
    int32_t dm;         // receiver shift dm_i
    int32_t mask;       // ring length - 1 (F, S rings; transient y rings)
    int64_t f_off;      // this entry's factors: f_off + l
    int64_t r_off;      // ring base (rings for F, S; yrings for the transient) + first rank of the entry
    int32_t cnt;        // ranks of this entry: a block of high rank is split over several
    int32_t pad;
};
constexpr int RECV_SPLIT = 16;  // ranks per gather entry

// Static tail of one near pair, in its receiver's list.
struct TailPair {
    int32_t src;        // source element
    int32_t w;          // window W_ij (the near windows hold K_ij,m - K^S_ij dt below it)
    double ks;          // K^S_ij dt
};

struct NearTile {
    int32_t nr, ns;
    int32_t recv[TILE];
    int32_t src[TILE];
    int64_t pair_begin;     // pairs (r, s) at pair_begin + r*ns + s
    int32_t hz;             // lag count of the tile's problem
    int32_t pad;
};

struct FdphHost;  // host-side setup products (kept for export)

// Scenarios sharing one FDP=H operator: scenario r's state sits r strides past
// the base of each array, and its values in a step row of D and T at r * N.
struct Scn {
    int64_t D = 0;      // Dring: N * L
    int64_t U = 0;      // running slip sum: 2 * N
    int64_t Drec = 0;   // N * Lf
    int64_t ring = 0;   // F and S rings and transient u rings
    int64_t y = 0;      // transient y rings
    int64_t q = 0;      // staircase running sums
    int64_t part = 0;   // near partial sums
    int64_t row = 0;    // values per step row of D and T: R * N
};

// Launch configuration of the near-field kernel (set at setup, changed by the
// autotuner).
struct NearTune {
    int unroll = 16;                // source-loop unroll (8 or 16)
    int wide = 1;                   // 1: window loads of twice the narrow width per lane (16 bytes, else 8)
    int lds_pad = 0;                // unused LDS per workgroup: caps workgroups per CU
    int order = 0;                  // 0: items in build order; 1: grouped by sources per XCD; 2: largest first
    int mfma = 1;                   // time blocks: 1 the matrix-core kernel, 2 the same with chunk groups, 0 the lane-per-lag one
    int grid = 0;                   // workgroups when perm is set
    const int32_t *perm = nullptr;  // workgroup -> item (-1: padding), or null
};

struct FdphOp {
    Frame *dfr = nullptr;           // device copy of the element frames
    int N = 0, M = 0;
    int L = 0;              // near history ring (power of two > max W)
    int Lf = 0;             // recent history ring for the far FIR (power of two)
    int precision = BIE_FP64;
    int near_chunk = NEAR_CHUNK_DEFAULT;
    int R = 1;                  // scenarios (slip-rate histories) sharing the operator
    int tb = 1;                 // steps per time block of bie_run / bie_run_graph (1: none)
    Scn scn;                    // their strides
    NearTune tune;              // near-kernel launch configuration (single steps)
    NearTune tune_tb;           // the same for time blocks
    int32_t *perm_grouped = nullptr;  // item order grouped by source slice and XCD
    int grid_grouped = 0;
    int32_t *perm_size = nullptr;     // item order by size, largest first
    // time blocks, matrix-core kernel with chunk groups (NearTune::mfma == 2):
    // a work item is up to NEAR_GROUP consecutive lag chunks of one tile
    int n_grp = 0;
    int32_t *grp = nullptr;           // [n_grp][2]: first item, items
    int32_t *gperm_grouped = nullptr; // group orders, as the item orders above
    int ggrid_grouped = 0;
    int32_t *gperm_size = nullptr;
    int32_t *gslot = nullptr;         // [n_grp][TILE] slot in `partial` of (group, tile receiver)
    int32_t *rn_ptr_g = nullptr;      // [N+1] receiver i owns [rn_ptr_g[i], rn_ptr_g[i+1]) of the groups' slots
    int64_t tune_step = 0;      // step index used when timing near-kernel variants
    double dt = 0.5;

    // histories
    double *Dring = nullptr;    // [N][L], slot (-t) & (L-1)
    double *Drec = nullptr;     // [Lf][N], slot t & (Lf-1)
    double *Uring = nullptr;    // [U_SLOTS][N] running sum of D, slot t & (U_SLOTS-1) (U_t = U_{t-1} + D_t)

    // near field
    int n_tiles = 0;
    NearTile *tiles = nullptr;
    int64_t n_pairs = 0;
    int32_t *pW = nullptr;      // window per pair
    int32_t *pSrc = nullptr;    // source of each pair
    double *Kw = nullptr;       // FP64 windows
    float *Kw32 = nullptr;      // FP32 windows (mixed precision)
    int n_items = 0;
    int64_t near_lags = 0;      // window elements; the 64 after them are zero
    int32_t *items = nullptr;   // [n_items][2] (tile, chunk)
    int64_t *item_base = nullptr;  // [n_items] start of the item's window region in Kw
    int32_t *item_rel = nullptr;   // [n_items][TILE*TILE] segment offset of each pair
    uint16_t *item_rng = nullptr;  // [n_items][TILE] lo | hi << 8: sources of each receiver with lags in the chunk
    double *partial = nullptr;  // near partial sums, receiver-major: receiver i owns [rn_ptr[i], rn_ptr[i+1]);
                                // max(R, tb) copies (scenario or step of a time block) at scn.part strides
    int32_t *pslot = nullptr;   // [n_items][TILE] slot in `partial` of (item, tile receiver)
    int32_t *rn_ptr = nullptr;  // [N+1]
    // near pairs with a static tail (W_ij below the lag count), receiver-major
    int32_t *rp_ptr = nullptr;  // [N+1]
    TailPair *tails = nullptr;

    // far field
    int n_blocks = 0;
    FarBlock *blocks = nullptr;
    double *fdat = nullptr, *gdat = nullptr;
    float *fdat32 = nullptr, *gdat32 = nullptr;
    uint16_t *fdat16 = nullptr, *gdat16 = nullptr;  // BF16 bit patterns
    double *rings = nullptr;    // F and S rings, transient u rings
    double *yrings = nullptr;   // transient y rings
    size_t rings_bytes = 0, yrings_bytes = 0;
    double *hdat = nullptr;     // degenerate waveforms
    double *htr = nullptr;      // transient waveforms
    int n_groups = 0;
    SrcGroup *groups = nullptr;
    GroupSrc *gsrc = nullptr;
    double *xs = nullptr;       // time blocks: source inputs of the block's steps, [tb][group source]
    int n_gsrc = 0;             // group sources (a row of xs)
    ScatItem *scat = nullptr;   // time blocks: the scatter's work items
    int n_scat = 0;
    bool scat_tb = true;        // time blocks: one scatter launch per block (else one per step)
    int32_t *tr_list = nullptr; // [n_tr][2] (block, rank) of transient blocks
    int n_tr = 0;
    int32_t *re_ptr = nullptr;  // [N+1]
    RecvEntry *re = nullptr;

    // staircase transient (BIE_FLAG_QUANTIZE_TRANSIENT)
    int32_t *qbounds = nullptr;
    double *qrep = nullptr;
    double *qstate = nullptr;
    size_t qstate_bytes = 0;
    bool quantized = false;

    int32_t *hz = nullptr;      // [N] lag count of each receiver's problem
    double *TS = nullptr;       // [N] running Domain-S stress (FP64)
    double *self0 = nullptr;    // [N] FP64 self term K_ii,0 (mixed precision only)
    double *first_lag = nullptr; // [N] K_ii,0 of every receiver (all precisions)

    // side stream (default priority) for the far-field source side
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool side_pending = false;  // side-stream work recorded in ev_join that no step has joined

    std::shared_ptr<const FdphHost> host;  // tree and integer setup data (exports)
};

// Event pairs around the dominant kernel of each step (optional).
struct KernelTimer {
    static constexpr int CAP = 16384;
    bool enabled = false;
    std::vector<hipEvent_t> start, stop;
    int used = 0;
    int begin(hipStream_t s);       // returns the pair index or -1
    void end(int k, hipStream_t s);
    void release();
};

// ------------------------------------------------------------------ plans --
// Host products of the plain form's plan (bie_plan_dense).
struct DensePlan {
    Geometry g;
    int N = 0, M = 0, L = 0, ncomp = 1;
    int lag_chunk = 0, n_chunks = 0;
    int V = 1;
    std::vector<int32_t> blo;       // [M * N] causal band of each (lag, receiver)
    std::vector<int64_t> off;       // [M * N + 1]
};

// Host products of the FDP=H plan (bie_plan_fdph), completed by the window
// scan (bie_plan_windows): everything the operator holds, in host memory, and
// the sizes of its device arrays.
struct FdphPlan {
    Geometry g;
    bie_fdph_params par{};
    int count = 1;
    int N = 0, M = 0, R = 1, NC = 1;
    int precision = BIE_FP64;
    int near_chunk = NEAR_CHUNK_DEFAULT;
    bool quant = false;
    NearTune tune;
    int64_t horizon = 0;            // smallest lag count of the problems
    std::shared_ptr<FdphHost> host;
    // far field (FP64 factors; converted to the storage precision on upload)
    std::vector<std::array<double, 2>> comp;  // stress components (one: the traction of a planar fault)
    std::vector<FarBlock> fb;
    std::vector<std::array<int, 2>> fb_src;   // per block: leaf, component
    std::vector<double> fdat, gdat, hdat, htrdat;
    std::vector<SrcGroup> groups;
    std::vector<GroupSrc> gsrc;
    std::vector<ScatItem> scat;
    bool scat_tb = true;
    std::vector<int32_t> trl;
    std::vector<int32_t> re_ptr;
    std::vector<RecvEntry> re;
    std::vector<int32_t> qbounds;
    std::vector<double> qreps;
    int64_t ring_total = 0, y_total = 0, qstate_total = 0, max_dmj = 1;
    int64_t rank_sum[3] = {0, 0, 0}, rank_max[3] = {0, 0, 0}, fallbacks = 0, aca_sweeps = 0;
    int64_t bf16_split = 0;         // BF16 storage: cross terms kept as hi + lo pairs
    int tb = 1;                     // steps per time block (1: none)
    bool aca_pending = true;        // ACA+ factors not computed yet (device ACA+ runs in bie_plan_windows)
    int64_t aca_host_blocks = 0;    // blocks factored on the host after the device reached their rank cap
    double aca_seconds = 0.0;       // wall time of ACA+ (device kernel and transfers, or host)
    int64_t n_adm = 0, n_inadm = 0;
    // near field: tiles and pair slots (placeholders between packed sub-blocks: prec = -1)
    std::vector<NearTile> tiles;
    std::vector<int32_t> prec, psrc;
    int64_t near_pairs = 0, pair_slots = 0;
    // after the window scan
    bool windows = false;
    std::vector<int32_t> W;         // per pair slot
    std::vector<double> ks;         // K^S_ij dt per pair slot
    std::vector<int32_t> items, item_rel, tile_item0, pTile, pQ, perm, rn_ptr, pslot, rp_ptr;
    std::vector<int64_t> item_base, self_off;
    std::vector<uint16_t> item_rng;
    std::vector<double> self0;
    std::vector<double> self_ks;    // K^S_ii dt of the self pairs at self_off
    std::vector<TailPair> tails;
    int64_t near_lags = 0, maxW = 1, n_partial = 1;
    int n_items = 0, grid_grouped = 0;
    std::vector<int32_t> perm_size;
    std::vector<int32_t> grp, gperm, gperm_size, gslot, rn_ptr_g;  // chunk groups (time blocks)
    int n_grp = 0, ggrid_grouped = 0;
    int64_t tune_step = 0;
    int L = 2, Lf = 2;
    Scn scn;
    bie_stats stats{};
    double plan_seconds = 0.0;
};

struct bie_plan_impl {
    int kind = 0;                   // BIE_KIND_DENSE or BIE_KIND_FDPH
    DensePlan dense;
    FdphPlan fdph;
};

struct bie_op_impl {
    int kind = 0;
    int N = 0, M = 0;
    int64_t step = 0;
    int64_t *step_dev = nullptr;    // device step counter of captured steps
    hipGraphExec_t graph_exec = nullptr;  // last captured step (bie_run_graph)
    hipStream_t graph_stream = nullptr;
    const double *graph_D = nullptr;      // inputs, outputs and first step of the cached graph
    double *graph_T = nullptr;
    int64_t graph_n0 = -1;
    int64_t graph_steps = 0;              // steps per launch of the cached graph
    hipStream_t cap_stream = nullptr;     // capture stream (default priority)
    KernelTimer timer;
    double *zero_in = nullptr;      // [N] zeros (advance, predict)
    double *scratch_out = nullptr;  // [N] discarded tractions (advance)
    int64_t *nonfinite = nullptr;   // first (step * N + index) with a non-finite traction (debug scan)
    bool scan_finite = false;
    // coupled stepping (predict / commit)
    int mode = BIE_MODE_ANTIPLANE;
    double dt = 0.5;
    bool first_lag_diag = false;
    int64_t horizon = INT64_MAX;    // steps the operator's problems all run (FDP=H: smallest lag count)
    bool predicted = false;         // a predict of the current step awaits its commit
    double *k0 = nullptr;           // [N] K_ii,0 (rupture runs)
    bool k0_ready = false;
    DevArena arena;                 // the caller's workspace
    DenseOp dense;
    FdphOp fdph;
    bie_stats stats{};
};

// plans (host) and operators inside a caller workspace, returning BIE_* codes
int plan_dense(const bie_problem *p, bie_plan_impl *pl);
int plan_fdph(const bie_problem *p, int count, const bie_fdph_params *q, bie_plan_impl *pl);
size_t plan_scratch_bytes(const FdphPlan &P);
int plan_windows(FdphPlan &P, void *scratch, size_t bytes, hipStream_t s);
// A is dry (sizing) or holds the workspace; op receives the device arrays
int materialize_dense(const DensePlan &P, DevArena &A, hipStream_t s, bie_op_impl *op);
int materialize_fdph(const FdphPlan &P, DevArena &A, hipStream_t s, bie_op_impl *op);
int export_fdph(const bie_op_impl *op, int what, int64_t *buf, int64_t cap, int64_t *rows);
bie_stats dense_stats(const DensePlan &D);
int workspace_bytes(const bie_plan_impl *pl, size_t *bytes);
int fdph_steps_ok(const bie_op_impl *op, int64_t steps, const char *who);
int static_scratch_ptr(double **out);
int diag_aca(int nr, int ns, const double *A, double eps, uint64_t seed, int *rank, int *fallback, int *sweeps,
             double *rel_err);
int plan_block_errors(const FdphPlan &P, double *buf, int64_t cap, int64_t *rows);
int launch_scan_finite(const double *t, int64_t row, const StepIdx &si, int64_t *word, hipStream_t s);

// per-step launchers (si.dev set: launches for a captured step)
// (advance = false: the step's traction is computed but the step counter
// stays, for a predict that its commit completes)
int dense_step(bie_op_impl *op, const double *d, double *t, hipStream_t s, const StepIdx &si, bool advance = true);
int fdph_step(bie_op_impl *op, const double *d, double *t, hipStream_t s, const StepIdx &si, bool advance = true);
// The op->fdph.tb steps starting at si (a time block of a prescribed-slip
// run): D rows of all of them in, T rows out, the near field in one pass.
int fdph_block(bie_op_impl *op, const double *d, double *t, hipStream_t s, const StepIdx &si);
// commit of a predicted step: D_n into the history (and the far-field rings)
int dense_commit(bie_op_impl *op, const double *d, hipStream_t s);
int fdph_commit(bie_op_impl *op, const double *d, hipStream_t s);
int fdph_join_side(bie_op_impl *op, hipStream_t s);
int launch_first_lag(const bie_op_impl *op, double *k0, hipStream_t s);
int launch_friction(int N, const bie_friction &fr, double dt, const double *t0, const double *k0, double *slip,
                    int32_t *state, double *t, double *d, hipStream_t s);
int launch_step_advance(int64_t *n_dev, hipStream_t s, int64_t by = 1);
int launch_step_set(int64_t *n_dev, int64_t value, hipStream_t s);
int dense_reset(bie_op_impl *op, hipStream_t s);
int dense_advance(bie_op_impl *op, int64_t steps, hipStream_t s);
int fdph_reset(bie_op_impl *op, hipStream_t s);
int launch_near(const FdphOp &F, const NearTune &c, hipStream_t s, const StepIdx &si);
int launch_near_tb(const FdphOp &F, const NearTune &c, hipStream_t s, const StepIdx &si);
int fdph_autotune(bie_op_impl *op, int reps, hipStream_t s, bie_tune *out);
size_t near_lds_bytes(const FdphOp &F, bool mfma);

// device setup kernels (fdph_kernels.hip)
int launch_near_windows(const Geometry &g, const Frame *dfr, const int32_t *d_prec, const int32_t *d_psrc,
                        const int32_t *d_hz, int64_t n_pairs, double eps_q, double eps_st_abs, int32_t *d_W,
                        double *d_ks, hipStream_t s);
int launch_near_fill(const Geometry &g, const FdphOp &f, const int32_t *d_prec, const int32_t *d_ptile,
                     const int32_t *d_pq, const int32_t *d_tile_item0, const double *d_ks, hipStream_t s);
int launch_set_self(const FdphOp &f, const int64_t *d_self_off, const double *d_self_ks, int n_self, hipStream_t s);
int launch_dense_build(const Geometry &g, const DenseOp &d, hipStream_t s);
int launch_first_lag_dense(const DenseOp &d, double *k0, hipStream_t s);

inline int ilog2ceil(int64_t v) {
    int k = 0;
    while ((int64_t(1) << k) < v) ++k;
    return k;
}

}  // namespace bie

struct bie_op : public bie::bie_op_impl {};
struct bie_plan : public bie::bie_plan_impl {};
