// dmm.hip - host orchestration of Dual_MM (dm_solve_discrete) and its small kernels.
//
// Paper: Sec. 2.3 (Alg. Dual_MM, dual decomposition and the lower bound of
// eq. DD-dual), App. A.3.2 (iterative minorant).  The chain sweep kernels are in
// dmm_kernels.h; each (lanes, labels-per-lane) tile is compiled in its own unit.
#include <hip/hip_fp16.h>

#include <map>
#include <mutex>
#include <tuple>

#include "dmm_adjoint.h"
#include "dmm_hier.h"
#include "tiles.h"

namespace dm {

#define DM_EXTERN_TILE(g, l)                                                            \
    extern template hipError_t launch_tile<g, l>(const SweepArgs&, dm_dtype, hipStream_t); \
    extern template hipError_t launch_adjoint_tile<g, l, false>(const AdjArgs&, dm_dtype, hipStream_t); \
    extern template hipError_t launch_adjoint_tile<g, l, true>(const AdjArgs&, dm_dtype, hipStream_t);
DM_FOR_EACH_TILE(DM_EXTERN_TILE)
#undef DM_EXTERN_TILE

// ------------------------------------------------------------------ small kernels
__global__ void fill_f32_kernel(float* __restrict__ p, long long n, float v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void copy_f32_kernel(const float* __restrict__ a, float* __restrict__ b, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) b[i] = a[i];
}

// Lower-bound adjoint of one chain family's optima at a dual lambda: the derivative of a
// chain optimum with respect to its unaries is the one-hot of its (unique) optimal
// labeling `lab`, and with respect to an edge weight the truncated distance of the two
// labels.  Rows have unaries cost - lambda (cost gets +g, dual -g), columns lambda (+g).
__global__ void lb_inject_kernel(const int* __restrict__ lab, int W, int H, int K, int T, const double* __restrict__ gp,
                                 int rows, float* __restrict__ lbar, float* __restrict__ gcost, double* __restrict__ gw) {
    const double g = gp[0];
    const long long n = (long long)W * H;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        const int l = min(max(lab[p], 0), K - 1);
        const int x = (int)(p % W), y = (int)(p / W);
        if (rows) {
            lbar[p * K + l] -= (float)g;
            gcost[p * K + l] += (float)g;
            if (x + 1 < W) {
                const int d = abs(l - min(max(lab[p + 1], 0), K - 1));
                gw[(long long)y * (W - 1) + x] += g * (double)(d < T ? d : T);
            }
        } else {
            lbar[p * K + l] += (float)g;
            if (y + 1 < H) {
                const int d = abs(l - min(max(lab[p + W], 0), K - 1));
                gw[p] += g * (double)(d < T ? d : T);
            }
        }
    }
}

// Adjoint of the energy of the output labeling, E(x) = sum_i cost_i(x_i) + sum_edges w rho(x_i - x_j):
// the labels are piecewise constant in the inputs, so dE/dcost is the one-hot of x and
// dE/dw the truncated label distance of each edge.
__global__ void energy_adjoint_kernel(const int* __restrict__ lab, int W, int H, int K, int T,
                                      const double* __restrict__ gp, float* __restrict__ gcost,
                                      double* __restrict__ gwh, double* __restrict__ gwv) {
    const double g = gp[1];
    const long long n = (long long)W * H;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        const int l = min(max(lab[p], 0), K - 1);
        const int x = (int)(p % W), y = (int)(p / W);
        gcost[p * K + l] += (float)g;
        if (x + 1 < W) {
            const int d = abs(l - min(max(lab[p + 1], 0), K - 1));
            gwh[(long long)y * (W - 1) + x] += g * (double)(d < T ? d : T);
        }
        if (y + 1 < H) {
            const int d = abs(l - min(max(lab[p + W], 0), K - 1));
            gwv[p] += g * (double)(d < T ? d : T);
        }
    }
}

__global__ void zero_f64_kernel(double* __restrict__ p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void edge_out_kernel(const double* __restrict__ acc, long long n, int accumulate, float* __restrict__ out) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = (accumulate ? out[i] : 0.0f) + (float)acc[i];
}

// Per-block FP64 partial sums of the grid energy, fixed order.
template <typename TT>
__global__ __launch_bounds__(256) void energy_partial_kernel(const TT* __restrict__ theta, const float* __restrict__ w_h,
                                                             const float* __restrict__ w_v, const int* __restrict__ lab,
                                                             int W, int H, int K, int T, double* __restrict__ partial) {
    __shared__ double sh[256];
    double acc = 0.0;
    const long long npx = (long long)W * H;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(p / W), x = (int)(p % W);
        const int l = min(max(lab[p], 0), K - 1);
        acc += (double)to_f<TT>(theta[p * K + l]);
        if (x + 1 < W) {
            int d = abs(l - min(max(lab[p + 1], 0), K - 1));
            acc += (double)w_h[(long long)y * (W - 1) + x] * (double)(d < T ? d : T);
        }
        if (y + 1 < H) {
            int d = abs(l - min(max(lab[p + W], 0), K - 1));
            acc += (double)w_v[p] * (double)(d < T ? d : T);
        }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__device__ double block_sum(const double* __restrict__ v, int n, double* sh) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += v[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Lower bound after each half-step k = 0..S-1 (one block per k):
//   slot k holds the chain optima of half-step k's family (k even: H rows, odd: W columns),
//   slot S the row optima of the final pass, slot S+1 the column optima of a final column pass.
// After half-step k the bound is (optimum of the family just updated, preserved by the
// exact minorant) + (optimum of the other family, recorded by the next pass over it).
__global__ __launch_bounds__(256) void lb_trace_kernel(const double* __restrict__ opt, long long max_chains, int S,
                                                       int H, int W, double* __restrict__ trace) {
    __shared__ double sh[256];
    const int k = blockIdx.x;
    if (k >= S) return;
    const int count_a = (k % 2 == 0) ? H : W;
    int slot_b = k + 1, count_b;
    if (k == S - 1 && (S % 2) == 1) {
        slot_b = S + 1;  // last half-step horizontal: pair with the final column pass
        count_b = W;
    } else if (slot_b == S) {
        count_b = H;
    } else {
        count_b = (slot_b % 2 == 0) ? H : W;
    }
    double a = block_sum(opt + (long long)k * max_chains, count_a, sh);
    double b = block_sum(opt + (long long)slot_b * max_chains, count_b, sh);
    if (threadIdx.x == 0) trace[k] = a + b;
}

// bounds[0] = sum(slot a) + sum(slot b); bounds[1] = sum of energy partials.
__global__ __launch_bounds__(256) void bounds_kernel(const double* __restrict__ opt, long long max_chains, int slot_a,
                                                     int count_a, int slot_b, int count_b,
                                                     const double* __restrict__ partial, int n_partial,
                                                     double* __restrict__ bounds) {
    __shared__ double sh[256];
    double a = block_sum(opt + (long long)slot_a * max_chains, count_a, sh);
    double b = block_sum(opt + (long long)slot_b * max_chains, count_b, sh);
    double e = block_sum(partial, n_partial, sh);
    if (threadIdx.x == 0) {
        bounds[0] = a + b;
        bounds[1] = e;
    }
}

// ------------------------------------------------------------------ host side
namespace {

struct Tile {
    int G, LPL;
};

// Tiles compiled into the library; a chain of K labels needs G*LPL >= K.
#define DM_TILE_ENTRY(g, l) {g, l},
constexpr Tile kTiles[] = {DM_FOR_EACH_TILE(DM_TILE_ENTRY)};
#undef DM_TILE_ENTRY

bool tile_compiled(int G, int LPL) {
    for (const Tile& t : kTiles)
        if (t.G == G && t.LPL == LPL) return true;
    return false;
}

// Default tile: the smallest compiled tile that holds K labels (fewest idle lanes),
// preferring exact fits.
Tile default_tile(int K) {
    Tile best{64, 4};
    int best_waste = 1 << 30;
    for (const Tile& t : kTiles) {
        const int cap = t.G * t.LPL;
        if (cap < K) continue;
        const int waste = cap - K;
        if (waste < best_waste || (waste == best_waste && t.G > best.G)) {
            best = t;
            best_waste = waste;
        }
    }
    return best;
}

Tile row_tile(const dm_shape& s, const dm_discrete_params& p) {
    return p.tile_lanes != 0 ? Tile{p.tile_lanes, p.labels_per_lane} : default_tile(s.K);
}
Tile col_tile(const dm_shape& s, const dm_discrete_params& p) {
    return p.tile_lanes_v != 0 ? Tile{p.tile_lanes_v, p.labels_per_lane_v} : row_tile(s, p);
}

hipError_t launch_sweep(Tile t, const SweepArgs& a, dm_dtype dt, hipStream_t st) {
#define DM_TILE_CASE(g, l) \
    if (t.G == g && t.LPL == l) return launch_tile<g, l>(a, dt, st);
    DM_FOR_EACH_TILE(DM_TILE_CASE)
#undef DM_TILE_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint(Tile t, const AdjArgs& a, dm_dtype dt, hipStream_t st) {
#define DM_TILE_CASE(g, l)                                                                          \
    if (t.G == g && t.LPL == l)                                                                     \
        return a.tape[0] != nullptr ? launch_adjoint_tile<g, l, true>(a, dt, st)                    \
                                    : launch_adjoint_tile<g, l, false>(a, dt, st);
    DM_FOR_EACH_TILE(DM_TILE_CASE)
#undef DM_TILE_CASE
    return hipErrorInvalidValue;
}

// Algorithmic HBM bytes of one sweep launch: what the passes must read and write per
// label-node (cost b bytes, dual / messages / min-marginals 4 bytes), times the labels.
double sweep_bytes(const SweepArgs& a, dm_dtype dt) {
    const double b = a.theta != nullptr ? (dt == DM_F16 ? 2.0 : 4.0) : 0.0;
    const double nodes = (double)a.n * a.n_chains * a.K;
    double per = 0.0;
    // record mode (dual checkpoints with every pass's messages) also stores the last
    // pass's messages; tape mode instead writes every pass's tape
    const bool tape = (a.mode & kRecordFlag) && a.tape[0] != nullptr;
    const double rec = ((a.mode & kRecordFlag) && !tape) ? 4.0 : 0.0;
    if (tape) {
        const int P = (a.mode & ~kRecordFlag) == kModeIterative ? a.n_pass : 1;
        per += (P + 1) * (double)a.tape_px / a.K;
    }
    switch (a.mode & ~kRecordFlag) {
        case kModeIterative:
            per += b + 8.0 + rec;                          // R0: cost, dual; message out
            for (int s = 0; s < a.n_pass; ++s) per += (s < a.n_pass - 1) ? b + 16.0 : b + 12.0;
            break;
        case kModeNaive: per += (b + 8.0) + (b + 12.0) + rec; break;
        case kModeOptimum: per = b + 4.0; break;
        case kModeFinal: per = (b + 8.0) + (b + 8.0) + (a.minmarg != nullptr ? 4.0 : 0.0); break;
        default: break;
    }
    return per * nodes + (a.mode == kModeFinal ? 4.0 * a.n * a.n_chains : 0.0);
}

// Algorithmic HBM bytes of one adjoint launch (per label-node: what its passes read and
// write; cost b bytes, every other volume 4).
double adjoint_bytes(const AdjArgs& a, dm_dtype dt) {
    const bool theta = a.theta != nullptr;
    const double b = theta ? (dt == DM_F16 ? 2.0 : 4.0) : 0.0;
    const double nodes = (double)a.n * a.n_chains * a.K;
    // kind: 0 R0, 1 update, 3 final; first: the half-step's last update pass
    const bool tape = a.tape[0] != nullptr;
    auto pass = [&](int kind, bool first, bool has_bin) {
        // cost, dual, carried and reverse messages (recomputing form) or the tape
        double x = tape ? (double)a.tape_px / a.K : b + 8.0 + (kind != 0 ? 4.0 : 0.0);
        if (kind != 3) x += 4.0;                                  // dual adjoint in
        if (has_bin) x += 4.0;                                    // stored-message adjoint in
        const bool gx = kind == 3 || (theta && (first || kind == 0));
        if (gx) x += 4.0;                                         // dL/dcost or dL/dminmarg in
        x += 4.0;                                                 // dual adjoint out
        if (kind != 0) x += 4.0;                                  // reverse-message adjoint out
        if (theta && (first || kind == 0)) x += 4.0;              // dL/dcost out
        return x;
    };
    double per = 0.0;
    if (a.mode == kModeFinal) {
        per = pass(3, false, false) + pass(0, false, true);
    } else {
        const int P = a.mode == kModeIterative ? a.n_pass : 1;
        for (int s = P; s >= 1; --s) per += pass(1, s == P, s < P);
        per += pass(0, false, true);
    }
    return per * nodes;
}

hipError_t launch_sweep_prof(Tile t, const SweepArgs& a, dm_dtype dt, hipStream_t st) {
    int kind = DM_PROF_SWEEP_H;
    if (a.mode == kModeFinal) kind = DM_PROF_SWEEP_FINAL;
    else if (a.mode == kModeOptimum) kind = DM_PROF_SWEEP_OPT;
    else if (a.mode & kRecordFlag) kind = a.theta != nullptr ? DM_PROF_RECORD_H : DM_PROF_RECORD_V;
    else if (a.theta == nullptr) kind = DM_PROF_SWEEP_V;
    ProfScope ps(kind, profiler_on() ? sweep_bytes(a, dt) : 0.0, st);
    return launch_sweep(t, a, dt, st);
}

struct WsLayout {
    size_t msg, msg2, opt, partial, labels, ckpt, total;  // msg2: hierarchical minorant only
    size_t vol_bytes;
    long long max_chains;
    int n_slots, n_partial;
    size_t slab_bytes;  // kept per half-step
    bool tape;          // the selections are kept as tapes
    size_t tape_bytes;  // bytes of one tape
};

// Update passes of a half-step (the adjoint's P).
int pass_count(const dm_discrete_params& p) { return p.minorant == DM_MINORANT_ITERATIVE ? p.max_pass : 1; }

// Volumes kept per half-step: none; its input dual (checkpoint, messages recomputed in the
// backward); or its input dual, the messages of every pass (P + 1) and the duals after
// update passes 1 .. P-1 (recorded in the forward, no recompute).
int slab_volumes(const dm_discrete_params& p) {
    if (p.keep_checkpoints == 1) return 1;
    if (p.keep_checkpoints == 2) return 1 + (pass_count(p) + 1) + (pass_count(p) - 1);
    return 0;
}

// Tape bytes per pixel of a tile, and whether the tape form covers its distance
// transform (the truncation reaches at most one lane across).
size_t tape_px_bytes(Tile t) { return (size_t)t.G * kTapeWords(t.LPL) * 4; }
bool tape_tile_ok(Tile t, int T) {
    const int need = (T - 1 + t.LPL - 1) / t.LPL;
    return (need < t.G - 1 ? need : t.G - 1) <= 1;
}
// The backward reads selection tapes instead of recomputing the selections when both
// families' tiles allow it, the caller did not ask for recomputation and one tape fits
// the 32-bit buffer range.  Returns the bytes of one tape (0: no tapes).
size_t tape_bytes_for(const dm_shape& s, const dm_discrete_params& p) {
    if (p.recompute_selections) return 0;
    const Tile r = row_tile(s, p), c = col_tile(s, p);
    if (!tape_tile_ok(r, p.trunc_T) || !tape_tile_ok(c, p.trunc_T)) return 0;
    const size_t px = tape_px_bytes(r) > tape_px_bytes(c) ? tape_px_bytes(r) : tape_px_bytes(c);
    const size_t b = align_up((size_t)s.W * s.H * px, 256);
    return b <= kMaxVolBytes ? b : 0;
}

constexpr int kEnergyBlocks = 1024;

int half_step_count(const dm_discrete_params& p) { return p.n_half_steps > 0 ? p.n_half_steps : 2 * p.n_iters; }

WsLayout layout(const dm_shape& s, const dm_discrete_params& p) {
    WsLayout L{};
    const size_t vol = (size_t)s.W * s.H * s.K;
    const int S = half_step_count(p);
    L.max_chains = s.W > s.H ? s.W : s.H;
    L.n_slots = S + 2;
    L.n_partial = kEnergyBlocks;
    size_t off = 0;
    L.msg = off;
    off = align_up(off + vol * sizeof(float), 256);
    L.msg2 = off;  // messages from the right of the hierarchical minorant
    if (p.minorant == DM_MINORANT_HIERARCHICAL) off = align_up(off + vol * sizeof(float), 256);
    L.opt = off;
    off = align_up(off + (size_t)L.n_slots * L.max_chains * sizeof(double), 256);
    L.partial = off;
    off = align_up(off + (size_t)L.n_partial * sizeof(double), 256);
    L.labels = off;
    off = align_up(off + (size_t)s.W * s.H * sizeof(int), 256);
    L.vol_bytes = align_up(vol * sizeof(float), 256);
    L.ckpt = off;
    L.tape_bytes = tape_bytes_for(s, p);
    L.tape = L.tape_bytes != 0;
    // per half-step: its input dual, plus (keep_checkpoints 2) every pass's tape or its
    // messages and intermediate duals
    if (p.keep_checkpoints == 2 && L.tape)
        L.slab_bytes = L.vol_bytes + (size_t)(pass_count(p) + 1) * L.tape_bytes;
    else
        L.slab_bytes = (size_t)slab_volumes(p) * L.vol_bytes;
    off += (size_t)S * L.slab_bytes;
    L.total = off;
    return L;
}

int validate_params(const dm_shape& s, const dm_discrete_params* p) {
    int st = validate_shape(s);
    if (st != DM_OK) return st;
    DM_REQUIRE(p != nullptr, DM_ERR_NULL, "params is NULL");
    DM_REQUIRE(p->n_iters >= 0 && p->n_iters <= 100000, DM_ERR_PARAM, "n_iters=%d out of range", p->n_iters);
    DM_REQUIRE(p->n_half_steps >= 0 && p->n_half_steps <= 200000, DM_ERR_PARAM, "n_half_steps=%d out of range",
               p->n_half_steps);
    DM_REQUIRE(p->trunc_T >= 1, DM_ERR_PARAM, "trunc_T=%d must be >= 1", p->trunc_T);
    DM_REQUIRE(p->minorant == DM_MINORANT_ITERATIVE || p->minorant == DM_MINORANT_NAIVE ||
                   p->minorant == DM_MINORANT_HIERARCHICAL,
               DM_ERR_PARAM, "unknown minorant %d", p->minorant);
    DM_REQUIRE(p->minorant != DM_MINORANT_HIERARCHICAL || p->keep_checkpoints == 0, DM_ERR_UNSUPPORTED,
               "the hierarchical minorant has no backward: keep_checkpoints must be 0");
    if (p->minorant == DM_MINORANT_ITERATIVE) {
        DM_REQUIRE(p->max_pass >= 1 && p->max_pass <= 8, DM_ERR_PARAM, "max_pass=%d out of range [1, 8]", p->max_pass);
        for (int i = 0; i < p->max_pass; ++i)
            DM_REQUIRE(p->gamma[i] > 0.0f && p->gamma[i] <= 1.0f, DM_ERR_PARAM, "gamma[%d]=%g not in (0, 1]", i,
                       (double)p->gamma[i]);
        DM_REQUIRE(p->gamma[p->max_pass - 1] == 1.0f, DM_ERR_PARAM,
                   "gamma[max_pass-1] must be 1 for a maximal minorant (got %g)", (double)p->gamma[p->max_pass - 1]);
    }
    DM_REQUIRE(p->warm_start == 0 || p->warm_start == 1, DM_ERR_PARAM, "warm_start must be 0 or 1");
    DM_REQUIRE(p->keep_checkpoints >= 0 && p->keep_checkpoints <= 2, DM_ERR_PARAM, "keep_checkpoints must be 0, 1 or 2");
    DM_REQUIRE(p->recompute_selections == 0 || p->recompute_selections == 1, DM_ERR_PARAM,
               "recompute_selections must be 0 or 1");
    if (p->tile_lanes != 0 || p->labels_per_lane != 0) {
        DM_REQUIRE(tile_compiled(p->tile_lanes, p->labels_per_lane), DM_ERR_UNSUPPORTED,
                   "tile %d lanes x %d labels is not compiled in", p->tile_lanes, p->labels_per_lane);
        DM_REQUIRE(p->tile_lanes * p->labels_per_lane >= s.K, DM_ERR_PARAM, "tile %dx%d holds fewer than K=%d labels",
                   p->tile_lanes, p->labels_per_lane, s.K);
    }
    if (p->tile_lanes_v != 0 || p->labels_per_lane_v != 0) {
        DM_REQUIRE(tile_compiled(p->tile_lanes_v, p->labels_per_lane_v), DM_ERR_UNSUPPORTED,
                   "column tile %d lanes x %d labels is not compiled in", p->tile_lanes_v, p->labels_per_lane_v);
        DM_REQUIRE(p->tile_lanes_v * p->labels_per_lane_v >= s.K, DM_ERR_PARAM,
                   "column tile %dx%d holds fewer than K=%d labels", p->tile_lanes_v, p->labels_per_lane_v, s.K);
    }
    return DM_OK;
}

}  // namespace

}  // namespace dm

using namespace dm;

extern "C" size_t dm_solve_discrete_workspace(dm_shape s, dm_dtype cost_dtype, const dm_discrete_params* p) {
    (void)cost_dtype;
    if (validate_params(s, p) != DM_OK) return 0;
    return layout(s, *p).total;
}

extern "C" int dm_solve_discrete(const void* cost, dm_dtype cost_dtype, const float* w_h, const float* w_v, dm_shape s,
                                 const dm_discrete_params* p, int32_t* labels_out, float* minmarg_out,
                                 float* dual_inout, double* bounds_out, double* lb_trace_out, void* workspace,
                                 size_t workspace_bytes, void* hip_stream) {
    clear_error();
    int st = validate_params(s, p);
    if (st != DM_OK) return st;
    DM_REQUIRE(cost_dtype == DM_F32 || cost_dtype == DM_F16, DM_ERR_DTYPE, "unknown cost dtype %d", (int)cost_dtype);
    DM_REQUIRE(cost != nullptr && dual_inout != nullptr, DM_ERR_NULL, "cost and dual_inout are required");
    DM_REQUIRE(s.W == 1 || w_h != nullptr, DM_ERR_NULL, "w_h is required when W > 1");
    DM_REQUIRE(s.H == 1 || w_v != nullptr, DM_ERR_NULL, "w_v is required when H > 1");
    const WsLayout L = layout(s, *p);
    DM_REQUIRE(workspace != nullptr && workspace_bytes >= L.total, DM_ERR_WORKSPACE,
               "workspace %zu bytes, need %zu", workspace_bytes, L.total);
    DM_REQUIRE(((uintptr_t)cost % 16) == 0 && ((uintptr_t)dual_inout % 16) == 0 &&
                   ((uintptr_t)minmarg_out % 16) == 0 && ((uintptr_t)workspace % 256) == 0,
               DM_ERR_PARAM, "cost, dual and min-marginal volumes need 16-byte alignment, workspace 256");
    {
        hipError_t e = hipGetLastError();  // surface a sticky error from earlier work
        if (e != hipSuccess) {
            set_error("pending HIP error before dm_solve_discrete: %s", hipGetErrorString(e));
            return DM_ERR_HIP;
        }
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    char* ws = static_cast<char*>(workspace);
    float* msg = reinterpret_cast<float*>(ws + L.msg);
    double* opt = reinterpret_cast<double*>(ws + L.opt);
    double* partial = reinterpret_cast<double*>(ws + L.partial);
    int* labels = labels_out != nullptr ? labels_out : reinterpret_cast<int*>(ws + L.labels);

    const Tile tile = row_tile(s, *p), tile_v = col_tile(s, *p);
    const long long vol = (long long)s.W * s.H * s.K;
    DM_REQUIRE(vol * 4 < (long long)kOOB, DM_ERR_UNSUPPORTED, "volume of %lld labels exceeds the 4 GiB buffer range", vol);
    const int S = half_step_count(*p);
    // With checkpoints, half-step k reads the dual from ckpt[k] and writes ckpt[k+1] (the
    // last one writes dual_inout): the checkpoints cost no extra traffic.
    float* ckpt0 = reinterpret_cast<float*>(ws + L.ckpt);
    auto slab_vol = [&](int k, int i) {
        return reinterpret_cast<float*>(ws + L.ckpt + (size_t)k * L.slab_bytes + (size_t)i * L.vol_bytes);
    };
    auto slab_tape = [&](int k, int i) {
        return reinterpret_cast<unsigned*>(ws + L.ckpt + (size_t)k * L.slab_bytes + L.vol_bytes +
                                           (size_t)i * L.tape_bytes);
    };
    auto ckpt = [&](int k) { return slab_vol(k, 0); };
    const int P = pass_count(*p);
    const bool record = p->keep_checkpoints == 2;
    const bool use_ckpt = p->keep_checkpoints && S > 0;
    if (use_ckpt) {
        ProfScope ps(DM_PROF_OTHER, 8.0 * vol, stream);
        if (p->warm_start)
            hipLaunchKernelGGL(copy_f32_kernel, dim3(2048), dim3(256), 0, stream, dual_inout, ckpt0, vol);
        else
            hipLaunchKernelGGL(fill_f32_kernel, dim3(2048), dim3(256), 0, stream, ckpt0, vol, 0.0f);
        DM_HIP_TRY(hipGetLastError(), "init checkpoint");
    } else if (!p->warm_start) {
        ProfScope ps(DM_PROF_OTHER, 4.0 * vol, stream);
        hipLaunchKernelGGL(fill_f32_kernel, dim3(2048), dim3(256), 0, stream, dual_inout, vol, 0.0f);
        DM_HIP_TRY(hipGetLastError(), "fill dual");
    }

    SweepArgs rows{};
    rows.theta = cost;
    rows.lam = dual_inout;
    rows.msg = msg;
    rows.w = w_h;
    rows.chain_px = s.W;
    rows.node_px = 1;
    rows.w_chain = s.W - 1;
    rows.w_node = 1;
    rows.vol_bytes_f32 = (unsigned)(vol * 4);
    rows.vol_bytes_theta = (unsigned)(vol * (cost_dtype == DM_F16 ? 2 : 4));
    rows.w_bytes = (unsigned)((long long)s.H * (s.W - 1) * 4);
    rows.K = s.K;
    rows.n = s.W;
    rows.n_chains = s.H;
    rows.T = p->trunc_T;
    rows.sign = 1.0f;
    rows.inv_n = 1.0f / (float)s.W;
    rows.n_pass = p->max_pass;
    for (int i = 0; i < 8; ++i) rows.gamma[i] = p->gamma[i];
    rows.mode = p->minorant == DM_MINORANT_NAIVE ? kModeNaive : kModeIterative;

    SweepArgs cols = rows;
    cols.theta = nullptr;
    cols.w = w_v;
    cols.w_bytes = (unsigned)((long long)(s.H - 1) * s.W * 4);
    cols.chain_px = 1;
    cols.node_px = s.W;
    cols.w_chain = 1;
    cols.w_node = s.W;
    cols.n = s.H;
    cols.n_chains = s.W;
    cols.sign = -1.0f;
    cols.inv_n = 1.0f / (float)s.H;

    const bool want_bounds = bounds_out != nullptr || lb_trace_out != nullptr;
    for (int k = 0; k < S; ++k) {
        SweepArgs a = (k % 2 == 0) ? rows : cols;
        a.opt = want_bounds ? opt + (long long)k * L.max_chains : nullptr;
        if (use_ckpt) {
            a.lam_in = ckpt(k);
            a.lam = (k + 1 < S) ? ckpt(k + 1) : dual_inout;
        }
        if (record && L.tape) {
            // every pass's selection tape into the half-step's slab; messages and duals
            // in place as in the plain half-step
            a.mode |= kRecordFlag;
            for (int i = 0; i < 9; ++i) a.rec_msg[i] = msg;
            for (int i = 0; i < 8; ++i) a.rec_lam[i] = a.lam;
            for (int i = 0; i <= P && i < 9; ++i) a.tape[i] = slab_tape(k, i);
            a.tape_bytes = (unsigned)L.tape_bytes;
            a.tape_px = (unsigned)tape_px_bytes(k % 2 == 0 ? tile : tile_v);
        } else if (record) {
            // every pass's messages and intermediate duals into the half-step's slab
            a.mode |= kRecordFlag;
            for (int i = 0; i <= P && i < 9; ++i) a.rec_msg[i] = slab_vol(k, 1 + i);
            for (int i = 1; i < P && i < 8; ++i) a.rec_lam[i] = slab_vol(k, P + 1 + i);
        }
        if (p->minorant == DM_MINORANT_HIERARCHICAL) {
            ProfScope ps(k % 2 == 0 ? DM_PROF_SWEEP_H : DM_PROF_SWEEP_V,
                         profiler_on() ? hier_half_step_bytes(a, cost_dtype) : 0.0, stream);
            DM_HIP_TRY(launch_hier_half_step(a, reinterpret_cast<float*>(ws + L.msg2), cost_dtype, stream),
                       "hierarchical half-step launch");
            continue;
        }
        DM_HIP_TRY(launch_sweep_prof(k % 2 == 0 ? tile : tile_v, a, cost_dtype, stream), "half-step launch");
    }
    // Final row pass: normalized min-marginals of F, labels, row optima (slot S).
    {
        SweepArgs a = rows;
        a.mode = kModeFinal;
        a.minmarg = minmarg_out;
        a.labels = labels;
        a.opt = want_bounds ? opt + (long long)S * L.max_chains : nullptr;
        DM_HIP_TRY(launch_sweep_prof(tile, a, cost_dtype, stream), "final pass launch");
    }
    if (want_bounds) {
        // G's optimum: preserved from the last vertical half-step if that was the last
        // half-step, else measured by a column message pass into slot S+1.
        int slot_g = S - 1;
        if (S == 0 || (S % 2) == 1) {
            SweepArgs a = cols;
            a.mode = kModeOptimum;
            a.opt = opt + (long long)(S + 1) * L.max_chains;
            DM_HIP_TRY(launch_sweep_prof(tile_v, a, cost_dtype, stream), "column optimum launch");
            slot_g = S + 1;
        }
        ProfScope ps(DM_PROF_BOUNDS, (double)s.W * s.H * ((cost_dtype == DM_F16 ? 2 : 4) + 12), stream);
        if (bounds_out != nullptr) {
            if (cost_dtype == DM_F16)
                hipLaunchKernelGGL(energy_partial_kernel<_Float16>, dim3(kEnergyBlocks), dim3(256), 0, stream,
                                   static_cast<const _Float16*>(cost), w_h, w_v, labels, s.W, s.H, s.K, p->trunc_T,
                                   partial);
            else
                hipLaunchKernelGGL(energy_partial_kernel<float>, dim3(kEnergyBlocks), dim3(256), 0, stream,
                                   static_cast<const float*>(cost), w_h, w_v, labels, s.W, s.H, s.K, p->trunc_T,
                                   partial);
            DM_HIP_TRY(hipGetLastError(), "energy launch");
            hipLaunchKernelGGL(bounds_kernel, dim3(1), dim3(256), 0, stream, opt, L.max_chains, S, s.H, slot_g,
                               s.W, partial, kEnergyBlocks, bounds_out);
            DM_HIP_TRY(hipGetLastError(), "bounds launch");
        }
        if (lb_trace_out != nullptr && S > 0) {
            hipLaunchKernelGGL(lb_trace_kernel, dim3(S), dim3(256), 0, stream, opt, L.max_chains, S, s.H, s.W,
                               lb_trace_out);
            DM_HIP_TRY(hipGetLastError(), "lb trace launch");
        }
    }
    return DM_OK;
}

// ------------------------------------------------------------------ backward
namespace dm {
namespace {

struct BwdLayout {
    size_t vol, msg, lam, tape, bbar, lbar, gwh, gwv, lab, total;
    size_t tape_bytes;  // one tape (0: the selections are recomputed)
    int P;
};

BwdLayout bwd_layout(const dm_shape& s, const dm_discrete_params& p) {
    BwdLayout L{};
    // recompute volumes: every pass of a half-step, or (records kept by the forward) only
    // the final pass's two
    L.P = p.keep_checkpoints == 2 ? 1 : pass_count(p);
    L.vol = align_up((size_t)s.W * s.H * s.K * sizeof(float), 256);
    L.tape_bytes = tape_bytes_for(s, p);
    const bool tape = L.tape_bytes != 0;
    size_t off = 0;
    L.msg = off;
    // with tapes, messages and intermediate duals of a recompute stay in place
    off += (size_t)(tape ? 1 : L.P + 1) * L.vol;
    L.lam = off;
    off += (size_t)(L.P > 1 ? (tape ? 1 : L.P - 1) : 0) * L.vol;
    L.tape = off;
    off += tape ? (size_t)(L.P + 1) * L.tape_bytes : 0;
    L.bbar = off;
    off += 2 * L.vol;
    L.lbar = off;
    off += L.vol;
    L.gwh = off;
    off += align_up((size_t)s.H * (s.W > 1 ? s.W - 1 : 1) * sizeof(double), 256);
    L.gwv = off;
    off += align_up((size_t)(s.H > 1 ? s.H - 1 : 1) * s.W * sizeof(double), 256);
    L.lab = off;
    off += align_up((size_t)s.W * s.H * sizeof(int), 256);
    L.total = off;
    return L;
}

}  // namespace
}  // namespace dm

extern "C" size_t dm_solve_discrete_backward_workspace(dm_shape s, const dm_discrete_params* p) {
    if (validate_params(s, p) != DM_OK) return 0;
    return bwd_layout(s, *p).total;
}

extern "C" int dm_solve_discrete_backward(const float* grad_minmarg, const double* grad_bounds, const void* cost,
                                          dm_dtype cost_dtype, const float* w_h, const float* w_v, dm_shape s,
                                          const dm_discrete_params* p, const float* dual, const void* fwd_workspace,
                                          size_t fwd_workspace_bytes, float* grad_cost, float* grad_w_h,
                                          float* grad_w_v, int accumulate, void* workspace, size_t workspace_bytes,
                                          void* hip_stream) {
    clear_error();
    int st = validate_params(s, p);
    if (st != DM_OK) return st;
    DM_REQUIRE(cost_dtype == DM_F32 || cost_dtype == DM_F16, DM_ERR_DTYPE, "unknown cost dtype %d", (int)cost_dtype);
    DM_REQUIRE(cost != nullptr && dual != nullptr && grad_cost != nullptr && fwd_workspace != nullptr, DM_ERR_NULL,
               "cost, dual, grad_cost and the forward workspace are required");
    DM_REQUIRE(s.W == 1 || w_h != nullptr, DM_ERR_NULL, "w_h is required when W > 1");
    DM_REQUIRE(s.H == 1 || w_v != nullptr, DM_ERR_NULL, "w_v is required when H > 1");
    DM_REQUIRE(p->keep_checkpoints == 1 || p->keep_checkpoints == 2, DM_ERR_PARAM,
               "the forward must have been run with keep_checkpoints = 1 or 2");
    DM_REQUIRE(accumulate == 0 || accumulate == 1, DM_ERR_PARAM, "accumulate must be 0 or 1");
    const WsLayout LF = layout(s, *p);
    DM_REQUIRE(fwd_workspace_bytes >= LF.total, DM_ERR_WORKSPACE, "forward workspace %zu bytes, need %zu",
               fwd_workspace_bytes, LF.total);
    const BwdLayout LB = bwd_layout(s, *p);
    DM_REQUIRE(workspace != nullptr && workspace_bytes >= LB.total, DM_ERR_WORKSPACE, "workspace %zu bytes, need %zu",
               workspace_bytes, LB.total);
    const long long vol = (long long)s.W * s.H * s.K;
    DM_REQUIRE(vol * 4 < (long long)kOOB, DM_ERR_UNSUPPORTED, "volume exceeds the 4 GiB buffer range");
    DM_REQUIRE(((uintptr_t)cost % 16) == 0 && ((uintptr_t)dual % 16) == 0 && ((uintptr_t)grad_cost % 16) == 0 &&
                   ((uintptr_t)grad_minmarg % 16) == 0 && ((uintptr_t)workspace % 256) == 0,
               DM_ERR_PARAM, "volumes need 16-byte alignment, workspace 256");
    {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_error("pending HIP error before dm_solve_discrete_backward: %s", hipGetErrorString(e));
            return DM_ERR_HIP;
        }
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const char* fws = static_cast<const char*>(fwd_workspace);
    char* ws = static_cast<char*>(workspace);
    auto vol_at = [&](size_t off, int i) { return reinterpret_cast<float*>(ws + off + (size_t)i * LB.vol); };
    float* lbar = vol_at(LB.lbar, 0);
    double* gwh = reinterpret_cast<double*>(ws + LB.gwh);
    double* gwv = reinterpret_cast<double*>(ws + LB.gwv);
    int* lab = reinterpret_cast<int*>(ws + LB.lab);
    const Tile tile = row_tile(s, *p), tile_v = col_tile(s, *p);
    const int S = half_step_count(*p);
    const int P = LB.P;
    const long long n_wh = (long long)s.H * (s.W - 1), n_wv = (long long)(s.H - 1) * s.W;

    if (!accumulate) {
        hipLaunchKernelGGL(fill_f32_kernel, dim3(2048), dim3(256), 0, stream, grad_cost, vol, 0.0f);
        DM_HIP_TRY(hipGetLastError(), "zero grad");
    }
    if (n_wh > 0) hipLaunchKernelGGL(zero_f64_kernel, dim3(512), dim3(256), 0, stream, gwh, n_wh);
    if (n_wv > 0) hipLaunchKernelGGL(zero_f64_kernel, dim3(512), dim3(256), 0, stream, gwv, n_wv);
    DM_HIP_TRY(hipGetLastError(), "zero edge grads");

    // Sweep descriptions (same as the forward) and the adjoint descriptions.
    SweepArgs rows{};
    rows.theta = cost;
    rows.w = w_h;
    rows.chain_px = s.W;
    rows.node_px = 1;
    rows.w_chain = s.W - 1;
    rows.w_node = 1;
    rows.vol_bytes_f32 = (unsigned)(vol * 4);
    rows.vol_bytes_theta = (unsigned)(vol * (cost_dtype == DM_F16 ? 2 : 4));
    rows.w_bytes = (unsigned)(n_wh * 4);
    rows.K = s.K;
    rows.n = s.W;
    rows.n_chains = s.H;
    rows.T = p->trunc_T;
    rows.sign = 1.0f;
    rows.inv_n = 1.0f / (float)s.W;
    rows.n_pass = p->max_pass;
    for (int i = 0; i < 8; ++i) rows.gamma[i] = p->gamma[i];
    rows.mode = p->minorant == DM_MINORANT_NAIVE ? kModeNaive : kModeIterative;
    const bool tape = LB.tape_bytes != 0;
    if (tape) {
        for (int i = 0; i < 9; ++i) rows.rec_msg[i] = vol_at(LB.msg, 0);
        for (int i = 1; i < 8; ++i) rows.rec_lam[i] = P > 1 ? vol_at(LB.lam, 0) : nullptr;
        for (int i = 0; i <= P && i < 9; ++i)
            rows.tape[i] = reinterpret_cast<unsigned*>(ws + LB.tape + (size_t)i * LB.tape_bytes);
        rows.tape_bytes = (unsigned)LB.tape_bytes;
        rows.tape_px = (unsigned)tape_px_bytes(tile);
    } else {
        for (int i = 0; i <= P && i < 9; ++i) rows.rec_msg[i] = vol_at(LB.msg, i);
        for (int i = 1; i < P && i < 8; ++i) rows.rec_lam[i] = vol_at(LB.lam, i - 1);
    }
    rows.msg = rows.rec_msg[0];
    rows.labels = lab;
    SweepArgs cols = rows;
    cols.theta = nullptr;
    cols.w = w_v;
    cols.w_bytes = (unsigned)(n_wv * 4);
    cols.chain_px = 1;
    cols.node_px = s.W;
    cols.w_chain = 1;
    cols.w_node = s.W;
    cols.n = s.H;
    cols.n_chains = s.W;
    cols.sign = -1.0f;
    cols.inv_n = 1.0f / (float)s.H;
    if (tape) cols.tape_px = (unsigned)tape_px_bytes(tile_v);

    auto adj_from = [&](const SweepArgs& a, double* gw) {
        AdjArgs b{};
        b.theta = a.theta;
        b.w = a.w;
        b.lbar = lbar;
        b.bbar[0] = vol_at(LB.bbar, 0);
        b.bbar[1] = vol_at(LB.bbar, 1);
        b.grad_theta = a.theta != nullptr ? grad_cost : nullptr;
        b.grad_w = gw;
        for (int i = 0; i < 9; ++i) b.rec_msg[i] = a.rec_msg[i];
        for (int i = 0; i < 8; ++i) b.rec_lam[i] = a.rec_lam[i];
        for (int i = 0; i < 9; ++i) b.tape[i] = a.tape[i];
        b.tape_bytes = a.tape_bytes;
        b.tape_px = a.tape_px;
        b.chain_px = a.chain_px;
        b.node_px = a.node_px;
        b.w_chain = a.w_chain;
        b.w_node = a.w_node;
        b.vol_bytes_f32 = a.vol_bytes_f32;
        b.vol_bytes_theta = a.vol_bytes_theta;
        b.w_bytes = a.w_bytes;
        b.K = a.K;
        b.n = a.n;
        b.n_chains = a.n_chains;
        b.T = a.T;
        b.mode = a.mode;
        b.n_pass = a.n_pass;
        b.sign = a.sign;
        b.inv_n = a.inv_n;
        for (int i = 0; i < 8; ++i) b.gamma[i] = a.gamma[i];
        return b;
    };

    // Lower bound LB = sum of row optima + sum of column optima at the final dual.  A
    // half-step leaves the optimum of its own family unchanged as a function of the
    // inputs (it subtracts a minorant that vanishes on the family's optimal labeling),
    // while that family's chains are left with tied min-marginals (all of them for the
    // maximal iterative minorant), where no labeling gives the derivative.  So the
    // family X of the last half-step contributes the one-hot of its optimum at the dual
    // before that half-step; the other family at the final dual.
    const int lb_last = S >= 1 ? ((S - 1) % 2 == 0 ? 0 : 1) : -1;  // 0 rows, 1 columns, -1 none
    // optimal labels of one family's chains at a dual (argmin of the normalized
    // min-marginals, lowest label on ties) into `lab`
    auto labels_at = [&](bool rows_family, const float* lam_k) -> int {
        SweepArgs a = rows_family ? rows : cols;
        a.mode = kModeFinal;
        a.lam = const_cast<float*>(lam_k);
        a.lam_in = lam_k;
        a.msg = vol_at(LB.msg, 0);
        a.minmarg = nullptr;
        a.labels = lab;
        a.opt = nullptr;
        DM_HIP_TRY(launch_sweep(rows_family ? tile : tile_v, a, cost_dtype, stream), "optimum labels");
        return DM_OK;
    };
    auto lb_inject = [&](bool rows_family, const float* lam_k) -> int {
        const int st_l = labels_at(rows_family, lam_k);
        if (st_l != DM_OK) return st_l;
        hipLaunchKernelGGL(lb_inject_kernel, dim3(1024), dim3(256), 0, stream, lab, s.W, s.H, s.K, p->trunc_T,
                           grad_bounds, rows_family ? 1 : 0, lbar, grad_cost, rows_family ? gwh : gwv);
        DM_HIP_TRY(hipGetLastError(), "bound adjoint");
        return DM_OK;
    };

    // 1. final row pass: dL/dminmarg (and the row part of dL/dLB when the rows are taken
    //    at the final dual) -> dL/dcost, dL/d(final dual)
    {
        SweepArgs a = rows;
        a.mode = kModeFinal | kRecordFlag;
        a.lam_in = dual;
        a.lam = const_cast<float*>(dual);  // never written in record mode
        DM_HIP_TRY(launch_sweep(tile, a, cost_dtype, stream), "final recompute");
        AdjArgs b = adj_from(rows, gwh);
        b.mode = kModeFinal;
        b.lam0 = dual;
        b.grad_mm = grad_minmarg;
        b.g_lb = lb_last == 0 ? nullptr : grad_bounds;
        ProfScope ps(DM_PROF_ADJOINT_FINAL, profiler_on() ? adjoint_bytes(b, cost_dtype) : 0.0, stream);
        DM_HIP_TRY(launch_adjoint(tile, b, cost_dtype, stream), "final adjoint");
        // dL/dE(labels): the output labels are the row family's optimal labels at the final dual
        if (grad_bounds != nullptr) {
            st = labels_at(true, dual);
            if (st != DM_OK) return st;
            hipLaunchKernelGGL(energy_adjoint_kernel, dim3(1024), dim3(256), 0, stream, lab, s.W, s.H, s.K,
                               p->trunc_T, grad_bounds, grad_cost, gwh, gwv);
            DM_HIP_TRY(hipGetLastError(), "energy adjoint");
        }
    }
    // 2. column part of dL/dLB at the final dual
    if (grad_bounds != nullptr && lb_last != 1) {
        st = lb_inject(false, dual);
        if (st != DM_OK) return st;
    }
    // 3. half-steps in reverse: recompute from the checkpoint, then differentiate
    const int PF = pass_count(*p);
    for (int k = S - 1; k >= 0; --k) {
        auto fslab = [&](int i) {
            return reinterpret_cast<const float*>(fws + LF.ckpt + (size_t)k * LF.slab_bytes + (size_t)i * LF.vol_bytes);
        };
        const float* ck = fslab(0);
        const bool h = (k % 2) == 0;
        AdjArgs b = adj_from(h ? rows : cols, h ? gwh : gwv);
        if (p->keep_checkpoints == 2 && tape) {
            // the forward kept this half-step's tapes
            for (int i = 0; i < 9; ++i)
                b.tape[i] = i <= PF ? reinterpret_cast<const unsigned*>(fws + LF.ckpt + (size_t)k * LF.slab_bytes +
                                                                        LF.vol_bytes + (size_t)i * LF.tape_bytes)
                                    : nullptr;
            b.tape_bytes = (unsigned)LF.tape_bytes;
        } else if (p->keep_checkpoints == 2) {
            // the forward kept this half-step's messages and intermediate duals
            for (int i = 0; i <= PF && i < 9; ++i) b.rec_msg[i] = fslab(1 + i);
            for (int i = 1; i < PF && i < 8; ++i) b.rec_lam[i] = fslab(PF + 1 + i);
        } else {
            SweepArgs a = h ? rows : cols;
            a.mode = a.mode | kRecordFlag;
            a.lam_in = ck;
            a.lam = const_cast<float*>(ck);
            ProfScope ps(h ? DM_PROF_RECORD_H : DM_PROF_RECORD_V, profiler_on() ? sweep_bytes(a, cost_dtype) : 0.0,
                         stream);
            DM_HIP_TRY(launch_sweep(h ? tile : tile_v, a, cost_dtype, stream), "half-step recompute");
        }
        b.lam0 = ck;
        {
            ProfScope ps(h ? DM_PROF_ADJOINT_H : DM_PROF_ADJOINT_V, profiler_on() ? adjoint_bytes(b, cost_dtype) : 0.0,
                         stream);
            DM_HIP_TRY(launch_adjoint(h ? tile : tile_v, b, cost_dtype, stream), "half-step adjoint");
        }
        // the last half-step's family enters dL/dLB at the dual before that half-step
        if (k == S - 1 && grad_bounds != nullptr) {
            st = lb_inject(h, ck);
            if (st != DM_OK) return st;
        }
    }
    if (grad_w_h != nullptr && n_wh > 0)
        hipLaunchKernelGGL(edge_out_kernel, dim3(512), dim3(256), 0, stream, gwh, n_wh, accumulate, grad_w_h);
    if (grad_w_v != nullptr && n_wv > 0)
        hipLaunchKernelGGL(edge_out_kernel, dim3(512), dim3(256), 0, stream, gwv, n_wv, accumulate, grad_w_v);
    DM_HIP_TRY(hipGetLastError(), "edge grads");
    return DM_OK;
}

// ------------------------------------------------------------------ autotuner
namespace dm {
int validate_discrete(const dm_shape& s, const dm_discrete_params* p) { return validate_params(s, p); }

namespace {

__global__ void hash_fill_kernel(float* __restrict__ f32, _Float16* __restrict__ f16, long long n, unsigned seed) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        unsigned x = (unsigned)i * 2654435761u ^ seed;
        x ^= x >> 15;
        x *= 2246822519u;
        x ^= x >> 13;
        const float v = (float)(x & 0xFFFFFF) * (1.0f / 16777216.0f);
        if (f32) f32[i] = v;
        if (f16) f16[i] = (_Float16)v;
    }
}

struct TuneKey {
    int W, H, K, dt, minorant, max_pass;
    bool operator<(const TuneKey& o) const {
        return std::tie(W, H, K, dt, minorant, max_pass) < std::tie(o.W, o.H, o.K, o.dt, o.minorant, o.max_pass);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<Tile, Tile>> g_tune_cache;

}  // namespace
}  // namespace dm

// Picks, for the row and the column family separately, the compiled (lanes, labels per
// lane) tile with the shortest measured half-step on a synthetic instance of the same
// shape, and writes the choice into p (tile_lanes/labels_per_lane for rows, the _v fields
// for columns).  Allocates (and frees) scratch device memory; results are cached per
// (W, H, K, cost dtype, minorant, max_pass) for the process.
extern "C" int dm_default_tile(int K, int* tile_lanes, int* labels_per_lane) {
    clear_error();
    DM_REQUIRE(tile_lanes != nullptr && labels_per_lane != nullptr, DM_ERR_NULL, "null output");
    DM_REQUIRE(K >= 1 && K <= 256, DM_ERR_SHAPE, "K=%d out of range [1, 256]", K);
    const Tile t = default_tile(K);
    *tile_lanes = t.G;
    *labels_per_lane = t.LPL;
    return DM_OK;
}

extern "C" int dm_autotune_tiles(dm_shape s, dm_dtype cost_dtype, dm_discrete_params* p, void* hip_stream) {
    clear_error();
    DM_REQUIRE(p != nullptr, DM_ERR_NULL, "params is NULL");
    int st = validate_params(s, p);
    if (st != DM_OK) return st;
    DM_REQUIRE(p->minorant != DM_MINORANT_HIERARCHICAL, DM_ERR_UNSUPPORTED,
               "the hierarchical minorant uses no chain tiles");
    DM_REQUIRE(cost_dtype == DM_F32 || cost_dtype == DM_F16, DM_ERR_DTYPE, "unknown cost dtype");
    const TuneKey key{s.W, s.H, s.K, (int)cost_dtype, p->minorant, p->max_pass};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            p->tile_lanes = it->second.first.G;
            p->labels_per_lane = it->second.first.LPL;
            p->tile_lanes_v = it->second.second.G;
            p->labels_per_lane_v = it->second.second.LPL;
            return DM_OK;
        }
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const long long vol = (long long)s.W * s.H * s.K;
    DM_REQUIRE(vol * 4 < (long long)kOOB, DM_ERR_UNSUPPORTED, "volume exceeds the 4 GiB buffer range");
    void *theta = nullptr, *lam = nullptr, *msg = nullptr, *wh = nullptr, *wv = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (theta) (void)hipFree(theta);
        if (lam) (void)hipFree(lam);
        if (msg) (void)hipFree(msg);
        if (wh) (void)hipFree(wh);
        if (wv) (void)hipFree(wv);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    const size_t tb = (size_t)vol * (cost_dtype == DM_F16 ? 2 : 4);
    const long long n_wh = (long long)s.H * (s.W - 1), n_wv = (long long)(s.H - 1) * s.W;
    if (hipMalloc(&theta, tb) != hipSuccess || hipMalloc(&lam, vol * 4) != hipSuccess ||
        hipMalloc(&msg, vol * 4) != hipSuccess || hipMalloc(&wh, (n_wh > 0 ? n_wh : 1) * 4) != hipSuccess ||
        hipMalloc(&wv, (n_wv > 0 ? n_wv : 1) * 4) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        set_error("autotune: device allocation failed");
        return DM_ERR_HIP;
    }
    hipLaunchKernelGGL(hash_fill_kernel, dim3(2048), dim3(256), 0, stream,
                       cost_dtype == DM_F32 ? static_cast<float*>(theta) : nullptr,
                       cost_dtype == DM_F16 ? static_cast<_Float16*>(theta) : nullptr, vol, 12345u);
    hipLaunchKernelGGL(fill_f32_kernel, dim3(2048), dim3(256), 0, stream, static_cast<float*>(lam), vol, 0.0f);
    if (n_wh > 0) hipLaunchKernelGGL(fill_f32_kernel, dim3(256), dim3(256), 0, stream, static_cast<float*>(wh), n_wh, 0.1f);
    if (n_wv > 0) hipLaunchKernelGGL(fill_f32_kernel, dim3(256), dim3(256), 0, stream, static_cast<float*>(wv), n_wv, 0.1f);

    SweepArgs rows{};
    rows.theta = theta;
    rows.lam = static_cast<float*>(lam);
    rows.msg = static_cast<float*>(msg);
    rows.w = static_cast<float*>(wh);
    rows.chain_px = s.W;
    rows.node_px = 1;
    rows.w_chain = s.W - 1;
    rows.w_node = 1;
    rows.vol_bytes_f32 = (unsigned)(vol * 4);
    rows.vol_bytes_theta = (unsigned)tb;
    rows.w_bytes = (unsigned)(n_wh * 4);
    rows.K = s.K;
    rows.n = s.W;
    rows.n_chains = s.H;
    rows.T = p->trunc_T;
    rows.sign = 1.0f;
    rows.inv_n = 1.0f / (float)s.W;
    rows.n_pass = p->max_pass;
    for (int i = 0; i < 8; ++i) rows.gamma[i] = p->gamma[i];
    rows.mode = p->minorant == DM_MINORANT_NAIVE ? kModeNaive : kModeIterative;
    SweepArgs cols = rows;
    cols.theta = nullptr;
    cols.w = static_cast<float*>(wv);
    cols.w_bytes = (unsigned)(n_wv * 4);
    cols.chain_px = 1;
    cols.node_px = s.W;
    cols.w_chain = 1;
    cols.w_node = s.W;
    cols.n = s.H;
    cols.n_chains = s.W;
    cols.sign = -1.0f;
    cols.inv_n = 1.0f / (float)s.H;

    Tile best[2] = {default_tile(s.K), default_tile(s.K)};
    for (int fam = 0; fam < 2; ++fam) {
        const SweepArgs& a = fam == 0 ? rows : cols;
        float best_ms = 1e30f;
        for (const Tile& t : kTiles) {
            if (t.G * t.LPL < s.K) continue;
            if (launch_sweep(t, a, cost_dtype, stream) != hipSuccess) continue;  // warm-up
            float ms_min = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                (void)hipEventRecord(e0, stream);
                (void)launch_sweep(t, a, cost_dtype, stream);
                (void)hipEventRecord(e1, stream);
                if (hipEventSynchronize(e1) != hipSuccess) break;
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                ms_min = ms < ms_min ? ms : ms_min;
            }
            if (ms_min < best_ms) {
                best_ms = ms_min;
                best[fam] = t;
            }
        }
    }
    const hipError_t err = hipStreamSynchronize(stream);
    cleanup();
    if (err != hipSuccess) {
        set_error("autotune: %s", hipGetErrorString(err));
        return DM_ERR_HIP;
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = {best[0], best[1]};
    }
    p->tile_lanes = best[0].G;
    p->labels_per_lane = best[0].LPL;
    p->tile_lanes_v = best[1].G;
    p->labels_per_lane_v = best[1].LPL;
    return DM_OK;
}
