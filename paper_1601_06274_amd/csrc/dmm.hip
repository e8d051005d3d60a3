// dmm.hip - host orchestration of Dual_MM (dm_solve_discrete) and its small kernels.
//
// Paper: Sec. 2.3 (Alg. Dual_MM, dual decomposition and the lower bound of
// eq. DD-dual), App. A.3.2 (iterative minorant).  The chain sweep kernels are in
// dmm_kernels.h; each (lanes, labels-per-lane) tile is compiled in its own unit.
#include <hip/hip_fp16.h>

#include "dmm_kernels.h"

namespace dm {

#define DM_EXTERN_TILE(g, l) extern template hipError_t launch_tile<g, l>(const SweepArgs&, dm_dtype, hipStream_t);
DM_EXTERN_TILE(4, 1)
DM_EXTERN_TILE(4, 2)
DM_EXTERN_TILE(8, 4)
DM_EXTERN_TILE(16, 4)
DM_EXTERN_TILE(32, 3)
DM_EXTERN_TILE(32, 4)
DM_EXTERN_TILE(64, 3)
DM_EXTERN_TILE(64, 4)
#undef DM_EXTERN_TILE

// ------------------------------------------------------------------ small kernels
__global__ void fill_f32_kernel(float* __restrict__ p, long long n, float v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
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
constexpr Tile kTiles[] = {{4, 1}, {4, 2}, {8, 4}, {16, 4}, {32, 3}, {32, 4}, {64, 3}, {64, 4}};

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

hipError_t launch_sweep(Tile t, const SweepArgs& a, dm_dtype dt, hipStream_t st) {
#define DM_TILE_CASE(g, l) \
    if (t.G == g && t.LPL == l) return launch_tile<g, l>(a, dt, st);
    DM_TILE_CASE(4, 1)
    DM_TILE_CASE(4, 2)
    DM_TILE_CASE(8, 4)
    DM_TILE_CASE(16, 4)
    DM_TILE_CASE(32, 3)
    DM_TILE_CASE(32, 4)
    DM_TILE_CASE(64, 3)
    DM_TILE_CASE(64, 4)
#undef DM_TILE_CASE
    return hipErrorInvalidValue;
}

// Algorithmic HBM bytes of one sweep launch: what the passes must read and write per
// label-node (cost b bytes, dual / messages / min-marginals 4 bytes), times the labels.
double sweep_bytes(const SweepArgs& a, dm_dtype dt) {
    const double b = a.theta != nullptr ? (dt == DM_F16 ? 2.0 : 4.0) : 0.0;
    const double nodes = (double)a.n * a.n_chains * a.K;
    double per = 0.0;
    switch (a.mode) {
        case kModeIterative:
            per = b + 8.0;                                 // R0: cost, dual; message out
            for (int s = 0; s < a.n_pass; ++s) per += (s < a.n_pass - 1) ? b + 16.0 : b + 12.0;
            break;
        case kModeNaive: per = (b + 8.0) + (b + 12.0); break;
        case kModeOptimum: per = b + 4.0; break;
        case kModeFinal: per = (b + 8.0) + (b + 8.0) + (a.minmarg != nullptr ? 4.0 : 0.0); break;
        default: break;
    }
    return per * nodes + (a.mode == kModeFinal ? 4.0 * a.n * a.n_chains : 0.0);
}

hipError_t launch_sweep_prof(Tile t, const SweepArgs& a, dm_dtype dt, hipStream_t st) {
    int kind = DM_PROF_SWEEP_H;
    if (a.mode == kModeFinal) kind = DM_PROF_SWEEP_FINAL;
    else if (a.mode == kModeOptimum) kind = DM_PROF_SWEEP_OPT;
    else if (a.theta == nullptr) kind = DM_PROF_SWEEP_V;
    ProfScope ps(kind, profiler_on() ? sweep_bytes(a, dt) : 0.0, st);
    return launch_sweep(t, a, dt, st);
}

struct WsLayout {
    size_t msg, opt, partial, labels, total;
    long long max_chains;
    int n_slots, n_partial;
};

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
    L.opt = off;
    off = align_up(off + (size_t)L.n_slots * L.max_chains * sizeof(double), 256);
    L.partial = off;
    off = align_up(off + (size_t)L.n_partial * sizeof(double), 256);
    L.labels = off;
    off = align_up(off + (size_t)s.W * s.H * sizeof(int), 256);
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
    DM_REQUIRE(p->minorant == DM_MINORANT_ITERATIVE || p->minorant == DM_MINORANT_NAIVE, DM_ERR_PARAM,
               "unknown minorant %d", p->minorant);
    if (p->minorant == DM_MINORANT_ITERATIVE) {
        DM_REQUIRE(p->max_pass >= 1 && p->max_pass <= 8, DM_ERR_PARAM, "max_pass=%d out of range [1, 8]", p->max_pass);
        for (int i = 0; i < p->max_pass; ++i)
            DM_REQUIRE(p->gamma[i] > 0.0f && p->gamma[i] <= 1.0f, DM_ERR_PARAM, "gamma[%d]=%g not in (0, 1]", i,
                       (double)p->gamma[i]);
        DM_REQUIRE(p->gamma[p->max_pass - 1] == 1.0f, DM_ERR_PARAM,
                   "gamma[max_pass-1] must be 1 for a maximal minorant (got %g)", (double)p->gamma[p->max_pass - 1]);
    }
    DM_REQUIRE(p->warm_start == 0 || p->warm_start == 1, DM_ERR_PARAM, "warm_start must be 0 or 1");
    if (p->tile_lanes != 0 || p->labels_per_lane != 0) {
        DM_REQUIRE(tile_compiled(p->tile_lanes, p->labels_per_lane), DM_ERR_UNSUPPORTED,
                   "tile %d lanes x %d labels is not compiled in", p->tile_lanes, p->labels_per_lane);
        DM_REQUIRE(p->tile_lanes * p->labels_per_lane >= s.K, DM_ERR_PARAM, "tile %dx%d holds fewer than K=%d labels",
                   p->tile_lanes, p->labels_per_lane, s.K);
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

    const Tile tile = (p->tile_lanes != 0) ? Tile{p->tile_lanes, p->labels_per_lane} : default_tile(s.K);
    const long long vol = (long long)s.W * s.H * s.K;
    DM_REQUIRE(vol * 4 < (long long)kOOB, DM_ERR_UNSUPPORTED, "volume of %lld labels exceeds the 4 GiB buffer range", vol);
    if (!p->warm_start) {
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

    const int S = half_step_count(*p);
    const bool want_bounds = bounds_out != nullptr || lb_trace_out != nullptr;
    for (int k = 0; k < S; ++k) {
        SweepArgs a = (k % 2 == 0) ? rows : cols;
        a.opt = want_bounds ? opt + (long long)k * L.max_chains : nullptr;
        DM_HIP_TRY(launch_sweep_prof(tile, a, cost_dtype, stream), "half-step launch");
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
            DM_HIP_TRY(launch_sweep_prof(tile, a, cost_dtype, stream), "column optimum launch");
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
