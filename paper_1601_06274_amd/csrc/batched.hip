// batched.hip - many uneven instances in one hipGraph launch (plan / run / destroy).
//
// The plan groups instances by their autotuned chain tile, builds per-launch work tables
// (lane groups of chains, longest chains first) and captures the whole solve once into a
// hipGraph: per half-step one persistent work-queue launch per tile class (classes run as
// parallel graph branches), the final row pass, and optionally the batched refinement
// (one launch per iteration over all instances' tiles).  dm_run_batched replays it.
// Unlike the single-instance calls, the plan allocates and owns device memory (tables,
// message scratch, refinement state) until dm_plan_destroy.
#include <algorithm>
#include <map>
#include <vector>

#include "batched_kernels.h"
#include "common.h"
#include "plan.h"
#include "refine.h"
#include "tiles.h"

namespace dm {

#define DM_EXTERN_BTILE(g, l) \
    extern template hipError_t launch_batched_tile<g, l>(const BatchLaunch&, bool, dm_dtype, int, hipStream_t);
DM_FOR_EACH_TILE(DM_EXTERN_BTILE)
#undef DM_EXTERN_BTILE

namespace {

hipError_t launch_batched(int G, int LPL, const BatchLaunch& bl, bool full, dm_dtype dt, int workers, hipStream_t st) {
#define DM_BCASE(g, l) \
    if (G == g && LPL == l) return launch_batched_tile<g, l>(bl, full, dt, workers, st);
    DM_FOR_EACH_TILE(DM_BCASE)
#undef DM_BCASE
    return hipErrorInvalidValue;
}

__global__ void zero_i32_kernel(int* __restrict__ p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void zero_dual_kernel(const InstDesc* __restrict__ insts, int n) {
    for (int i = blockIdx.y; i < n; i += gridDim.y) {
        const InstDesc in = insts[i];
        const long long vol = (long long)in.W * in.H * in.K;
        for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < vol;
             e += (long long)gridDim.x * blockDim.x)
            in.lam[e] = 0.0f;
    }
}

// Energy of every instance's labels (one with a bounds buffer): FP64 partial sums per
// (instance, block) in a fixed order, as energy_partial_kernel for one instance.
template <typename TT>
__global__ __launch_bounds__(256) void batch_energy_kernel(const InstDesc* __restrict__ insts, int T,
                                                           double* __restrict__ partial) {
    __shared__ double sh[256];
    const InstDesc in = insts[blockIdx.y];
    double acc = 0.0;
    if (in.bounds != nullptr) {
        const TT* theta = static_cast<const TT*>(in.theta);
        const int W = in.W, H = in.H, K = in.K;
        const long long npx = (long long)W * H;
        for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npx;
             p += (long long)gridDim.x * blockDim.x) {
            const int y = (int)(p / W), x = (int)(p % W);
            const int l = min(max(in.labels[p], 0), K - 1);
            acc += (double)to_f<TT>(theta[p * K + l]);
            if (x + 1 < W) {
                const int d = abs(l - min(max(in.labels[p + 1], 0), K - 1));
                acc += (double)in.w_h[(long long)y * (W - 1) + x] * (double)(d < T ? d : T);
            }
            if (y + 1 < H) {
                const int d = abs(l - min(max(in.labels[p + W], 0), K - 1));
                acc += (double)in.w_v[p] * (double)(d < T ? d : T);
            }
        }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(long long)blockIdx.y * gridDim.x + blockIdx.x] = sh[0];
}

__device__ double batch_block_sum(const double* __restrict__ v, int n, double* sh) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += v[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// bounds = {sum of row optima + sum of column optima, sum of the energy partials}, one
// block per instance (the lower bound of eq. DD-dual at the final dual).
__global__ __launch_bounds__(256) void batch_bounds_kernel(const InstDesc* __restrict__ insts,
                                                           const double* __restrict__ partial, int n_part) {
    __shared__ double sh[256];
    const InstDesc in = insts[blockIdx.x];
    if (in.bounds == nullptr) return;  // uniform over the block
    const double a = batch_block_sum(in.opt_rows, in.H, sh);
    const double b = batch_block_sum(in.opt_cols, in.W, sh);
    const double e = batch_block_sum(partial + (long long)blockIdx.x * n_part, n_part, sh);
    if (threadIdx.x == 0) {
        in.bounds[0] = a + b;
        in.bounds[1] = e;
    }
}

constexpr int kBatchEnergyBlocks = 32;  // energy partial sums per instance

struct Class {
    int family, G, LPL;
    bool full;
    std::vector<BatchItem> items;
    BatchItem* d_items = nullptr;
};

}  // namespace

struct BatchPlan : PlanBase {
    int n = 0;
    dm_dtype dt = DM_F32;
    dm_discrete_params dp{};
    bool has_refine = false;
    dm_refine_params rp{};
    std::vector<Class> classes;
};

}  // namespace dm

using namespace dm;

extern "C" int dm_plan_batched(const dm_instance* inst, int n, dm_dtype cost_dtype, const dm_discrete_params* p,
                               const dm_refine_params* rp, void** plan_out) {
    clear_error();
    DM_REQUIRE(plan_out != nullptr && inst != nullptr && p != nullptr, DM_ERR_NULL, "inst, params and plan_out required");
    *plan_out = nullptr;
    DM_REQUIRE(n >= 1 && n <= 4096, DM_ERR_PARAM, "n=%d instances out of range [1, 4096]", n);
    DM_REQUIRE(cost_dtype == DM_F32 || cost_dtype == DM_F16, DM_ERR_DTYPE, "unknown cost dtype");
    DM_REQUIRE(p->minorant == DM_MINORANT_ITERATIVE || p->minorant == DM_MINORANT_NAIVE, DM_ERR_UNSUPPORTED,
               "batched plans take the iterative or the naive minorant (got %d)", p->minorant);
    for (int i = 0; i < n; ++i) {
        const dm_instance& I = inst[i];
        int st = validate_shape(I.s);
        if (st != DM_OK) return st;
        DM_REQUIRE(I.cost != nullptr && I.dual != nullptr && I.labels != nullptr, DM_ERR_NULL,
                   "instance %d: cost, dual and labels are required", i);
        DM_REQUIRE(I.s.W == 1 || I.w_h != nullptr, DM_ERR_NULL, "instance %d: w_h required", i);
        DM_REQUIRE(I.s.H == 1 || I.w_v != nullptr, DM_ERR_NULL, "instance %d: w_v required", i);
        DM_REQUIRE(rp == nullptr || I.u != nullptr, DM_ERR_NULL, "instance %d: u required with refinement", i);
        DM_REQUIRE((long long)I.s.W * I.s.H * I.s.K * 4 < (long long)kOOB, DM_ERR_UNSUPPORTED,
                   "instance %d exceeds the 4 GiB buffer range", i);
        DM_REQUIRE(((uintptr_t)I.cost % 16) == 0 && ((uintptr_t)I.dual % 16) == 0 &&
                       ((uintptr_t)I.minmarg % 16) == 0,
                   DM_ERR_PARAM, "instance %d: volumes need 16-byte alignment", i);
        dm_discrete_params q = *p;
        q.tile_lanes = q.labels_per_lane = q.tile_lanes_v = q.labels_per_lane_v = 0;
        q.keep_checkpoints = 0;
        // validate the schedule with the instance's shape (tiles are chosen below)
        if ((st = validate_discrete(I.s, &q)) != DM_OK) return st;
    }
    if (rp != nullptr) {
        int st = validate_refine(inst[0].s, rp);
        if (st != DM_OK) return st;
    }
    hipError_t e0 = hipGetLastError();
    DM_REQUIRE(e0 == hipSuccess, DM_ERR_HIP, "pending HIP error before dm_plan_batched: %s", hipGetErrorString(e0));

    auto plan = new (std::nothrow) BatchPlan();
    DM_REQUIRE(plan != nullptr, DM_ERR_HIP, "out of host memory");
    plan->n = n;
    plan->dt = cost_dtype;
    plan->dp = *p;
    plan->has_refine = rp != nullptr;
    if (rp) plan->rp = *rp;
    auto fail = [&](const char* what, hipError_t e) {
        set_error("dm_plan_batched: %s: %s", what, hipGetErrorString(e));
        delete plan;
        return DM_ERR_HIP;
    };

    // 1. tiles per (K, family): given in p, else autotuned on the largest instance of that K
    std::map<int, std::pair<std::pair<int, int>, std::pair<int, int>>> tile_of_k;
    for (int i = 0; i < n; ++i) {
        const int K = inst[i].s.K;
        if (tile_of_k.count(K)) continue;
        int big = i;
        for (int j = 0; j < n; ++j)
            if (inst[j].s.K == K && (long long)inst[j].s.W * inst[j].s.H > (long long)inst[big].s.W * inst[big].s.H)
                big = j;
        dm_discrete_params q = *p;
        q.keep_checkpoints = 0;
        if (p->tile_lanes == 0) {
            q.tile_lanes = q.labels_per_lane = q.tile_lanes_v = q.labels_per_lane_v = 0;
            const int st = dm_autotune_tiles(inst[big].s, cost_dtype, &q, nullptr);
            if (st != DM_OK) {
                delete plan;
                return st;
            }
        } else if (p->tile_lanes_v == 0) {
            q.tile_lanes_v = q.tile_lanes;
            q.labels_per_lane_v = q.labels_per_lane;
        }
        if (q.tile_lanes * q.labels_per_lane < K || q.tile_lanes_v * q.labels_per_lane_v < K) {
            set_error("tile holds fewer than K=%d labels", K);
            delete plan;
            return DM_ERR_PARAM;
        }
        tile_of_k[K] = {{q.tile_lanes, q.labels_per_lane}, {q.tile_lanes_v, q.labels_per_lane_v}};
    }

    // 2. device instance table and message scratch
    std::vector<InstDesc> hd(n);
    size_t msg_total = 0, opt_total = 0;
    bool any_bounds = false;
    for (int i = 0; i < n; ++i) {
        msg_total += align_up((size_t)inst[i].s.W * inst[i].s.H * inst[i].s.K * 4, 256);
        if (inst[i].bounds != nullptr) {
            any_bounds = true;
            opt_total += (size_t)inst[i].s.W + inst[i].s.H;
        }
    }
    char* msg_pool = plan->alloc<char>(msg_total);
    InstDesc* d_insts = plan->alloc<InstDesc>(n);
    double* opt_pool = any_bounds ? plan->alloc<double>(opt_total) : nullptr;
    double* partial = any_bounds ? plan->alloc<double>((size_t)n * kBatchEnergyBlocks) : nullptr;
    if (!msg_pool || !d_insts || (any_bounds && (!opt_pool || !partial))) return fail("allocation", hipErrorOutOfMemory);
    size_t opt_off = 0;
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        const dm_instance& I = inst[i];
        const long long vol = (long long)I.s.W * I.s.H * I.s.K;
        InstDesc& d = hd[i];
        d.theta = I.cost;
        d.lam = I.dual;
        d.msg = reinterpret_cast<float*>(msg_pool + off);
        off += align_up((size_t)vol * 4, 256);
        d.w_h = I.w_h;
        d.w_v = I.w_v;
        d.labels = I.labels;
        d.bounds = I.bounds;
        d.minmarg = I.minmarg;
        d.opt_rows = d.opt_cols = nullptr;
        if (I.bounds != nullptr) {
            d.opt_rows = opt_pool + opt_off;
            d.opt_cols = opt_pool + opt_off + I.s.H;
            opt_off += (size_t)I.s.W + I.s.H;
        }
        d.W = I.s.W;
        d.H = I.s.H;
        d.K = I.s.K;
        d.vol_bytes_f32 = (unsigned)(vol * 4);
        d.vol_bytes_theta = (unsigned)(vol * (cost_dtype == DM_F16 ? 2 : 4));
        d.wh_bytes = (unsigned)((long long)I.s.H * (I.s.W - 1) * 4);
        d.wv_bytes = (unsigned)((long long)(I.s.H - 1) * I.s.W * 4);
    }
    hipError_t e = hipMemcpy(d_insts, hd.data(), sizeof(InstDesc) * n, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail("copy instance table", e);

    // 3. classes (family, tile, full) with their work items, longest chains first
    std::map<std::tuple<int, int, int, int>, int> class_of;
    for (int fam = 0; fam < 2; ++fam) {
        for (int i = 0; i < n; ++i) {
            const auto t = fam == 0 ? tile_of_k[inst[i].s.K].first : tile_of_k[inst[i].s.K].second;
            const bool full = t.first * t.second == inst[i].s.K;
            const auto key = std::make_tuple(fam, t.first, t.second, full ? 1 : 0);
            if (!class_of.count(key)) {
                class_of[key] = (int)plan->classes.size();
                Class c;
                c.family = fam;
                c.G = t.first;
                c.LPL = t.second;
                c.full = full;
                plan->classes.push_back(c);
            }
            Class& c = plan->classes[class_of[key]];
            const int chains = fam == 0 ? inst[i].s.H : inst[i].s.W;
            const int cpw = 64 / c.G;
            for (int ch = 0; ch < chains; ch += cpw) c.items.push_back(BatchItem{i, ch});
        }
    }
    for (Class& c : plan->classes) {
        const int fam = c.family;
        std::stable_sort(c.items.begin(), c.items.end(), [&](const BatchItem& a, const BatchItem& b) {
            const int la = fam == 0 ? inst[a.inst].s.W : inst[a.inst].s.H;
            const int lb = fam == 0 ? inst[b.inst].s.W : inst[b.inst].s.H;
            return la > lb;
        });
        c.d_items = plan->alloc<BatchItem>(c.items.size());
        if (!c.d_items) return fail("allocation", hipErrorOutOfMemory);
        e = hipMemcpy(c.d_items, c.items.data(), sizeof(BatchItem) * c.items.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail("copy items", e);
    }
    const int S = p->n_half_steps > 0 ? p->n_half_steps : 2 * p->n_iters;
    const int n_cls = (int)plan->classes.size();
    const long long n_counters = (long long)(S + 2) * n_cls;
    int* counters = plan->alloc<int>(n_counters);
    if (!counters) return fail("allocation", hipErrorOutOfMemory);

    // 4. refinement state and tables
    RefBatchInst* d_rinst = nullptr;
    RefChunk* d_chunks = nullptr;
    RefTile* d_tiles = nullptr;
    int n_chunks = 0, n_tiles = 0;
    if (rp != nullptr) {
        std::vector<RefBatchInst> hr(n);
        std::vector<RefChunk> chunks;
        std::vector<RefTile> tiles;
        for (int i = 0; i < n; ++i) {
            const dm_instance& I = inst[i];
            const size_t px = (size_t)I.s.W * I.s.H;
            const size_t plane = align_up(px * sizeof(rfloat), 256);
            char* base = plan->alloc<char>(13 * plane);
            if (!base) return fail("allocation", hipErrorOutOfMemory);
            RefBatchInst& r = hr[i];
            r.theta = I.cost;
            r.labels = I.labels;
            r.w_h = I.w_h;
            r.w_v = I.w_v;
            r.u_out = I.u;
            r.S[0] = state_at(base, plane);
            r.S[1] = state_at(base + 5 * plane, plane);
            r.u0 = reinterpret_cast<rfloat*>(base + 10 * plane);
            r.sL = reinterpret_cast<rfloat*>(base + 11 * plane);
            r.sR = reinterpret_cast<rfloat*>(base + 12 * plane);
            r.W = I.s.W;
            r.H = I.s.H;
            r.K = I.s.K;
            for (long long st = 0; st < (long long)px; st += 4096)
                chunks.push_back(RefChunk{i, st, (int)std::min<long long>(4096, (long long)px - st)});
            int nbx, nby;
            refine_tile_extent(I.s.W, I.s.H, nbx, nby);
            for (int by = 0; by < nby; ++by)
                for (int bx = 0; bx < nbx; ++bx) tiles.push_back(RefTile{i, bx, by});
        }
        n_chunks = (int)chunks.size();
        n_tiles = (int)tiles.size();
        d_rinst = plan->alloc<RefBatchInst>(n);
        d_chunks = plan->alloc<RefChunk>(chunks.size());
        d_tiles = plan->alloc<RefTile>(tiles.size());
        if (!d_rinst || !d_chunks || !d_tiles) return fail("allocation", hipErrorOutOfMemory);
        if ((e = hipMemcpy(d_rinst, hr.data(), sizeof(RefBatchInst) * n, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(d_chunks, chunks.data(), sizeof(RefChunk) * chunks.size(), hipMemcpyHostToDevice)) !=
                hipSuccess ||
            (e = hipMemcpy(d_tiles, tiles.data(), sizeof(RefTile) * tiles.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return fail("copy refinement tables", e);
    }

    // 5. capture the whole solve into one graph
    int dev = 0, n_cu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    constexpr int kSide = 4;
    hipStream_t main_s = nullptr, side[kSide] = {};
    hipEvent_t ev_fork = nullptr, ev_join[kSide] = {};
    auto destroy_streams = [&]() {
        if (main_s) (void)hipStreamDestroy(main_s);
        for (auto& s2 : side)
            if (s2) (void)hipStreamDestroy(s2);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        for (auto& ev : ev_join)
            if (ev) (void)hipEventDestroy(ev);
    };
    if ((e = hipStreamCreateWithFlags(&main_s, hipStreamNonBlocking)) != hipSuccess) {
        destroy_streams();
        return fail("stream", e);
    }
    for (auto& s2 : side)
        if ((e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking)) != hipSuccess) {
            destroy_streams();
            return fail("stream", e);
        }
    if ((e = hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming)) != hipSuccess) {
        destroy_streams();
        return fail("event", e);
    }
    for (auto& ev : ev_join)
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) {
            destroy_streams();
            return fail("event", e);
        }
    if ((e = hipStreamBeginCapture(main_s, hipStreamCaptureModeRelaxed)) != hipSuccess) {
        destroy_streams();
        return fail("begin capture", e);
    }
    hipError_t ce = hipSuccess;
    auto note = [&](hipError_t x) {
        if (ce == hipSuccess && x != hipSuccess) ce = x;
    };
    hipLaunchKernelGGL(zero_i32_kernel, dim3(64), dim3(256), 0, main_s, counters, n_counters);
    note(hipGetLastError());
    if (!p->warm_start) {
        hipLaunchKernelGGL(zero_dual_kernel, dim3(256, std::min(n, 64)), dim3(256), 0, main_s, d_insts, n);
        note(hipGetLastError());
    }
    auto launch_step = [&](int slot, int family, int mode, bool want_opt) {
        // fork: every class of this family on its own side stream
        note(hipEventRecord(ev_fork, main_s));
        int used = 0;
        for (int ci = 0; ci < n_cls; ++ci) {
            const Class& c = plan->classes[ci];
            if (c.family != family) continue;
            hipStream_t s2 = side[used % kSide];
            if (used < kSide) note(hipStreamWaitEvent(s2, ev_fork, 0));
            BatchLaunch bl{};
            bl.insts = d_insts;
            bl.items = c.d_items;
            bl.n_items = (int)c.items.size();
            bl.counter = counters + (long long)slot * n_cls + ci;
            bl.family = family;
            bl.mode = mode;
            bl.want_opt = want_opt ? 1 : 0;
            bl.T = p->trunc_T;
            bl.n_pass = p->max_pass;
            for (int g = 0; g < 8; ++g) bl.gamma[g] = p->gamma[g];
            const int workers = std::max(1, std::min(bl.n_items, n_cu * 8));
            note(launch_batched(c.G, c.LPL, bl, c.full, cost_dtype, workers, s2));
            ++used;
        }
        for (int u = 0; u < std::min(used, kSide); ++u) {
            note(hipEventRecord(ev_join[u], side[u]));
            note(hipStreamWaitEvent(main_s, ev_join[u], 0));
        }
    };
    const int mode = p->minorant == DM_MINORANT_NAIVE ? kModeNaive : kModeIterative;
    // with bounds: the column optima at the final dual come from the last vertical
    // half-step when it is the last half-step (its family's optimum is unchanged by it),
    // else from a column optimum pass; the row optima from the final pass
    for (int k = 0; k < S; ++k) launch_step(k, k % 2, mode, any_bounds && k == S - 1 && k % 2 == 1);
    launch_step(S, 0, kModeFinal, any_bounds);
    if (any_bounds) {
        if (S == 0 || S % 2 == 1) launch_step(S + 1, 1, kModeOptimum, true);
        if (cost_dtype == DM_F16)
            hipLaunchKernelGGL(batch_energy_kernel<_Float16>, dim3(kBatchEnergyBlocks, n), dim3(256), 0, main_s,
                               d_insts, p->trunc_T, partial);
        else
            hipLaunchKernelGGL(batch_energy_kernel<float>, dim3(kBatchEnergyBlocks, n), dim3(256), 0, main_s,
                               d_insts, p->trunc_T, partial);
        note(hipGetLastError());
        hipLaunchKernelGGL(batch_bounds_kernel, dim3(n), dim3(256), 0, main_s, d_insts, partial, kBatchEnergyBlocks);
        note(hipGetLastError());
    }
    if (rp != nullptr) note(launch_batched_refine(d_rinst, d_chunks, n_chunks, d_tiles, n_tiles, cost_dtype, *rp, main_s));
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(main_s, &graph);
    destroy_streams();
    if (ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail("launch during capture", ce);
    }
    if (e != hipSuccess) return fail("end capture", e);
    plan->graph = graph;
    if ((e = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0)) != hipSuccess) return fail("instantiate", e);
    *plan_out = static_cast<PlanBase*>(plan);
    return DM_OK;
}

extern "C" int dm_run_batched(void* plan, void* hip_stream) {
    clear_error();
    DM_REQUIRE(plan != nullptr, DM_ERR_NULL, "plan is NULL");
    PlanBase* bp = static_cast<PlanBase*>(plan);
    DM_HIP_TRY(hipGraphLaunch(bp->exec, static_cast<hipStream_t>(hip_stream)), "graph launch");
    return DM_OK;
}

extern "C" size_t dm_plan_device_bytes(const void* plan) {
    return plan == nullptr ? 0 : static_cast<const PlanBase*>(plan)->device_bytes;
}

extern "C" void dm_plan_destroy(void* plan) { delete static_cast<PlanBase*>(plan); }
