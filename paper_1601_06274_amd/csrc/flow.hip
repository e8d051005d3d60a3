// flow.hip - optical flow on gfx950: two-dimensional SAD cost, the decoupled layer costs
// and the quadratic-fit refinement.
//
// Paper: Sec. 2.2 "Flow" (the two flow components as separate label layers with the
// optimistic costs of eq. flow decoupled costs, each layer then a stereo-like Dual_MM
// problem), Sec. 3.2 (refinement with the quadratic model eq. quadfit and its prox
// eq. prox_flow), Sec. 2.4 (the primal-dual iteration, shared with stereo).
//
// Layout: the cost table of a pixel is [K2][K1] (horizontal label fastest), pixel (x, y)
// at y*W + x: cost[((y*W + x)*K2 + j)*K1 + i] for the displacement (i - off1, j - off2).
//
// Kernels
//   flow_sad_kernel     : a block owns one image row, one vertical label j and 64 pixels; the
//                         three window rows of I1 (66 columns) and the three displaced rows of
//                         I2 (66 + K1 - 1 columns) are staged in LDS; each thread sums the
//                         3x3 window of |I1 - I2(displaced)| for its (pixel, i) pairs.
//                         flow_sad_cols_kernel (windows of 1, 3 or 5): the same staging,
//                         each lane one label i over 16 consecutive pixels, every window
//                         column's sum formed once and shared by the outputs that use it.
//   flow_project_kernel : each wave owns one pixel at a time (1 to 4 waves per block, as LDS
//                         allows); its K2 x K1 table goes into LDS (16-byte loads when a row
//                         holds whole vectors)
//                         (row stride K1 + 1, so row and column reads are conflict-free), then
//                         lane i takes the minimum down column i (f1) and lane j along row j
//                         (f2).  The minima are exact, so the unaries keep the cost dtype.
//                         HBM-bound: the table is read once, the two unary vectors written once.
//   flow_linearize_kernel: per pixel, L and the positive part of diag Q of the data term at
//                         the current (u1, u2) by central differences of the bilinearly
//                         interpolated table (FP64, like the stereo refinement).
//   flow_pdhg_kernel    : the stereo refinement's iteration (pdhg.h, several iterations per
//                         launch) with the quadratic prox, one component per blockIdx.z.
#include <algorithm>

#include "common.h"
#include "pdhg.h"
#include "refine.h"

namespace dm {
namespace {

constexpr int kFlowTX = 64;

template <typename OT>
__global__ __launch_bounds__(256) void flow_sad_kernel(const float* __restrict__ I1, const float* __restrict__ I2, int W,
                                                       int H, int K1, int K2, int off1, int off2, int r, float trunc,
                                                       float inv_area, OT* __restrict__ out) {
    extern __shared__ float lds[];
    const int x0 = blockIdx.x * kFlowTX;
    const int y = blockIdx.y;
    const int j = blockIdx.z;
    const int d2 = j - off2;
    const int nw = 2 * r + 1;              // window width
    const int nc1 = kFlowTX + 2 * r;       // I1 columns: window slots x0 - r .. x0 + TX - 1 + r (clamped)
    const int nc2 = nc1 + K1 - 1;          // I2 columns: base + [0, nc2)
    float* a1 = lds;                       // [nw][nc1]
    float* a2 = lds + nw * nc1;            // [nw][nc2]
    const int cx_first = min(max(x0 - r, 0), W - 1);
    const int base2 = cx_first - off1;     // I2 column of slot 0 at label i = 0
    for (int idx = threadIdx.x; idx < nw * nc1; idx += blockDim.x) {
        const int dy = idx / nc1, t = idx % nc1;
        const int cy = min(max(y + dy - r, 0), H - 1);
        const int cx = min(max(x0 - r + t, 0), W - 1);
        a1[idx] = I1[(long long)cy * W + cx];
    }
    for (int idx = threadIdx.x; idx < nw * nc2; idx += blockDim.x) {
        const int dy = idx / nc2, t = idx % nc2;
        const int my = min(max(min(max(y + dy - r, 0), H - 1) + d2, 0), H - 1);  // clamped: validity checked below
        const int mx = min(max(base2 + t, 0), W - 1);
        a2[idx] = I2[(long long)my * W + mx];
    }
    __syncthreads();
    const int n_out = kFlowTX * K1;
    for (int idx = threadIdx.x; idx < n_out; idx += blockDim.x) {
        const int xo = idx / K1, i = idx % K1;
        const int x = x0 + xo;
        if (x >= W) continue;
        const int d1 = i - off1;
        float acc = 0.0f;
        for (int dy = 0; dy < nw; ++dy) {
            const int cy = min(max(y + dy - r, 0), H - 1);
            const bool row_ok = cy + d2 >= 0 && cy + d2 < H;
            for (int dx = 0; dx < nw; ++dx) {
                const int t = xo + dx;                          // window slot of column x + dx - r
                const int cx = min(max(x0 - r + t, 0), W - 1);  // its clamped column
                const int mx = cx + d1;
                float e = trunc;
                if (row_ok && mx >= 0 && mx < W) e = fabsf(a1[dy * nc1 + t] - a2[dy * nc2 + (cx - cx_first) + i]);
                acc += e;
            }
        }
        out[(((long long)y * W + x) * K2 + j) * K1 + i] = (OT)fminf(trunc, acc * inv_area);
    }
}

// The same cost for windows of width 2R + 1 <= 5: each wave takes 16 consecutive pixels of
// the block's 64 and each lane one horizontal label at a time, so a window column's sum
// over the 2R + 1 rows is formed once and shared by the 2R + 1 outputs that use it (the
// window summed column by column: the same terms as the general kernel, another order of
// additions).  No divisions; the row validity is uniform and the column validity one
// compare per lane.
template <typename OT, int R>
__global__ __launch_bounds__(256) void flow_sad_cols_kernel(const float* __restrict__ I1, const float* __restrict__ I2,
                                                            int W, int H, int K1, int K2, int off1, int off2,
                                                            float trunc, float inv_area, OT* __restrict__ out) {
    constexpr int NW = 2 * R + 1, GX = 16, NC = GX + 2 * R;
    extern __shared__ float lds[];
    const int x0 = blockIdx.x * kFlowTX;
    const int y = blockIdx.y;
    const int j = blockIdx.z;
    const int d2 = j - off2;
    const int nc1 = kFlowTX + 2 * R;
    const int nc2 = nc1 + K1 - 1;
    float* a1 = lds;
    float* a2 = lds + NW * nc1;
    const int cx_first = min(max(x0 - R, 0), W - 1);
    const int base2 = cx_first - off1;
    for (int idx = threadIdx.x; idx < NW * nc1; idx += blockDim.x) {
        const int dy = idx / nc1, t = idx % nc1;
        const int cy = min(max(y + dy - R, 0), H - 1);
        const int cx = min(max(x0 - R + t, 0), W - 1);
        a1[idx] = I1[(long long)cy * W + cx];
    }
    for (int idx = threadIdx.x; idx < NW * nc2; idx += blockDim.x) {
        const int dy = idx / nc2, t = idx % nc2;
        const int my = min(max(min(max(y + dy - R, 0), H - 1) + d2, 0), H - 1);  // clamped: validity checked below
        const int mx = min(max(base2 + t, 0), W - 1);
        a2[idx] = I2[(long long)my * W + mx];
    }
    __syncthreads();
    bool row_ok[NW];
#pragma unroll
    for (int dy = 0; dy < NW; ++dy) {
        const int cy = min(max(y + dy - R, 0), H - 1);
        row_ok[dy] = cy + d2 >= 0 && cy + d2 < H;
    }
    const int g = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
    const int t0 = g * GX;  // the wave's first output slot
    for (int i = lane; i < K1; i += 64) {
        const int d1 = i - off1;
        float cs[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int t = t0 + c;                           // window slot of column x0 - R + t
            const int cx = min(max(x0 - R + t, 0), W - 1);  // its clamped column
            const int mx = cx + d1;
            const bool col_ok = mx >= 0 && mx < W;
            const int o2 = (cx - cx_first) + i;
            float sum = 0.0f;
#pragma unroll
            for (int dy = 0; dy < NW; ++dy) {
                const float e = (row_ok[dy] && col_ok) ? fabsf(a1[dy * nc1 + t] - a2[dy * nc2 + o2]) : trunc;
                sum += e;
            }
            cs[c] = sum;
        }
#pragma unroll
        for (int q = 0; q < GX; ++q) {
            const int x = x0 + t0 + q;
            float acc = cs[q];
#pragma unroll
            for (int dx = 1; dx < NW; ++dx) acc += cs[q + dx];
            if (x < W) out[(((long long)y * W + x) * K2 + j) * K1 + i] = (OT)fminf(trunc, acc * inv_area);
        }
    }
}

template <typename TT>
__global__ __launch_bounds__(256) void flow_project_kernel(const TT* __restrict__ cost, long long npx, int K1, int K2,
                                                           TT* __restrict__ f1, TT* __restrict__ f2) {
    extern __shared__ float lds[];
    const int nwv = blockDim.x / 64;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int ld = K1 + 1;
    float* tile = lds + (size_t)wave * K2 * ld;
    const int n = K1 * K2;
    // every wave of the block runs the same number of groups, so the barriers match
    for (long long g = blockIdx.x; g * nwv < npx; g += gridDim.x) {
        const long long p = g * nwv + wave;
        const bool live = p < npx;
        if (live) {
            const TT* src = cost + p * (long long)n;
            // 16-byte loads when a row holds whole vectors and the volume is 16-byte
            // aligned (every pixel's table then is too): the wave's loads are issued
            // together and a vector's elements share one row
            constexpr int EPV = 16 / (int)sizeof(TT);
            if (K1 % EPV == 0 && ((uintptr_t)cost & 15u) == 0) {
                const uint4* s4 = reinterpret_cast<const uint4*>(src);
                const int nv = n / EPV, vpr = K1 / EPV;
#pragma unroll 8
                for (int v = lane; v < nv; v += 64) {
                    const uint4 w = s4[v];
                    const TT* el = reinterpret_cast<const TT*>(&w);
                    const int r = v / vpr, c = (v - r * vpr) * EPV;
                    float* dst = tile + r * ld + c;
#pragma unroll
                    for (int k = 0; k < EPV; ++k) dst[k] = (float)el[k];
                }
            } else {
                for (int e = lane; e < n; e += 64) tile[(e / K1) * ld + (e % K1)] = (float)src[e];
            }
        }
        __syncthreads();
        if (live) {
            for (int i = lane; i < K1; i += 64) {
                float m = tile[i];
                for (int jj = 1; jj < K2; ++jj) m = fminf(m, tile[jj * ld + i]);
                f1[p * K1 + i] = (TT)m;
            }
            for (int jj = lane; jj < K2; jj += 64) {
                const float* row = tile + jj * ld;
                float m = row[0];
                for (int i = 1; i < K1; ++i) m = fminf(m, row[i]);
                f2[p * K2 + jj] = (TT)m;
            }
        }
        __syncthreads();
    }
}

// Bilinear interpolation of pixel p's table at (v1, v2), arguments clamped to the label ranges.
template <typename TT>
__device__ __forceinline__ rfloat interp2(const TT* __restrict__ c, long long p, int K1, int K2, rfloat v1, rfloat v2) {
    v1 = fmin(fmax(v1, 0.0), (rfloat)(K1 - 1));
    v2 = fmin(fmax(v2, 0.0), (rfloat)(K2 - 1));
    int a0 = (int)floor(v1), b0 = (int)floor(v2);
    a0 = a0 < K1 - 1 ? a0 : K1 - 1;
    b0 = b0 < K2 - 1 ? b0 : K2 - 1;
    const int a1 = a0 + 1 < K1 - 1 ? a0 + 1 : K1 - 1;
    const int b1 = b0 + 1 < K2 - 1 ? b0 + 1 : K2 - 1;
    const rfloat t = v1 - (rfloat)a0, s = v2 - (rfloat)b0;
    const TT* tab = c + p * (long long)K1 * K2;
    const rfloat d00 = (rfloat)(float)tab[b0 * K1 + a0], d01 = (rfloat)(float)tab[b0 * K1 + a1];
    const rfloat d10 = (rfloat)(float)tab[b1 * K1 + a0], d11 = (rfloat)(float)tab[b1 * K1 + a1];
    return (1.0 - s) * ((1.0 - t) * d00 + t * d01) + s * ((1.0 - t) * d10 + t * d11);
}

struct FlowComp {
    RefineState S[2];
    rfloat* u0;
    rfloat* L;
    rfloat* Q;
    int K;
};
struct FlowComps {
    FlowComp c[2];
};

template <typename TT>
__global__ __launch_bounds__(256) void flow_linearize_kernel(const TT* __restrict__ cost, long long npx, int K1, int K2,
                                                             rfloat h, FlowComps fc, int cur) {
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long long)gridDim.x * blockDim.x) {
        const rfloat u1 = fc.c[0].S[cur].u[p], u2 = fc.c[1].S[cur].u[p];
        const rfloat c = interp2(cost, p, K1, K2, u1, u2);
        const rfloat p1 = interp2(cost, p, K1, K2, u1 + h, u2), m1 = interp2(cost, p, K1, K2, u1 - h, u2);
        const rfloat p2 = interp2(cost, p, K1, K2, u1, u2 + h), m2 = interp2(cost, p, K1, K2, u1, u2 - h);
        fc.c[0].u0[p] = u1;
        fc.c[1].u0[p] = u2;
        fc.c[0].L[p] = (p1 - m1) / (2.0 * h);
        fc.c[1].L[p] = (p2 - m2) / (2.0 * h);
        fc.c[0].Q[p] = fmax((p1 - 2.0 * c + m1) / (h * h), 0.0);
        fc.c[1].Q[p] = fmax((p2 - 2.0 * c + m2) / (h * h), 0.0);
    }
}

// prox of tau D~ for the quadratic model of one component (eq. prox_flow with the
// denominator 1 + tau Q, the stationarity condition of the prox objective), then the box
// [u0 - h, u0 + h] n [0, K-1].  code: bits 2-3 clamp (0, 1 low, 2 high).
struct QuadProx {
    const rfloat* u0;
    const rfloat* L;
    const rfloat* Q;
    rfloat tau, h;
    struct Px {
        rfloat u0, L, Q;
    };
    __device__ __forceinline__ Px load(long long p) const { return Px{u0[p], L[p], Q[p]}; }
    __device__ __forceinline__ rfloat operator()(rfloat uh, long long p, rfloat kmax, int& code) const {
        return apply(uh, load(p), kmax, code);
    }
    __device__ __forceinline__ rfloat apply(rfloat uh, const Px& d, rfloat kmax, int& code) const {
        const rfloat c = d.u0, q = d.Q;
        rfloat v = (uh + tau * (q * c - d.L)) / (1.0 + tau * q);
        const rfloat lo = fmax(c - h, 0.0);
        const rfloat hi = fmin(c + h, kmax);
        int cl = 0;
        if (v < lo) {
            v = lo;
            cl = 1;
        } else if (v > hi) {
            v = hi;
            cl = 2;
        }
        code = cl << 2;
        return v;
    }
};

__global__ __launch_bounds__(256) void flow_pdhg_kernel(FlowComps fc, int cur, const float* __restrict__ w_h,
                                                        const float* __restrict__ w_v, int W, int H, RefineScalars sc,
                                                        int n_iter) {
    const FlowComp& c = fc.c[blockIdx.z];
    pdhg_fused_tile<kQTX, kQTY, kQS>(c.S[cur], c.S[cur ^ 1], QuadProx{c.u0, c.L, c.Q, sc.tau, sc.h}, w_h, w_v, W, H,
                                     c.K, sc, nullptr, 0, n_iter, blockIdx.x * kQTX, blockIdx.y * kQTY);
}

__global__ __launch_bounds__(256) void flow_init_kernel(const int* __restrict__ l1, const int* __restrict__ l2,
                                                        long long npx, FlowComps fc) {
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long long)gridDim.x * blockDim.x) {
        for (int k = 0; k < 2; ++k) {
            const RefineState s = fc.c[k].S[0];
            int l = (k == 0 ? l1 : l2)[p];
            l = l < 0 ? 0 : (l > fc.c[k].K - 1 ? fc.c[k].K - 1 : l);
            s.u[p] = (rfloat)l;
            s.ph[p] = 0.0;
            s.pv[p] = 0.0;
            s.qh[p] = 0.0;
            s.qv[p] = 0.0;
        }
    }
}

__global__ __launch_bounds__(256) void flow_narrow_kernel(FlowComps fc, int cur, long long npx, float* __restrict__ u1,
                                                          float* __restrict__ u2) {
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long long)gridDim.x * blockDim.x) {
        u1[p] = (float)fc.c[0].S[cur].u[p];
        u2[p] = (float)fc.c[1].S[cur].u[p];
    }
}

int validate_flow_shape(const dm_flow_shape& s) {
    DM_REQUIRE(s.W >= 1 && s.W <= 16384 && s.H >= 1 && s.H <= 16384, DM_ERR_SHAPE, "W=%d, H=%d out of range [1, 16384]",
               s.W, s.H);
    DM_REQUIRE(s.K1 >= 1 && s.K1 <= 256 && s.K2 >= 1 && s.K2 <= 256, DM_ERR_SHAPE, "K1=%d, K2=%d out of range [1, 256]",
               s.K1, s.K2);
    DM_REQUIRE(s.K1 * s.K2 <= 4096, DM_ERR_SHAPE, "K1*K2 = %d exceeds 4096", s.K1 * s.K2);
    const unsigned long long n = (unsigned long long)s.W * s.H * s.K1 * s.K2;
    DM_REQUIRE(n < (1ull << 32), DM_ERR_SHAPE, "W*H*K1*K2 = %llu exceeds 2^32", n);
    DM_REQUIRE(s.off1 >= 0 && s.off1 < s.K1 && s.off2 >= 0 && s.off2 < s.K2, DM_ERR_PARAM,
               "offsets (%d, %d) must lie in [0, K1) x [0, K2)", s.off1, s.off2);
    // each layer's unary volume is a dm_solve_discrete problem
    const unsigned long long v = (unsigned long long)s.W * s.H * (s.K1 > s.K2 ? s.K1 : s.K2) * 4ull;
    DM_REQUIRE(v <= 0xFE000000ull, DM_ERR_SHAPE, "a layer's FP32 unary volume of %llu bytes exceeds the solver's range", v);
    return DM_OK;
}

int pending(const char* where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("pending HIP error before %s: %s", where, hipGetErrorString(e));
        return DM_ERR_HIP;
    }
    return DM_OK;
}

struct FlowLayout {
    size_t plane, comp, total;  // per component: u0, L, Q, two states of 5 planes
};

FlowLayout flow_layout(const dm_flow_shape& s) {
    FlowLayout L{};
    L.plane = align_up((size_t)s.W * s.H * sizeof(rfloat), 256);
    L.comp = 13 * L.plane;
    L.total = 2 * L.comp;
    return L;
}

int validate_flow_refine(const dm_flow_shape& s, const dm_refine_params* p) {
    int st = validate_flow_shape(s);
    if (st != DM_OK) return st;
    st = validate_refine(dm_shape{s.W, s.H, s.K1 > s.K2 ? s.K1 : s.K2}, p);
    if (st != DM_OK) return st;
    DM_REQUIRE(p->keep_tape == 0, DM_ERR_UNSUPPORTED, "the flow refinement has no backward: keep_tape must be 0");
    return DM_OK;
}

}  // namespace
}  // namespace dm

using namespace dm;

extern "C" int dm_build_flow_cost_volume(const float* I1, const float* I2, dm_flow_shape s, const dm_cost_params* p,
                                         dm_dtype out_dtype, void* cost_out, float* w_h, float* w_v,
                                         void* hip_stream) {
    clear_error();
    int st = validate_flow_shape(s);
    if (st != DM_OK) return st;
    DM_REQUIRE(I1 != nullptr && I2 != nullptr && cost_out != nullptr && p != nullptr, DM_ERR_NULL,
               "images, params and cost_out are required");
    DM_REQUIRE(out_dtype == DM_F32 || out_dtype == DM_F16, DM_ERR_DTYPE, "unknown dtype %d", (int)out_dtype);
    DM_REQUIRE(p->window >= 1 && p->window <= 15 && (p->window & 1), DM_ERR_PARAM, "window must be odd in [1, 15]");
    DM_REQUIRE(p->trunc > 0.0f && p->lambda_pw >= 0.0f && p->contrast_sigma > 0.0f, DM_ERR_PARAM,
               "trunc > 0, lambda_pw >= 0, contrast_sigma > 0 required");
    if ((st = pending("dm_build_flow_cost_volume")) != DM_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int r = p->window / 2;
    const int nw = 2 * r + 1;
    const size_t lds = (size_t)nw * ((kFlowTX + 2 * r) + (kFlowTX + 2 * r + s.K1 - 1)) * sizeof(float);
    const dim3 grid((s.W + kFlowTX - 1) / kFlowTX, s.H, s.K2);
    const float inv_area = 1.0f / (float)(nw * nw);
    const long long npx = (long long)s.W * s.H;
    ProfScope ps(DM_PROF_FLOW_COST, (double)npx * s.K1 * s.K2 * (out_dtype == DM_F16 ? 2 : 4) + 8.0 * npx, stream);
#define DM_FLOW_COLS(OT, R)                                                                                   \
    hipLaunchKernelGGL((flow_sad_cols_kernel<OT, R>), grid, dim3(256), lds, stream, I1, I2, s.W, s.H, s.K1, s.K2, \
                       s.off1, s.off2, p->trunc, inv_area, static_cast<OT*>(cost_out))
    if (out_dtype == DM_F16) {
        if (r == 0) DM_FLOW_COLS(_Float16, 0);
        else if (r == 1) DM_FLOW_COLS(_Float16, 1);
        else if (r == 2) DM_FLOW_COLS(_Float16, 2);
        else
            hipLaunchKernelGGL(flow_sad_kernel<_Float16>, grid, dim3(256), lds, stream, I1, I2, s.W, s.H, s.K1, s.K2,
                               s.off1, s.off2, r, p->trunc, inv_area, static_cast<_Float16*>(cost_out));
    } else {
        if (r == 0) DM_FLOW_COLS(float, 0);
        else if (r == 1) DM_FLOW_COLS(float, 1);
        else if (r == 2) DM_FLOW_COLS(float, 2);
        else
            hipLaunchKernelGGL(flow_sad_kernel<float>, grid, dim3(256), lds, stream, I1, I2, s.W, s.H, s.K1, s.K2,
                               s.off1, s.off2, r, p->trunc, inv_area, static_cast<float*>(cost_out));
    }
#undef DM_FLOW_COLS
    ps.stop();
    DM_HIP_TRY(hipGetLastError(), "flow cost launch");
    if (w_h != nullptr || w_v != nullptr)
        DM_HIP_TRY(launch_contrast_weights(I1, s.W, s.H, p->lambda_pw, p->contrast_sigma, w_h, w_v, stream),
                   "contrast launch");
    return DM_OK;
}

extern "C" int dm_flow_project(const void* cost, dm_dtype cost_dtype, dm_flow_shape s, void* f1_out, void* f2_out,
                               void* hip_stream) {
    clear_error();
    int st = validate_flow_shape(s);
    if (st != DM_OK) return st;
    DM_REQUIRE(cost != nullptr && f1_out != nullptr && f2_out != nullptr, DM_ERR_NULL, "cost, f1_out and f2_out are required");
    DM_REQUIRE(cost_dtype == DM_F32 || cost_dtype == DM_F16, DM_ERR_DTYPE, "unknown dtype %d", (int)cost_dtype);
    if ((st = pending("dm_flow_project")) != DM_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const long long npx = (long long)s.W * s.H;
    // one pixel per wave; as many waves per block as 64 KiB of LDS holds (at most 4)
    const size_t per_wave = (size_t)s.K2 * (s.K1 + 1) * sizeof(float);
    const int nwv = (int)std::max<size_t>(1, std::min<size_t>(4, 65536 / per_wave));
    const size_t lds = (size_t)nwv * per_wave;
    const unsigned blocks = (unsigned)std::min<long long>((npx + nwv - 1) / nwv, 8192LL);
    const int es = cost_dtype == DM_F16 ? 2 : 4;
    ProfScope ps(DM_PROF_FLOW_PROJECT, (double)npx * ((double)s.K1 * s.K2 + s.K1 + s.K2) * es, stream);
    if (cost_dtype == DM_F16)
        hipLaunchKernelGGL(flow_project_kernel<_Float16>, dim3(blocks), dim3(64 * nwv), lds, stream,
                           static_cast<const _Float16*>(cost), npx, s.K1, s.K2, static_cast<_Float16*>(f1_out),
                           static_cast<_Float16*>(f2_out));
    else
        hipLaunchKernelGGL(flow_project_kernel<float>, dim3(blocks), dim3(64 * nwv), lds, stream,
                           static_cast<const float*>(cost), npx, s.K1, s.K2, static_cast<float*>(f1_out),
                           static_cast<float*>(f2_out));
    DM_HIP_TRY(hipGetLastError(), "flow projection launch");
    return DM_OK;
}

extern "C" size_t dm_refine_flow_workspace(dm_flow_shape s, const dm_refine_params* p) {
    if (validate_flow_refine(s, p) != DM_OK) return 0;
    return flow_layout(s).total;
}

extern "C" int dm_refine_flow(const void* cost, dm_dtype cost_dtype, const int32_t* labels1, const int32_t* labels2,
                              const float* w_h, const float* w_v, dm_flow_shape s, const dm_refine_params* p,
                              float* u1_out, float* u2_out, void* workspace, size_t workspace_bytes, void* hip_stream) {
    clear_error();
    int st = validate_flow_refine(s, p);
    if (st != DM_OK) return st;
    DM_REQUIRE(cost_dtype == DM_F32 || cost_dtype == DM_F16, DM_ERR_DTYPE, "unknown dtype %d", (int)cost_dtype);
    DM_REQUIRE(cost != nullptr && labels1 != nullptr && labels2 != nullptr && u1_out != nullptr && u2_out != nullptr,
               DM_ERR_NULL, "cost, both label maps and both outputs are required");
    DM_REQUIRE(s.W == 1 || w_h != nullptr, DM_ERR_NULL, "w_h is required when W > 1");
    DM_REQUIRE(s.H == 1 || w_v != nullptr, DM_ERR_NULL, "w_v is required when H > 1");
    const FlowLayout L = flow_layout(s);
    DM_REQUIRE(workspace != nullptr && workspace_bytes >= L.total, DM_ERR_WORKSPACE, "workspace %zu bytes, need %zu",
               workspace_bytes, L.total);
    if ((st = pending("dm_refine_flow")) != DM_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    char* ws = static_cast<char*>(workspace);
    FlowComps fc;
    for (int k = 0; k < 2; ++k) {
        char* b = ws + k * L.comp;
        fc.c[k].u0 = reinterpret_cast<rfloat*>(b);
        fc.c[k].L = reinterpret_cast<rfloat*>(b + L.plane);
        fc.c[k].Q = reinterpret_cast<rfloat*>(b + 2 * L.plane);
        fc.c[k].S[0] = state_at(b + 3 * L.plane, L.plane);
        fc.c[k].S[1] = state_at(b + 8 * L.plane, L.plane);
        fc.c[k].K = k == 0 ? s.K1 : s.K2;
    }
    const long long npx = (long long)s.W * s.H;
    const unsigned eb = (unsigned)std::min<long long>((npx + 255) / 256, 4096);
    hipLaunchKernelGGL(flow_init_kernel, dim3(eb), dim3(256), 0, stream, labels1, labels2, npx, fc);
    DM_HIP_TRY(hipGetLastError(), "flow refine init");
    const RefineScalars sc = refine_scalars(*p);
    const dim3 grid((s.W + kQTX - 1) / kQTX, (s.H + kQTY - 1) / kQTY, 2);
    int cur = 0;
    for (int wp = 0; wp < p->n_warps; ++wp) {
        ProfScope ps1(DM_PROF_REFINE_LINEARIZE, (double)npx * (16.0 + 20.0 * (cost_dtype == DM_F16 ? 2 : 4) + 48.0),
                      stream);
        if (cost_dtype == DM_F16)
            hipLaunchKernelGGL(flow_linearize_kernel<_Float16>, dim3(eb), dim3(256), 0, stream,
                               static_cast<const _Float16*>(cost), npx, s.K1, s.K2, (rfloat)p->h, fc, cur);
        else
            hipLaunchKernelGGL(flow_linearize_kernel<float>, dim3(eb), dim3(256), 0, stream,
                               static_cast<const float*>(cost), npx, s.K1, s.K2, (rfloat)p->h, fc, cur);
        ps1.stop();
        DM_HIP_TRY(hipGetLastError(), "flow linearize");
        for (int it0 = 0; it0 < p->n_iters; it0 += kQS) {
            const int nit = std::min(kQS, p->n_iters - it0);
            ProfScope ps2(DM_PROF_REFINE_ITER, 2.0 * nit * npx * (8.0 * 13.0 + 8.0), stream);
            hipLaunchKernelGGL(flow_pdhg_kernel, grid, dim3(256), 0, stream, fc, cur, w_h, w_v, s.W, s.H, sc, nit);
            cur ^= 1;
        }
        DM_HIP_TRY(hipGetLastError(), "flow pdhg");
    }
    hipLaunchKernelGGL(flow_narrow_kernel, dim3(eb), dim3(256), 0, stream, fc, cur, npx, u1_out, u2_out);
    DM_HIP_TRY(hipGetLastError(), "flow narrow");
    return DM_OK;
}
