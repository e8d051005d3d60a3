// refine.hip - continuous refinement by the non-linear primal-dual method on gfx950.
//
// Paper: Sec. 2.4 (Valkonen's iteration, eq. cont_iterates; difference-of-convex split
// eq. r-decompose; conjugate prox eq. pprox; the operator gradient) and Sec. 3.1 (two-slope
// convex model of the data term around the current point, its prox, warping).
//
// With x = (u, q), y = (p, d = 1) one iteration is, per pixel / edge,
//     u+ = prox_{tau D~}( u - tau A^T (p - q) )
//     q+ = prox_{tau R_-^*}( q + tau A u )
//     p+ = prox_{sigma R_+^*}( p + sigma A (2 u+ - u) ),
// with (Au)_e = u_i - u_j for the right / lower neighbour j of i.  R_+ uses
// r_{eps,delta}, R_- uses r_{0, C + delta - eps*delta}; both conjugate proxes are
// eq. pprox followed by the clamp to [-w, w].
//
// Kernels
//   linearize_kernel : u0 := u, slopes (s_L, s_R) of the data term at u0 by linear
//                      interpolation of the cost volume along the label axis (once per warp)
//   pdhg_kernel      : one full iteration.  A block owns a TX x TY tile; it first computes
//                      u+ on the tile plus a one-pixel halo to the right and below (the
//                      halo values are recomputed, not exchanged), keeps u and u+ in LDS,
//                      then updates q and p of the tile's edges.  State is double
//                      buffered (every read sees the previous iterate).
// State and arithmetic are FP64 (rfloat); the cost volume and edge weights are read in
// their storage types and widened.  The working set (about 11 doubles per pixel) stays
// in L2 / MALL at these sizes, so the iteration is bound by on-chip bandwidth and
// launch latency, not HBM.
#include "common.h"
#include "refine.h"

namespace dm {

template <typename TT>
__device__ __forceinline__ rfloat cost_at(const TT* __restrict__ th, long long p, int K, int k) {
    return (rfloat)(float)th[p * K + k];
}

template <typename TT>
__device__ __forceinline__ rfloat interp(const TT* __restrict__ th, long long p, int K, rfloat v) {
    v = fmin(fmax(v, 0.0), (rfloat)(K - 1));
    int k0 = (int)floor(v);
    k0 = k0 < K - 1 ? k0 : K - 1;
    const int k1 = k0 + 1 < K - 1 ? k0 + 1 : K - 1;
    const rfloat t = v - (rfloat)k0;
    return (1.0 - t) * cost_at(th, p, K, k0) + t * cost_at(th, p, K, k1);
}

template <typename TT>
__global__ __launch_bounds__(256) void linearize_kernel(const TT* __restrict__ th, const rfloat* __restrict__ u, int W,
                                                        int H, int K, rfloat h, rfloat* __restrict__ u0,
                                                        rfloat* __restrict__ sL, rfloat* __restrict__ sR) {
    const long long n = (long long)W * H;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        const rfloat c = u[p];
        const rfloat Dc = interp(th, p, K, c);
        const rfloat Dm = interp(th, p, K, c - h);
        const rfloat Dp = interp(th, p, K, c + h);
        rfloat l = (Dc - Dm) / h;
        rfloat r = (Dp - Dc) / h;
        const bool has_l = c - h >= 0.0;
        const bool has_r = c + h <= (rfloat)(K - 1);
        const rfloat l0 = l;
        l = has_l ? l : (has_r ? r : 0.0);
        r = has_r ? r : (has_l ? l0 : 0.0);
        if (l > r) {
            const rfloat m = 0.5 * (l + r);
            l = m;
            r = m;
        }
        u0[p] = c;
        sL[p] = l;
        sR[p] = r;
    }
}

// prox of step * (w r_{alpha,beta})^* at t (eq. pprox), then the clamp to [-w, w].
__device__ __forceinline__ rfloat prox_conj(rfloat t, rfloat w, rfloat alpha, rfloat beta, rfloat step) {
    const rfloat a = fabs(t);
    const rfloat aw = alpha * w;
    rfloat r = (a <= aw) ? t : copysign(fmax(aw, a - beta * step), t);
    return fmin(fmax(r, -w), w);
}

// prox of tau * D~ (two-slope soft threshold) and the box [u0 - h, u0 + h] n [0, K-1].
__device__ __forceinline__ rfloat prox_data(rfloat uh, rfloat u0, rfloat l, rfloat r, rfloat tau, rfloat h,
                                            rfloat kmax) {
    rfloat v = (uh > u0 + tau * r) ? uh - tau * r : ((uh < u0 + tau * l) ? uh - tau * l : u0);
    const rfloat lo = fmax(u0 - h, 0.0);
    const rfloat hi = fmin(u0 + h, kmax);
    return fmin(fmax(v, lo), hi);
}

constexpr int kTX = 64, kTY = 4;

// Edge arrays are stored per pixel: ph/qh at (x, y) belong to the edge (x, y)-(x+1, y)
// (unused in the last column), pv/qv to (x, y)-(x, y+1) (unused in the last row).
__global__ __launch_bounds__(256) void pdhg_kernel(const RefineState in, RefineState out, const rfloat* __restrict__ u0,
                                                   const rfloat* __restrict__ sL, const rfloat* __restrict__ sR,
                                                   const float* __restrict__ w_h, const float* __restrict__ w_v, int W,
                                                   int H, int K, RefineScalars sc) {
    __shared__ rfloat s_uo[kTY + 1][kTX + 1];
    __shared__ rfloat s_un[kTY + 1][kTX + 1];
    const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY;
    const rfloat kmax = (rfloat)(K - 1);
    // Phase A: u+ on the tile and its right / lower halo.
    for (int idx = threadIdx.x; idx < (kTX + 1) * (kTY + 1); idx += blockDim.x) {
        const int i = idx % (kTX + 1), j = idx / (kTX + 1);
        const int x = x0 + i, y = y0 + j;
        rfloat uo = 0.0, un = 0.0;
        if (x < W && y < H) {
            const long long p = (long long)y * W + x;
            // (A^T z)_i = z_h(i) + z_v(i) - z_h(left) - z_v(up), z = p - q
            rfloat at = 0.0;
            if (x + 1 < W) at += in.ph[p] - in.qh[p];
            if (y + 1 < H) at += in.pv[p] - in.qv[p];
            if (x > 0) at -= in.ph[p - 1] - in.qh[p - 1];
            if (y > 0) at -= in.pv[p - W] - in.qv[p - W];
            uo = in.u[p];
            un = prox_data(uo - sc.tau * at, u0[p], sL[p], sR[p], sc.tau, sc.h, kmax);
        }
        s_uo[j][i] = uo;
        s_un[j][i] = un;
    }
    __syncthreads();
    // Phase B: q+ (old u) and p+ (extrapolated 2u+ - u) on the tile's edges.
    const int i = threadIdx.x % kTX, j = threadIdx.x / kTX;
    const int x = x0 + i, y = y0 + j;
    if (x >= W || y >= H) return;
    const long long p = (long long)y * W + x;
    const rfloat uo = s_uo[j][i], un = s_un[j][i];
    out.u[p] = un;
    if (x + 1 < W) {
        const rfloat w = (rfloat)w_h[(long long)y * (W - 1) + x];
        const rfloat gq = uo - s_uo[j][i + 1];
        out.qh[p] = prox_conj(in.qh[p] + sc.tau * gq, w, 0.0, sc.beta_minus, sc.tau);
        const rfloat gp = (2.0 * un - uo) - (2.0 * s_un[j][i + 1] - s_uo[j][i + 1]);
        out.ph[p] = prox_conj(in.ph[p] + sc.sigma * gp, w, sc.eps, sc.delta, sc.sigma);
    }
    if (y + 1 < H) {
        const rfloat w = (rfloat)w_v[p];
        const rfloat gq = uo - s_uo[j + 1][i];
        out.qv[p] = prox_conj(in.qv[p] + sc.tau * gq, w, 0.0, sc.beta_minus, sc.tau);
        const rfloat gp = (2.0 * un - uo) - (2.0 * s_un[j + 1][i] - s_uo[j + 1][i]);
        out.pv[p] = prox_conj(in.pv[p] + sc.sigma * gp, w, sc.eps, sc.delta, sc.sigma);
    }
}

__global__ __launch_bounds__(256) void refine_init_kernel(const int* __restrict__ labels, long long n, int K,
                                                          RefineState s) {
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        int l = labels[p];
        l = l < 0 ? 0 : (l > K - 1 ? K - 1 : l);
        s.u[p] = (rfloat)l;
        s.ph[p] = 0.0;
        s.pv[p] = 0.0;
        s.qh[p] = 0.0;
        s.qv[p] = 0.0;
    }
}

__global__ __launch_bounds__(256) void narrow_kernel(const rfloat* __restrict__ a, float* __restrict__ b, long long n) {
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x)
        b[p] = (float)a[p];
}

// ------------------------------------------------------------------ host
RefineLayout refine_layout(const dm_shape& s) {
    RefineLayout L{};
    const size_t px = (size_t)s.W * s.H * sizeof(rfloat);
    const size_t a = align_up(px, 256);
    L.u0 = 0;
    L.sL = L.u0 + a;
    L.sR = L.sL + a;
    L.state0 = L.sR + a;             // 5 arrays
    L.state1 = L.state0 + 5 * a;     // 5 arrays
    L.total = L.state1 + 5 * a;
    L.plane = a;
    return L;
}

RefineState state_at(char* base, size_t plane) {
    RefineState s;
    s.u = reinterpret_cast<rfloat*>(base);
    s.ph = reinterpret_cast<rfloat*>(base + plane);
    s.pv = reinterpret_cast<rfloat*>(base + 2 * plane);
    s.qh = reinterpret_cast<rfloat*>(base + 3 * plane);
    s.qv = reinterpret_cast<rfloat*>(base + 4 * plane);
    return s;
}

int validate_refine(const dm_shape& s, const dm_refine_params* p) {
    int st = validate_shape(s);
    if (st != DM_OK) return st;
    DM_REQUIRE(p != nullptr, DM_ERR_NULL, "params is NULL");
    DM_REQUIRE(p->C > 0.0f, DM_ERR_PARAM, "C must be > 0");
    DM_REQUIRE(p->eps >= 0.0f && p->eps <= 1.0f, DM_ERR_PARAM, "eps must be in [0, 1]");
    DM_REQUIRE(p->delta >= 0.0f, DM_ERR_PARAM, "delta must be >= 0");
    DM_REQUIRE(p->h > 0.0f, DM_ERR_PARAM, "h must be > 0");
    DM_REQUIRE(p->tau > 0.0f && p->sigma > 0.0f, DM_ERR_PARAM, "tau and sigma must be > 0");
    DM_REQUIRE(p->n_warps >= 0 && p->n_iters >= 0, DM_ERR_PARAM, "n_warps and n_iters must be >= 0");
    return DM_OK;
}

RefineScalars refine_scalars(const dm_refine_params& p) {
    RefineScalars sc;
    sc.tau = p.tau;
    sc.sigma = p.sigma;
    sc.h = p.h;
    sc.eps = p.eps;
    sc.delta = p.delta;
    sc.beta_minus = p.C + p.delta - p.eps * p.delta;
    return sc;
}

}  // namespace dm

using namespace dm;

extern "C" size_t dm_refine_continuous_workspace(dm_shape s, const dm_refine_params* p) {
    if (validate_refine(s, p) != DM_OK) return 0;
    return refine_layout(s).total;
}

extern "C" int dm_refine_continuous(const void* cost, dm_dtype cost_dtype, const int32_t* labels, const float* w_h,
                                    const float* w_v, dm_shape s, const dm_refine_params* p, float* u_out,
                                    void* workspace, size_t workspace_bytes, void* hip_stream) {
    clear_error();
    int st = validate_refine(s, p);
    if (st != DM_OK) return st;
    DM_REQUIRE(cost_dtype == DM_F32 || cost_dtype == DM_F16, DM_ERR_DTYPE, "unknown cost dtype %d", (int)cost_dtype);
    DM_REQUIRE(cost != nullptr && labels != nullptr && u_out != nullptr, DM_ERR_NULL,
               "cost, labels and u_out are required");
    DM_REQUIRE(s.W == 1 || w_h != nullptr, DM_ERR_NULL, "w_h is required when W > 1");
    DM_REQUIRE(s.H == 1 || w_v != nullptr, DM_ERR_NULL, "w_v is required when H > 1");
    const RefineLayout L = refine_layout(s);
    DM_REQUIRE(workspace != nullptr && workspace_bytes >= L.total, DM_ERR_WORKSPACE, "workspace %zu bytes, need %zu",
               workspace_bytes, L.total);
    {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_error("pending HIP error before dm_refine_continuous: %s", hipGetErrorString(e));
            return DM_ERR_HIP;
        }
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    char* ws = static_cast<char*>(workspace);
    rfloat* u0 = reinterpret_cast<rfloat*>(ws + L.u0);
    rfloat* sL = reinterpret_cast<rfloat*>(ws + L.sL);
    rfloat* sR = reinterpret_cast<rfloat*>(ws + L.sR);
    RefineState S[2] = {state_at(ws + L.state0, L.plane), state_at(ws + L.state1, L.plane)};
    const long long npx = (long long)s.W * s.H;
    const unsigned eb = (unsigned)std::min<long long>((npx + 255) / 256, 4096);
    ProfScope ps0(DM_PROF_OTHER, 44.0 * npx, stream);
    hipLaunchKernelGGL(refine_init_kernel, dim3(eb), dim3(256), 0, stream, labels, npx, s.K, S[0]);
    ps0.stop();
    DM_HIP_TRY(hipGetLastError(), "refine init");
    const RefineScalars sc = refine_scalars(*p);
    const dim3 grid((s.W + kTX - 1) / kTX, (s.H + kTY - 1) / kTY);
    int cur = 0;
    for (int wp = 0; wp < p->n_warps; ++wp) {
        ProfScope ps1(DM_PROF_REFINE_LINEARIZE, npx * (4.0 + 4.0 * (cost_dtype == DM_F16 ? 2 : 4) + 12.0), stream);
        if (cost_dtype == DM_F16)
            hipLaunchKernelGGL(linearize_kernel<_Float16>, dim3(eb), dim3(256), 0, stream,
                               static_cast<const _Float16*>(cost), S[cur].u, s.W, s.H, s.K, (rfloat)p->h, u0, sL, sR);
        else
            hipLaunchKernelGGL(linearize_kernel<float>, dim3(eb), dim3(256), 0, stream, static_cast<const float*>(cost),
                               S[cur].u, s.W, s.H, s.K, (rfloat)p->h, u0, sL, sR);
        ps1.stop();
        DM_HIP_TRY(hipGetLastError(), "linearize");
        for (int it = 0; it < p->n_iters; ++it) {
            // per pixel: reads u, u0, sL, sR, 4 duals, 2 weights; writes u and 4 duals
            ProfScope ps2(DM_PROF_REFINE_ITER, npx * (8.0 * 13.0 + 8.0), stream);
            hipLaunchKernelGGL(pdhg_kernel, grid, dim3(256), 0, stream, S[cur], S[cur ^ 1], u0, sL, sR, w_h, w_v, s.W,
                               s.H, s.K, sc);
            cur ^= 1;
        }
        DM_HIP_TRY(hipGetLastError(), "pdhg");
    }
    ProfScope ps3(DM_PROF_OTHER, 12.0 * npx, stream);
    hipLaunchKernelGGL(narrow_kernel, dim3(eb), dim3(256), 0, stream, S[cur].u, u_out, npx);
    DM_HIP_TRY(hipGetLastError(), "copy u");
    return DM_OK;
}
