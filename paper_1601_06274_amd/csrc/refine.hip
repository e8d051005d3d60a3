// refine.hip - continuous refinement by the non-linear primal-dual method on gfx950,
// and its adjoint.
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
//   pdhg_fused_kernel: kFS iterations per launch on a tile extended by kFS pixels, the state
//                      in LDS between iterations (temporal tiling, pdhg.h).  Optionally
//                      records the branch taken by every prox (16-bit mask per pixel and
//                      iteration) for the adjoint.  batched_pdhg_fused_kernel: the same
//                      per (instance, tile) of a batched plan's table.
// State and arithmetic are FP64 (rfloat); the cost volume and edge weights are read in
// their storage types and widened.  The working set (about 11 doubles per pixel) stays
// in L2 / MALL at these sizes, so the iteration is bound by on-chip bandwidth and
// launch latency, not HBM.
//
// Adjoint (reverse mode).  Every map of the iteration is piecewise linear; given the
// recorded branches, the adjoint of one iteration is a linear stencil reaching one pixel,
// run kAS reverse iterations per launch by temporal tiling (pdhg_adjoint_fused_kernel).
// At the start of each warp (processed in reverse) the accumulated adjoints of the
// slopes and of u0 are pushed through the linearisation into the cost volume and into u
// (linearize_adjoint_kernel).  At kinks
// (exact ties of a branch test) the derivative of the branch that the forward took is
// used; on the interpolated data term at integer arguments the segment [k, k+1].
#include <algorithm>

#include "common.h"
#include "pdhg.h"
#include "refine.h"

namespace dm {

template <typename TT>
__device__ __forceinline__ rfloat cost_at(const TT* __restrict__ th, long long p, int K, int k) {
    return (rfloat)(float)th[p * K + k];
}

// Linear interpolation of the cost along the label axis; also the segment used.
template <typename TT>
__device__ __forceinline__ rfloat interp(const TT* __restrict__ th, long long p, int K, rfloat v, int* k0_out = nullptr,
                                         rfloat* t_out = nullptr) {
    v = fmin(fmax(v, 0.0), (rfloat)(K - 1));
    int k0 = (int)floor(v);
    k0 = k0 < K - 1 ? k0 : K - 1;
    const int k1 = k0 + 1 < K - 1 ? k0 + 1 : K - 1;
    const rfloat t = v - (rfloat)k0;
    if (k0_out) *k0_out = k0;
    if (t_out) *t_out = t;
    return (1.0 - t) * cost_at(th, p, K, k0) + t * cost_at(th, p, K, k1);
}

template <typename TT>
__device__ __forceinline__ void linearize_px(const TT* __restrict__ th, const rfloat* __restrict__ u, long long p,
                                             int K, rfloat h, rfloat* __restrict__ u0, rfloat* __restrict__ sL,
                                             rfloat* __restrict__ sR) {
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

template <typename TT>
__global__ __launch_bounds__(256) void linearize_kernel(const TT* __restrict__ th, const rfloat* __restrict__ u, int W,
                                                        int H, int K, rfloat h, rfloat* __restrict__ u0,
                                                        rfloat* __restrict__ sL, rfloat* __restrict__ sR) {
    const long long n = (long long)W * H;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x)
        linearize_px(th, u, p, K, h, u0, sL, sR);
}

// prox of tau * D~ (two-slope soft threshold) and the box [u0 - h, u0 + h] n [0, K-1].
// code: bits 0-1 zone (0 middle, 1 right slope, 2 left slope), bits 2-3 clamp (0, 1 low, 2 high).
// (with selects: every candidate computed, no divergent branches)
__device__ __forceinline__ rfloat prox_data(rfloat uh, rfloat u0, rfloat l, rfloat r, rfloat tau, rfloat h, rfloat kmax,
                                            int& code) {
    const bool zr = uh > u0 + tau * r;
    const bool zl = !zr && uh < u0 + tau * l;
    rfloat v = zr ? uh - tau * r : (zl ? uh - tau * l : u0);
    const int zone = zr ? 1 : (zl ? 2 : 0);
    const rfloat lo = fmax(u0 - h, 0.0);
    const rfloat hi = fmin(u0 + h, kmax);
    const bool below = v < lo, above = !below && v > hi;
    v = below ? lo : (above ? hi : v);
    const int cl = below ? 1 : (above ? 2 : 0);
    code = zone | (cl << 2);
    return v;
}

struct TwoSlopeProx {
    const rfloat* u0;
    const rfloat* sL;
    const rfloat* sR;
    rfloat tau, h;
    struct Px {
        rfloat u0, sL, sR;
    };
    __device__ __forceinline__ rfloat operator()(rfloat uh, long long p, rfloat kmax, int& code) const {
        return prox_data(uh, u0[p], sL[p], sR[p], tau, h, kmax, code);
    }
    __device__ __forceinline__ Px load(long long p) const { return Px{u0[p], sL[p], sR[p]}; }
    __device__ __forceinline__ rfloat apply(rfloat uh, const Px& d, rfloat kmax, int& code) const {
        return prox_data(uh, d.u0, d.sL, d.sR, tau, h, kmax, code);
    }
};

__global__ __launch_bounds__(256, 2) void pdhg_fused_kernel(const RefineState in, RefineState out,
                                                         const rfloat* __restrict__ u0, const rfloat* __restrict__ sL,
                                                         const rfloat* __restrict__ sR, const float* __restrict__ w_h,
                                                         const float* __restrict__ w_v, int W, int H, int K,
                                                         RefineScalars sc, uint16_t* __restrict__ mask0,
                                                         size_t mask_stride, int n_iter) {
    pdhg_fused_tile<kFTX, kFTY, kFS>(in, out, TwoSlopeProx{u0, sL, sR, sc.tau, sc.h}, w_h, w_v, W, H, K, sc, mask0,
                                     mask_stride, n_iter, blockIdx.x * kFTX, blockIdx.y * kFTY);
}

// ------------------------------------------------------------------ batched forms
// Many instances of (possibly) different sizes: block b of a launch works on the
// pixel chunk or tile listed at index b of a table built by the plan.
__global__ __launch_bounds__(256) void batched_refine_init_kernel(const RefBatchInst* __restrict__ insts,
                                                                  const RefChunk* __restrict__ chunks, int cur) {
    const RefChunk c = chunks[blockIdx.x];
    const RefBatchInst& in = insts[c.inst];
    const RefineState s = in.S[cur];
    for (long long p = c.start + threadIdx.x; p < c.start + c.count; p += blockDim.x) {
        int l = in.labels[p];
        l = l < 0 ? 0 : (l > in.K - 1 ? in.K - 1 : l);
        s.u[p] = (rfloat)l;
        s.ph[p] = 0.0;
        s.pv[p] = 0.0;
        s.qh[p] = 0.0;
        s.qv[p] = 0.0;
    }
}

template <typename TT>
__global__ __launch_bounds__(256) void batched_linearize_kernel(const RefBatchInst* __restrict__ insts,
                                                                const RefChunk* __restrict__ chunks, int cur,
                                                                rfloat h) {
    const RefChunk c = chunks[blockIdx.x];
    const RefBatchInst& in = insts[c.inst];
    for (long long p = c.start + threadIdx.x; p < c.start + c.count; p += blockDim.x)
        linearize_px(static_cast<const TT*>(in.theta), in.S[cur].u, p, in.K, h, in.u0, in.sL, in.sR);
}

__global__ __launch_bounds__(256, 2) void batched_pdhg_fused_kernel(const RefBatchInst* __restrict__ insts,
                                                                    const RefTile* __restrict__ tiles, int cur,
                                                                    RefineScalars sc, int n_iter) {
    const RefTile t = tiles[blockIdx.x];
    const RefBatchInst& in = insts[t.inst];
    pdhg_fused_tile<kFTX, kFTY, kFS>(in.S[cur], in.S[cur ^ 1], TwoSlopeProx{in.u0, in.sL, in.sR, sc.tau, sc.h},
                                     in.w_h, in.w_v, in.W, in.H, in.K, sc, nullptr, 0, n_iter, t.bx * kFTX,
                                     t.by * kFTY);
}

__global__ __launch_bounds__(256) void batched_narrow_kernel(const RefBatchInst* __restrict__ insts,
                                                             const RefChunk* __restrict__ chunks, int cur) {
    const RefChunk c = chunks[blockIdx.x];
    const RefBatchInst& in = insts[c.inst];
    for (long long p = c.start + threadIdx.x; p < c.start + c.count; p += blockDim.x) in.u_out[p] = (float)in.S[cur].u[p];
}

void refine_tile_extent(int W, int H, int& nbx, int& nby) {
    nbx = (W + kFTX - 1) / kFTX;
    nby = (H + kFTY - 1) / kFTY;
}

hipError_t launch_batched_refine(const RefBatchInst* insts, const RefChunk* chunks, int n_chunks, const RefTile* tiles,
                                 int n_tiles, dm_dtype dt, const dm_refine_params& p, hipStream_t st) {
    const RefineScalars sc = refine_scalars(p);
    hipLaunchKernelGGL(batched_refine_init_kernel, dim3(n_chunks), dim3(256), 0, st, insts, chunks, 0);
    int cur = 0;
    for (int wp = 0; wp < p.n_warps; ++wp) {
        if (dt == DM_F16)
            hipLaunchKernelGGL(batched_linearize_kernel<_Float16>, dim3(n_chunks), dim3(256), 0, st, insts, chunks, cur,
                               (rfloat)p.h);
        else
            hipLaunchKernelGGL(batched_linearize_kernel<float>, dim3(n_chunks), dim3(256), 0, st, insts, chunks, cur,
                               (rfloat)p.h);
        // kFS iterations per launch, as the single-instance refinement
        for (int it0 = 0; it0 < p.n_iters; it0 += kFS) {
            const int nit = std::min(kFS, p.n_iters - it0);
            hipLaunchKernelGGL(batched_pdhg_fused_kernel, dim3(n_tiles), dim3(256), 0, st, insts, tiles, cur, sc, nit);
            cur ^= 1;
        }
    }
    hipLaunchKernelGGL(batched_narrow_kernel, dim3(n_chunks), dim3(256), 0, st, insts, chunks, cur);
    return hipGetLastError();
}

// d(prox)/dt for a conjugate-prox branch code, and d(prox)/dw (alpha, -alpha, 1, -1 for
// codes 1-4, else 0), as selects.
__device__ __forceinline__ rfloat conj_dt(int code) { return code == 0 ? 1.0 : 0.0; }
__device__ __forceinline__ rfloat conj_dw(int code, rfloat alpha) {
    const rfloat s = (code == 1 || code == 3) ? 1.0 : ((code == 2 || code == 4) ? -1.0 : 0.0);
    return code >= 3 ? s : s * alpha;
}

// n_iter <= kAS reverse iterations per launch (temporal tiling, as pdhg_fused_tile): the
// adjoint of iteration it reaches one pixel (diagonals included), so a kATX x kATY output
// tile is exact after n_iter iterations on the tile extended by kAS pixels on every side.
// The adjoint state sits in LDS between iterations; the accumulators of the tile's pixels
// (u0, slopes, edge weights) are loaded once, carried in registers in the order of the
// additions of one reverse iteration at a time and stored once, so the results do not
// depend on the tiling (bit for bit).  Per iteration: the branch masks of the region into
// LDS; phase A the adjoint of u-hat and the new u adjoint (from the own and the left /
// upper edges); phase B the edge adjoints in place and the accumulators.  mask_hi: the mask plane of
// the launch's first (latest) iteration; earlier iterations lie mask_stride elements
// below, one plane each.
__global__ __launch_bounds__(256) void pdhg_adjoint_fused_kernel(const RefineState nxt, RefineState prv,
                                                                 const uint16_t* __restrict__ mask_hi,
                                                                 size_t mask_stride, int n_iter,
                                                                 const rfloat* __restrict__ u0, int W, int H, int K,
                                                                 RefineScalars sc, rfloat* __restrict__ acc_u0,
                                                                 rfloat* __restrict__ acc_sL, rfloat* __restrict__ acc_sR,
                                                                 rfloat* __restrict__ acc_wh,
                                                                 rfloat* __restrict__ acc_wv) {
    constexpr int TX = kATX, TY = kATY, S = kAS;
    constexpr int RX = TX + 2 * S, RY = TY + 2 * S, NP = RX * RY;
    constexpr int NT = 256, PPT = (NP + NT - 1) / NT;
    // the u adjoint of a pixel is read and written by that pixel only: in registers
    __shared__ rfloat s_ph[NP], s_pv[NP], s_qh[NP], s_qv[NP], s_uhb[NP];
    __shared__ uint16_t s_m[NP];
    const int ox = (int)blockIdx.x * TX - S, oy = (int)blockIdx.y * TY - S;
    const rfloat kmax = (rfloat)(K - 1);
    // per slot: the pixel's u0, and for the tile's own pixels the accumulators
    rfloat su[PPT], c0[PPT], a_u0[PPT], a_sL[PPT], a_sR[PPT], a_wh[PPT], a_wv[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        su[k] = c0[k] = a_u0[k] = a_sL[k] = a_sR[k] = a_wh[k] = a_wv[k] = 0.0;
        if (idx >= NP) break;
        const int rx = idx % RX, ry = idx / RX;
        const int x = ox + rx, y = oy + ry;
        rfloat u = 0.0, ph = 0.0, pv = 0.0, qh = 0.0, qv = 0.0;
        if (x >= 0 && x < W && y >= 0 && y < H) {
            const long long p = (long long)y * W + x;
            u = nxt.u[p];
            ph = nxt.ph[p];
            pv = nxt.pv[p];
            qh = nxt.qh[p];
            qv = nxt.qv[p];
            c0[k] = u0[p];
            if (rx >= S && rx < S + TX && ry >= S && ry < S + TY) {
                a_u0[k] = acc_u0[p];
                a_sL[k] = acc_sL[p];
                a_sR[k] = acc_sR[p];
                a_wh[k] = acc_wh[p];
                a_wv[k] = acc_wv[p];
            }
        }
        su[k] = u;
        s_ph[idx] = ph;
        s_pv[idx] = pv;
        s_qh[idx] = qh;
        s_qv[idx] = qv;
    }
    for (int it = 0; it < n_iter; ++it) {
        const uint16_t* mask = mask_hi - (size_t)it * mask_stride;
        uint32_t mm[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int idx = (int)threadIdx.x + k * NT;
            mm[k] = 0u;
            if (idx >= NP) break;
            const int x = ox + idx % RX, y = oy + idx / RX;
            if (x >= 0 && x < W && y >= 0 && y < H) mm[k] = mask[(long long)y * W + x];
            s_m[idx] = (uint16_t)mm[k];
        }
        __syncthreads();  // the masks, and (it > 0) the previous iteration's edges
        rfloat ubt[PPT];
        // Phase A: adjoint of u-hat, and the adjoint of the iteration's input u.
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int idx = (int)threadIdx.x + k * NT;
            ubt[k] = 0.0;
            if (idx >= NP) break;
            const int rx = idx % RX, ry = idx / RX;
            const int x = ox + rx, y = oy + ry;
            rfloat uhb = 0.0, un = 0.0;
            if (x >= 0 && x < W && y >= 0 && y < H) {
                const uint32_t m = mm[k];
                // (A^T p-bar-hat) and (A^T q-bar-hat): own edges, then the left / upper ones
                rfloat atp = 0.0, atq = 0.0;
                if (x + 1 < W) {
                    atp += s_ph[idx] * conj_dt(mfield(m, 10, 3));
                    atq += s_qh[idx] * conj_dt(mfield(m, 4, 3));
                }
                if (y + 1 < H) {
                    atp += s_pv[idx] * conj_dt(mfield(m, 13, 3));
                    atq += s_qv[idx] * conj_dt(mfield(m, 7, 3));
                }
                if (x > 0 && rx > 0) {
                    const uint32_t ml = s_m[idx - 1];
                    atp -= s_ph[idx - 1] * conj_dt(mfield(ml, 10, 3));
                    atq -= s_qh[idx - 1] * conj_dt(mfield(ml, 4, 3));
                }
                if (y > 0 && ry > 0) {
                    const uint32_t mu = s_m[idx - RX];
                    atp -= s_pv[idx - RX] * conj_dt(mfield(mu, 13, 3));
                    atq -= s_qv[idx - RX] * conj_dt(mfield(mu, 7, 3));
                }
                ubt[k] = su[k] + 2.0 * sc.sigma * atp;
                const int zone = mfield(m, 0, 2), cl = mfield(m, 2, 2);
                uhb = (cl == 0 && zone != 0) ? ubt[k] : 0.0;
                un = uhb - sc.sigma * atp + sc.tau * atq;
            }
            s_uhb[idx] = uhb;
            su[k] = un;
        }
        __syncthreads();
        // Phase B: the edges' adjoints in place, the accumulators of the tile's pixels.
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int idx = (int)threadIdx.x + k * NT;
            if (idx >= NP) break;
            const int rx = idx % RX, ry = idx / RX;
            const int x = ox + rx, y = oy + ry;
            if (x < 0 || x >= W || y < 0 || y >= H) continue;
            const uint32_t m = mm[k];
            const rfloat uhb = s_uhb[idx];
            if (x + 1 < W) {
                const int cq = mfield(m, 4, 3), cp = mfield(m, 10, 3);
                const int r = rx + 1 < RX ? idx + 1 : idx;  // beyond the region: a value that is never used
                const rfloat du = uhb - s_uhb[r];
                const rfloat ph = s_ph[idx], qh = s_qh[idx];
                s_ph[idx] = ph * conj_dt(cp) - sc.tau * du;
                s_qh[idx] = qh * conj_dt(cq) + sc.tau * du;
                a_wh[k] += ph * conj_dw(cp, sc.eps) + qh * conj_dw(cq, 0.0);
            }
            if (y + 1 < H) {
                const int cq = mfield(m, 7, 3), cp = mfield(m, 13, 3);
                const int d = ry + 1 < RY ? idx + RX : idx;
                const rfloat du = uhb - s_uhb[d];
                const rfloat pv = s_pv[idx], qv = s_qv[idx];
                s_pv[idx] = pv * conj_dt(cp) - sc.tau * du;
                s_qv[idx] = qv * conj_dt(cq) + sc.tau * du;
                a_wv[k] += pv * conj_dw(cp, sc.eps) + qv * conj_dw(cq, 0.0);
            }
            // u-prox adjoint into u0 and the slopes (selects)
            const int zone = mfield(m, 0, 2), cl = mfield(m, 2, 2);
            const bool pass_u0 = cl == 0 ? zone == 0 : (cl == 1 ? c0[k] - sc.h >= 0.0 : c0[k] + sc.h <= kmax);
            a_u0[k] += ubt[k] * (pass_u0 ? 1.0 : 0.0);
            a_sR[k] = (cl == 0 && zone == 1) ? a_sR[k] - sc.tau * ubt[k] : a_sR[k];
            a_sL[k] = (cl == 0 && zone == 2) ? a_sL[k] - sc.tau * ubt[k] : a_sL[k];
        }
        __syncthreads();  // phase B's edges before the next iteration reads them
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        if (idx >= NP) break;
        const int rx = idx % RX, ry = idx / RX;
        const int x = ox + rx, y = oy + ry;
        if (rx < S || rx >= S + TX || ry < S || ry >= S + TY || x >= W || y >= H) continue;
        const long long p = (long long)y * W + x;
        prv.u[p] = su[k];
        prv.ph[p] = s_ph[idx];
        prv.pv[p] = s_pv[idx];
        prv.qh[p] = s_qh[idx];
        prv.qv[p] = s_qv[idx];
        acc_u0[p] = a_u0[k];
        acc_sL[p] = a_sL[k];
        acc_sR[p] = a_sR[k];
        acc_wh[p] = a_wh[k];
        acc_wv[p] = a_wv[k];
    }
}

// Adjoint of the per-warp linearisation at u0: pushes the accumulated slope / u0
// adjoints into the cost volume gradient and into the adjoint of u at the warp start
// (only when that u is a variable, i.e. not the first warp).  Clears the accumulators.
template <typename TT>
__global__ __launch_bounds__(256) void linearize_adjoint_kernel(const TT* __restrict__ th, const rfloat* __restrict__ u0w,
                                                                int W, int H, int K, rfloat h, rfloat* __restrict__ acc_u0,
                                                                rfloat* __restrict__ acc_sL,
                                                                rfloat* __restrict__ acc_sR, rfloat* __restrict__ ubar,
                                                                int add_to_u, float* __restrict__ grad_cost) {
    const long long n = (long long)W * H;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        const rfloat c = u0w[p];
        const rfloat lb = acc_sL[p], rb = acc_sR[p];
        rfloat u0b = acc_u0[p];
        acc_u0[p] = 0.0;
        acc_sL[p] = 0.0;
        acc_sR[p] = 0.0;
        const rfloat Dc = interp(th, p, K, c);
        const rfloat Dm = interp(th, p, K, c - h);
        const rfloat Dp = interp(th, p, K, c + h);
        const rfloat l_raw = (Dc - Dm) / h, r_raw = (Dp - Dc) / h;
        const bool has_l = c - h >= 0.0;
        const bool has_r = c + h <= (rfloat)(K - 1);
        const rfloat l1 = has_l ? l_raw : (has_r ? r_raw : 0.0);
        const rfloat r1 = has_r ? r_raw : (has_l ? l_raw : 0.0);
        rfloat l1b = lb, r1b = rb;
        if (l1 > r1) {
            l1b = 0.5 * (lb + rb);
            r1b = l1b;
        }
        const rfloat lrb = (has_l ? l1b : 0.0) + ((!has_r && has_l) ? r1b : 0.0);
        const rfloat rrb = (has_r ? r1b : 0.0) + ((!has_l && has_r) ? l1b : 0.0);
        const rfloat Dcb = (lrb - rrb) / h, Dmb = -lrb / h, Dpb = rrb / h;
        const rfloat vs[3] = {c, c - h, c + h};
        const rfloat Db[3] = {Dcb, Dmb, Dpb};
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            if (Db[e] == 0.0) continue;
            int k0;
            rfloat t;
            interp(th, p, K, vs[e], &k0, &t);
            const int k1 = k0 + 1 < K - 1 ? k0 + 1 : K - 1;
            grad_cost[p * K + k0] += (float)((1.0 - t) * Db[e]);
            grad_cost[p * K + k1] += (float)(t * Db[e]);
            const bool inside = vs[e] >= 0.0 && vs[e] <= (rfloat)(K - 1);
            if (inside) u0b += Db[e] * (cost_at(th, p, K, k1) - cost_at(th, p, K, k0));
        }
        if (add_to_u) ubar[p] += u0b;
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

__global__ __launch_bounds__(256) void adjoint_init_kernel(const float* __restrict__ grad_u, long long n, RefineState s,
                                                           rfloat* __restrict__ a0, rfloat* __restrict__ a1,
                                                           rfloat* __restrict__ a2, rfloat* __restrict__ a3,
                                                           rfloat* __restrict__ a4) {
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        s.u[p] = (rfloat)grad_u[p];
        s.ph[p] = 0.0;
        s.pv[p] = 0.0;
        s.qh[p] = 0.0;
        s.qv[p] = 0.0;
        a0[p] = 0.0;
        a1[p] = 0.0;
        a2[p] = 0.0;
        a3[p] = 0.0;
        a4[p] = 0.0;
    }
}

__global__ __launch_bounds__(256) void narrow_kernel(const rfloat* __restrict__ a, float* __restrict__ b, long long n) {
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x)
        b[p] = (float)a[p];
}

// Edge-weight gradients from the per-pixel FP64 accumulators (overwrite or add).
__global__ __launch_bounds__(256) void edge_grad_kernel(const rfloat* __restrict__ acc_wh,
                                                        const rfloat* __restrict__ acc_wv, int W, int H, int accumulate,
                                                        float* __restrict__ gw_h, float* __restrict__ gw_v) {
    const long long n = (long long)W * H;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(p % W), y = (int)(p / W);
        if (gw_h != nullptr && x + 1 < W) {
            const long long e = (long long)y * (W - 1) + x;
            gw_h[e] = (accumulate ? gw_h[e] : 0.0f) + (float)acc_wh[p];
        }
        if (gw_v != nullptr && y + 1 < H) gw_v[p] = (accumulate ? gw_v[p] : 0.0f) + (float)acc_wv[p];
    }
}

__global__ void fill_zero_f32_kernel(float* __restrict__ p, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// ------------------------------------------------------------------ host
RefineLayout refine_layout(const dm_shape& s, const dm_refine_params* p) {
    RefineLayout L{};
    const size_t px = (size_t)s.W * s.H;
    const size_t a = align_up(px * sizeof(rfloat), 256);
    L.u0 = 0;
    L.sL = L.u0 + a;
    L.sR = L.sL + a;
    L.state0 = L.sR + a;             // 5 arrays
    L.state1 = L.state0 + 5 * a;     // 5 arrays
    L.total = L.state1 + 5 * a;
    L.plane = a;
    L.tape_u0 = L.tape_mask = 0;
    if (p != nullptr && p->keep_tape) {
        L.tape_u0 = L.total;
        L.total += (size_t)p->n_warps * a;
        L.tape_mask = L.total;
        L.mask_plane = align_up(px * sizeof(uint16_t), 256);
        L.total += (size_t)p->n_warps * p->n_iters * L.mask_plane;
    }
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
    DM_REQUIRE(p->keep_tape == 0 || p->keep_tape == 1, DM_ERR_PARAM, "keep_tape must be 0 or 1");
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

struct RefineBwdLayout {
    size_t state0, state1, acc, total, plane;
};

RefineBwdLayout refine_bwd_layout(const dm_shape& s) {
    RefineBwdLayout L{};
    const size_t a = align_up((size_t)s.W * s.H * sizeof(rfloat), 256);
    L.plane = a;
    L.state0 = 0;
    L.state1 = 5 * a;
    L.acc = 10 * a;  // acc_u0, acc_sL, acc_sR, acc_wh, acc_wv
    L.total = 15 * a;
    return L;
}

int pending_hip(const char* where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("pending HIP error before %s: %s", where, hipGetErrorString(e));
        return DM_ERR_HIP;
    }
    return DM_OK;
}

}  // namespace dm

using namespace dm;

extern "C" size_t dm_refine_continuous_workspace(dm_shape s, const dm_refine_params* p) {
    if (validate_refine(s, p) != DM_OK) return 0;
    return refine_layout(s, p).total;
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
    const RefineLayout L = refine_layout(s, p);
    DM_REQUIRE(workspace != nullptr && workspace_bytes >= L.total, DM_ERR_WORKSPACE, "workspace %zu bytes, need %zu",
               workspace_bytes, L.total);
    if ((st = pending_hip("dm_refine_continuous")) != DM_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    char* ws = static_cast<char*>(workspace);
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
    const dim3 fgrid((s.W + kFTX - 1) / kFTX, (s.H + kFTY - 1) / kFTY);
    int cur = 0;
    for (int wp = 0; wp < p->n_warps; ++wp) {
        // with a tape, every warp keeps its own u0 (the adjoint needs it)
        rfloat* u0 = p->keep_tape ? reinterpret_cast<rfloat*>(ws + L.tape_u0 + (size_t)wp * L.plane)
                                  : reinterpret_cast<rfloat*>(ws + L.u0);
        ProfScope ps1(DM_PROF_REFINE_LINEARIZE, npx * (4.0 + 4.0 * (cost_dtype == DM_F16 ? 2 : 4) + 12.0), stream);
        if (cost_dtype == DM_F16)
            hipLaunchKernelGGL(linearize_kernel<_Float16>, dim3(eb), dim3(256), 0, stream,
                               static_cast<const _Float16*>(cost), S[cur].u, s.W, s.H, s.K, (rfloat)p->h, u0, sL, sR);
        else
            hipLaunchKernelGGL(linearize_kernel<float>, dim3(eb), dim3(256), 0, stream, static_cast<const float*>(cost),
                               S[cur].u, s.W, s.H, s.K, (rfloat)p->h, u0, sL, sR);
        ps1.stop();
        DM_HIP_TRY(hipGetLastError(), "linearize");
        // kFS iterations per launch, the state on chip in between
        for (int it0 = 0; it0 < p->n_iters; it0 += kFS) {
            const int nit = std::min(kFS, p->n_iters - it0);
            uint16_t* mask0 = p->keep_tape ? reinterpret_cast<uint16_t*>(
                                                 ws + L.tape_mask + ((size_t)wp * p->n_iters + it0) * L.mask_plane)
                                           : nullptr;
            // per pixel and iteration: reads u, u0, sL, sR, 4 duals, 2 weights; writes u and 4 duals
            ProfScope ps2(DM_PROF_REFINE_ITER, nit * npx * (8.0 * 13.0 + 8.0), stream);
            hipLaunchKernelGGL(pdhg_fused_kernel, fgrid, dim3(256), 0, stream, S[cur], S[cur ^ 1], u0, sL, sR, w_h,
                               w_v, s.W, s.H, s.K, sc, mask0, L.mask_plane / sizeof(uint16_t), nit);
            cur ^= 1;
        }
        DM_HIP_TRY(hipGetLastError(), "pdhg");
    }
    ProfScope ps3(DM_PROF_OTHER, 12.0 * npx, stream);
    hipLaunchKernelGGL(narrow_kernel, dim3(eb), dim3(256), 0, stream, S[cur].u, u_out, npx);
    DM_HIP_TRY(hipGetLastError(), "copy u");
    return DM_OK;
}

extern "C" size_t dm_refine_continuous_backward_workspace(dm_shape s, const dm_refine_params* p) {
    if (validate_refine(s, p) != DM_OK) return 0;
    return refine_bwd_layout(s).total;
}

extern "C" int dm_refine_continuous_backward(const float* grad_u, const void* cost, dm_dtype cost_dtype,
                                             const float* w_h, const float* w_v, dm_shape s,
                                             const dm_refine_params* p, const void* fwd_workspace,
                                             size_t fwd_workspace_bytes, float* grad_cost, float* grad_w_h,
                                             float* grad_w_v, int accumulate, void* workspace, size_t workspace_bytes,
                                             void* hip_stream) {
    clear_error();
    int st = validate_refine(s, p);
    if (st != DM_OK) return st;
    DM_REQUIRE(p->keep_tape == 1, DM_ERR_PARAM, "the forward must have been run with keep_tape = 1");
    DM_REQUIRE(cost_dtype == DM_F32 || cost_dtype == DM_F16, DM_ERR_DTYPE, "unknown cost dtype %d", (int)cost_dtype);
    DM_REQUIRE(grad_u != nullptr && cost != nullptr && grad_cost != nullptr && fwd_workspace != nullptr, DM_ERR_NULL,
               "grad_u, cost, grad_cost and the forward workspace are required");
    DM_REQUIRE(accumulate == 0 || accumulate == 1, DM_ERR_PARAM, "accumulate must be 0 or 1");
    const RefineLayout LF = refine_layout(s, p);
    DM_REQUIRE(fwd_workspace_bytes >= LF.total, DM_ERR_WORKSPACE, "forward workspace %zu bytes, need %zu",
               fwd_workspace_bytes, LF.total);
    const RefineBwdLayout LB = refine_bwd_layout(s);
    DM_REQUIRE(workspace != nullptr && workspace_bytes >= LB.total, DM_ERR_WORKSPACE, "workspace %zu bytes, need %zu",
               workspace_bytes, LB.total);
    if ((st = pending_hip("dm_refine_continuous_backward")) != DM_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const char* fws = static_cast<const char*>(fwd_workspace);
    char* ws = static_cast<char*>(workspace);
    RefineState A[2] = {state_at(ws + LB.state0, LB.plane), state_at(ws + LB.state1, LB.plane)};
    rfloat* acc = reinterpret_cast<rfloat*>(ws + LB.acc);
    rfloat* acc_u0 = acc;
    rfloat* acc_sL = reinterpret_cast<rfloat*>(ws + LB.acc + LB.plane);
    rfloat* acc_sR = reinterpret_cast<rfloat*>(ws + LB.acc + 2 * LB.plane);
    rfloat* acc_wh = reinterpret_cast<rfloat*>(ws + LB.acc + 3 * LB.plane);
    rfloat* acc_wv = reinterpret_cast<rfloat*>(ws + LB.acc + 4 * LB.plane);
    const long long npx = (long long)s.W * s.H;
    const unsigned eb = (unsigned)std::min<long long>((npx + 255) / 256, 4096);
    if (!accumulate) {
        const long long vol = npx * s.K;
        hipLaunchKernelGGL(fill_zero_f32_kernel, dim3(2048), dim3(256), 0, stream, grad_cost, vol);
        DM_HIP_TRY(hipGetLastError(), "zero grad");
    }
    hipLaunchKernelGGL(adjoint_init_kernel, dim3(eb), dim3(256), 0, stream, grad_u, npx, A[0], acc_u0, acc_sL, acc_sR,
                       acc_wh, acc_wv);
    DM_HIP_TRY(hipGetLastError(), "adjoint init");
    const RefineScalars sc = refine_scalars(*p);
    const dim3 fgrid((s.W + kATX - 1) / kATX, (s.H + kATY - 1) / kATY);
    int cur = 0;
    for (int wp = p->n_warps - 1; wp >= 0; --wp) {
        const rfloat* u0 = reinterpret_cast<const rfloat*>(fws + LF.tape_u0 + (size_t)wp * LF.plane);
        // kAS reverse iterations per launch, the adjoint state on chip in between
        for (int hi = p->n_iters - 1; hi >= 0; hi -= kAS) {
            const int nit = std::min(kAS, hi + 1);
            const uint16_t* mask = reinterpret_cast<const uint16_t*>(
                fws + LF.tape_mask + ((size_t)wp * p->n_iters + hi) * LF.mask_plane);
            hipLaunchKernelGGL(pdhg_adjoint_fused_kernel, fgrid, dim3(256), 0, stream, A[cur], A[cur ^ 1], mask,
                               LF.mask_plane / sizeof(uint16_t), nit, u0, s.W, s.H, s.K, sc, acc_u0, acc_sL, acc_sR,
                               acc_wh, acc_wv);
            cur ^= 1;
        }
        DM_HIP_TRY(hipGetLastError(), "pdhg adjoint");
        if (cost_dtype == DM_F16)
            hipLaunchKernelGGL(linearize_adjoint_kernel<_Float16>, dim3(eb), dim3(256), 0, stream,
                               static_cast<const _Float16*>(cost), u0, s.W, s.H, s.K, (rfloat)p->h, acc_u0, acc_sL,
                               acc_sR, A[cur].u, wp > 0 ? 1 : 0, grad_cost);
        else
            hipLaunchKernelGGL(linearize_adjoint_kernel<float>, dim3(eb), dim3(256), 0, stream,
                               static_cast<const float*>(cost), u0, s.W, s.H, s.K, (rfloat)p->h, acc_u0, acc_sL,
                               acc_sR, A[cur].u, wp > 0 ? 1 : 0, grad_cost);
        DM_HIP_TRY(hipGetLastError(), "linearize adjoint");
    }
    if (grad_w_h != nullptr || grad_w_v != nullptr) {
        hipLaunchKernelGGL(edge_grad_kernel, dim3(eb), dim3(256), 0, stream, acc_wh, acc_wv, s.W, s.H, accumulate,
                           grad_w_h, grad_w_v);
        DM_HIP_TRY(hipGetLastError(), "edge grads");
    }
    return DM_OK;
}
