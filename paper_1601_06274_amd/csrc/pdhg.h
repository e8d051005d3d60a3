// pdhg.h - one primal-dual iteration of the refinement on a tile (Sec. 2.4, eq. cont_iterates),
// shared by the stereo refinement (two-slope data model, Sec. 3.1) and the flow refinement
// (quadratic data model per component, Sec. 3.2): the iteration differs only in the prox
// of the data term, a template argument.
//
// With x = (u, q), y = (p, d = 1), per pixel / edge:
//     u+ = prox_{tau D~}( u - tau A^T (p - q) )
//     q+ = prox_{tau R_-^*}( q + tau A u )
//     p+ = prox_{sigma R_+^*}( p + sigma A (2 u+ - u) ),
// (Au)_e = u_i - u_j for the right / lower neighbour j of i.  Edge arrays are stored per
// pixel: ph/qh at (x, y) belong to the edge (x, y)-(x+1, y) (unused in the last column),
// pv/qv to (x, y)-(x, y+1) (unused in the last row).  State is double buffered between
// launches (every read of a launch sees the previous launch's iterate).  DataProx is the
// prox of tau D~ of a pixel around its model: load(p) reads the pixel's model once per
// launch, apply(uh, model, kmax, code) returns the prox and its branch code (4 bits).
#pragma once

#include "refine.h"

namespace dm {

// Branch codes of the conjugate prox (3 bits): 0 = identity slope in t, 1 / 2 = flat at
// +alpha*w / -alpha*w, 3 / 4 = clamped at +w / -w.
// Written with selects (every candidate computed, no divergent branches).
__device__ __forceinline__ rfloat prox_conj(rfloat t, rfloat w, rfloat alpha, rfloat beta, rfloat step, int& code) {
    const rfloat a = fabs(t);
    const rfloat aw = alpha * w;
    const rfloat sh = a - beta * step;
    const bool inner = a <= aw;
    const bool flat = !inner && sh < aw;
    rfloat r = inner ? t : copysign(flat ? aw : sh, t);
    const int c = flat ? (t > 0.0 ? 1 : 2) : 0;
    const bool lo = r < -w, hi = r > w;
    r = lo ? -w : (hi ? w : r);
    code = lo ? 4 : (hi ? 3 : c);
    return r;
}

// Mask layout (uint16 per pixel and iteration): [0,4) u-prox, [4,7) qh, [7,10) qv,
// [10,13) ph, [13,16) pv.
__device__ __forceinline__ int mfield(uint32_t m, int shift, int bits) { return (int)((m >> shift) & ((1u << bits) - 1u)); }

// n_iter <= S iterations in one launch (temporal tiling).  A block owns a TX x TY output
// tile and loads the state of the tile extended by S pixels on every side into LDS; each
// iteration runs phases A (u+) and B (q+, p+) on the whole region.  Values within s pixels
// of the region's border are wrong after s iterations (their neighbours outside the region
// are missing), but every dependency of the iteration reaches one pixel, so after n_iter
// <= S iterations the output tile is exact, and the arithmetic per pixel and iteration
// (the same expressions in the same order for every tile shape and S) does not depend on
// the tiling: the results equal one iteration per launch bit for bit.
// mask0: the branch-mask plane of the first iteration (nullptr: no tape), mask_stride the
// element distance between consecutive iterations' planes.
template <int TX, int TY, int S, class DataProx>
__device__ __forceinline__ void pdhg_fused_tile(const RefineState& in, const RefineState& out, const DataProx& prox,
                                                const float* __restrict__ w_h, const float* __restrict__ w_v, int W,
                                                int H, int K, const RefineScalars& sc, uint16_t* __restrict__ mask0,
                                                size_t mask_stride, int n_iter, int x0, int y0) {
    constexpr int RX = TX + 2 * S, RY = TY + 2 * S, NP = RX * RY;
    constexpr int NT = 256, PPT = (NP + NT - 1) / NT;
    __shared__ rfloat s_u[2][NP];
    __shared__ rfloat s_ph[NP], s_pv[NP], s_qh[NP], s_qv[NP];
    const int ox = x0 - S, oy = y0 - S;
    const rfloat kmax = (rfloat)(K - 1);
    // per-pixel constants of the launch stay in registers: the data model and the weights
    // (in their storage type, widened where used)
    typename DataProx::Px dm[PPT];
    float wh[PPT], wv[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        wh[k] = 0.0f;
        wv[k] = 0.0f;
        dm[k] = typename DataProx::Px{};
        if (idx >= NP) break;
        const int x = ox + idx % RX, y = oy + idx / RX;
        rfloat u = 0.0, ph = 0.0, pv = 0.0, qh = 0.0, qv = 0.0;
        if (x >= 0 && x < W && y >= 0 && y < H) {
            const long long p = (long long)y * W + x;
            u = in.u[p];
            ph = in.ph[p];
            pv = in.pv[p];
            qh = in.qh[p];
            qv = in.qv[p];
            dm[k] = prox.load(p);
            if (x + 1 < W) wh[k] = w_h[(long long)y * (W - 1) + x];
            if (y + 1 < H) wv[k] = w_v[p];
        }
        s_u[0][idx] = u;
        s_ph[idx] = ph;
        s_pv[idx] = pv;
        s_qh[idx] = qh;
        s_qv[idx] = qv;
    }
    __syncthreads();
    int cur = 0;
    for (int it = 0; it < n_iter; ++it) {
        int code[PPT];
        // Phase A: u+ on the region.
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            code[k] = 0;
            const int idx = (int)threadIdx.x + k * NT;
            if (idx >= NP) break;
            const int rx = idx % RX, ry = idx / RX;
            const int x = ox + rx, y = oy + ry;
            rfloat un = 0.0;
            if (x >= 0 && x < W && y >= 0 && y < H) {
                // (A^T z)_i = z_h(i) + z_v(i) - z_h(left) - z_v(up), z = p - q
                rfloat at = 0.0;
                if (x + 1 < W) at += s_ph[idx] - s_qh[idx];
                if (y + 1 < H) at += s_pv[idx] - s_qv[idx];
                if (x > 0) at -= rx > 0 ? s_ph[idx - 1] - s_qh[idx - 1] : 0.0;
                if (y > 0) at -= ry > 0 ? s_pv[idx - RX] - s_qv[idx - RX] : 0.0;
                un = prox.apply(s_u[cur][idx] - sc.tau * at, dm[k], kmax, code[k]);
            }
            s_u[cur ^ 1][idx] = un;
        }
        __syncthreads();
        // Phase B: q+ (old u) and p+ (extrapolated 2u+ - u) on the region's edges, in place.
        uint16_t* mask = mask0 != nullptr ? mask0 + (size_t)it * mask_stride : nullptr;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int idx = (int)threadIdx.x + k * NT;
            if (idx >= NP) break;
            const int rx = idx % RX, ry = idx / RX;
            const int x = ox + rx, y = oy + ry;
            if (x < 0 || x >= W || y < 0 || y >= H) continue;
            const rfloat uo = s_u[cur][idx], un = s_u[cur ^ 1][idx];
            uint32_t m = (uint32_t)code[k];
            int c;
            if (x + 1 < W) {
                const int r = rx + 1 < RX ? idx + 1 : idx;  // beyond the region: a value that is never used
                const rfloat gq = uo - s_u[cur][r];
                const rfloat w = (rfloat)wh[k];
                s_qh[idx] = prox_conj(s_qh[idx] + sc.tau * gq, w, 0.0, sc.beta_minus, sc.tau, c);
                m |= (uint32_t)c << 4;
                const rfloat gp = (2.0 * un - uo) - (2.0 * s_u[cur ^ 1][r] - s_u[cur][r]);
                s_ph[idx] = prox_conj(s_ph[idx] + sc.sigma * gp, w, sc.eps, sc.delta, sc.sigma, c);
                m |= (uint32_t)c << 10;
            }
            if (y + 1 < H) {
                const int d = ry + 1 < RY ? idx + RX : idx;
                const rfloat gq = uo - s_u[cur][d];
                const rfloat w = (rfloat)wv[k];
                s_qv[idx] = prox_conj(s_qv[idx] + sc.tau * gq, w, 0.0, sc.beta_minus, sc.tau, c);
                m |= (uint32_t)c << 7;
                const rfloat gp = (2.0 * un - uo) - (2.0 * s_u[cur ^ 1][d] - s_u[cur][d]);
                s_pv[idx] = prox_conj(s_pv[idx] + sc.sigma * gp, w, sc.eps, sc.delta, sc.sigma, c);
                m |= (uint32_t)c << 13;
            }
            const bool central = rx >= S && rx < S + TX && ry >= S && ry < S + TY;
            if (mask != nullptr && central) mask[(long long)y * W + x] = (uint16_t)m;
        }
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        if (idx >= NP) break;
        const int rx = idx % RX, ry = idx / RX;
        const int x = ox + rx, y = oy + ry;
        if (rx < S || rx >= S + TX || ry < S || ry >= S + TY || x >= W || y >= H) continue;
        const long long p = (long long)y * W + x;
        out.u[p] = s_u[cur][idx];
        out.ph[p] = s_ph[idx];
        out.pv[p] = s_pv[idx];
        out.qh[p] = s_qh[idx];
        out.qv[p] = s_qv[idx];
    }
}

// Fused tile shapes.  The stereo forward: 40 x 24 outputs, 4 iterations per launch, a
// 48 x 32 region (73.7 KB of LDS, 6 pixels per thread), so two blocks share a CU and the
// 512 blocks of a 1242 x 375 frame are all resident at once; 40 iterations per warp take
// 10 launches.  Its adjoint: 32 x 16 outputs, 4 reverse iterations per launch, a 40 x 24
// region (40.3 KB of LDS, 4 pixels per thread, 113 VGPRs), four blocks per CU and the 936
// blocks of a frame resident (with 6 pixels per thread the adjoint's accumulators exceed
// the register file).  The flow refinement (quadratic-fit model): 32 x 20 outputs, 3
// iterations per launch, a 38 x 26 region, three blocks per CU.
constexpr int kFTX = 40, kFTY = 24, kFS = 4;
constexpr int kATX = 32, kATY = 16, kAS = 4;
constexpr int kQTX = 32, kQTY = 20, kQS = 3;


}  // namespace dm
