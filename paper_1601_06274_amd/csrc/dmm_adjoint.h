// dmm_adjoint.h - reverse-mode adjoint of the Dual_MM chain passes on gfx950.
//
// The paper gives no derivative; this is the exact derivative of the piecewise-linear
// maps of Sec. 2.3 / App. A.1 / App. A.3.2 (iterative and naive minorants) as the
// forward computes them: minimisations route the adjoint to the selected candidate
// (lowest label on exact ties; in a message, window candidates in the order
// 0, -1, +1, -2, +2, ... before the truncation term on ties), normalisations subtract
// the summed adjoint at the argmin.
//
// One half-step of the forward is recomputed from its dual checkpoint by the record
// mode of chain_kernel, which keeps the messages of every pass (M[0] .. M[P]) and the
// dual after every update pass but the last (Lam[1] .. Lam[P-1]).  The adjoint kernel
// then walks, per chain, the passes in reverse order and each pass against its
// direction, carrying the adjoint of the in-register message and exchanging the
// adjoints of stored messages through two ping-pong volumes.  The adjoint of the dual
// (in units of the half-step's family unaries r) is updated in place in `lbar`.
//
// Message adjoint: the adjoint of phi(b) = v(src(b)) + w*dist(b) - vmin goes to
// v(src(b)) (window source or, for the truncation term, the argmin of v) and to w;
// the subtraction of vmin sends minus the total to argmin v.  Sources are found in
// LDS (the group's v), the gather back is a fixed-order sum (no atomics, bitwise
// deterministic).
#pragma once

#include "dmm_kernels.h"

namespace dm {

struct AdjArgs {
    const void* theta;        // horizontal family: cost [H][W][K]; nullptr for the vertical family
    const float* lam0;        // dual before the first update pass (the checkpoint)
    const float* rec_lam[8];  // dual after update pass s (s = 1 .. P-1)
    const float* rec_msg[9];  // messages of pass s (0: backward message pass)
    const float* w;           // edge weights of the family
    float* lbar;              // in: adjoint of the half-step output (dual); out: of its input
    float* bbar[2];           // adjoints of stored messages (ping-pong)
    float* grad_theta;        // horizontal family: dL/dcost accumulated (may be null)
    double* grad_w;           // dL/dw accumulated in FP64, indexed like w
    const float* grad_mm;     // final mode: dL/d(normalized row min-marginals), may be null
    double g_lb;              // final mode: dL/d(lower bound)
    long long chain_px, node_px, w_chain, w_node;
    unsigned vol_bytes_f32, vol_bytes_theta, w_bytes;
    int K, n, n_chains, T, mode, n_pass;
    float sign;               // +1 horizontal (lambda += h), -1 vertical
    float inv_n;
    float gamma[8];
};

template <int G>
__device__ __forceinline__ float group_sum(float x) {
    if constexpr (G >= 2) x += dpp<kQuadXor1>(x);
    if constexpr (G >= 4) x += dpp<kQuadXor2>(x);
    if constexpr (G >= 8) x += dpp<kRowHalfMirror>(x);
    if constexpr (G >= 16) x += dpp<kRowMirror>(x);
    if constexpr (G >= 32) {
        uint32_t a = __builtin_bit_cast(uint32_t, x);
        auto p = __builtin_amdgcn_permlane16_swap(a, opaque_copy(a), false, false);
        x = __builtin_bit_cast(float, (uint32_t)p[0]) + __builtin_bit_cast(float, (uint32_t)p[1]);
    }
    if constexpr (G >= 64) {
        uint32_t a = __builtin_bit_cast(uint32_t, x);
        auto p = __builtin_amdgcn_permlane32_swap(a, opaque_copy(a), false, false);
        x = __builtin_bit_cast(float, (uint32_t)p[0]) + __builtin_bit_cast(float, (uint32_t)p[1]);
    }
    return x;
}

// Adjoint pass kinds: update pass of the iterative minorant, naive update pass, final
// min-marginal pass, backward message pass (R0).
enum AdjKind : int { kAdjIter = 1, kAdjNaive = 2, kAdjFinal = 3, kAdjR0 = 0 };

template <int G, int LPL, int PF, typename TT, bool FULL, bool HAS_THETA>
struct AdjWalker {
    static constexpr int CPW = 64 / G;
    static constexpr int GK = G * LPL;

    struct Node {
        RawVec<TT, LPL, FULL> th;
        RawVec<float, LPL, FULL> lam, cmsg, rmsg, abar, bin;
        RawVec<float, LPL, FULL> gx;  // dL/dcost (first / R0 passes) or dL/dminmarg (final pass)
        float w;
    };

    __amdgpu_buffer_rsrc_t r_theta, r_w;
    __amdgpu_buffer_rsrc_t r_lam, r_cmsg, r_rmsg, r_abar, r_bin, r_bout, r_gth, r_gmm;
    float* __restrict__ lbar;
    float* __restrict__ grad_theta;
    double* __restrict__ grad_w;
    const float* __restrict__ grad_mm;
    long long base_px, wbase, node_px, w_node;
    int sub, grp, n, K, T;
    float sign, inv_n;
    unsigned vb;
    bool ok;
    bool lv[LPL];
    float* s_v;    // LDS: this group's v
    float* s_cb;   // LDS: this group's message adjoint
    int* s_src;    // LDS: source label of each message entry (-1: truncation term)

    __device__ AdjWalker(const AdjArgs& a, int chain, int sub_, int grp_, float* sv, float* scb, int* ssrc)
        : lbar(a.lbar), grad_theta(a.grad_theta), grad_w(a.grad_w), grad_mm(a.grad_mm), node_px(a.node_px),
          w_node(a.w_node), sub(sub_), grp(grp_), n(a.n), K(a.K), T(a.T), sign(a.sign), inv_n(a.inv_n),
          vb(a.vol_bytes_f32) {
        ok = chain < a.n_chains;
        base_px = (long long)(ok ? chain : 0) * a.chain_px;
        wbase = (long long)(ok ? chain : 0) * a.w_chain;
        r_theta = make_rsrc(a.theta, HAS_THETA ? a.vol_bytes_theta : 0u);
        r_w = make_rsrc(a.w, a.w_bytes);
        r_abar = make_rsrc(a.lbar, vb);
        r_gth = make_rsrc(a.grad_theta, a.grad_theta != nullptr ? vb : 0u);
        r_gmm = make_rsrc(a.grad_mm, a.grad_mm != nullptr ? vb : 0u);
#pragma unroll
        for (int i = 0; i < LPL; ++i) lv[i] = FULL ? true : (sub * LPL + i < K);
        s_v = sv + grp * GK;
        s_cb = scb + grp * GK;
        s_src = ssrc + grp * GK;
    }

    __device__ __forceinline__ long long elem(int j) const { return (base_px + (long long)j * node_px) * K + sub * LPL; }

    template <int ES>
    __device__ __forceinline__ void offsets(int j, bool valid, unsigned& off0, unsigned (&offs)[LPL]) const {
        const unsigned base = (unsigned)(elem(j) * ES);
        off0 = (valid && ok) ? base : kOOB;
#pragma unroll
        for (int i = 0; i < LPL; ++i) offs[i] = (valid && ok && lv[i]) ? base + (unsigned)(i * ES) : kOOB;
    }

    // FWD: the direction of the forward pass being differentiated (the adjoint walks the
    // other way).  The message produced at node j sits at slot j (FWD) or j-1; the carried
    // message used at j at slot j-1 (FWD) or j; the reverse message at slot j (FWD) or j-1.
    template <bool FWD, int KIND, bool IS_FIRST>
    __device__ __forceinline__ void load(Node& nd, int j, bool has_bin) const {
        unsigned o0, os[LPL];
        if constexpr (HAS_THETA) {
            offsets<(int)sizeof(TT)>(j, true, o0, os);
            nd.th.load(r_theta, o0, os);
        }
        offsets<4>(j, true, o0, os);
        nd.lam.load(r_lam, o0, os);
        nd.abar.load(r_abar, o0, os);
        if constexpr (KIND == kAdjFinal) nd.gx.load(r_gmm, o0, os);
        else if constexpr (HAS_THETA && (IS_FIRST || KIND == kAdjR0)) nd.gx.load(r_gth, o0, os);
        const bool out = FWD ? (j < n - 1) : (j > 0);  // a message leaves node j
        const int out_slot = FWD ? j : j - 1;
        const bool has_c = FWD ? (j > 0) : (j < n - 1);
        offsets<4>(FWD ? j - 1 : j, has_c, o0, os);
        nd.cmsg.load(r_cmsg, o0, os);
        if constexpr (KIND != kAdjR0) {
            const bool has_r = FWD ? (j < n - 1) : (j > 0);
            offsets<4>(FWD ? j : j - 1, has_r, o0, os);
            nd.rmsg.load(r_rmsg, o0, os);
        }
        offsets<4>(out_slot, out && has_bin, o0, os);
        nd.bin.load(r_bin, o0, os);
        const long long ei = wbase + (long long)out_slot * w_node;
        const unsigned wo = (out && ok) ? (unsigned)(ei * 4) : kOOB;
        nd.w = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r_w, (int)wo, 0, 0));
    }

    __device__ __forceinline__ float lane_min(const float (&x)[LPL]) const {
        float m = x[0];
#pragma unroll
        for (int i = 1; i < LPL; ++i) m = fminf(m, x[i]);
        return m;
    }

    // Lowest label attaining the group minimum `mn` of x.
    __device__ __forceinline__ int group_argmin(const float (&x)[LPL], float mn) const {
        int first = 0x7fffffff;
#pragma unroll
        for (int i = LPL - 1; i >= 0; --i)
            if (lv[i] && x[i] == mn) first = sub * LPL + i;
        return group_min_i<G>(first);
    }

    // Adjoint of out(b) = min(window, vmin + wT) - vmin given cb = d L / d out; returns
    // d L / d v in vbar and d L / d w.
    __device__ __forceinline__ float message_adjoint(const float (&v)[LPL], float wt, const float (&cb)[LPL],
                                                     float (&vbar)[LPL]) {
        const float vmin = group_min<G>(lane_min(v));
        const int astar = group_argmin(v, vmin);
#pragma unroll
        for (int i = 0; i < LPL; ++i) s_v[sub * LPL + i] = v[i];
        __syncthreads();
        const float cap = vmin + wt * (float)T;
        float wpart = 0.0f, tpart = 0.0f, apart = 0.0f;
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            const int b = sub * LPL + i;
            int src = -1;
            float dist = (float)T;
            if (lv[i]) {
                float best = v[i];
                int bd = 0;
                for (int t = 1; t < T && t < K; ++t) {
                    const int lo = b - t, hi = b + t;
                    if (lo >= 0) {
                        const float c = s_v[lo] + wt * (float)t;
                        if (c < best) { best = c; bd = -t; }
                    }
                    if (hi < K) {
                        const float c = s_v[hi] + wt * (float)t;
                        if (c < best) { best = c; bd = t; }
                    }
                }
                if (best <= cap) {
                    src = b + bd;
                    dist = (float)(bd < 0 ? -bd : bd);
                }
                wpart += cb[i] * dist;
                if (src < 0) tpart += cb[i];
                apart += cb[i];
            }
            s_cb[b] = lv[i] ? cb[i] : 0.0f;
            s_src[b] = src;
        }
        __syncthreads();
        const float wsum = group_sum<G>(wpart);
        const float tsum = group_sum<G>(tpart);
        const float asum = group_sum<G>(apart);
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            const int a = sub * LPL + i;
            float acc = 0.0f;
            if (lv[i]) {
                const int lo = a - (T - 1) > 0 ? a - (T - 1) : 0;
                const int hi = a + (T - 1) < K - 1 ? a + (T - 1) : K - 1;
                for (int b = lo; b <= hi; ++b)
                    if (s_src[b] == a) acc += s_cb[b];
                if (a == astar) acc += tsum - asum;
            }
            vbar[i] = acc;
        }
        __syncthreads();
        return wsum;
    }

    // One adjoint pass.  IS_FIRST: first adjoint pass of the half-step (reads the
    // half-step output adjoint from lbar, scales it to the family's unaries and, for the
    // horizontal family, adds it to dL/dcost).  IS_LAST: the R0 adjoint, which writes the
    // half-step input adjoint back to lbar (and adds to dL/dcost).
    template <bool FWD, int KIND, bool IS_FIRST>
    __device__ void pass(float gamma, bool has_bin) {
        float carry[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) carry[i] = 0.0f;
        int next_label = 0;  // final mode: label of the node visited before (LB pairwise term)
        Node ring[PF];
        // The adjoint walks against FWD: step t visits node FWD ? n-1-t : t.
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int t = q < n ? q : n - 1;
            load<FWD, KIND, IS_FIRST>(ring[q], FWD ? n - 1 - t : t, has_bin);
        }
        int t0 = 0;
        for (; t0 + PF <= n; t0 += PF) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int t = t0 + q;
                Node cur = ring[q];
                const int tn = (t + PF < n) ? t + PF : n - 1;
                load<FWD, KIND, IS_FIRST>(ring[q], FWD ? n - 1 - tn : tn, has_bin);
                step<FWD, KIND, IS_FIRST>(cur, FWD ? n - 1 - t : t, carry, gamma, next_label);
            }
        }
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int t = t0 + q;
            if (t < n) step<FWD, KIND, IS_FIRST>(ring[q], FWD ? n - 1 - t : t, carry, gamma, next_label);
        }
    }

    template <bool FWD, int KIND, bool IS_FIRST>
    __device__ __forceinline__ void step(const Node& nd, int j, float (&carry)[LPL], float gamma, int& next_label) {
        const bool out = FWD ? (j < n - 1) : (j > 0);
        const int out_slot = FWD ? j : j - 1;
        float r[LPL], ab[LPL], cbo[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            const float lam = nd.lam.get(i);
            const float x = HAS_THETA ? nd.th.get(i) - lam : lam;
            r[i] = lv[i] ? x : kBig;
            ab[i] = nd.abar.get(i);
            cbo[i] = out ? carry[i] + nd.bin.get(i) : 0.0f;
        }
        unsigned o0, os[LPL];
        offsets<4>(j, true, o0, os);
        if constexpr (IS_FIRST) {
            // lbar holds dL/d(dual after the half-step); the family's last-pass unaries r
            // relate to it by lambda = cost - r (horizontal) or lambda = r (vertical)
            if constexpr (HAS_THETA) {
                float g[LPL];
#pragma unroll
                for (int i = 0; i < LPL; ++i) g[i] = nd.gx.get(i) + ab[i];
                store_f32<LPL, FULL>(r_gth, o0, os, g);
            }
#pragma unroll
            for (int i = 0; i < LPL; ++i) ab[i] = (sign > 0.0f) ? -ab[i] : ab[i];
        }
        float v[LPL], vbar[LPL], rbar[LPL], cbar[LPL];
        if constexpr (KIND == kAdjR0) {
#pragma unroll
            for (int i = 0; i < LPL; ++i) v[i] = nd.cmsg.get(i) + r[i];
        } else {
            float m[LPL];
#pragma unroll
            for (int i = 0; i < LPL; ++i) m[i] = r[i] + nd.cmsg.get(i) + nd.rmsg.get(i);
            const float mmin = group_min<G>(lane_min(m));
            const int kstar = group_argmin(m, mmin);
            float madj[LPL];
            if constexpr (KIND == kAdjFinal) {
                // normalized min-marginal adjoint + lower-bound term at the row optimum
                float gs = 0.0f;
#pragma unroll
                for (int i = 0; i < LPL; ++i) gs += lv[i] ? nd.gx.get(i) : 0.0f;
                gs = group_sum<G>(gs);
#pragma unroll
                for (int i = 0; i < LPL; ++i) {
                    madj[i] = lv[i] ? nd.gx.get(i) : 0.0f;
                    if (sub * LPL + i == kstar) madj[i] -= gs;
                    v[i] = nd.cmsg.get(i) + r[i];
                }
            } else {
                // the message leaving node j is computed from r' = r - delta (iterative) or
                // from r (naive); madj is filled after the message adjoint
                const float g = KIND == kAdjIter ? gamma : inv_n;
#pragma unroll
                for (int i = 0; i < LPL; ++i) {
                    float dl = g * (m[i] - mmin);
                    dl = lv[i] ? dl : 0.0f;
                    v[i] = nd.cmsg.get(i) + (KIND == kAdjIter ? r[i] - dl : r[i]);
                }
            }
            float wsum = 0.0f;
            if (out) {
                wsum = message_adjoint(v, nd.w, cbo, vbar);
            } else {
#pragma unroll
                for (int i = 0; i < LPL; ++i) vbar[i] = 0.0f;
            }
            if constexpr (KIND == kAdjFinal) {
#pragma unroll
                for (int i = 0; i < LPL; ++i) {
                    rbar[i] = madj[i] + vbar[i];
                    cbar[i] = madj[i] + vbar[i];
                }
                // lower bound: d opt / d r_j = one-hot of the row optimum's label (kstar)
                if (g_lb_f != 0.0f) {
#pragma unroll
                    for (int i = 0; i < LPL; ++i)
                        if (sub * LPL + i == kstar) rbar[i] += g_lb_f;
                }
                if (out) {
                    int dd = kstar - next_label;
                    dd = dd < 0 ? -dd : dd;
                    wsum += g_lb_f * (float)(dd < T ? dd : T);
                }
                next_label = kstar;
            } else {
                const float g = KIND == kAdjIter ? gamma : inv_n;
                float rbp[LPL], s = 0.0f;
#pragma unroll
                for (int i = 0; i < LPL; ++i) {
                    rbp[i] = (KIND == kAdjIter) ? ab[i] + vbar[i] : ab[i];
                    s += lv[i] ? -rbp[i] : 0.0f;
                }
                s = group_sum<G>(s);
#pragma unroll
                for (int i = 0; i < LPL; ++i) {
                    float mb = lv[i] ? g * (-rbp[i]) : 0.0f;
                    if (sub * LPL + i == kstar) mb -= g * s;
                    madj[i] = mb;
                    rbar[i] = rbp[i] + (KIND == kAdjNaive ? vbar[i] : 0.0f) + mb;
                    cbar[i] = vbar[i] + mb;
                }
            }
            // adjoint of the reverse message read at node j, for the pass that wrote it
            const bool has_r = FWD ? (j < n - 1) : (j > 0);
            unsigned ro0, ros[LPL];
            offsets<4>(FWD ? j : j - 1, has_r, ro0, ros);
            store_f32<LPL, FULL>(r_bout, ro0, ros, madj);
            if (ok && sub == 0 && out && wsum != 0.0f) grad_w[wbase + (long long)out_slot * w_node] += (double)wsum;
#pragma unroll
            for (int i = 0; i < LPL; ++i) carry[i] = lv[i] ? cbar[i] : 0.0f;
            store_f32<LPL, FULL>(r_abar, o0, os, rbar);
            return;
        }
        // R0 adjoint
        float wsum = 0.0f;
        if (out) {
            wsum = message_adjoint(v, nd.w, cbo, vbar);
        } else {
#pragma unroll
            for (int i = 0; i < LPL; ++i) vbar[i] = 0.0f;
        }
        if (ok && sub == 0 && out && wsum != 0.0f) grad_w[wbase + (long long)out_slot * w_node] += (double)wsum;
        float rt[LPL], outv[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            rt[i] = ab[i] + vbar[i];
            carry[i] = lv[i] ? vbar[i] : 0.0f;
            outv[i] = sign > 0.0f ? -rt[i] : rt[i];  // dL/d(dual before the half-step)
        }
        if constexpr (HAS_THETA) {
            float g[LPL];
#pragma unroll
            for (int i = 0; i < LPL; ++i) g[i] = nd.gx.get(i) + rt[i];
            store_f32<LPL, FULL>(r_gth, o0, os, g);
        }
        store_f32<LPL, FULL>(r_abar, o0, os, outv);
    }

    float g_lb_f = 0.0f;
};

template <int G, int LPL, int PF, typename TT, bool FULL, bool HAS_THETA>
__global__ __launch_bounds__(64) void adjoint_kernel(AdjArgs a) {
    using AW = AdjWalker<G, LPL, PF, TT, FULL, HAS_THETA>;
    __shared__ float s_v[64 * LPL];
    __shared__ float s_cb[64 * LPL];
    __shared__ int s_src[64 * LPL];
    constexpr int CPW = 64 / G;
    const int lane = threadIdx.x;
    const int sub = lane % G;
    const int grp = lane / G;
    const int chain = blockIdx.x * CPW + grp;
    AW wk(a, chain, sub, grp, s_v, s_cb, s_src);
    const unsigned vb = a.vol_bytes_f32;
    if (a.mode == kModeFinal) {
        // final row pass: forward min-marginal pass (messages M[1], reverse M[0]), then R0
        wk.g_lb_f = (float)a.g_lb;
        wk.r_lam = make_rsrc(a.lam0, vb);
        wk.r_cmsg = make_rsrc(a.rec_msg[1], vb);
        wk.r_rmsg = make_rsrc(a.rec_msg[0], vb);
        wk.r_bin = make_rsrc(nullptr, 0u);
        wk.r_bout = make_rsrc(a.bbar[0], vb);
        wk.template pass<true, kAdjFinal, false>(0.0f, false);
        wk.r_cmsg = make_rsrc(a.rec_msg[0], vb);
        wk.r_bin = make_rsrc(a.bbar[0], vb);
        wk.r_bout = make_rsrc(nullptr, 0u);
        // the final pass's R0 adjoint turns dL/dr into dL/dcost and dL/d(dual) = -dL/dr
        wk.template pass<false, kAdjR0, false>(0.0f, true);
        return;
    }
    const int P = a.mode == kModeIterative ? a.n_pass : 1;
    for (int s = P; s >= 1; --s) {
        const float* lam_s = a.lam0;
        const float* msg_s = a.rec_msg[1];
        const float* msg_r = a.rec_msg[0];
        float g = a.gamma[0];
#pragma unroll
        for (int i = 1; i <= 8; ++i) {
            if (s == i) {
                if (i > 1) lam_s = a.rec_lam[i - 1 < 8 ? i - 1 : 7];
                msg_s = a.rec_msg[i];
                msg_r = a.rec_msg[i - 1];
                g = a.gamma[i - 1];
            }
        }
        wk.r_lam = make_rsrc(lam_s, vb);
        wk.r_cmsg = make_rsrc(msg_s, vb);
        wk.r_rmsg = make_rsrc(msg_r, vb);
        const bool has_bin = s < P;
        wk.r_bin = make_rsrc(a.bbar[s & 1], has_bin ? vb : 0u);
        wk.r_bout = make_rsrc(a.bbar[(s - 1) & 1], vb);
        const bool fwd = ((s - 1) & 1) == 0;
        if (a.mode == kModeNaive) {
            wk.template pass<true, kAdjNaive, true>(0.0f, false);
        } else if (s == P) {
            if (fwd) wk.template pass<true, kAdjIter, true>(g, has_bin);
            else wk.template pass<false, kAdjIter, true>(g, has_bin);
        } else {
            if (fwd) wk.template pass<true, kAdjIter, false>(g, has_bin);
            else wk.template pass<false, kAdjIter, false>(g, has_bin);
        }
    }
    wk.r_lam = make_rsrc(a.lam0, vb);
    wk.r_cmsg = make_rsrc(a.rec_msg[0], vb);
    wk.r_bin = make_rsrc(a.bbar[0], vb);
    wk.r_bout = make_rsrc(nullptr, 0u);
    wk.template pass<false, kAdjR0, false>(0.0f, true);
}

constexpr int kAdjPF = 4;

template <int G, int LPL, typename TT, bool HAS_THETA>
hipError_t launch_adjoint_tt(const AdjArgs& a, hipStream_t st) {
    constexpr int CPW = 64 / G;
    const unsigned blocks = (unsigned)((a.n_chains + CPW - 1) / CPW);
    if (a.K == G * LPL)
        hipLaunchKernelGGL((adjoint_kernel<G, LPL, kAdjPF, TT, true, HAS_THETA>), dim3(blocks), dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL((adjoint_kernel<G, LPL, kAdjPF, TT, false, HAS_THETA>), dim3(blocks), dim3(64), 0, st, a);
    return hipGetLastError();
}

template <int G, int LPL>
hipError_t launch_adjoint_tile(const AdjArgs& a, dm_dtype dt, hipStream_t st) {
    if (a.theta == nullptr) return launch_adjoint_tt<G, LPL, float, false>(a, st);
    if (dt == DM_F16) return launch_adjoint_tt<G, LPL, _Float16, true>(a, st);
    return launch_adjoint_tt<G, LPL, float, true>(a, st);
}

}  // namespace dm
