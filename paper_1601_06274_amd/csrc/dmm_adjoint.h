// dmm_adjoint.h - reverse-mode adjoint of the Dual_MM chain passes on gfx950.
//
// The paper gives no derivative; this is the exact derivative of the piecewise-linear
// maps of Sec. 2.3 / App. A.1 / App. A.3.2 (iterative and naive minorants) as the
// forward computes them: minimisations route the adjoint to the selected candidate
// (lowest label on exact ties; in a message, window candidates in the order
// 0, -1, +1, -2, +2, ... before the truncation term on ties), normalisations subtract
// the summed adjoint at the argmin.
//
// The adjoint kernel walks, per chain, the passes of a half-step in reverse order and
// each pass against its direction, carrying the adjoint of the in-register message and
// exchanging the adjoints of stored messages through two ping-pong volumes.  The
// adjoint of the dual (in units of the half-step's family unaries r) is updated in
// place in `lbar`.  Two forms:
//   * tape form (default): the record mode of chain_kernel (in the forward, or in a
//     recompute from the dual checkpoint) wrote per pass, node and label which
//     candidate each min took and the node's two argmins; the adjoint routes along
//     those selections and reads no forward values;
//   * recomputing form: the record mode kept every pass's messages (M[0] .. M[P]) and
//     the duals between passes (Lam[1] .. Lam[P-1]); the adjoint replays each node's
//     forward step with the same arithmetic and recomputes the selections (in-lane
//     scans, or a window search in LDS).
// Both give the same gradients bit for bit (up to the sign of zeros).
//
// Message adjoint: the adjoint of phi(b) = v(src(b)) + w*dist(b) - vmin goes to
// v(src(b)) (window source or, for the truncation term, the argmin of v) and to w;
// the subtraction of vmin sends minus the total to argmin v.  The gather back is a
// fixed-order sum (no atomics, bitwise deterministic).  The kernel's workgroup is one
// wave, so LDS exchanges need only the LDS wait, not a workgroup barrier.
#pragma once

#include "dmm_kernels.h"

namespace dm {

using lds_f32 = __attribute__((address_space(3))) float;
using lds_i32 = __attribute__((address_space(3))) int;
using gbl_f64 = __attribute__((address_space(1))) double;

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
    const double* g_lb;       // final mode: device dL/d(lower bound), nullptr = 0
    long long chain_px, node_px, w_chain, w_node;
    unsigned vol_bytes_f32, vol_bytes_theta, w_bytes;
    int K, n, n_chains, T, mode, n_pass;
    float sign;               // +1 horizontal (lambda += h), -1 vertical
    float inv_n;
    float gamma[8];
    const unsigned* tape[9];  // tape mode: selection tape of pass s (0: backward message pass)
    unsigned tape_bytes;      // bytes of one tape
    unsigned tape_px;         // tape bytes per pixel of this tile (byte accounting only)
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

// Two / three independent group sums (every lane of a group gets its group's sums).
// For G = 64 the cross-row steps carry two values in the operands of one permlane swap.
template <int G>
__device__ __forceinline__ void group_sum2(float& a, float& b) {
    if constexpr (G == 64) {
        a = group_sum<16>(a);
        b = group_sum<16>(b);
        auto p = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(uint32_t, a), __builtin_bit_cast(uint32_t, b), false,
                                                  false);
        // lanes 0-31: a over rows {0,2}, {1,3}; lanes 32-63: b likewise; then rows r <-> r^1
        const uint32_t ux = __builtin_bit_cast(uint32_t, __builtin_bit_cast(float, (uint32_t)p[0]) +
                                                             __builtin_bit_cast(float, (uint32_t)p[1]));
        auto h = __builtin_amdgcn_permlane16_swap(ux, opaque_copy(ux), false, false);
        const float c = __builtin_bit_cast(float, (uint32_t)h[0]) + __builtin_bit_cast(float, (uint32_t)h[1]);
        const uint32_t uc = __builtin_bit_cast(uint32_t, c);
        auto q = __builtin_amdgcn_permlane32_swap(uc, opaque_copy(uc), false, false);
        a = __builtin_bit_cast(float, (uint32_t)q[0]);
        b = __builtin_bit_cast(float, (uint32_t)q[1]);
    } else {
        a = group_sum<G>(a);
        b = group_sum<G>(b);
    }
}

// Lowest label of the group whose value equals the group minimum mn (attained by some
// existing label).  A whole-wave group uses a ballot instead of an integer reduction.
template <int G, int LPL, bool FULL>
__device__ __forceinline__ int group_argmin_eq(const float (&x)[LPL], float mn, const bool (&lv)[LPL], int sub) {
    if constexpr (G == 64) {
        int first = LPL;
#pragma unroll
        for (int i = LPL - 1; i >= 0; --i)
            if ((FULL || lv[i]) && x[i] == mn) first = i;
        const unsigned long long mask = __builtin_amdgcn_ballot_w64(first < LPL);
        const int lane = (int)__builtin_ctzll(mask);
        return lane * LPL + __builtin_amdgcn_readlane(first, lane);
    } else {
        int first = 0x7fffffff;
#pragma unroll
        for (int i = LPL - 1; i >= 0; --i)
            if ((FULL || lv[i]) && x[i] == mn) first = sub * LPL + i;
        return group_min_i<G>(first);
    }
}

// Adjoint pass kinds: update pass of the iterative minorant, naive update pass, final
// min-marginal pass, backward message pass (R0).
enum AdjKind : int { kAdjIter = 1, kAdjNaive = 2, kAdjFinal = 3, kAdjR0 = 0 };
enum OutMode : int { kOutRuntime = 0, kOutYes = 1, kOutNo = 2 };

template <int G, int LPL, int PF, typename TT, bool FULL, bool HAS_THETA>
struct AdjWalker {
    static constexpr int ES = (int)sizeof(TT);
    static constexpr int GK = G * LPL;
    static constexpr int kFar = 1 << 20;  // distance of a missing neighbour's candidate

    struct Node {
        RawVec<TT, LPL, FULL> th;
        RawVec<float, LPL, FULL> lam, cmsg, rmsg, abar, bin;
        RawVec<float, LPL, FULL> gx;  // dL/dcost (first / R0 passes) or dL/dminmarg (final pass)
        float w;
        uint32_t tw[kTapeWords(LPL)];  // tape mode: the node's selection bytes
    };
    struct Cursor {
        unsigned th, f, w, tp;
    };
    static constexpr int kTW = kTapeWords(LPL);

    __amdgpu_buffer_rsrc_t r_theta, r_w;
    __amdgpu_buffer_rsrc_t r_lam, r_cmsg, r_rmsg, r_abar, r_bin, r_bout, r_gth, r_gmm;
    __amdgpu_buffer_rsrc_t r_tape;  // tape mode: the current pass's tape
    unsigned tp0, tp_step;
    gbl_f64* grad_w;
    // Offsets as in the forward walker: node 0 of this lane's chain and label, edge (0, 1),
    // per-node steps; missing chains sit at kOOB with step 0.
    unsigned th0, f0, w0, th_step, f_step, w_step;
    int sub, grp, n, K, T;
    float sign, inv_n, Tf;
    bool ok;
    bool lv[LPL];
    int dt_steps;
    bool direct;  // the forward used the direct window form (T <= 3)
    float g_lb_f = 0.0f;
    // LDS (typed in the local address space: a generic pointer would make every access a
    // flat instruction, which waits on the vector-memory counter too)
    lds_f32* s_v;    // this group's v
    lds_f32* s_cb;   // this group's message adjoint
    lds_i32* s_src;  // source label of each message entry (-1: truncation term)

    __device__ __forceinline__ AdjWalker(const AdjArgs& a, int chain, int sub_, int grp_, float* sv, float* scb, int* ssrc)
        : grad_w((gbl_f64*)a.grad_w), sub(sub_), grp(grp_), n(a.n), K(a.K), T(a.T), sign(a.sign), inv_n(a.inv_n) {
        ok = chain < a.n_chains;
        Tf = (float)a.T;
        const unsigned long long cpx = (unsigned long long)(ok ? chain : 0) * (unsigned long long)a.chain_px;
        const unsigned long long e0 = cpx * (unsigned long long)a.K + (unsigned long long)(sub * LPL);
        const unsigned long long nk = (unsigned long long)a.node_px * (unsigned long long)a.K;
        f0 = ok ? (unsigned)(e0 * 4ull) : kOOB;
        th0 = ok ? (unsigned)(e0 * (unsigned long long)ES) : kOOB;
        f_step = ok ? (unsigned)(nk * 4ull) : 0u;
        th_step = ok ? (unsigned)(nk * (unsigned long long)ES) : 0u;
        w0 = ok ? (unsigned)((unsigned long long)chain * (unsigned long long)a.w_chain * 4ull) : kOOB;
        w_step = ok ? (unsigned)(a.w_node * 4) : 0u;
        const unsigned vb = a.vol_bytes_f32;
        r_theta = make_rsrc(a.theta, HAS_THETA ? a.vol_bytes_theta : 0u);
        r_w = make_rsrc(a.w, a.w_bytes);
        r_abar = make_rsrc(a.lbar, vb);
        r_gth = make_rsrc(a.grad_theta, a.grad_theta != nullptr ? vb : 0u);
        r_gmm = make_rsrc(a.grad_mm, a.grad_mm != nullptr ? vb : 0u);
#pragma unroll
        for (int i = 0; i < LPL; ++i) lv[i] = FULL ? true : (ok && sub * LPL + i < K);
        const int need = (a.T - 1 + LPL - 1) / LPL;
        dt_steps = need < G - 1 ? need : G - 1;
        direct = a.T <= 3 && a.T - 1 <= LPL;
        const unsigned long long ts = (unsigned long long)(G * kTW * 4);
        tp0 = ok ? (unsigned)(cpx * ts + (unsigned long long)(sub * kTW * 4)) : kOOB;
        tp_step = ok ? (unsigned)((unsigned long long)a.node_px * ts) : 0u;
        r_tape = make_rsrc(nullptr, 0u);
        s_v = (lds_f32*)sv + grp * GK;
        s_cb = (lds_f32*)scb + grp * GK;
        s_src = (lds_i32*)ssrc + grp * GK;
    }

    // dL/dw of an edge += x (lane 0 of the group).  A returning read-modify-write would
    // make the node wait for all loads in flight (the wait counter is in order); a
    // no-return atomic does not.  Each edge belongs to one chain, so its updates come
    // from one wave in program order (and from launches in stream order): the summation
    // order is fixed and the result deterministic.
    __device__ __forceinline__ void add_edge_grad(unsigned w_off, float x) const {
        __hip_atomic_fetch_add(grad_w + (w_off >> 2), (double)x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }

    template <int E>
    __device__ __forceinline__ void label_offsets(unsigned off, unsigned (&o)[LPL]) const {
#pragma unroll
        for (int i = 0; i < LPL; ++i) o[i] = (FULL || lv[i]) ? off + (unsigned)(i * E) : kOOB;
    }

    // Cursor at the first node the adjoint visits (the forward pass's last node).
    __device__ __forceinline__ Cursor cursor_start(bool fwd) const {
        const unsigned j = fwd ? (unsigned)(n - 1) : 0u;
        const unsigned e = fwd ? (unsigned)(n - 1) : 0xFFFFFFFFu;  // edge leaving node j in the pass
        return Cursor{th0 + j * th_step, f0 + j * f_step, w0 + e * w_step, tp0 + j * tp_step};
    }
    template <bool FWD>
    __device__ __forceinline__ void advance(Cursor& c) const {
        // the adjoint walks against the forward pass
        if constexpr (FWD) {
            c.th -= th_step; c.f -= f_step; c.w -= w_step; c.tp -= tp_step;
        } else {
            c.th += th_step; c.f += f_step; c.w += w_step; c.tp += tp_step;
        }
    }

    // Node j of a forward pass in direction FWD: the message leaving j and the reverse
    // message read at j sit in slot j (FWD) or j-1, the carried message arriving at j in
    // slot j-1 (FWD) or j.  Issue order: what the step uses last first.
    template <bool FWD, int KIND, bool IS_FIRST>
    __device__ __forceinline__ void load(Node& nd, Cursor& c) const {
        unsigned os[LPL];
        const unsigned rs = FWD ? c.f : c.f - f_step;
        const unsigned cs = FWD ? c.f - f_step : c.f;
        nd.w = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r_w, (int)c.w, 0, 0));
        label_offsets<4>(rs, os);
        nd.bin.load(r_bin, rs, os);
        if constexpr (KIND != kAdjR0) nd.rmsg.load(r_rmsg, rs, os);
        label_offsets<4>(c.f, os);
        if constexpr (KIND == kAdjFinal) nd.gx.load(r_gmm, c.f, os);
        else if constexpr (HAS_THETA && (IS_FIRST || KIND == kAdjR0)) nd.gx.load(r_gth, c.f, os);
        if constexpr (KIND != kAdjFinal) nd.abar.load(r_abar, c.f, os);
        nd.lam.load(r_lam, c.f, os);
        label_offsets<4>(cs, os);
        nd.cmsg.load(r_cmsg, cs, os);
        if constexpr (HAS_THETA) {
            label_offsets<ES>(c.th, os);
            nd.th.load(r_theta, c.th, os);
        }
        advance<FWD>(c);
    }

    __device__ __forceinline__ float lane_min(const float (&x)[LPL]) const {
        float m = x[0];
#pragma unroll
        for (int i = 1; i < LPL; ++i) m = fminf(m, x[i]);
        return m;
    }

    // Neighbour-lane moves inside the group: value of lane sub-1 / sub+1, `fill` at the
    // group's first / last lane.
    template <typename V>
    __device__ __forceinline__ V from_left(V x, V fill) const {
        const int r = __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, fill), __builtin_bit_cast(int, x), kWaveShr1,
                                                  0xF, 0xF, false);
        const V y = __builtin_bit_cast(V, r);
        return (G < 64 && sub == 0) ? fill : y;
    }
    template <typename V>
    __device__ __forceinline__ V from_right(V x, V fill) const {
        const int r = __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, fill), __builtin_bit_cast(int, x), kWaveShl1,
                                                  0xF, 0xF, false);
        const V y = __builtin_bit_cast(V, r);
        return (G < 64 && sub == G - 1) ? fill : y;
    }

    // Adjoint of the truncated-linear message out = min(DT(v), vmin + wT) - vmin for the
    // output adjoint cb: the part that reaches v through the selected sources (vbar), and
    // per-lane partial sums of dL/dw (wl) and of dL/dvmin (zl: truncated entries minus all
    // entries; the caller routes the group total to the minimiser).
    //
    // DTM 0 / 1 (the distance transform reaches 0 / 1 lanes across): the forward's scans
    // are replayed with the same arithmetic, recording which operand each min took and
    // the distance of its source, and the adjoint runs the scans in reverse.  Ties go to
    // the closer source, then to the lower label; a source at distance >= T, or above
    // the truncation level, gives the truncation term.  DTM 2 (longer reach): sources are
    // searched in LDS over the window (candidates 0, -1, +1, -2, +2, ... in that order).
    template <int DTM>
    __device__ __forceinline__ void msg_adjoint(const float (&v)[LPL], float vmin, float wt, const float (&cb)[LPL],
                                                float (&vbar)[LPL], float& wl, float& zl) {
        const float cap = __builtin_fmaf(wt, Tf, vmin);
        if constexpr (DTM == 2) {
#pragma unroll
            for (int i = 0; i < LPL; ++i) s_v[sub * LPL + i] = v[i];
            wave_lds_sync();
            float wpart = 0.0f, cpart = 0.0f, apart = 0.0f;
#pragma unroll
            for (int i = 0; i < LPL; ++i) {
                const int b = sub * LPL + i;
                int src = -1;
                float dist = Tf;
                if (FULL || lv[i]) {
                    float best = v[i];
                    int bd = 0;
                    for (int t = 1; t < T && t < K; ++t) {
                        const int lo = b - t, hi = b + t;
                        if (lo >= 0) {
                            const float c = wdist(wt, t, s_v[lo]);
                            if (c < best) { best = c; bd = -t; }
                        }
                        if (hi < K) {
                            const float c = wdist(wt, t, s_v[hi]);
                            if (c < best) { best = c; bd = t; }
                        }
                    }
                    if (best <= cap) {
                        src = b + bd;
                        dist = (float)(bd < 0 ? -bd : bd);
                    }
                    wpart = __builtin_fmaf(cb[i], dist, wpart);
                    if (src < 0) cpart += cb[i];
                    apart += cb[i];
                }
                s_cb[b] = (FULL || lv[i]) ? cb[i] : 0.0f;
                s_src[b] = src;
            }
            wave_lds_sync();
#pragma unroll
            for (int i = 0; i < LPL; ++i) {
                const int a = sub * LPL + i;
                float acc = 0.0f;
                if (FULL || lv[i]) {
                    const int lo = a - (T - 1) > 0 ? a - (T - 1) : 0;
                    const int hi = a + (T - 1) < K - 1 ? a + (T - 1) : K - 1;
                    for (int b = lo; b <= hi; ++b)
                        if (s_src[b] == a) acc += s_cb[b];
                }
                vbar[i] = acc;
            }
            wave_lds_sync();
            wl = wpart;
            zl = cpart - apart;
        } else {
            // forward in-lane scans (values as the forward computes them) with choices
            float f[LPL], b[LPL];
            int df[LPL], db[LPL];
            bool fi[LPL], bi[LPL];  // took the neighbour (inherit) rather than v itself
            f[0] = v[0];
            df[0] = 0;
            fi[0] = false;
#pragma unroll
            for (int i = 1; i < LPL; ++i) {
                const float c = f[i - 1] + wt;
                fi[i] = c < v[i];
                f[i] = fi[i] ? c : v[i];
                df[i] = fi[i] ? df[i - 1] + 1 : 0;
            }
            b[LPL - 1] = v[LPL - 1];
            db[LPL - 1] = 0;
            bi[LPL - 1] = false;
#pragma unroll
            for (int i = LPL - 2; i >= 0; --i) {
                const float c = b[i + 1] + wt;
                bi[i] = c < v[i];
                b[i] = bi[i] ? c : v[i];
                db[i] = bi[i] ? db[i + 1] + 1 : 0;
            }
            float cl = kBig, cr = kBig;
            int dcl = kFar, dcr = kFar;
            if constexpr (DTM == 1) {
                cl = from_left(f[LPL - 1], kBig);
                cr = from_right(b[0], kBig);
                dcl = from_left(df[LPL - 1], kFar);
                dcr = from_right(db[0], kFar);
            }
            float fb[LPL], bb[LPL];
            float CL = 0.0f, CR = 0.0f, wpart = 0.0f, cpart = 0.0f, apart = 0.0f;
#pragma unroll
            for (int i = 0; i < LPL; ++i) {
                // left side: in-lane forward chain, or (DTM 1) the left lane's chain end
                float lvv = f[i];
                int ld = df[i];
                bool useF = true;
                if constexpr (DTM == 1) {
                    const float vl = wdist(wt, i + 1, cl);
                    useF = f[i] <= vl;
                    lvv = useF ? f[i] : vl;
                    ld = useF ? df[i] : dcl + i + 1;
                }
                float rvv = b[i];
                int rd = db[i];
                bool useB = true;
                if constexpr (DTM == 1) {
                    const float vr = wdist(wt, LPL - i, cr);
                    useB = b[i] <= vr;
                    rvv = useB ? b[i] : vr;
                    rd = useB ? db[i] : dcr + LPL - i;
                }
                const bool left = (lvv < rvv) | ((lvv == rvv) & (ld <= rd));
                const float wv = left ? lvv : rvv;
                const int wd = left ? ld : rd;
                const bool win = (wv <= cap) & (wd < T);
                const float c = (FULL || lv[i]) ? cb[i] : 0.0f;
                fb[i] = (win & left & useF) ? c : 0.0f;
                bb[i] = (win & !left & useB) ? c : 0.0f;
                if constexpr (DTM == 1) {
                    const float cL = (win & left & !useF) ? c : 0.0f;
                    const float cR = (win & !left & !useB) ? c : 0.0f;
                    CL += cL;
                    CR += cR;
                    wpart += __builtin_fmaf(cL, (float)(i + 1), cR * (float)(LPL - i));
                }
                cpart += win ? 0.0f : c;
                apart += c;
            }
            if constexpr (DTM == 1) {
                // the left lane's chain end fed this lane's left candidates, and vice versa
                fb[LPL - 1] += from_right(CL, 0.0f);
                bb[0] += from_left(CR, 0.0f);
            }
            // reverse scans
#pragma unroll
            for (int i = 0; i < LPL; ++i) vbar[i] = 0.0f;
#pragma unroll
            for (int i = LPL - 1; i >= 1; --i) {
                if (fi[i]) {
                    fb[i - 1] += fb[i];
                    wpart += fb[i];
                } else {
                    vbar[i] += fb[i];
                }
            }
            vbar[0] += fb[0];
#pragma unroll
            for (int i = 0; i < LPL - 1; ++i) {
                if (bi[i]) {
                    bb[i + 1] += bb[i];
                    wpart += bb[i];
                } else {
                    vbar[i] += bb[i];
                }
            }
            vbar[LPL - 1] += bb[LPL - 1];
            wl = __builtin_fmaf(Tf, cpart, wpart);
            zl = cpart - apart;
        }
    }

    // ---------------------------------------------------------------- tape mode
    // The forward's record sweep stored, per pass, node and label, which operand each
    // min of the message took and the node's two argmins (TapeBit).  The adjoint then
    // routes adjoints along those selections without the forward's values: it reads
    // the tape, the stored-message adjoint and the dual adjoint only.

    // Tape-mode loads (issue order: what the step uses last first).
    template <bool FWD, int KIND, bool IS_FIRST>
    __device__ __forceinline__ void load_tape(Node& nd, Cursor& c) const {
        unsigned os[LPL];
        const unsigned rs = FWD ? c.f : c.f - f_step;
        label_offsets<4>(rs, os);
        nd.bin.load(r_bin, rs, os);
        label_offsets<4>(c.f, os);
        if constexpr (KIND == kAdjFinal) nd.gx.load(r_gmm, c.f, os);
        else if constexpr (HAS_THETA && (IS_FIRST || KIND == kAdjR0)) nd.gx.load(r_gth, c.f, os);
        if constexpr (KIND != kAdjFinal) nd.abar.load(r_abar, c.f, os);
        load_words<kTW>(r_tape, c.tp, nd.tw);
        advance<FWD>(c);
    }

    // Tape bit BIT of label i (as a 32-bit word position).
    static constexpr int tape_pos(int i, unsigned bit) { return 8 * (i & 3) + __builtin_ctz(bit); }
    // c where the tape bit is set, else +0: the bit sign-extended into a mask (no compare).
    template <unsigned BIT>
    __device__ __forceinline__ float sel(const Node& nd, int i, float c) const {
        const int m = __builtin_amdgcn_sbfe((int)nd.tw[i >> 2], tape_pos(i, BIT), 1);
        return __builtin_bit_cast(float, __builtin_bit_cast(int, c) & m);
    }
    __device__ __forceinline__ bool has(const Node& nd, int i, unsigned bit) const {
        return ((nd.tw[i >> 2] >> (8 * (i & 3))) & bit) != 0u;
    }

    // msg_adjoint<DTM> (DTM 0 / 1) with the selections read from the tape: the same
    // routing and the same order of additions as the recomputing form, so the results
    // agree with it bit for bit (up to the sign of zeros: an unselected term adds +0).
    template <bool DT1>
    __device__ __forceinline__ void msg_adjoint_tape(const Node& nd, const float (&cb)[LPL], float (&vbar)[LPL],
                                                     float& wl, float& zl) {
        float fb[LPL], bb[LPL];
        float CL = 0.0f, CR = 0.0f, wpart = 0.0f, cpart = 0.0f, apart = 0.0f;
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            const float c = (FULL || lv[i]) ? cb[i] : 0.0f;
            fb[i] = sel<kTapeF>(nd, i, c);
            bb[i] = sel<kTapeB>(nd, i, c);
            if constexpr (DT1) {
                const float cL = sel<kTapeCL>(nd, i, c);
                const float cR = sel<kTapeCR>(nd, i, c);
                CL += cL;
                CR += cR;
                wpart += __builtin_fmaf(cL, (float)(i + 1), cR * (float)(LPL - i));
            }
            cpart += has(nd, i, kTapeF | kTapeB | kTapeCL | kTapeCR) ? 0.0f : c;
            apart += c;
        }
        if constexpr (DT1) {
            fb[LPL - 1] += from_right(CL, 0.0f);
            bb[0] += from_left(CR, 0.0f);
        }
#pragma unroll
        for (int i = 0; i < LPL; ++i) vbar[i] = 0.0f;
#pragma unroll
        for (int i = LPL - 1; i >= 1; --i) {
            const float t = sel<kTapeFI>(nd, i, fb[i]);  // passed on to the left neighbour
            fb[i - 1] += t;
            wpart += t;
            vbar[i] += fb[i] - t;
        }
        vbar[0] += fb[0];
#pragma unroll
        for (int i = 0; i < LPL - 1; ++i) {
            const float t = sel<kTapeBI>(nd, i, bb[i]);
            bb[i + 1] += t;
            wpart += t;
            vbar[i] += bb[i] - t;
        }
        vbar[LPL - 1] += bb[LPL - 1];
        wl = __builtin_fmaf(Tf, cpart, wpart);
        zl = cpart - apart;
    }

    // Message adjoint from a direct window tape (codes 0-5, distance in bits 3-4): the
    // routing, the order of additions and the edge and minimum terms of the window search
    // of msg_adjoint<2>, so the two agree bit for bit (up to the sign of zeros).  Each
    // source label sums, in ascending target order, what the left lane sends (its
    // targets before this lane), its own targets, then the right lane's targets one by
    // one.
    __device__ __forceinline__ void msg_adjoint_direct(const Node& nd, const float (&cb)[LPL], float (&vbar)[LPL],
                                                       float& wl, float& zl) {
        float t[5][LPL];  // t[k][i]: the adjoint of target i if its message took class k
        float wpart = 0.0f, cpart = 0.0f, apart = 0.0f;
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            const unsigned x = nd.tw[i >> 2] >> (8 * (i & 3));
            const unsigned code = x & 7u;
            const float c = (FULL || lv[i]) ? cb[i] : 0.0f;
#pragma unroll
            for (int k = 0; k < 5; ++k) t[k][i] = code == (unsigned)k ? c : 0.0f;
            const float dist = (float)((x >> 3) & 3u);
            const float cc = code == 5u ? c : 0.0f;
            // sums start from their first term (equal to 0 + term up to the sign of zero)
            wpart = i == 0 ? c * dist : __builtin_fmaf(c, dist, wpart);
            cpart = i == 0 ? cc : cpart + cc;
            apart = i == 0 ? c : apart + c;
        }
        // class of a target at offset d from its source: +2 -> 4, +1 -> 2, 0 -> 0, -1 -> 1, -2 -> 3
        constexpr int cls[5] = {3, 1, 0, 2, 4};  // indexed by d + 2, d = source - target
        float toR0, toR1 = 0.0f;
        if constexpr (LPL >= 2) {
            toR0 = t[4][LPL - 2] + t[2][LPL - 1];
            toR1 = t[4][LPL - 1];
        } else {
            toR0 = t[2][0];
        }
        const float fL0 = from_left(toR0, 0.0f);
        const float fL1 = LPL >= 2 ? from_left(toR1, 0.0f) : 0.0f;
        const float rA = from_right(t[1][0], 0.0f);
        const float rB = LPL >= 2 ? from_right(t[3][1], 0.0f) : 0.0f;
        const float rC = LPL >= 2 ? from_right(t[3][0], 0.0f) : 0.0f;
#pragma unroll
        for (int j = 0; j < LPL; ++j) {
            const int b0 = j - 2 > 0 ? j - 2 : 0;
            float acc = j == 0 ? fL0 + t[cls[j - b0 + 2]][b0]
                               : (j == 1 ? fL1 + t[cls[j - b0 + 2]][b0] : t[cls[j - b0 + 2]][b0]);
#pragma unroll
            for (int b = b0 + 1; b <= (j + 2 < LPL - 1 ? j + 2 : LPL - 1); ++b)
                acc += t[cls[j - b + 2]][b];
            if (j == LPL - 1) {
                acc += rA;
                if constexpr (LPL >= 2) acc += rB;
            } else if (j == LPL - 2) {
                acc += rC;
            }
            vbar[j] = acc;
        }
        wl = wpart;
        zl = cpart - apart;
    }

    // MF: the forward's message form - 1 scans reaching one lane, 2 direct window.
    template <bool FWD, int KIND, bool IS_FIRST, int MF>
    __device__ __forceinline__ void pass_tape(float gamma) {
        float cbar[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) cbar[i] = 0.0f;
        int next_label = 0;
        float unused_w = 0.0f;  // nodes outside the steady blocks add their edge sums one by one
        Cursor lc = cursor_start(FWD);
        Cursor sc = lc;
        Node ring[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            load_tape<FWD, KIND, IS_FIRST>(ring[q], lc);
            __builtin_amdgcn_sched_barrier(0);
        }
        int t0 = 0;
        if (n >= PF) {
            // first block: the first visited node (the forward pass's last) sends no
            // message; the steady loop's nodes all do
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                if (q == 0)
                    step_tape<FWD, KIND, IS_FIRST, MF, kOutNo>(ring[q], q, cbar, gamma, next_label, sc, unused_w);
                else
                    step_tape<FWD, KIND, IS_FIRST, MF, kOutYes>(ring[q], q, cbar, gamma, next_label, sc, unused_w);
                load_tape<FWD, KIND, IS_FIRST>(ring[q], lc);
            }
            // steady blocks: node q's edge sum goes to lane q, and the block's PF edges get
            // one atomic (lanes 0..PF-1) instead of one lane-0 atomic per node
            constexpr bool kBatchW = G >= PF;
            for (t0 = PF; t0 + PF <= n; t0 += PF) {
                float wacc = 0.0f;
                const unsigned w_blk = sc.w;
#pragma unroll
                for (int q = 0; q < PF; ++q) {
                    step_tape<FWD, KIND, IS_FIRST, MF, kOutYes, kBatchW>(ring[q], t0 + q, cbar, gamma, next_label, sc,
                                                                         wacc, q);
                    load_tape<FWD, KIND, IS_FIRST>(ring[q], lc);
                }
                if constexpr (kBatchW)
                    if (ok && sub < PF)
                        add_edge_grad(FWD ? w_blk - (unsigned)sub * w_step : w_blk + (unsigned)sub * w_step, wacc);
            }
        }
#pragma unroll
        for (int q = 0; q < PF; ++q)
            if (t0 + q < n)
                step_tape<FWD, KIND, IS_FIRST, MF, kOutRuntime>(ring[q], t0 + q, cbar, gamma, next_label, sc,
                                                                unused_w);
    }

    template <bool FWD, int KIND, bool IS_FIRST>
    __device__ __forceinline__ void run_pass_tape(float gamma) {
        if (direct)
            pass_tape<FWD, KIND, IS_FIRST, 2>(gamma);
        else
            pass_tape<FWD, KIND, IS_FIRST, 1>(gamma);
    }

    // Adjoint of the forward step at the node visited t-th, from the tape (the same
    // formulas as step()).
    // OUTM: whether the node sends a message in the forward pass (kOutYes / kOutNo), or
    // decided at run time (t != 0).  BATCH: the node's edge sum goes to lane wb of wacc
    // (the caller adds a block of edges at once); else lane 0 adds it now.
    template <bool FWD, int KIND, bool IS_FIRST, int MF, int OUTM, bool BATCH = false>
    __device__ __forceinline__ void step_tape(const Node& nd, int t, float (&cbar)[LPL], float gamma, int& next_label,
                                              Cursor& sc, float& wacc, int wb = 0) {
        const bool out = OUTM == kOutYes ? true : (OUTM == kOutNo ? false : t != 0);
        const unsigned rs = FWD ? sc.f : sc.f - f_step;
        unsigned os[LPL];
        float ab[LPL], cb[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            ab[i] = KIND == kAdjFinal ? 0.0f : nd.abar.get(i);
            cb[i] = out ? cbar[i] + nd.bin.get(i) : 0.0f;
        }
        if constexpr (IS_FIRST) {
            if constexpr (HAS_THETA) {
                float g[LPL];
#pragma unroll
                for (int i = 0; i < LPL; ++i) g[i] = nd.gx.get(i) + ab[i];
                label_offsets<4>(sc.f, os);
                store_f32<LPL, FULL>(r_gth, sc.f, os, g);
            }
#pragma unroll
            for (int i = 0; i < LPL; ++i) ab[i] = (sign > 0.0f) ? -ab[i] : ab[i];
        }
        // the last node of a forward pass sends no message: its selection bits are 0 and
        // its message adjoint cb is 0, so the message adjoint below adds nothing there
        float vbar[LPL], wl = 0.0f, zl = 0.0f;
        if constexpr (MF == 2)
            msg_adjoint_direct(nd, cb, vbar, wl, zl);
        else
            msg_adjoint_tape<true>(nd, cb, vbar, wl, zl);
        if constexpr (KIND == kAdjR0) {
            group_sum2<G>(wl, zl);
            float rt[LPL], outv[LPL];
#pragma unroll
            for (int i = 0; i < LPL; ++i) {
                vbar[i] += sel<kTapeA>(nd, i, zl);
                rt[i] = ab[i] + vbar[i];
                cbar[i] = (FULL || lv[i]) ? vbar[i] : 0.0f;
                outv[i] = sign > 0.0f ? -rt[i] : rt[i];
            }
            label_offsets<4>(sc.f, os);
            if constexpr (HAS_THETA) {
                float g[LPL];
#pragma unroll
                for (int i = 0; i < LPL; ++i) g[i] = nd.gx.get(i) + rt[i];
                store_f32<LPL, FULL>(r_gth, sc.f, os, g);
            }
            store_f32<LPL, FULL>(r_abar, sc.f, os, outv);
        } else {
            float al = 0.0f;
#pragma unroll
            for (int i = 0; i < LPL; ++i)
                al += (FULL || lv[i]) ? (KIND == kAdjFinal ? nd.gx.get(i) : ab[i]) : 0.0f;
            group_sum2<G>(wl, zl);
            al = group_sum<G>(al);
            float rbar[LPL], revb[LPL];
            if constexpr (KIND == kAdjIter) {
                const float mminb = gamma * al;
#pragma unroll
                for (int i = 0; i < LPL; ++i) {
                    const bool valid = FULL || lv[i];
                    const float ub = sel<kTapeA>(nd, i, zl);
                    const float dbar = valid ? -vbar[i] - ab[i] : 0.0f;
                    float mb = __builtin_fmaf(gamma, dbar, -(gamma * ub));
                    mb += sel<kTapeK>(nd, i, mminb);
                    mb = valid ? mb : 0.0f;
                    const float rcb = vbar[i] + ub + mb;
                    revb[i] = out ? mb : 0.0f;
                    rbar[i] = ab[i] + rcb;
                    cbar[i] = valid ? rcb : 0.0f;
                }
            } else if constexpr (KIND == kAdjNaive) {
                const float mminb = inv_n * al;
#pragma unroll
                for (int i = 0; i < LPL; ++i) {
                    const bool valid = FULL || lv[i];
                    vbar[i] += sel<kTapeA>(nd, i, zl);
                    const float mb = valid ? __builtin_fmaf(-inv_n, ab[i], sel<kTapeK>(nd, i, mminb)) : 0.0f;
                    const float rcb = vbar[i] + mb;
                    revb[i] = out ? mb : 0.0f;
                    rbar[i] = ab[i] + rcb;
                    cbar[i] = valid ? rcb : 0.0f;
                }
            } else {  // final pass
                int first = 0x7fffffff;
#pragma unroll
                for (int i = 0; i < LPL; ++i) {
                    const bool valid = FULL || lv[i];
                    const bool isk = has(nd, i, kTapeK);
                    vbar[i] += sel<kTapeA>(nd, i, zl);
                    float mb = valid ? nd.gx.get(i) : 0.0f;
                    mb -= sel<kTapeK>(nd, i, al);
                    const float rcb = vbar[i] + mb;
                    revb[i] = out ? mb : 0.0f;
                    rbar[i] = rcb + sel<kTapeK>(nd, i, g_lb_f);
                    cbar[i] = valid ? rcb : 0.0f;
                    if (isk) first = sub * LPL + i;
                }
                const int kstar = group_min_i<G>(first);
                if (out) {
                    int dd = kstar - next_label;
                    dd = dd < 0 ? -dd : dd;
                    wl = __builtin_fmaf(g_lb_f, (float)(dd < T ? dd : T), wl);
                }
                next_label = kstar;
            }
            label_offsets<4>(rs, os);
            store_f32<LPL, FULL>(r_bout, rs, os, revb);
            label_offsets<4>(sc.f, os);
            store_f32<LPL, FULL>(r_abar, sc.f, os, rbar);
        }
        if constexpr (BATCH)
            wacc = sub == wb ? wl : wacc;
        else if (ok && sub == 0 && out)
            add_edge_grad(sc.w, wl);
        advance<FWD>(sc);
    }

    // One adjoint pass over the forward pass FWD of kind KIND.  IS_FIRST: the half-step's
    // last update pass (its input adjoint in lbar is dL/d(dual after the half-step); it is
    // turned into units of the family's unaries r = cost - dual (rows) or dual (columns)
    // and, for rows, added to dL/dcost).  R0: writes dL/d(dual before the half-step) back
    // to lbar and adds dL/dr to dL/dcost for rows.
    template <bool FWD, int KIND, bool IS_FIRST, int DTM>
    __device__ __forceinline__ void pass(float gamma) {
        float cbar[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) cbar[i] = 0.0f;
        int next_label = 0;  // final pass: optimum label of the node visited before
        Cursor lc = cursor_start(FWD);
        Cursor sc = lc;
        Node ring[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            load<FWD, KIND, IS_FIRST>(ring[q], lc);
            __builtin_amdgcn_sched_barrier(0);  // keep slot order (the loop's waits assume it)
        }
        int t0 = 0;
        for (; t0 + PF <= n; t0 += PF) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                step<FWD, KIND, IS_FIRST, DTM>(ring[q], t0 + q, cbar, gamma, next_label, sc);
                load<FWD, KIND, IS_FIRST>(ring[q], lc);
            }
        }
#pragma unroll
        for (int q = 0; q < PF; ++q)
            if (t0 + q < n) step<FWD, KIND, IS_FIRST, DTM>(ring[q], t0 + q, cbar, gamma, next_label, sc);
    }

    // The recomputing form: scans for a forward that used them with one lane of reach,
    // else the window search (the direct window forward's rule, and the general reach).
    template <bool FWD, int KIND, bool IS_FIRST>
    __device__ __forceinline__ void run_pass(float gamma) {
        if (!direct && dt_steps == 1)
            pass<FWD, KIND, IS_FIRST, 1>(gamma);
        else
            pass<FWD, KIND, IS_FIRST, 2>(gamma);
    }

    // Adjoint of the forward step at the node visited t-th (t = 0: the pass's last node).
    template <bool FWD, int KIND, bool IS_FIRST, int DTM>
    __device__ __forceinline__ void step(const Node& nd, int t, float (&cbar)[LPL], float gamma, int& next_label,
                                         Cursor& sc) {
        const bool out = t != 0;        // a message leaves this node in the forward pass
        const bool has_c = t != n - 1;  // a carried message arrives at it
        const unsigned rs = FWD ? sc.f : sc.f - f_step;
        unsigned os[LPL];
        float r[LPL], carry[LPL], ab[LPL], cb[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            const float lam = nd.lam.get(i);
            const float x = HAS_THETA ? nd.th.get(i) - lam : lam;
            r[i] = (FULL || lv[i]) ? x : kBig;
            carry[i] = has_c ? nd.cmsg.get(i) : 0.0f;
            ab[i] = KIND == kAdjFinal ? 0.0f : nd.abar.get(i);
            cb[i] = out ? cbar[i] + nd.bin.get(i) : 0.0f;
        }
        if constexpr (IS_FIRST) {
            if constexpr (HAS_THETA) {
                float g[LPL];
#pragma unroll
                for (int i = 0; i < LPL; ++i) g[i] = nd.gx.get(i) + ab[i];
                label_offsets<4>(sc.f, os);
                store_f32<LPL, FULL>(r_gth, sc.f, os, g);
            }
#pragma unroll
            for (int i = 0; i < LPL; ++i) ab[i] = (sign > 0.0f) ? -ab[i] : ab[i];
        }
        float vbar[LPL], wl = 0.0f, zl = 0.0f;
        if constexpr (KIND == kAdjR0) {
            float v[LPL];
#pragma unroll
            for (int i = 0; i < LPL; ++i) v[i] = carry[i] + r[i];
            const float vmin = group_min<G>(lane_min(v));
            msg_adjoint<DTM>(v, vmin, nd.w, cb, vbar, wl, zl);
            group_sum2<G>(wl, zl);
            const int a_v = group_argmin_eq<G, LPL, FULL>(v, vmin, lv, sub);
            float rt[LPL], outv[LPL];
#pragma unroll
            for (int i = 0; i < LPL; ++i) {
                if (sub * LPL + i == a_v) vbar[i] += zl;
                rt[i] = ab[i] + vbar[i];
                cbar[i] = (FULL || lv[i]) ? vbar[i] : 0.0f;
                outv[i] = sign > 0.0f ? -rt[i] : rt[i];  // dL/d(dual before the half-step)
            }
            label_offsets<4>(sc.f, os);
            if constexpr (HAS_THETA) {
                float g[LPL];
#pragma unroll
                for (int i = 0; i < LPL; ++i) g[i] = nd.gx.get(i) + rt[i];
                store_f32<LPL, FULL>(r_gth, sc.f, os, g);
            }
            store_f32<LPL, FULL>(r_abar, sc.f, os, outv);
        } else {
            // replay the forward step (same arithmetic as the forward walker)
            float v[LPL], m[LPL], vn[LPL];
#pragma unroll
            for (int i = 0; i < LPL; ++i) {
                v[i] = r[i] + carry[i];
                m[i] = v[i] + (out ? nd.rmsg.get(i) : 0.0f);
            }
            // message input: v (naive, final) or u = rc - gamma*m (iterative; the updated
            // r' + carry up to the node constant gamma*mmin)
            float mmin = lane_min(m), bmin;
#pragma unroll
            for (int i = 0; i < LPL; ++i)
                vn[i] = KIND == kAdjIter ? ((FULL || lv[i]) ? __builtin_fmaf(-gamma, m[i], v[i]) : kBig) : v[i];
            bmin = lane_min(vn);
            group_min2<G>(mmin, bmin);
            const int kstar = group_argmin_eq<G, LPL, FULL>(m, mmin, lv, sub);
            if (out) {
                msg_adjoint<DTM>(vn, bmin, nd.w, cb, vbar, wl, zl);
            } else {
#pragma unroll
                for (int i = 0; i < LPL; ++i) vbar[i] = 0.0f;
            }
            // third sum: dL/d(r out) (update passes) or dL/dminmarg (final pass)
            float al = 0.0f;
#pragma unroll
            for (int i = 0; i < LPL; ++i)
                al += (FULL || lv[i]) ? (KIND == kAdjFinal ? nd.gx.get(i) : ab[i]) : 0.0f;
            group_sum2<G>(wl, zl);
            al = group_sum<G>(al);
            const int a_b = group_argmin_eq<G, LPL, FULL>(vn, bmin, lv, sub);
            float rbar[LPL], revb[LPL];
            if constexpr (KIND == kAdjIter) {
                // message of u = rc - gamma m, d = gamma (m - mmin), r' = r - d;
                // dL/dmmin sums to gamma * sum(dL/dr')
                const float mminb = gamma * al;
#pragma unroll
                for (int i = 0; i < LPL; ++i) {
                    const bool valid = FULL || lv[i];
                    const int lab = sub * LPL + i;
                    const float ub = lab == a_b ? zl : 0.0f;
                    const float dbar = valid ? -vbar[i] - ab[i] : 0.0f;
                    float mb = __builtin_fmaf(gamma, dbar, -(gamma * ub));
                    if (lab == kstar) mb += mminb;
                    mb = valid ? mb : 0.0f;
                    const float rcb = vbar[i] + ub + mb;
                    revb[i] = out ? mb : 0.0f;
                    rbar[i] = ab[i] + rcb;
                    cbar[i] = valid ? rcb : 0.0f;
                }
            } else if constexpr (KIND == kAdjNaive) {
                const float mminb = inv_n * al;
#pragma unroll
                for (int i = 0; i < LPL; ++i) {
                    const bool valid = FULL || lv[i];
                    const int lab = sub * LPL + i;
                    if (lab == a_b) vbar[i] += zl;
                    const float mb = valid ? __builtin_fmaf(-inv_n, ab[i], lab == kstar ? mminb : 0.0f) : 0.0f;
                    const float rcb = vbar[i] + mb;
                    revb[i] = out ? mb : 0.0f;
                    rbar[i] = ab[i] + rcb;
                    cbar[i] = valid ? rcb : 0.0f;
                }
            } else {  // final pass: normalized min-marginals mm = m - mmin, lower bound
#pragma unroll
                for (int i = 0; i < LPL; ++i) {
                    const bool valid = FULL || lv[i];
                    const int lab = sub * LPL + i;
                    if (lab == a_b) vbar[i] += zl;
                    float mb = valid ? nd.gx.get(i) : 0.0f;
                    if (lab == kstar) mb -= al;
                    const float rcb = vbar[i] + mb;
                    revb[i] = out ? mb : 0.0f;
                    // d(row optimum)/dr = one-hot of the optimum's label
                    rbar[i] = rcb + ((lab == kstar) ? g_lb_f : 0.0f);
                    cbar[i] = valid ? rcb : 0.0f;
                }
                if (out) {
                    int dd = kstar - next_label;
                    dd = dd < 0 ? -dd : dd;
                    wl = __builtin_fmaf(g_lb_f, (float)(dd < T ? dd : T), wl);
                }
                next_label = kstar;
            }
            label_offsets<4>(rs, os);
            store_f32<LPL, FULL>(r_bout, rs, os, revb);
            label_offsets<4>(sc.f, os);
            store_f32<LPL, FULL>(r_abar, sc.f, os, rbar);
        }
        if (ok && sub == 0 && out && wl != 0.0f) add_edge_grad(sc.w, wl);
        advance<FWD>(sc);
    }
};

// One adjoint pass, recomputing the selections (TAPE false) or reading them from the
// pass's tape.
template <bool TAPE, bool FWD, int KIND, bool IS_FIRST, typename AW>
__device__ __forceinline__ void adjoint_pass(AW& wk, const unsigned* tape, unsigned tape_bytes, float g) {
    if constexpr (TAPE) {
        wk.r_tape = make_rsrc(tape, tape_bytes);
        wk.template run_pass_tape<FWD, KIND, IS_FIRST>(g);
    } else {
        wk.template run_pass<FWD, KIND, IS_FIRST>(g);
    }
}

// The adjoint passes of one launch (a half-step's, or the final row pass's) for the chain
// walked by `wk` (an AdjWalker, or a walker of the same interface).
template <bool TAPE, class AW>
__device__ __forceinline__ void run_adjoint_walker(const AdjArgs& a, AW& wk) {
    const unsigned vb = a.vol_bytes_f32;
    const unsigned tb = a.tape_bytes;
    if (a.mode == kModeFinal) {
        // final row pass: forward min-marginal pass (messages M[1], reverse M[0]), then R0
        wk.g_lb_f = a.g_lb != nullptr ? (float)a.g_lb[0] : 0.0f;
        wk.r_lam = make_rsrc(a.lam0, vb);
        wk.r_cmsg = make_rsrc(a.rec_msg[1], vb);
        wk.r_rmsg = make_rsrc(a.rec_msg[0], vb);
        wk.r_bin = make_rsrc(nullptr, 0u);
        wk.r_bout = make_rsrc(a.bbar[0], vb);
        adjoint_pass<TAPE, true, kAdjFinal, false>(wk, a.tape[1], tb, 0.0f);
        wk.r_cmsg = make_rsrc(a.rec_msg[0], vb);
        wk.r_bin = make_rsrc(a.bbar[0], vb);
        wk.r_bout = make_rsrc(nullptr, 0u);
        // the final pass's R0 adjoint turns dL/dr into dL/dcost and dL/d(dual) = -dL/dr
        adjoint_pass<TAPE, false, kAdjR0, false>(wk, a.tape[0], tb, 0.0f);
        return;
    }
    const int P = a.mode == kModeIterative ? a.n_pass : 1;
    for (int s = P; s >= 1; --s) {
        const float* lam_s = a.lam0;
        const float* msg_s = a.rec_msg[1];
        const float* msg_r = a.rec_msg[0];
        const unsigned* tp = a.tape[1];
        float g = a.gamma[0];
#pragma unroll
        for (int i = 1; i <= 8; ++i) {
            if (s == i) {
                if (i > 1) lam_s = a.rec_lam[i - 1 < 8 ? i - 1 : 7];
                msg_s = a.rec_msg[i];
                msg_r = a.rec_msg[i - 1];
                tp = a.tape[i];
                g = a.gamma[i - 1];
            }
        }
        wk.r_lam = make_rsrc(lam_s, vb);
        wk.r_cmsg = make_rsrc(msg_s, vb);
        wk.r_rmsg = make_rsrc(msg_r, vb);
        const bool has_bin = s < P;
        // selects, not a dynamic index (which would put the argument block in scratch)
        float* const b_odd = a.bbar[1];
        float* const b_even = a.bbar[0];
        wk.r_bin = make_rsrc((s & 1) ? b_odd : b_even, has_bin ? vb : 0u);
        wk.r_bout = make_rsrc((s & 1) ? b_even : b_odd, vb);
        const bool fwd = ((s - 1) & 1) == 0;
        if (a.mode == kModeNaive) {
            adjoint_pass<TAPE, true, kAdjNaive, true>(wk, tp, tb, 0.0f);
        } else if (s == P) {
            if (fwd) adjoint_pass<TAPE, true, kAdjIter, true>(wk, tp, tb, g);
            else adjoint_pass<TAPE, false, kAdjIter, true>(wk, tp, tb, g);
        } else {
            if (fwd) adjoint_pass<TAPE, true, kAdjIter, false>(wk, tp, tb, g);
            else adjoint_pass<TAPE, false, kAdjIter, false>(wk, tp, tb, g);
        }
    }
    wk.r_lam = make_rsrc(a.lam0, vb);
    wk.r_cmsg = make_rsrc(a.rec_msg[0], vb);
    wk.r_bin = make_rsrc(a.bbar[0], vb);
    wk.r_bout = make_rsrc(nullptr, 0u);
    adjoint_pass<TAPE, false, kAdjR0, false>(wk, a.tape[0], tb, 0.0f);
}

template <int G, int LPL, int PF, typename TT, bool FULL, bool HAS_THETA, bool TAPE>
__global__ __launch_bounds__(64) void adjoint_kernel(AdjArgs a) {
    using AW = AdjWalker<G, LPL, PF, TT, FULL, HAS_THETA>;
    // LDS for the recomputing form's long-reach message adjoint (unused with a tape)
    __shared__ float s_v[TAPE ? 1 : 64 * LPL];
    __shared__ float s_cb[TAPE ? 1 : 64 * LPL];
    __shared__ int s_src[TAPE ? 1 : 64 * LPL];
    constexpr int CPW = 64 / G;
    const int lane = threadIdx.x;
    const int sub = lane % G;
    const int grp = lane / G;
    const int chain = blockIdx.x * CPW + grp;
    AW wk(a, chain, sub, grp, s_v, s_cb, s_src);
    run_adjoint_walker<TAPE>(a, wk);
}

constexpr int kAdjPF = 4;      // recomputing form: a node's ring slot holds cost, dual and two messages
constexpr int kAdjTapePF = 8;  // tape form: a slot holds the tape word and two adjoints only

template <int G, int LPL, typename TT, bool HAS_THETA, bool TAPE>
hipError_t launch_adjoint_tt(const AdjArgs& a, hipStream_t st) {
    constexpr int CPW = 64 / G;
    const unsigned blocks = (unsigned)((a.n_chains + CPW - 1) / CPW);
    constexpr int PF = TAPE ? kAdjTapePF : kAdjPF;
    if (a.K == G * LPL)
        hipLaunchKernelGGL((adjoint_kernel<G, LPL, PF, TT, true, HAS_THETA, TAPE>), dim3(blocks), dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL((adjoint_kernel<G, LPL, PF, TT, false, HAS_THETA, TAPE>), dim3(blocks), dim3(64), 0, st, a);
    return hipGetLastError();
}

// TAPE: the selections come from the tapes a.tape[] written by the record sweep in tape
// mode (distance transforms that reach at most one lane across).
template <int G, int LPL, bool TAPE>
hipError_t launch_adjoint_tile(const AdjArgs& a, dm_dtype dt, hipStream_t st) {
    if (a.theta == nullptr) return launch_adjoint_tt<G, LPL, float, false, TAPE>(a, st);
    if (dt == DM_F16) return launch_adjoint_tt<G, LPL, _Float16, true, TAPE>(a, st);
    return launch_adjoint_tt<G, LPL, float, true, TAPE>(a, st);
}

}  // namespace dm
