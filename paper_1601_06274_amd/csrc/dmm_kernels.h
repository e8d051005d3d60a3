// dmm_kernels.h - Dual_MM on gfx950: chain sweeps over the horizontal / vertical families.
//
// Paper: Sec. 2.3 (dual decomposition into horizontal and vertical chains,
// Alg. Dual_MM), App. A.1 (min-marginals via left/right messages, eq. msg-pass and
// eq. min-marg-expression), App. A.3.2 (Alg. Iterative Minorant), Sec. 2.3 / App. A.1
// (naive minorant m/n).
//
// Mapping to the hardware
//   * One chain is owned by a group of G lanes of one wavefront; each lane holds LPL
//     consecutive labels (label k = sub*LPL + i), so a node's K-vector is one
//     contiguous, coalesced read of the label-major volume for rows and for columns.
//   * A pass walks the chain node by node.  The message arriving from the side not
//     yet visited is read from the message buffer; the message in the walking
//     direction is carried in registers.  Loads run PF nodes ahead of the
//     computation through a register ring, so memory latency overlaps the
//     per-node critical path.  All loads and stores are buffer instructions whose
//     out-of-range offsets read 0 / are dropped by the hardware, so the loop has no
//     branches around memory operations and the wait counters stay exact.
//   * Min over labels = in-lane min + DPP butterfly (quad_perm, row mirrors) +
//     gfx950 permlane16/32 swaps for groups of 32/64 lanes.
//   * Message for the truncated-linear pairwise term w*min(|a-b|, T): the two-pass
//     L1 distance transform (a forward and a backward lower-envelope scan, in-lane,
//     extended across lane boundaries with wave_shr/wave_shl DPP for as many lanes as
//     the truncation radius T-1 needs) followed by min(., min v + wT).  O(K) work per
//     message for fixed T.
//   * Messages are renormalised to minimum 0 at every step (they are defined up to a
//     constant); the subtracted constants add up to the chain optimum, accumulated in
//     FP64 for the lower bound.
//   * All passes of one half-step for a chain run inside one launch by the owning
//     wave; the only dependency between chains is the half-step boundary, which is
//     the kernel boundary.
//
// Message buffer convention: slot j of a chain (stored at node j's position) holds
// the message on edge (j, j+1) - the backward message phi_{j+1,j} after a backward
// pass, the forward message phi_{j,j+1} after a forward pass.  Each pass overwrites a
// slot only after reading it, so one volume serves all passes.
#pragma once

#include <hip/hip_fp16.h>

#include "common.h"
#include "wave.h"

namespace dm {

enum SweepMode : int {
    kModeIterative = 0,  // iterative-minorant half-step
    kModeNaive = 1,      // naive-minorant half-step
    kModeOptimum = 2,    // chain optimum only (backward message pass, no stores)
    kModeFinal = 3,      // normalized min-marginals + argmin labels + optimum
};
// Launch flag (added to mode): recompute a half-step keeping every pass's messages and
// intermediate duals (the adjoint's input).
constexpr int kRecordFlag = 16;

struct SweepArgs {
    const void* theta;   // [H][W][K] cost (horizontal family) or nullptr (vertical family)
    float* lam;          // [H][W][K] dual variables (written; read after the first update pass)
    const float* lam_in; // dual variables read by the message pass and the first update pass
                         // (== lam for an in-place half-step; a checkpoint otherwise)
    float* msg;          // [H][W][K] message buffer
    const float* w;      // edge weights of this family
    float* minmarg;      // kModeFinal: [H][W][K] (may be null)
    int* labels;         // kModeFinal: [H][W]
    double* opt;         // per-chain optimum (may be null)
    long long chain_px;  // pixel offset between consecutive chains
    long long node_px;   // pixel offset between consecutive nodes of a chain
    long long w_chain;   // edge-array offset between chains
    long long w_node;    // edge-array offset between consecutive edges of a chain
    unsigned vol_bytes_f32;  // bytes of one FP32 [H][W][K] volume (< 4 GiB)
    unsigned vol_bytes_theta;
    unsigned w_bytes;        // bytes of the edge array
    int K, n, n_chains, T, mode, n_pass;
    float sign;          // +1: lambda += delta (horizontal), -1: lambda -= delta (vertical)
    float inv_n;         // 1/n for the naive minorant
    float gamma[8];
    float* rec_lam[8];   // record mode: dual after update pass s (s = 1 .. n_pass-1)
    float* rec_msg[9];   // record mode: messages written by pass s (s = 0: backward message pass)
};

// Offset that is outside every buffer: loads return 0, stores are dropped.
constexpr unsigned kOOB = 0xFFFFFFF0u;
constexpr int kBufWord3 = 0x00020000;  // gfx9 raw buffer descriptor word 3

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kBufWord3);
}

template <typename TT> __device__ __forceinline__ float to_f(TT x);
template <> __device__ __forceinline__ float to_f<float>(float x) { return x; }
template <> __device__ __forceinline__ float to_f<_Float16>(_Float16 x) { return (float)x; }

__device__ __forceinline__ float f16_bits_to_f(uint32_t b) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(b & 0xFFFFu));
}

// Raw words of LPL consecutive elements of type TT, loaded with one vector buffer load
// when the tile is full (all labels exist), else one scalar load per label.
template <typename TT, int LPL, bool FULL>
struct RawVec;

template <int LPL, bool FULL>
struct RawVec<float, LPL, FULL> {
    uint32_t w[LPL];
    // off[i]: byte offset of element i (only off[0] used for the vector form)
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, unsigned off0, const unsigned (&offs)[LPL]) {
        if constexpr (FULL && LPL == 4) {
            auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off0, 0, 0);
            w[0] = v[0]; w[1] = v[1]; w[2] = v[2]; w[3] = v[3];
        } else if constexpr (FULL && LPL == 3) {
            auto v = __builtin_amdgcn_raw_buffer_load_b96(r, (int)off0, 0, 0);
            w[0] = v[0]; w[1] = v[1]; w[2] = v[2];
        } else if constexpr (FULL && LPL == 2) {
            auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off0, 0, 0);
            w[0] = v[0]; w[1] = v[1];
        } else {
#pragma unroll
            for (int i = 0; i < LPL; ++i) w[i] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)offs[i], 0, 0);
        }
    }
    __device__ __forceinline__ float get(int i) const { return __builtin_bit_cast(float, w[i]); }
};

template <int LPL, bool FULL>
struct RawVec<_Float16, LPL, FULL> {
    static constexpr bool kPacked = FULL && (LPL == 2 || LPL == 4);
    static constexpr int kWords = kPacked ? LPL / 2 : LPL;
    uint32_t w[kWords];
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, unsigned off0, const unsigned (&offs)[LPL]) {
        if constexpr (FULL && LPL == 4) {
            auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off0, 0, 0);
            w[0] = v[0]; w[1] = v[1];
        } else if constexpr (FULL && LPL == 2) {
            w[0] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)off0, 0, 0);
        } else {
#pragma unroll
            for (int i = 0; i < LPL; ++i) w[i] = __builtin_amdgcn_raw_buffer_load_b16(r, (int)offs[i], 0, 0);
        }
    }
    __device__ __forceinline__ float get(int i) const {
        if constexpr (kPacked) return f16_bits_to_f(w[i >> 1] >> (16 * (i & 1)));
        else return f16_bits_to_f(w[i]);
    }
};

template <int LPL, bool FULL>
__device__ __forceinline__ void store_f32(__amdgpu_buffer_rsrc_t r, unsigned off0, const unsigned (&offs)[LPL],
                                          const float (&v)[LPL]) {
    if constexpr (FULL && LPL == 4) {
        __builtin_amdgcn_raw_buffer_store_b128(
            (__attribute__((ext_vector_type(4))) unsigned){__builtin_bit_cast(uint32_t, v[0]), __builtin_bit_cast(uint32_t, v[1]),
                                                           __builtin_bit_cast(uint32_t, v[2]), __builtin_bit_cast(uint32_t, v[3])},
            r, (int)off0, 0, 0);
    } else if constexpr (FULL && LPL == 3) {
        __builtin_amdgcn_raw_buffer_store_b96(
            (__attribute__((ext_vector_type(3))) unsigned){__builtin_bit_cast(uint32_t, v[0]), __builtin_bit_cast(uint32_t, v[1]),
                                                           __builtin_bit_cast(uint32_t, v[2])},
            r, (int)off0, 0, 0);
    } else if constexpr (FULL && LPL == 2) {
        __builtin_amdgcn_raw_buffer_store_b64(
            (__attribute__((ext_vector_type(2))) unsigned){__builtin_bit_cast(uint32_t, v[0]), __builtin_bit_cast(uint32_t, v[1])},
            r, (int)off0, 0, 0);
    } else {
#pragma unroll
        for (int i = 0; i < LPL; ++i) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v[i]), r, (int)offs[i], 0, 0);
    }
}

// ------------------------------------------------------------------ chain walker
template <int G, int LPL, int PF, typename TT, bool FULL, bool HAS_THETA>
struct Walker {
    // One prefetched node: raw cost words, dual, reverse message, edge weight.
    struct Node {
        RawVec<TT, LPL, FULL> th;
        RawVec<float, LPL, FULL> lam;
        RawVec<float, LPL, FULL> rev;
        float w;
    };

    __amdgpu_buffer_rsrc_t r_theta, r_w, r_mm;
    // buffers of the current pass: dual loads / stores, reverse-message loads, message stores
    __amdgpu_buffer_rsrc_t r_lam_ld, r_lam_st, r_msg_ld, r_msg_st;
    unsigned vol_bytes;
    int* __restrict__ labels;
    long long base_px, wbase, node_px, w_node;
    int sub, n, K, T;
    float sign, inv_n;
    bool ok;          // this group's chain exists
    bool lv[LPL];     // label valid
    int dt_steps;     // lanes the distance transform must reach across

    __device__ Walker(SweepArgs args, int chain, int sub_)
        : labels(args.labels), node_px(args.node_px), w_node(args.w_node), sub(sub_), n(args.n), K(args.K),
          T(args.T), sign(args.sign), inv_n(args.inv_n) {
        ok = chain < args.n_chains;
        base_px = (long long)(ok ? chain : 0) * args.chain_px;
        wbase = (long long)(ok ? chain : 0) * args.w_chain;
        r_theta = make_rsrc(args.theta, HAS_THETA ? args.vol_bytes_theta : 0u);
        vol_bytes = args.vol_bytes_f32;
        r_lam_ld = make_rsrc(args.lam_in != nullptr ? args.lam_in : args.lam, vol_bytes);
        r_lam_st = make_rsrc(args.lam, vol_bytes);
        r_msg_ld = make_rsrc(args.msg, vol_bytes);
        r_msg_st = r_msg_ld;
        r_w = make_rsrc(args.w, args.w_bytes);
        r_mm = make_rsrc(args.minmarg, args.minmarg != nullptr ? args.vol_bytes_f32 : 0u);
#pragma unroll
        for (int i = 0; i < LPL; ++i) lv[i] = FULL ? true : (sub * LPL + i < K);
        const int need = (args.T - 1 + LPL - 1) / LPL;
        dt_steps = need < G - 1 ? need : G - 1;
    }

    // Element index of this lane's first label at node j.
    __device__ __forceinline__ long long elem(int j) const { return (base_px + (long long)j * node_px) * K + sub * LPL; }

    // Byte offsets (element size ES) of this lane's labels at node j; out of range when
    // `valid` is false or the label does not exist.
    template <int ES>
    __device__ __forceinline__ void offsets(int j, bool valid, unsigned& off0, unsigned (&offs)[LPL]) const {
        const unsigned base = (unsigned)(elem(j) * ES);
        off0 = (valid && ok) ? base : kOOB;
#pragma unroll
        for (int i = 0; i < LPL; ++i) offs[i] = (valid && ok && lv[i]) ? base + (unsigned)(i * ES) : kOOB;
    }

    // Loads node j of a pass in direction FWD (j is clamped by the caller to [0, n-1]).
    template <bool FWD, bool WANT_REV>
    __device__ __forceinline__ void load(Node& nd, int j) const {
        unsigned o0, os[LPL];
        if constexpr (HAS_THETA) {
            offsets<(int)sizeof(TT)>(j, true, o0, os);
            nd.th.load(r_theta, o0, os);
        }
        offsets<4>(j, true, o0, os);
        nd.lam.load(r_lam_ld, o0, os);
        const bool has = FWD ? (j < n - 1) : (j > 0);
        if constexpr (WANT_REV) {
            offsets<4>(FWD ? j : j - 1, has, o0, os);
            nd.rev.load(r_msg_ld, o0, os);
        }
        const long long ei = wbase + (long long)(FWD ? j : j - 1) * w_node;
        const unsigned wo = (has && ok) ? (unsigned)(ei * 4) : kOOB;
        nd.w = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r_w, (int)wo, 0, 0));
    }

    // Truncated-linear message of v (normalised by its minimum vmin), into out.
    __device__ __forceinline__ void message(const float (&v)[LPL], float vmin, float wt, float (&out)[LPL]) const {
        float f[LPL], b[LPL];
        f[0] = v[0];
#pragma unroll
        for (int i = 1; i < LPL; ++i) f[i] = fminf(v[i], f[i - 1] + wt);
        b[LPL - 1] = v[LPL - 1];
#pragma unroll
        for (int i = LPL - 2; i >= 0; --i) b[i] = fminf(v[i], b[i + 1] + wt);
        for (int s = 0; s < dt_steps; ++s) {
            float cl = dpp_fill<kWaveShr1>(f[LPL - 1], kBig);
            float cr = dpp_fill<kWaveShl1>(b[0], kBig);
            if (sub == 0) cl = kBig;
            if (sub == G - 1) cr = kBig;
#pragma unroll
            for (int i = 0; i < LPL; ++i) {
                f[i] = fminf(f[i], cl + wt * (float)(i + 1));
                b[i] = fminf(b[i], cr + wt * (float)(LPL - i));
            }
        }
        const float cap = vmin + wt * (float)T;
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            float d = fminf(fminf(f[i], b[i]), cap) - vmin;
            out[i] = lv[i] ? d : 0.0f;
        }
    }

    __device__ __forceinline__ float lane_min(const float (&x)[LPL]) const {
        float m = x[0];
#pragma unroll
        for (int i = 1; i < LPL; ++i) m = fminf(m, x[i]);
        return m;
    }

    // One directional pass.  KIND: 0 = backward message pass (R0), 1 = iterative update,
    // 2 = naive update, 3 = final min-marginals.  Adds the normalisation constants of a
    // message pass (= chain optimum) to `opt`.
    template <bool FWD, int KIND>
    __device__ void pass(float gamma, bool store_msg, double& opt) {
        constexpr bool WANT_REV = KIND != 0;
        float carry[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) carry[i] = 0.0f;
        Node ring[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int t = q < n ? q : n - 1;
            load<FWD, WANT_REV>(ring[q], FWD ? t : n - 1 - t);
        }
        int t0 = 0;
        // Steady state: PF nodes per iteration, loads for node t+PF issued before node t
        // is processed (clamped to the last node near the end: a redundant reload).
        for (; t0 + PF <= n; t0 += PF) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int t = t0 + q;
                Node cur = ring[q];
                const int tn = (t + PF < n) ? t + PF : n - 1;
                load<FWD, WANT_REV>(ring[q], FWD ? tn : n - 1 - tn);
                step<FWD, KIND>(cur, FWD ? t : n - 1 - t, carry, gamma, store_msg, opt);
            }
        }
        // Tail: fewer than PF nodes left, already in the ring.
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int t = t0 + q;
            if (t < n) step<FWD, KIND>(ring[q], FWD ? t : n - 1 - t, carry, gamma, store_msg, opt);
        }
    }

    template <bool FWD, int KIND>
    __device__ __forceinline__ void step(const Node& nd, int j, float (&carry)[LPL], float gamma, bool store_msg,
                                         double& opt) {
        float r[LPL], lamv[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            lamv[i] = nd.lam.get(i);
            const float x = HAS_THETA ? nd.th.get(i) - lamv[i] : lamv[i];
            r[i] = lv[i] ? x : kBig;
        }
        float v[LPL];
        if constexpr (KIND == 0) {
#pragma unroll
            for (int i = 0; i < LPL; ++i) v[i] = carry[i] + r[i];
        } else {
            float m[LPL];
#pragma unroll
            for (int i = 0; i < LPL; ++i) m[i] = r[i] + carry[i] + nd.rev.get(i);
            const float mmin = group_min<G>(lane_min(m));
            if constexpr (KIND == 1 || KIND == 2) {
                float nl[LPL];
#pragma unroll
                for (int i = 0; i < LPL; ++i) {
                    float d = (KIND == 1 ? gamma : inv_n) * (m[i] - mmin);
                    d = lv[i] ? d : 0.0f;
                    if (KIND == 1) r[i] -= d;
                    nl[i] = lamv[i] + sign * d;
                }
                unsigned o0, os[LPL];
                offsets<4>(j, true, o0, os);
                store_f32<LPL, FULL>(r_lam_st, o0, os, nl);
            } else {  // KIND == 3: normalized min-marginals and argmin
                float mm[LPL];
                int first = 0x7fffffff;
#pragma unroll
                for (int i = LPL - 1; i >= 0; --i) {
                    mm[i] = m[i] - mmin;
                    if (lv[i] && m[i] == mmin) first = sub * LPL + i;
                }
                int lab = group_min_i<G>(first);
                lab = lab < K ? lab : K - 1;  // defensive: a label always exists for finite costs
                unsigned o0, os[LPL];
                offsets<4>(j, true, o0, os);
                store_f32<LPL, FULL>(r_mm, o0, os, mm);
                if (ok && sub == 0) labels[base_px + (long long)j * node_px] = lab;
            }
#pragma unroll
            for (int i = 0; i < LPL; ++i) v[i] = carry[i] + r[i];
        }
        const bool has_next = FWD ? (j < n - 1) : (j > 0);
        if (KIND == 0 || has_next) {
            const float vmin = group_min<G>(lane_min(v));
            if constexpr (KIND == 0) opt += (double)vmin;
            if (has_next) {
                message(v, vmin, nd.w, carry);
                if (store_msg) {
                    unsigned o0, os[LPL];
                    offsets<4>(FWD ? j : j - 1, true, o0, os);
                    store_f32<LPL, FULL>(r_msg_st, o0, os, carry);
                }
            }
        }
    }
};

// Mode groups compiled as separate kernels (separate symbols in profiles, and each
// kernel holds only the passes it runs): half-step (iterative or naive minorant),
// final row pass, column optimum pass.
enum ModeGroup : int { kGroupHalfStep = 0, kGroupFinal = 1, kGroupOptimum = 2, kGroupRecord = 3 };

// All passes of one mode group for the chain owned by this lane group.
template <int G, int LPL, int PF, typename TT, bool FULL, bool HAS_THETA, int MG>
__device__ __forceinline__ void run_chain(const SweepArgs& a, int chain, int sub) {
    Walker<G, LPL, PF, TT, FULL, HAS_THETA> wk(a, chain, sub);
    double opt = 0.0;
    if constexpr (MG == kGroupHalfStep) {
        // R0 and the first update pass read lam_in; update passes write lam
        const __amdgpu_buffer_rsrc_t lam_out = wk.r_lam_st;
        wk.r_lam_st = make_rsrc(nullptr, 0u);
        wk.template pass<false, 0>(0.0f, true, opt);
        wk.r_lam_st = lam_out;
        if (a.mode == kModeIterative) {
            for (int s = 0; s < a.n_pass; ++s) {
                const bool last = s == a.n_pass - 1;
                if (s == 1) wk.r_lam_ld = lam_out;
                // select instead of a dynamic index: keeps the argument block out of scratch
                float g = a.gamma[0];
#pragma unroll
                for (int i = 1; i < 8; ++i)
                    if (s == i) g = a.gamma[i];
                if ((s & 1) == 0)
                    wk.template pass<true, 1>(g, !last, opt);
                else
                    wk.template pass<false, 1>(g, !last, opt);
            }
        } else {
            wk.template pass<true, 2>(0.0f, false, opt);
        }
    } else if constexpr (MG == kGroupFinal) {
        wk.template pass<false, 0>(0.0f, true, opt);
        wk.template pass<true, 3>(0.0f, false, opt);
    } else if constexpr (MG == kGroupOptimum) {
        wk.template pass<false, 0>(0.0f, false, opt);
    } else {  // kGroupRecord: recompute a half-step keeping every pass's messages and duals
        const unsigned vb = wk.vol_bytes;
        wk.r_lam_st = make_rsrc(nullptr, 0u);
        wk.r_msg_st = make_rsrc(a.rec_msg[0], vb);
        wk.template pass<false, 0>(0.0f, true, opt);
        const int P = a.mode == kModeIterative ? a.n_pass : 1;
        for (int s = 0; s < P; ++s) {
            const float* ld = a.lam_in;
            float* st = nullptr;
            float* mld = a.rec_msg[0];
            float* mst = a.rec_msg[1];
#pragma unroll
            for (int i = 1; i < 8; ++i) {
                if (s == i) {
                    ld = a.rec_lam[i];
                    mld = a.rec_msg[i];
                    mst = a.rec_msg[i + 1];
                }
            }
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (s == i && s + 1 < P) st = a.rec_lam[i + 1];
            wk.r_lam_ld = make_rsrc(ld, vb);
            wk.r_lam_st = make_rsrc(st, st != nullptr ? vb : 0u);
            wk.r_msg_ld = make_rsrc(mld, vb);
            wk.r_msg_st = make_rsrc(mst, vb);
            float g = a.gamma[0];
#pragma unroll
            for (int i = 1; i < 8; ++i)
                if (s == i) g = a.gamma[i];
            if (a.mode != kModeIterative)
                wk.template pass<true, 2>(0.0f, true, opt);
            else if ((s & 1) == 0)
                wk.template pass<true, 1>(g, true, opt);
            else
                wk.template pass<false, 1>(g, true, opt);
        }
    }
    if (a.opt != nullptr && wk.ok && sub == 0) a.opt[chain] = opt;
}

template <int G, int LPL, int PF, typename TT, bool FULL, bool HAS_THETA, int MG>
__global__ __launch_bounds__(64) void chain_kernel(SweepArgs a) {
    constexpr int CPW = 64 / G;
    const int lane = threadIdx.x;
    run_chain<G, LPL, PF, TT, FULL, HAS_THETA, MG>(a, blockIdx.x * CPW + lane / G, lane % G);
}

// ------------------------------------------------------------------ launch
constexpr int kPF = 8;

template <int G, int LPL, typename TT, bool HAS_THETA, int MG>
hipError_t launch_mg(const SweepArgs& a, hipStream_t st) {
    constexpr int CPW = 64 / G;
    const unsigned blocks = (unsigned)((a.n_chains + CPW - 1) / CPW);
    if (a.K == G * LPL)
        hipLaunchKernelGGL((chain_kernel<G, LPL, kPF, TT, true, HAS_THETA, MG>), dim3(blocks), dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL((chain_kernel<G, LPL, kPF, TT, false, HAS_THETA, MG>), dim3(blocks), dim3(64), 0, st, a);
    return hipGetLastError();
}

template <int G, int LPL, typename TT, bool HAS_THETA>
hipError_t launch_tt(const SweepArgs& a, hipStream_t st) {
    if (a.mode & kRecordFlag) {
        SweepArgs b = a;
        b.mode = a.mode & ~kRecordFlag;
        return launch_mg<G, LPL, TT, HAS_THETA, kGroupRecord>(b, st);
    }
    if (a.mode == kModeFinal) return launch_mg<G, LPL, TT, HAS_THETA, kGroupFinal>(a, st);
    if (a.mode == kModeOptimum) {
        if constexpr (!HAS_THETA) return launch_mg<G, LPL, TT, false, kGroupOptimum>(a, st);
        return hipErrorInvalidValue;
    }
    return launch_mg<G, LPL, TT, HAS_THETA, kGroupHalfStep>(a, st);
}

template <int G, int LPL>
hipError_t launch_tile(const SweepArgs& a, dm_dtype dt, hipStream_t st) {
    if (a.theta == nullptr) return launch_tt<G, LPL, float, false>(a, st);
    if (dt == DM_F16) return launch_tt<G, LPL, _Float16, true>(a, st);
    return launch_tt<G, LPL, float, true>(a, st);
}

}  // namespace dm
