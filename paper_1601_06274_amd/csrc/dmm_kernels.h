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
//   * Message for the truncated-linear pairwise term w*min(|a-b|, T): for T <= 3 the
//     window itself (the label and up to two labels on each side, neighbour lanes'
//     values by wave_shr/wave_shl DPP, each candidate rounded once); for larger T the
//     two-pass L1 distance transform (a forward and a backward lower-envelope scan,
//     in-lane, extended across lane boundaries for as many lanes as the truncation
//     radius T-1 needs); then min(., min v + wT).  O(K) work per message for fixed T.
//   * Record mode (the backward's input): the same passes also write, per node and
//     label, which candidate each min took (the selection tape), or keep every pass's
//     messages and duals.
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
    unsigned* tape[9];   // tape mode: selection tape of pass s (s = 0: backward message pass)
    unsigned tape_bytes; // bytes of one tape
    unsigned tape_px;    // tape bytes per pixel of this tile (byte accounting only)
};

// Selection tape: what the adjoint of a pass needs from the forward, one byte per label
// and node: which candidate the label's message took, and the node's two argmins.  Per
// lane and node the bytes of its LPL labels are packed into kTapeWords(LPL) dwords
// (label i in byte i % 4 of word i / 4); a node's lanes are contiguous, so the tape of a
// pass is [pixel][lane][word].  Messages in the direct window form (T <= 3) store in
// bits 0-2 the candidate code (0: the label itself, 1: d = -1, 2: +1, 3: -2, 4: +2,
// 5: the cap) and in bits 3-4 its distance (T for the cap); messages from the scans
// store the bits below.  Bits K and A are common to both.
enum TapeBit : unsigned {
    kTapeFI = 1,    // forward in-lane scan: took the left neighbour + w (not v itself)
    kTapeBI = 2,    // backward in-lane scan: took the right neighbour + w
    kTapeF = 4,     // message entry from the forward scan of this lane
    kTapeB = 8,     // from the backward scan of this lane
    kTapeCL = 16,   // from the left lane's forward-scan end
    kTapeCR = 32,   // from the right lane's backward-scan end (none of F/B/CL/CR: the cap)
    kTapeK = 64,    // argmin of the min-marginal m (lowest label)
    kTapeA = 128,   // argmin of the message input (lowest label)
};
__host__ __device__ constexpr int kTapeWords(int lpl) { return (lpl + 3) / 4; }

// Offset that is outside every buffer (volumes are at most kMaxVolBytes): loads return 0,
// stores are dropped, also for the vector chunks at kOOB + 16*k (no 32-bit wrap).
// Cursor offsets that step below 0 wrap to >= 2^32 - 16 MiB (one node of the largest
// volume), which the size limit also keeps out of range.
constexpr unsigned kOOB = 0xFFFFFF00u;
constexpr unsigned long long kMaxVolBytes = 0xFE000000ull;
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

// NW consecutive dwords at byte offset off: vector buffer loads of up to 4 dwords (the
// chunk offsets go into the instruction's immediate field).
template <int NW>
__device__ __forceinline__ void load_words(__amdgpu_buffer_rsrc_t r, unsigned off, uint32_t* w) {
    if constexpr (NW >= 4) {
        auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
        w[0] = v[0]; w[1] = v[1]; w[2] = v[2]; w[3] = v[3];
        if constexpr (NW > 4) load_words<NW - 4>(r, off + 16u, w + 4);
    } else if constexpr (NW == 3) {
        auto v = __builtin_amdgcn_raw_buffer_load_b96(r, (int)off, 0, 0);
        w[0] = v[0]; w[1] = v[1]; w[2] = v[2];
    } else if constexpr (NW == 2) {
        auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
        w[0] = v[0]; w[1] = v[1];
    } else if constexpr (NW == 1) {
        w[0] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
    }
}

template <int NW>
__device__ __forceinline__ void store_words(__amdgpu_buffer_rsrc_t r, unsigned off, const uint32_t* w) {
    using u4 = __attribute__((ext_vector_type(4))) unsigned;
    using u3 = __attribute__((ext_vector_type(3))) unsigned;
    using u2 = __attribute__((ext_vector_type(2))) unsigned;
    if constexpr (NW >= 4) {
        __builtin_amdgcn_raw_buffer_store_b128((u4){w[0], w[1], w[2], w[3]}, r, (int)off, 0, 0);
        if constexpr (NW > 4) store_words<NW - 4>(r, off + 16u, w + 4);
    } else if constexpr (NW == 3) {
        __builtin_amdgcn_raw_buffer_store_b96((u3){w[0], w[1], w[2]}, r, (int)off, 0, 0);
    } else if constexpr (NW == 2) {
        __builtin_amdgcn_raw_buffer_store_b64((u2){w[0], w[1]}, r, (int)off, 0, 0);
    } else if constexpr (NW == 1) {
        __builtin_amdgcn_raw_buffer_store_b32(w[0], r, (int)off, 0, 0);
    }
}

// Raw words of LPL consecutive elements of type TT: vector buffer loads when the tile is
// full (all labels exist), else one scalar load per label (offsets of missing labels are
// out of range).
template <typename TT, int LPL, bool FULL>
struct RawVec;

template <int LPL, bool FULL>
struct RawVec<float, LPL, FULL> {
    uint32_t w[LPL];
    // off0: byte offset of element 0 (vector form); offs[i]: of element i (scalar form)
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, unsigned off0, const unsigned (&offs)[LPL]) {
        if constexpr (FULL) {
            load_words<LPL>(r, off0, w);
        } else {
#pragma unroll
            for (int i = 0; i < LPL; ++i) w[i] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)offs[i], 0, 0);
        }
    }
    __device__ __forceinline__ float get(int i) const { return __builtin_bit_cast(float, w[i]); }
};

template <int LPL, bool FULL>
struct RawVec<_Float16, LPL, FULL> {
    // pairs of halves per dword when the lane's labels start 4-byte aligned (even LPL)
    static constexpr bool kPacked = FULL && (LPL % 2 == 0);
    static constexpr int kWords = kPacked ? LPL / 2 : LPL;
    uint32_t w[kWords];
    __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t r, unsigned off0, const unsigned (&offs)[LPL]) {
        if constexpr (kPacked) {
            load_words<kWords>(r, off0, w);
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
    if constexpr (FULL) {
        uint32_t w[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) w[i] = __builtin_bit_cast(uint32_t, v[i]);
        store_words<LPL>(r, off0, w);
    } else {
#pragma unroll
        for (int i = 0; i < LPL; ++i) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v[i]), r, (int)offs[i], 0, 0);
    }
}

// Candidate value base + w*k of a source k labels away, as one fused operation (the
// forward, the tape recording and the adjoint's recomputation round it alike whatever
// the compiler contracts elsewhere).
__device__ __forceinline__ float wdist(float w, int k, float base) { return __builtin_fmaf(w, (float)k, base); }

// Tape byte BIT of the group's lowest label whose value equals the group minimum mn,
// or'ed into the owning lane's tape words (label sub*LPL + i: byte i % 4 of word i / 4).
template <int G, int LPL, bool FULL, int NW>
__device__ __forceinline__ void tape_argmin(const float (&x)[LPL], float mn, const bool (&lv)[LPL], int sub,
                                            unsigned bit, uint32_t (&tw)[NW]) {
    int first = LPL;
#pragma unroll
    for (int i = LPL - 1; i >= 0; --i)
        if ((FULL || lv[i]) && x[i] == mn) first = i;
    bool own;
    if constexpr (G == 64) {
        const unsigned long long mask = __builtin_amdgcn_ballot_w64(first < LPL);
        own = first < LPL && (int)__builtin_ctzll(mask) == sub;
    } else {
        const int g = group_min_i<G>(first < LPL ? sub * LPL + first : 0x7fffffff);
        own = first < LPL && g == sub * LPL + first;
    }
    const unsigned b = bit << (8 * (first & 3));
#pragma unroll
    for (int j = 0; j < NW; ++j) tw[j] |= (own && (first >> 2) == j) ? b : 0u;
}

// ------------------------------------------------------------------ chain walker
template <int G, int LPL, int PF, typename TT, bool FULL, bool HAS_THETA>
struct Walker {
    static constexpr int ES = (int)sizeof(TT);
    // One prefetched node: raw cost words, dual, reverse message, edge weight.
    struct Node {
        RawVec<TT, LPL, FULL> th;
        RawVec<float, LPL, FULL> lam;
        RawVec<float, LPL, FULL> rev;
        float w;
    };
    // Byte offsets of the node a load stream is at.
    struct Cursor {
        unsigned th, f, w;
    };

    __amdgpu_buffer_rsrc_t r_theta, r_w, r_mm, r_lab;
    // buffers of the current pass: dual loads / stores, reverse-message loads, message stores
    __amdgpu_buffer_rsrc_t r_lam_ld, r_lam_st, r_msg_ld, r_msg_st;
    unsigned vol_bytes;
    // Offsets (bytes) of this lane's first label at node 0, of the edge (0, 1) and of the
    // node's label slot, and their per-node steps.  Lanes whose chain does not exist sit
    // at kOOB with step 0, so every access of theirs is out of range.
    unsigned th0, f0, w0, lab0, th_step, f_step, w_step, lab_step;
    int sub, n, K, T;
    float sign, inv_n, Tf;
    // 1.0 that the compiler cannot see as a constant: cost - dual as fma(cost, one, -dual)
    // (the same rounding as the subtraction) takes one mixed-precision FMA for FP16 cost
    float one;
    bool ok;          // this group's chain exists
    bool lv[LPL];     // label exists (and the chain exists)
    int dt_steps;     // lanes the distance transform must reach across
    float dl, dr;     // distance-transform lane shifts; lanes without a source keep kBig
    float dl2, dr2;   // direct window: the second label across the lane edge
    bool direct;      // direct window form of the message (T <= 3, reach within one lane)
    // tape mode: store descriptor of the current pass's tape, this lane's tape offset at
    // node 0 and its per-node step
    static constexpr int kTW = kTapeWords(LPL);
    static constexpr int kFar = 1 << 20;  // source distance of a missing neighbour lane
    __amdgpu_buffer_rsrc_t r_tape_st;
    unsigned tp0, tp_step;

    __device__ __forceinline__ Walker(SweepArgs args, int chain, int sub_)
        : sub(sub_), n(args.n), K(args.K), T(args.T), sign(args.sign), inv_n(args.inv_n) {
        ok = chain < args.n_chains;
        Tf = (float)args.T;
        one = args.sign * args.sign;
        const unsigned long long cpx = (unsigned long long)(ok ? chain : 0) * (unsigned long long)args.chain_px;
        const unsigned long long e0 = cpx * (unsigned long long)args.K + (unsigned long long)(sub * LPL);
        const unsigned long long nk = (unsigned long long)args.node_px * (unsigned long long)args.K;
        f0 = ok ? (unsigned)(e0 * 4ull) : kOOB;
        th0 = ok ? (unsigned)(e0 * (unsigned long long)ES) : kOOB;
        f_step = ok ? (unsigned)(nk * 4ull) : 0u;
        th_step = ok ? (unsigned)(nk * (unsigned long long)ES) : 0u;
        w0 = ok ? (unsigned)((unsigned long long)chain * (unsigned long long)args.w_chain * 4ull) : kOOB;
        w_step = ok ? (unsigned)(args.w_node * 4) : 0u;
        const bool lab_lane = ok && sub == 0;
        lab0 = lab_lane ? (unsigned)(cpx * 4ull) : kOOB;
        lab_step = lab_lane ? (unsigned)(args.node_px * 4) : 0u;
        r_theta = make_rsrc(args.theta, HAS_THETA ? args.vol_bytes_theta : 0u);
        vol_bytes = args.vol_bytes_f32;
        r_lam_ld = make_rsrc(args.lam_in != nullptr ? args.lam_in : args.lam, vol_bytes);
        r_lam_st = make_rsrc(args.lam, vol_bytes);
        r_msg_ld = make_rsrc(args.msg, vol_bytes);
        r_msg_st = r_msg_ld;
        r_w = make_rsrc(args.w, args.w_bytes);
        r_mm = make_rsrc(args.minmarg, args.minmarg != nullptr ? vol_bytes : 0u);
        r_lab = make_rsrc(args.labels, args.labels != nullptr ? vol_bytes / (unsigned)args.K : 0u);
#pragma unroll
        for (int i = 0; i < LPL; ++i) lv[i] = FULL ? true : (ok && sub * LPL + i < K);
        const int need = (args.T - 1 + LPL - 1) / LPL;
        dt_steps = need < G - 1 ? need : G - 1;
        direct = args.T <= 3 && args.T - 1 <= LPL;
        const unsigned long long ts = (unsigned long long)(G * kTW * 4);
        tp0 = ok ? (unsigned)(cpx * ts + (unsigned long long)(sub * kTW * 4)) : kOOB;
        tp_step = ok ? (unsigned)((unsigned long long)args.node_px * ts) : 0u;
        r_tape_st = make_rsrc(nullptr, 0u);
    }

    // Per-label byte offsets of an access at `off` (element size E).  A full tile uses
    // `off` alone (vector access); otherwise labels that do not exist are out of range.
    template <int E>
    __device__ __forceinline__ void label_offsets(unsigned off, unsigned (&o)[LPL]) const {
#pragma unroll
        for (int i = 0; i < LPL; ++i) o[i] = (FULL || lv[i]) ? off + (unsigned)(i * E) : kOOB;
    }

    __device__ __forceinline__ Cursor cursor_at(bool fwd) const {
        const unsigned j = fwd ? 0u : (unsigned)(n - 1);
        // edge of node j in a pass: (j, j+1) forward, (j-1, j) backward
        const unsigned e = fwd ? 0u : (unsigned)(n - 2);
        return Cursor{th0 + j * th_step, f0 + j * f_step, w0 + e * w_step};
    }

    // Loads the node at the cursor and moves the cursor one node in direction FWD.
    // Beyond the chain end the loads read other data or zeros; such nodes are never used.
    template <bool FWD, bool WANT_REV>
    __device__ __forceinline__ void load(Node& nd, Cursor& c) const {
        // Issue order: edge weight (used last), reverse message, dual, cost (used first),
        // so one wait for the cost covers the node's other loads.
        unsigned os[LPL];
        nd.w = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r_w, (int)c.w, 0, 0));
        if constexpr (WANT_REV) {
            // message slot of the edge toward the unvisited side: j forward, j-1 backward
            const unsigned ro = FWD ? c.f : c.f - f_step;
            label_offsets<4>(ro, os);
            nd.rev.load(r_msg_ld, ro, os);
        }
        label_offsets<4>(c.f, os);
        nd.lam.load(r_lam_ld, c.f, os);
        if constexpr (HAS_THETA) {
            label_offsets<ES>(c.th, os);
            nd.th.load(r_theta, c.th, os);
        }
        if constexpr (FWD) {
            c.th += th_step; c.f += f_step; c.w += w_step;
        } else {
            c.th -= th_step; c.f -= f_step; c.w -= w_step;
        }
    }

    // Value arriving from the left / right neighbour lane of the group (kBig at the
    // group's first / last lane).  For 64- and 16-lane groups the shifted-in value is
    // kept in a register (`keep`) whose edge lanes are never written.
    __device__ __forceinline__ float from_left_r(float x, float& keep) {
        if constexpr (G == 64) {
            keep = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, keep),
                                                                         __builtin_bit_cast(int, x), kWaveShr1, 0xF,
                                                                         0xF, false));
            return keep;
        } else if constexpr (G == 16) {
            keep = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, keep),
                                                                         __builtin_bit_cast(int, x), kRowShr1, 0xF,
                                                                         0xF, false));
            return keep;
        } else {
            const float c = dpp_fill<kWaveShr1>(x, kBig);
            return sub == 0 ? kBig : c;
        }
    }
    __device__ __forceinline__ float from_right_r(float x, float& keep) {
        if constexpr (G == 64) {
            keep = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, keep),
                                                                         __builtin_bit_cast(int, x), kWaveShl1, 0xF,
                                                                         0xF, false));
            return keep;
        } else if constexpr (G == 16) {
            keep = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, keep),
                                                                         __builtin_bit_cast(int, x), kRowShl1, 0xF,
                                                                         0xF, false));
            return keep;
        } else {
            const float c = dpp_fill<kWaveShl1>(x, kBig);
            return sub == G - 1 ? kBig : c;
        }
    }
    __device__ __forceinline__ float from_left(float x) { return from_left_r(x, dl); }
    __device__ __forceinline__ float from_right(float x) { return from_right_r(x, dr); }

    // Direct window form of the message for T <= 3 (window |d| < T reaching at most one
    // lane across): each label takes the minimum of the window candidates v(a) + w|a-b|,
    // rounded once each, and of the cap vmin + wT.  TP: also records in tape byte bits
    // 0-2 which candidate the minimum took - the first in the order d = 0, -1, +1, -2,
    // +2 that attains it, the cap only when strictly lower (codes 0-4, 5 for the cap) -
    // and in bits 3-4 its distance (T for the cap).
    // T3: T is 3 (both window distances enabled; no per-node selection of the weights).
    template <bool TP, bool T3>
    __device__ __forceinline__ void message_direct(const float (&v)[LPL], float vmin, float wt, float (&out)[LPL],
                                                   uint32_t (&tw)[kTW]) {
        const float w1 = (T3 || T > 1) ? wt : kBig;  // disabled candidates sit above every window value
        const float w2 = T > 2 ? wt + wt : kBig;     // 2w is exact: v + 2w rounds like fma(w, 2, v)
        const float cap = __builtin_fmaf(wt, Tf, vmin);
        const float l1 = from_left_r(v[LPL - 1], dl);
        const float r1 = from_right_r(v[0], dr);
        float l2 = kBig, r2 = kBig;
        if constexpr (LPL >= 2) {
            l2 = from_left_r(v[LPL - 2], dl2);
            r2 = from_right_r(v[1], dr2);
        }
        auto val = [&](int a) -> float {
            return a < 0 ? (a == -1 ? l1 : l2) : (a >= LPL ? (a == LPL ? r1 : r2) : v[a]);
        };
        const unsigned cap_code = 5u | ((unsigned)(T3 ? 3 : T) << 3);
#pragma unroll
        for (int j = 0; j < kTW; ++j) tw[j] = 0u;
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            const bool valid = FULL || lv[i];
            const float s0 = v[i];
            const float cm1 = val(i - 1) + w1, cp1 = val(i + 1) + w1;
            const float cm2 = T3 ? __builtin_fmaf(wt, 2.0f, val(i - 2)) : val(i - 2) + w2;
            const float cp2 = T3 ? __builtin_fmaf(wt, 2.0f, val(i + 2)) : val(i + 2) + w2;
            const float e = fminf(fminf(fminf(s0, cm1), cp1), fminf(cm2, cp2));
            out[i] = valid ? fminf(e, cap) - vmin : 0.0f;
            if constexpr (TP) {
                unsigned x = 4u | (2u << 3);
                x = cm2 == e ? (3u | (2u << 3)) : x;
                x = cp1 == e ? (2u | (1u << 3)) : x;
                x = cm1 == e ? (1u | (1u << 3)) : x;
                x = s0 == e ? 0u : x;
                x = cap < e ? cap_code : x;
                tw[i >> 2] |= (valid ? x : 0u) << (8 * (i & 3));
            }
        }
    }

    // Truncated-linear message of v (normalised by its minimum vmin), into out:
    // min over labels k' of v[k'] + wt*min(|k - k'|, T), minus vmin.  DT1: the
    // distance transform reaches exactly one lane across (dt_steps == 1).
    template <bool DT1>
    __device__ __forceinline__ void message(const float (&v)[LPL], float vmin, float wt, float (&out)[LPL]) {
        float f[LPL], b[LPL];
        f[0] = v[0];
#pragma unroll
        for (int i = 1; i < LPL; ++i) f[i] = fminf(v[i], f[i - 1] + wt);
        b[LPL - 1] = v[LPL - 1];
#pragma unroll
        for (int i = LPL - 2; i >= 0; --i) b[i] = fminf(v[i], b[i + 1] + wt);
        const float cap = __builtin_fmaf(wt, Tf, vmin);
        if constexpr (DT1) {
            const float cl = from_left(f[LPL - 1]);
            const float cr = from_right(b[0]);
#pragma unroll
            for (int i = 0; i < LPL; ++i) {
                const float e = fminf(fminf(f[i], b[i]), cap);
                const float d = fminf(e, fminf(wdist(wt, i + 1, cl), wdist(wt, LPL - i, cr))) - vmin;
                out[i] = (FULL || lv[i]) ? d : 0.0f;
            }
        } else {
            for (int s = 0; s < dt_steps; ++s) {
                const float cl = from_left(f[LPL - 1]);
                const float cr = from_right(b[0]);
#pragma unroll
                for (int i = 0; i < LPL; ++i) {
                    f[i] = fminf(f[i], wdist(wt, i + 1, cl));
                    b[i] = fminf(b[i], wdist(wt, LPL - i, cr));
                }
            }
#pragma unroll
            for (int i = 0; i < LPL; ++i) {
                const float d = fminf(fminf(f[i], b[i]), cap) - vmin;
                out[i] = (FULL || lv[i]) ? d : 0.0f;
            }
        }
    }

    // Integer value of the neighbour lane (kFar at the group's first / last lane).
    __device__ __forceinline__ int from_left_i(int x) const {
        if constexpr (G == 16) return __builtin_amdgcn_update_dpp(kFar, x, kRowShr1, 0xF, 0xF, false);
        const int y = __builtin_amdgcn_update_dpp(kFar, x, kWaveShr1, 0xF, 0xF, false);
        return (G < 64 && sub == 0) ? kFar : y;
    }
    __device__ __forceinline__ int from_right_i(int x) const {
        if constexpr (G == 16) return __builtin_amdgcn_update_dpp(kFar, x, kRowShl1, 0xF, 0xF, false);
        const int y = __builtin_amdgcn_update_dpp(kFar, x, kWaveShl1, 0xF, 0xF, false);
        return (G < 64 && sub == G - 1) ? kFar : y;
    }

    // message<DT1> (same values, same arithmetic) that also records, per label, the
    // operand each min took (tape bits FI, BI, F, B, CL, CR).  The distance transform
    // reaches at most one lane across (dt_steps 0 or 1).  Ties between candidates go to
    // the closer source, then to the left one (lower label); the cap (vmin + wT) wins
    // over a window candidate only if strictly lower, and a source at distance >= T is
    // the cap.
    //
    // Fast form (T >= LPL, so an in-lane source is always within the window): the left
    // candidate wins a tie with the right one when it is the label itself (distance 0),
    // which covers the ties of untouched labels; a wave with any other tie between the
    // left and right candidates takes the general form with per-label source distances.
    template <bool DT1>
    __device__ __forceinline__ void message_tp(const float (&v)[LPL], float vmin, float wt, float (&out)[LPL],
                                               uint32_t (&tw)[kTW]) {
        float f[LPL], b[LPL];
        bool fi[LPL], bi[LPL];
        f[0] = v[0];
        fi[0] = false;
#pragma unroll
        for (int i = 1; i < LPL; ++i) {
            const float c = f[i - 1] + wt;
            f[i] = fminf(v[i], c);
            fi[i] = c < v[i];
        }
        b[LPL - 1] = v[LPL - 1];
        bi[LPL - 1] = false;
#pragma unroll
        for (int i = LPL - 2; i >= 0; --i) {
            const float c = b[i + 1] + wt;
            b[i] = fminf(v[i], c);
            bi[i] = c < v[i];
        }
        // source distances of the lane's chain ends (the neighbour lanes' candidates)
        int df_end = 0, db_beg = 0;
#pragma unroll
        for (int i = 1; i < LPL; ++i) df_end = fi[i] ? df_end + 1 : 0;
#pragma unroll
        for (int i = LPL - 2; i >= 0; --i) db_beg = bi[i] ? db_beg + 1 : 0;
        const float cap = __builtin_fmaf(wt, Tf, vmin);
        float cl = kBig, cr = kBig;
        int dcl = kFar, dcr = kFar;
        if constexpr (DT1) {
            cl = from_left(f[LPL - 1]);
            cr = from_right(b[0]);
            dcl = from_left_i(df_end);
            dcr = from_right_i(db_beg);
        }
        float vl[LPL], vr[LPL];
        bool useF[LPL], useB[LPL];
        bool hard = T < LPL;
#pragma unroll
        for (int j = 0; j < kTW; ++j) tw[j] = 0u;
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            const bool valid = FULL || lv[i];
            vl[i] = wdist(wt, i + 1, cl);
            vr[i] = wdist(wt, LPL - i, cr);
            if constexpr (DT1) {
                const float e = fminf(fminf(f[i], b[i]), cap);
                const float d = fminf(e, fminf(vl[i], vr[i])) - vmin;
                out[i] = valid ? d : 0.0f;
            } else {
                const float d = fminf(fminf(f[i], b[i]), cap) - vmin;
                out[i] = valid ? d : 0.0f;
            }
            useF[i] = !DT1 || f[i] <= vl[i];
            useB[i] = !DT1 || b[i] <= vr[i];
            const float lvv = useF[i] ? f[i] : vl[i];
            const float rvv = useB[i] ? b[i] : vr[i];
            const bool left = lvv <= rvv;
            // a tie is decided here only when the left candidate is the label itself
            hard |= valid & (lvv == rvv) & (fi[i] | !useF[i]);
            const float wv = left ? lvv : rvv;
            const bool near = left ? (useF[i] | (dcl + i + 1 < T)) : (useB[i] | (dcr + LPL - i < T));
            const bool win = (wv <= cap) & near;
            const unsigned t1 = useF[i] ? kTapeF : kTapeCL;
            const unsigned t2 = useB[i] ? kTapeB : kTapeCR;
            const unsigned route = win ? (left ? t1 : t2) : 0u;
            const unsigned x = route | (fi[i] ? kTapeFI : 0u) | (bi[i] ? kTapeBI : 0u);
            tw[i >> 2] |= (valid ? x : 0u) << (8 * (i & 3));
        }
        if (__builtin_amdgcn_ballot_w64(hard) != 0ull) {
            // general form: per-label source distances decide the ties
            int df[LPL], db[LPL];
            df[0] = 0;
#pragma unroll
            for (int i = 1; i < LPL; ++i) df[i] = fi[i] ? df[i - 1] + 1 : 0;
            db[LPL - 1] = 0;
#pragma unroll
            for (int i = LPL - 2; i >= 0; --i) db[i] = bi[i] ? db[i + 1] + 1 : 0;
#pragma unroll
            for (int j = 0; j < kTW; ++j) tw[j] = 0u;
#pragma unroll
            for (int i = 0; i < LPL; ++i) {
                const bool valid = FULL || lv[i];
                const float lvv = useF[i] ? f[i] : vl[i];
                const int ld = useF[i] ? df[i] : dcl + i + 1;
                const float rvv = useB[i] ? b[i] : vr[i];
                const int rd = useB[i] ? db[i] : dcr + LPL - i;
                const bool left = (lvv < rvv) | ((lvv == rvv) & (ld <= rd));
                const float wv = left ? lvv : rvv;
                const int wd = left ? ld : rd;
                const bool win = (wv <= cap) & (wd < T);
                unsigned x = (fi[i] ? kTapeFI : 0u) | (bi[i] ? kTapeBI : 0u);
                x |= (win & left & useF[i]) ? kTapeF : 0u;
                x |= (win & !left & useB[i]) ? kTapeB : 0u;
                x |= (win & left & !useF[i]) ? kTapeCL : 0u;
                x |= (win & !left & !useB[i]) ? kTapeCR : 0u;
                tw[i >> 2] |= (valid ? x : 0u) << (8 * (i & 3));
            }
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
    // MF: message form - 0 scans reaching several lanes, 1 scans reaching one lane (DT1),
    // 2 direct window, 3 direct window with T = 3.
    template <bool FWD, int KIND, int MF, bool TP>
    __device__ __forceinline__ void pass(float gamma, bool store_msg, double& opt) {
        constexpr bool WANT_REV = KIND != 0;
        float carry[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) carry[i] = 0.0f;
        dl = kBig;
        dr = kBig;
        dl2 = kBig;
        dr2 = kBig;
        const __amdgpu_buffer_rsrc_t msg_st = store_msg ? r_msg_st : make_rsrc(nullptr, 0u);
        Cursor lc = cursor_at(FWD);
        unsigned sf = lc.f;                                           // store cursor (dual, messages)
        unsigned sl = lab0 + (FWD ? 0u : (unsigned)(n - 1)) * lab_step;  // label slot
        unsigned stp = tp0 + (FWD ? 0u : (unsigned)(n - 1)) * tp_step;   // tape slot
        Node ring[PF];
        // Issued in slot order (the scheduler may not reorder them): the steady-state loop
        // waits for slot q's loads assuming the later slots' loads were issued after them.
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            load<FWD, WANT_REV>(ring[q], lc);
            __builtin_amdgcn_sched_barrier(0);
        }
        int t0 = 0;
        // Steady state: every node here has a successor in the walking direction.  Node
        // t is processed, then its ring slot is refilled with node t + PF.
        for (; t0 + PF < n; t0 += PF) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                step<FWD, KIND, false, MF, TP>(ring[q], true, carry, gamma, msg_st, opt, sf, sl, stp);
                load<FWD, WANT_REV>(ring[q], lc);
            }
        }
        // Tail: the last 1..PF nodes, already in the ring; the chain's last node has no
        // successor.
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int t = t0 + q;
            if (t < n) step<FWD, KIND, true, MF, TP>(ring[q], t < n - 1, carry, gamma, msg_st, opt, sf, sl, stp);
        }
    }

    // A pass with the distance-transform variant this walker's truncation needs.  TP:
    // also write the pass's selection tape (the host enables it only for dt_steps <= 1).
    template <bool FWD, int KIND, bool TP = false>
    __device__ __forceinline__ void run_pass(float gamma, bool store_msg, double& opt) {
        if (direct) {
            if (T == 3)
                pass<FWD, KIND, 3, TP>(gamma, store_msg, opt);
            else
                pass<FWD, KIND, 2, TP>(gamma, store_msg, opt);
        } else if constexpr (TP) {
            pass<FWD, KIND, 1, TP>(gamma, store_msg, opt);  // the host enables tapes for dt_steps <= 1 only
        } else {
            if (dt_steps == 1)
                pass<FWD, KIND, 1, TP>(gamma, store_msg, opt);
            else
                pass<FWD, KIND, 0, TP>(gamma, store_msg, opt);
        }
    }

    template <bool FWD, int KIND, bool TAIL, int MF, bool TP>
    __device__ __forceinline__ void step(const Node& nd, bool has_next, float (&carry)[LPL], float gamma,
                                         __amdgpu_buffer_rsrc_t msg_st, double& opt, unsigned& sf, unsigned& sl,
                                         unsigned& stp) {
        if constexpr (!TAIL) has_next = true;
        float vmin = 0.0f;
        uint32_t tw[kTW];  // tape: message selections and the two argmins
#pragma unroll
        for (int j = 0; j < kTW; ++j) tw[j] = 0u;
        float r[LPL], lamv[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            lamv[i] = nd.lam.get(i);
            const float x = HAS_THETA ? __builtin_fmaf(nd.th.get(i), one, -lamv[i]) : lamv[i];
            r[i] = (FULL || lv[i]) ? x : kBig;
        }
        float v[LPL];
        if constexpr (KIND == 0) {
#pragma unroll
            for (int i = 0; i < LPL; ++i) v[i] = carry[i] + r[i];
        } else {
            float m[LPL];
#pragma unroll
            for (int i = 0; i < LPL; ++i) {
                v[i] = r[i] + carry[i];
                const float rv = nd.rev.get(i);
                m[i] = v[i] + ((TAIL && !has_next) ? 0.0f : rv);  // no message beyond the chain end
            }
            // The minimum of the message input is reduced together with mmin.  Naive
            // update and final pass: the input is v = r + carry.  Iterative update: the
            // updated r' + carry = rc - gamma*(m - mmin) (rc = r + carry) differs from
            // u = rc - gamma*m by the node constant gamma*mmin, and messages are defined up
            // to constants, so the message is taken of u: it does not wait for mmin.
            float mmin = lane_min(m), bmin;
            if constexpr (KIND == 1) {
#pragma unroll
                for (int i = 0; i < LPL; ++i) v[i] = (FULL || lv[i]) ? __builtin_fmaf(-gamma, m[i], v[i]) : kBig;
            }
            bmin = lane_min(v);
            group_min2<G>(mmin, bmin);
            vmin = bmin;
            if constexpr (TP) {
                // the message selections are or'ed in later: keep the argmin byte apart
                uint32_t tk[kTW];
#pragma unroll
                for (int j = 0; j < kTW; ++j) tk[j] = 0u;
                tape_argmin<G, LPL, FULL, kTW>(m, mmin, lv, sub, kTapeK, tk);
#pragma unroll
                for (int j = 0; j < kTW; ++j) tw[j] = tk[j];
            }
            if constexpr (KIND == 1 || KIND == 2) {
                float nl[LPL];
#pragma unroll
                for (int i = 0; i < LPL; ++i) {
                    float d = (KIND == 1 ? gamma : inv_n) * (m[i] - mmin);
                    d = (FULL || lv[i]) ? d : 0.0f;
                    nl[i] = __builtin_fmaf(sign, d, lamv[i]);
                }
                unsigned os[LPL];
                label_offsets<4>(sf, os);
                store_f32<LPL, FULL>(r_lam_st, sf, os, nl);
            } else {  // KIND == 3: normalized min-marginals and argmin
                float mm[LPL];
                int first = 0x7fffffff;
#pragma unroll
                for (int i = LPL - 1; i >= 0; --i) {
                    mm[i] = m[i] - mmin;
                    if ((FULL || lv[i]) && m[i] == mmin) first = sub * LPL + i;
                }
                int lab = group_min_i<G>(first);
                lab = lab < K ? lab : K - 1;  // defensive: a label always exists for finite costs
                unsigned os[LPL];
                label_offsets<4>(sf, os);
                store_f32<LPL, FULL>(r_mm, sf, os, mm);
                __builtin_amdgcn_raw_buffer_store_b32((uint32_t)lab, r_lab, (int)sl, 0, 0);
                sl = FWD ? sl + lab_step : sl - lab_step;
            }
        }
        if (KIND == 0 || has_next) {
            if constexpr (KIND == 0) vmin = group_min<G>(lane_min(v));
            if constexpr (KIND == 0) opt += (double)vmin;
            if (has_next) {
                if constexpr (MF >= 2) {
                    uint32_t tm[kTW];
                    message_direct<TP, MF == 3>(v, vmin, nd.w, carry, tm);
                    if constexpr (TP) {
#pragma unroll
                        for (int j = 0; j < kTW; ++j) tw[j] |= tm[j];
                        tape_argmin<G, LPL, FULL, kTW>(v, vmin, lv, sub, kTapeA, tw);
                    }
                } else if constexpr (TP) {
                    uint32_t tm[kTW];
                    message_tp<MF == 1>(v, vmin, nd.w, carry, tm);
#pragma unroll
                    for (int j = 0; j < kTW; ++j) tw[j] |= tm[j];
                    tape_argmin<G, LPL, FULL, kTW>(v, vmin, lv, sub, kTapeA, tw);
                } else {
                    message<MF == 1>(v, vmin, nd.w, carry);
                }
                // slot of edge (j, j+1) / (j-1, j); a pass that keeps no messages stores
                // through an empty descriptor (dropped) rather than branching per node
                const unsigned mo = FWD ? sf : sf - f_step;
                unsigned os[LPL];
                label_offsets<4>(mo, os);
                store_f32<LPL, FULL>(msg_st, mo, os, carry);
            }
        }
        if constexpr (TP) {
            store_words<kTW>(r_tape_st, stp, tw);
            stp = FWD ? stp + tp_step : stp - tp_step;
        }
        sf = FWD ? sf + f_step : sf - f_step;
    }
};

// Mode groups compiled as separate kernels (separate symbols in profiles, and each
// kernel holds only the passes it runs): half-step (iterative or naive minorant),
// final row pass, column optimum pass.
// Record: a half-step keeping every pass's messages and intermediate duals.  Tape: a
// half-step writing every pass's selection tape (messages and duals in place, as in the
// plain half-step).
enum ModeGroup : int { kGroupHalfStep = 0, kGroupFinal = 1, kGroupOptimum = 2, kGroupRecord = 3, kGroupTape = 4 };

// All passes of one mode group for the chain walked by `wk` (a Walker, or a walker of
// the same interface); `writer`: this lane stores the chain optimum.
template <int MG, class WK>
__device__ __forceinline__ void run_walker(const SweepArgs& a, WK& wk, int chain, bool writer) {
    double opt = 0.0;
    if constexpr (MG == kGroupHalfStep) {
        // R0 and the first update pass read lam_in; update passes write lam
        const __amdgpu_buffer_rsrc_t lam_out = wk.r_lam_st;
        wk.r_lam_st = make_rsrc(nullptr, 0u);
        wk.template run_pass<false, 0>(0.0f, true, opt);
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
                    wk.template run_pass<true, 1>(g, !last, opt);
                else
                    wk.template run_pass<false, 1>(g, !last, opt);
            }
        } else {
            wk.template run_pass<true, 2>(0.0f, false, opt);
        }
    } else if constexpr (MG == kGroupFinal) {
        wk.template run_pass<false, 0>(0.0f, true, opt);
        wk.template run_pass<true, 3>(0.0f, false, opt);
    } else if constexpr (MG == kGroupOptimum) {
        wk.template run_pass<false, 0>(0.0f, false, opt);
    } else {
        // kGroupRecord: a half-step keeping every pass's messages and duals.  kGroupTape:
        // the same walk with the message and dual buffers aliased by the caller (a.msg for
        // every message volume; one volume for the intermediate duals), each pass writing
        // its selection tape; the last pass's messages are not stored.
        constexpr bool TP = MG == kGroupTape;
        const unsigned vb = wk.vol_bytes;
        wk.r_lam_st = make_rsrc(nullptr, 0u);
        wk.r_msg_st = make_rsrc(a.rec_msg[0], vb);
        if constexpr (TP) wk.r_tape_st = make_rsrc(a.tape[0], a.tape_bytes);
        wk.template run_pass<false, 0, TP>(0.0f, true, opt);
        const int P = a.mode == kModeIterative ? a.n_pass : 1;
        for (int s = 0; s < P; ++s) {
            const float* ld = a.lam_in;
            float* st = nullptr;
            float* mld = a.rec_msg[0];
            float* mst = a.rec_msg[1];
            unsigned* tp = a.tape[1];
#pragma unroll
            for (int i = 1; i < 8; ++i) {
                if (s == i) {
                    ld = a.rec_lam[i];
                    mld = a.rec_msg[i];
                    mst = a.rec_msg[i + 1];
                    tp = a.tape[i + 1];
                }
            }
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (s == i && s + 1 < P) st = a.rec_lam[i + 1];
            // the last pass writes the half-step's output dual unless it would overwrite
            // the input (the backward's recompute from a checkpoint)
            if (s + 1 == P && a.lam != a.lam_in) st = a.lam;
            wk.r_lam_ld = make_rsrc(ld, vb);
            wk.r_lam_st = make_rsrc(st, st != nullptr ? vb : 0u);
            wk.r_msg_ld = make_rsrc(mld, vb);
            wk.r_msg_st = make_rsrc(mst, vb);
            if constexpr (TP) wk.r_tape_st = make_rsrc(tp, a.tape_bytes);
            const bool keep_msg = !TP || s + 1 < P;
            float g = a.gamma[0];
#pragma unroll
            for (int i = 1; i < 8; ++i)
                if (s == i) g = a.gamma[i];
            if (a.mode != kModeIterative)
                wk.template run_pass<true, 2, TP>(0.0f, keep_msg, opt);
            else if ((s & 1) == 0)
                wk.template run_pass<true, 1, TP>(g, keep_msg, opt);
            else
                wk.template run_pass<false, 1, TP>(g, keep_msg, opt);
        }
    }
    if (a.opt != nullptr && wk.ok && writer) a.opt[chain] = opt;
}

// All passes of one mode group for the chain owned by this lane group.
template <int G, int LPL, int PF, typename TT, bool FULL, bool HAS_THETA, int MG>
__device__ __forceinline__ void run_chain(const SweepArgs& a, int chain, int sub) {
    Walker<G, LPL, PF, TT, FULL, HAS_THETA> wk(a, chain, sub);
    run_walker<MG>(a, wk, chain, sub == 0);
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
        if (a.tape[0] != nullptr) return launch_mg<G, LPL, TT, HAS_THETA, kGroupTape>(b, st);
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
