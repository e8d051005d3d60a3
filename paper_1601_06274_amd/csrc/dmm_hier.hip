// dmm_hier.hip - hierarchical-minorant half-step of Dual_MM on gfx950.
//
// Paper App. A.3.3 (Alg. Handshake and the figure of the messages passed): a chain is cut
// at the edge (i, i+1) in its middle; with the message into i from the left part and
// the message into i+1 from the right part, the Handshake over that edge passes half of
// the min-marginal at i to the right (phi_ij, the new message into i+1) and bounces
// back what cannot be passed (phi_ji, the new message into i).  The two parts are then
// separate chains, each cut again in its middle, down to single nodes.  In a part, the
// messages of the level above stay valid on the side whose boundary did not change;
// only the other side's messages are recomputed, from the new boundary message up to
// the part's cut.  Node k's minorant is its unary plus the two Handshake messages it
// received, its minimum subtracted; the family's dual moves by it as for the other
// minorants (rows: lambda += h, columns: lambda -= h).
//
// Mapping: one chain per workgroup of one or four wave64s (lane l holds labels l*LPL ..
// l*LPL+LPL-1), the parts processed level by level; parts of at most a few nodes are
// finished in the wave's LDS, depth first from a per-wave stack.  When the chains are few
// a half-step is two launches: a block of four waves per chain for the levels above a
// split depth D, then a block per subtree at depth D (the parts of a depth are independent
// once the passes above them have written their boundary messages).  Messages live in two HBM volumes
// (into each node from the left and from the right), normalised by the minimum of the
// message input; the per-node normalisation of the result makes those constants
// irrelevant.  The message is the truncated-linear distance transform: for T - 1 <= LPL
// the window minimum over this lane's labels and T - 1 from each neighbouring lane (DPP
// lane shifts), else in-lane scans and a 64-lane min-plus scan with the linear
// distance; then the cap min v + wT.  Passes prefetch the next nodes' unaries kHierPF
// nodes ahead (with the weights of their edges); a Handshake issues its four loads
// together.  Every HBM access is a raw buffer instruction at a 32-bit byte offset (node
// offset = first node's + node * per-node step): vector loads and stores of a lane's
// labels when K fills the tile (FULL), else one access per label with the labels that
// do not exist at an out-of-range offset (reads 0, writes dropped) - no predicates.
// Built once per labels-per-lane count (-DDM_HIER_LPL=1..4: that count's kernels) and
// once with -DDM_HIER_LPL=0 (the dispatch and the byte count), so the many kernel
// instantiations compile in parallel.
#include "dmm_hier.h"

#ifndef DM_HIER_LPL
#error "DM_HIER_LPL must be defined (0: dispatch, 1..4: the kernels of that labels-per-lane count)"
#endif

namespace dm {

// Parts of at most this many nodes are finished in LDS by one wave (App. A.3.3's
// iteration count assumes that short parts sit in fast memory).  A wave stages
// 3 x chunk x 64 x LPL floats: 8 nodes keep it at 18.4 KB for K = 192, so two blocks of
// four waves, or eight blocks of one, share a CU.  (12 nodes for one wave per chain took
// one more level off the HBM passes but left five waves per CU: 7 % slower on the
// subtrees of the 1242 x 375 frame's columns, whose blocks outnumber the CU slots.)
constexpr int hier_chunk(int, int) { return 8; }
// Waves per chain: several when the chains alone leave most of the 1024 SIMDs idle.
inline int hier_waves(int n_chains, int n) { return n_chains <= 512 && n >= 64 ? 4 : 1; }

hipError_t launch_hier_lpl1(const SweepArgs& a, float* msg_right, dm_dtype dt, hipStream_t st);
hipError_t launch_hier_lpl2(const SweepArgs& a, float* msg_right, dm_dtype dt, hipStream_t st);
hipError_t launch_hier_lpl3(const SweepArgs& a, float* msg_right, dm_dtype dt, hipStream_t st);
hipError_t launch_hier_lpl4(const SweepArgs& a, float* msg_right, dm_dtype dt, hipStream_t st);

#if DM_HIER_LPL > 0
namespace {

// LDS pointers typed in the local address space (a generic pointer would make every
// access a flat instruction, which also waits on the vector-memory counter)
using lds_f32 = __attribute__((address_space(3))) float;
using lds_i32 = __attribute__((address_space(3))) int;

constexpr int kHierPF = 8;

__device__ __forceinline__ int hsplit(int s, int e) { return s + (e - s + 1) / 2 - 1; }

// TW: the truncation's reach T - 1 when it is at most LPL (the window of a label then
// spans at most the neighbouring lanes: the message is the window minimum, no scans);
// -1: any T, by scans.
// NW: waves per chain (a workgroup of NW waves).
template <int LPL, typename TT, bool HAS_THETA, int TW, int NW, bool FULL>
struct HierChain {
    static constexpr int kHierChunk = hier_chunk(NW, LPL);
    static constexpr int kLdsFloats = 3 * kHierChunk * 64 * LPL + kHierChunk;  // per wave
    static constexpr int ES = (int)sizeof(TT);
    // buffers: cost, dual read, dual written, messages from the left / right, weights
    __amdgpu_buffer_rsrc_t r_th, r_lin, r_lout, r_mL, r_mR, r_w;
    // byte offsets of this lane's first label at node 0 (FP32 volumes, cost volume) and of
    // edge 0, and their per-node / per-edge steps; lanes without labels sit at kOOB
    unsigned f0, f_step, c0, c_step, w0, w_step;
    int K, n, lane, wv;
    float Tf, sign;
    bool lv[LPL];
    lds_f32* lds;        // this wave's staging of one small part
    lds_i32* stk_small;  // this wave's part stack inside a small part

    __device__ HierChain(const SweepArgs& a, float* msg_right, int chain) {
        K = a.K;
        n = a.n;
        lane = (int)threadIdx.x & 63;
        wv = (int)threadIdx.x >> 6;
        Tf = (float)a.T;
        sign = a.sign;
#pragma unroll
        for (int i = 0; i < LPL; ++i) lv[i] = FULL || lane * LPL + i < K;
        const bool any = FULL || lane * LPL < K;
        const unsigned long long e0 =
            (unsigned long long)chain * (unsigned long long)a.chain_px * (unsigned long long)K + (unsigned)(lane * LPL);
        const unsigned long long nk = (unsigned long long)a.node_px * (unsigned long long)K;
        f0 = any ? (unsigned)(e0 * 4ull) : kOOB;
        f_step = any ? (unsigned)(nk * 4ull) : 0u;
        c0 = any ? (unsigned)(e0 * (unsigned long long)ES) : kOOB;
        c_step = any ? (unsigned)(nk * (unsigned long long)ES) : 0u;
        w0 = (unsigned)((unsigned long long)chain * (unsigned long long)a.w_chain * 4ull);
        w_step = (unsigned)(a.w_node * 4);
        const unsigned vb = a.vol_bytes_f32;
        r_th = make_rsrc(a.theta, HAS_THETA ? a.vol_bytes_theta : 0u);
        r_lin = make_rsrc(a.lam_in != nullptr ? a.lam_in : a.lam, vb);
        r_lout = make_rsrc(a.lam, vb);
        r_mL = make_rsrc(a.msg, vb);
        r_mR = make_rsrc(msg_right, vb);
        r_w = make_rsrc(a.w, a.w_bytes);
    }

    // Per-label byte offsets of the access at `off` (element size E): labels that do not
    // exist are out of range.
    template <int E>
    __device__ __forceinline__ void offs(unsigned off, unsigned (&o)[LPL]) const {
#pragma unroll
        for (int i = 0; i < LPL; ++i) o[i] = lv[i] ? off + (unsigned)(i * E) : kOOB;
    }
    // The raw words of a node's unaries (dual, and cost for rows), as loaded.
    struct RawNode {
        RawVec<float, LPL, FULL> l;
        RawVec<TT, LPL, FULL> c;
    };
    __device__ __forceinline__ void load_raw(int node, RawNode& nd) const {
        unsigned o[LPL];
        const unsigned fo = f0 + (unsigned)node * f_step;
        offs<4>(fo, o);
        nd.l.load(r_lin, fo, o);
        if constexpr (HAS_THETA) {
            const unsigned co = c0 + (unsigned)node * c_step;
            offs<ES>(co, o);
            nd.c.load(r_th, co, o);
        }
    }
    // unaries of the family at a node: cost - dual (rows) or dual (columns); kBig for
    // labels that do not exist
    __device__ __forceinline__ void unary_of(const RawNode& nd, float (&r)[LPL]) const {
#pragma unroll
        for (int i = 0; i < LPL; ++i) r[i] = lv[i] ? (HAS_THETA ? nd.c.get(i) - nd.l.get(i) : nd.l.get(i)) : kBig;
    }
    __device__ __forceinline__ void load_r(int node, float (&r)[LPL]) const {
        RawNode nd;
        load_raw(node, nd);
        unary_of(nd, r);
    }
    // the dual at a node (0 for labels that do not exist)
    __device__ __forceinline__ void load_lam(int node, float (&x)[LPL]) const {
        unsigned o[LPL];
        const unsigned fo = f0 + (unsigned)node * f_step;
        offs<4>(fo, o);
        RawVec<float, LPL, FULL> l;
        l.load(r_lin, fo, o);
#pragma unroll
        for (int i = 0; i < LPL; ++i) x[i] = l.get(i);
    }
    __device__ __forceinline__ void store_lam(int node, const float (&x)[LPL]) const {
        unsigned o[LPL];
        const unsigned fo = f0 + (unsigned)node * f_step;
        offs<4>(fo, o);
        store_f32<LPL, FULL>(r_lout, fo, o, x);
    }
    __device__ __forceinline__ void load_msg(bool left, int node, float (&m)[LPL]) const {
        unsigned o[LPL];
        const unsigned fo = f0 + (unsigned)node * f_step;
        offs<4>(fo, o);
        RawVec<float, LPL, FULL> v;
        v.load(left ? r_mL : r_mR, fo, o);
#pragma unroll
        for (int i = 0; i < LPL; ++i) m[i] = v.get(i);
    }
    __device__ __forceinline__ void store_msg(bool left, int node, const float (&m)[LPL]) const {
        unsigned o[LPL];
        const unsigned fo = f0 + (unsigned)node * f_step;
        offs<4>(fo, o);
        store_f32<LPL, FULL>(left ? r_mL : r_mR, fo, o, m);
    }
    __device__ __forceinline__ float weight(int edge) const {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r_w, (int)(w0 + (unsigned)edge * w_step),
                                                                              0, 0));
    }

    __device__ __forceinline__ float wave_min(const float (&x)[LPL]) const {
        float m = x[0];
#pragma unroll
        for (int i = 1; i < LPL; ++i) m = fminf(m, x[i]);
        return group_min<64>(m);
    }

    // out = min_a [v(a) + wt * min(|a - b|, T)] - min v over the chain's labels; returns
    // min v.  Labels that do not exist take no part and get 0.
    __device__ __forceinline__ float message(const float (&vin)[LPL], float wt, float (&out)[LPL]) const {
        float v[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) v[i] = lv[i] ? vin[i] : kBig;
        const float vmin = wave_min(v);
        const float cap = vmin + wt * Tf;
        if constexpr (TW >= 0) {
            // window |a - b| <= TW: this lane's labels and TW from each neighbouring lane
            float e[LPL + 2 * (TW > 0 ? TW : 0)];
#pragma unroll
            for (int j = 0; j < TW; ++j) e[j] = dpp_fill<kWaveShr1>(v[LPL - TW + j], kBig);
#pragma unroll
            for (int i = 0; i < LPL; ++i) e[TW + i] = v[i];
#pragma unroll
            for (int j = 0; j < TW; ++j) e[TW + LPL + j] = dpp_fill<kWaveShl1>(v[j], kBig);
#pragma unroll
            for (int i = 0; i < LPL; ++i) {
                float m = v[i];
#pragma unroll
                for (int d = 1; d <= TW; ++d) m = fminf(m, fminf(e[TW + i - d], e[TW + i + d]) + wt * (float)d);
                out[i] = lv[i] ? fminf(m, cap) - vmin : 0.0f;
            }
            return vmin;
        }
        float f[LPL], b[LPL];
        f[0] = v[0];
#pragma unroll
        for (int i = 1; i < LPL; ++i) f[i] = fminf(v[i], f[i - 1] + wt);
        b[LPL - 1] = v[LPL - 1];
#pragma unroll
        for (int i = LPL - 2; i >= 0; --i) b[i] = fminf(v[i], b[i + 1] + wt);
        // lane scans with the linear distance: g = best value at this lane's last label
        // over labels at or left of it, h = at its first label over labels at or right
        const float lane_w = wt * (float)LPL;
        float g = f[LPL - 1], h = b[0];
#pragma unroll
        for (int s = 1; s < 64; s <<= 1) {
            const float go = __shfl_up(g, s);
            const float ho = __shfl_down(h, s);
            const float d = lane_w * (float)s;
            if (lane >= s) g = fminf(g, go + d);
            if (lane + s < 64) h = fminf(h, ho + d);
        }
        float inl = __shfl_up(g, 1), inr = __shfl_down(h, 1);
        if (lane == 0) inl = kBig;
        if (lane == 63) inr = kBig;
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            const float fl = fminf(f[i], inl + wt * (float)(i + 1));
            const float br = fminf(b[i], inr + wt * (float)(LPL - i));
            out[i] = lv[i] ? fminf(fminf(fl, br), cap) - vmin : 0.0f;
        }
        return vmin;
    }

    // Where a pass or a Handshake reads unaries and messages: the HBM volumes (Glob) or a
    // part staged in LDS (Lds: unaries, messages from the left, from the right, node
    // index relative to the part's first node).
    struct Glob {
        const HierChain* h;
        // a pass's prefetched node: raw unary words and the weight of its outgoing edge
        struct Node {
            RawNode u;
            float w;
        };
        __device__ __forceinline__ void load_node(int k, int edge, Node& nd) const {
            h->load_raw(k, nd.u);
            nd.w = h->weight(edge);
        }
        __device__ __forceinline__ void unary(const Node& nd, float (&r)[LPL]) const { h->unary_of(nd.u, r); }
        __device__ __forceinline__ void load_r(int k, float (&r)[LPL]) const { h->load_r(k, r); }
        __device__ __forceinline__ void load_m(bool left, int k, float (&m)[LPL]) const { h->load_msg(left, k, m); }
        __device__ __forceinline__ void store_m(bool left, int k, const float (&m)[LPL]) const {
            h->store_msg(left, k, m);
        }
        __device__ __forceinline__ float w(int edge) const { return h->weight(edge); }
    };
    struct Lds {
        const HierChain* h;
        lds_f32* base;  // [3][kHierChunk][64 * LPL] then the part's kHierChunk - 1 edge weights
        int s;
        __device__ __forceinline__ lds_f32* at(int arr, int k) const {
            return base + ((size_t)arr * kHierChunk + (k - s)) * (64 * LPL) + h->lane * LPL;
        }
        struct Node {
            float r[LPL];
            float w;
        };
        __device__ __forceinline__ void load_node(int k, int edge, Node& nd) const {
            load_r(k, nd.r);
            nd.w = w(edge);
        }
        __device__ __forceinline__ void unary(const Node& nd, float (&r)[LPL]) const {
#pragma unroll
            for (int i = 0; i < LPL; ++i) r[i] = nd.r[i];
        }
        __device__ __forceinline__ void load_r(int k, float (&r)[LPL]) const {
            const lds_f32* p = at(0, k);
#pragma unroll
            for (int i = 0; i < LPL; ++i) r[i] = h->lv[i] ? p[i] : kBig;
        }
        __device__ __forceinline__ void load_m(bool left, int k, float (&m)[LPL]) const {
            const lds_f32* p = at(left ? 1 : 2, k);
#pragma unroll
            for (int i = 0; i < LPL; ++i) m[i] = p[i];
        }
        __device__ __forceinline__ void store_m(bool left, int k, const float (&m)[LPL]) const {
            lds_f32* p = at(left ? 1 : 2, k);
#pragma unroll
            for (int i = 0; i < LPL; ++i) p[i] = m[i];
        }
        __device__ __forceinline__ float w(int edge) const {
            return base[(size_t)3 * kHierChunk * (64 * LPL) + (edge - s)];
        }
    };

    // Message pass over `count` nodes starting at `start` in direction dir (+1: from the
    // left, the message of node k goes into k + 1; -1: into k - 1), carrying the message
    // in c.  Adds the normalisation constants to opt.
    template <class M>
    __device__ __forceinline__ void pass(const M& mem, int start, int count, int dir, float (&c)[LPL], double& opt) const {
        if (count <= 0) return;
        // ring of the next nodes' raw unary words and the weights of their outgoing edges,
        // as loaded (the arithmetic at use); a slot is refilled only after its node's
        // message, so no slot is live across its refill and the loop keeps each slot in
        // the same registers (no copies, no drain of the loads in flight).  The loads go
        // unconditionally to a node of the pass (clamped to its last), so the full blocks
        // have no branches and the waits stay exact.
        typename M::Node ring[kHierPF];
        const int eo = dir > 0 ? 0 : -1;  // edge of node k in the walking direction: k + eo
        auto node_of = [&](int t) { return start + dir * (t < count ? t : count - 1); };
        // issued in slot order: the loop waits for slot q assuming later slots came after
#pragma unroll
        for (int q = 0; q < kHierPF; ++q) {
            const int k = node_of(q);
            mem.load_node(k, k + eo, ring[q]);
            __builtin_amdgcn_sched_barrier(0);
        }
        int t0 = 0;
        for (; t0 + kHierPF <= count; t0 += kHierPF) {
#pragma unroll
            for (int q = 0; q < kHierPF; ++q) {
                const int t = t0 + q;
                const int k = start + dir * t;
                float r[LPL], v[LPL];
                mem.unary(ring[q], r);
#pragma unroll
                for (int i = 0; i < LPL; ++i) v[i] = c[i] + r[i];
                opt += (double)message(v, ring[q].w, c);
                mem.store_m(dir > 0, k + dir, c);
                const int kn = node_of(t + kHierPF);
                mem.load_node(kn, kn + eo, ring[q]);
                // one node per scheduling region: a later slot's conversions hoisted
                // above this node would wait for its just-issued loads
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int q = 0; q < kHierPF; ++q) {
            const int t = t0 + q;
            if (t < count) {
                const int k = start + dir * t;
                float r[LPL], v[LPL];
                mem.unary(ring[q], r);
#pragma unroll
                for (int i = 0; i < LPL; ++i) v[i] = c[i] + r[i];
                opt += (double)message(v, ring[q].w, c);
                mem.store_m(dir > 0, k + dir, c);
            }
        }
    }

    // Handshake over the edge (i, i+1) (Alg. Handshake): reads the messages into i from
    // the left and into i+1 from the right, writes the new boundary messages; returns
    // them in pji (into i) and pij (into i+1).  first: adds the chain optimum's remaining
    // terms to opt (the min-marginal at i of the whole chain).
    template <class M>
    __device__ __forceinline__ void handshake(const M& mem, int i, float (&pji)[LPL], float (&pij)[LPL], bool first,
                                              double& opt) const {
        HsIn in;
        hs_load(mem, i, in);  // the four loads issued together
        hs_compute(mem, i, in, pji, pij, first, opt);
    }
    // A Handshake's inputs: the unaries of i and i+1, the messages into them, the weight.
    struct HsIn {
        float r1[LPL], mr[LPL], r0[LPL], ml[LPL], wt;
    };
    template <class M>
    __device__ __forceinline__ void hs_load(const M& mem, int i, HsIn& in) const {
        mem.load_r(i + 1, in.r1);
        mem.load_m(false, i + 1, in.mr);
        mem.load_r(i, in.r0);
        mem.load_m(true, i, in.ml);
        in.wt = mem.w(i);
    }
    template <class M>
    __device__ __forceinline__ void hs_compute(const M& mem, int i, const HsIn& in, float (&pji)[LPL],
                                               float (&pij)[LPL], bool first, double& opt) const {
        float m[LPL], t[LPL];
#pragma unroll
        for (int q = 0; q < LPL; ++q) t[q] = in.r1[q] + in.mr[q];
        const float c0 = message(t, in.wt, pji);  // from i+1 to i
#pragma unroll
        for (int q = 0; q < LPL; ++q) m[q] = lv[q] ? in.ml[q] + in.r0[q] + pji[q] : kBig;  // min-marginal at i
        if (first) opt += (double)c0 + (double)wave_min(m);
#pragma unroll
        for (int q = 0; q < LPL; ++q) t[q] = 0.5f * m[q] - pji[q];
        message(t, in.wt, pij);  // a half of it shared to the right
#pragma unroll
        for (int q = 0; q < LPL; ++q) t[q] = -pij[q];
        message(t, in.wt, pji);  // what cannot be shared comes back
        mem.store_m(false, i, pji);
        mem.store_m(true, i + 1, pij);
    }

    // Cuts the part s..e (length >= 2; on entry the messages from the left are valid on
    // s..cut and those from the right on cut+1..e) and its parts depth first, down to
    // single nodes.
    template <class M>
    __device__ __forceinline__ void split_parts(const M& mem, lds_i32* stk, int s0, int e0, bool& first,
                                                double& opt) const {
        double unused = 0.0;  // the parts' normalisation constants are not the optimum's
        float pji[LPL], pij[LPL];
        int sp = 1;
        stk[0] = s0;
        stk[1] = e0;
        while (sp > 0) {
            --sp;
            const int s = stk[2 * sp], e = stk[2 * sp + 1];
            const int i = hsplit(s, e);
            handshake(mem, i, pji, pij, first, opt);
            first = false;
            if (i > s) {  // left part s..i: messages from the right, from i down to its cut
                const int i2 = hsplit(s, i);
                pass(mem, i, i - i2 - 1, -1, pji, unused);
                stk[2 * sp] = s;
                stk[2 * sp + 1] = i;
                ++sp;
            }
            if (e > i + 1) {  // right part i+1..e: messages from the left, up to its cut
                const int j2 = hsplit(i + 1, e);
                pass(mem, i + 1, j2 - i - 1, +1, pij, unused);
                stk[2 * sp] = i + 1;
                stk[2 * sp + 1] = e;
                ++sp;
            }
        }
    }

    // A part of at most kHierChunk nodes (length >= 2): its unaries and valid messages
    // are staged in LDS, its parts are cut down to single nodes there, and the minorant
    // of its nodes moves the dual.  In three steps, so that the next part's loads are in
    // flight while this part is computed: small_load issues every load of a part
    // (nodes past its end read its last node again, edges past it its last edge: no
    // branches, the waits stay exact); small_stage writes them to LDS and keeps the
    // duals; small_finish cuts the part in LDS and moves the dual.
    // The next part's loads in flight during the current part pay off with several waves
    // per chain (the row family); with one wave per chain the extra registers and code
    // cost more than the latency they hide (measured), so those load and compute in turn.
    static constexpr bool kPrefetchSmall = NW > 1;
    struct SmallIn {
        RawNode u[kHierChunk];         // unaries as loaded (their dual words are the dual)
        float mg[kHierChunk][LPL];     // the valid message of each node
        float ew[kHierChunk - 1];      // edge weights
    };
    __device__ __forceinline__ void small_load(int s, int e, SmallIn& in) const {
        const int m = e - s + 1;
        const int cut = hsplit(s, e);
#pragma unroll
        for (int j = 0; j < kHierChunk; ++j) load_raw(s + (j < m ? j : m - 1), in.u[j]);
#pragma unroll
        for (int j = 0; j < kHierChunk - 1; ++j) in.ew[j] = weight(s + (j < m - 1 ? j : m - 2));
#pragma unroll
        for (int j = 0; j < kHierChunk; ++j) {
            const int k = s + (j < m ? j : m - 1);
            load_msg(k <= cut, k, in.mg[j]);
        }
    }
    __device__ __forceinline__ void small_stage(int s, int e, const SmallIn& in, float (&lam)[kHierChunk][LPL]) const {
        const int m = e - s + 1;
        const int cut = hsplit(s, e);
        const Lds L{this, lds, s};
#pragma unroll
        for (int j = 0; j < kHierChunk; ++j) {
#pragma unroll
            for (int i = 0; i < LPL; ++i) lam[j][i] = in.u[j].l.get(i);
            if (j < m) {
                float r[LPL];
                unary_of(in.u[j], r);
                lds_f32* p = L.at(0, s + j);
#pragma unroll
                for (int i = 0; i < LPL; ++i) p[i] = r[i];
                L.store_m(s + j <= cut, s + j, in.mg[j]);
            }
        }
        lds_f32* wl = lds + (size_t)3 * kHierChunk * (64 * LPL);
        if (lane == 0) {
#pragma unroll
            for (int j = 0; j < kHierChunk - 1; ++j)
                if (j < m - 1) wl[j] = in.ew[j];
        }
        wave_lds_sync();
    }
    // fill: 0, or the side of its parent this part is (-1 left, +1 right) when the parent
    // left out its passes (every child at most kHierChunk long): the part then computes
    // the messages its parent's pass would have written, from the one valid message at
    // its outer end (the Handshake's) to its own cut, in LDS with the same pass.
    __device__ __forceinline__ void small_finish(int s, int e, const float (&lam)[kHierChunk][LPL], bool first,
                                                 double& opt, int fill) const {
        const int m = e - s + 1;
        const Lds L{this, lds, s};
        if (fill != 0) {
            double unused = 0.0;
            float c[LPL];
            const int cut = hsplit(s, e);
            if (fill < 0) {  // left child: messages from the right, from e down to the cut
                L.load_m(false, e, c);
                pass(L, e, e - cut - 1, -1, c, unused);
            } else {  // right child: messages from the left, from s up to the cut
                L.load_m(true, s, c);
                pass(L, s, cut - s, +1, c, unused);
            }
            wave_lds_sync();
        }
        bool f = first;
        split_parts(L, stk_small, s, e, f, opt);
        wave_lds_sync();
#pragma unroll
        for (int j = 0; j < kHierChunk; ++j) {
            if (j < m) {
                float r[LPL], a[LPL], b[LPL], mm[LPL];
                L.load_r(s + j, r);
                L.load_m(true, s + j, a);
                L.load_m(false, s + j, b);
#pragma unroll
                for (int i = 0; i < LPL; ++i) mm[i] = lv[i] ? r[i] + a[i] + b[i] : kBig;
                const float mn = wave_min(mm);
                float out[LPL];
#pragma unroll
                for (int i = 0; i < LPL; ++i) out[i] = lam[j][i] + sign * (mm[i] - mn);
                store_lam(s + j, out);
            }
        }
        wave_lds_sync();  // the next part reuses the LDS
    }

    // The part at `depth` with index p (its path from the whole chain: bit depth-1-d of
    // p chooses the right part at depth d); false if an ancestor was at most
    // kHierChunk long (finished in LDS, not cut further).  A cut leaves parts of at most
    // the parent's length, so the parent is the shortest ancestor and the only one to
    // test; the walk itself has no branches (scalar selects).
    __device__ __forceinline__ bool part_at(int depth, int p, int& s, int& e) const {
        int plen;
        return part_at(depth, p, s, e, plen);
    }
    // ... and the parent's length (0x7fffffff at depth 0)
    __device__ __forceinline__ bool part_at(int depth, int p, int& s, int& e, int& plen) const {
        s = 0;
        e = n - 1;
        plen = 0x7fffffff;  // the parent's length (depth 0: no parent, the whole chain exists)
        for (int d = depth - 1; d >= 0; --d) {
            plen = e - s + 1;
            const int i = hsplit(s, e);
            const bool right = (p >> d) & 1;
            s = right ? i + 1 : s;
            e = right ? e : i;
        }
        return plen > kHierChunk;
    }

    // Level order: at each depth, first the cuts of the parts (Handshakes; parts of at
    // most kHierChunk nodes are finished in LDS instead), then the messages of their two
    // parts up to the parts' own cuts, the work spread over the workgroup's waves with a
    // barrier after each step.  The whole chain's optimum is measured by the level-0
    // passes (waves 0 and 1) and the first cut (wave 0).
    // d_root, p_root: the subtree of part p_root at depth d_root (0, 0: the whole chain,
    // with the level-0 passes); the parts of one depth are independent once the passes of
    // the depth above have written their boundary messages, so the subtrees of a depth
    // are separate work.  d_stop: the depth whose cuts are left out (with those below).
    __device__ __forceinline__ void run(double* opt_out, double* opt_share, int d_root, int p_root, int d_stop) {
        double opt = 0.0;
        if (n >= 2) {
            const Glob G{this};
            float c[LPL];
            if (d_root == 0) {
                const int i0 = hsplit(0, n - 1);
                if (wv == 0) {
#pragma unroll
                    for (int q = 0; q < LPL; ++q) c[q] = 0.0f;
                    store_msg(true, 0, c);
                    pass(G, 0, i0, +1, c, opt);
                }
                if (wv == (NW > 1 ? 1 : 0)) {
#pragma unroll
                    for (int q = 0; q < LPL; ++q) c[q] = 0.0f;
                    store_msg(false, n - 1, c);
                    pass(G, n - 1, n - 2 - i0, -1, c, opt);
                }
                __syncthreads();
            }
            int maxlen = n;  // longest part at this depth
            for (int d = 0; d < d_root; ++d) maxlen = (maxlen + 1) / 2;
            for (int depth = d_root; depth < d_stop; ++depth) {
                const int np = 1 << (depth - d_root);  // the subtree's parts at this depth
                const int pb = p_root << (depth - d_root);  // the index of its first
                // this wave's cuts, the inputs of the next one loaded while the current
                // one is computed
                HsIn nxt;
                int nxt_i = -1;
                auto next_big = [&](int from) -> int {  // the next part of this wave longer than the chunk
                    for (int p = from; p < np; p += NW) {
                        int s1, e1;
                        if (part_at(depth, pb + p, s1, e1) && e1 - s1 + 1 > kHierChunk) return hsplit(s1, e1);
                    }
                    return -1;
                };
                if (maxlen > kHierChunk) {
                    nxt_i = next_big(wv);
                    if (nxt_i >= 0) hs_load(G, nxt_i, nxt);
                }
                // this wave's parts of at most the chunk, the next one's loads issued
                // while the current one is computed
                auto next_small = [&](int from, int& s1, int& e1) -> bool {
                    for (int p = from; p < np; p += NW)
                        if (part_at(depth, pb + p, s1, e1) && e1 - s1 + 1 <= kHierChunk) return true;
                    return false;
                };
                SmallIn sm;
                int sm_s, sm_e;
                if constexpr (kPrefetchSmall)
                    if (next_small(wv, sm_s, sm_e)) small_load(sm_s, sm_e, sm);
                for (int p = wv; p < np; p += NW) {
                    int s0, e0, plen;
                    if (!part_at(depth, pb + p, s0, e0, plen)) continue;
                    if (e0 - s0 + 1 <= kHierChunk) {
                        // with the prefetch, sm holds this part's loads (parts are visited in order)
                        if constexpr (!kPrefetchSmall) small_load(s0, e0, sm);
                        float lam[kHierChunk][LPL];
                        small_stage(s0, e0, sm, lam);
                        if constexpr (kPrefetchSmall)
                            if (next_small(p + NW, sm_s, sm_e)) small_load(sm_s, sm_e, sm);
                        const int fill = plen <= 2 * kHierChunk ? (((pb + p) & 1) ? +1 : -1) : 0;
                        small_finish(s0, e0, lam, depth == 0, opt, fill);
                    } else {
                        const int i = nxt_i;  // == hsplit(s0, e0): parts are visited in order
                        const HsIn cur = nxt;
                        nxt_i = next_big(p + NW);
                        if (nxt_i >= 0) hs_load(G, nxt_i, nxt);
                        float pji[LPL], pij[LPL];
                        hs_compute(G, i, cur, pji, pij, depth == 0, opt);
                    }
                }
                __syncthreads();
                if (maxlen <= kHierChunk) break;
                // item 2p: the left part's messages from the right, from the cut down to
                // its own cut; 2p + 1: the right part's from the left, up to its cut.  A
                // part of at most 2 kHierChunk nodes leaves them to its two parts (both
                // finished in LDS, which recompute them there: no HBM round trip for a
                // pass of a few nodes)
                for (int q = wv; q < 2 * np; q += NW) {
                    int s0, e0;
                    if (!part_at(depth, pb + (q >> 1), s0, e0) || e0 - s0 + 1 <= 2 * kHierChunk) continue;
                    const int i = hsplit(s0, e0);
                    double unused = 0.0;  // the parts' normalisation constants are not the optimum's
                    if ((q & 1) == 0) {
                        if (i > s0) {
                            load_msg(false, i, c);
                            pass(G, i, i - hsplit(s0, i) - 1, -1, c, unused);
                        }
                    } else if (e0 > i + 1) {
                        load_msg(true, i + 1, c);
                        pass(G, i + 1, hsplit(i + 1, e0) - i - 1, +1, c, unused);
                    }
                }
                __syncthreads();
                maxlen = (maxlen + 1) / 2;
            }
        } else if (wv == 0) {
            // one node: its minorant is its unary
            float r[LPL], l0[LPL], out[LPL];
            load_r(0, r);
            load_lam(0, l0);
            const float mn = wave_min(r);
            opt = (double)mn;
#pragma unroll
            for (int i = 0; i < LPL; ++i) out[i] = l0[i] + sign * (r[i] - mn);
            store_lam(0, out);
        }
        if constexpr (NW > 1) {
            if (wv == 1 && lane == 0) *opt_share = opt;
            __syncthreads();
            if (wv == 0) opt += *opt_share;
        }
        if (opt_out != nullptr && wv == 0 && lane == 0) *opt_out = opt;
    }
};

// split: 0, a block per chain; else the depth D at which the chains' work is split:
// split > 0 launches a block per chain for the levels above D (no LDS parts there),
// split < 0 a block per subtree at depth D (2^D blocks per chain, chain-major).
template <int LPL, typename TT, bool HAS_THETA, int TW, int NW, bool FULL>
__global__ __launch_bounds__(64 * NW) void hier_chain_kernel(SweepArgs a, float* msg_right, int split) {
    using HC = HierChain<LPL, TT, HAS_THETA, TW, NW, FULL>;
    __shared__ int stk[NW][2 * 64];  // each wave's part stack (depth <= 32)
    __shared__ double opt_share[1];
    extern __shared__ float part[];  // per wave: [3][chunk][64 * LPL], then chunk weights
    const int d = split < 0 ? -split : 0;
    const int chain = (int)(blockIdx.x >> d);
    HC hc(a, msg_right, chain);
    hc.lds = (lds_f32*)(part + (size_t)hc.wv * HC::kLdsFloats);
    hc.stk_small = (lds_i32*)stk[hc.wv];
    hc.run(a.opt != nullptr && split >= 0 ? a.opt + chain : nullptr, opt_share, d, (int)(blockIdx.x & ((1u << d) - 1u)),
           split > 0 ? split : 0x7fff);
}

// Depth at which the chains' work is split into separate blocks, 0 for none.  A block
// per chain leaves the CUs unevenly loaded when the chains are few (the 375 rows of a
// 1242 x 375 frame in blocks of four waves: some CUs hold one chain, some two, and the
// kernel waits for the latter); the subtrees at depth D are 2^D times as many blocks of
// equal work.  D is the shallowest depth giving at least 8192 waves (about eight per
// SIMD, over several rounds of resident blocks), at most 4, and only while every part
// at depth D is longer than the LDS part (n >= (chunk + 1) 2^D: a part at depth d has at
// least floor(n / 2^d) nodes), so the block per chain meets no LDS part and runs the
// passes of every depth above D (its parts are longer than twice the LDS part).
inline int hier_split_depth(int n_chains, int nw, int chunk, int n) {
    int D = 0;
    while (D < 4 && (long long)n_chains * nw << D < 8192 && n >= ((chunk + 1) << (D + 1))) ++D;
    return D;
}

template <int LPL, int TW, int NW, bool FULL>
void launch_blocks(const SweepArgs& a, float* msg_right, dm_dtype dt, hipStream_t st, int split, unsigned blocks,
                   size_t shm) {
    const dim3 grid(blocks), block(64 * NW);
    if (a.theta == nullptr)
        hipLaunchKernelGGL((hier_chain_kernel<LPL, float, false, TW, NW, FULL>), grid, block, shm, st, a, msg_right,
                           split);
    else if (dt == DM_F16)
        hipLaunchKernelGGL((hier_chain_kernel<LPL, _Float16, true, TW, NW, FULL>), grid, block, shm, st, a, msg_right,
                           split);
    else
        hipLaunchKernelGGL((hier_chain_kernel<LPL, float, true, TW, NW, FULL>), grid, block, shm, st, a, msg_right,
                           split);
}

template <int LPL, int TW, int NW, bool FULL>
hipError_t launch_full(const SweepArgs& a, float* msg_right, dm_dtype dt, hipStream_t st) {
    const size_t lds = (size_t)NW * HierChain<LPL, float, false, TW, NW, FULL>::kLdsFloats * sizeof(float);
    const int D = hier_split_depth(a.n_chains, NW, hier_chunk(NW, LPL), a.n);
    if (D == 0) {
        launch_blocks<LPL, TW, NW, FULL>(a, msg_right, dt, st, 0, (unsigned)a.n_chains, lds);
    } else {
        // the levels above D: four waves per chain whatever NW (the two level-0 passes side
        // by side, up to four passes per depth), no LDS parts, so no dynamic LDS
        launch_blocks<LPL, TW, 4, FULL>(a, msg_right, dt, st, D, (unsigned)a.n_chains, 0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        launch_blocks<LPL, TW, NW, FULL>(a, msg_right, dt, st, -D, (unsigned)a.n_chains << D, lds);
    }
    return hipGetLastError();
}

template <int LPL, int TW, int NW>
hipError_t launch_nw(const SweepArgs& a, float* msg_right, dm_dtype dt, hipStream_t st) {
    if (a.K == 64 * LPL) return launch_full<LPL, TW, NW, true>(a, msg_right, dt, st);
    return launch_full<LPL, TW, NW, false>(a, msg_right, dt, st);
}

template <int LPL, int TW>
hipError_t launch_tw(const SweepArgs& a, float* msg_right, dm_dtype dt, hipStream_t st) {
    if (hier_waves(a.n_chains, a.n) == 4) return launch_nw<LPL, TW, 4>(a, msg_right, dt, st);
    return launch_nw<LPL, TW, 1>(a, msg_right, dt, st);
}

template <int LPL>
hipError_t launch_lpl(const SweepArgs& a, float* msg_right, dm_dtype dt, hipStream_t st) {
    const int tw = a.T - 1;
    if (tw == 0) return launch_tw<LPL, 0>(a, msg_right, dt, st);
    if (tw == 1) return launch_tw<LPL, 1>(a, msg_right, dt, st);
    if constexpr (LPL >= 2)
        if (tw == 2) return launch_tw<LPL, 2>(a, msg_right, dt, st);
    if constexpr (LPL >= 3)
        if (tw == 3) return launch_tw<LPL, 3>(a, msg_right, dt, st);
    return launch_tw<LPL, -1>(a, msg_right, dt, st);
}

}  // namespace

#define DM_HIER_FN2(n) launch_hier_lpl##n
#define DM_HIER_FN(n) DM_HIER_FN2(n)
hipError_t DM_HIER_FN(DM_HIER_LPL)(const SweepArgs& a, float* msg_right, dm_dtype dt, hipStream_t st) {
    return launch_lpl<DM_HIER_LPL>(a, msg_right, dt, st);
}

#else  // DM_HIER_LPL == 0

hipError_t launch_hier_half_step(const SweepArgs& a, float* msg_right, dm_dtype dt, hipStream_t st) {
    if (a.K <= 64) return launch_hier_lpl1(a, msg_right, dt, st);
    if (a.K <= 128) return launch_hier_lpl2(a, msg_right, dt, st);
    if (a.K <= 192) return launch_hier_lpl3(a, msg_right, dt, st);
    if (a.K <= 256) return launch_hier_lpl4(a, msg_right, dt, st);
    return hipErrorInvalidValue;
}

double hier_half_step_bytes(const SweepArgs& a, dm_dtype dt) {
    // per label-node, HBM only: the two level-0 passes read every node's unaries (cost
    // and dual for rows, the dual for columns) and write its message; at every depth whose
    // parts are longer than twice the LDS part, the passes after the cuts do so for half
    // of the nodes (shorter parts leave those passes to their parts, in LDS); a part of at
    // most the LDS part's length is read once (unaries, one message) into LDS and its
    // nodes' duals written.  The Handshakes' own loads and stores (two nodes per cut, about
    // one cut per LDS part) are left out.
    const double b = a.theta != nullptr ? (dt == DM_F16 ? 2.0 : 4.0) : 0.0;
    const int lpl = a.K <= 64 ? 1 : a.K <= 128 ? 2 : a.K <= 192 ? 3 : 4;
    const int chunk = hier_chunk(hier_waves(a.n_chains, a.n), lpl);
    int deep = 0;  // depths whose parts are longer than twice the LDS part
    for (int m = a.n; m > 2 * chunk; m = (m + 1) / 2) ++deep;
    const double step = b + 4.0 + 4.0;                 // unaries read, message written
    const double per = step * (1.0 + 0.5 * deep) + (b + 4.0 + 4.0) + 4.0;  // + LDS part in, dual out
    return per * (double)a.n * a.n_chains * a.K;
}

#endif  // DM_HIER_LPL

}  // namespace dm
