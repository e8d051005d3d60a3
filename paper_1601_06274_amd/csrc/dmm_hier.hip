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
// Mapping: one chain per wave64 (lane l holds labels l*LPL .. l*LPL+LPL-1), the parts
// processed depth first from a per-wave stack in LDS.  Messages live in two HBM volumes
// (into each node from the left and from the right), normalised by the minimum of the
// message input; the per-node normalisation of the result makes those constants
// irrelevant.  The message is the truncated-linear distance transform: in-lane scans
// and a 64-lane min-plus scan with the linear distance, then the cap min v + wT.  The
// passes prefetch the next nodes' unaries kHierPF nodes ahead.
#include "dmm_hier.h"

namespace dm {
namespace {

constexpr int kHierPF = 4;

__device__ __forceinline__ int hsplit(int s, int e) { return s + (e - s + 1) / 2 - 1; }

template <int LPL, typename TT, bool HAS_THETA>
struct HierChain {
    const TT* th;
    const float* lin;
    float* lout;
    float* msgL;  // message into a node from the left (within its current part)
    float* msgR;  // message into a node from the right
    const float* w;
    long long px0, npx, w0, wn;
    int K, n, lane;
    float Tf, sign;
    bool lv[LPL];

    __device__ HierChain(const SweepArgs& a, float* msg_right, int chain) {
        th = static_cast<const TT*>(a.theta);
        lin = a.lam_in != nullptr ? a.lam_in : a.lam;
        lout = a.lam;
        msgL = a.msg;
        msgR = msg_right;
        w = a.w;
        px0 = (long long)chain * a.chain_px;
        npx = a.node_px;
        w0 = (long long)chain * a.w_chain;
        wn = a.w_node;
        K = a.K;
        n = a.n;
        lane = (int)threadIdx.x;
        Tf = (float)a.T;
        sign = a.sign;
#pragma unroll
        for (int i = 0; i < LPL; ++i) lv[i] = lane * LPL + i < K;
    }

    __device__ __forceinline__ long long el(int node, int i) const {
        return (px0 + (long long)node * npx) * K + lane * LPL + i;
    }
    // unaries of the family at a node: cost - dual (rows) or dual (columns); kBig for
    // labels that do not exist
    __device__ __forceinline__ void load_r(int node, float (&r)[LPL]) const {
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            float x = kBig;
            if (lv[i]) {
                const long long e = el(node, i);
                const float l = lin[e];
                x = HAS_THETA ? (float)th[e] - l : l;
            }
            r[i] = x;
        }
    }
    __device__ __forceinline__ void load_msg(const float* buf, int node, float (&m)[LPL]) const {
#pragma unroll
        for (int i = 0; i < LPL; ++i) m[i] = lv[i] ? buf[el(node, i)] : 0.0f;
    }
    __device__ __forceinline__ void store_msg(float* buf, int node, const float (&m)[LPL]) const {
#pragma unroll
        for (int i = 0; i < LPL; ++i)
            if (lv[i]) buf[el(node, i)] = m[i];
    }
    __device__ __forceinline__ float weight(int edge) const { return w[w0 + (long long)edge * wn]; }

    __device__ __forceinline__ float wave_min(const float (&x)[LPL]) const {
        float m = x[0];
#pragma unroll
        for (int i = 1; i < LPL; ++i) m = fminf(m, x[i]);
        return group_min<64>(m);
    }

    // out = min_a [v(a) + wt * min(|a - b|, T)] - min v over the chain's labels; returns
    // min v.  Labels that do not exist take no part and get 0.
    __device__ float message(const float (&vin)[LPL], float wt, float (&out)[LPL]) const {
        float v[LPL], f[LPL], b[LPL];
#pragma unroll
        for (int i = 0; i < LPL; ++i) v[i] = lv[i] ? vin[i] : kBig;
        const float vmin = wave_min(v);
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
        const float cap = vmin + wt * Tf;
#pragma unroll
        for (int i = 0; i < LPL; ++i) {
            const float fl = fminf(f[i], inl + wt * (float)(i + 1));
            const float br = fminf(b[i], inr + wt * (float)(LPL - i));
            out[i] = lv[i] ? fminf(fminf(fl, br), cap) - vmin : 0.0f;
        }
        return vmin;
    }

    // Message pass over `count` nodes starting at `start` in direction dir (+1: from the
    // left, the message of node k goes into k + 1 and is stored in msgL; -1: into k - 1,
    // stored in msgR), carrying the message in c.  Adds the normalisation constants to opt.
    __device__ void pass(int start, int count, int dir, float (&c)[LPL], double& opt) const {
        if (count <= 0) return;
        float ring[kHierPF][LPL];
#pragma unroll
        for (int q = 0; q < kHierPF; ++q)
            if (q < count) load_r(start + dir * q, ring[q]);
        for (int t0 = 0; t0 < count; t0 += kHierPF) {
#pragma unroll
            for (int q = 0; q < kHierPF; ++q) {
                const int t = t0 + q;
                if (t < count) {
                    const int k = start + dir * t;
                    float v[LPL];
#pragma unroll
                    for (int i = 0; i < LPL; ++i) v[i] = c[i] + ring[q][i];
                    if (t + kHierPF < count) load_r(k + dir * kHierPF, ring[q]);
                    opt += (double)message(v, weight(dir > 0 ? k : k - 1), c);
                    store_msg(dir > 0 ? msgL : msgR, k + dir, c);
                }
            }
        }
    }

    // Handshake over the edge (i, i+1) (Alg. Handshake): reads the messages into i from
    // the left and into i+1 from the right, writes the new boundary messages; returns
    // them in pji (into i) and pij (into i+1).  first: adds the chain optimum's remaining
    // terms to opt (the min-marginal at i of the whole chain).
    __device__ void handshake(int i, float (&pji)[LPL], float (&pij)[LPL], bool first, double& opt) const {
        float r[LPL], m[LPL], t[LPL];
        load_r(i + 1, r);
        load_msg(msgR, i + 1, m);
#pragma unroll
        for (int q = 0; q < LPL; ++q) t[q] = r[q] + m[q];
        const float wt = weight(i);
        const float c0 = message(t, wt, pji);  // from i+1 to i
        load_r(i, r);
        load_msg(msgL, i, m);
#pragma unroll
        for (int q = 0; q < LPL; ++q) m[q] = lv[q] ? m[q] + r[q] + pji[q] : kBig;  // min-marginal at i
        if (first) opt += (double)c0 + (double)wave_min(m);
#pragma unroll
        for (int q = 0; q < LPL; ++q) t[q] = 0.5f * m[q] - pji[q];
        message(t, wt, pij);  // a half of it shared to the right
#pragma unroll
        for (int q = 0; q < LPL; ++q) t[q] = -pij[q];
        message(t, wt, pji);  // what cannot be shared comes back
        store_msg(msgR, i, pji);
        store_msg(msgL, i + 1, pij);
    }

    __device__ void run(int* stk, double* opt_out) {
        double opt = 0.0;
        float c[LPL], pji[LPL], pij[LPL];
        if (n >= 2) {
            const int i0 = hsplit(0, n - 1);
#pragma unroll
            for (int q = 0; q < LPL; ++q) c[q] = 0.0f;
            store_msg(msgL, 0, c);
            pass(0, i0, +1, c, opt);
#pragma unroll
            for (int q = 0; q < LPL; ++q) c[q] = 0.0f;
            store_msg(msgR, n - 1, c);
            pass(n - 1, n - 2 - i0, -1, c, opt);
            int sp = 0;
            stk[0] = 0;
            stk[1] = n - 1;
            sp = 1;
            bool first = true;
            double unused = 0.0;  // the parts' normalisation constants are not the optimum's
            while (sp > 0) {
                --sp;
                const int s = stk[2 * sp], e = stk[2 * sp + 1];
                const int i = hsplit(s, e);
                handshake(i, pji, pij, first, opt);
                first = false;
                if (i > s) {  // left part s..i: messages from the right, from i down to its cut
                    const int i2 = hsplit(s, i);
                    pass(i, i - i2 - 1, -1, pji, unused);
                    stk[2 * sp] = s;
                    stk[2 * sp + 1] = i;
                    ++sp;
                }
                if (e > i + 1) {  // right part i+1..e: messages from the left, up to its cut
                    const int j2 = hsplit(i + 1, e);
                    pass(i + 1, j2 - i - 1, +1, pij, unused);
                    stk[2 * sp] = i + 1;
                    stk[2 * sp + 1] = e;
                    ++sp;
                }
            }
        }
        // the minorant: unary plus both boundary messages, normalised per node
        float ring[kHierPF][LPL];
#pragma unroll
        for (int q = 0; q < kHierPF; ++q)
            if (q < n) load_r(q, ring[q]);
        for (int t0 = 0; t0 < n; t0 += kHierPF) {
#pragma unroll
            for (int q = 0; q < kHierPF; ++q) {
                const int k = t0 + q;
                if (k < n) {
                    float m[LPL], lm[LPL], rm[LPL];
                    load_msg(msgL, k, lm);
                    load_msg(msgR, k, rm);
                    if (n == 1) {
#pragma unroll
                        for (int i = 0; i < LPL; ++i) lm[i] = rm[i] = 0.0f;
                    }
#pragma unroll
                    for (int i = 0; i < LPL; ++i) m[i] = lv[i] ? ring[q][i] + lm[i] + rm[i] : kBig;
                    if (k + kHierPF < n) load_r(k + kHierPF, ring[q]);
                    const float mn = wave_min(m);
                    if (n == 1) opt = (double)mn;
#pragma unroll
                    for (int i = 0; i < LPL; ++i) {
                        if (lv[i]) {
                            const long long e = el(k, i);
                            lout[e] = lin[e] + sign * (m[i] - mn);
                        }
                    }
                }
            }
        }
        if (opt_out != nullptr && lane == 0) *opt_out = opt;
    }
};

template <int LPL, typename TT, bool HAS_THETA>
__global__ __launch_bounds__(64) void hier_chain_kernel(SweepArgs a, float* msg_right) {
    // depth-first stack of parts: at most one more entry per level, levels <= 32
    __shared__ int stk[2 * 64];
    const int chain = blockIdx.x;
    HierChain<LPL, TT, HAS_THETA> hc(a, msg_right, chain);
    hc.run(stk, a.opt != nullptr ? a.opt + chain : nullptr);
}

template <int LPL>
hipError_t launch_lpl(const SweepArgs& a, float* msg_right, dm_dtype dt, hipStream_t st) {
    const dim3 grid((unsigned)a.n_chains), block(64);
    if (a.theta == nullptr)
        hipLaunchKernelGGL((hier_chain_kernel<LPL, float, false>), grid, block, 0, st, a, msg_right);
    else if (dt == DM_F16)
        hipLaunchKernelGGL((hier_chain_kernel<LPL, _Float16, true>), grid, block, 0, st, a, msg_right);
    else
        hipLaunchKernelGGL((hier_chain_kernel<LPL, float, true>), grid, block, 0, st, a, msg_right);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_hier_half_step(const SweepArgs& a, float* msg_right, dm_dtype dt, hipStream_t st) {
    if (a.K <= 64) return launch_lpl<1>(a, msg_right, dt, st);
    if (a.K <= 128) return launch_lpl<2>(a, msg_right, dt, st);
    if (a.K <= 192) return launch_lpl<3>(a, msg_right, dt, st);
    if (a.K <= 256) return launch_lpl<4>(a, msg_right, dt, st);
    return hipErrorInvalidValue;
}

double hier_half_step_bytes(const SweepArgs& a, dm_dtype dt) {
    // per label-node: the level-0 passes read the unaries of every node and write a
    // message; each further level does so for half of the nodes (about log2(n) - 1
    // levels); the final pass reads the unaries and both messages and writes the dual
    const double b = a.theta != nullptr ? (dt == DM_F16 ? 2.0 : 4.0) : 0.0;
    int levels = 0;
    for (int m = a.n; m > 1; m = (m + 1) / 2) ++levels;
    const double step = b + 4.0 + 4.0;  // cost, dual read; message written
    const double per = step * (1.0 + 0.5 * (levels > 1 ? levels - 1 : 0)) + (b + 4.0 + 8.0 + 4.0);
    return per * (double)a.n * a.n_chains * a.K;
}

}  // namespace dm
