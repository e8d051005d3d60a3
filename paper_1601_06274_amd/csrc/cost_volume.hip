// cost_volume.hip - truncated windowed SAD cost volume and contrast edge weights.
//
// Paper: the data term sampled at every label forms the unary cost vectors
// (Sec. 2.2 "Stereo"), precomputed for all labels before the discrete stage
// (Table tab:timing "Cost Vol.").  The paper's own data term is Census + Hamming
// (Sec. 3.1); this kernel provides a truncated windowed SAD in the same role.
// Edge strengths are image dependent, lower across image edges (Sec. 2.1).
//
// Layout: the volume is label-major ([y][x][d], d fastest).  A block owns one image row
// and TX consecutive pixels; its threads are the labels (blockDim = K rounded up to a
// wave), so each pixel's K costs are one contiguous, coalesced write.  The window rows of
// both images are staged in LDS; each thread first sums the window vertically for the
// TX + 2R window columns of its label (registers), then slides the horizontal sum.
// Border handling: window positions are clamped to the image (clamp-to-edge), and a
// right-image column left of 0 costs `trunc`.
#include "common.h"

namespace dm {

constexpr int kSadTX = 16;  // pixels per block

template <typename OT, int R>
__global__ __launch_bounds__(256) void sad_tile_kernel(const float* __restrict__ IL, const float* __restrict__ IR, int W,
                                                       int H, int K, float trunc, float inv_area,
                                                       OT* __restrict__ out) {
    constexpr int TX = kSadTX;
    constexpr int NR = 2 * R + 1;   // window rows
    constexpr int NC = TX + 2 * R;  // window columns of the tile
    __shared__ float sL[NR][NC];
    __shared__ float sR[NR][NC + 255];
    const int y = blockIdx.y;
    const int x0 = blockIdx.x * TX;
    const int lr = x0 - R;            // image column of sL[.][0]
    const int rr = x0 - R - (K - 1);  // image column of sR[.][0]
    const int nrc = NC + K - 1;
    for (int e = threadIdx.x; e < NR * nrc; e += blockDim.x) {
        const int row = e / nrc, j = e - row * nrc;
        const int yy = min(max(y + row - R, 0), H - 1);
        const int xc = rr + j;
        sR[row][j] = (xc >= 0 && xc < W) ? IR[(long long)yy * W + xc] : 0.0f;
        if (j < NC) sL[row][j] = IL[(long long)yy * W + min(max(lr + j, 0), W - 1)];
    }
    __syncthreads();
    const int d = threadIdx.x;
    if (d >= K) return;
    // vertical window sums at the (clamped) columns lr + i
    float col[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        const int xx = min(max(lr + i, 0), W - 1);  // clamped image column
        const int li = xx - lr;                     // its index in sL
        const int xr = xx - d;                      // matching right-image column
        const int ri = xr - rr;
        float acc = 0.0f;
#pragma unroll
        for (int row = 0; row < NR; ++row) acc += (xr >= 0) ? fabsf(sL[row][li] - sR[row][ri]) : trunc;
        col[i] = acc;
    }
#pragma unroll
    for (int xi = 0; xi < TX; ++xi) {
        const int x = x0 + xi;
        if (x >= W) break;
        float acc = 0.0f;
#pragma unroll
        for (int dx = 0; dx < NR; ++dx) acc += col[xi + dx];
        out[((long long)y * W + x) * K + d] = (OT)fminf(trunc, acc * inv_area);
    }
}

// Any odd window (the tiled kernel covers radii 1..3): one thread per (pixel, label).
template <typename OT>
__global__ __launch_bounds__(256) void sad_kernel(const float* __restrict__ IL, const float* __restrict__ IR, int W,
                                                  int H, int K, int r, float trunc, float inv_area,
                                                  OT* __restrict__ out) {
    const long long total = (long long)W * H * K;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int d = (int)(idx % K);
        const long long p = idx / K;
        const int x = (int)(p % W), y = (int)(p / W);
        float acc = 0.0f;
        for (int dx = -r; dx <= r; ++dx) {
            const int xx = min(max(x + dx, 0), W - 1);
            const int xr = xx - d;
            for (int dy = -r; dy <= r; ++dy) {
                const int yy = min(max(y + dy, 0), H - 1);
                acc += (xr >= 0) ? fabsf(IL[(long long)yy * W + xx] - IR[(long long)yy * W + xr]) : trunc;
            }
        }
        out[idx] = (OT)fminf(trunc, acc * inv_area);
    }
}

__global__ __launch_bounds__(256) void contrast_kernel(const float* __restrict__ IL, int W, int H, float lambda_pw,
                                                       float inv_sigma, float* __restrict__ w_h,
                                                       float* __restrict__ w_v) {
    const long long total = (long long)W * H;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < total;
         p += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(p % W), y = (int)(p / W);
        const float c = IL[p];
        if (w_h != nullptr && x + 1 < W) w_h[(long long)y * (W - 1) + x] = lambda_pw * expf(-fabsf(IL[p + 1] - c) * inv_sigma);
        if (w_v != nullptr && y + 1 < H) w_v[p] = lambda_pw * expf(-fabsf(IL[p + W] - c) * inv_sigma);
    }
}

hipError_t launch_contrast_weights(const float* I, int W, int H, float lambda_pw, float contrast_sigma, float* w_h,
                                   float* w_v, hipStream_t stream) {
    const long long npx = (long long)W * H;
    const unsigned b2 = (unsigned)std::min<long long>((npx + 255) / 256, 65535LL);
    hipLaunchKernelGGL(contrast_kernel, dim3(b2), dim3(256), 0, stream, I, W, H, lambda_pw, 1.0f / contrast_sigma, w_h,
                       w_v);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Census + Hamming
// The paper's data term (Sec. 3.1): each image's Census transform over a small patch,
// compared by the Hamming distance.  Readings: bit b of a pixel's code is
// [I(q_b) < I(centre)] for the b-th non-centre position q_b of the (2R+1)^2 window in
// raster order (dy outer, dx inner), coordinates clamped to the image; the cost is the
// number of differing bits over n = (2R+1)^2 - 1, truncated at `trunc`; a match outside
// the image costs `trunc`.  Left view: pixel x matches x - d of the right image; right
// view: pixel x of the right image matches x + d of the left image.
//
// A block owns one image row and TX consecutive pixels; each thread owns a pair of
// labels (d, d + 1).  The window rows of the reference image (TX codes) and of the
// matched image (TX + K - 1 codes) are staged in LDS and every code is computed once per
// block; then each thread writes its two labels' costs for the TX pixels: per label one
// xor, two popcounts and a table lookup (the table holds min(trunc, h / n) for h = 0..n,
// each an IEEE division, so every value is the correctly rounded quotient).  PACK (K
// even): the pair is one 2-element store (its element offset is even, so it is aligned).
constexpr int kCensusTX = 64;

template <typename OT, int R, bool LEFT, bool PACK>
__global__ __launch_bounds__(128) void census_tile_kernel(const float* __restrict__ IL, const float* __restrict__ IR,
                                                          int W, int H, int K, float trunc, OT* __restrict__ out) {
    constexpr int TX = kCensusTX;
    constexpr int NR = 2 * R + 1;
    constexpr int NA = TX + 2 * R;  // staged columns of the reference image
    __shared__ float sA[NR][NA];
    __shared__ float sB[NR][TX + 255 + 2 * R];
    __shared__ uint64_t cA[TX];
    __shared__ uint64_t cB[TX + 255];
    __shared__ float lut[64];
    const float* __restrict__ A = LEFT ? IL : IR;  // reference image of the view
    const float* __restrict__ B = LEFT ? IR : IL;  // matched image
    const int y = blockIdx.y;
    const int x0 = blockIdx.x * TX;
    const int nb = TX + K - 1;                // codes of the matched image
    const int bA = x0;                         // image column of code cA[0]
    const int bB = LEFT ? x0 - (K - 1) : x0;  // image column of code cB[0]
    const int nbs = nb + 2 * R;
#pragma unroll
    for (int row = 0; row < NR; ++row) {
        const long long yy = min(max(y + row - R, 0), H - 1);
        const float* __restrict__ Brow = B + yy * W;
        for (int j = threadIdx.x; j < nbs; j += blockDim.x) sB[row][j] = Brow[min(max(bB - R + j, 0), W - 1)];
        const float* __restrict__ Arow = A + yy * W;
        for (int j = threadIdx.x; j < NA; j += blockDim.x) sA[row][j] = Arow[min(max(bA - R + j, 0), W - 1)];
    }
    constexpr int n = NR * NR - 1;
    if (threadIdx.x <= n) lut[threadIdx.x] = fminf(trunc, (float)threadIdx.x / (float)n);
    __syncthreads();
    // codes: staged column c's window is columns c .. c + 2R of the staged rows
    for (int c = threadIdx.x; c < TX + nb; c += blockDim.x) {
        const bool isA = c < TX;
        const int cc = isA ? c : c - TX;
        uint64_t v = 0;
        int b = 0;
        if (isA) {
            const float ctr = sA[R][cc + R];
#pragma unroll
            for (int dy = 0; dy < NR; ++dy)
#pragma unroll
                for (int dx = 0; dx < NR; ++dx) {
                    if (dy == R && dx == R) continue;
                    v |= (uint64_t)(sA[dy][cc + dx] < ctr) << b;
                    ++b;
                }
            cA[cc] = v;
        } else {
            const float ctr = sB[R][cc + R];
#pragma unroll
            for (int dy = 0; dy < NR; ++dy)
#pragma unroll
                for (int dx = 0; dx < NR; ++dx) {
                    if (dy == R && dx == R) continue;
                    v |= (uint64_t)(sB[dy][cc + dx] < ctr) << b;
                    ++b;
                }
            cB[cc] = v;
        }
    }
    __syncthreads();
    const int d0 = 2 * (int)threadIdx.x;
    if (d0 >= K) return;
    const bool two = d0 + 1 < K;  // always with PACK
    const int nx = min(TX, W - x0);
    const float tr = trunc;
    auto cost = [&](int xi, int d) -> float {
        const int x = x0 + xi;
        const int xo = LEFT ? x - d : x + d;            // matched column
        const int jb = LEFT ? xi + K - 1 - d : xi + d;  // its code index
        return (xo >= 0 && xo < W) ? lut[__popcll(cA[xi] ^ cB[jb])] : tr;
    };
    OT* __restrict__ o = out + ((long long)y * W + x0) * K + d0;
#pragma unroll 8
    for (int xi = 0; xi < nx; ++xi) {
        const float c0 = cost(xi, d0);
        if constexpr (PACK) {
            typedef OT pair_t __attribute__((ext_vector_type(2)));
            pair_t v;
            v.x = (OT)c0;
            v.y = (OT)cost(xi, d0 + 1);
            *reinterpret_cast<pair_t*>(o) = v;
        } else {
            o[0] = (OT)c0;
            if (two) o[1] = (OT)cost(xi, d0 + 1);
        }
        o += K;
    }
}

// Left-right consistency check (Sec. 4.1): a left pixel keeps its disparity iff the
// right view's disparity at its match x - round(u) (round half up) differs by at most
// max_diff; otherwise it gets `invalid`.  The rounding is exact (floor plus the
// fraction's comparison with 1/2), the difference and its comparison are FP32.
__global__ __launch_bounds__(256) void lr_check_kernel(const float* __restrict__ uL, const float* __restrict__ uR,
                                                       int W, int H, float max_diff, float invalid,
                                                       float* __restrict__ out) {
    const long long total = (long long)W * H;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < total;
         p += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(p % W);
        const float u = uL[p];
        const float fl = floorf(u);
        const float r = fl + ((u - fl) >= 0.5f ? 1.0f : 0.0f);
        const float xr = (float)x - r;
        float o = invalid;
        if (xr >= 0.0f && xr <= (float)(W - 1)) {
            const float v = uR[p - x + (long long)xr];
            if (fabsf(u - v) <= max_diff) o = u;
        }
        out[p] = o;
    }
}

}  // namespace dm

using namespace dm;

extern "C" int dm_build_cost_volume_census(const float* I_left, const float* I_right, dm_shape s,
                                           const dm_cost_params* p, int view, dm_dtype out_dtype, void* cost_out,
                                           float* w_h, float* w_v, void* hip_stream) {
    clear_error();
    int st = validate_shape(s);
    if (st != DM_OK) return st;
    DM_REQUIRE(p != nullptr, DM_ERR_NULL, "params is NULL");
    DM_REQUIRE(I_left != nullptr && I_right != nullptr && cost_out != nullptr, DM_ERR_NULL,
               "images and cost_out are required");
    DM_REQUIRE(out_dtype == DM_F32 || out_dtype == DM_F16, DM_ERR_DTYPE, "unknown dtype %d", (int)out_dtype);
    DM_REQUIRE(view == DM_VIEW_LEFT || view == DM_VIEW_RIGHT, DM_ERR_PARAM, "view=%d must be 0 (left) or 1 (right)",
               view);
    DM_REQUIRE(p->window == 3 || p->window == 5 || p->window == 7, DM_ERR_PARAM, "census window=%d must be 3, 5 or 7",
               p->window);
    DM_REQUIRE(p->trunc > 0.0f && p->trunc <= 1.0f, DM_ERR_PARAM, "census trunc must be in (0, 1]");
    DM_REQUIRE(p->lambda_pw >= 0.0f && p->contrast_sigma > 0.0f, DM_ERR_PARAM,
               "lambda_pw >= 0 and contrast_sigma > 0 required");
    {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_error("pending HIP error before dm_build_cost_volume_census: %s", hipGetErrorString(e));
            return DM_ERR_HIP;
        }
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const long long total = (long long)s.W * s.H * s.K;
    ProfScope ps(DM_PROF_CENSUS, (double)total * (out_dtype == DM_F16 ? 2 : 4) + 8.0 * s.W * s.H, stream);
    const dim3 grid((unsigned)((s.W + kCensusTX - 1) / kCensusTX), (unsigned)s.H);
    const dim3 block((unsigned)(((s.K + 1) / 2 + 63) / 64 * 64));  // one thread per label pair
    const bool left = view == DM_VIEW_LEFT;
    const bool pack = (s.K % 2) == 0;
#define DM_CENSUS_V(OT, RR, LF, PK)                                                                                 \
    hipLaunchKernelGGL((census_tile_kernel<OT, RR, LF, PK>), grid, block, 0, stream, I_left, I_right, s.W, s.H, s.K, \
                       p->trunc, static_cast<OT*>(cost_out))
#define DM_CENSUS(OT, RR)                                     \
    do {                                                      \
        if (left) {                                           \
            if (pack) DM_CENSUS_V(OT, RR, true, true);        \
            else DM_CENSUS_V(OT, RR, true, false);            \
        } else {                                              \
            if (pack) DM_CENSUS_V(OT, RR, false, true);       \
            else DM_CENSUS_V(OT, RR, false, false);           \
        }                                                     \
    } while (0)
    const int r = p->window / 2;
    if (out_dtype == DM_F16) {
        if (r == 1) DM_CENSUS(_Float16, 1);
        else if (r == 2) DM_CENSUS(_Float16, 2);
        else DM_CENSUS(_Float16, 3);
    } else {
        if (r == 1) DM_CENSUS(float, 1);
        else if (r == 2) DM_CENSUS(float, 2);
        else DM_CENSUS(float, 3);
    }
#undef DM_CENSUS
#undef DM_CENSUS_V
    ps.stop();
    DM_HIP_TRY(hipGetLastError(), "census launch");
    if (w_h != nullptr || w_v != nullptr) {
        const long long npx = (long long)s.W * s.H;
        const unsigned b2 = (unsigned)std::min<long long>((npx + 255) / 256, 65535LL);
        hipLaunchKernelGGL(contrast_kernel, dim3(b2), dim3(256), 0, stream, left ? I_left : I_right, s.W, s.H,
                           p->lambda_pw, 1.0f / p->contrast_sigma, w_h, w_v);
        DM_HIP_TRY(hipGetLastError(), "contrast launch");
    }
    return DM_OK;
}

extern "C" int dm_lr_check(const float* u_left, const float* u_right, int W, int H, float max_diff, float invalid,
                           float* u_out, void* hip_stream) {
    clear_error();
    DM_REQUIRE(u_left != nullptr && u_right != nullptr && u_out != nullptr, DM_ERR_NULL,
               "u_left, u_right and u_out are required");
    DM_REQUIRE(W >= 1 && H >= 1 && (long long)W * H <= (1LL << 31), DM_ERR_SHAPE, "W=%d H=%d out of range", W, H);
    DM_REQUIRE(W <= (1 << 24), DM_ERR_SHAPE, "W=%d above 2^24", W);
    DM_REQUIRE(max_diff >= 0.0f, DM_ERR_PARAM, "max_diff must be >= 0");
    {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_error("pending HIP error before dm_lr_check: %s", hipGetErrorString(e));
            return DM_ERR_HIP;
        }
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const long long npx = (long long)W * H;
    ProfScope ps(DM_PROF_LR_CHECK, 12.0 * npx, stream);
    const unsigned blocks = (unsigned)std::min<long long>((npx + 255) / 256, 65535LL * 4);
    hipLaunchKernelGGL(lr_check_kernel, dim3(blocks), dim3(256), 0, stream, u_left, u_right, W, H, max_diff, invalid,
                       u_out);
    ps.stop();
    DM_HIP_TRY(hipGetLastError(), "lr check launch");
    return DM_OK;
}

extern "C" int dm_build_cost_volume(const float* I_left, const float* I_right, dm_shape s, const dm_cost_params* p,
                                    dm_dtype out_dtype, void* cost_out, float* w_h, float* w_v, void* hip_stream) {
    clear_error();
    int st = validate_shape(s);
    if (st != DM_OK) return st;
    DM_REQUIRE(p != nullptr, DM_ERR_NULL, "params is NULL");
    DM_REQUIRE(I_left != nullptr && I_right != nullptr && cost_out != nullptr, DM_ERR_NULL,
               "images and cost_out are required");
    DM_REQUIRE(out_dtype == DM_F32 || out_dtype == DM_F16, DM_ERR_DTYPE, "unknown dtype %d", (int)out_dtype);
    DM_REQUIRE(p->window >= 1 && p->window <= 15 && (p->window % 2) == 1, DM_ERR_PARAM,
               "window=%d must be odd in [1, 15]", p->window);
    DM_REQUIRE(p->trunc > 0.0f, DM_ERR_PARAM, "trunc must be > 0");
    DM_REQUIRE(p->lambda_pw >= 0.0f && p->contrast_sigma > 0.0f, DM_ERR_PARAM,
               "lambda_pw >= 0 and contrast_sigma > 0 required");
    {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_error("pending HIP error before dm_build_cost_volume: %s", hipGetErrorString(e));
            return DM_ERR_HIP;
        }
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const long long total = (long long)s.W * s.H * s.K;
    const unsigned blocks = (unsigned)std::min<long long>((total + 255) / 256, 65535LL * 8);
    const int r = p->window / 2;
    const float inv_area = 1.0f / (float)(p->window * p->window);
    // algorithmic bytes: the volume written once, the two images read once
    ProfScope ps(DM_PROF_COST_VOLUME, (double)total * (out_dtype == DM_F16 ? 2 : 4) + 8.0 * s.W * s.H, stream);
    const dim3 tgrid((unsigned)((s.W + kSadTX - 1) / kSadTX), (unsigned)s.H);
    const dim3 tblock((unsigned)((s.K + 63) / 64 * 64));
#define DM_SAD_TILE(OT, RR) \
    hipLaunchKernelGGL((sad_tile_kernel<OT, RR>), tgrid, tblock, 0, stream, I_left, I_right, s.W, s.H, s.K, p->trunc, \
                       inv_area, static_cast<OT*>(cost_out))
    if (out_dtype == DM_F16) {
        if (r == 1) DM_SAD_TILE(_Float16, 1);
        else if (r == 2) DM_SAD_TILE(_Float16, 2);
        else if (r == 3) DM_SAD_TILE(_Float16, 3);
        else
            hipLaunchKernelGGL(sad_kernel<_Float16>, dim3(blocks), dim3(256), 0, stream, I_left, I_right, s.W, s.H, s.K,
                               r, p->trunc, inv_area, static_cast<_Float16*>(cost_out));
    } else {
        if (r == 1) DM_SAD_TILE(float, 1);
        else if (r == 2) DM_SAD_TILE(float, 2);
        else if (r == 3) DM_SAD_TILE(float, 3);
        else
            hipLaunchKernelGGL(sad_kernel<float>, dim3(blocks), dim3(256), 0, stream, I_left, I_right, s.W, s.H, s.K, r,
                               p->trunc, inv_area, static_cast<float*>(cost_out));
    }
#undef DM_SAD_TILE
    ps.stop();
    DM_HIP_TRY(hipGetLastError(), "sad launch");
    if (w_h != nullptr || w_v != nullptr) {
        const long long npx = (long long)s.W * s.H;
        const unsigned b2 = (unsigned)std::min<long long>((npx + 255) / 256, 65535LL);
        hipLaunchKernelGGL(contrast_kernel, dim3(b2), dim3(256), 0, stream, I_left, s.W, s.H, p->lambda_pw,
                           1.0f / p->contrast_sigma, w_h, w_v);
        DM_HIP_TRY(hipGetLastError(), "contrast launch");
    }
    return DM_OK;
}
