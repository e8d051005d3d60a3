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

}  // namespace dm

using namespace dm;

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
