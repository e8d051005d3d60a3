// cost_volume.hip - truncated windowed SAD cost volume and contrast edge weights.
//
// Paper: the data term sampled at every label forms the unary cost vectors
// (Sec. 2.2 "Stereo"), precomputed for all labels before the discrete stage
// (Table tab:timing "Cost Vol.").  The paper's own data term is Census + Hamming
// (Sec. 3.1); this kernel provides a truncated windowed SAD in the same role.
// Edge strengths are image dependent, lower across image edges (Sec. 2.1).
//
// Layout: one thread per (pixel, label), label fastest, so each wavefront writes a
// contiguous run of the label-major volume (the kernel is bound by those writes);
// the image reads of a window hit the caches.
#include "common.h"

namespace dm {

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
        for (int dy = -r; dy <= r; ++dy) {
            const int yy = min(max(y + dy, 0), H - 1);
            const float* Lrow = IL + (long long)yy * W;
            const float* Rrow = IR + (long long)yy * W;
            for (int dx = -r; dx <= r; ++dx) {
                const int xx = min(max(x + dx, 0), W - 1);
                const int xr = xx - d;
                acc += (xr >= 0) ? fabsf(Lrow[xx] - Rrow[xr]) : trunc;
            }
        }
        const float v = fminf(trunc, acc * inv_area);
        out[idx] = (OT)v;
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
    if (out_dtype == DM_F16)
        hipLaunchKernelGGL(sad_kernel<_Float16>, dim3(blocks), dim3(256), 0, stream, I_left, I_right, s.W, s.H, s.K, r,
                           p->trunc, inv_area, static_cast<_Float16*>(cost_out));
    else
        hipLaunchKernelGGL(sad_kernel<float>, dim3(blocks), dim3(256), 0, stream, I_left, I_right, s.W, s.H, s.K, r,
                           p->trunc, inv_area, static_cast<float*>(cost_out));
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
