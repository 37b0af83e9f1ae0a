// Multi-resolution reconstruction (Sec. 5.2): the irradiance is filtered
// at several resolutions, each level with its own predicted weight maps,
// and adjacent levels are blended from the coarsest with Eq. 7:
//   o_p = i^f_p - alpha_p [U D i^f]_p + alpha_p [U i^c]_p
// (D: 2x2 mean, U: nearest-neighbour upsampling).  The per-level filtering
// is the weight-sharing decode (decode.hip, tensor form); this file holds
// the 2x2 mean of the irradiance and the blend.
#include "wskp_internal.h"

namespace wskp {

constexpr int kMrThreads = 256;

// out [H/2, W/2, 3] = 2x2 means of in [H, W, 3] (H, W even)
__global__ __launch_bounds__(kMrThreads) void pool2_kernel(int H, int W, const float *in, float *out)
{
    const int Hc = H / 2, Wc = W / 2;
    const int p = blockIdx.x * kMrThreads + threadIdx.x;
    if (p >= Hc * Wc) return;
    const int y = p / Wc, x = p - y * Wc;
    const float *a = in + ((size_t)(2 * y) * W + 2 * x) * 3;
    const float *b = a + (size_t)W * 3;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
        gstore(out + (size_t)p * 3 + ch,
               0.25f * (((gload(a + ch) + gload(a + 3 + ch)) + gload(b + ch)) + gload(b + 3 + ch)));
}

// One thread per 2x2 block of fine pixels: the block's mean of the fine
// image is formed once and serves its four outputs.  mod (optional)
// remodulates the result.  The four outputs are stored after all loads,
// each pixel's three channels in consecutive stores, so that the L2
// receives whole lines rather than parts of them spread over the kernel.
__global__ __launch_bounds__(kMrThreads) void mr_blend_kernel(int H, int W, const float *fine, const float *coarse,
                                                               const float *alpha, const float *mod, float *out)
{
    const int Hc = H / 2, Wc = W / 2;
    const int p = blockIdx.x * kMrThreads + threadIdx.x;
    if (p >= Hc * Wc) return;
    const int y = p / Wc, x = p - y * Wc;
    size_t q[4];
    q[0] = (size_t)(2 * y) * W + 2 * x;
    q[1] = q[0] + 1;
    q[2] = q[0] + W;
    q[3] = q[2] + 1;
    float f[4][3], a[4], c[3];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a[k] = gload(alpha + q[k]);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) f[k][ch] = gload(fine + q[k] * 3 + ch);
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) c[ch] = gload(coarse + (size_t)p * 3 + ch);
    float o[4][3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float df = 0.25f * (((f[0][ch] + f[1][ch]) + f[2][ch]) + f[3][ch]);
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k][ch] = f[k][ch] - a[k] * df + a[k] * c[ch];
    }
    if (mod) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) o[k][ch] *= gload(mod + q[k] * 3 + ch);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) gstore(out + q[k] * 3 + ch, o[k][ch]);
}

hipError_t launch_pool2(int H, int W, const float *in, float *out, hipStream_t s)
{
    const int n = (H / 2) * (W / 2);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(pool2_kernel, dim3((n + kMrThreads - 1) / kMrThreads), dim3(kMrThreads), 0, s, H, W, in,
                       out);
    return hipGetLastError();
}

hipError_t launch_mr_blend(int H, int W, const float *fine, const float *coarse, const float *alpha,
                           const float *mod, float *out, hipStream_t s)
{
    const int n = (H / 2) * (W / 2);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mr_blend_kernel, dim3((n + kMrThreads - 1) / kMrThreads), dim3(kMrThreads), 0, s, H, W,
                       fine, coarse, alpha, mod, out);
    return hipGetLastError();
}

}  // namespace wskp
