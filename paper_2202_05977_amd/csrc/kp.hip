// Explicit kernel-map reconstruction: the baseline of the memory and time
// comparison of Sec. 5.3.  A kernel-prediction network without weight
// sharing predicts, for every pixel p and kernel size k_i, all k_i^2 weights
// of p's own kernel; reconstruction then reads that H x W x k_i^2 map.  The
// weight-sharing form (decode.hip) reads one scalar per pixel and size.
// Here the explicit maps are filled from the weight maps (kernel weight of
// neighbour q in p's window = W_i(q), 0 outside the image), so both forms
// compute the same Eq. 3-5 result and their difference is only the memory
// each reads.
//
//   kp_expand_kernel  writes the maps, planar per tap: map_i[t][H][W], tap
//                     t = (dy + r_i) k_i + (dx + r_i)
//   kp_decode_kernel  one thread per centre: for each size, the normalised
//                     map-weighted sum of c over the window, the softmax
//                     blend with the logits and the remodulation
#include "wskp_internal.h"

namespace wskp {

constexpr int kKpThreads = 256;

// head [H,W,2M] as wskp_decode takes it: weights W_i, then logits.
__global__ __launch_bounds__(kKpThreads) void kp_expand_kernel(DecodeCfg dc, int H, int W, const float *head,
                                                                float *maps)
{
    const int P = H * W, twoM = 2 * dc.M;
    const int p = blockIdx.x * kKpThreads + threadIdx.x;
    if (p >= P) return;
    const int y = p / W, x = p - y * W;
    size_t off = 0;
    for (int i = 0; i < dc.M; ++i) {
        const int r = dc.radius[i], k = 2 * r + 1;
        for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx) {
                const int qy = y + dy, qx = x + dx;
                const bool in = qy >= 0 && qy < H && qx >= 0 && qx < W;
                const size_t t = (size_t)(dy + r) * k + (dx + r);
                gstore(maps + off + t * P + p, in ? gload(head + ((size_t)qy * W + qx) * twoM + i) : 0.f);
            }
        off += (size_t)k * k * P;
    }
}

// c [H,W,3], mod [H,W,3] (or null = 1), head [H,W,2M] (its logits).
__global__ __launch_bounds__(kKpThreads) void kp_decode_kernel(DecodeCfg dc, int H, int W, const float *maps,
                                                                const float *head, const float *c,
                                                                const float *mod, float *out)
{
    const int P = H * W;
    const int p = blockIdx.x * kKpThreads + threadIdx.x;
    if (p >= P) return;
    const int y = p / W, x = p - y * W;
    const float *lg = head + (size_t)p * 2 * dc.M + dc.M;
    float lmax = -INFINITY;
    for (int i = 0; i < dc.M; ++i) lmax = fmaxf(lmax, gload(lg + i));
    float esum = 0.f, F0 = 0.f, F1 = 0.f, F2 = 0.f;
    size_t off = 0;
    for (int i = 0; i < dc.M; ++i) {
        const int r = dc.radius[i], k = 2 * r + 1;
        float S = 0.f, N0 = 0.f, N1 = 0.f, N2 = 0.f;
        for (int dy = -r; dy <= r; ++dy) {
            const int qy = min(max(y + dy, 0), H - 1);
            for (int dx = -r; dx <= r; ++dx) {
                const int qx = min(max(x + dx, 0), W - 1);
                // taps outside the image carry weight 0 in the map
                const float w = gload(maps + off + ((size_t)(dy + r) * k + (dx + r)) * P + p);
                const float *cq = c + ((size_t)qy * W + qx) * 3;
                S += w;
                N0 += w * gload(cq);
                N1 += w * gload(cq + 1);
                N2 += w * gload(cq + 2);
            }
        }
        off += (size_t)k * k * P;
        const float inv = 1.f / fmaxf(S, dc.eps_norm);
        const float e = expf(gload(lg + i) - lmax);
        esum += e;
        F0 += e * (N0 * inv);
        F1 += e * (N1 * inv);
        F2 += e * (N2 * inv);
    }
    const float inv = 1.f / esum;
    const float *m = mod ? mod + (size_t)p * 3 : nullptr;
    gstore(out + (size_t)p * 3 + 0, (m ? gload(m) : 1.f) * F0 * inv);
    gstore(out + (size_t)p * 3 + 1, (m ? gload(m + 1) : 1.f) * F1 * inv);
    gstore(out + (size_t)p * 3 + 2, (m ? gload(m + 2) : 1.f) * F2 * inv);
}

size_t kp_map_floats(const DecodeCfg &dc, int H, int W)
{
    size_t taps = 0;
    for (int i = 0; i < dc.M; ++i) taps += (size_t)(2 * dc.radius[i] + 1) * (2 * dc.radius[i] + 1);
    return taps * H * W;
}

hipError_t launch_kp_expand(const DecodeCfg &dc, int H, int W, const float *head, float *maps, hipStream_t s)
{
    const int blocks = (H * W + kKpThreads - 1) / kKpThreads;
    hipLaunchKernelGGL(kp_expand_kernel, dim3(blocks), dim3(kKpThreads), 0, s, dc, H, W, head, maps);
    return hipGetLastError();
}

hipError_t launch_kp_decode(const DecodeCfg &dc, int H, int W, const float *maps, const float *head,
                            const float *c, const float *mod, float *out, hipStream_t s)
{
    const int blocks = (H * W + kKpThreads - 1) / kKpThreads;
    hipLaunchKernelGGL(kp_decode_kernel, dim3(blocks), dim3(kKpThreads), 0, s, dc, H, W, maps, head, c, mod,
                       out);
    return hipGetLastError();
}

}  // namespace wskp
