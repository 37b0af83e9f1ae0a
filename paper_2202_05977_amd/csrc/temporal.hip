// Temporal accumulation before denoising (Sec. 4.1, last paragraph): the
// previous frame's accumulated radiance is reprojected with the motion
// vector and, where world position and shading normal agree, blended with
// the current 1-spp radiance; elsewhere the current radiance is kept.
//
// Per pixel p: q = p + mv(p) in the previous frame; the four pixels around
// q carry bilinear weights, and a tap counts if it lies in the image, its
// world position is within pos_tol of p's and its normal has a dot product
// of at least normal_tol with p's.  With S the counted weight:
//   S > 0: history h and length L are the S-normalised weighted means,
//          alpha = max(1 / (L + 1), alpha_min), out = (1 - alpha) h + alpha r,
//          length L + 1
//   S = 0: out = r, length 1
// The tap tests are evaluated in double: for float inputs the squared
// distance and the dot product are then exact or correctly rounded, so the
// accept/reject decision is the same in any implementation that does so.
// One thread per pixel; the four taps of neighbouring threads overlap, so
// the previous frame's buffers are read about once from HBM.
#include "wskp_internal.h"

namespace wskp {

constexpr int kTmpThreads = 256;

struct TemporalArgs {
    int H, W;
    const float *r, *n, *wp, *mv;
    const float *pr, *pl, *pn, *pw;   // previous frame (pr == nullptr: first frame)
    float *out, *len;
    float alpha_min;
    double pos_tol2, normal_tol;
};

__global__ __launch_bounds__(kTmpThreads) void temporal_kernel(TemporalArgs a)
{
    const int P = a.H * a.W;
    const int p = blockIdx.x * kTmpThreads + threadIdx.x;
    if (p >= P) return;
    const int y = p / a.W, x = p - y * a.W;
    const float r0 = gload(a.r + 3 * p), r1 = gload(a.r + 3 * p + 1), r2 = gload(a.r + 3 * p + 2);
    float o0 = r0, o1 = r1, o2 = r2, L = 1.f;
    if (a.pr) {
        const double n0 = gload(a.n + 3 * p), n1 = gload(a.n + 3 * p + 1), n2 = gload(a.n + 3 * p + 2);
        const double w0 = gload(a.wp + 3 * p), w1 = gload(a.wp + 3 * p + 1), w2 = gload(a.wp + 3 * p + 2);
        // the reprojected position, its cell and its fraction exactly (in
        // double), so that every implementation picks the same four taps
        const double qx = (double)x + (double)gload(a.mv + 2 * p);
        const double qy = (double)y + (double)gload(a.mv + 2 * p + 1);
        const double cx = floor(qx), cy = floor(qy);
        const float fx = (float)(qx - cx), fy = (float)(qy - cy);
        const int x0 = (int)fmax(fmin(cx, 1e9), -1e9), y0 = (int)fmax(fmin(cy, 1e9), -1e9);
        float S = 0.f, Ls = 0.f, h0 = 0.f, h1 = 0.f, h2 = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int tx = x0 + (t & 1), ty = y0 + (t >> 1);
            if (tx < 0 || tx >= a.W || ty < 0 || ty >= a.H) continue;
            const int q = ty * a.W + tx;
            const double d0 = (double)gload(a.pw + 3 * q) - w0;
            const double d1 = (double)gload(a.pw + 3 * q + 1) - w1;
            const double d2 = (double)gload(a.pw + 3 * q + 2) - w2;
            // each product is exact in double, so contraction into fma does
            // not change the rounded sums
            const double dist2 = d0 * d0 + d1 * d1 + d2 * d2;
            const double dot = (double)gload(a.pn + 3 * q) * n0 + (double)gload(a.pn + 3 * q + 1) * n1 +
                               (double)gload(a.pn + 3 * q + 2) * n2;
            if (!(dist2 <= a.pos_tol2 && dot >= a.normal_tol)) continue;
            const float w = ((t & 1) ? fx : 1.f - fx) * ((t >> 1) ? fy : 1.f - fy);
            S += w;
            Ls += w * gload(a.pl + q);
            h0 += w * gload(a.pr + 3 * q);
            h1 += w * gload(a.pr + 3 * q + 1);
            h2 += w * gload(a.pr + 3 * q + 2);
        }
        if (S > 0.f) {
            const float inv = 1.f / S;
            const float Lh = Ls * inv;
            const float al = fmaxf(1.f / (Lh + 1.f), a.alpha_min);
            o0 = (1.f - al) * (h0 * inv) + al * r0;
            o1 = (1.f - al) * (h1 * inv) + al * r1;
            o2 = (1.f - al) * (h2 * inv) + al * r2;
            L = Lh + 1.f;
        }
    }
    gstore(a.out + 3 * p, o0);
    gstore(a.out + 3 * p + 1, o1);
    gstore(a.out + 3 * p + 2, o2);
    gstore(a.len + p, L);
}

hipError_t launch_temporal(int H, int W, const float *r, const float *n, const float *wp, const float *mv,
                           const float *pr, const float *pl, const float *pn, const float *pw, float alpha_min,
                           float pos_tol, float normal_tol, float *out, float *len, hipStream_t s)
{
    TemporalArgs a{H, W, r, n, wp, mv, pr, pl, pn, pw, out, len, alpha_min,
                   (double)pos_tol * (double)pos_tol, (double)normal_tol};
    const int blocks = (H * W + kTmpThreads - 1) / kTmpThreads;
    hipLaunchKernelGGL(temporal_kernel, dim3(blocks), dim3(kTmpThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace wskp
