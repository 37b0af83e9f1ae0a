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
// the previous frame's buffers are read about once from HBM.  Byte offsets
// are 32-bit: the host limits frames to fewer than 2^28 pixels.
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

constexpr unsigned kTmpNoPixel = 0xfffffff0u;   // offset beyond every buffer: loads read 0

__device__ __forceinline__ float3 ld3(rsrc_t r, unsigned off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b96(r, off, 0, 0);
    return make_float3(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]));
}

// All of a pixel's loads (its own buffers, then the four taps' world
// position, normal, history length and radiance) are issued before any
// test, as 12-byte buffer loads from 32-bit offsets; a tap outside the image
// reads zeros from an offset beyond the buffers and is not counted.
__global__ __launch_bounds__(kTmpThreads) void temporal_kernel(TemporalArgs a)
{
    const int P = a.H * a.W;
    const int p = blockIdx.x * kTmpThreads + threadIdx.x;
    if (p >= P) return;
    const int y = p / a.W, x = p - y * a.W;
    const unsigned P12 = (unsigned)P * 12u, P4 = (unsigned)P * 4u;
    const float3 r = ld3(make_rsrc(a.r, P12), (unsigned)p * 12u);
    float o0 = r.x, o1 = r.y, o2 = r.z, L = 1.f;
    if (a.pr) {
        const float3 nf = ld3(make_rsrc(a.n, P12), (unsigned)p * 12u);
        const float3 wf = ld3(make_rsrc(a.wp, P12), (unsigned)p * 12u);
        const auto mv = __builtin_amdgcn_raw_buffer_load_b64(make_rsrc(a.mv, (unsigned)P * 8u), (unsigned)p * 8u, 0, 0);
        // the reprojected position, its cell and its fraction exactly (in
        // double), so that every implementation picks the same four taps
        const double qx = (double)x + (double)__uint_as_float(mv[0]);
        const double qy = (double)y + (double)__uint_as_float(mv[1]);
        const double cx = floor(qx), cy = floor(qy);
        const float fx = (float)(qx - cx), fy = (float)(qy - cy);
        const int x0 = (int)fmax(fmin(cx, 1e9), -1e9), y0 = (int)fmax(fmin(cy, 1e9), -1e9);
        const rsrc_t rpw = make_rsrc(a.pw, P12), rpn = make_rsrc(a.pn, P12), rpr = make_rsrc(a.pr, P12);
        const rsrc_t rpl = make_rsrc(a.pl, P4);
        unsigned q[4];
        bool inside[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int tx = x0 + (t & 1), ty = y0 + (t >> 1);
            inside[t] = tx >= 0 && tx < a.W && ty >= 0 && ty < a.H;
            q[t] = inside[t] ? (unsigned)(ty * a.W + tx) : 0u;
        }
        float3 pw[4], pn[4], pr[4];
        float pl[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const unsigned o3 = inside[t] ? q[t] * 12u : kTmpNoPixel;
            pw[t] = ld3(rpw, o3);
            pn[t] = ld3(rpn, o3);
            pl[t] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rpl, inside[t] ? q[t] * 4u : kTmpNoPixel, 0, 0));
            pr[t] = ld3(rpr, o3);
        }
        const double n0 = nf.x, n1 = nf.y, n2 = nf.z, w0 = wf.x, w1 = wf.y, w2 = wf.z;
        float S = 0.f, Ls = 0.f, h0 = 0.f, h1 = 0.f, h2 = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const double d0 = (double)pw[t].x - w0;
            const double d1 = (double)pw[t].y - w1;
            const double d2 = (double)pw[t].z - w2;
            // each product is exact in double, so contraction into fma does
            // not change the rounded sums
            const double dist2 = d0 * d0 + d1 * d1 + d2 * d2;
            const double dot = (double)pn[t].x * n0 + (double)pn[t].y * n1 + (double)pn[t].z * n2;
            if (!(inside[t] && dist2 <= a.pos_tol2 && dot >= a.normal_tol)) continue;
            const float w = ((t & 1) ? fx : 1.f - fx) * ((t >> 1) ? fy : 1.f - fy);
            S += w;
            Ls += w * pl[t];
            h0 += w * pr[t].x;
            h1 += w * pr[t].y;
            h2 += w * pr[t].z;
        }
        if (S > 0.f) {
            const float inv = 1.f / S;
            const float Lh = Ls * inv;
            const float al = fmaxf(1.f / (Lh + 1.f), a.alpha_min);
            o0 = (1.f - al) * (h0 * inv) + al * r.x;
            o1 = (1.f - al) * (h1 * inv) + al * r.y;
            o2 = (1.f - al) * (h2 * inv) + al * r.z;
            L = Lh + 1.f;
        }
    }
    typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
    __builtin_amdgcn_raw_buffer_store_b96(u32x3{__float_as_uint(o0), __float_as_uint(o1), __float_as_uint(o2)},
                                          make_rsrc(a.out, P12), (unsigned)p * 12u, 0, 0);
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
