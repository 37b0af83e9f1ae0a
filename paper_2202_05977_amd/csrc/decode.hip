// Weight-sharing kernel construction + filtering + fusion + remodulation
// (Sec. 4.2; Eq. 3, Eq. 4, Eq. 5) in one memory-bound pass, and its adjoint.
//
// The normalised kernel weight of Eq. 3 depends on the neighbour only
// through its own scalar W_i(q) and on the centre only through the window
// sum, so every filtered value is a ratio of two box sums:
//     out_i(p) = sum_{q in Omega_i(p)} W_i(q) c(q) / max(sum_{q in Omega_i(p)} W_i(q), eps)
// with windows truncated at the border.  No k x k kernel map is ever formed.
//
// Two input forms:
//   frames   (decode_tile_kernel, the denoising path) a workgroup of 512
//            threads owns a tile of 40 x 45 centres (1280 x 720: 512 tiles,
//            two per CU), forms c = r / (a + eps_a) while staging its halo,
//            keeps it in registers, and for each kernel size sums the plane
//            (W_i, W_i c) in LDS along the rows, then down the columns;
//            head (planar [2M][H][W]), r, a and out come from the frame
//            descriptors of a batch; mod = a + eps_a
//   tensors  (decode_fwd_kernel<DK_TENSORS>, wskp_decode) head [N,H,W,2M],
//            c, mod (optional) and out are plain tensors of equal-size
//            frames; 32 x 16-centre tiles of 256 threads
// Adjoint: decode_fwd_kernel<DK_ADJ_A> (32 x 16 tiles; the forward window
// sums plus the per-centre adjoint terms) and decode_adj_b_kernel (the same
// box sums of those terms).
#include "wskp_internal.h"

namespace wskp {

// 32 x 16-centre tiles (8 row groups of kDTY/8 rows).  The adjoint's
// results are validated at this height only.
constexpr int kDTX = 32, kDTY = 16;
static_assert(kDTY % 8 == 0, "8 row groups of kDTY/8 rows");
// minimum resident workgroups per CU the forward kernel's registers must
// allow (a build-time tuning knob)
#ifndef WSKP_DECODE_MIN_WG
#define WSKP_DECODE_MIN_WG 4
#endif

struct DecodeIO {
    int H, W;
    const float *head;  // map j of pixel q at head[q * hs_pix + j * hs_map]
    size_t hs_pix, hs_map;
    const float *r, *a; // frames form
    const float *c;     // tensors form
    const float *mod;   // tensors form, may be null
    float *out;
    const float *g;
    float *grad_head;
    float4 *scratch;
    float *dlogit;
};

struct DecodeTensors {
    int N, H, W;
    const float *head, *c, *mod;
    float *out;
    // adjoint only
    const float *g;     // dL/dout [N,H,W,3]
    float *grad_head;   // [N,H,W,2M]
    float4 *scratch;    // [N,M,H,W] x (u_0, u_1, u_2, dS)
    float *dlogit;      // [N,M,H,W]: the logits' gradients, pass A to pass B
};

// Tile u of nbk (u in launch order) -> frame, tile origin and I/O pointers.
template <bool FRAMES>
__device__ __forceinline__ bool decode_locate_at(const DecodeCfg &dc, const FrameArg &fa,
                                                 const DecodeTensors &dt, int u, int nbk,
                                                 DecodeIO &io, int &x0, int &y0)
{
    const int twoM = 2 * dc.M;
    auto tiles = [](int H, int W) { return ((W + kDTX - 1) / kDTX) * ((H + kDTY - 1) / kDTY); };
    int t = xcd_logical_id(u, nbk);
    if constexpr (FRAMES) {
        int n;
        t = batch_tile_id(fa, u, nbk, n);
        if (t < 0) return false;
        const int f = batch_frame(fa, n, t, tiles);
        if (f < 0) return false;
        const FrameDesc &fd = frame_at(fa, f);
        io.H = fd.H;
        io.W = fd.W;
        io.head = fd.head;              // planar [2M][H][W] (written by the head conv)
        io.hs_pix = 1;
        io.hs_map = (size_t)fd.H * fd.W;
        io.r = fd.r;
        io.a = fd.a;
        io.c = nullptr;
        io.mod = nullptr;
        io.out = fd.out;
        io.g = nullptr;
        io.grad_head = nullptr;
        io.scratch = nullptr;
        io.dlogit = nullptr;
    } else {
        // equal-size frames: the frame index is a division
        const int cnt = tiles(dt.H, dt.W);
        const int f = t / cnt;
        if (f >= dt.N) return false;
        t -= f * cnt;
        const size_t P = (size_t)dt.H * dt.W;
        io.H = dt.H;
        io.W = dt.W;
        io.head = dt.head + (size_t)f * P * twoM;   // interleaved [H][W][2M]
        io.hs_pix = twoM;
        io.hs_map = 1;
        io.r = io.a = nullptr;
        io.c = dt.c + (size_t)f * P * 3;
        io.mod = dt.mod ? dt.mod + (size_t)f * P * 3 : nullptr;
        io.out = dt.out ? dt.out + (size_t)f * P * 3 : nullptr;
        io.g = dt.g ? dt.g + (size_t)f * P * 3 : nullptr;
        io.grad_head = dt.grad_head ? dt.grad_head + (size_t)f * P * twoM : nullptr;
        io.scratch = dt.scratch ? dt.scratch + (size_t)f * P * dc.M : nullptr;
        io.dlogit = dt.dlogit ? dt.dlogit + (size_t)f * P * dc.M : nullptr;
    }
    const int txn = (io.W + kDTX - 1) / kDTX;
    x0 = (t % txn) * kDTX;
    y0 = (t / txn) * kDTY;
    return true;
}

template <bool FRAMES>
__device__ __forceinline__ bool decode_locate(const DecodeCfg &dc, const FrameArg &fa,
                                              const DecodeTensors &dt, DecodeIO &io, int &x0,
                                              int &y0)
{
    return decode_locate_at<FRAMES>(dc, fa, dt, blockIdx.x, gridDim.x, io, x0, y0);
}

enum DecodeKind { DK_FRAMES = 0, DK_TENSORS = 1, DK_ADJ_A = 2 };

// e^x for the softmax numerators (x = l_i - max_j l_j <= 0): the hardware
// 2^x of x log2(e) instead of the library expf.  Relative error about
// 1 ulp + |x| * 6e-8 (the rounding of x log2(e)); the numerators with a
// large |x| are the small ones, whose errors hardly move the blend.
__device__ __forceinline__ float exp_softmax(float x)
{
    return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
}

__device__ __forceinline__ float4 f4add(float4 a, float4 b)
{
    return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}

// Window sums of K consecutive values for N consecutive window starts:
//   s[t] = v[t] + ... + v[t+K-1],  t = 0..N-1,
// with additions only (no running sum with subtraction, so a large value
// leaving the window cannot cancel the small ones that remain).  For K >= N
// the part v[N-1..K-1] is common to all N windows and is summed once; each
// window adds a suffix of the run's head and a prefix of its tail.
template <int K, int N, typename LD>
__device__ __forceinline__ void box_run(LD v, float4 *s)
{
    // v(j) reads value j where it is needed; the partial sums are formed in
    // an order that keeps only the outputs and two running sums live:
    //   s[t] = (v(t) + ... + v(N-2)) + C + (v(K) + ... + v(K+t-1))
    if constexpr (K < N || K <= 3) {
#pragma unroll
        for (int t = 0; t < N; ++t) {
            float4 a = v(t);
#pragma unroll
            for (int j = 1; j < K; ++j) a = f4add(a, v(t + j));
            s[t] = a;
        }
    } else {
        float4 C = v(N - 1);
#pragma unroll
        for (int j = N; j < K; ++j) C = f4add(C, v(j));
        s[N - 1] = C;
        if constexpr (N >= 2) {
            float4 L = v(N - 2);
            s[N - 2] = f4add(L, C);
#pragma unroll
            for (int t = N - 3; t >= 0; --t) {
                L = f4add(v(t), L);
                s[t] = f4add(L, C);
            }
            float4 Rt = v(K);
            s[1] = f4add(s[1], Rt);
#pragma unroll
            for (int t = 2; t < N; ++t) {
                Rt = f4add(Rt, v(K + t - 1));
                s[t] = f4add(s[t], Rt);
            }
        }
    }
}

// Tile geometry: 32 x kDTY centres per workgroup; a thread owns a column
// tx and a run of kRun = kDTY/8 rows (kRun*ty .. kRun*ty+kRun-1); the
// horizontal pass gives each thread runs of kHRun columns.
constexpr int kRun = kDTY / 8;
constexpr int kHRun = 4;
// Halo pixels per thread for a largest radius of at most RM.  The kernels
// are instantiated for RM = 5 (kernel sizes up to 11) and RM = 7 (up to 15):
// the smaller bound needs fewer registers.
template <int RM>
constexpr int max_pix() { return ((32 + 2 * RM + 1) * (kDTY + 2 * RM) + kThreads - 1) / kThreads; }

// Row stride (in float4) of the halo planes.  A 16-byte LDS read serves 8
// lanes per cycle from 32 banks and the horizontal pass gives consecutive
// lanes consecutive rows, so 8 consecutive rows must fall in distinct
// 16-byte bank groups: an odd stride does that.
__device__ __host__ __forceinline__ int halo_stride(int R) { return 32 + 2 * R + 1; }
constexpr int kHB = 33;   // row-sum buffer stride (float4): rows land in distinct bank groups

// Horizontal then vertical window sums of a float4 plane st [HY][HXS] for
// kernel size K: returns in acc[t] the K x K window sums of the 4 components
// for this thread's kRun centres.  hb holds the row sums [HY][kHB].
// Horizontal items are numbered row-fastest, so the lanes of a wave read
// and write different rows at the same columns (no bank conflicts).
template <int K>
__device__ __forceinline__ void window_sums4(int R, int HXS, const float4 *st, float4 *hb,
                                             float4 *acc)
{
    constexpr int r = K / 2;
    const int tid = threadIdx.x;
    constexpr int nrows = kDTY + 2 * r;
    constexpr int RPR = 32 / kHRun;
    for (int it = tid; it < nrows * RPR; it += kThreads) {
        const int hy = R - r + it % nrows, xr = (it / nrows) * kHRun;
        const int base = hy * HXS + xr + R - r;
        float4 s[kHRun];
        box_run<K, kHRun>([&](int j) { return st[base + j]; }, s);
#pragma unroll
        for (int t = 0; t < kHRun; ++t) hb[hy * kHB + xr + t] = s[t];
    }
    lds_sync();
    const int tx = tid & 31, ty = tid >> 5;
    const int vb = (kRun * ty + R - r) * kHB + tx;
    box_run<K, kRun>([&](int j) { return hb[vb + j * kHB]; }, acc);
    // no barrier here: the next writer of hb runs after the caller's next
    // barrier, and the horizontal reads of st ended at the barrier above
}

#define WSKP_SWITCH_K(RM, k, CALL)                       \
    switch (k) {                                         \
    case 1: CALL(1); break;                              \
    case 3: CALL(3); break;                              \
    case 5: CALL(5); break;                              \
    case 7: CALL(7); break;                              \
    case 9: CALL(9); break;                              \
    case 11: CALL(11); break;                            \
    case 13: if constexpr (RM >= 6) { CALL(13); } break; \
    default: if constexpr (RM >= 7) { CALL(15); } break; \
    }

// Global pixel index of each of this thread's halo slots (-1 outside the
// image or past the halo), computed once per workgroup.  The halo width HX
// is a runtime value: one division gives the first slot's row and column,
// and each further slot (kThreads later) steps them by the wave-uniform
// quotient and remainder of kThreads / HX (the remainder is below HX, so
// the column wraps at most once).
template <int RM>
__device__ __forceinline__ void halo_pixels(int x0, int y0, int R, int HX, int HXY, int H, int W,
                                            int *gp)
{
    const int sy = kThreads / HX, sx = kThreads - sy * HX;
    int ly = threadIdx.x / HX, lx = threadIdx.x - ly * HX;
#pragma unroll
    for (int k = 0; k < max_pix<RM>(); ++k) {
        const int p = threadIdx.x + k * kThreads;
        const int gy = y0 - R + ly, gx = x0 - R + lx;
        gp[k] = (p < HXY && gy >= 0 && gy < H && gx >= 0 && gx < W) ? gy * W + gx : -1;
        lx += sx;
        ly += sy;
        if (lx >= HX) {
            lx -= HX;
            ++ly;
        }
    }
}

// Frames form: byte offset of a slot that holds no image pixel, beyond
// every buffer the decode reads (frames hold at most 2^28 pixels, so the
// largest, radiance and albedo, stay below 3.3e9 bytes); such loads read 0.
constexpr unsigned kNoPixel = 0xfffffff0u;

// Frames form: weight map i (a plane of the head record) at this thread's
// halo slots, from byte offsets o1 (4 * pixel, or kNoPixel: reads 0).
template <int RM>
__device__ __forceinline__ void load_w_frames(const DecodeIO &io, int i, const unsigned *o1, float *w)
{
    const unsigned P = (unsigned)(io.H * io.W);
    const rsrc_t rs = make_rsrc(io.head + (size_t)i * P, P * 4u);
#pragma unroll
    for (int k = 0; k < max_pix<RM>(); ++k)
        w[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, o1[k], 0, 0));
}

// Loads weight map i at this thread's halo pixels, unconditionally (pixels
// outside the image read pixel 0; the caller masks them with gp < 0).
template <int M, int RM>
__device__ __forceinline__ void load_w(const DecodeIO &io, int i, const int *gp, float *w)
{
#pragma unroll
    for (int k = 0; k < max_pix<RM>(); ++k)
        w[k] = gload(io.head + (size_t)(gp[k] >= 0 ? gp[k] : 0) * io.hs_pix + i * io.hs_map);
}

// Dynamic LDS: product plane float4 [HXY] (W_i, W_i c) rebuilt for each
// kernel size, row sums float4 [(kDTY+2R)][kHB].
//   DK_FRAMES / DK_TENSORS: forward, writes out.
//   DK_ADJ_A: first half of the vector-Jacobian product.  Per centre p,
//     with dF = g * mod, da_i = <dF, out_i>:
//       dlogit_i   = alpha_i (da_i - sum_j alpha_j da_j)
//       u_i,ch(p)  = alpha_i dF_ch / max(S_i, eps)
//       dS_i(p)    = -[S_i > eps] sum_ch u_i,ch(p) out_i,ch(p)
//     (u_i, dS_i) and dlogit_i go to scratch (planes per size, coalesced
//     stores); decode_adj_b_kernel box-sums (u_i, dS_i) and writes each
//     pixel's whole grad_head record.
template <int M, int KIND, int RM>
__global__ __launch_bounds__(kThreads, WSKP_DECODE_MIN_WG) void decode_fwd_kernel(DecodeCfg dc, FrameArg fa,
                                                               DecodeTensors dt)
{
    constexpr bool FRAMES = KIND == DK_FRAMES;
    constexpr bool ADJ = KIND == DK_ADJ_A;
    extern __shared__ float4 lds4[];
    DecodeIO io;
    int x0, y0;
    if (!decode_locate<FRAMES>(dc, fa, dt, io, x0, y0)) return;

    const int R = dc.R;
    const int HX = halo_stride(R), HXY = HX * (kDTY + 2 * R);
    float4 *pr = lds4;
    float4 *hb = pr + HXY;
    const int H = io.H, W = io.W;
    const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;

    constexpr int kMaxPix = max_pix<RM>();
    int gp[kMaxPix];
    halo_pixels<RM>(x0, y0, R, HX, HXY, H, W, gp);
    // irradiance of this thread's halo pixels, kept in registers; c = r /
    // (a + eps_a) uses the hardware reciprocal.  The weight map of each size
    // is fetched one size ahead.
    // All loads are unconditional (pixels outside the image or the halo read
    // pixel 0 and are masked afterwards), so that every request is in flight
    // before the first result is used.
    // The frames form uses buffer loads from precomputed byte offsets: a
    // slot outside the image gets kNoPixel and reads zeros (c = 0 * rcp(eps_a)
    // = 0, W = 0), so nothing needs masking afterwards.
    float cv[kMaxPix][3], av[FRAMES ? kMaxPix : 1][3], wv[kMaxPix];
    unsigned o1[FRAMES ? kMaxPix : 1];
    if constexpr (FRAMES) {
        const unsigned P = (unsigned)(H * W);
        const rsrc_t rr = make_rsrc(io.r, P * 12u), ra = make_rsrc(io.a, P * 12u);
#pragma unroll
        for (int k = 0; k < kMaxPix; ++k) {
            const unsigned o3 = gp[k] >= 0 ? (unsigned)gp[k] * 12u : kNoPixel;
            o1[k] = gp[k] >= 0 ? (unsigned)gp[k] * 4u : kNoPixel;
            const auto r3 = __builtin_amdgcn_raw_buffer_load_b96(rr, o3, 0, 0);
            const auto a3 = __builtin_amdgcn_raw_buffer_load_b96(ra, o3, 0, 0);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                cv[k][ch] = __uint_as_float(r3[ch]);
                av[k][ch] = __uint_as_float(a3[ch]);
            }
        }
        load_w_frames<RM>(io, 0, o1, wv);
    } else {
#pragma unroll
        for (int k = 0; k < kMaxPix; ++k) {
            const size_t q = (size_t)(gp[k] >= 0 ? gp[k] : 0) * 3;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) cv[k][ch] = gload(io.c + q + ch);
        }
        load_w<M, RM>(io, 0, gp, wv);
    }
#pragma unroll
    for (int k = 0; k < kMaxPix; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            if constexpr (FRAMES)
                cv[k][ch] *= __builtin_amdgcn_rcpf(av[FRAMES ? k : 0][ch] + dc.eps_albedo);
            else
                cv[k][ch] = gp[k] >= 0 ? cv[k][ch] : 0.f;
        }

    // Fusion (Eq. 5) of this thread's kRun centres (column tx, rows
    // kRun*ty + o).  Forward: softmax numerators exp(l_i - max_j l_j) weight
    // the filtered values as they are produced and the sum of the
    // numerators divides once at the end; no per-size state is kept, so the
    // size loop need not be unrolled.  Adjoint: the normalised alpha_i are
    // kept for the gradient.
    const float *lp[kRun];
    unsigned lo[FRAMES ? kRun : 1];   // frames: byte offset of the centre in a plane
    // frames: logit i of this thread's centres, from plane M + i by buffer load
    auto logit_frames = [&](int i, int o) {
        const unsigned P = (unsigned)(H * W);
        const rsrc_t rs = make_rsrc(io.head + (size_t)(M + i) * P, P * 4u);
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, lo[FRAMES ? o : 0], 0, 0));
    };
    float lmax[kRun], esum[kRun], F[kRun][3];
    float alpha[ADJ ? kRun : 1][ADJ ? M : 1];
#pragma unroll
    for (int o = 0; o < kRun; ++o) {
        const int y = y0 + kRun * ty + o, x = x0 + tx;
        const bool in = y < H && x < W;
        lp[o] = io.head + ((size_t)(in ? y : 0) * W + (in ? x : 0)) * io.hs_pix + M * io.hs_map;
        if constexpr (FRAMES) lo[o] = in ? (unsigned)(y * W + x) * 4u : 0u;
        float m = -INFINITY;
#pragma unroll
        for (int i = 0; i < M; ++i) m = fmaxf(m, FRAMES ? logit_frames(i, o) : gload(lp[o] + i * io.hs_map));
        lmax[o] = m;
        esum[o] = 0.f;
        F[o][0] = F[o][1] = F[o][2] = 0.f;
        if constexpr (ADJ) {
            float sum = 0.f;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                alpha[o][i] = expf(gload(lp[o] + i * io.hs_map) - m);
                sum += alpha[o][i];
            }
            const float inv = 1.f / sum;
#pragma unroll
            for (int i = 0; i < M; ++i) alpha[o][i] *= inv;
        }
    }
    float outv[ADJ ? kRun : 1][ADJ ? M : 1][3];
    float Sv[ADJ ? kRun : 1][ADJ ? M : 1];
    float mv[ADJ ? 1 : kRun][3];   // forward: remodulation factor of the centres

    // one kernel size: product plane, window sums, normalisation, fusion
    auto size_step = [&](int i) {
        // this size's logits of the thread's centres, requested first so
        // that the window sums hide their latency
        float lgv[ADJ ? 1 : kRun];
        if constexpr (!ADJ) {
#pragma unroll
            for (int o = 0; o < kRun; ++o) lgv[o] = FRAMES ? logit_frames(i, o) : gload(lp[o] + i * io.hs_map);
        }
        // product plane of this size from this thread's registers, then
        // fetch the next size's weights
#pragma unroll
        for (int k = 0; k < kMaxPix; ++k) {
            const int p = tid + k * kThreads;
            const float w = (FRAMES || gp[k] >= 0) ? wv[k] : 0.f;
            if (p < HXY) pr[p] = make_float4(w, w * cv[k][0], w * cv[k][1], w * cv[k][2]);
        }
        if (i + 1 < M) {
            if constexpr (FRAMES) load_w_frames<RM>(io, i + 1, o1, wv);
            else load_w<M, RM>(io, i + 1, gp, wv);
        }
        lds_sync();
        float4 acc[kRun];
#define WSKP_WS(KK) window_sums4<KK>(R, HX, pr, hb, acc)
        WSKP_SWITCH_K(RM, 2 * dc.radius[i] + 1, WSKP_WS)
#undef WSKP_WS
#pragma unroll
        for (int o = 0; o < kRun; ++o) {
            const float inv = __builtin_amdgcn_rcpf(fmaxf(acc[o].x, dc.eps_norm));
            const float o0 = acc[o].y * inv, o1 = acc[o].z * inv, o2 = acc[o].w * inv;
            if constexpr (ADJ) {
                outv[o][i][0] = o0;
                outv[o][i][1] = o1;
                outv[o][i][2] = o2;
                Sv[o][i] = acc[o].x;
            } else {
                const float e = exp_softmax(lgv[o] - lmax[o]);
                esum[o] += e;
                F[o][0] += e * o0;
                F[o][1] += e * o1;
                F[o][2] += e * o2;
            }
        }
    };
    if constexpr (ADJ) {
#pragma unroll
        for (int i = 0; i < M; ++i) size_step(i);
    } else {
#pragma unroll 1
        for (int i = 0; i < M - 1; ++i) size_step(i);
        // the centres' remodulation factors are requested before the last
        // size's window sums, which hide their latency (centres outside the
        // image read pixel 0 and are not stored)
#pragma unroll
        for (int o = 0; o < kRun; ++o) {
            if constexpr (FRAMES) {
                const unsigned P = (unsigned)(H * W);
                const auto a3 = __builtin_amdgcn_raw_buffer_load_b96(make_rsrc(io.a, P * 12u), lo[o] * 3u, 0, 0);
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) mv[o][ch] = __uint_as_float(a3[ch]) + dc.eps_albedo;
            } else {
                const int y = y0 + kRun * ty + o, x = x0 + tx;
                const size_t pix = (y < H && x < W) ? (size_t)y * W + x : 0;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) mv[o][ch] = io.mod ? gload(io.mod + pix * 3 + ch) : 1.f;
            }
        }
        size_step(M - 1);
#pragma unroll
        for (int o = 0; o < kRun; ++o) {
            const float inv = 1.f / esum[o];
            F[o][0] *= inv;
            F[o][1] *= inv;
            F[o][2] *= inv;
        }
    }

#pragma unroll
    for (int o = 0; o < kRun; ++o) {
        const int y = y0 + kRun * ty + o, x = x0 + tx;
        if (y >= H || x >= W) continue;
        const size_t pix = (size_t)y * W + x;
        if constexpr (!ADJ) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) gstore(io.out + pix * 3 + ch, mv[o][ch] * F[o][ch]);
        } else {
            float dF[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                dF[ch] = gload(io.g + pix * 3 + ch) * (io.mod ? gload(io.mod + pix * 3 + ch) : 1.f);
            float da[M], adot = 0.f;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                da[i] = dF[0] * outv[o][i][0] + dF[1] * outv[o][i][1] + dF[2] * outv[o][i][2];
                adot += alpha[o][i] * da[i];
            }
            const size_t P = (size_t)H * W;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                gstore(io.dlogit + (size_t)i * P + pix, alpha[o][i] * (da[i] - adot));
                const float S = Sv[o][i];
                const float inv = 1.f / fmaxf(S, dc.eps_norm);
                float4 v;
                v.x = alpha[o][i] * dF[0] * inv;
                v.y = alpha[o][i] * dF[1] * inv;
                v.z = alpha[o][i] * dF[2] * inv;
                v.w = S > dc.eps_norm
                          ? -(v.x * outv[o][i][0] + v.y * outv[o][i][1] + v.z * outv[o][i][2])
                          : 0.f;
                gstore(reinterpret_cast<gf32x4 *>(io.scratch + (size_t)i * P + pix), gf32x4{v.x, v.y, v.z, v.w});
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Forward decode, one tile of TW x TH centres per workgroup of 512 threads.
//
// Separable window sums, horizontal first.  Per kernel size i, r = r_i:
//   1. each thread writes the plane (W_i, W_i c) of its halo pixels into
//      LDS, P[hy][hx] (row stride HXS, odd);
//   2. horizontal pass: thread (halo row hy, run of kNR columns) sums the
//      r-windows of the TW output columns into the row-sum buffer
//      S[hy][x] (rows R-r .. R+TH+r-1: the rows the vertical pass reads);
//   3. vertical pass: thread (column x, run of kNC rows) sums r-windows of
//      the row sums down its column: the k x k window sums of its kNC
//      centres, which it normalises and blends into their fusion state.
// Two barriers per size: after 1 (the plane is complete) and after 2 (the
// row sums are complete).  The vertical pass of size i and the plane write
// of size i + 1 use different buffers and run in the same phase.
// The thread of step 3 owns those centres for the whole kernel: their
// logits, fusion state and output.  Its lanes hold consecutive columns, so
// the centres' global loads and stores are coalesced row segments.  The
// irradiance c of the thread's halo pixels stays in registers.  Each size's
// weight map is fetched two sizes ahead and its logits one size ahead, with
// the size loop unrolled so that the prefetched registers are never copied
// (a copy would wait for its load): the loads of the next sizes stay in
// flight across the barriers of this one.  With exp weights (whose halo
// maximum takes more registers) the map is fetched one size ahead and the
// logits while the plane is built, in a loop that is not unrolled.
//
// Fusion (Eq. 5) is an online softmax: the state of a centre is the largest
// logit seen so far (m, in base-2 units), the sum of the numerators 2^(l-m)
// and the numerator-weighted sum of the filtered values; a larger logit
// rescales both by 2^(m_old - m_new).  Only the first size's logits are
// needed before filtering starts.
//
// EXPW: the head holds raw pre-activations h and W = exp(h).  Window ratios
// are unchanged by a common factor, so each tile uses W = exp(h - m_i) with
// m_i the largest h_i over its halo (no overflow for any finite h) and the
// floor eps e^{-m_i} in place of eps: out = N / max(S, eps) as with exp(h).
constexpr int kFThreads = 512;
constexpr int kFSlots = 6;          // halo pixels per thread: HXS * (TH + 2R) <= 3072
constexpr int kNR = 5;              // row sums per thread (horizontal run)
constexpr int kNC = 5;              // centres per thread (vertical run)
constexpr int kTileW = 40;          // centres per tile row (multiple of kNR)
constexpr int kSRow = kTileW + 1;   // row-sum buffer stride (float4): odd
constexpr float kLog2e = 1.4426950408889634f;


__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
    return v;
}

template <int M, int RM, bool EXPW>
__global__ __launch_bounds__(kFThreads, 4) void decode_tile_kernel(DecodeCfg dc, FrameArg fa)
{
    extern __shared__ float4 lds4[];
    __shared__ float red[2][kFThreads / 64];
    const int TW = dc.tw, TH = dc.th, HXS = dc.hxs, R = dc.R;
    const int HX = TW + 2 * R, HY = TH + 2 * R, HXY = HXS * HY;
    const int tid = threadIdx.x;

    // ---- tile -> frame, origin, I/O
    DecodeIO io;
    int x0, y0;
    {
        auto tiles = [&](int H, int W) { return ((W + TW - 1) / TW) * ((H + TH - 1) / TH); };
        int n;
        int t = batch_tile_id(fa, blockIdx.x, gridDim.x, n);
        if (t < 0) return;
        const int f = batch_frame(fa, n, t, tiles);   // t becomes the tile within frame f
        if (f < 0) return;
        const FrameDesc &fd = frame_at(fa, f);
        io.H = fd.H;
        io.W = fd.W;
        io.head = fd.head;
        io.hs_pix = 1;
        io.hs_map = (size_t)fd.H * fd.W;
        io.r = fd.r;
        io.a = fd.a;
        io.c = nullptr;
        io.mod = nullptr;
        io.out = fd.out;
        const int txn = (io.W + TW - 1) / TW;
        x0 = (t % txn) * TW;
        y0 = (t / txn) * TH;
    }
    const int H = io.H, W = io.W;
    const unsigned P = (unsigned)(H * W);

    // ---- this thread's halo slots p = tid + k * 512: row-major over
    // [HY][HXS].  gp[k] is the slot's pixel index in the frame, or -1 (a
    // slot outside the image, a padding column hx >= HX, or past the plane):
    // such slots hold W = 0.  Slots past the plane write their zeros to the
    // plane's last cell, a padding column (TW + 2R is even, so HXS = HX + 1)
    // that no pass reads.
    int gp[kFSlots];
    {
        const int sy = kFThreads / HXS, sx = kFThreads - sy * HXS;
        int ly = tid / HXS, lx = tid - ly * HXS;
#pragma unroll
        for (int k = 0; k < kFSlots; ++k) {
            const int gy = y0 - R + ly, gx = x0 - R + lx;
            gp[k] = (ly < HY && lx < HX && gy >= 0 && gy < H && gx >= 0 && gx < W) ? gy * W + gx : -1;
            lx += sx;
            ly += sy;
            if (lx >= HXS) {
                lx -= HXS;
                ++ly;
            }
        }
    }
    // the thread's centres: column cx of the tile, rows cy .. cy + kNC - 1
    // (the last run of a column is moved up to end at row TH - 1; centres it
    // shares with the run above are computed, and stored, twice with the
    // same values).  nc: how many of them lie in the image.
    const int nv_items = TW * ((TH + kNC - 1) / kNC);
    const bool owner = tid < nv_items;
    const int cx = tid % TW, cy = min((tid / TW) * kNC, TH - kNC);
    const int gcx = x0 + cx, gcy = y0 + cy;
    const int nc = (owner && gcx < W) ? max(0, min(kNC, H - gcy)) : 0;
    auto centre_off = [&](int q) { return q < nc ? (unsigned)((gcy + q) * W + gcx) * 4u : kNoPixel; };
    auto centre_pix = [&](int q) { return q < nc ? (size_t)(gcy + q) * W + gcx : (size_t)0; };

    // ---- loads: irradiance of the halo slots, the first weight map.  All
    // are buffer loads from 32-bit byte offsets (kNoPixel outside the image:
    // reads zeros).  Map j of pixel q sits at (j P + q) * 4 (planar record).
    const unsigned hstride = 4u;
    auto map_rsrc = [&](int j) { return make_rsrc(io.head + (size_t)j * P, P * 4u); };
    constexpr bool kAhead2 = !EXPW;     // weights two sizes ahead, logits one
    float cv[kFSlots][3], wv[kFSlots], wn[kFSlots];
    auto load_w = [&](int i, float *dst) {
        const rsrc_t rs = map_rsrc(i);
#pragma unroll
        for (int k = 0; k < kFSlots; ++k)
            dst[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                rs, gp[k] >= 0 ? (unsigned)gp[k] * hstride : kNoPixel, 0, 0));
    };
    auto load_logit = [&](int i, float *lg) {
        const rsrc_t rs = map_rsrc(M + i);
#pragma unroll
        for (int q = 0; q < kNC; ++q) {
            const unsigned o = centre_off(q);
            lg[q] = __uint_as_float(
                __builtin_amdgcn_raw_buffer_load_b32(rs, o == kNoPixel ? kNoPixel : (o >> 2) * hstride, 0, 0));
        }
    };
    float lg[kNC];
    {
        const rsrc_t rr = make_rsrc(io.r, P * 12u), ra = make_rsrc(io.a, P * 12u);
        float av[kFSlots][3];
#pragma unroll
        for (int k = 0; k < kFSlots; ++k) {
            const unsigned o3 = gp[k] >= 0 ? (unsigned)gp[k] * 12u : kNoPixel;
            const auto r3 = __builtin_amdgcn_raw_buffer_load_b96(rr, o3, 0, 0);
            const auto a3 = __builtin_amdgcn_raw_buffer_load_b96(ra, o3, 0, 0);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                cv[k][ch] = __uint_as_float(r3[ch]);
                av[k][ch] = __uint_as_float(a3[ch]);
            }
        }
        load_w(0, wv);
        load_logit(0, lg);
        if (kAhead2 && M > 1) load_w(1, wn);
#pragma unroll
        for (int k = 0; k < kFSlots; ++k)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                // c = r / (a + eps_a) by the hardware reciprocal; slots outside
                // the image hold c = 0 (also when eps_a = 0, where the
                // reciprocal of their zero albedo is infinite)
                const float c = cv[k][ch] * __builtin_amdgcn_rcpf(av[k][ch] + dc.eps_albedo);
                cv[k][ch] = gp[k] >= 0 ? c : 0.f;
            }
    }

    // ---- online fusion state of the thread's centres
    float lm[kNC], esum[kNC], F[kNC][3];
#pragma unroll
    for (int q = 0; q < kNC; ++q) {
        lm[q] = -INFINITY;
        esum[q] = 0.f;
        F[q][0] = F[q][1] = F[q][2] = 0.f;
    }

    float4 *pl = lds4;                  // plane [HY][HXS]
    float4 *sr = lds4 + HXY;            // row sums [HY][kSRow]
    const int wave = tid >> 6;
    // EXPW: the halo maximum of the loaded map, per wave into red[buf]
    auto wave_max_to_lds = [&](int buf) {
        float m = -INFINITY;
#pragma unroll
        for (int k = 0; k < kFSlots; ++k) m = gp[k] >= 0 ? fmaxf(m, wv[k]) : m;
        m = wave_max(m);
        if ((tid & 63) == 0) red[buf][wave] = m;
    };
    if constexpr (EXPW) {
        wave_max_to_lds(0);
        lds_sync();
    }
    float mv[kNC][3];                   // remodulation factor of the centres

    constexpr int kUnroll = kAhead2 ? M : 1;
#pragma unroll kUnroll
    for (int i = 0; i < M; ++i) {
        const int r = dc.radius[i];
        float eps = dc.eps_norm;
        // 1. the plane (W_i, W_i c) of the halo slots
        {
            float mi = 0.f;
            if constexpr (EXPW) {
                mi = red[i & 1][0];
#pragma unroll
                for (int w = 1; w < kFThreads / 64; ++w) mi = fmaxf(mi, red[i & 1][w]);
                // a tile without image pixels in its halo has nothing to filter
                mi = mi == -INFINITY ? 0.f : mi;
                eps = fmaxf(eps * __builtin_amdgcn_exp2f(-mi * kLog2e), 1.17549435e-38f);
            }
#pragma unroll
            for (int k = 0; k < kFSlots; ++k) {
                const int p = min(tid + k * kFThreads, HXY - 1);
                float w = wv[k];
                if constexpr (EXPW) w = __builtin_amdgcn_exp2f((w - mi) * kLog2e);
                w = gp[k] >= 0 ? w : 0.f;
                pl[p] = make_float4(w, w * cv[k][0], w * cv[k][1], w * cv[k][2]);
            }
        }
        // the prefetches (see above); before the last size, the centres'
        // remodulation factors
        float w2[kFSlots], l1[kNC];
        if constexpr (kAhead2) {
            if (i + 2 < M) load_w(i + 2, w2);
            if (i + 1 < M) load_logit(i + 1, l1);
        } else {
            if (i > 0) load_logit(i, lg);
            if (i + 1 < M) load_w(i + 1, wv);
        }
        if (i + 1 == M) {
            const rsrc_t ra = make_rsrc(io.a, P * 12u);
#pragma unroll
            for (int q = 0; q < kNC; ++q) {
                const unsigned o = centre_off(q);
                const auto a3 = __builtin_amdgcn_raw_buffer_load_b96(ra, o == kNoPixel ? kNoPixel : o * 3u, 0, 0);
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) mv[q][ch] = __uint_as_float(a3[ch]) + dc.eps_albedo;
            }
        }
        lds_sync();

        // 2. horizontal pass: halo row hy (of the TH + 2r the vertical pass
        // reads), output columns x .. x + kNR - 1, into the row-sum buffer
        {
            const int nrows = TH + 2 * r;
            if (tid < nrows * (TW / kNR)) {
                const int hrow = R - r + tid % nrows;
                const int hx = (tid / nrows) * kNR;
                const int base = hrow * HXS + R - r + hx;
                float4 hs[kNR];
#define WSKP_H(KK) box_run<KK, kNR>([&](int j) { return pl[base + j]; }, hs)
                WSKP_SWITCH_K(RM, 2 * r + 1, WSKP_H)
#undef WSKP_H
#pragma unroll
                for (int t = 0; t < kNR; ++t) sr[hrow * kSRow + hx + t] = hs[t];
            }
        }
        if constexpr (EXPW) {
            if (i + 1 < M) wave_max_to_lds((i + 1) & 1);
        }
        lds_sync();

        // 3. vertical pass over the row sums: the kNC centres' window sums
        // (S, N_0, N_1, N_2), normalised and blended
        if (owner) {
            float4 acc[kNC];
            const int base = (cy + R - r) * kSRow + cx;
#define WSKP_V(KK) box_run<KK, kNC>([&](int j) { return sr[base + j * kSRow]; }, acc)
            WSKP_SWITCH_K(RM, 2 * r + 1, WSKP_V)
#undef WSKP_V
#pragma unroll
            for (int q = 0; q < kNC; ++q) {
                const float inv = __builtin_amdgcn_rcpf(fmaxf(acc[q].x, eps));
                const float l2 = lg[q] * kLog2e;
                const float mn = fmaxf(lm[q], l2);
                const float sc = __builtin_amdgcn_exp2f(lm[q] - mn);   // 0 for the first size
                const float e = __builtin_amdgcn_exp2f(l2 - mn);
                lm[q] = mn;
                esum[q] = esum[q] * sc + e;
                const float ei = e * inv;
                F[q][0] = F[q][0] * sc + ei * acc[q].y;
                F[q][1] = F[q][1] * sc + ei * acc[q].z;
                F[q][2] = F[q][2] * sc + ei * acc[q].w;
            }
        }
        if constexpr (kAhead2) {
            // size i + 1 becomes current (no copies once unrolled)
#pragma unroll
            for (int k = 0; k < kFSlots; ++k) {
                wv[k] = wn[k];
                wn[k] = w2[k];
            }
            if (i + 1 < M) {
#pragma unroll
                for (int q = 0; q < kNC; ++q) lg[q] = l1[q];
            }
        }
    }

    // ---- remodulation (y = mod * F / sum of numerators) and store
#pragma unroll
    for (int q = 0; q < kNC; ++q) {
        if (q >= nc) break;
        const float inv = 1.f / esum[q];
        float *op = io.out + centre_pix(q) * 3;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) gstore(op + ch, mv[q][ch] * (F[q][ch] * inv));
    }
}

// Second half of the vector-Jacobian product.  Windows are symmetric and
// truncated the same way at the border (p in Omega(q) <=> q in Omega(p)), so
// the adjoint of a box sum is the same box sum:
//   dW_i(q)  = sum_ch c_ch(q) box_i(u_i,ch)(q) + box_i(dS_i)(q)  -> grad_head[q][i]
//   dc_ch(q) = sum_i W_i(q) box_i(u_i,ch)(q)                      -> grad_c[q][ch]
// One size at a time: stage the halo of (u_i, dS_i) as float4, row sums,
// column sums.  LDS: float4 [HXY] staged + float4 [(kDTY+2R)][kHB] row sums.
template <int M, int RM>
__global__ __launch_bounds__(kThreads) void decode_adj_b_kernel(DecodeCfg dc, DecodeTensors dt,
                                                                 float *grad_c)
{
    extern __shared__ float4 lds4[];
    FrameArg fa{};
    DecodeIO io;
    int x0, y0;
    if (!decode_locate<false>(dc, fa, dt, io, x0, y0)) return;
    const int R = dc.R;
    const int HX = halo_stride(R), HXY = HX * (kDTY + 2 * R);
    float4 *st = lds4;
    float4 *hb = st + HXY;
    const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
    const int H = io.H, W = io.W;
    const size_t P = (size_t)H * W;
    const int fidx = (int)((io.head - dt.head) / ((size_t)P * 2 * M));
    float *gc = grad_c + (size_t)fidx * P * 3;

    constexpr int kMaxPix = max_pix<RM>();
    int gp[kMaxPix];
    halo_pixels<RM>(x0, y0, R, HX, HXY, H, W, gp);
    // the centres' irradiance and weights, read once; dW_i and dc summed
    // over the sizes in registers
    float cvv[kRun][3], wvv[kRun][M], dwv[kRun][M], dcv[kRun][3];
#pragma unroll
    for (int o = 0; o < kRun; ++o) {
        const int y = y0 + kRun * ty + o, x = x0 + tx;
        const size_t pix = (y < H && x < W) ? (size_t)y * W + x : 0;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            cvv[o][ch] = gload(io.c + pix * 3 + ch);
            dcv[o][ch] = 0.f;
        }
#pragma unroll
        for (int i = 0; i < M; ++i) wvv[o][i] = gload(io.head + pix * (2 * M) + i);
    }
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const float4 *sp = io.scratch + (size_t)i * P;
        float4 v[kMaxPix];
#pragma unroll
        for (int k = 0; k < kMaxPix; ++k) {
            const gf32x4 q = gload(reinterpret_cast<const gf32x4 *>(sp + (gp[k] >= 0 ? gp[k] : 0)));
            v[k] = gp[k] >= 0 ? make_float4(q.x, q.y, q.z, q.w) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int k = 0; k < kMaxPix; ++k) {
            const int p = tid + k * kThreads;
            if (p < HXY) st[p] = v[k];
        }
        lds_sync();
        float4 acc[kRun];
#define WSKP_WS(KK) window_sums4<KK>(R, HX, st, hb, acc)
        WSKP_SWITCH_K(RM, 2 * dc.radius[i] + 1, WSKP_WS)
#undef WSKP_WS
#pragma unroll
        for (int o = 0; o < kRun; ++o) {
            // acc = box sums of (u_0, u_1, u_2, dS)
            dwv[o][i] = cvv[o][0] * acc[o].x + cvv[o][1] * acc[o].y + cvv[o][2] * acc[o].z + acc[o].w;
            dcv[o][0] += wvv[o][i] * acc[o].x;
            dcv[o][1] += wvv[o][i] * acc[o].y;
            dcv[o][2] += wvv[o][i] * acc[o].z;
        }
    }
    // each centre's record [dW_0 .. dW_{M-1}, dlogit_0 .. dlogit_{M-1}] in
    // consecutive stores, so that its lines are written whole (grad_head
    // needs only the 4-byte alignment of a float)
#pragma unroll
    for (int o = 0; o < kRun; ++o) {
        const int y = y0 + kRun * ty + o, x = x0 + tx;
        if (y < H && x < W) {
            const size_t pix = (size_t)y * W + x;
            float rec[2 * M];
#pragma unroll
            for (int i = 0; i < M; ++i) {
                rec[i] = dwv[o][i];
                rec[M + i] = gload(io.dlogit + (size_t)i * P + pix);
            }
            float *gh = io.grad_head + pix * (2 * M);
#pragma unroll
            for (int j = 0; j < 2 * M; ++j) gstore(gh + j, rec[j]);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) gstore(gc + pix * 3 + ch, dcv[o][ch]);
        }
    }
}

static size_t decode_lds_bytes(const DecodeCfg &dc)
{
    const size_t HX = halo_stride(dc.R), HY = kDTY + 2 * dc.R;
    return sizeof(float4) * (HX * HY + HY * kHB);
}

static size_t adj_b_lds_bytes(const DecodeCfg &dc)
{
    const size_t HX = halo_stride(dc.R), HY = kDTY + 2 * dc.R;
    return sizeof(float4) * (HX * HY + HY * kHB);
}

template <typename K>
static void allow_lds(K kernel, size_t bytes)
{
    if (bytes > 48 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int KIND>
static hipError_t launch_decode(const DecodeCfg &dc, const FrameArg &fa, const DecodeTensors &dt,
                                int blocks, hipStream_t s)
{
    if (blocks <= 0) return hipSuccess;
    const size_t lds = decode_lds_bytes(dc);
    // the largest radius selects the register-lean instantiation when it can
    const bool r5 = dc.R <= 5;
    switch (dc.M) {
#define WSKP_M(m)                                                                                  \
    case m:                                                                                        \
        if (r5) {                                                                                  \
            allow_lds(decode_fwd_kernel<m, KIND, 5>, lds);                                         \
            hipLaunchKernelGGL((decode_fwd_kernel<m, KIND, 5>), dim3(blocks), dim3(kThreads), lds, \
                               s, dc, fa, dt);                                                     \
        } else {                                                                                   \
            allow_lds(decode_fwd_kernel<m, KIND, 7>, lds);                                         \
            hipLaunchKernelGGL((decode_fwd_kernel<m, KIND, 7>), dim3(blocks), dim3(kThreads), lds, \
                               s, dc, fa, dt);                                                     \
        }                                                                                          \
        break;
        WSKP_M(1) WSKP_M(2) WSKP_M(3) WSKP_M(4) WSKP_M(5) WSKP_M(6) WSKP_M(7) WSKP_M(8)
#undef WSKP_M
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Tile shape of the forward decode for the handle's largest radius: 40
// centres wide; as tall as the workgroup's 512 threads allow (at most 45
// rows): every thread holds at most kFSlots halo pixels, one horizontal run
// and one vertical run.  At 720p, 1080p and 1440p with R <= 6 the 45-row
// tiles divide the frame exactly (1280 x 720: 32 x 16 = 512 tiles).
void decode_tile_shape(DecodeCfg &dc)
{
    dc.tw = kTileW;
    dc.hxs = (dc.tw + 2 * dc.R) | 1;   // odd row stride: lanes on consecutive rows hit distinct banks
    int th = 45;
    auto lds = [&](int t) { return sizeof(float4) * (size_t)(dc.hxs + kSRow) * (t + 2 * dc.R) + 64; };
    while (th > kNC && (dc.hxs * (th + 2 * dc.R) > kFSlots * kFThreads ||
                        (th + 2 * dc.R) * (dc.tw / kNR) > kFThreads ||
                        dc.tw * ((th + kNC - 1) / kNC) > kFThreads ||
                        2 * lds(th) > 160 * 1024))      // two workgroups per CU
        --th;
    dc.th = th;
}

int decode_grid(const DecodeCfg &dc, int n, const int *H, const int *W)
{
    long total = 0;
    for (int f = 0; f < n; ++f)
        total += (long)((W[f] + dc.tw - 1) / dc.tw) * ((H[f] + dc.th - 1) / dc.th);
    return (int)total;
}

static size_t tile_lds_bytes(const DecodeCfg &dc)
{
    // the plane [HY][HXS] and the row sums [HY][kSRow]
    return sizeof(float4) * (size_t)(dc.hxs + kSRow) * (dc.th + 2 * dc.R);
}

template <int M, int RM, bool EXPW>
static hipError_t launch_tile_inst(const DecodeCfg &dc, const FrameArg &fa, int blocks, hipStream_t s)
{
    const size_t lds = tile_lds_bytes(dc);
    allow_lds(decode_tile_kernel<M, RM, EXPW>, lds);
    hipLaunchKernelGGL((decode_tile_kernel<M, RM, EXPW>), dim3(blocks), dim3(kFThreads), lds, s, dc, fa);
    return hipGetLastError();
}

hipError_t launch_decode_frames(const DecodeCfg &dc, const FrameArg &fa, int blocks, hipStream_t s)
{
    // one instantiation covers every kernel size up to 15 (the size only
    // selects the window-sum code; the registers do not depend on it)
    if (blocks <= 0) return hipSuccess;
    switch (dc.M) {
#define WSKP_M(m)                                                                 \
    case m:                                                                       \
        if (dc.exp_weights) return launch_tile_inst<m, 7, true>(dc, fa, blocks, s); \
        return launch_tile_inst<m, 7, false>(dc, fa, blocks, s);
        WSKP_M(1) WSKP_M(2) WSKP_M(3) WSKP_M(4) WSKP_M(5) WSKP_M(6) WSKP_M(7) WSKP_M(8)
#undef WSKP_M
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_decode_tensors(const DecodeCfg &dc, int N, int H, int W, const float *head,
                                 const float *c, const float *mod, float *out, hipStream_t s)
{
    // the 32 x 16-tile kernel: on equal-size stacks it measured faster than
    // the 40 x 45 tile kernel (29 vs 35 us for 8 x 256^2, 42 vs 45 us at 720p)
    DecodeTensors dt{N, H, W, head, c, mod, out, nullptr, nullptr, nullptr, nullptr};
    FrameArg fa{};
    const int blocks = N * ((W + kDTX - 1) / kDTX) * ((H + kDTY - 1) / kDTY);
    return launch_decode<DK_TENSORS>(dc, fa, dt, blocks, s);
}

size_t decode_backward_scratch_bytes(const DecodeCfg &dc, int N, int H, int W)
{
    // (u_i, dS_i) as float4 and dlogit_i as float, per size and pixel
    return (size_t)N * dc.M * H * W * (sizeof(float4) + sizeof(float));
}

hipError_t launch_decode_backward(const DecodeCfg &dc, int N, int H, int W, const float *head,
                                  const float *c, const float *mod, const float *g,
                                  float *grad_head, float *grad_c, void *scratch, hipStream_t s)
{
    FrameArg fa{};
    float4 *s4 = reinterpret_cast<float4 *>(scratch);
    DecodeTensors dt{N, H, W, head, c, mod, nullptr, g, grad_head, s4,
                     reinterpret_cast<float *>(s4 + (size_t)N * dc.M * H * W)};
    const int blocks = N * ((W + kDTX - 1) / kDTX) * ((H + kDTY - 1) / kDTY);
    hipError_t e = launch_decode<DK_ADJ_A>(dc, fa, dt, blocks, s);
    if (e != hipSuccess) return e;
    const size_t lds = adj_b_lds_bytes(dc);
    const bool r5 = dc.R <= 5;
    switch (dc.M) {
#define WSKP_M(m)                                                                                 \
    case m:                                                                                       \
        if (r5) {                                                                                 \
            allow_lds(decode_adj_b_kernel<m, 5>, lds);                                            \
            hipLaunchKernelGGL((decode_adj_b_kernel<m, 5>), dim3(blocks), dim3(kThreads), lds, s, \
                               dc, dt, grad_c);                                                   \
        } else {                                                                                  \
            allow_lds(decode_adj_b_kernel<m, 7>, lds);                                            \
            hipLaunchKernelGGL((decode_adj_b_kernel<m, 7>), dim3(blocks), dim3(kThreads), lds, s, \
                               dc, dt, grad_c);                                                   \
        }                                                                                         \
        break;
        WSKP_M(1) WSKP_M(2) WSKP_M(3) WSKP_M(4) WSKP_M(5) WSKP_M(6) WSKP_M(7) WSKP_M(8)
#undef WSKP_M
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace wskp
