// 3x3 convolutions of the prediction network (Sec. 4.1, Eq. 2) as implicit
// GEMMs on the gfx950 matrix cores.
//
// GEMM view of one layer: rows = output pixels, columns = output channels,
// reduction K = 9 taps x C_in.  A workgroup (4 wave64s) owns a tile of
// TH x 32 output pixels and 16*NB output channels.  The reduction runs over
// chunks of CK input channels: the (TH+2) x 34 input halo of the chunk and
// the matching 9*CK x 16*NB weight slice are staged in LDS, then every wave
// issues MFMAs over the 9 taps.  The operation that produces the layer's
// input is fused into the staging step, so that input never exists in
// memory:
//   CONV_PACK   network input (Sec. 5.1): gamma-tonemapped radiance, albedo,
//               (normal+1)/2 and clamped scaled depth, from the raw buffers
//   CONV_POOL   2x2 mean of the finer level (encoder down path)
//   CONV_CAT    [nearest x2 upsample of the coarser level, skip] (decoder)
//   CONV_PLAIN  the map itself (head)
// The epilogue adds the bias and applies ReLU, or for the head the weight
// activation (softplus or exp) on channels 0..M-1 and nothing on the logits.
//
// Two arithmetic forms:
//   fp32: v_mfma_f32_16x16x4f32; LDS holds channel planes so that the 16
//         pixels x 4 channels of an A fragment are bank-conflict free.
//   bf16: v_mfma_f32_16x16x32_bf16; LDS holds pixels with 8-channel runs so
//         that each lane reads its A fragment with one 16-byte load.
//   Both accumulate in fp32.
#include "wskp_internal.h"

namespace wskp {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// ---- element conversions ---------------------------------------------------
__device__ __forceinline__ float bf16_to_f32(unsigned short h)
{
    return __uint_as_float(((unsigned int)h) << 16);
}

// Round to nearest, ties to even (the standard bit-level method); NaN stays NaN.
__device__ __forceinline__ unsigned short f32_to_bf16(float f)
{
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

template <typename T> struct Elem;
template <> struct Elem<float> {
    __device__ static __forceinline__ void load4(const float *p, float v[4])
    {
        const float4 q = *reinterpret_cast<const float4 *>(p);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    }
    __device__ static __forceinline__ void store(float *p, float v) { *p = v; }
};
template <> struct Elem<unsigned short> {
    __device__ static __forceinline__ void load4(const unsigned short *p, float v[4])
    {
        const uint2 q = *reinterpret_cast<const uint2 *>(p);
        v[0] = __uint_as_float(q.x << 16);
        v[1] = __uint_as_float(q.x & 0xffff0000u);
        v[2] = __uint_as_float(q.y << 16);
        v[3] = __uint_as_float(q.y & 0xffff0000u);
    }
    __device__ static __forceinline__ void store(unsigned short *p, float v) { *p = f32_to_bf16(v); }
};

// ---- tile lookup -------------------------------------------------------------
// Maps this workgroup to (frame, output-channel group, tile).  Returns false
// for workgroups beyond the batch's tile count (capacity launches).
template <int TH>
__device__ __forceinline__ bool conv_locate(const ConvLayer &L, const FrameArg &fa, int &f, int &g,
                                            int &x0, int &y0, int &Hl, int &Wl)
{
    const int nbk = gridDim.x;
    int t = xcd_logical_id(blockIdx.x, nbk);
    if (fa.reverse) t = nbk - 1 - t;
    for (f = 0; f < fa.n; ++f) {
        const FrameDesc &fd = frame_at(fa, f);
        Hl = fd.H >> L.level;
        Wl = fd.W >> L.level;
        const int txn = (Wl + kConvTW - 1) / kConvTW, tyn = (Hl + TH - 1) / TH;
        const int cnt = txn * tyn * L.groups;
        if (t < cnt) {
            g = t % L.groups;
            t /= L.groups;
            x0 = (t % txn) * kConvTW;
            y0 = (t / txn) * TH;
            return true;
        }
        t -= cnt;
    }
    return false;
}

// Four consecutive virtual input channels c..c+3 at pixel (gy, gx) of the
// layer's resolution, produced by the fused input operation.
template <int MODE, typename SrcT>
__device__ __forceinline__ void fetch4(const ConvLayer &L, const FrameDesc &fd, const SrcT *s0,
                                       const SrcT *s1, int gy, int gx, int Wl, int c, float v[4])
{
    if (MODE == CONV_PLAIN) {
        Elem<SrcT>::load4(s0 + ((size_t)gy * Wl + gx) * L.C0 + c, v);
    } else if (MODE == CONV_POOL) {
        const int W0 = Wl * 2;
        const SrcT *b = s0 + ((size_t)(2 * gy) * W0 + 2 * gx) * L.C0 + c;
        float p0[4], p1[4], p2[4], p3[4];
        Elem<SrcT>::load4(b, p0);
        Elem<SrcT>::load4(b + L.C0, p1);
        Elem<SrcT>::load4(b + (size_t)W0 * L.C0, p2);
        Elem<SrcT>::load4(b + (size_t)W0 * L.C0 + L.C0, p3);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = 0.25f * (p0[j] + p1[j] + p2[j] + p3[j]);
    } else if (MODE == CONV_CAT) {
        if (c < L.C0)
            Elem<SrcT>::load4(s0 + ((size_t)(gy >> 1) * (Wl >> 1) + (gx >> 1)) * L.C0 + c, v);
        else
            Elem<SrcT>::load4(s1 + ((size_t)gy * Wl + gx) * L.C1 + (c - L.C0), v);
    } else {  // CONV_PACK: [T(r) 3, a 3, (n+1)/2 3, depth 1, zero padding]
        const size_t pix = (size_t)gy * Wl + gx;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int ch = c + j;
            float x = 0.f;
            if (ch < 3) {
                const float r = fd.r[pix * 3 + ch];
                x = powf(fminf(fmaxf(r, 0.f), 1.f), L.inv_gamma);
            } else if (ch < 6) {
                x = fd.a[pix * 3 + ch - 3];
            } else if (ch < 9) {
                x = (fd.n[pix * 3 + ch - 6] + 1.f) * 0.5f;
            } else if (ch == 9) {
                x = fminf(fmaxf((fd.d[pix] - L.dnear) * L.dinv, 0.f), 1.f);
            }
            v[j] = x;
        }
    }
}

template <int EPI>
__device__ __forceinline__ float epilogue(float v, int co, int M)
{
    if (EPI == EPI_RELU) return fmaxf(v, 0.f);
    if (co < M) {
        if (EPI == EPI_HEAD_EXP) return expf(v);
        return fmaxf(v, 0.f) + log1pf(expf(-fabsf(v)));
    }
    return v;
}

template <typename OutT>
__device__ __forceinline__ OutT *conv_dst(const ConvLayer &L, const FrameDesc &fd)
{
    if (L.out_kind == 2) return reinterpret_cast<OutT *>(fd.head);
    return reinterpret_cast<OutT *>(L.out_kind ? fd.u[L.out_idx] : fd.e[L.out_idx]);
}

// =============================================================================
// fp32 form
// =============================================================================
template <int TH, int CK, int NB>
struct F32Geom {
    static constexpr int TW = kConvTW, HP = TH + 2, WP = TW + 2;
    static constexpr int PL = ((HP * WP - 16 + 31) / 32) * 32 + 16;  // plane stride = 16 mod 32
    static constexpr int BS = NB * 16 + ((NB % 2 == 0) ? 16 : 0);     // weight row stride
    static constexpr int MB = TH / 2;                                  // 16-px blocks per wave
};

template <int MODE, int EPI, int TH, int CK, int NB, typename SrcT, typename OutT>
__global__ __launch_bounds__(kThreads) void conv3x3_f32_kernel(ConvLayer L, FrameArg fa)
{
    using G = F32Geom<TH, CK, NB>;
    __shared__ float As[CK * G::PL];
    __shared__ float Bs[9 * CK * G::BS];

    int f, g, x0, y0, Hl, Wl;
    if (!conv_locate<TH>(L, fa, f, g, x0, y0, Hl, Wl)) return;
    const FrameDesc &fd = frame_at(fa, f);
    const SrcT *s0 = reinterpret_cast<const SrcT *>(L.src0_kind ? fd.u[L.src0_idx] : fd.e[L.src0_idx]);
    const SrcT *s1 = reinterpret_cast<const SrcT *>(fd.e[L.src1_idx]);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lj = lane & 15, lk = lane >> 4;

    f32x4 acc[G::MB][NB];
#pragma unroll
    for (int i = 0; i < G::MB; ++i)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[i][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int nchunks = L.Cin_pad / CK;
    for (int cc = 0; cc < nchunks; ++cc) {
        if (cc) __syncthreads();
        // input halo of this chunk -> channel planes
        constexpr int NG = CK / 4;
        for (int it = tid; it < G::HP * G::WP * NG; it += kThreads) {
            const int p = it / NG, cg = it - p * NG;
            const int ly = p / G::WP, lx = p - ly * G::WP;
            const int gy = y0 - 1 + ly, gx = x0 - 1 + lx;
            float v[4] = {0.f, 0.f, 0.f, 0.f};
            if (gy >= 0 && gy < Hl && gx >= 0 && gx < Wl)
                fetch4<MODE, SrcT>(L, fd, s0, s1, gy, gx, Wl, cc * CK + cg * 4, v);
#pragma unroll
            for (int j = 0; j < 4; ++j) As[(cg * 4 + j) * G::PL + p] = v[j];
        }
        // weight slice [9*CK][16*NB]
        const float *wsrc = reinterpret_cast<const float *>(L.w) +
                            (size_t)cc * 9 * CK * L.Cout_pad + g * NB * 16;
        for (int it = tid; it < 9 * CK * NB * 4; it += kThreads) {
            const int e = it / (NB * 4), q = it - e * (NB * 4);
            const float4 v = *reinterpret_cast<const float4 *>(wsrc + (size_t)e * L.Cout_pad + q * 4);
            float *d = &Bs[e * G::BS + q * 4];
            d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
        }
        __syncthreads();

#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap % 3;
#pragma unroll
            for (int c4 = 0; c4 < CK / 4; ++c4) {
                float b[NB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    b[nb] = Bs[(tap * CK + c4 * 4 + lk) * G::BS + nb * 16 + lj];
#pragma unroll
                for (int i = 0; i < G::MB; ++i) {
                    const int blk = wave * G::MB + i, row = blk >> 1, cb = blk & 1;
                    const float a = As[(c4 * 4 + lk) * G::PL + (row + dy) * G::WP + cb * 16 + lj + dx];
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[i][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[nb], acc[i][nb], 0, 0, 0);
                }
            }
        }
    }

    // epilogue: lane holds channel lj of pixels 4*lk + v of each 16-px block
    OutT *dst = conv_dst<OutT>(L, fd);
#pragma unroll
    for (int i = 0; i < G::MB; ++i) {
        const int blk = wave * G::MB + i, row = blk >> 1, cb = blk & 1;
        const int y = y0 + row;
        if (y >= Hl) continue;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int co = g * NB * 16 + nb * 16 + lj;
            if (co >= L.Cout) continue;
            const float bias = L.bias[co];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int x = x0 + cb * 16 + lk * 4 + v;
                if (x >= Wl) continue;
                const float val = epilogue<EPI>(acc[i][nb][v] + bias, co, L.M);
                Elem<OutT>::store(dst + ((size_t)y * Wl + x) * L.Cout + co, val);
            }
        }
    }
}

// =============================================================================
// bf16 form
// =============================================================================
// LDS input: pixel-major rows of CK bf16 channels plus 8 padding channels,
// so the byte stride of a pixel is 2*(CK+8): for CK = 32 that is 80 bytes,
// which spreads the 16-byte fragment reads of 8 consecutive pixels over all
// banks.  A fragment for 16x16x32: lane (i = l%16, q = l/16) holds 8
// consecutive K values; the K order inside a chunk is (tap, channel) with the
// channel fastest, and each MFMA covers 32 consecutive K values: 4 runs of 8
// channels.  For CK = 16 (the 10-channel network input padded) one MFMA
// spans two taps.
template <int TH, int CK, int NB>
struct BF16Geom {
    static constexpr int TW = kConvTW, HP = TH + 2, WP = TW + 2;
    static constexpr int PS = CK + 8;                 // pixel stride (bf16 elements)
    static constexpr int KE = 9 * CK;                 // K values per chunk
    static constexpr int NK = (KE + 31) / 32;         // MFMAs per chunk (K padded)
    static constexpr int BSK = NK * 32 + 8;           // weight: per output channel, K run + pad
    static constexpr int MB = TH / 2;
};

template <int MODE, int EPI, int TH, int CK, int NB, typename SrcT, typename OutT>
__global__ __launch_bounds__(kThreads) void conv3x3_bf16_kernel(ConvLayer L, FrameArg fa)
{
    using G = BF16Geom<TH, CK, NB>;
    __shared__ __attribute__((aligned(16))) unsigned short As[G::HP * G::WP * G::PS];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[NB * 16 * G::BSK];

    int f, g, x0, y0, Hl, Wl;
    if (!conv_locate<TH>(L, fa, f, g, x0, y0, Hl, Wl)) return;
    const FrameDesc &fd = frame_at(fa, f);
    const SrcT *s0 = reinterpret_cast<const SrcT *>(L.src0_kind ? fd.u[L.src0_idx] : fd.e[L.src0_idx]);
    const SrcT *s1 = reinterpret_cast<const SrcT *>(fd.e[L.src1_idx]);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lj = lane & 15, lq = lane >> 4;

    f32x4 acc[G::MB][NB];
#pragma unroll
    for (int i = 0; i < G::MB; ++i)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[i][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int nchunks = L.Cin_pad / CK;
    for (int cc = 0; cc < nchunks; ++cc) {
        if (cc) __syncthreads();
        constexpr int NG = CK / 4;
        for (int it = tid; it < G::HP * G::WP * NG; it += kThreads) {
            const int p = it / NG, cg = it - p * NG;
            const int ly = p / G::WP, lx = p - ly * G::WP;
            const int gy = y0 - 1 + ly, gx = x0 - 1 + lx;
            float v[4] = {0.f, 0.f, 0.f, 0.f};
            if (gy >= 0 && gy < Hl && gx >= 0 && gx < Wl)
                fetch4<MODE, SrcT>(L, fd, s0, s1, gy, gx, Wl, cc * CK + cg * 4, v);
            uint2 pk;
            pk.x = (unsigned)f32_to_bf16(v[0]) | ((unsigned)f32_to_bf16(v[1]) << 16);
            pk.y = (unsigned)f32_to_bf16(v[2]) | ((unsigned)f32_to_bf16(v[3]) << 16);
            *reinterpret_cast<uint2 *>(&As[p * G::PS + cg * 4]) = pk;
        }
        // weights: packed per chunk as [Cout_pad][NK*32] bf16 (K fastest)
        const unsigned short *wsrc = reinterpret_cast<const unsigned short *>(L.w) +
                                     ((size_t)cc * L.Cout_pad + g * NB * 16) * (G::NK * 32);
        constexpr int KV = G::NK * 32 / 8;  // 16-byte vectors per channel row
        for (int it = tid; it < NB * 16 * KV; it += kThreads) {
            const int co = it / KV, q = it - co * KV;
            const uint4 v = *reinterpret_cast<const uint4 *>(wsrc + (size_t)co * (G::NK * 32) + q * 8);
            *reinterpret_cast<uint4 *>(&Bs[co * G::BSK + q * 8]) = v;
        }
        __syncthreads();

#pragma unroll
        for (int s = 0; s < G::NK; ++s) {
            // this lane's run of 8 K values: k = s*32 + lq*8 .. +7 -> (tap, c0)
            const int k0 = s * 32 + lq * 8;
            const int tap = k0 / CK, c0 = k0 - tap * CK;
            const bool live = tap < 9;
            const int dy = live ? tap / 3 : 0, dx = live ? tap % 3 : 0;
            bf16x8 b[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const u16x8 q = *reinterpret_cast<const u16x8 *>(&Bs[(nb * 16 + lj) * G::BSK + k0]);
                b[nb] = __builtin_bit_cast(bf16x8, q);
            }
#pragma unroll
            for (int i = 0; i < G::MB; ++i) {
                const int blk = wave * G::MB + i, row = blk >> 1, cb = blk & 1;
                const int p = (row + dy) * G::WP + cb * 16 + lj + dx;
                u16x8 q = *reinterpret_cast<const u16x8 *>(&As[p * G::PS + (live ? c0 : 0)]);
                if (!live) q = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
                const bf16x8 a = __builtin_bit_cast(bf16x8, q);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[i][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[nb], acc[i][nb], 0, 0, 0);
            }
        }
    }

    OutT *dst = conv_dst<OutT>(L, fd);
#pragma unroll
    for (int i = 0; i < G::MB; ++i) {
        const int blk = wave * G::MB + i, row = blk >> 1, cb = blk & 1;
        const int y = y0 + row;
        if (y >= Hl) continue;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int co = g * NB * 16 + nb * 16 + lj;
            if (co >= L.Cout) continue;
            const float bias = L.bias[co];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int x = x0 + cb * 16 + lq * 4 + v;
                if (x >= Wl) continue;
                const float val = epilogue<EPI>(acc[i][nb][v] + bias, co, L.M);
                Elem<OutT>::store(dst + ((size_t)y * Wl + x) * L.Cout + co, val);
            }
        }
    }
}

// =============================================================================
// dispatch
// =============================================================================
constexpr int kTH = 8;
int conv_tile_rows(int) { return kTH; }

int conv_chunk(int prec, int mode, int Cin, int C0)
{
    if (mode == CONV_PACK) return prec == 0 ? 12 : 16;
    if (prec != 0 && Cin % 32 == 0 && (mode != CONV_CAT || C0 % 32 == 0)) return 32;
    return 16;
}

int conv_grid(const ConvLayer &L, int n, const int *H, const int *W)
{
    long total = 0;
    for (int f = 0; f < n; ++f) {
        const int Hl = H[f] >> L.level, Wl = W[f] >> L.level;
        total += (long)((Wl + kConvTW - 1) / kConvTW) * ((Hl + kTH - 1) / kTH) * L.groups;
    }
    return (int)total;
}

template <int MODE, int EPI, int CK, int NB, typename SrcT, typename OutT>
static void launch_one(int prec, const ConvLayer &L, const FrameArg &fa, int blocks, hipStream_t s)
{
    if (prec == 0)
        hipLaunchKernelGGL((conv3x3_f32_kernel<MODE, EPI, kTH, CK, NB, SrcT, OutT>), dim3(blocks),
                           dim3(kThreads), 0, s, L, fa);
    else
        hipLaunchKernelGGL((conv3x3_bf16_kernel<MODE, EPI, kTH, CK, NB, SrcT, OutT>), dim3(blocks),
                           dim3(kThreads), 0, s, L, fa);
}

template <int MODE, int EPI, typename SrcT, typename OutT>
static bool launch_ck_nb(int prec, const ConvLayer &L, const FrameArg &fa, int blocks, hipStream_t s)
{
#define WSKP_CASE(ck, nb)                                                   \
    if (L.CK == ck && L.NB == nb) {                                         \
        launch_one<MODE, EPI, ck, nb, SrcT, OutT>(prec, L, fa, blocks, s); \
        return true;                                                        \
    }
    if (MODE == CONV_PACK) {
        if (prec == 0) { WSKP_CASE(12, 1) WSKP_CASE(12, 2) }
        else { WSKP_CASE(16, 1) WSKP_CASE(16, 2) }
        return false;
    }
    WSKP_CASE(16, 1)
    WSKP_CASE(16, 2)
    if (prec != 0) { WSKP_CASE(32, 1) WSKP_CASE(32, 2) }
#undef WSKP_CASE
    return false;
}

template <typename SrcT, typename OutT>
static bool dispatch_typed(const ConvLayer &L, int mode, int prec, const FrameArg &fa, int blocks,
                           hipStream_t s)
{
    switch (mode) {
    case CONV_PACK: return launch_ck_nb<CONV_PACK, EPI_RELU, SrcT, OutT>(prec, L, fa, blocks, s);
    case CONV_POOL: return launch_ck_nb<CONV_POOL, EPI_RELU, SrcT, OutT>(prec, L, fa, blocks, s);
    case CONV_CAT: return launch_ck_nb<CONV_CAT, EPI_RELU, SrcT, OutT>(prec, L, fa, blocks, s);
    default: return false;
    }
}

template <typename SrcT>
static bool dispatch_head(const ConvLayer &L, int epi, int prec, const FrameArg &fa, int blocks,
                          hipStream_t s)
{
    if (epi == EPI_HEAD_EXP)
        return launch_ck_nb<CONV_PLAIN, EPI_HEAD_EXP, SrcT, float>(prec, L, fa, blocks, s);
    return launch_ck_nb<CONV_PLAIN, EPI_HEAD_SOFTPLUS, SrcT, float>(prec, L, fa, blocks, s);
}

hipError_t launch_conv(const ConvLayer &L, int mode, int epi, int prec, const FrameArg &fa,
                       int blocks, hipStream_t s)
{
    if (blocks <= 0) return hipSuccess;
    bool ok;
    if (prec == 0)
        ok = mode == CONV_PLAIN ? dispatch_head<float>(L, epi, prec, fa, blocks, s)
                                : dispatch_typed<float, float>(L, mode, prec, fa, blocks, s);
    else
        ok = mode == CONV_PLAIN ? dispatch_head<unsigned short>(L, epi, prec, fa, blocks, s)
                                : dispatch_typed<unsigned short, unsigned short>(L, mode, prec, fa, blocks, s);
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace wskp
