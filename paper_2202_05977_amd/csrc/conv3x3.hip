// Convolutions of the prediction network (Sec. 4.1, Eq. 2) as implicit
// GEMMs on the gfx950 matrix cores: 3x3, or 5x5 for a net whose convs are
// merged RepVGG blocks (Sec. 4.1, prediction phase).
//
// GEMM view of one layer: output pixels x output channels, reduction K =
// KS*KS taps x C_in (the MFMAs take the weights as their first operand, so
// each lane ends with 4 consecutive channels of one pixel, which the
// epilogue stores directly).  A workgroup (4 wave64s) owns a tile of
// TH x 32 output pixels and 16*NB output channels.  The reduction runs over
// chunks of CK input channels: the (TH+KS-1) x (32+KS-1) input halo of the
// chunk and the matching KS*KS*CK x 16*NB weight slice are staged in LDS,
// then every wave issues MFMAs over the taps.  The operation that produces the layer's
// input is fused into the staging step, so that input never exists in
// memory:
//   CONV_PACK   network input (Sec. 5.1): gamma-tonemapped radiance, albedo,
//               (normal+1)/2 and clamped scaled depth, from the raw buffers
//   CONV_POOL   2x2 mean of the finer level (encoder down path)
//   CONV_CAT    [nearest x2 upsample of the coarser level, skip] (decoder)
//   CONV_PLAIN  the map itself (the head; in the bf16 plan also the encoders
//               >= 1, whose input is the 2x2-mean copy the previous encoder's
//               epilogue wrote)
// The epilogue adds the bias and applies ReLU, or for the head the weight
// activation (softplus or exp) on channels 0..M-1 and nothing on the logits.
//
// Three arithmetic forms:
//   fp32: v_mfma_f32_16x16x4f32; LDS holds channel planes so that the 16
//         pixels x 4 channels of an A fragment are bank-conflict free.
//   bf16: v_mfma_f32_16x16x32_bf16; LDS holds pixels with 8-channel runs so
//         that each lane reads its A fragment with one 16-byte load.
//   fp8:  v_mfma_f32_16x16x128_f8f6f4 on e4m3 operands (bf16 activations in
//         memory, quantised with the layer's input scale while staging).
//   All accumulate in fp32.
#include "wskp_internal.h"

#include <type_traits>

namespace wskp {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// ---- element conversions ---------------------------------------------------
__device__ __forceinline__ float bf16_to_f32(unsigned short h)
{
    return __uint_as_float(((unsigned int)h) << 16);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// fp32 -> bf16 with round-to-nearest-even: one v_cvt_pk_bf16_f32 for a pair
__device__ __forceinline__ unsigned cvt_pk_bf16(float a, float b)
{
    return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2{a, b}), bf16x2));
}

__device__ __forceinline__ unsigned short f32_to_bf16(float f) { return (unsigned short)cvt_pk_bf16(f, 0.f); }

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
    const int lev = L.level, groups = L.groups;
    auto tiles = [=](int H, int W) {
        return (((W >> lev) + kConvTW - 1) / kConvTW) * (((H >> lev) + TH - 1) / TH) * groups;
    };
    int n;
    int t = batch_tile_id(fa, blockIdx.x, gridDim.x, n);
    if (t < 0) return false;
    f = batch_frame(fa, n, t, tiles);
    if (f < 0) return false;
    const FrameDesc &fd = frame_at(fa, f);
    Hl = fd.H >> lev;
    Wl = fd.W >> lev;
    const int txn = (Wl + kConvTW - 1) / kConvTW;
    g = t % groups;
    t /= groups;
    x0 = (t % txn) * kConvTW;
    y0 = (t / txn) * TH;
    return true;
}

// ---- fast transcendental helpers -------------------------------------------
// v_exp_f32 / v_log_f32 compute 2^x and log2(x) to about 1 ulp for normal
// inputs.  log1p uses the compensated form log(u) * t / (u - 1), u = 1 + t,
// which removes the rounding of 1 + t (Goldberg's method), so the result keeps
// full relative accuracy for small t.
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

__device__ __forceinline__ float log1p_small(float t)
{
    const float u = 1.f + t;
    if (u == 1.f) return t;
    // t / (u - 1) is 1 up to the rounding of u: the hardware reciprocal
    // (1 ulp) instead of an IEEE division
    return fast_log2(u) * 0.69314718055994531f * (t * __builtin_amdgcn_rcpf(u - 1.f));
}

// softplus(x) = max(x, 0) + log(1 + e^{-|x|})
__device__ __forceinline__ float softplus_f(float x)
{
    const float t = fast_exp2(-fabsf(x) * 1.4426950408889634f);
    return fmaxf(x, 0.f) + log1p_small(t);
}

template <int EPI>
__device__ __forceinline__ float epilogue(float v, int co, int M)
{
    if (EPI == EPI_RELU) return fmaxf(v, 0.f);
    // exp weights: the raw pre-activation is stored; the decode takes the
    // exponential with a per-tile shift (no overflow for any finite h)
    if (co < M && EPI == EPI_HEAD_SOFTPLUS) return softplus_f(v);
    return v;
}

__device__ __forceinline__ const void *conv_src0(const ConvLayer &L, const FrameDesc &fd)
{
    return L.src0_kind == 0 ? fd.e[L.src0_idx] : (L.src0_kind == 1 ? fd.u[L.src0_idx] : fd.p[L.src0_idx]);
}

template <typename OutT>
__device__ __forceinline__ OutT *conv_dst(const ConvLayer &L, const FrameDesc &fd)
{
    if (L.out_kind == 2) return reinterpret_cast<OutT *>(fd.head);
    return reinterpret_cast<OutT *>(L.out_kind ? fd.u[L.out_idx] : fd.e[L.out_idx]);
}

__device__ __forceinline__ unsigned pack2(float a, float b)
{
    return cvt_pk_bf16(a, b);
}

typedef int i32x8 __attribute__((ext_vector_type(8)));

// Four floats -> four OCP e4m3 bytes (round to nearest even), saturated to
// the largest finite magnitude 448 first so that no value becomes NaN.
__device__ __forceinline__ unsigned fp8x4(float a, float b, float c, float d)
{
    const float m = 448.f;
    a = fminf(fmaxf(a, -m), m);
    b = fminf(fmaxf(b, -m), m);
    c = fminf(fmaxf(c, -m), m);
    d = fminf(fmaxf(d, -m), m);
    int r = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    r = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, r, true);
    return (unsigned)r;
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 g_u32x4;
// 16-byte load through a global-address-space pointer (a global_load
// instead of a flat load).
__device__ __forceinline__ uint4 gload16(const void *p)
{
    const u32x4 v = *(g_u32x4 *)(p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// Network input of Sec. 5.1 at one pixel: [T(r) 3, a 3, (n+1)/2 3, depth 1],
// T(x) = clamp(x,0,1)^(1/gamma) = 2^(log2(x)/gamma), depth scaled to [0,1]
// and clamped.  pack_load only loads the raw values (so that the loads of
// every item are in flight before any result is used); pack_transform maps
// them in place.
__device__ __forceinline__ void pack_load(const FrameDesc &fd, size_t pix, float x[10])
{
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        x[ch] = gload(fd.r + pix * 3 + ch);
        x[3 + ch] = gload(fd.a + pix * 3 + ch);
        x[6 + ch] = gload(fd.n + pix * 3 + ch);
    }
    x[9] = gload(fd.d + pix);
}

__device__ __forceinline__ void pack_transform(const ConvLayer &L, float x[10])
{
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        x[ch] = fast_exp2(fast_log2(fminf(fmaxf(x[ch], 0.f), 1.f)) * L.inv_gamma);
        x[6 + ch] = (x[6 + ch] + 1.f) * 0.5f;
    }
    x[9] = fminf(fmaxf((x[9] - L.dnear) * L.dinv, 0.f), 1.f);
}

// =============================================================================
// Staging of one reduction chunk: the (TH+KS-1) x (32+KS-1) input halo
// (virtual channels [cc*CK, cc*CK+CK)) and the weight slice.  init() computes each
// item's source offsets once; fetch() only issues global loads into
// registers (and, for pooling, averages them); commit() writes the registers
// to LDS.  The main loop fetches chunk cc+1 while the MFMAs of chunk cc run.
// =============================================================================
template <int PREC, int MODE, int CK, int TH, int NB, typename SrcT, int KS>
struct Stage {
    static constexpr bool BF = PREC == 1;       // bf16 operands
    static constexpr bool F8 = PREC == 2;       // fp8 (e4m3) operands, bf16 activations in HBM
    static constexpr int KR = KS / 2;           // halo width
    static constexpr int TW = kConvTW, HP = TH + KS - 1, WP = TW + KS - 1;
    // input items: a 16-byte run of one pixel's channels (PACK: one pixel)
    static constexpr int G = (MODE == CONV_PACK) ? CK : 16 / (int)sizeof(SrcT);
    static constexpr int NG = CK / G;
    static constexpr int TOT = HP * WP * NG;
    static constexpr int IT = (TOT + kThreads - 1) / kThreads;
    static constexpr int RW = (MODE == CONV_PACK) ? (BF || F8 ? 2 : 3) : 1;  // 16-byte words per item
    // LDS geometry
    static constexpr int PL = ((HP * WP - 16 + 31) / 32) * 32 + 16;     // fp32 plane stride
    static constexpr int PS = CK + 8;                                    // bf16 pixel stride (elements)
    static constexpr int PS8 = CK + 16;                                  // fp8 pixel stride (bytes)
    static constexpr int KE = KS * KS * CK;
    static constexpr int NR = KE / 32;                                   // fp8: runs of 32 K values
    static constexpr int NK = F8 ? (NR + 3) / 4 : (BF ? (KE + 31) / 32 : KE / 4);  // MFMAs per chunk
    static constexpr int BS = NB * 16 + ((NB % 2 == 0) ? 16 : 0);        // fp32 weight row stride
    static constexpr int BSK = NK * 32 + 8;                              // bf16 weight row stride
    static constexpr int BSK8 = NK * 128 + 16;                           // fp8 weight row stride (bytes)
    static constexpr int A_BYTES = F8 ? HP * WP * PS8 : (BF ? HP * WP * PS * 2 : CK * PL * 4);
    static constexpr int B_BYTES = F8 ? NB * 16 * BSK8 : (BF ? NB * 16 * BSK * 2 : KE * BS * 4);
    // weight items: 16 bytes of the packed chunk
    static constexpr int WTOT = F8 ? NB * 16 * NK * 8 : (BF ? NB * 16 * (BSK / 8) : KE * NB * 4);
    static constexpr int WIT = (WTOT + kThreads - 1) / kThreads;
    // per-chunk stride of the packed weights, in elements of the packed type, per output channel
    static constexpr int WCHUNK = F8 ? NK * 128 : (BF ? BSK : KE);

    uint4 in[IT][RW];
    uint4 w[WIT];
    int off0[IT], off1[IT];   // element offsets of the item in source 0 / source 1
    unsigned live;            // bit k: item k lies inside the image
    int woff[WIT];            // element offset of weight item k in chunk 0

    __device__ __forceinline__ void init(const ConvLayer &L, int g, int x0, int y0, int Hl, int Wl)
    {
        const int tid = threadIdx.x;
        live = 0;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int it = tid + k * kThreads;
            const int p = it / NG, cg = it - p * NG;
            const int ly = p / WP, lx = p - ly * WP;
            const int gy = y0 - KR + ly, gx = x0 - KR + lx;
            off0[k] = off1[k] = 0;
            if (it < TOT && gy >= 0 && gy < Hl && gx >= 0 && gx < Wl) {
                live |= 1u << k;
                if constexpr (MODE == CONV_PACK) {
                    off0[k] = gy * Wl + gx;                                    // pixel index
                } else if constexpr (MODE == CONV_PLAIN) {
                    off0[k] = (gy * Wl + gx) * L.C0 + cg * G;
                } else if constexpr (MODE == CONV_CAT) {
                    off0[k] = ((gy >> 1) * (Wl >> 1) + (gx >> 1)) * L.C0 + cg * G;
                    off1[k] = (gy * Wl + gx) * L.C1 + cg * G;
                } else {  // POOL: top-left of the 2x2 window in the finer level
                    off0[k] = ((2 * gy) * (2 * Wl) + 2 * gx) * L.C0 + cg * G;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < WIT; ++k) {
            const int it = tid + k * kThreads;
            woff[k] = 0;
            if (it < WTOT) {
                if constexpr (F8) {
                    const int co = it / (NK * 8), q = it - co * (NK * 8);
                    woff[k] = (g * NB * 16 + co) * (NK * 128) + q * 16;
                } else if constexpr (BF) {
                    // the group's padded rows are one contiguous block
                    woff[k] = g * NB * 16 * BSK + it * 8;
                } else {
                    const int e = it / (NB * 4), q = it - e * (NB * 4);
                    woff[k] = e * L.Cout_pad + g * NB * 16 + q * 4;
                }
            }
        }
    }

    __device__ __forceinline__ void fetch(const ConvLayer &L, const FrameDesc &fd, const SrcT *s0,
                                          const SrcT *s1, int cc, int Wl)
    {
        const int tid = threadIdx.x;
        const int c0 = cc * CK;
        // decoder input: the whole chunk comes from one source (CK divides C0)
        const bool from_up = (MODE != CONV_CAT) || c0 < L.C0;
        // network input: the raw values of every item (items outside the
        // image read pixel 0 and are zeroed below) are loaded first
        float raw[MODE == CONV_PACK ? IT : 1][10];
        if constexpr (MODE == CONV_PACK) {
#pragma unroll
            for (int k = 0; k < IT; ++k) pack_load(fd, (size_t)off0[k], raw[k]);
        }
#pragma unroll
        for (int k = 0; k < IT; ++k) {
#pragma unroll
            for (int q = 0; q < RW; ++q) in[k][q] = make_uint4(0, 0, 0, 0);
            if (!((live >> k) & 1u)) continue;
            if constexpr (MODE == CONV_PACK) {
                float *x = raw[k];
                pack_transform(L, x);
                if constexpr (F8) {
                    unsigned q[3];
#pragma unroll
                    for (int j = 0; j < 3; ++j) q[j] = fp8x4(x[4 * j] * L.in_qscale, x[4 * j + 1] * L.in_qscale,
                                                       j < 2 ? x[4 * j + 2] * L.in_qscale : 0.f,
                                                       j < 2 ? x[4 * j + 3] * L.in_qscale : 0.f);
                    in[k][0] = make_uint4(q[0], q[1], q[2], 0);
                    in[k][1] = make_uint4(0, 0, 0, 0);
                } else if constexpr (BF) {
                    in[k][0] = make_uint4(pack2(x[0], x[1]), pack2(x[2], x[3]), pack2(x[4], x[5]),
                                          pack2(x[6], x[7]));
                    in[k][1] = make_uint4(pack2(x[8], x[9]), 0, 0, 0);
                } else {
                    in[k][0] = make_uint4(__float_as_uint(x[0]), __float_as_uint(x[1]),
                                          __float_as_uint(x[2]), __float_as_uint(x[3]));
                    in[k][1] = make_uint4(__float_as_uint(x[4]), __float_as_uint(x[5]),
                                          __float_as_uint(x[6]), __float_as_uint(x[7]));
                    in[k][2] = make_uint4(__float_as_uint(x[8]), __float_as_uint(x[9]), 0, 0);
                }
            } else if constexpr (MODE == CONV_PLAIN) {
                in[k][0] = gload16(s0 + off0[k] + c0);
            } else if constexpr (MODE == CONV_CAT) {
                in[k][0] = from_up ? gload16(s0 + off0[k] + c0) : gload16(s1 + off1[k] + (c0 - L.C0));
            } else {  // CONV_POOL: 2x2 mean of the finer level
                const SrcT *b = s0 + off0[k] + c0;
                const size_t rs = (size_t)(2 * Wl) * L.C0;
                const uint4 q0 = gload16(b);
                const uint4 q1 = gload16(b + L.C0);
                const uint4 q2 = gload16(b + rs);
                const uint4 q3 = gload16(b + rs + L.C0);
                if constexpr (BF || F8) {
                    const unsigned *a0 = &q0.x, *a1 = &q1.x, *a2 = &q2.x, *a3 = &q3.x;
                    unsigned o[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float lo = 0.25f * (bf16_to_f32(a0[j] & 0xffff) + bf16_to_f32(a1[j] & 0xffff) +
                                                  bf16_to_f32(a2[j] & 0xffff) + bf16_to_f32(a3[j] & 0xffff));
                        const float hi = 0.25f * (bf16_to_f32(a0[j] >> 16) + bf16_to_f32(a1[j] >> 16) +
                                                  bf16_to_f32(a2[j] >> 16) + bf16_to_f32(a3[j] >> 16));
                        o[j] = pack2(lo, hi);
                    }
                    in[k][0] = make_uint4(o[0], o[1], o[2], o[3]);
                } else {
                    const float *f0 = reinterpret_cast<const float *>(&q0), *f1 = reinterpret_cast<const float *>(&q1);
                    const float *f2 = reinterpret_cast<const float *>(&q2), *f3 = reinterpret_cast<const float *>(&q3);
                    float o[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) o[j] = 0.25f * (f0[j] + f1[j] + f2[j] + f3[j]);
                    in[k][0] = make_uint4(__float_as_uint(o[0]), __float_as_uint(o[1]),
                                          __float_as_uint(o[2]), __float_as_uint(o[3]));
                }
            }
        }
        // weight slice of this chunk
        using WT = typename std::conditional<F8, unsigned char,
                   typename std::conditional<BF, unsigned short, float>::type>::type;
        const WT *wsrc = reinterpret_cast<const WT *>(L.w) + (size_t)cc * WCHUNK * L.Cout_pad;
#pragma unroll
        for (int k = 0; k < WIT; ++k)
            if (tid + k * kThreads < WTOT) w[k] = gload16(wsrc + woff[k]);
    }

    __device__ __forceinline__ void commit(void *As_, void *Bs_, float qs) const
    {
        const int tid = threadIdx.x;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int it = tid + k * kThreads;
            if (it >= TOT) continue;
            const int p = it / NG, cg = it - p * NG;
            if constexpr (F8) {
                unsigned char *As = static_cast<unsigned char *>(As_);
                if constexpr (MODE == CONV_PACK) {
                    *reinterpret_cast<uint4 *>(&As[p * PS8]) = in[k][0];
                    *reinterpret_cast<uint4 *>(&As[p * PS8 + 16]) = in[k][1];
                } else {
                    // 8 bf16 channels -> 8 scaled e4m3 bytes
                    const unsigned *v = &in[k][0].x;
                    uint2 o;
                    o.x = fp8x4(bf16_to_f32(v[0] & 0xffff) * qs, bf16_to_f32(v[0] >> 16) * qs,
                                bf16_to_f32(v[1] & 0xffff) * qs, bf16_to_f32(v[1] >> 16) * qs);
                    o.y = fp8x4(bf16_to_f32(v[2] & 0xffff) * qs, bf16_to_f32(v[2] >> 16) * qs,
                                bf16_to_f32(v[3] & 0xffff) * qs, bf16_to_f32(v[3] >> 16) * qs);
                    *reinterpret_cast<uint2 *>(&As[p * PS8 + cg * 8]) = o;
                }
            } else if constexpr (BF) {
                unsigned short *As = static_cast<unsigned short *>(As_);
#pragma unroll
                for (int q = 0; q < RW; ++q)
                    *reinterpret_cast<uint4 *>(&As[p * PS + cg * G + q * 8]) = in[k][q];
            } else {
                float *As = static_cast<float *>(As_);
#pragma unroll
                for (int q = 0; q < RW; ++q) {
                    const unsigned *v = &in[k][q].x;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int ch = cg * G + q * 4 + j;
                        if (ch < CK) As[ch * PL + p] = __uint_as_float(v[j]);
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < WIT; ++k) {
            const int it = tid + k * kThreads;
            if (it >= WTOT) continue;
            if constexpr (F8) {
                const int co = it / (NK * 8), q = it - co * (NK * 8);
                *reinterpret_cast<uint4 *>(static_cast<unsigned char *>(Bs_) + co * BSK8 + q * 16) = w[k];
            } else if constexpr (BF) {
                *reinterpret_cast<uint4 *>(static_cast<unsigned short *>(Bs_) + it * 8) = w[k];
            } else {
                const int e = it / (NB * 4), q = it - e * (NB * 4);
                *reinterpret_cast<uint4 *>(static_cast<float *>(Bs_) + e * BS + q * 4) = w[k];
            }
        }
    }
};

// One chunk's MFMAs.  fp32: KS*KS*CK/4 steps of v_mfma_f32_16x16x4f32 (K
// order tap, channel); bf16: NK steps of v_mfma_f32_16x16x32_bf16, each
// covering 32 consecutive K values as 4 runs of 8 channels (a run never
// crosses a tap because CK is a multiple of 8; for CK = 16 one MFMA spans
// two taps).
template <int PREC, int MODE, int CK, int TH, int NB, typename SrcT, int KS>
__device__ __forceinline__ void chunk_mfma(const void *As_, const void *Bs_, f32x4 (*acc)[NB])
{
    using S = Stage<PREC, MODE, CK, TH, NB, SrcT, KS>;
    constexpr int MB = TH / 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lj = lane & 15, lq = lane >> 4;
    if constexpr (PREC == 0) {
        const float *As = static_cast<const float *>(As_);
        const float *Bs = static_cast<const float *>(Bs_);
#pragma unroll
        for (int tap = 0; tap < KS * KS; ++tap) {
            const int dy = tap / KS, dx = tap % KS;
#pragma unroll
            for (int c4 = 0; c4 < CK / 4; ++c4) {
                float b[NB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) b[nb] = Bs[(tap * CK + c4 * 4 + lq) * S::BS + nb * 16 + lj];
#pragma unroll
                for (int i = 0; i < MB; ++i) {
                    const int blk = wave * MB + i, row = blk >> 1, cb = blk & 1;
                    const float a = As[(c4 * 4 + lq) * S::PL + (row + dy) * S::WP + cb * 16 + lj + dx];
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[i][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[nb], a, acc[i][nb], 0, 0, 0);
                }
            }
        }
    } else if constexpr (PREC == 2) {
        // v_mfma_f32_16x16x128_f8f6f4: lane (i, q) holds 32 consecutive K
        // values (one run of 32 channels of one tap); one MFMA = 4 runs.
        const unsigned char *As = static_cast<const unsigned char *>(As_);
        const unsigned char *Bs = static_cast<const unsigned char *>(Bs_);
#pragma unroll
        for (int s = 0; s < S::NK; ++s) {
            const int run = 4 * s + lq;
            const int k0 = run * 32;
            const int tap = k0 / CK, c0 = k0 - tap * CK;
            const bool live = run < S::NR;
            const int dy = live ? tap / KS : 0, dx = live ? tap % KS : 0;
            i32x8 b[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const unsigned char *bp = &Bs[(nb * 16 + lj) * S::BSK8 + s * 128 + lq * 32];
                const uint4 u0 = *reinterpret_cast<const uint4 *>(bp);
                const uint4 u1 = *reinterpret_cast<const uint4 *>(bp + 16);
                b[nb] = i32x8{(int)u0.x, (int)u0.y, (int)u0.z, (int)u0.w,
                              (int)u1.x, (int)u1.y, (int)u1.z, (int)u1.w};
            }
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                const int blk = wave * MB + i, row = blk >> 1, cb = blk & 1;
                const int p = (row + dy) * S::WP + cb * 16 + lj + dx;
                const unsigned char *ap = &As[p * S::PS8 + (live ? c0 : 0)];
                uint4 u0 = *reinterpret_cast<const uint4 *>(ap);
                uint4 u1 = *reinterpret_cast<const uint4 *>(ap + 16);
                if (!live) u0 = u1 = make_uint4(0, 0, 0, 0);
                const i32x8 a = i32x8{(int)u0.x, (int)u0.y, (int)u0.z, (int)u0.w,
                                      (int)u1.x, (int)u1.y, (int)u1.z, (int)u1.w};
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[i][nb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                        b[nb], a, acc[i][nb], 0, 0, 0, 0, 0, 0);
            }
        }
    } else {
        const unsigned short *As = static_cast<const unsigned short *>(As_);
        const unsigned short *Bs = static_cast<const unsigned short *>(Bs_);
#pragma unroll
        for (int s = 0; s < S::NK; ++s) {
            const int k0 = s * 32 + lq * 8;
            const int tap = k0 / CK, c0 = k0 - tap * CK;
            const bool live = tap < KS * KS;
            const int dy = live ? tap / KS : 0, dx = live ? tap % KS : 0;
            bf16x8 b[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                b[nb] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&Bs[(nb * 16 + lj) * S::BSK + k0]));
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                const int blk = wave * MB + i, row = blk >> 1, cb = blk & 1;
                const int p = (row + dy) * S::WP + cb * 16 + lj + dx;
                u16x8 q = *reinterpret_cast<const u16x8 *>(&As[p * S::PS + (live ? c0 : 0)]);
                if (!live) q = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
                const bf16x8 a = __builtin_bit_cast(bf16x8, q);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[i][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[nb], a, acc[i][nb], 0, 0, 0);
            }
        }
    }
}

// Epilogue shared by the conv kernels.  The MFMAs take the weights as their
// first operand, so in output block (i, nb) lane (j, q) holds pixel j of the
// block and the 4 consecutive output channels nb*16 + 4q .. 4q+3.  Bias (and
// the fp8 dequantisation factor) and the activation are applied in
// registers.  Activations (bf16 or fp32 NHWC): each lane writes its 4
// channels with one 8- or 16-byte store; the 4 lanes of a pixel cover 16
// contiguous channels.  The head record (fp32) is planar [2M][H][W], the
// layout the decode reads one map at a time.
//
// With L.pool_idx >= 0 (bf16 activations, a wave owning whole row pairs:
// TH >= 8) the epilogue also writes the 2x2 means of the stored (rounded)
// values to the next level, summed in the order (2y,2x), (2y,2x+1),
// (2y+1,2x), (2y+1,2x+1): the column partner is the neighbouring lane, the
// row partner is block i+2 of the same lane.
// Value held by the neighbouring lane (lane ^ 1), through a DPP quad
// permutation [1, 0, 3, 2] (a VALU move, no LDS round trip).
__device__ __forceinline__ float lane_xor1(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// Per-lane output-channel constants of the epilogue: the bias and, for fp8,
// the dequantisation factor of this lane's 4 channels in each block.
template <int PREC, int NB>
struct EpiConsts {
    float bias[NB][4], dq[NB][4];
    __device__ __forceinline__ void load(const ConvLayer &L, int g)
    {
        const int lq = (threadIdx.x & 63) >> 4;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int co = g * NB * 16 + nb * 16 + 4 * lq + v;
                bias[nb][v] = co < L.Cout ? gload(L.bias + co) : 0.f;
                dq[nb][v] = (PREC == 2 && co < L.Cout) ? gload(L.out_scale + co) : 1.f;
            }
    }
};

template <int PREC, int EPI, int TH, int NB, typename OutT>
__device__ __forceinline__ void conv_epilogue(const ConvLayer &L, const FrameDesc &fd, int g, int x0,
                                              int y0, int Hl, int Wl, f32x4 (*acc)[NB],
                                              const EpiConsts<PREC, NB> &ec)
{
    constexpr int MB = TH / 2;
    constexpr int NC = NB * 16;
    constexpr bool CAN_POOL = !std::is_same<OutT, float>::value && EPI == EPI_RELU && MB >= 4;
    // bf16 activations of an even number of blocks: stored in pairs
    constexpr bool PAIR = !std::is_same<OutT, float>::value && EPI == EPI_RELU && NB % 2 == 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lj = lane & 15, lq = lane >> 4;
    OutT *dst = conv_dst<OutT>(L, fd);
    const bool pool = CAN_POOL && L.pool_idx >= 0;
    OutT *pdst = pool ? reinterpret_cast<OutT *>(fd.p[L.pool_idx]) : nullptr;
    const auto &bias = ec.bias;
    const auto &dq = ec.dq;
    float pe[CAN_POOL ? 2 : 1][CAN_POOL ? NB : 1][4];   // even-row partial sums
    // head record: element offset of this lane's first channel plane, per block
    const size_t P = (size_t)Hl * Wl;
    size_t plane0[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) plane0[nb] = (size_t)(g * NC + nb * 16 + 4 * lq) * P;
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int blk = wave * MB + i, row = blk >> 1, cb = blk & 1;
        const int y = y0 + row, x = x0 + cb * 16 + lj;
        const bool in = y < Hl && x < Wl;
        OutT *pp = dst + ((size_t)y * Wl + x) * L.Cout;
        uint2 qs[NB];   // packed bf16 of each block (paired stores)
        uint2 pm[NB];   // packed 2x2 means of each block (odd rows, paired stores)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int co = g * NC + nb * 16 + 4 * lq;
            const bool cin = co < L.Cout;
            float v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = epilogue<EPI>(acc[i][nb][k] * dq[nb][k] + bias[nb][k], co + k, L.M);
            if constexpr (EPI == EPI_HEAD_SOFTPLUS || EPI == EPI_HEAD_EXP) {
                // head record, planar [2M][H][W]: the 16 lanes of a channel
                // write 16 consecutive pixels of its plane
                if (in) {
                    OutT *q = dst + plane0[nb] + (unsigned)(y * Wl + x);
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (co + k < L.Cout) gstore(q + k * P, v[k]);
                }
            } else if constexpr (std::is_same<OutT, float>::value) {
                // fp32 activations: Cout is a multiple of 16
                if (in && cin) gstore(reinterpret_cast<gf32x4 *>(pp + co), gf32x4{v[0], v[1], v[2], v[3]});
            } else {
                // activations: Cout is a multiple of 16
                const uint2 q = make_uint2(pack2(v[0], v[1]), pack2(v[2], v[3]));
                qs[nb] = q;
                if constexpr (!PAIR) {
                    if (in && cin) gstore(reinterpret_cast<gu32x2 *>(pp + co), gu32x2{q.x, q.y});
                }
                if constexpr (CAN_POOL) {
                    if (pool) {
                        const float r[4] = {__uint_as_float(q.x << 16), __uint_as_float(q.x & 0xffff0000u),
                                            __uint_as_float(q.y << 16), __uint_as_float(q.y & 0xffff0000u)};
                        const bool odd_row = (i >> 1) & 1;
                        if (!odd_row) {
#pragma unroll
                            for (int k = 0; k < 4; ++k) pe[cb][nb][k] = r[k] + lane_xor1(r[k]);
                        } else {
                            float m[4];
#pragma unroll
                            for (int k = 0; k < 4; ++k) m[k] = 0.25f * ((pe[cb][nb][k] + r[k]) + lane_xor1(r[k]));
                            pm[nb] = make_uint2(pack2(m[0], m[1]), pack2(m[2], m[3]));
                            if constexpr (!PAIR) {
                                const int Y = y >> 1, X = x >> 1;
                                if ((lj & 1) == 0 && Y < (Hl >> 1) && X < (Wl >> 1) && cin) {
                                    OutT *pd = pdst + ((size_t)Y * (Wl >> 1) + X) * L.Cout + co;
                                    gstore(reinterpret_cast<gu32x2 *>(pd), gu32x2{pm[nb].x, pm[nb].y});
                                }
                            }
                        }
                    }
                }
            }
        }
        if constexpr (PAIR) {
            // Blocks nb and nb+1 together: lane row q holds channels 4q..4q+3
            // of each.  v_permlane16_swap exchanges the odd rows of the first
            // operand with the even rows of the second, after which even rows
            // hold 8 consecutive channels of block nb (from rows q, q+1) and
            // odd rows 8 of block nb+1 (rows q-1, q): one 16-byte store per
            // lane, and the 4 lanes of a pixel cover its 32 channels.
#pragma unroll
            for (int nb = 0; nb < NB; nb += 2) {
                const auto s0 = __builtin_amdgcn_permlane16_swap(qs[nb].x, qs[nb + 1].x, false, false);
                const auto s1 = __builtin_amdgcn_permlane16_swap(qs[nb].y, qs[nb + 1].y, false, false);
                const int c = g * NC + ((lq & 1) ? (nb + 1) * 16 + 4 * (lq - 1) : nb * 16 + 4 * lq);
                if (in && c < L.Cout)
                    gstore(reinterpret_cast<gu32x4 *>(pp + c), gu32x4{s0[0], s1[0], s0[1], s1[1]});
                if constexpr (CAN_POOL) {
                    // the 2x2 means of a row pair, the same way (even lanes)
                    if (pool && ((i >> 1) & 1)) {
                        const auto t0 = __builtin_amdgcn_permlane16_swap(pm[nb].x, pm[nb + 1].x, false, false);
                        const auto t1 = __builtin_amdgcn_permlane16_swap(pm[nb].y, pm[nb + 1].y, false, false);
                        const int Y = y >> 1, X = x >> 1;
                        if ((lj & 1) == 0 && Y < (Hl >> 1) && X < (Wl >> 1) && c < L.Cout) {
                            OutT *pd = pdst + ((size_t)Y * (Wl >> 1) + X) * L.Cout + c;
                            gstore(reinterpret_cast<gu32x4 *>(pd), gu32x4{t0[0], t1[0], t0[1], t1[1]});
                        }
                    }
                }
            }
        }
    }
}

template <int PREC, int MODE, int EPI, int TH, int CK, int NB, typename SrcT, typename OutT, int KS = 3>
#ifndef WSKP_CONV_MIN_WG
#define WSKP_CONV_MIN_WG 1
#endif
__global__ __launch_bounds__(kThreads, (MODE == CONV_PACK && PREC == 1 && KS == 3) ? 4 : WSKP_CONV_MIN_WG) void conv3x3_kernel(ConvLayer L, FrameArg fa)
{
    using S = Stage<PREC, MODE, CK, TH, NB, SrcT, KS>;
    constexpr int MB = TH / 2;
    constexpr int LDS_BYTES = S::A_BYTES + S::B_BYTES;
    __shared__ __attribute__((aligned(16))) unsigned char smem[LDS_BYTES];
    void *As = smem;
    void *Bs = smem + S::A_BYTES;

    int f, g, x0, y0, Hl, Wl;
    if (!conv_locate<TH>(L, fa, f, g, x0, y0, Hl, Wl)) return;
    const FrameDesc &fd = frame_at(fa, f);
    const SrcT *s0 = reinterpret_cast<const SrcT *>(conv_src0(L, fd));
    const SrcT *s1 = reinterpret_cast<const SrcT *>(fd.e[L.src1_idx]);
    f32x4 acc[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[i][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

    S st;
    st.init(L, g, x0, y0, Hl, Wl);
    const int nchunks = L.Cin_pad / CK;
    st.fetch(L, fd, s0, s1, 0, Wl);
    EpiConsts<PREC, NB> ec;
    if constexpr (MODE == CONV_PACK) {
        // the network input is one chunk: the epilogue's constants are
        // requested once the staged values are in LDS (their registers are
        // free again) and the MFMAs hide their latency; the barrier waits for
        // LDS only, not for these loads
        st.commit(As, Bs, L.in_qscale);
        ec.load(L, g);
        lds_sync();
        chunk_mfma<PREC, MODE, CK, TH, NB, SrcT, KS>(As, Bs, acc);
    } else {
        for (int cc = 0; cc < nchunks; ++cc) {
            if (cc) __syncthreads();
            st.commit(As, Bs, L.in_qscale);
            __syncthreads();
            if (cc + 1 < nchunks) st.fetch(L, fd, s0, s1, cc + 1, Wl);
            chunk_mfma<PREC, MODE, CK, TH, NB, SrcT, KS>(As, Bs, acc);
        }
        ec.load(L, g);
    }

    conv_epilogue<PREC, EPI, TH, NB, OutT>(L, fd, g, x0, y0, Hl, Wl, acc, ec);
}

// =============================================================================
// bf16 decoder and head convs with direct-to-LDS buffer loads
// =============================================================================
// Every 16-byte slot of the input halo (8 bf16 channels of one pixel) and of
// the weight slice goes from memory straight into LDS with
// buffer_load_dwordx4 ... lds: no registers hold staged data and no commit
// pass rewrites it.  A wave-level load writes 64 consecutive slots, so the
// LDS image of the halo is pixel-major with 4 slots per pixel (CK = 32
// channels).  A 16-byte LDS read serves 8 lanes per cycle from 32 banks, so
// the 8 pixels a fragment read takes in one cycle must land in 8 distinct
// 16-byte bank groups of a 128-byte line: the 4 slots of pixel p hold channel
// groups in the order g ^ ((p >> 1) & 3), which with the pixel's position
// in the line (p & 1) enumerates all 8 groups for any 8 consecutive pixels.
// Each lane realises the order by choosing which group it fetches.  Pixels outside the image
// get an offset beyond the buffer's range, and the hardware returns zeros:
// that is the conv's zero padding.

#ifndef WSKP_DIRECT_SWZ
#define WSKP_DIRECT_SWZ 1
#endif
constexpr int kDirectSwz = WSKP_DIRECT_SWZ;

__device__ __forceinline__ void load_lds16(rsrc_t r, unsigned char *lds, unsigned voff)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void *)lds, 16,
                                             (int)voff, 0, 0, 0);
}

constexpr unsigned kOutOfRange = 0x7ffffff0u;

// vmcnt(N) with lgkmcnt(0): waits until at most N vector-memory loads of
// this wave are outstanding (loads complete in order); N = 0 waits for the
// direct-to-LDS loads of the stage.
template <int N>
__device__ __forceinline__ void wait_vmem()
{
    static_assert(N >= 0 && N < 64, "vmcnt is a 6-bit field");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (0 << 8));
}

// Each wave computes HW = TH/4 output rows of the tile (both 16-pixel column
// blocks, all NB output blocks).  For one column offset dx it reads the A
// fragments of its HW+KS-1 input rows once and uses each for up to KS
// vertical taps dy (input row r+dy feeds output row r), so a 3x3 chunk costs
// 6 (HW+2) A fragment reads instead of 18 HW: the LDS bytes per MFMA, which
// bound this loop, fall with HW.
// Workgroups per CU that the stage's LDS (160 KiB per CU) admits, at most
// four (at TH = 8: 40, 49 and 58 KiB for 2, 3 and 4 output blocks, so 4, 3
// and 2; 5x5 layers with one output block, 52 KiB, 3); the register budget
// is capped to match.
constexpr int direct_stage_bytes(int NB, int KS, int TH)
{
    return ((TH + KS - 1) * (kConvTW + KS - 1) * 64 + NB * 16 * KS * KS * 64 + 1023) / 1024 * 1024;
}
constexpr int direct_min_wg(int NB, int KS, int TH)
{
    return 163840 / direct_stage_bytes(NB, KS, TH) < 4 ? 163840 / direct_stage_bytes(NB, KS, TH) : 4;
}

template <int MODE, int EPI, int TH, int NB, typename OutT, int KS = 3>
__global__ __launch_bounds__(kThreads, direct_min_wg(NB, KS, TH)) void conv3x3_bf16_direct(ConvLayer L, FrameArg fa)
{
    constexpr int CK = 32, WP = kConvTW + KS - 1, HP = TH + KS - 1, NPIX = HP * WP;
    constexpr int A_SLOTS = NPIX * 4;
    constexpr int NK = KS * KS;                            // one tap (32 channels) per MFMA
    // Weight rows are unpadded (k^2 taps x 32 channels: 576 B for 3x3,
    // 1600 B for 5x5); in row co
    // the 16-byte column groups are stored XOR-ed with 2 * ((co >> 2) & 1)
    // (host packing), so the 16 rows x 4 groups of a B-fragment read fall
    // on distinct banks (a 592-byte padded row costs 4 extra LDS cycles per
    // read on gfx950).
    constexpr int BSK = NK * 32;
    constexpr int B_SLOTS = NB * 16 * BSK / 8;
    // The stage is one array of 16-byte slots, halo first, weights right
    // after it; load instruction j fills slots [64j, 64j + 64).  The
    // instruction that straddles the boundary is issued twice, once per
    // source, each with only its own lanes active.
    constexpr int SLOTS = A_SLOTS + B_SLOTS;
    constexpr int INS = (SLOTS + 63) / 64;
    constexpr int PW = (INS + 3) / 4;                      // load instructions per wave
    constexpr int A_BYTES = A_SLOTS * 16, STAGE = INS * 1024;
    static_assert(STAGE == direct_stage_bytes(NB, KS, TH), "stage size");
    constexpr int MB = TH / 2, NC = NB * 16, HW = TH / 4;
    static_assert(TH % 4 == 0, "each wave owns TH/4 whole rows");
    __shared__ __attribute__((aligned(1024))) unsigned char smem[STAGE];

    int f, g, x0, y0, Hl, Wl;
    if (!conv_locate<TH>(L, fa, f, g, x0, y0, Hl, Wl)) return;
    const FrameDesc &fd = frame_at(fa, f);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lj = lane & 15, lq = lane >> 4;
    const int bq = lq ^ (((lj >> 2) & 1) << 1);   // swizzled weight column group

    const unsigned short *s0 =
        reinterpret_cast<const unsigned short *>(conv_src0(L, fd));
    const unsigned short *s1 = reinterpret_cast<const unsigned short *>(fd.e[L.src1_idx]);
    const int H0 = MODE == CONV_CAT ? Hl >> 1 : Hl, W0 = MODE == CONV_CAT ? Wl >> 1 : Wl;
    const rsrc_t r0 = make_rsrc(s0, (unsigned)((size_t)H0 * W0 * L.C0 * 2));
    const rsrc_t r1 = make_rsrc(s1, MODE == CONV_CAT ? (unsigned)((size_t)Hl * Wl * L.C1 * 2) : 0u);
    const int nchunks = L.Cin_pad / CK;
    const rsrc_t rw = make_rsrc(L.w, (unsigned)((size_t)nchunks * L.Cout_pad * BSK * 2));

    // byte offsets of this wave's A slots in source 0 and source 1 (chunk 0).
    // The lane's k-th slot is slot0 + 256 k: halo pixel p0 + 64 k with the
    // same channel group (adding 64 leaves bits 1-2 of the pixel index
    // unchanged), so its row and column step by the quotient and remainder
    // of 64 / WP.  Row and pixel pitches are below 2^24, so the products are
    // 24-bit multiplies (full rate, unlike 32-bit ones).
    const unsigned cp0 = (unsigned)L.C0 * 2u, rp0 = (unsigned)W0 * cp0;
    const unsigned cp1 = (unsigned)L.C1 * 2u, rp1 = (unsigned)Wl * cp1;
    const int slot0 = wave * 64 + lane, p0 = slot0 >> 2;
    const unsigned goff = (unsigned)(((slot0 & 3) ^ ((p0 >> kDirectSwz) & 3)) * 16);
    constexpr int SY = 64 / WP, SX = 64 - SY * WP;
    int ly = p0 / WP, lx = p0 - ly * WP;
    unsigned oa0[PW], oa1[PW];
#pragma unroll
    for (int k = 0; k < PW; ++k) {
        const int gy = y0 - KS / 2 + ly, gx = x0 - KS / 2 + lx;
        const bool in = p0 + 64 * k < NPIX && (unsigned)gy < (unsigned)Hl && (unsigned)gx < (unsigned)Wl;
        if (MODE == CONV_CAT) {
            oa0[k] = in ? __umul24((unsigned)gy >> 1, rp0) + __umul24((unsigned)gx >> 1, cp0) + goff : kOutOfRange;
            oa1[k] = in ? __umul24((unsigned)gy, rp1) + __umul24((unsigned)gx, cp1) + goff : kOutOfRange;
        } else {
            oa0[k] = in ? __umul24((unsigned)gy, rp0) + __umul24((unsigned)gx, cp0) + goff : kOutOfRange;
            oa1[k] = kOutOfRange;
        }
        lx += SX;
        ly += SY;
        if (lx >= WP) {
            lx -= WP;
            ++ly;
        }
    }

    // issues chunk cc's halo and weight slices into the stage at `buf`
    auto issue = [&](int cc, unsigned char *buf) {
        const int c0 = cc * CK;
        const bool up = MODE != CONV_CAT || c0 < L.C0;
        const unsigned da = (unsigned)((up ? c0 : c0 - L.C0) * 2);
        const unsigned wb = (unsigned)((cc * L.Cout_pad + g * NC) * BSK * 2);
#pragma unroll
        for (int k = 0; k < PW; ++k) {
            const int ins = wave + 4 * k;
            if (ins >= INS) break;
            const int slot = ins * 64 + lane;
            unsigned char *dst = buf + ins * 1024;
            if (ins * 64 < A_SLOTS && slot < A_SLOTS) {
                if (up) load_lds16(r0, dst, oa0[k] + da);
                else load_lds16(r1, dst, oa1[k] + da);
            }
            if (ins * 64 + 64 > A_SLOTS && slot >= A_SLOTS && slot < SLOTS)
                load_lds16(rw, dst, wb + (unsigned)((slot - A_SLOTS) * 16));
        }
    };

    f32x4 acc[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[i][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

    // MFMAs of one chunk from the stage at As (halo) / As + A_BYTES (weights)
    auto compute = [&](const unsigned char *As) {
        const unsigned char *Bs = As + A_BYTES;
#pragma unroll
        for (int dx = 0; dx < KS; ++dx) {
            bf16x8 a[HW + KS - 1][2];
#pragma unroll
            for (int rr = 0; rr < HW + KS - 1; ++rr)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) {
                    const int p = (wave * HW + rr) * WP + cb * 16 + lj + dx;
                    const int slot = p * 4 + (lq ^ ((p >> kDirectSwz) & 3));
                    a[rr][cb] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(As + slot * 16));
                }
#pragma unroll
            for (int dy = 0; dy < KS; ++dy) {
                const int s = dy * KS + dx;
                bf16x8 b[NB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    b[nb] = __builtin_bit_cast(
                        bf16x8, *reinterpret_cast<const u16x8 *>(Bs + ((nb * 16 + lj) * BSK + s * 32 + bq * 8) * 2));
#pragma unroll
                for (int r = 0; r < HW; ++r)
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb)
                            acc[2 * r + cb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                b[nb], a[r + dy][cb], acc[2 * r + cb][nb], 0, 0, 0);
            }
        }
    };

    issue(0, smem);
    for (int cc = 0; cc < nchunks; ++cc) {
        wait_vmem<0>();
        lds_barrier();
        compute(smem);
        wait_lds();
        lds_barrier();   // the stage has been read before it is refilled
        if (cc + 1 < nchunks) issue(cc + 1, smem);
    }
    EpiConsts<1, NB> ec;
    ec.load(L, g);
    conv_epilogue<1, EPI, TH, NB, OutT>(L, fd, g, x0, y0, Hl, Wl, acc, ec);
}

// =============================================================================
// dispatch
// =============================================================================
// Output rows per conv tile (build-time tuning knobs): kTH for the kernels
// that stage through registers, kTHD (a multiple of 4) for the direct-load
// bf16 kernel.
#ifndef WSKP_CONV_TH
#define WSKP_CONV_TH 4
#endif
#ifndef WSKP_DIRECT_TH
#define WSKP_DIRECT_TH 8
#endif
#ifndef WSKP_CONV_DIRECT
#define WSKP_CONV_DIRECT 1
#endif
constexpr int kTH = WSKP_CONV_TH;
// the network-input layer (one reduction chunk) gets its own knob
#ifndef WSKP_PACK_TH
#define WSKP_PACK_TH 8
#endif
constexpr int kTHP = WSKP_PACK_TH;
constexpr int kTHD = WSKP_DIRECT_TH;

static bool uses_direct(int prec, int mode, int CK, int ks)
{
    return WSKP_CONV_DIRECT && (ks == 3 || ks == 5) && prec == 1 && CK == 32 &&
           (mode == CONV_CAT || mode == CONV_PLAIN);
}

bool conv_uses_direct(int prec, int mode, int CK, int ks) { return uses_direct(prec, mode, CK, ks); }

// Tile rows per layer: the input layer uses kTHP; the direct-load kernel uses
// kTHD, or 4 rows (and one output block per workgroup) on the levels from
// WSKP_COARSE_LEVEL on, which have few pixels, so that they still spread
// over all CUs, unless the layer passes on 2x2 means (that needs whole row
// pairs per wave, 8 rows).  From level 4: with level 3 on 4-row tiles too
// (the fourth level of the 720p net, 160 x 90) one frame's launch was
// slightly faster alone but three-stream throughput 1 % lower.
#ifndef WSKP_COARSE_LEVEL
#define WSKP_COARSE_LEVEL 4
#endif
int conv_tile_rows(int prec, int mode, int CK, int level, bool pool, int ks)
{
    if (mode == CONV_PACK) return kTHP;
    if (!uses_direct(prec, mode, CK, ks)) return kTH;
    return (level >= WSKP_COARSE_LEVEL && !pool) ? 4 : kTHD;
}

int conv_chunk(int prec, int mode, int Cin, int C0)
{
    if (prec == 2) return 32;   // fp8: runs of 32 channels (the network input padded to 32)
    if (mode == CONV_PACK) return prec == 0 ? 12 : 16;
    if (prec != 0 && Cin % 32 == 0 && (mode != CONV_CAT || C0 % 32 == 0)) return 32;
    return 16;
}

#ifndef WSKP_CONV_MAX_NB
#define WSKP_CONV_MAX_NB 4
#endif
#ifndef WSKP_DIRECT_MAX_NB
#define WSKP_DIRECT_MAX_NB 2
#endif
// Wider groups stage and read each input tile fewer times (the A operand is
// reused across NB blocks); narrower groups give more workgroups and a
// smaller stage, so more of them fit a CU.  The direct-load kernel measured
// fastest with at most two blocks (stage <= 40 KiB, four workgroups per CU)
// and one block on the coarsest levels.  5x5 layers take one block per
// group: their weight slices are 25/9 times larger.
int conv_blocks_per_group(int prec, int mode, int CK, int nblk, int level, int ks)
{
    if (ks != 3) return 1;
    if (mode == CONV_PACK) return nblk % 2 == 0 ? 2 : 1;
    const bool direct = uses_direct(prec, mode, CK, ks);
    if (direct && level >= WSKP_COARSE_LEVEL) return 1;
    for (int nb = direct ? WSKP_DIRECT_MAX_NB : WSKP_CONV_MAX_NB; nb > 1; --nb)
        if (nb <= 4 && nblk % nb == 0) return nb;
    return 1;
}

int conv_grid(const ConvLayer &L, int n, const int *H, const int *W)
{
    long total = 0;
    for (int f = 0; f < n; ++f) {
        const int Hl = H[f] >> L.level, Wl = W[f] >> L.level;
        total += (long)((Wl + kConvTW - 1) / kConvTW) * ((Hl + L.th - 1) / L.th) * L.groups;
    }
    return (int)total;
}

template <int PREC, int MODE, int EPI, int CK, int NB, typename OutT>
static void launch_one(const ConvLayer &L, const FrameArg &fa, int blocks, hipStream_t s)
{
    using SrcT = typename std::conditional<PREC == 0, float, unsigned short>::type;
    constexpr int TH = MODE == CONV_PACK ? kTHP : kTH;
    if constexpr (WSKP_CONV_DIRECT && NB == 1 && PREC == 1 && CK == 32 && (MODE == CONV_CAT || MODE == CONV_PLAIN)) {
        if (L.ks == 5) {
            if (L.th == 4)
                hipLaunchKernelGGL((conv3x3_bf16_direct<MODE, EPI, 4, 1, OutT, 5>), dim3(blocks), dim3(kThreads), 0, s,
                                   L, fa);
            else
                hipLaunchKernelGGL((conv3x3_bf16_direct<MODE, EPI, kTHD, 1, OutT, 5>), dim3(blocks), dim3(kThreads),
                                   0, s, L, fa);
            return;
        }
    }
    if constexpr (NB == 1 && PREC != 2) {
        if (L.ks == 5) {
            hipLaunchKernelGGL((conv3x3_kernel<PREC, MODE, EPI, TH, CK, NB, SrcT, OutT, 5>), dim3(blocks),
                               dim3(kThreads), 0, s, L, fa);
            return;
        }
    }
    if constexpr (WSKP_CONV_DIRECT && PREC == 1 && CK == 32 && (MODE == CONV_CAT || MODE == CONV_PLAIN)) {
        if (L.th == 4)
            hipLaunchKernelGGL((conv3x3_bf16_direct<MODE, EPI, 4, NB, OutT>), dim3(blocks),
                               dim3(kThreads), 0, s, L, fa);
        else
            hipLaunchKernelGGL((conv3x3_bf16_direct<MODE, EPI, kTHD, NB, OutT>), dim3(blocks),
                               dim3(kThreads), 0, s, L, fa);
        return;
    }
    // fp32 activations travel with the fp32 MFMA form; the bf16 and fp8 forms
    // keep bf16 activations in memory
    hipLaunchKernelGGL((conv3x3_kernel<PREC, MODE, EPI, TH, CK, NB, SrcT, OutT>), dim3(blocks),
                       dim3(kThreads), 0, s, L, fa);
}

// Chunk sizes: fp32 uses CK = 12 (network input) or 16; bf16 uses 16 (input
// padded from 10) or 32 where the channel counts allow it.
template <int PREC, int MODE, int EPI, typename OutT>
static bool launch_ck_nb(const ConvLayer &L, const FrameArg &fa, int blocks, hipStream_t s)
{
#define WSKP_CASE(ck, nb)                                                   \
    if (L.CK == ck && L.NB == nb) {                                         \
        launch_one<PREC, MODE, EPI, ck, nb, OutT>(L, fa, blocks, s);       \
        return true;                                                        \
    }
    if constexpr (PREC == 2) {
        WSKP_CASE(32, 1) WSKP_CASE(32, 2)
        if constexpr (MODE != CONV_PACK && MODE != CONV_PLAIN) { WSKP_CASE(32, 3) WSKP_CASE(32, 4) }
    } else if constexpr (MODE == CONV_PACK) {
        if constexpr (PREC == 0) { WSKP_CASE(12, 1) WSKP_CASE(12, 2) }
        else { WSKP_CASE(16, 1) WSKP_CASE(16, 2) }
    } else if constexpr (MODE == CONV_PLAIN) {
        WSKP_CASE(16, 1)
        if constexpr (PREC == 0 && EPI == EPI_LINEAR) { WSKP_CASE(16, 2) WSKP_CASE(16, 4) }
        if constexpr (PREC != 0) { WSKP_CASE(32, 1) }
        if constexpr (PREC == 1 && EPI == EPI_RELU) { WSKP_CASE(32, 2) WSKP_CASE(32, 3) WSKP_CASE(32, 4) }
    } else {
        WSKP_CASE(16, 1) WSKP_CASE(16, 2) WSKP_CASE(16, 3) WSKP_CASE(16, 4)
        if constexpr (PREC != 0) { WSKP_CASE(32, 1) WSKP_CASE(32, 2) WSKP_CASE(32, 3) WSKP_CASE(32, 4) }
    }
#undef WSKP_CASE
    return false;
}

template <int PREC>
static bool dispatch(const ConvLayer &L, int mode, int epi, const FrameArg &fa, int blocks,
                     hipStream_t s)
{
    using ActT = typename std::conditional<PREC == 0, float, unsigned short>::type;
    switch (mode) {
    case CONV_PACK: return launch_ck_nb<PREC, CONV_PACK, EPI_RELU, ActT>(L, fa, blocks, s);
    case CONV_POOL: return launch_ck_nb<PREC, CONV_POOL, EPI_RELU, ActT>(L, fa, blocks, s);
    case CONV_CAT: return launch_ck_nb<PREC, CONV_CAT, EPI_RELU, ActT>(L, fa, blocks, s);
    case CONV_PLAIN:
        // encoders on pooled maps (bf16); the head record is fp32 in every precision
        if (epi == EPI_RELU) return launch_ck_nb<PREC, CONV_PLAIN, EPI_RELU, ActT>(L, fa, blocks, s);
        if constexpr (PREC == 0) {
            // training: the input gradient of a conv, fp32 NHWC
            if (epi == EPI_LINEAR) return launch_ck_nb<PREC, CONV_PLAIN, EPI_LINEAR, float>(L, fa, blocks, s);
        }
        if (epi == EPI_HEAD_EXP) return launch_ck_nb<PREC, CONV_PLAIN, EPI_HEAD_EXP, float>(L, fa, blocks, s);
        return launch_ck_nb<PREC, CONV_PLAIN, EPI_HEAD_SOFTPLUS, float>(L, fa, blocks, s);
    default: return false;
    }
}

hipError_t launch_conv(const ConvLayer &L, int mode, int epi, int prec, const FrameArg &fa,
                       int blocks, hipStream_t s)
{
    if (blocks <= 0) return hipSuccess;
    // 5x5 layers run the register-staged kernel with one block per group
    if (L.ks != 3 && (L.ks != 5 || L.NB != 1 || prec == 2)) return hipErrorInvalidValue;
    const bool ok = prec == 0   ? dispatch<0>(L, mode, epi, fa, blocks, s)
                    : prec == 1 ? dispatch<1>(L, mode, epi, fa, blocks, s)
                                : dispatch<2>(L, mode, epi, fa, blocks, s);
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace wskp
