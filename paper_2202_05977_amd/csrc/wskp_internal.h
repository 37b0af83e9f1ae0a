// Internal declarations shared by the HIP kernels and the C ABI layer of
// libwskp.  Not part of the public interface (include/wskp.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace wskp {

constexpr int kMaxLevels = 6;
constexpr int kMaxKernels = 8;
constexpr int kThreads = 256;  // every kernel runs 4 wave64s per workgroup

// Everything one frame's layers need: its size, the caller's input and
// output buffers, and where its intermediate maps sit in the workspace.
struct FrameDesc {
    int H, W;
    const float *r, *a, *n, *d;  // radiance, albedo, normal [H,W,3]; depth [H,W,1]
    float *out;                  // [H,W,3]
    void *e[kMaxLevels];         // encoder outputs e_l  [H>>l, W>>l, C_l]
    void *u[kMaxLevels];         // decoder outputs u_l  [H>>l, W>>l, C_l]; u[L-1] == e[L-1]
    void *p[kMaxLevels];         // bf16 form: 2x2 means of e_l [H>>(l+1), W>>(l+1), C_l]
    float *head;                 // [H,W,2M]: weights W_i then logits
};

// Global-memory access through address-space-1 pointers.  Pointers that
// reach a kernel inside a structure are generic, and generic (flat)
// accesses also count against the LDS wait counter: every wait for an LDS
// read would then also wait for the global loads still in flight.
template <typename T>
__device__ __forceinline__ T gload(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ void gstore(T *p, T v)
{
    *(__attribute__((address_space(1))) T *)p = v;
}
typedef float gf32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int gu32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int gu32x4 __attribute__((ext_vector_type(4)));

// Workgroup barrier without the memory fence of __syncthreads(): the fence
// waits for every global load in flight (prefetches included).  Callers make
// the data they need visible explicitly (wait_lds / a vmcnt wait before the
// barrier); the empty asm statements keep the compiler from moving memory
// accesses across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// lgkmcnt(0): this wave's LDS reads and writes have completed.
__device__ __forceinline__ void wait_lds() { __builtin_amdgcn_s_waitcnt((15) | (3 << 14) | (7 << 4) | (0 << 8)); }

// Barrier for LDS producer/consumer phases: this wave's LDS accesses are
// complete, then every wave of the workgroup has arrived.  Global loads
// stay in flight.
__device__ __forceinline__ void lds_sync()
{
    wait_lds();
    lds_barrier();
}

// A batch of frames for one launch: either one frame passed by value or a
// device-resident table of n frames.
struct FrameArg {
    const FrameDesc *table;  // device pointer, or nullptr to use `one`
    int n;
    int reverse;             // walk tiles in reverse order
    // capacity launch (graph replay): when non-null, dev_n[0] is the frame
    // count and dev_n[1 + launch] this launch's tile count, both in device
    // memory, and the grid is an upper bound on those tiles; workgroups
    // beyond them exit
    const int *dev_n;
    int launch;
    FrameDesc one;
};

__device__ __forceinline__ const FrameDesc &frame_at(const FrameArg &fa, int f)
{
    return fa.table ? fa.table[f] : fa.one;
}

// Raw buffer resource over `bytes` bytes at `base`.  Loads through it
// whose offset lies beyond `bytes` return zeros.  The descriptor must live
// in scalar registers: base and size are made visibly wave-uniform (the
// callers pass wave-uniform values).
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, unsigned bytes)
{
    const unsigned long long b = reinterpret_cast<unsigned long long>(base);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    void *ub = reinterpret_cast<void *>(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(ub, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes),
                                             0x00020000);
}

// Spread consecutive logical tile ids over one XCD.  The hardware deals
// workgroups round-robin to the 8 XCDs (block b runs on XCD b % 8); this
// bijection gives each XCD a contiguous run of logical ids so that tiles
// that share halos (and output-channel groups that share an input tile)
// share that XCD's L2.
__device__ __forceinline__ int xcd_logical_id(int b, int nb)
{
    const int x = b & 7, i = b >> 3;
    const int q = nb >> 3, rmd = nb & 7;
    return x * q + (x < rmd ? x : rmd) + i;
}

// Finds the frame of a batch that holds logical tile t, given the tile
// count of a frame of size H x W, and rewrites t as the tile index inside
// that frame.  Each lane reads one frame's size, a wave-wide inclusive scan
// turns the counts into cumulative ends, and a ballot counts the frames
// that end at or before t: one round of loads per 64 frames instead of one
// dependent load per frame.  Returns -1 past the batch's last tile.  Every
// lane of the wave calls it with the same t; the results are wave-uniform.
template <typename Count>
__device__ __forceinline__ int batch_frame(const FrameArg &fa, int n, int &t, Count count)
{
    if (!fa.table) return t < count(fa.one.H, fa.one.W) ? 0 : -1;
    const int lane = threadIdx.x & 63;
    int base = 0;
    for (int f0 = 0; f0 < n; f0 += 64) {
        const int f = f0 + lane;
        int c = f < n ? count(gload(&fa.table[f].H), gload(&fa.table[f].W)) : 0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(c, d, 64);
            if (lane >= d) c += v;
        }
        const int end = base + c;
        const int k = __popcll(__ballot(f < n && end <= t));
        const int valid = n - f0 < 64 ? n - f0 : 64;
        if (k < valid) {
            t = __builtin_amdgcn_readfirstlane(t - (k > 0 ? __shfl(end, k - 1, 64) : base));
            return __builtin_amdgcn_readfirstlane(f0 + k);
        }
        base = __shfl(end, 63, 64);
    }
    return -1;
}

// Logical tile of workgroup b of a launch of nb workgroups, and the batch's
// frame count n.  Capacity launches read n and the launch's tile count from
// device memory (one load round: the two words share a cache line); there
// the tile count is below nb, and workgroups beyond it get -1.  Then the
// XCD-aware spread of the ids over the real tile count and the optional
// reversal.
__device__ __forceinline__ int batch_tile_id(const FrameArg &fa, int b, int nb, int &n)
{
    n = fa.n;
    if (fa.dev_n) {
        const int dn = gload(fa.dev_n), dt = gload(fa.dev_n + 1 + fa.launch);
        n = __builtin_amdgcn_readfirstlane(dn);
        nb = __builtin_amdgcn_readfirstlane(dt);
        if (b >= nb) return -1;
    }
    int t = xcd_logical_id(b, nb);
    if (fa.reverse) t = nb - 1 - t;
    return t;
}


enum ConvMode { CONV_PACK = 0, CONV_POOL = 1, CONV_CAT = 2, CONV_PLAIN = 3 };
// EPI_LINEAR: bias only, NHWC fp32 store (the input gradient of a conv in
// training runs the forward kernel with transposed, flipped weights).
enum ConvEpi { EPI_RELU = 0, EPI_HEAD_SOFTPLUS = 1, EPI_HEAD_EXP = 2, EPI_LINEAR = 3 };
enum ActType { ACT_F32 = 0, ACT_BF16 = 1 };

// One 3x3 conv layer as the kernels see it.
struct ConvLayer {
    int level;         // output resolution level (H >> level, W >> level)
    int src0_kind;     // 0: e[src0_idx], 1: u[src0_idx], 2: p[src0_idx]
    int src0_idx;
    int src1_idx;      // CAT: skip e[src1_idx]
    int C0, C1;        // channels of source 0 / source 1 (CAT: up, skip)
    int Cin_pad;       // virtual input channels padded to the chunk size
    int Cout;          // real output channels
    int Cout_pad;      // padded to 16 * NB * groups
    int groups;        // output-channel groups (one workgroup each)
    int out_kind;      // 0: e[out_idx], 1: u[out_idx], 2: head
    int out_idx;
    int M;             // head: channels 0..M-1 get the weight activation
    int CK;            // input channels per reduction chunk (weights packed to match)
    int NB;            // 16-channel output blocks per workgroup
    int th;            // output rows per tile of the kernel that runs this layer
    int ks;            // kernel size: 3, or 5 (a merged RepVGG block)
    int pool_idx;      // >= 0: the epilogue also writes the 2x2 means of the output to p[pool_idx]
    const void *w;     // packed weights
    const float *bias; // [Cout]
    float inv_gamma, dnear, dinv;  // CONV_PACK preprocessing constants
    float in_qscale;           // fp8: 1 / (input activation scale)
    const float *out_scale;    // fp8: per output channel, input scale x weight scale
};

struct DecodeCfg {
    int M;
    int R;                    // max radius
    int radius[kMaxKernels];  // (k_i - 1)/2
    float eps_norm;
    float eps_albedo;
    int exp_weights;          // frames form: the head holds h, W = exp(h) (per-tile shift)
    int tw, th;               // forward decode tile: centres per row, rows
    int hxs;                  // row stride (float4) of its LDS plane
};

// ---- launchers (defined in the .hip files) --------------------------------
// Launches one conv layer over `blocks` workgroups (conv_grid of the batch;
// a larger count is allowed: surplus workgroups exit at once).
hipError_t launch_conv(const ConvLayer &L, int mode, int epi, int prec, const FrameArg &fa,
                       int blocks, hipStream_t s);
int conv_grid(const ConvLayer &L, int n, const int *H, const int *W);
int conv_chunk(int prec, int mode, int Cin, int C0);
// 16-channel output blocks per workgroup for a layer with nblk blocks.
int conv_blocks_per_group(int prec, int mode, int CK, int nblk, int level, int ks);
// Decode + fusion + remodulation over frames of fa (denoise mode: c and mod
// derive from r, a) -- or over plain tensors (decode mode).
hipError_t launch_decode_frames(const DecodeCfg &dc, const FrameArg &fa, int blocks, hipStream_t s);
// Sets dc.tw, dc.th, dc.hxs from dc.R (the forward decode's tile shape).
void decode_tile_shape(DecodeCfg &dc);
int decode_grid(const DecodeCfg &dc, int n, const int *H, const int *W);
hipError_t launch_decode_tensors(const DecodeCfg &dc, int N, int H, int W, const float *head,
                                 const float *c, const float *mod, float *out, hipStream_t s);
hipError_t launch_decode_backward(const DecodeCfg &dc, int N, int H, int W, const float *head,
                                  const float *c, const float *mod, const float *g,
                                  float *grad_head, float *grad_c, void *scratch,
                                  hipStream_t s);
size_t decode_backward_scratch_bytes(const DecodeCfg &dc, int N, int H, int W);
// Training kernels (train.hip): see the file's header for each operation.
// Kernels with an nf argument run over nf frames of one size: frame f's
// operand X is at X + f sX (strides in floats); their outputs are contiguous
// per frame.
// Up to kTrGroup frames' own buffers (radiance, albedo, normal, depth, the
// denoised output, the reference) for the per-frame training kernels, which
// run over the frames of a group in one launch
constexpr int kTrGroup = 16;
struct TrFrames {
    const float *r[kTrGroup], *a[kTrGroup], *n[kTrGroup], *d[kTrGroup], *y[kTrGroup], *t[kTrGroup];
};
hipError_t tr_pack(long P, int nf, const TrFrames &fr, float inv_gamma, float dnear, float dinv, float *X,
                   hipStream_t s);
hipError_t tr_pool(int H, int W, int C, int nf, const float *in, long sin, float *out, hipStream_t s);
hipError_t tr_head_prep(long P, int M, int nf, const float *planar, long sp, const TrFrames &fr, float eps_a,
                        float *head, float *c, float *mod, hipStream_t s);
int tr_smape_blocks(long n);
// loss[0] (+)= the SMAPE of nf frames of n values (partial: nf x
// tr_smape_blocks(n) floats)
hipError_t tr_smape(long n, int nf, const TrFrames &fr, float eps, float inv_n, float *g, float *partial, float *loss,
                    int accumulate, hipStream_t s);
// dh[p][j] for j < 2M, zero for 2M <= j < ld (rows ld floats apart)
hipError_t tr_head_act_bwd(long P, int M, int ld, int nf, const float *grad_head, const float *planar, long sp,
                           float *dh, hipStream_t s);
// gm = (act > 0) g over nf frames of n values (gm may be g)
hipError_t tr_mask(long n, int nf, const float *g, const float *act, long sa, float *gm, hipStream_t s);
// Weights of the input-gradient conv in the fp32 forward kernels' packing
// ([Co_pad/16][9][16][Cout_pad], 16-channel chunks): element (c, t, ci) is
// w[c][ci][8 - t], zero beyond Co or Ci.
hipError_t tr_pack_dgrad(int Ci, int Co, int Co_pad, int Cout_pad, const float *w, float *packed, hipStream_t s);
// partial sums of a weight gradient over nf frames of P pixels
size_t tr_wgrad_part_floats(long P, int Ci, int Co, int nf);
// The conv's input: Cu channels of `up` (H/2 x W/2) upsampled x2, then Cf
// channels of `in` (H x W) (Cu = 0: `in` alone); gm rows are ldg >= Co
// floats apart; dw and db accumulate the nf frames
hipError_t tr_wgrad(int H, int W, int Co, int ldg, int nf, const float *gm, long sgm, const float *in, long sin,
                    int Cf, const float *up, long sup, int Cu, float *part, float *dw, float *db, hipStream_t s);
// gu = (act_u > 0) * (the upsampled part's gradient); ge = the skip part's
hipError_t tr_cat_bwd(int H, int W, int Cu, int Ce, int nf, const float *gcat, const float *act_u, long sa, float *gu,
                      float *ge, hipStream_t s);
// ge = (act > 0) * (ge + the 2x2 mean's adjoint of gp)
hipError_t tr_pool_bwd(int H, int W, int C, int nf, const float *gp, const float *act, long sa, float *ge,
                       hipStream_t s);
// table of nf frames of H x W for an input-gradient conv: e[0] = src + f ss,
// e[1] = dst + f sd
hipError_t tr_frame_table(FrameDesc *tab, int nf, int H, int W, const float *src, long ss, float *dst, long sd,
                          hipStream_t s);
hipError_t tr_fill(long n, float v, float *b, hipStream_t s);
hipError_t tr_adam(long n, float *w, const float *g, float *m, float *v, float lr, float b1, float b2, float c1,
                   float c2, float eps, hipStream_t s);
hipError_t tr_repack(int Cin, int Cout, int CK, int nch, int Cout_pad, const float *blob, float *packed, float *bias,
                     hipStream_t s);
// Multi-resolution reconstruction pieces (mr.hip): 2x2 mean of a 3-channel
// image, and the Eq. 7 blend (optionally remodulated).
hipError_t launch_pool2(int H, int W, const float *in, float *out, hipStream_t s);
hipError_t launch_mr_blend(int H, int W, const float *fine, const float *coarse, const float *alpha,
                           const float *mod, float *out, hipStream_t s);
// Temporal accumulation of one frame (temporal.hip); pr == nullptr: first frame.
hipError_t launch_temporal(int H, int W, const float *r, const float *n, const float *wp, const float *mv,
                           const float *pr, const float *pl, const float *pn, const float *pw, float alpha_min,
                           float pos_tol, float normal_tol, float *out, float *len, hipStream_t s);
// Explicit kernel-map reconstruction (the comparison of Sec. 5.3, kp.hip).
size_t kp_map_floats(const DecodeCfg &dc, int H, int W);
hipError_t launch_kp_expand(const DecodeCfg &dc, int H, int W, const float *head, float *maps, hipStream_t s);
hipError_t launch_kp_decode(const DecodeCfg &dc, int H, int W, const float *maps, const float *head,
                            const float *c, const float *mod, float *out, hipStream_t s);

// Tile geometry of the conv kernels (host and device agree on these).
constexpr int kConvTW = 32;  // output columns per tile (two 16-pixel MFMA blocks)
int conv_tile_rows(int prec, int mode, int CK, int level, bool pool, int ks);
// true if the layer runs the direct-to-LDS bf16 kernel (its weights are
// packed without row padding and with swizzled column groups)
bool conv_uses_direct(int prec, int mode, int CK, int ks);

}  // namespace wskp
