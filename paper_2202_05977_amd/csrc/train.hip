// One training step of the network (Eq. 1: the network's parameters are
// fitted by minimising a loss between the reconstruction and the reference;
// Eq. 6: the SMAPE loss; Sec. 5.3: Adam), FP32 throughout.
//
// The forward pass is the fp32 denoising path (its workspace keeps every
// layer's output).  The backward pass (the frames of one size together):
//   SMAPE gradient at the output -> adjoint of decode and fusion (decode.hip)
//   -> derivative of the weight activation -> for each conv, from the head
//   back to the first encoder: the weight and bias gradient (accumulated
//   over the frames of the batch) and the input gradient, which the adjoints
//   of the nearest x2 upsampling, the channel concatenation and the 2x2 mean
//   distribute to the layers that fed it.  The adjoint that writes the last
//   contribution to an activation's gradient also applies that activation's
//   ReLU mask, and the first contribution overwrites, so no gradient buffer
//   is cleared and no separate mask pass runs (except the head's input).
// The weight gradient's input is written out where it is computed (the
// network input, a 2x2 mean); a decoder's, the [upsampled, skip]
// concatenation, is read from its two sources.  Frames of one size run the
// backward pass together: every kernel once per layer over all of them.
//
// Gradient kernels (NHWC fp32, zero padding, conv = 3x3 cross-correlation):
//   dgrad  gin[p][ci] = sum_{tap,co} gm[p - off(tap)][co] w[co][ci][tap]:
//          itself a 3x3 conv of gm with the kernel flipped and its channel
//          axes swapped, run by the fp32 forward conv kernel (MFMA,
//          conv3x3.hip) on weights that tr_pack_dgrad lays out for it; the
//          head's 2M output channels are padded with zeros to a multiple
//          of 16 (its gradient dh is written with that row stride)
//   wgrad  dw[co][ci][tap] = sum_p gm[p][co] in[p + off(tap)][ci],
//          db[co] = sum_p gm[p][co]: a GEMM over pixels,
//          tr_wgrad_mfma_kernel (v_mfma_f32_16x16x4f32, 4 pixels per step;
//          channel counts that are not multiples of 16 are padded with
//          zeros).  Each workgroup sums one chunk of 256 to 1024 pixels
//          and a second pass adds the chunks' partial sums in a fixed
//          order, so the result does not depend on scheduling
#include "wskp_internal.h"

namespace wskp {

constexpr int kTrThreads = 256;

static inline int tr_blocks(long n) { return (int)((n + kTrThreads - 1) / kTrThreads); }

// The per-frame kernels below run over a group of frames (blockIdx.y), the
// frames' own buffers passed by pointer (TrFrames) and the group's scratch
// contiguous per frame.

// network input X [P][10] (Sec. 5.1), as the first conv's staging forms it
__global__ __launch_bounds__(kTrThreads) void tr_pack_kernel(long P, TrFrames fr, float inv_gamma, float dnear,
                                                              float dinv, float *X)
{
    const long p = (long)blockIdx.x * kTrThreads + threadIdx.x;
    if (p >= P) return;
    const int f = blockIdx.y;
    const float *r = fr.r[f], *a = fr.a[f], *n = fr.n[f], *d = fr.d[f];
    X += f * P * 10;
    float x[10];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float rv = fminf(fmaxf(gload(r + p * 3 + ch), 0.f), 1.f);
        x[ch] = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(rv) * inv_gamma);
        x[3 + ch] = gload(a + p * 3 + ch);
        x[6 + ch] = (gload(n + p * 3 + ch) + 1.f) * 0.5f;
    }
    x[9] = fminf(fmaxf((gload(d + p) - dnear) * dinv, 0.f), 1.f);
#pragma unroll
    for (int ch = 0; ch < 10; ++ch) gstore(X + p * 10 + ch, x[ch]);
}

// Kernels over nf frames of one size: frame f's operand X sits at X + f sX
// (floats); outputs are contiguous per frame.

// out [nf][H/2][W/2][C] = 2x2 means of in [H][W][C] (frame stride sin)
__global__ __launch_bounds__(kTrThreads) void tr_pool_kernel(int H, int W, int C, int nf, const float *in, long sin,
                                                              float *out)
{
    const int Wo = W / 2;
    const long n = (long)(H / 2) * Wo * C;
    const long i = (long)blockIdx.x * kTrThreads + threadIdx.x;
    if (i >= n * nf) return;
    const long f = i / n, j = i - f * n;
    const int ch = (int)(j % C);
    const long q = j / C;
    const int y = (int)(q / Wo), x = (int)(q % Wo);
    const float *s = in + f * sin + ((long)(2 * y) * W + 2 * x) * C + ch;
    gstore(out + i, 0.25f * (((gload(s) + gload(s + C)) + gload(s + (long)W * C)) + gload(s + (long)W * C + C)));
}

// interleaved head [P][2M] from the planar record [2M][P]; c = r/(a+eps_a),
// mod = a + eps_a (the decode adjoint's inputs)
__global__ __launch_bounds__(kTrThreads) void tr_head_prep_kernel(long P, int M, const float *planar, long sp,
                                                                   TrFrames fr, float eps_a, float *head, float *c,
                                                                   float *mod)
{
    const long p = (long)blockIdx.x * kTrThreads + threadIdx.x;
    if (p >= P) return;
    const int f = blockIdx.y;
    const float *r = fr.r[f], *a = fr.a[f];
    planar += f * sp;
    head += f * P * 2 * M;
    c += f * P * 3;
    mod += f * P * 3;
    for (int j = 0; j < 2 * M; ++j) gstore(head + p * 2 * M + j, gload(planar + (long)j * P + p));
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float m = gload(a + p * 3 + ch) + eps_a;
        gstore(mod + p * 3 + ch, m);
        gstore(c + p * 3 + ch, gload(r + p * 3 + ch) / m);
    }
}

// SMAPE (Eq. 6) gradient g = dL/dy for n values of each frame with mean
// weight inv_n, and the block's share of the loss in
// partial[frame * gridDim.x + blockIdx.x]
__global__ __launch_bounds__(kTrThreads) void tr_smape_kernel(long n, TrFrames fr, float eps, float inv_n, float *g,
                                                               float *partial)
{
    __shared__ float red[kTrThreads];
    const long i = (long)blockIdx.x * kTrThreads + threadIdx.x;
    const int f = blockIdx.y;
    const float *y = fr.y[f], *t = fr.t[f];
    g += f * n;
    partial += (long)f * gridDim.x;
    float l = 0.f;
    if (i < n) {
        const float yv = gload(y + i), tv = gload(t + i);
        const float d = yv - tv, den = fabsf(yv) + fabsf(tv) + eps;
        const float sd = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
        const float sr = yv > 0.f ? 1.f : (yv < 0.f ? -1.f : 0.f);
        l = fabsf(d) / den;
        gstore(g + i, (sd * den - fabsf(d) * sr) / (den * den) * inv_n);
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = kTrThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) gstore(partial + blockIdx.x, red[0] * inv_n);
}

// loss[0] (+)= sum of partial[0..nb): thread i sums partial[i], [i + 256],
// ... in order, then the 256 sums are added pairwise in LDS (a fixed order)
__global__ __launch_bounds__(kTrThreads) void tr_sum_kernel(int nb, const float *partial, float *loss, int accumulate)
{
    __shared__ float red[kTrThreads];
    float v = 0.f;
    for (int b = threadIdx.x; b < nb; b += kTrThreads) v += gload(partial + b);
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = kTrThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) gstore(loss, (accumulate ? gload(loss) : 0.f) + red[0]);
}

// gradient at the head conv's output: weight channels through softplus'
// (the logistic of h, = 1 - e^{-W} = -expm1(-W) in terms of W = softplus(h),
// accurate also where W is tiny); logits as is
__global__ __launch_bounds__(kTrThreads) void tr_head_act_bwd_kernel(long P, int M, int ld, const float *grad_head,
                                                                      const float *planar, long sp, float *dh)
{
    const long i = (long)blockIdx.x * kTrThreads + threadIdx.x;
    if (i >= P * ld) return;
    const int f = blockIdx.y;
    grad_head += f * P * 2 * M;
    planar += f * sp;
    dh += f * P * ld;
    const int j = (int)(i % ld);
    const long p = i / ld;
    float g = 0.f;
    if (j < 2 * M) {
        g = gload(grad_head + p * 2 * M + j);
        if (j < M) g *= -expm1f(-gload(planar + (long)j * P + p));
    }
    gstore(dh + i, g);
}

// gm = g * (act > 0) (the ReLU's derivative) over nf frames of n values
// (g and gm contiguous, act frame stride sa)
__global__ __launch_bounds__(kTrThreads) void tr_mask_kernel(long n, int nf, const float *g, const float *act, long sa,
                                                              float *gm)
{
    const long i = (long)blockIdx.x * kTrThreads + threadIdx.x;
    if (i >= n * nf) return;
    const long f = i / n, j = i - f * n;
    const float v = gload(g + i);
    gstore(gm + i, gload(act + f * sa + j) > 0.f ? v : 0.f);
}

// Partial weight gradients on the matrix cores, part[chunk][co][ci][tap]
// and partb[chunk][co]: a GEMM over
// pixels, D[co][ci] += sum_p gm[p][co] * in[p + off(tap)][ci] for each tap,
// with v_mfma_f32_16x16x4f32 taking 4 pixels per step (lane (g, j): pixel
// g of the step; A = gm[p_g][co0 + j] (gm rows ldg floats apart),
// B = in[p_g + off][ci0 + j]).  One workgroup per (chunk of `chunk`
// pixels, CB output blocks of 16, one input block of 16); its kWgWaves waves
// take consecutive quarters of the chunk, each loading the operands of its
// next step before the MFMAs of the current one, and add their sums in LDS
// in a fixed order, (w0 + w2) + (w1 + w3).  Operands are raw buffer loads
// with 32-bit offsets into windows: the chunk's gm rows, and the whole
// source rows of the image rows the chunk touches and one either side (the
// input block's source: the H x W map, or the half-size map the input
// upsamples).  Channels beyond Co or Ci (the network input's 10, the
// head's 2M), taps outside the image and pixels past the chunk take an
// offset beyond the window and read zeros, so no load is conditional.  The workgroups of input block 0 also sum gm
// (B = 1) for the bias.  Lane (g, j) ends with D[4g + r][j], r = 0..3.
typedef float trf32x4 __attribute__((ext_vector_type(4)));
// Chunks are 256 pixels, doubled (up to kWgChunkMax) while a launch still
// has kWgMinGroups workgroups: fewer partial sums to write and reduce.
constexpr int kWgChunk = 256, kWgChunkMax = 1024, kWgMinGroups = 2048, kWgWaves = 4;
constexpr unsigned kWgOut = 0x80000000u;   // beyond every window (windows are < 2 GiB)
template <int CB>
__global__ __launch_bounds__(64 * kWgWaves) void tr_wgrad_mfma_kernel(int H, int W, int Co, int ldg, int chunk,
                                                                      int nch, const float *gm, long sgm,
                                                                      const float *in, long sin, int Cf,
                                                                      const float *up, long sup, int Cu,
                                                                      float *part, float *partb)
{
    __shared__ trf32x4 red[2][CB * 10][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
    const int co0 = blockIdx.y * (16 * CB), ci0 = blockIdx.z * 16;
    const long P = (long)H * W;
    // workgroup x: frame f, chunk x - f nch of that frame; partial sum x
    const int fr = blockIdx.x / nch;
    gm += fr * sgm;
    const long c0 = (long)(blockIdx.x - fr * nch) * chunk;
    const int n = (int)min((long)chunk, P - c0);
    const rsrc_t rg = make_rsrc(gm + c0 * ldg, (unsigned)n * (unsigned)ldg * 4u);
    // The input block's source: the map that the upsampling makes H x W
    // (channels 0 .. Cu-1 of the layer's input, read at (y/2, x/2)) or the
    // H x W map (channels Cu ..).  Its window: the source rows of image rows
    // ylo .. yhi (the chunk's rows and one either side), whole rows.
    const int Ci = Cu + Cf;
    const bool coarse = ci0 < Cu;
    const int sh = coarse ? 1 : 0, Cs = coarse ? Cu : Cf, cs0 = coarse ? ci0 : ci0 - Cu;
    const int Wsrc = W >> sh;
    const float *src = coarse ? up + fr * sup : in + fr * sin;
    const int ylo = max(0, (int)(c0 / W) - 1), yhi = min(H - 1, (int)((c0 + n - 1) / W) + 1);
    const int rlo = ylo >> sh, rhi = yhi >> sh;
    const unsigned rowb = (unsigned)Wsrc * (unsigned)Cs * 4u, pixb = (unsigned)Cs * 4u;
    const rsrc_t ri = make_rsrc(src + (long)rlo * Wsrc * Cs, (unsigned)(rhi - rlo + 1) * rowb);
    const bool bias = blockIdx.z == 0;
    bool cok[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) cok[c] = co0 + c * 16 + j < Co;
    const bool ciok = cs0 + j < Cs;
    const unsigned chb = (unsigned)(cs0 + j) * 4u;
    trf32x4 acc[CB][10];
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int t = 0; t < 10; ++t) acc[c][t] = trf32x4{0.f, 0.f, 0.f, 0.f};
    // this wave's pixels qa .. qb - 1 of the chunk
    const int qa = wave * (chunk / kWgWaves), qb = min(n, qa + chunk / kWgWaves);
    float a[CB], b[9];
    // operands of the step at chunk pixel q, for this lane's pixel q + g at
    // image position (y, x)
    // (offsets are made out of range by setting bit 31, with no select, so
    // that the compiler keeps every load unconditional)
    auto out = [](bool ok) { return (0u - (unsigned)!ok) & kWgOut; };
    auto load = [&](int q, int y, int x, float (&av)[CB], float (&bv)[9]) {
        const int p = q + g;
        const bool valid = p < qb;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const unsigned off = ((unsigned)p * (unsigned)ldg + (unsigned)(co0 + c * 16 + j)) * 4u | out(valid & cok[c]);
            av[c] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rg, off, 0, 0));
        }
        // tap (dy, dx) reads source row ((y + dy - 1) >> sh) - rlo, column
        // (x + dx - 1) >> sh of the window (valid taps lie inside it)
        const bool vc = valid & ciok;
        const bool rok[3] = {y >= 1, true, y + 1 < H}, xok[3] = {x >= 1, true, x + 1 < W};
        unsigned rt[3], ct[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            rt[d] = (unsigned)(((y + d - 1) >> sh) - rlo) * rowb + chb;
            ct[d] = (unsigned)((x + d - 1) >> sh) * pixb;
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dy = t / 3, dx = t % 3;
            const unsigned off = (rt[dy] + ct[dx]) | out(vc & rok[dy] & xok[dx]);
            bv[t] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ri, off, 0, 0));
        }
    };
    const long p0 = c0 + qa + g;
    int y = (int)(p0 / W), x = (int)(p0 - (long)y * W);
    load(qa, y, x, a, b);
    for (int q = qa; q < qb; q += 4) {
        int yn = y, xn = x + 4;
        if (W >= 4) {
            const bool wrap = xn >= W;
            xn -= wrap ? W : 0;
            yn += wrap ? 1 : 0;
        } else {
            while (xn >= W) {
                xn -= W;
                ++yn;
            }
        }
        float an[CB], bn[9];
        load(q + 4, yn, xn, an, bn);
#pragma unroll
        for (int c = 0; c < CB; ++c) {
#pragma unroll
            for (int t = 0; t < 9; ++t) acc[c][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[c], b[t], acc[c][t], 0, 0, 0);
            if (bias) acc[c][9] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[c], 1.f, acc[c][9], 0, 0, 0);
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) a[c] = an[c];
#pragma unroll
        for (int t = 0; t < 9; ++t) b[t] = bn[t];
        y = yn;
        x = xn;
    }
    // (w0 + w2) + (w1 + w3)
    if (wave >= 2)
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
            for (int t = 0; t < 10; ++t) red[wave - 2][c * 10 + t][lane] = acc[c][t];
    __syncthreads();
    if (wave < 2)
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
            for (int t = 0; t < 10; ++t) acc[c][t] += red[wave][c * 10 + t][lane];
    __syncthreads();
    if (wave == 1)
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
            for (int t = 0; t < 10; ++t) red[0][c * 10 + t][lane] = acc[c][t];
    __syncthreads();
    if (wave != 0) return;
    const long base = (long)blockIdx.x * Co * Ci * 9;
    const int ci = ci0 + j;
#pragma unroll
    for (int c = 0; c < CB; ++c) {
#pragma unroll
        for (int t = 0; t < 10; ++t) acc[c][t] += red[0][c * 10 + t][lane];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = co0 + c * 16 + 4 * g + r;
            if (co >= Co) continue;
            if (ci < Ci)
#pragma unroll
                for (int t = 0; t < 9; ++t) gstore(part + base + ((long)co * Ci + ci) * 9 + t, acc[c][t][r]);
            if (bias && j == 0) gstore(partb + (long)blockIdx.x * Co + co, acc[c][9][r]);
        }
    }
}

// First level of a sliced reduce: out[y][i] = sum of part rows (chunks)
// y S .. y S + S - 1 (fixed order: four interleaved sums added pairwise), for
// the nw weights then the Co biases; blockIdx.y = slice y.  Used when a layer
// has few weights and many chunks, so that more workgroups share the sums.
__global__ __launch_bounds__(kTrThreads) void tr_wgrad_slice_kernel(long nw, int Co, int nchunk, int S,
                                                                     const float *part, const float *partb,
                                                                     float *out)
{
    __shared__ float sred[4][64];
    const int li = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const long i = (long)blockIdx.x * 64 + li;
    const bool inw = i < nw, in = i < nw + Co;
    const float *src = inw ? part + i : partb + (in ? i - nw : 0);
    const long stride = inw ? nw : Co;
    const int c0 = blockIdx.y * S, c1 = min(nchunk, c0 + S);
    float s0 = 0.f;
    if (in)
        for (int c = c0 + grp; c < c1; c += 4) s0 += gload(src + (long)c * stride);
    sred[grp][li] = s0;
    __syncthreads();
    if (grp == 0 && in)
        gstore(out + (long)blockIdx.y * (nw + Co) + i, (sred[0][li] + sred[1][li]) + (sred[2][li] + sred[3][li]));
}

// dw (+)= sum over chunks of part, likewise db: 64 weights per workgroup,
// its four waves take the chunks c = wave (mod 4) and each sums them in
// order on two alternating accumulators; the waves' sums are added in a
// fixed order, so the result does not depend on scheduling
__global__ __launch_bounds__(kTrThreads) void tr_wgrad_reduce_kernel(long nw, int Co, int nchunk, const float *part,
                                                                      const float *partb, float *dw, float *db)
{
    __shared__ float sred[4][64];
    const int li = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const long i = (long)blockIdx.x * 64 + li;
    const bool inw = i < nw, in = i < nw + Co;
    const float *src = inw ? part + i : partb + (in ? i - nw : 0);
    const long stride = inw ? nw : Co;
    float s0 = 0.f, s1 = 0.f;
    if (in) {
        int c = grp;
        for (; c + 4 < nchunk; c += 8) {
            s0 += gload(src + (long)c * stride);
            s1 += gload(src + (long)(c + 4) * stride);
        }
        if (c < nchunk) s0 += gload(src + (long)c * stride);
    }
    sred[grp][li] = s0 + s1;
    __syncthreads();
    if (grp == 0 && in) {
        float *dst = inw ? dw + i : db + (i - nw);
        gstore(dst, gload(dst) + ((sred[0][li] + sred[1][li]) + (sred[2][li] + sred[3][li])));
    }
}

// adjoint of [upsample(u), e]: the upsampled part's gradient, the sum of
// gcat[2y+i][2x+j][c] (c < Cu), masked by u's ReLU (its only contribution)
// into gu[y][x][c]; the skip part's, gcat[p][Cu+c], into ge[p][c] (its first
// contribution: both overwrite)
__global__ __launch_bounds__(kTrThreads) void tr_cat_bwd_kernel(int H, int W, int Cu, int Ce, int nf,
                                                                 const float *gcat, const float *act_u, long sa,
                                                                 float *gu, float *ge)
{
    const int C = Cu + Ce;
    const int Hc = H / 2, Wc = W / 2;
    const long nu = (long)Hc * Wc * Cu, ne = (long)H * W * Ce;
    const long i = (long)blockIdx.x * kTrThreads + threadIdx.x;
    if (i >= (nu + ne) * nf) return;
    const long f = i / (nu + ne), k = i - f * (nu + ne);
    const float *gc = gcat + f * H * W * C;
    if (k < nu) {
        const int c = (int)(k % Cu);
        const long q = k / Cu;
        const int y = (int)(q / Wc), x = (int)(q % Wc);
        const float *s = gc + ((long)(2 * y) * W + 2 * x) * C + c;
        const float v = ((gload(s) + gload(s + C)) + gload(s + (long)W * C)) + gload(s + (long)W * C + C);
        gstore(gu + f * nu + k, gload(act_u + f * sa + k) > 0.f ? v : 0.f);
    } else {
        const long j = k - nu;
        const int c = (int)(j % Ce);
        const long p = j / Ce;
        gstore(ge + f * ne + j, gload(gc + p * C + Cu + c));
    }
}

// ge[p][c] = (act[p][c] > 0) (ge[p][c] + gp[p/2][c] / 4): the 2x2 mean's
// adjoint added to what the concatenation's adjoint wrote, then the ReLU mask
// of e (its last contribution)
__global__ __launch_bounds__(kTrThreads) void tr_pool_bwd_kernel(int H, int W, int C, int nf, const float *gp,
                                                                  const float *act, long sa, float *ge)
{
    const long n = (long)H * W * C;
    const long i = (long)blockIdx.x * kTrThreads + threadIdx.x;
    if (i >= n * nf) return;
    const long f = i / n, j = i - f * n;
    const int c = (int)(j % C);
    const long p = j / C;
    const int y = (int)(p / W), x = (int)(p % W);
    const long np = (long)(H / 2) * (W / 2) * C;
    const float v = gload(ge + i) + 0.25f * gload(gp + f * np + ((long)(y / 2) * (W / 2) + x / 2) * C + c);
    gstore(ge + i, gload(act + f * sa + j) > 0.f ? v : 0.f);
}

// frame table of an input-gradient conv over nf frames: e[0] = the gradient
// it reads (frame stride ss), e[1] = the input gradient it writes (sd)
__global__ void tr_frame_table_kernel(FrameDesc *tab, int nf, int H, int W, const float *src, long ss, float *dst,
                                      long sd)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    FrameDesc d{};
    d.H = H;
    d.W = W;
    d.e[0] = const_cast<float *>(src + f * ss);
    d.e[1] = dst + f * sd;
    tab[f] = d;
}

__global__ __launch_bounds__(kTrThreads) void tr_fill_kernel(long n, float v, float *b)
{
    const long i = (long)blockIdx.x * kTrThreads + threadIdx.x;
    if (i < n) gstore(b + i, v);
}

// Adam (Kingma and Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// w -= lr (m / c1) / (sqrt(v / c2) + eps) with c1 = 1 - b1^t, c2 = 1 - b2^t
__global__ __launch_bounds__(kTrThreads) void tr_adam_kernel(long n, float *w, const float *g, float *m, float *v,
                                                              float lr, float b1, float b2, float c1, float c2,
                                                              float eps)
{
    const long i = (long)blockIdx.x * kTrThreads + threadIdx.x;
    if (i >= n) return;
    const float gi = gload(g + i);
    const float mi = b1 * gload(m + i) + (1.f - b1) * gi;
    const float vi = b2 * gload(v + i) + (1.f - b2) * gi * gi;
    gstore(m + i, mi);
    gstore(v + i, vi);
    gstore(w + i, gload(w + i) - lr * (mi / c1) / (sqrtf(vi / c2) + eps));
}

// fp32 weights of one conv from the blob layout (OIHW, then bias) into the
// layout the fp32 conv kernel reads: [chunk][tap][c][Cout_pad], zero padded;
// bias copied
__global__ __launch_bounds__(kTrThreads) void tr_repack_kernel(int Cin, int Cout, int CK, int nch, int Cout_pad,
                                                                const float *blob, float *packed, float *bias)
{
    const long n = (long)nch * 9 * CK * Cout_pad;
    const long i = (long)blockIdx.x * kTrThreads + threadIdx.x;
    if (i < n) {
        const int co = (int)(i % Cout_pad);
        long q = i / Cout_pad;
        const int c = (int)(q % CK);
        q /= CK;
        const int tap = (int)(q % 9);
        const int cc = (int)(q / 9);
        const int ci = cc * CK + c;
        gstore(packed + i, (co < Cout && ci < Cin) ? gload(blob + ((long)co * Cin + ci) * 9 + tap) : 0.f);
    } else if (i < n + Cout) {
        const int co = (int)(i - n);
        gstore(bias + co, gload(blob + (long)Cout * Cin * 9 + co));
    }
}

// ---- launchers ---------------------------------------------------------------
#define TR_LAUNCH(kernel, n, ...)                                                                          \
    do {                                                                                                   \
        const long n_ = (n);                                                                               \
        if (n_ > 0) hipLaunchKernelGGL(kernel, dim3(tr_blocks(n_)), dim3(kTrThreads), 0, s, __VA_ARGS__); \
    } while (0)

// grid of one frame's blocks (x) over the group's nf frames (y)
#define TR_LAUNCH_F(kernel, n, nf, ...)                                                                    \
    do {                                                                                                   \
        const long n_ = (n);                                                                               \
        if (n_ > 0 && (nf) > 0)                                                                            \
            hipLaunchKernelGGL(kernel, dim3(tr_blocks(n_), (unsigned)(nf)), dim3(kTrThreads), 0, s, __VA_ARGS__); \
    } while (0)

hipError_t tr_pack(long P, int nf, const TrFrames &fr, float inv_gamma, float dnear, float dinv, float *X,
                   hipStream_t s)
{
    TR_LAUNCH_F(tr_pack_kernel, P, nf, P, fr, inv_gamma, dnear, dinv, X);
    return hipGetLastError();
}
hipError_t tr_pool(int H, int W, int C, int nf, const float *in, long sin, float *out, hipStream_t s)
{
    TR_LAUNCH(tr_pool_kernel, (long)(H / 2) * (W / 2) * C * nf, H, W, C, nf, in, sin, out);
    return hipGetLastError();
}
hipError_t tr_head_prep(long P, int M, int nf, const float *planar, long sp, const TrFrames &fr, float eps_a,
                        float *head, float *c, float *mod, hipStream_t s)
{
    TR_LAUNCH_F(tr_head_prep_kernel, P, nf, P, M, planar, sp, fr, eps_a, head, c, mod);
    return hipGetLastError();
}
int tr_smape_blocks(long n) { return tr_blocks(n); }
hipError_t tr_smape(long n, int nf, const TrFrames &fr, float eps, float inv_n, float *g, float *partial, float *loss,
                    int accumulate, hipStream_t s)
{
    TR_LAUNCH_F(tr_smape_kernel, n, nf, n, fr, eps, inv_n, g, partial);
    hipLaunchKernelGGL(tr_sum_kernel, dim3(1), dim3(kTrThreads), 0, s, tr_blocks(n) * nf, partial, loss, accumulate);
    return hipGetLastError();
}
hipError_t tr_head_act_bwd(long P, int M, int ld, int nf, const float *grad_head, const float *planar, long sp,
                           float *dh, hipStream_t s)
{
    TR_LAUNCH_F(tr_head_act_bwd_kernel, P * ld, nf, P, M, ld, grad_head, planar, sp, dh);
    return hipGetLastError();
}
hipError_t tr_mask(long n, int nf, const float *g, const float *act, long sa, float *gm, hipStream_t s)
{
    TR_LAUNCH(tr_mask_kernel, n * nf, n, nf, g, act, sa, gm);
    return hipGetLastError();
}
__global__ __launch_bounds__(kTrThreads) void tr_pack_dgrad_kernel(int Ci, int Co, int Co_pad, int Cout_pad,
                                                                    const float *w, float *packed)
{
    const long n = (long)Co_pad * 9 * Cout_pad;
    const long i = (long)blockIdx.x * kTrThreads + threadIdx.x;
    if (i >= n) return;
    const int ci = (int)(i % Cout_pad);
    const long ct = i / Cout_pad;            // (chunk * 9 + tap) * 16 + c
    const int c16 = (int)(ct % 16), ctap = (int)(ct / 16);
    const int t = ctap % 9, co = (ctap / 9) * 16 + c16;
    gstore(packed + i, ci < Ci && co < Co ? gload(w + ((long)co * Ci + ci) * 9 + (8 - t)) : 0.f);
}

hipError_t tr_pack_dgrad(int Ci, int Co, int Co_pad, int Cout_pad, const float *w, float *packed, hipStream_t s)
{
    TR_LAUNCH(tr_pack_dgrad_kernel, (long)Co_pad * 9 * Cout_pad, Ci, Co, Co_pad, Cout_pad, w, packed);
    return hipGetLastError();
}

static int wgrad_blocks(int Ci, int Co)
{
    const int cib = (Ci + 15) / 16, cob = (Co + 15) / 16;
    return cib * (cob % 2 == 0 ? cob / 2 : cob);
}
// pixels per chunk for nf frames of P pixels (a multiple of 16: four waves
// of whole 4-pixel steps)
static int wgrad_chunk(long P, int Ci, int Co, int nf)
{
    int c = kWgChunk;
    while (c < kWgChunkMax && (long)nf * ((P + 2 * c - 1) / (2 * c)) * wgrad_blocks(Ci, Co) >= kWgMinGroups) c *= 2;
    return c;
}
// slices of the two-level reduce (at most kWgSlices)
constexpr int kWgSlices = 64;
static int wgrad_slices(long nw, int Co, int nall)
{
    const long gx = (nw + Co + 63) / 64;
    int G = 1;
    while (G < kWgSlices && gx * G < 1024 && nall / (2 * G) >= 32) G *= 2;
    return G;
}
size_t tr_wgrad_part_floats(long P, int Ci, int Co, int nf)
{
    const int c = wgrad_chunk(P, Ci, Co, nf);
    // the chunks' partial sums, then the slices' sums of the two-level reduce
    return ((size_t)nf * ((P + c - 1) / c) + kWgSlices) * ((size_t)Co * Ci * 9 + Co);
}
hipError_t tr_wgrad(int H, int W, int Co, int ldg, int nf, const float *gm, long sgm, const float *in, long sin,
                    int Cf, const float *up, long sup, int Cu, float *part, float *dw, float *db, hipStream_t s)
{
    const int Ci = Cu + Cf;
    const long P = (long)H * W;
    const int chunk = wgrad_chunk(P, Ci, Co, nf);
    const int nch = (int)((P + chunk - 1) / chunk), nall = nf * nch;
    const long nw = (long)Co * Ci * 9;
    float *partb = part + (size_t)nall * nw;
    // the kernel's buffer windows and offsets stay below 2 GiB
    if ((double)(chunk + 3.0 * W) * std::max(std::max(Cf, Cu), ldg) * 4.0 >= 2147483648.0) return hipErrorInvalidValue;
    if (Cu % 16 || (Cu > 0 && (H % 2 || W % 2))) return hipErrorInvalidValue;   // whole blocks per source
    const unsigned cib = (unsigned)((Ci + 15) / 16), cob = (unsigned)((Co + 15) / 16);
    if (cob % 2 == 0)
        hipLaunchKernelGGL(tr_wgrad_mfma_kernel<2>, dim3((unsigned)nall, cob / 2, cib), dim3(64 * kWgWaves), 0, s, H,
                           W, Co, ldg, chunk, nch, gm, sgm, in, sin, Cf, up, sup, Cu, part, partb);
    else
        hipLaunchKernelGGL(tr_wgrad_mfma_kernel<1>, dim3((unsigned)nall, cob, cib), dim3(64 * kWgWaves), 0, s, H, W,
                           Co, ldg, chunk, nch, gm, sgm, in, sin, Cf, up, sup, Cu, part, partb);
    const unsigned gx = (unsigned)((nw + Co + 63) / 64);
    // (the second level treats the biases as weights nw .. nw + Co - 1, so
    // db must follow dw, as in the weight blob)
    const int G = db == dw + nw ? wgrad_slices(nw, Co, nall) : 1;
    if (G == 1) {
        hipLaunchKernelGGL(tr_wgrad_reduce_kernel, dim3(gx), dim3(kTrThreads), 0, s, nw, Co, nall, part, partb, dw, db);
    } else {
        // slice sums into the rows after the chunks' partials, then their sum
        float *sl = partb + (size_t)nall * Co;
        const int S = (nall + G - 1) / G;
        hipLaunchKernelGGL(tr_wgrad_slice_kernel, dim3(gx, (unsigned)G), dim3(kTrThreads), 0, s, nw, Co, nall, S, part,
                           partb, sl);
        // rows of sl are nw + Co floats: weights, then biases
        hipLaunchKernelGGL(tr_wgrad_reduce_kernel, dim3(gx), dim3(kTrThreads), 0, s, nw + Co, 0, G, sl, sl, dw, db);
    }
    return hipGetLastError();
}
hipError_t tr_cat_bwd(int H, int W, int Cu, int Ce, int nf, const float *gcat, const float *act_u, long sa, float *gu,
                      float *ge, hipStream_t s)
{
    TR_LAUNCH(tr_cat_bwd_kernel, ((long)(H / 2) * (W / 2) * Cu + (long)H * W * Ce) * nf, H, W, Cu, Ce, nf, gcat, act_u,
              sa, gu, ge);
    return hipGetLastError();
}
hipError_t tr_pool_bwd(int H, int W, int C, int nf, const float *gp, const float *act, long sa, float *ge,
                       hipStream_t s)
{
    TR_LAUNCH(tr_pool_bwd_kernel, (long)H * W * C * nf, H, W, C, nf, gp, act, sa, ge);
    return hipGetLastError();
}
hipError_t tr_frame_table(FrameDesc *tab, int nf, int H, int W, const float *src, long ss, float *dst, long sd,
                          hipStream_t s)
{
    hipLaunchKernelGGL(tr_frame_table_kernel, dim3((unsigned)((nf + 63) / 64)), dim3(64), 0, s, tab, nf, H, W, src, ss,
                       dst, sd);
    return hipGetLastError();
}
hipError_t tr_fill(long n, float v, float *b, hipStream_t s)
{
    TR_LAUNCH(tr_fill_kernel, n, n, v, b);
    return hipGetLastError();
}
hipError_t tr_adam(long n, float *w, const float *g, float *m, float *v, float lr, float b1, float b2, float c1,
                   float c2, float eps, hipStream_t s)
{
    TR_LAUNCH(tr_adam_kernel, n, n, w, g, m, v, lr, b1, b2, c1, c2, eps);
    return hipGetLastError();
}
hipError_t tr_repack(int Cin, int Cout, int CK, int nch, int Cout_pad, const float *blob, float *packed, float *bias,
                     hipStream_t s)
{
    TR_LAUNCH(tr_repack_kernel, (long)nch * 9 * CK * Cout_pad + Cout, Cin, Cout, CK, nch, Cout_pad, blob, packed,
              bias);
    return hipGetLastError();
}

}  // namespace wskp
