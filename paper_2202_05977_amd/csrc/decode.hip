// Weight-sharing kernel construction + filtering + fusion + remodulation
// (Sec. 4.2; Eq. 3, Eq. 4, Eq. 5) in one memory-bound pass.
//
// The normalised kernel weight of Eq. 3 depends on the neighbour only
// through its own scalar W_i(q) and on the centre only through the window
// sum, so every filtered value is a ratio of two box sums:
//     out_i(p) = sum_{q in Omega_i(p)} W_i(q) c(q) / max(sum_{q in Omega_i(p)} W_i(q), eps)
// with windows truncated at the image border.  No k x k kernel map is ever
// formed.  Each workgroup owns a 32 x 16 tile of centres; it stages the
// (32+2R) x (16+2R) halo of all M weight maps and of the irradiance c once in
// LDS (R = largest radius), then for each kernel size runs a horizontal pass
// (row sums of W and W*c, 4 values per position) into LDS and a vertical
// pass over those, and accumulates softmax(logits)_i * out_i in registers.
// The last step multiplies by the remodulation factor.
//
// Two input forms share the kernel:
//   frames   c = r / (a + eps_a) is formed while staging; mod = a + eps_a;
//            head, r, a and out come from the frame descriptors
//   tensors  head, c, mod (optional) and out are plain [N,H,W,*] tensors
#include "wskp_internal.h"

namespace wskp {

constexpr int kDTX = 32, kDTY = 16;

struct DecodeIO {
    int H, W;
    const float *head;  // [H,W,2M]
    const float *r, *a; // frames form
    const float *c;     // tensors form
    const float *mod;   // tensors form, may be null
    float *out;
    const float *g;
    float *grad_head;
    float4 *scratch;
};

struct DecodeTensors {
    int N, H, W;
    const float *head, *c, *mod;
    float *out;
    // adjoint only
    const float *g;     // dL/dout [N,H,W,3]
    float *grad_head;   // [N,H,W,2M]
    float4 *scratch;    // [N,M,H,W] x (u_0, u_1, u_2, dS)
};

template <bool FRAMES>
__device__ __forceinline__ bool decode_locate(const DecodeCfg &dc, const FrameArg &fa,
                                              const DecodeTensors &dt, DecodeIO &io, int &x0,
                                              int &y0)
{
    const int nbk = gridDim.x;
    int t = xcd_logical_id(blockIdx.x, nbk);
    if (FRAMES && fa.reverse) t = nbk - 1 - t;
    const int n = FRAMES ? fa.n : dt.N;
    const int twoM = 2 * dc.M;
    for (int f = 0; f < n; ++f) {
        int H, W;
        if (FRAMES) {
            const FrameDesc &fd = frame_at(fa, f);
            H = fd.H;
            W = fd.W;
        } else {
            H = dt.H;
            W = dt.W;
        }
        const int txn = (W + kDTX - 1) / kDTX, tyn = (H + kDTY - 1) / kDTY;
        const int cnt = txn * tyn;
        if (t < cnt) {
            x0 = (t % txn) * kDTX;
            y0 = (t / txn) * kDTY;
            io.H = H;
            io.W = W;
            if (FRAMES) {
                const FrameDesc &fd = frame_at(fa, f);
                io.head = fd.head;
                io.r = fd.r;
                io.a = fd.a;
                io.c = nullptr;
                io.mod = nullptr;
                io.out = fd.out;
                io.g = nullptr;
                io.grad_head = nullptr;
                io.scratch = nullptr;
            } else {
                const size_t P = (size_t)H * W;
                io.head = dt.head + (size_t)f * P * twoM;
                io.r = io.a = nullptr;
                io.c = dt.c + (size_t)f * P * 3;
                io.mod = dt.mod ? dt.mod + (size_t)f * P * 3 : nullptr;
                io.out = dt.out ? dt.out + (size_t)f * P * 3 : nullptr;
                io.g = dt.g ? dt.g + (size_t)f * P * 3 : nullptr;
                io.grad_head = dt.grad_head ? dt.grad_head + (size_t)f * P * twoM : nullptr;
                io.scratch = dt.scratch ? dt.scratch + (size_t)f * P * dc.M : nullptr;
            }
            return true;
        }
        t -= cnt;
    }
    return false;
}

enum DecodeKind { DK_FRAMES = 0, DK_TENSORS = 1, DK_ADJ_A = 2 };

// Dynamic LDS (floats): W planes [M][HY*HX], c planes [3][HY*HX],
// row sums [4][HY*32].
//   DK_FRAMES / DK_TENSORS: forward, writes out.
//   DK_ADJ_A: first half of the vector-Jacobian product.  Per centre p,
//     with dF = g * mod, da_i = <dF, out_i>:
//       dlogit_i   = alpha_i (da_i - sum_j alpha_j da_j)      -> grad_head[p][M+i]
//       u_i,ch(p)  = alpha_i dF_ch / max(S_i, eps)
//       dS_i(p)    = -[S_i > eps] sum_ch u_i,ch(p) out_i,ch(p)
//     (u_i, dS_i) go to scratch; decode_adj_b_kernel box-sums them.
template <int M, int KIND>
__global__ __launch_bounds__(kThreads) void decode_fwd_kernel(DecodeCfg dc, FrameArg fa,
                                                               DecodeTensors dt)
{
    constexpr bool FRAMES = KIND == DK_FRAMES;
    constexpr bool ADJ = KIND == DK_ADJ_A;
    extern __shared__ float lds[];
    DecodeIO io;
    int x0, y0;
    if (!decode_locate<FRAMES>(dc, fa, dt, io, x0, y0)) return;

    const int R = dc.R;
    const int HX = kDTX + 2 * R, HY = kDTY + 2 * R, HXY = HX * HY;
    float *Wl = lds;
    float *cl = Wl + M * HXY;
    float *hb = cl + 3 * HXY;
    const int HB = HY * kDTX;
    const int tid = threadIdx.x;
    const int H = io.H, W = io.W;

    // stage the halo: weights and irradiance, zero outside the image
    for (int p = tid; p < HXY; p += kThreads) {
        const int ly = p / HX, lx = p - ly * HX;
        const int gy = y0 - R + ly, gx = x0 - R + lx;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
            const size_t pix = (size_t)gy * W + gx;
            const float *hp = io.head + pix * (2 * M);
#pragma unroll
            for (int i = 0; i < M; ++i) Wl[i * HXY + p] = hp[i];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float c;
                if (FRAMES) c = io.r[pix * 3 + ch] / (io.a[pix * 3 + ch] + dc.eps_albedo);
                else c = io.c[pix * 3 + ch];
                cl[ch * HXY + p] = c;
            }
        } else {
#pragma unroll
            for (int i = 0; i < M; ++i) Wl[i * HXY + p] = 0.f;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) cl[ch * HXY + p] = 0.f;
        }
    }

    // each thread owns centres (tx, ty) and (tx, ty + 8)
    const int tx = tid & 31, ty = tid >> 5;
    float alpha[2][M], F[2][3];
    float outv[ADJ ? 2 : 1][ADJ ? M : 1][3];
    float Sv[ADJ ? 2 : 1][ADJ ? M : 1];
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        const int y = y0 + ty + 8 * o, x = x0 + tx;
        float lmax = -INFINITY;
        if (y < H && x < W) {
            const float *lp = io.head + ((size_t)y * W + x) * (2 * M) + M;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                alpha[o][i] = lp[i];
                lmax = fmaxf(lmax, alpha[o][i]);
            }
            float s = 0.f;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                alpha[o][i] = expf(alpha[o][i] - lmax);
                s += alpha[o][i];
            }
            const float inv = 1.f / s;
#pragma unroll
            for (int i = 0; i < M; ++i) alpha[o][i] *= inv;
        } else {
#pragma unroll
            for (int i = 0; i < M; ++i) alpha[o][i] = 0.f;
        }
        F[o][0] = F[o][1] = F[o][2] = 0.f;
    }
    __syncthreads();

#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int r = dc.radius[i];
        // horizontal pass over the rows this size needs: [R - r, R + 16 + r)
        const int row0 = R - r, nrows = kDTY + 2 * r;
        for (int it = tid; it < nrows * kDTX; it += kThreads) {
            const int hy = row0 + it / kDTX, xx = it % kDTX;
            const int base = hy * HX + xx + R;
            float S = 0.f, N0 = 0.f, N1 = 0.f, N2 = 0.f;
            for (int dx = -r; dx <= r; ++dx) {
                const float w = Wl[i * HXY + base + dx];
                S += w;
                N0 += w * cl[base + dx];
                N1 += w * cl[HXY + base + dx];
                N2 += w * cl[2 * HXY + base + dx];
            }
            const int q = hy * kDTX + xx;
            hb[q] = S;
            hb[HB + q] = N0;
            hb[2 * HB + q] = N1;
            hb[3 * HB + q] = N2;
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < 2; ++o) {
            const int yl = ty + 8 * o;
            float S = 0.f, N0 = 0.f, N1 = 0.f, N2 = 0.f;
            for (int dy = -r; dy <= r; ++dy) {
                const int q = (yl + R + dy) * kDTX + tx;
                S += hb[q];
                N0 += hb[HB + q];
                N1 += hb[2 * HB + q];
                N2 += hb[3 * HB + q];
            }
            const float inv = 1.f / fmaxf(S, dc.eps_norm);
            const float o0 = N0 * inv, o1 = N1 * inv, o2 = N2 * inv;
            if (ADJ) {
                outv[ADJ ? o : 0][ADJ ? i : 0][0] = o0;
                outv[ADJ ? o : 0][ADJ ? i : 0][1] = o1;
                outv[ADJ ? o : 0][ADJ ? i : 0][2] = o2;
                Sv[ADJ ? o : 0][ADJ ? i : 0] = S;
            } else {
                F[o][0] += alpha[o][i] * o0;
                F[o][1] += alpha[o][i] * o1;
                F[o][2] += alpha[o][i] * o2;
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int o = 0; o < 2; ++o) {
        const int y = y0 + ty + 8 * o, x = x0 + tx;
        if (y >= H || x >= W) continue;
        const size_t pix = (size_t)y * W + x;
        if (!ADJ) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float m = 1.f;
                if (FRAMES) m = io.a[pix * 3 + ch] + dc.eps_albedo;
                else if (io.mod) m = io.mod[pix * 3 + ch];
                io.out[pix * 3 + ch] = m * F[o][ch];
            }
        } else {
            float dF[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                dF[ch] = io.g[pix * 3 + ch] * (io.mod ? io.mod[pix * 3 + ch] : 1.f);
            float da[M], adot = 0.f;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const int oo = ADJ ? o : 0, ii = ADJ ? i : 0;
                da[i] = dF[0] * outv[oo][ii][0] + dF[1] * outv[oo][ii][1] + dF[2] * outv[oo][ii][2];
                adot += alpha[o][i] * da[i];
            }
            float *gh = io.grad_head + pix * (2 * M);
            const size_t P = (size_t)H * W;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const int oo = ADJ ? o : 0, ii = ADJ ? i : 0;
                gh[M + i] = alpha[o][i] * (da[i] - adot);
                const float S = Sv[oo][ii];
                const float inv = 1.f / fmaxf(S, dc.eps_norm);
                float4 v;
                v.x = alpha[o][i] * dF[0] * inv;
                v.y = alpha[o][i] * dF[1] * inv;
                v.z = alpha[o][i] * dF[2] * inv;
                v.w = S > dc.eps_norm
                          ? -(v.x * outv[oo][ii][0] + v.y * outv[oo][ii][1] + v.z * outv[oo][ii][2])
                          : 0.f;
                io.scratch[(size_t)i * P + pix] = v;
            }
        }
    }
}

// Second half of the vector-Jacobian product.  Windows are symmetric and
// truncated the same way at the border (p in Omega(q) <=> q in Omega(p)), so
// the adjoint of a box sum is the same box sum:
//   dW_i(q)  = sum_ch c_ch(q) box_i(u_i,ch)(q) + box_i(dS_i)(q)  -> grad_head[q][i]
//   dc_ch(q) = sum_i W_i(q) box_i(u_i,ch)(q)                      -> grad_c[q][ch]
// One size at a time: stage the halo of (u_i, dS_i) as float4, row sums,
// column sums.  LDS: [4][HY*HX] staged + [4][HY*32] row sums.
template <int M>
__global__ __launch_bounds__(kThreads) void decode_adj_b_kernel(DecodeCfg dc, DecodeTensors dt,
                                                                 float *grad_c)
{
    extern __shared__ float lds[];
    FrameArg fa{};
    DecodeIO io;
    int x0, y0;
    if (!decode_locate<false>(dc, fa, dt, io, x0, y0)) return;
    const int R = dc.R;
    const int HX = kDTX + 2 * R, HY = kDTY + 2 * R, HXY = HX * HY;
    float *st = lds;
    float *hb = st + 4 * HXY;
    const int HB = HY * kDTX;
    const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
    const int H = io.H, W = io.W;
    const size_t P = (size_t)H * W;
    const int fidx = (int)((io.head - dt.head) / ((size_t)P * 2 * M));
    float *gc = grad_c + (size_t)fidx * P * 3;

    float dcv[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    for (int i = 0; i < M; ++i) {
        const float4 *sp = io.scratch + (size_t)i * P;
        for (int p = tid; p < HXY; p += kThreads) {
            const int ly = p / HX, lx = p - ly * HX;
            const int gy = y0 - R + ly, gx = x0 - R + lx;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (gy >= 0 && gy < H && gx >= 0 && gx < W) v = sp[(size_t)gy * W + gx];
            st[p] = v.x;
            st[HXY + p] = v.y;
            st[2 * HXY + p] = v.z;
            st[3 * HXY + p] = v.w;
        }
        __syncthreads();
        const int r = dc.radius[i];
        const int row0 = R - r, nrows = kDTY + 2 * r;
        for (int it = tid; it < nrows * kDTX; it += kThreads) {
            const int hy = row0 + it / kDTX, xx = it % kDTX;
            const int base = hy * HX + xx + R;
            float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
            for (int dx = -r; dx <= r; ++dx) {
                a0 += st[base + dx];
                a1 += st[HXY + base + dx];
                a2 += st[2 * HXY + base + dx];
                a3 += st[3 * HXY + base + dx];
            }
            const int q = hy * kDTX + xx;
            hb[q] = a0;
            hb[HB + q] = a1;
            hb[2 * HB + q] = a2;
            hb[3 * HB + q] = a3;
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < 2; ++o) {
            const int yl = ty + 8 * o, y = y0 + yl, x = x0 + tx;
            float b0 = 0.f, b1 = 0.f, b2 = 0.f, b3 = 0.f;
            for (int dy = -r; dy <= r; ++dy) {
                const int q = (yl + R + dy) * kDTX + tx;
                b0 += hb[q];
                b1 += hb[HB + q];
                b2 += hb[2 * HB + q];
                b3 += hb[3 * HB + q];
            }
            if (y < H && x < W) {
                const size_t pix = (size_t)y * W + x;
                const float *cp = io.c + pix * 3;
                const float w = io.head[pix * (2 * M) + i];
                io.grad_head[pix * (2 * M) + i] = cp[0] * b0 + cp[1] * b1 + cp[2] * b2 + b3;
                dcv[o][0] += w * b0;
                dcv[o][1] += w * b1;
                dcv[o][2] += w * b2;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        const int y = y0 + ty + 8 * o, x = x0 + tx;
        if (y < H && x < W) {
            const size_t pix = (size_t)y * W + x;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) gc[pix * 3 + ch] = dcv[o][ch];
        }
    }
}

static size_t decode_lds_bytes(const DecodeCfg &dc)
{
    const int HX = kDTX + 2 * dc.R, HY = kDTY + 2 * dc.R;
    return sizeof(float) * ((size_t)(dc.M + 3) * HX * HY + 4 * (size_t)HY * kDTX);
}

static size_t adj_b_lds_bytes(const DecodeCfg &dc)
{
    const int HX = kDTX + 2 * dc.R, HY = kDTY + 2 * dc.R;
    return sizeof(float) * (4 * (size_t)HX * HY + 4 * (size_t)HY * kDTX);
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
    switch (dc.M) {
#define WSKP_M(m)                                                                                 \
    case m:                                                                                       \
        allow_lds(decode_fwd_kernel<m, KIND>, lds);                                               \
        hipLaunchKernelGGL((decode_fwd_kernel<m, KIND>), dim3(blocks), dim3(kThreads), lds, s, dc, \
                           fa, dt);                                                               \
        break;
        WSKP_M(1) WSKP_M(2) WSKP_M(3) WSKP_M(4) WSKP_M(5) WSKP_M(6) WSKP_M(7) WSKP_M(8)
#undef WSKP_M
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int decode_grid(int n, const int *H, const int *W)
{
    long total = 0;
    for (int f = 0; f < n; ++f)
        total += (long)((W[f] + kDTX - 1) / kDTX) * ((H[f] + kDTY - 1) / kDTY);
    return (int)total;
}

hipError_t launch_decode_frames(const DecodeCfg &dc, const FrameArg &fa, int blocks, hipStream_t s)
{
    DecodeTensors dt{};
    return launch_decode<DK_FRAMES>(dc, fa, dt, blocks, s);
}

hipError_t launch_decode_tensors(const DecodeCfg &dc, int N, int H, int W, const float *head,
                                 const float *c, const float *mod, float *out, hipStream_t s)
{
    FrameArg fa{};
    DecodeTensors dt{N, H, W, head, c, mod, out, nullptr, nullptr, nullptr};
    const int blocks = N * ((W + kDTX - 1) / kDTX) * ((H + kDTY - 1) / kDTY);
    return launch_decode<DK_TENSORS>(dc, fa, dt, blocks, s);
}

size_t decode_backward_scratch_bytes(const DecodeCfg &dc, int N, int H, int W)
{
    return (size_t)N * dc.M * H * W * sizeof(float4);
}

hipError_t launch_decode_backward(const DecodeCfg &dc, int N, int H, int W, const float *head,
                                  const float *c, const float *mod, const float *g,
                                  float *grad_head, float *grad_c, void *scratch, hipStream_t s)
{
    FrameArg fa{};
    DecodeTensors dt{N, H, W, head, c, mod, nullptr, g, grad_head,
                     reinterpret_cast<float4 *>(scratch)};
    const int blocks = N * ((W + kDTX - 1) / kDTX) * ((H + kDTY - 1) / kDTY);
    hipError_t e = launch_decode<DK_ADJ_A>(dc, fa, dt, blocks, s);
    if (e != hipSuccess) return e;
    const size_t lds = adj_b_lds_bytes(dc);
    switch (dc.M) {
#define WSKP_M(m)                                                                                 \
    case m:                                                                                       \
        allow_lds(decode_adj_b_kernel<m>, lds);                                                   \
        hipLaunchKernelGGL((decode_adj_b_kernel<m>), dim3(blocks), dim3(kThreads), lds, s, dc, dt, \
                           grad_c);                                                               \
        break;
        WSKP_M(1) WSKP_M(2) WSKP_M(3) WSKP_M(4) WSKP_M(5) WSKP_M(6) WSKP_M(7) WSKP_M(8)
#undef WSKP_M
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace wskp
