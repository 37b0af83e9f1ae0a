/*
 * Plain FP64 CPU oracle of the weight-sharing kernel-prediction (WSKP)
 * denoiser's per-frame path (Fan, Wang, Huo, Bao, "Real-time Monte Carlo
 * Denoising with Weight Sharing Kernel Prediction Network", EGSR 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the package's smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header, table or
 * helper with the HIP path.
 *
 * Every routine is the plain definition of its step, written as direct
 * loops: no tiling, no separable sums, no fused passes.  Inputs arrive as
 * float32 (the same arrays the GPU path reads) and are widened to double;
 * all arithmetic is double.
 *
 * Pins: every step below is checked by the tests against something other
 * than itself (closed forms, brute force, library routines, invariants,
 * finite differences).  End-to-end values of the whole path (preprocess,
 * U-Net, activation and decode composed) are parity unpinned against the
 * paper, which prints no numeric example and whose trained weights do not
 * exist here.
 *
 * Layouts: images are NHWC without the batch axis, i.e. element (y, x, ch)
 * of an H x W x C image sits at ((y * W) + x) * C + ch.  Conv weights are
 * OIHW: w[co][ci][ky][kx], followed in the blob by b[co].
 *
 * Build: gcc -O3 -fopenmp -shared -fPIC wskp_oracle.c -o libwskp_oracle.so -lm
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IDX(y, x, ch, W, C) ((((long)(y)) * (W) + (x)) * (C) + (ch))

/* ------------------------------------------------------------------------
 * Step 0: network input and albedo demodulation.
 * Sec. 5.1: the network sees LDR radiance (gamma tone mapping for the 1-spp
 * data), albedo, and normal and depth linearly scaled to [0, 1] -- ten
 * channels in this order.  Sec. 4.2 (end): the filter runs on the irradiance,
 * i.e. the radiance with the albedo divided out, and the albedo is
 * multiplied back at the end.
 *   X = [ clamp(r,0,1)^(1/gamma), a, (n+1)/2, clamp((d-near)/(far-near),0,1) ]
 *   c = r / (a + eps_a),  mod = a + eps_a
 * ---------------------------------------------------------------------- */
void wo_preprocess(long H, long W, const float *r, const float *a, const float *n,
                   const float *d, double gamma, double dnear, double dfar, double eps_a,
                   double *X, double *c, double *mod)
{
    for (long p = 0; p < H * W; ++p) {
        for (int ch = 0; ch < 3; ++ch) {
            double rv = r[p * 3 + ch];
            double lo = rv < 0.0 ? 0.0 : (rv > 1.0 ? 1.0 : rv);
            X[p * 10 + ch] = pow(lo, 1.0 / gamma);
            X[p * 10 + 3 + ch] = a[p * 3 + ch];
            X[p * 10 + 6 + ch] = (n[p * 3 + ch] + 1.0) * 0.5;
            double m = (double)a[p * 3 + ch] + eps_a;
            if (c) c[p * 3 + ch] = rv / m;
            if (mod) mod[p * 3 + ch] = m;
        }
        double t = ((double)d[p] - dnear) / (dfar - dnear);
        X[p * 10 + 9] = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    }
}

/* k x k cross-correlation (k odd), stride 1, zero padding (k-1)/2, plus
 * bias (the usual CNN convolution); optional ReLU.  With r = (k-1)/2:
 *   out[y][x][co] = b[co] +
 *     sum_{ci,ky,kx} w[co][ci][ky][kx] * in[y+ky-r][x+kx-r][ci].
 * k = 3 is the prediction network's conv (Sec. 4.1); k = 1, 3 and 5 are the
 * branches of a RepVGG block and k = 5 its merged inference form (Sec. 4.1,
 * prediction phase). */
void wo_conv2d(long H, long W, long Cin, long Cout, int k, const double *in,
               const double *w, const double *b, int relu, double *out)
{
    const int r = (k - 1) / 2;
#pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x)
            for (long co = 0; co < Cout; ++co) {
                double acc = b[co];
                for (long ci = 0; ci < Cin; ++ci)
                    for (int ky = 0; ky < k; ++ky) {
                        long yy = y + ky - r;
                        if (yy < 0 || yy >= H) continue;
                        for (int kx = 0; kx < k; ++kx) {
                            long xx = x + kx - r;
                            if (xx < 0 || xx >= W) continue;
                            acc += w[((co * Cin + ci) * k + ky) * k + kx] * in[IDX(yy, xx, ci, W, Cin)];
                        }
                    }
                out[IDX(y, x, co, W, Cout)] = (relu && acc < 0.0) ? 0.0 : acc;
            }
}

void wo_conv3x3(long H, long W, long Cin, long Cout, const double *in,
                const double *w, const double *b, int relu, double *out)
{
    wo_conv2d(H, W, Cin, Cout, 3, in, w, b, relu, out);
}

/* 2x2 mean, stride 2 (the D operator of Sec. 5.2). out is [H/2, W/2, C]. */
void wo_avgpool2(long H, long W, long C, const double *in, double *out)
{
    long Ho = H / 2, Wo = W / 2;
    for (long y = 0; y < Ho; ++y)
        for (long x = 0; x < Wo; ++x)
            for (long ch = 0; ch < C; ++ch)
                out[IDX(y, x, ch, Wo, C)] = 0.25 * (in[IDX(2 * y, 2 * x, ch, W, C)] +
                                                    in[IDX(2 * y, 2 * x + 1, ch, W, C)] +
                                                    in[IDX(2 * y + 1, 2 * x, ch, W, C)] +
                                                    in[IDX(2 * y + 1, 2 * x + 1, ch, W, C)]);
}

/* Nearest-neighbour x2 upsampling (the U operator of Sec. 5.2).
 * in is [H, W, C], out is [2H, 2W, C]. */
void wo_upsample2(long H, long W, long C, const double *in, double *out)
{
    for (long y = 0; y < 2 * H; ++y)
        for (long x = 0; x < 2 * W; ++x)
            for (long ch = 0; ch < C; ++ch)
                out[IDX(y, x, ch, 2 * W, C)] = in[IDX(y / 2, x / 2, ch, W, C)];
}

/* Channel concatenation [a, b] of two images with P pixels. */
void wo_concat(long P, long Ca, const double *a, long Cb, const double *b, double *out)
{
    for (long p = 0; p < P; ++p) {
        for (long ch = 0; ch < Ca; ++ch) out[p * (Ca + Cb) + ch] = a[p * Ca + ch];
        for (long ch = 0; ch < Cb; ++ch) out[p * (Ca + Cb) + Ca + ch] = b[p * Cb + ch];
    }
}

static double *widen(const float *src, long n)
{
    double *d = (double *)malloc(sizeof(double) * (size_t)n);
    for (long i = 0; i < n; ++i) d[i] = src[i];
    return d;
}

/* Runs one k x k conv of the blob: reads w (Cout*Cin*k*k) then b (Cout) at *off. */
static void blob_conv(const float *blob, long *off, long H, long W, long Cin, long Cout, int k,
                      const double *in, int relu, double *out)
{
    double *w = widen(blob + *off, Cout * Cin * k * k);
    *off += Cout * Cin * k * k;
    double *b = widen(blob + *off, Cout);
    *off += Cout;
    wo_conv2d(H, W, Cin, Cout, k, in, w, b, relu, out);
    free(w);
    free(b);
}

/* ------------------------------------------------------------------------
 * The prediction network (Sec. 4.1, Eq. 2): a U-Net of L levels.
 *   e_0 = ReLU(conv(X));  e_l = ReLU(conv(pool(e_{l-1}))),  l = 1..L-1
 *   u_{L-1} = e_{L-1};    u_l = ReLU(conv([up(u_{l+1}), e_l])),  l = L-2..0
 *   h = conv(u_0)         (Cout = 2M raw outputs, no activation)
 * Every conv is k x k (k = 3, or k = 5 for a net of merged RepVGG blocks).
 * H and W must be multiples of 2^(L-1).  Weights in blob order
 * enc0..enc_{L-1}, dec_{L-2}..dec_0, head.  Returns 0 on success.
 * ---------------------------------------------------------------------- */
int wo_unet(long H, long W, int L, const int *ch, int Cin, int Cout, int k, const float *blob,
            const double *X, double *h)
{
    if (L < 1 || L > 8 || k < 1 || k % 2 == 0) return -1;
    double *e[8], *u[8];
    long Hl[8], Wl[8];
    long off = 0;
    for (int l = 0; l < L; ++l) {
        Hl[l] = H >> l;
        Wl[l] = W >> l;
        if ((Hl[l] << l) != H || (Wl[l] << l) != W) return -2;
        e[l] = (double *)malloc(sizeof(double) * (size_t)(Hl[l] * Wl[l] * ch[l]));
        u[l] = NULL;
    }
    blob_conv(blob, &off, H, W, Cin, ch[0], k, X, 1, e[0]);
    for (int l = 1; l < L; ++l) {
        double *p = (double *)malloc(sizeof(double) * (size_t)(Hl[l] * Wl[l] * ch[l - 1]));
        wo_avgpool2(Hl[l - 1], Wl[l - 1], ch[l - 1], e[l - 1], p);
        blob_conv(blob, &off, Hl[l], Wl[l], ch[l - 1], ch[l], k, p, 1, e[l]);
        free(p);
    }
    u[L - 1] = e[L - 1];
    for (int l = L - 2; l >= 0; --l) {
        long P = Hl[l] * Wl[l];
        double *up = (double *)malloc(sizeof(double) * (size_t)(P * ch[l + 1]));
        wo_upsample2(Hl[l + 1], Wl[l + 1], ch[l + 1], u[l + 1], up);
        double *cat = (double *)malloc(sizeof(double) * (size_t)(P * (ch[l + 1] + ch[l])));
        wo_concat(P, ch[l + 1], up, ch[l], e[l], cat);
        u[l] = (double *)malloc(sizeof(double) * (size_t)(P * ch[l]));
        blob_conv(blob, &off, Hl[l], Wl[l], ch[l + 1] + ch[l], ch[l], k, cat, 1, u[l]);
        free(up);
        free(cat);
    }
    blob_conv(blob, &off, H, W, ch[0], Cout, k, u[0], 0, h);
    for (int l = 0; l < L; ++l) {
        if (u[l] && u[l] != e[l]) free(u[l]);
        free(e[l]);
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Step 2: the per-pixel weight maps and the fusion logits (Eq. 2, Eq. 3,
 * Sec. 4.2 "Kernel Fusion").  head[p][i] = act(h[p][i]) for i < M, where act
 * is softplus(x) = log(1 + e^x) (act == 0) or exp (act == 1, the paper's
 * Eq. 3 numerator); head[p][M + i] = h[p][M + i] (raw logits).
 * ---------------------------------------------------------------------- */
void wo_activate(long P, int M, int act, const double *h, double *head)
{
    for (long p = 0; p < P; ++p)
        for (int i = 0; i < 2 * M; ++i) {
            double v = h[p * 2 * M + i];
            if (i < M) {
                if (act == 1) v = exp(v);
                else v = (v > 0.0 ? v : 0.0) + log1p(exp(-fabs(v)));
            }
            head[p * 2 * M + i] = v;
        }
}

/* ------------------------------------------------------------------------
 * Steps 3-5: kernel construction, filtering, fusion and remodulation.
 *   Eq. 3 / Eq. 4:  for each size k_i with radius r_i = (k_i - 1)/2 and
 *     window Omega_i(p) = pixels q inside the image with |q - p|_inf <= r_i,
 *       S_i(p)    = sum_{q in Omega_i(p)} W_i(q)
 *       N_i,ch(p) = sum_{q in Omega_i(p)} W_i(q) c_ch(q)
 *       out_i,ch(p) = N_i,ch(p) / max(S_i(p), eps)
 *   (The normalised weight W_i(q)/S_i(p) is the kernel weight of Eq. 3;
 *   with W = exp(I) it is exactly the window softmax.)
 *   Eq. 5:  alpha = softmax_i(logit_i(p)),  F(p) = sum_i alpha_i out_i(p)
 *   Sec. 4.2 (end):  y = mod * F.
 * head is [H, W, 2M] (weights then logits), c and mod are [H, W, 3]; mod may
 * be NULL (taken as 1).  y is [H, W, 3].  outs ([H, W, M, 3]) and alpha
 * ([H, W, M]) are optional diagnostics (NULL to skip).
 * ---------------------------------------------------------------------- */
void wo_decode(long H, long W, int M, const int *ks, const double *head, const double *c,
               const double *mod, double eps, double *y, double *outs, double *alpha)
{
#pragma omp parallel for schedule(static)
    for (long py = 0; py < H; ++py)
        for (long px = 0; px < W; ++px) {
            long p = py * W + px;
            double o[16][3], lmax = -INFINITY, al[16], asum = 0.0;
            for (int i = 0; i < M; ++i) {
                long r = (ks[i] - 1) / 2;
                double S = 0.0, N[3] = {0.0, 0.0, 0.0};
                for (long qy = py - r; qy <= py + r; ++qy) {
                    if (qy < 0 || qy >= H) continue;
                    for (long qx = px - r; qx <= px + r; ++qx) {
                        if (qx < 0 || qx >= W) continue;
                        long q = qy * W + qx;
                        double w = head[q * 2 * M + i];
                        S += w;
                        for (int ch = 0; ch < 3; ++ch) N[ch] += w * c[q * 3 + ch];
                    }
                }
                double den = S > eps ? S : eps;
                for (int ch = 0; ch < 3; ++ch) o[i][ch] = N[ch] / den;
                double l = head[p * 2 * M + M + i];
                if (l > lmax) lmax = l;
            }
            for (int i = 0; i < M; ++i) {
                al[i] = exp(head[p * 2 * M + M + i] - lmax);
                asum += al[i];
            }
            for (int ch = 0; ch < 3; ++ch) {
                double F = 0.0;
                for (int i = 0; i < M; ++i) F += (al[i] / asum) * o[i][ch];
                y[p * 3 + ch] = (mod ? mod[p * 3 + ch] : 1.0) * F;
            }
            if (outs)
                for (int i = 0; i < M; ++i)
                    for (int ch = 0; ch < 3; ++ch) outs[(p * M + i) * 3 + ch] = o[i][ch];
            if (alpha)
                for (int i = 0; i < M; ++i) alpha[p * M + i] = al[i] / asum;
        }
}

/* ------------------------------------------------------------------------
 * Vector-Jacobian product of wo_decode: given g = dL/dy [H, W, 3], returns
 * dhead = dL/d(head) [H, W, 2M] (weights, then logits) and dc = dL/dc
 * [H, W, 3].  Reverse mode of the loops above, taken literally: every
 * centre p scatters into the window it read.  mod is treated as a constant.
 * Single-threaded (the scatter has write conflicts).
 * ---------------------------------------------------------------------- */
void wo_decode_vjp(long H, long W, int M, const int *ks, const double *head, const double *c,
                   const double *mod, double eps, const double *g, double *dhead, double *dc)
{
    memset(dhead, 0, sizeof(double) * (size_t)(H * W * 2 * M));
    memset(dc, 0, sizeof(double) * (size_t)(H * W * 3));
    for (long py = 0; py < H; ++py)
        for (long px = 0; px < W; ++px) {
            long p = py * W + px;
            double S[16], N[16][3], o[16][3], al[16], lmax = -INFINITY, asum = 0.0;
            for (int i = 0; i < M; ++i) {
                long r = (ks[i] - 1) / 2;
                S[i] = 0.0;
                N[i][0] = N[i][1] = N[i][2] = 0.0;
                for (long qy = py - r; qy <= py + r; ++qy) {
                    if (qy < 0 || qy >= H) continue;
                    for (long qx = px - r; qx <= px + r; ++qx) {
                        if (qx < 0 || qx >= W) continue;
                        long q = qy * W + qx;
                        double w = head[q * 2 * M + i];
                        S[i] += w;
                        for (int ch = 0; ch < 3; ++ch) N[i][ch] += w * c[q * 3 + ch];
                    }
                }
                double den = S[i] > eps ? S[i] : eps;
                for (int ch = 0; ch < 3; ++ch) o[i][ch] = N[i][ch] / den;
                double l = head[p * 2 * M + M + i];
                if (l > lmax) lmax = l;
            }
            for (int i = 0; i < M; ++i) {
                al[i] = exp(head[p * 2 * M + M + i] - lmax);
                asum += al[i];
            }
            for (int i = 0; i < M; ++i) al[i] /= asum;
            /* y = mod * sum_i alpha_i o_i  ->  dF = g * mod */
            double dF[3];
            for (int ch = 0; ch < 3; ++ch) dF[ch] = g[p * 3 + ch] * (mod ? mod[p * 3 + ch] : 1.0);
            /* d alpha_i = <dF, o_i>; softmax backward to the logits */
            double da[16], adot = 0.0;
            for (int i = 0; i < M; ++i) {
                da[i] = dF[0] * o[i][0] + dF[1] * o[i][1] + dF[2] * o[i][2];
                adot += al[i] * da[i];
            }
            for (int i = 0; i < M; ++i) dhead[p * 2 * M + M + i] += al[i] * (da[i] - adot);
            /* o_i = N_i / max(S_i, eps) */
            for (int i = 0; i < M; ++i) {
                double den = S[i] > eps ? S[i] : eps;
                double dN[3], dS = 0.0;
                for (int ch = 0; ch < 3; ++ch) {
                    double dO = al[i] * dF[ch];
                    dN[ch] = dO / den;
                    if (S[i] > eps) dS -= dO * N[i][ch] / (den * den);
                }
                long r = (ks[i] - 1) / 2;
                for (long qy = py - r; qy <= py + r; ++qy) {
                    if (qy < 0 || qy >= H) continue;
                    for (long qx = px - r; qx <= px + r; ++qx) {
                        if (qx < 0 || qx >= W) continue;
                        long q = qy * W + qx;
                        double w = head[q * 2 * M + i];
                        double dw = dS;
                        for (int ch = 0; ch < 3; ++ch) {
                            dw += dN[ch] * c[q * 3 + ch];
                            dc[q * 3 + ch] += dN[ch] * w;
                        }
                        dhead[q * 2 * M + i] += dw;
                    }
                }
            }
        }
}

/* L1 loss mean|y - t| over n elements and its gradient sign(y - t)/n with
 * sign(0) = 0. */
double wo_l1(long n, const double *y, const double *t, double *g)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) {
        double d = y[i] - t[i];
        s += fabs(d);
        if (g) g[i] = (d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0)) / (double)n;
    }
    return s / (double)n;
}

/* ------------------------------------------------------------------------
 * Temporal accumulation before denoising (Sec. 4.1, last paragraph): the
 * previous frame's accumulated radiance is reprojected to the current frame
 * with the motion vector; where the geometry agrees (world position and
 * shading normal) it is blended with the current 1-spp radiance, elsewhere
 * the current radiance is kept.  The paper gives no formulas; the reading
 * taken here (the usual one for such filters):
 *   q = p + mv(p)            position of p's surface point in the previous
 *                            frame (pixel-centre units)
 *   taps: the 4 pixels around q with bilinear weights; a tap counts if it
 *   lies in the image, |wp_prev(tap) - wp(p)|^2 <= pos_tol^2 and
 *   n_prev(tap) . n(p) >= normal_tol
 *   with S = sum of the counted weights:
 *     S > 0:  h = sum w prev_r / S,  L = sum w prev_len / S,
 *             alpha = max(1 / (L + 1), alpha_min),
 *             out = (1 - alpha) h + alpha r,  len = L + 1
 *     S = 0:  out = r,  len = 1
 *   prev_r == NULL (first frame): out = r, len = 1 everywhere.
 * The tap tests take fp32 inputs; their squared distance and dot product
 * are exact or correctly rounded in double, so any implementation that
 * evaluates them in double reaches the same decisions.
 * ---------------------------------------------------------------------- */
void wo_temporal(long H, long W, const float *r, const float *n, const float *wp, const float *mv,
                 const float *prev_r, const float *prev_len, const float *prev_n,
                 const float *prev_wp, double alpha_min, double pos_tol, double normal_tol,
                 double *out, double *len)
{
#pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            const long p = y * W + x;
            if (!prev_r) {
                for (int ch = 0; ch < 3; ++ch) out[p * 3 + ch] = (double)r[p * 3 + ch];
                len[p] = 1.0;
                continue;
            }
            const double qx = (double)x + (double)mv[p * 2 + 0];
            const double qy = (double)y + (double)mv[p * 2 + 1];
            const double x0 = floor(qx), y0 = floor(qy);
            const double fx = qx - x0, fy = qy - y0;
            double S = 0.0, L = 0.0, h[3] = {0.0, 0.0, 0.0};
            for (int t = 0; t < 4; ++t) {
                const long tx = (long)x0 + (t & 1), ty = (long)y0 + (t >> 1);
                const double w = ((t & 1) ? fx : 1.0 - fx) * ((t >> 1) ? fy : 1.0 - fy);
                if (tx < 0 || tx >= W || ty < 0 || ty >= H) continue;
                const long q = ty * W + tx;
                double d2 = 0.0, dot = 0.0;
                for (int k = 0; k < 3; ++k) {
                    const double d = (double)prev_wp[q * 3 + k] - (double)wp[p * 3 + k];
                    d2 += d * d;
                    dot += (double)prev_n[q * 3 + k] * (double)n[p * 3 + k];
                }
                if (!(d2 <= pos_tol * pos_tol && dot >= normal_tol)) continue;
                S += w;
                L += w * (double)prev_len[q];
                for (int ch = 0; ch < 3; ++ch) h[ch] += w * (double)prev_r[q * 3 + ch];
            }
            if (S > 0.0) {
                L /= S;
                double a = 1.0 / (L + 1.0);
                if (a < alpha_min) a = alpha_min;
                for (int ch = 0; ch < 3; ++ch)
                    out[p * 3 + ch] = (1.0 - a) * (h[ch] / S) + a * (double)r[p * 3 + ch];
                len[p] = L + 1.0;
            } else {
                for (int ch = 0; ch < 3; ++ch) out[p * 3 + ch] = (double)r[p * 3 + ch];
                len[p] = 1.0;
            }
        }
}

/* ------------------------------------------------------------------------
 * Multi-resolution blend (Eq. 7, Sec. 5.2): filtered images of two adjacent
 * resolutions, fine i^f [H,W,3] and coarse i^c [H/2,W/2,3], are combined
 * with a per-pixel weight alpha [H,W] as
 *   o_p = i^f_p - alpha_p [U D i^f]_p + alpha_p [U i^c]_p
 * D: 2x2 mean (downsampling), U: nearest-neighbour upsampling, so for fine
 * pixel (y, x) both bracketed terms are taken at coarse pixel (y/2, x/2).
 * H and W are even.
 * ---------------------------------------------------------------------- */
void wo_mr_blend(long H, long W, const double *fine, const double *coarse, const double *alpha,
                 double *out)
{
    const long Wc = W / 2;
#pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            const long yc = y / 2, xc = x / 2;
            const double a = alpha[y * W + x];
            for (int ch = 0; ch < 3; ++ch) {
                const double dfine = 0.25 * (fine[IDX(2 * yc, 2 * xc, ch, W, 3)] +
                                             fine[IDX(2 * yc, 2 * xc + 1, ch, W, 3)] +
                                             fine[IDX(2 * yc + 1, 2 * xc, ch, W, 3)] +
                                             fine[IDX(2 * yc + 1, 2 * xc + 1, ch, W, 3)]);
                out[IDX(y, x, ch, W, 3)] =
                    fine[IDX(y, x, ch, W, 3)] - a * dfine + a * coarse[IDX(yc, xc, ch, Wc, 3)];
            }
        }
}

/* ------------------------------------------------------------------------
 * Training (Eq. 1: the network's parameters minimise the loss between the
 * reconstruction and the reference; Eq. 6: SMAPE; Sec. 5.3: Adam).  Plain
 * definitions of each step's derivative.
 * ---------------------------------------------------------------------- */

/* SMAPE over n = 3N values (Eq. 6) and its gradient with respect to R:
 *   s = (1/n) sum |R - t| / (|R| + |t| + eps)
 *   ds/dR = (1/n) [sign(R - t) (|R| + |t| + eps) - |R - t| sign(R)] / (|R| + |t| + eps)^2
 * with sign(0) = 0. */
double wo_smape(long n, const double *R, const double *t, double eps, double *g)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) {
        const double d = R[i] - t[i];
        const double den = fabs(R[i]) + fabs(t[i]) + eps;
        s += fabs(d) / den;
        if (g) {
            const double sd = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
            const double sr = R[i] > 0.0 ? 1.0 : (R[i] < 0.0 ? -1.0 : 0.0);
            g[i] = (sd * den - fabs(d) * sr) / (den * den) / (double)n;
        }
    }
    return s / (double)n;
}

/* Backward of out = conv3x3(in; w, b) (before any ReLU):
 *   din[y][x][ci] = sum_{co,ky,kx} g[y-ky+1][x-kx+1][co] w[co][ci][ky][kx]
 *   dw[co][ci][ky][kx] = sum_{y,x} g[y][x][co] in[y+ky-1][x+kx-1][ci]
 *   db[co] = sum_{y,x} g[y][x][co]
 * (zero padding; din may be NULL).  dw and db are overwritten. */
void wo_conv3x3_backward(long H, long W, long Cin, long Cout, const double *in, const double *w,
                         const double *g, double *din, double *dw, double *db)
{
    if (din) {
#pragma omp parallel for schedule(static)
        for (long y = 0; y < H; ++y)
            for (long x = 0; x < W; ++x)
                for (long ci = 0; ci < Cin; ++ci) {
                    double acc = 0.0;
                    for (int ky = 0; ky < 3; ++ky) {
                        const long yy = y - ky + 1;
                        if (yy < 0 || yy >= H) continue;
                        for (int kx = 0; kx < 3; ++kx) {
                            const long xx = x - kx + 1;
                            if (xx < 0 || xx >= W) continue;
                            for (long co = 0; co < Cout; ++co)
                                acc += g[IDX(yy, xx, co, W, Cout)] * w[((co * Cin + ci) * 3 + ky) * 3 + kx];
                        }
                    }
                    din[IDX(y, x, ci, W, Cin)] = acc;
                }
    }
#pragma omp parallel for schedule(static)
    for (long co = 0; co < Cout; ++co) {
        double sb = 0.0;
        for (long p = 0; p < H * W; ++p) sb += g[p * Cout + co];
        db[co] = sb;
        for (long ci = 0; ci < Cin; ++ci)
            for (int ky = 0; ky < 3; ++ky)
                for (int kx = 0; kx < 3; ++kx) {
                    double acc = 0.0;
                    for (long y = 0; y < H; ++y) {
                        const long yy = y + ky - 1;
                        if (yy < 0 || yy >= H) continue;
                        for (long x = 0; x < W; ++x) {
                            const long xx = x + kx - 1;
                            if (xx < 0 || xx >= W) continue;
                            acc += g[IDX(y, x, co, W, Cout)] * in[IDX(yy, xx, ci, W, Cin)];
                        }
                    }
                    dw[((co * Cin + ci) * 3 + ky) * 3 + kx] = acc;
                }
    }
}

/* Backward of the 2x2 mean: din[y][x] = dout[y/2][x/2] / 4 (din [H,W,C]). */
void wo_avgpool2_backward(long H, long W, long C, const double *dout, double *din)
{
    const long Wo = W / 2;
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x)
            for (long ch = 0; ch < C; ++ch)
                din[IDX(y, x, ch, W, C)] = 0.25 * dout[IDX(y / 2, x / 2, ch, Wo, C)];
}

/* Backward of nearest x2 upsampling: din[y][x] = sum of dout over the 2x2
 * block (din [H,W,C], dout [2H,2W,C]). */
void wo_upsample2_backward(long H, long W, long C, const double *dout, double *din)
{
    const long W2 = 2 * W;
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x)
            for (long ch = 0; ch < C; ++ch)
                din[IDX(y, x, ch, W, C)] = dout[IDX(2 * y, 2 * x, ch, W2, C)] +
                                           dout[IDX(2 * y, 2 * x + 1, ch, W2, C)] +
                                           dout[IDX(2 * y + 1, 2 * x, ch, W2, C)] +
                                           dout[IDX(2 * y + 1, 2 * x + 1, ch, W2, C)];
}

/* Adam (Kingma and Ba; Sec. 5.3 trains with it): for step t >= 1,
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
void wo_adam(long n, double *w, const double *g, double *m, double *v, long t, double lr, double b1,
             double b2, double eps)
{
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (long i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        w[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
