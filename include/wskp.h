/*
 * wskp.h -- C ABI of the MI355X (gfx950) weight-sharing kernel-prediction
 * (WSKP) Monte Carlo denoiser.
 *
 * Method: Fan, Wang, Huo, Bao, "Real-time Monte Carlo Denoising with Weight
 * Sharing Kernel Prediction Network" (EGSR 2021).  A convolutional network
 * (Sec. 4.1, Eq. 2) predicts one scalar weight per pixel for each of M
 * filter sizes plus M per-pixel fusion logits.  Every pixel's k x k kernel
 * is built from its neighbours' scalars and normalised over the window
 * (Eq. 3), applied to the albedo-demodulated irradiance (Eq. 4, Sec. 4.2),
 * the M filtered images are blended with softmax weights (Eq. 5) and the
 * albedo is multiplied back (Sec. 4.2, last paragraph).
 *
 * Conventions shared by every entry point:
 *  - Images are NHWC float32, channels innermost, rows of W pixels, fully
 *    contiguous.  A batch of N frames of one size is N images back to back.
 *  - Every tensor pointer is a DEVICE pointer owned by the caller.  It must
 *    stay valid until the work queued on `stream` has completed.  The
 *    library never frees or retains caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    All work is queued asynchronously on it.  wskp_create, wskp_destroy and
 *    wskp_timing_enable synchronise the device; wskp_denoise_batch may wait
 *    for the host-to-device copy of its own frame table from 8 calls earlier
 *    (its pinned staging ring), and with WSKP_BATCH_GRAPH the first batch of
 *    a new capacity bucket allocates and captures a graph; no other call
 *    waits for the device.
 *  - Calls validate their arguments synchronously and return a status; no
 *    exception crosses the ABI.  A failed call queues no work.  Faults that
 *    happen later on the device surface at the caller's next
 *    synchronisation.  wskp_last_error() gives a thread-local message for
 *    the last failing call.
 *  - A handle may be used from several host threads at once only with
 *    distinct streams and distinct workspaces.
 */
#ifndef WSKP_H
#define WSKP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wskp_ctx *wskp_handle_t;

typedef enum {
    WSKP_OK = 0,
    WSKP_E_INVALID_ARG = -1, /* NULL pointer, bad config value, weight count mismatch */
    WSKP_E_SHAPE = -2,       /* H or W < 1, or not a multiple of 2^(levels-1) for the net */
    WSKP_E_UNSUPPORTED = -3, /* valid request the library does not implement */
    WSKP_E_DEVICE = -4,      /* no usable gfx950 device, or a HIP runtime error */
    WSKP_E_OOM = -5,         /* device or pinned-host allocation failed */
    WSKP_E_BUDGET = -6,      /* workspace too small for the request */
    WSKP_E_LAUNCH = -7,      /* a kernel launch was rejected by the runtime */
    WSKP_E_INTERNAL = -8
} wskp_status_t;

/* Arithmetic of the convolutions.  Decode, normalisation and fusion are
 * always float32. */
typedef enum {
    WSKP_PREC_FP32 = 0,    /* fp32 operands, fp32 MFMA accumulate */
    WSKP_PREC_BF16 = 1,    /* bf16 operands (round to nearest even), fp32 accumulate */
    WSKP_PREC_FP8_E4M3 = 2 /* OCP e4m3 operands with scales, fp32 accumulate */
} wskp_precision_t;

/* Map from the network's raw output h to the positive per-pixel weight W. */
typedef enum {
    WSKP_ACT_SOFTPLUS = 0, /* W = log(1 + e^h) */
    WSKP_ACT_EXP = 1       /* W = e^h: the numerator of the window softmax, Eq. 3 */
} wskp_weight_act_t;

#define WSKP_MAX_LEVELS 6
#define WSKP_MAX_KERNELS 8
#define WSKP_MAX_KERNEL_SIZE 15

/* Network and filter configuration.
 *  levels         U-Net depth L (1..6); frame sides must be multiples of 2^(L-1)
 *  channels[l]    width of level l, multiples of 16 (level 0 = full resolution)
 *  num_kernels    M, number of filter sizes (1..8); the net outputs 2M channels
 *  kernel_sizes   odd sizes k_i (1..15), one per weight map (Sec. 4.2, "Kernel
 *                 Fusion": k_i = k_b + i k_s)
 *  precision      wskp_precision_t of the convolutions
 *  weight_act     wskp_weight_act_t
 *  eps_norm       floor of the window sum: out = N / max(S, eps_norm)
 *  eps_albedo     c = r / (a + eps_albedo); the same factor remodulates
 *  gamma          tone map of the network's radiance input: clamp(r,0,1)^(1/gamma)
 *  depth_near/far depth scaled as clamp((d - near)/(far - near), 0, 1)
 *  conv_size      3, or 5: every conv is a k x k conv with k = conv_size; 5 is
 *                 the inference form of a RepVGG block (Sec. 4.1, prediction
 *                 phase; see wskp_repvgg_merge).  5 supports FP32 and BF16.
 * Network input channels (Sec. 5.1): [tonemapped r (3), albedo (3),
 * (normal + 1)/2 (3), scaled depth (1)]. */
typedef struct {
    uint32_t struct_size; /* sizeof(wskp_config_t) */
    int32_t levels;
    int32_t channels[8];
    int32_t num_kernels;
    int32_t kernel_sizes[8];
    int32_t precision;
    int32_t weight_act;
    float eps_norm;
    float eps_albedo;
    float gamma;
    float depth_near;
    float depth_far;
    int32_t conv_size;
} wskp_config_t;

/* One frame of a batch.  Device pointers, NHWC float32:
 * radiance/albedo/normal [H,W,3], depth [H,W,1], out [H,W,3]. */
typedef struct {
    int32_t H, W;
    const float *radiance;
    const float *albedo;
    const float *normal;
    const float *depth;
    float *out;
} wskp_frame_t;

/* Number of float32 values in the weight blob for `cfg`.  Blob order:
 * enc0..enc_{L-1}, dec_{L-2}..dec_0, head; each conv is w[C_out][C_in][k][k]
 * (k = conv_size) followed by b[C_out].  enc0 has C_in = 10, enc_l has C_in = C_{l-1},
 * dec_l has C_in = C_{l+1} + C_l (upsampled coarse features first), head
 * has C_in = C_0 and C_out = 2M (M weight channels, then M logits).
 * Returns 0 for an invalid config. */
size_t wskp_num_weights(const wskp_config_t *cfg);

/* Creates a handle on HIP device `device` for the prediction network of
 * Sec. 4.1 (Eq. 2: the network maps the noisy frame and its auxiliary
 * buffers to the per-pixel scalars that define every kernel) and the kernel
 * set of Sec. 4.2: validates cfg, copies the host weight blob (n_weights
 * floats, owned by the caller, not retained) to the device in the layout
 * the kernels read.  Synchronous.
 * host_act_scales: for WSKP_PREC_FP8_E4M3 only (ignored otherwise, may be
 * NULL), one positive float per conv in blob order: the scale s of that
 * conv's input activations, which are stored as e4m3(x / s) (values beyond
 * +-448 s saturate).  Weights are quantised per output channel with
 * s_w = max|w| / 448.  FP8 needs every level width to be a multiple of 32. */
wskp_status_t wskp_create(const wskp_config_t *cfg, const float *host_weights, size_t n_weights,
                          const float *host_act_scales, int device, wskp_handle_t *out);

/* RepVGG re-parameterisation (Sec. 4.1, prediction phase): a block that is,
 * during training, the sum of a 1x1, a 3x3 and a 5x5 conv branch (each with
 * its bias, zero padding (k-1)/2) plus, when C_in == C_out, the identity,
 * computes the same map as ONE 5x5 conv; this writes that conv's weights.
 * Host arrays, OIHW: w1 [cout][cin][1][1], w3 [cout][cin][3][3],
 * w5 [cout][cin][5][5], biases [cout]; a branch whose w and b are both NULL
 * is absent (exactly one of them NULL: WSKP_E_INVALID_ARG).  identity != 0
 * adds the identity branch (needs cin == cout).
 * Output: w_out [cout][cin][5][5] (each branch's kernel centred, the identity
 * a unit centre tap of (c, c)) and b_out [cout] (the biases summed), in the
 * layout of one conv of the weight blob with conv_size = 5.  Pure host
 * arithmetic in float32, synchronous, no device needed. */
wskp_status_t wskp_repvgg_merge(int cin, int cout, const float *w1, const float *b1,
                                const float *w3, const float *b3, const float *w5,
                                const float *b5, int identity, float *w_out, float *b_out);

/* Releases the handle's device memory.  Synchronises the device first. */
wskp_status_t wskp_destroy(wskp_handle_t h);

/* Bytes of device workspace that wskp_denoise (n = 1) or
 * wskp_denoise_batch needs for n frames of sizes H[i] x W[i]. */
wskp_status_t wskp_workspace_size(wskp_handle_t h, int n, const int *H, const int *W,
                                  size_t *bytes);

/* Denoises one frame (the problem of Sec. 3: noisy radiance plus albedo,
 * normal and depth in, denoised radiance out).  Inputs as wskp_frame_t;
 * `out` [H,W,3] receives albedo * fused filtered irradiance.  `ws` is a
 * device workspace of ws_bytes >= wskp_workspace_size(h, 1, &H, &W);
 * its content is scratch (the intermediate feature maps and the head
 * record, planar [2M][H][W]: weight maps W_i, then logits).  H and W must be
 * multiples of 2^(levels-1), at most 16384, and every level's feature map
 * (H>>l) x (W>>l) x channels[l] must stay below 2^29 values (the kernels
 * use 32-bit byte offsets); otherwise WSKP_E_SHAPE. */
wskp_status_t wskp_denoise(wskp_handle_t h, void *stream, int H, int W, const float *radiance,
                           const float *albedo, const float *normal, const float *depth,
                           float *out, void *ws, size_t ws_bytes);

/* Size of the device-resident scratch that wskp_denoise_static uses (each
 * device holds one, until the process ends). */
#define WSKP_STATIC_SCRATCH_BYTES (256ull << 20)

/* wskp_denoise without a workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, serving loops that
 * forbid allocation): the intermediate maps and the head record live in a
 * scratch array of WSKP_STATIC_SCRATCH_BYTES in device memory that the
 * library holds for each device (its address is looked up by wskp_create).
 * Same arguments, result and layout rules as wskp_denoise; it allocates
 * nothing.  A frame whose workspace (wskp_workspace_size(h, 1, &H, &W))
 * exceeds the scratch returns WSKP_E_BUDGET (e.g. 1280x720 fits with bf16
 * or FP8 convolutions, not with FP32).  Every call on one device shares
 * that device's scratch: calls that overlap in time on one device (other
 * streams, other handles, other host threads) race and give undefined
 * results; the caller must order them (e.g. one stream). */
wskp_status_t wskp_denoise_static(wskp_handle_t h, void *stream, int H, int W,
                                  const float *radiance, const float *albedo, const float *normal,
                                  const float *depth, float *out);

/* WSKP_STATIC_SCRATCH_BYTES, as built into the library. */
size_t wskp_static_scratch_bytes(void);

#define WSKP_BATCH_REVERSE_TILES 1u /* walk tiles in reverse order (result must not change) */
#define WSKP_BATCH_GRAPH 2u         /* replay one HIP graph per stream and capacity bucket */

/* Denoises n independent frames of possibly different sizes with one
 * launch per network layer.  `frames` is a HOST array of n descriptors
 * (read during the call only).  Each frame's result is the same as that of
 * wskp_denoise on it alone: no arithmetic crosses frames.  Workspace from
 * wskp_workspace_size(h, n, H, W).
 * WSKP_BATCH_GRAPH: the launches run as one HIP graph per (stream, flags,
 * capacity bucket).  A bucket is the batch's workgroup count of every
 * launch rounded up to a power of two; the first batch of a bucket captures
 * the graph (and allocates its device frame table, header plus 1024
 * descriptors, owned by the handle until wskp_destroy); every batch then
 * uploads its frame count and descriptors to that table on `stream` and
 * replays the graph, whose workgroups beyond the batch's tiles exit at once.
 * Results are identical to the direct launches.  Up to 256 graphs per
 * handle; beyond that, batches of new buckets are launched directly.  Calls
 * on the same stream are ordered; the caller must not capture this call
 * into a graph of its own. */
wskp_status_t wskp_denoise_batch(wskp_handle_t h, void *stream, int n, const wskp_frame_t *frames,
                                 uint32_t flags, void *ws, size_t ws_bytes);

/* Decode + fusion + remodulation alone (Eq. 3, 4, 5), for N frames of
 * H x W.  head [N,H,W,2M]: channels 0..M-1 are the positive weight maps
 * W_i (already activated), M..2M-1 the fusion logits.  c [N,H,W,3] is the
 * irradiance to filter, mod [N,H,W,3] the remodulation factor (NULL = 1).
 * out [N,H,W,3] = mod * sum_i softmax(logits)_i * (box_i(W_i c) /
 * max(box_i(W_i), eps_norm)), with windows truncated at the border.  Any
 * H, W >= 1. */
wskp_status_t wskp_decode(wskp_handle_t h, void *stream, int N, int H, int W, const float *head,
                          const float *c, const float *mod, float *out);

/* Vector-Jacobian product of wskp_decode (the gradient of Eq. 3-5, through
 * which the paper trains its network, Sec. 5.2): given grad_out = dL/dout
 * [N,H,W,3], writes grad_head = dL/dhead [N,H,W,2M] (weights, then
 * logits) and grad_c = dL/dc [N,H,W,3] (mod is treated as a constant).
 * Both outputs are overwritten, not accumulated.  ws is a device scratch
 * buffer of ws_bytes >= wskp_backward_workspace_size(h, N, H, W). */
wskp_status_t wskp_backward(wskp_handle_t h, void *stream, int N, int H, int W, const float *head,
                            const float *c, const float *mod, const float *grad_out,
                            float *grad_head, float *grad_c, void *ws, size_t ws_bytes);

/* Bytes of device scratch wskp_backward needs for N frames of H x W
 * (20 * M bytes per pixel: per-centre adjoint terms of every kernel size). */
wskp_status_t wskp_backward_workspace_size(wskp_handle_t h, int N, int H, int W, size_t *bytes);

/* Training (Eq. 1: the network's weights minimise a loss between its
 * reconstruction and the reference; Eq. 6: SMAPE; Sec. 5.3: Adam).  For
 * handles with WSKP_PREC_FP32 and WSKP_ACT_SOFTPLUS (others:
 * WSKP_E_UNSUPPORTED).  The handle keeps the weight blob (the layout of
 * wskp_num_weights) on the device as the trained parameters.
 * wskp_train_workspace_size: workspace bytes of wskp_train_grads for n
 *   frames of sizes H[i] x W[i].  Frames of one size run the backward pass
 *   together (every kernel once per layer over all n), so the workspace
 *   grows with n; frames of mixed sizes run it one at a time in scratch for
 *   the largest.
 * wskp_train_grads: forward pass of the n frames (each frame's `out`
 *   receives its reconstruction), loss = SMAPE(out, target) over all
 *   frames' values (Eq. 6 with eps_smape; N = all pixels of the batch) into
 *   the device scalar *loss, and its gradient with respect to every weight
 *   and bias into grad (device, wskp_num_weights floats, overwritten).
 *   targets: HOST array of n device pointers to [H_i,W_i,3] references.
 *   Gradients are accumulated over frames in a fixed order (run-to-run
 *   identical).  Errors: WSKP_E_BUDGET when ws_bytes is below
 *   wskp_train_workspace_size; WSKP_E_LAUNCH when a frame is too wide for
 *   the 32-bit buffer windows of the weight-gradient kernel (about 10^6
 *   pixels per row at 200 channels).
 * wskp_adam: one Adam step (step >= 1) on the handle's weights with the
 *   gradient grad and the moment buffers m, v (device, wskp_num_weights
 *   floats each, zero before step 1, updated in place); afterwards every
 *   denoising call uses the new weights.
 * wskp_get_weights: copies the handle's current weight blob to the device
 *   buffer dst (wskp_num_weights floats) on `stream`. */
wskp_status_t wskp_train_workspace_size(wskp_handle_t h, int n, const int *H, const int *W, size_t *bytes);
wskp_status_t wskp_train_grads(wskp_handle_t h, void *stream, int n, const wskp_frame_t *frames,
                               const float *const *targets, float eps_smape, float *grad, float *loss,
                               void *ws, size_t ws_bytes);
wskp_status_t wskp_adam(wskp_handle_t h, void *stream, const float *grad, float *m, float *v, int step,
                        float lr, float beta1, float beta2, float eps);
wskp_status_t wskp_get_weights(wskp_handle_t h, void *stream, float *dst);

/* Multi-resolution reconstruction (Sec. 5.2, the paper's network for
 * high-spp input): the irradiance is filtered at L resolutions, level l
 * with its own head record (wskp_decode on the 2x2-pooled irradiance, mod
 * NULL), and adjacent levels are combined from the coarsest by Eq. 7:
 *   o_p = fine_p - alpha_p [U D fine]_p + alpha_p [U coarse]_p
 * with D the 2x2 mean and U nearest-neighbour upsampling.
 * wskp_pool2: out [H/2,W/2,3] = 2x2 means of in [H,W,3].
 * wskp_mr_blend: fine [H,W,3], coarse [H/2,W/2,3], alpha [H,W] -> out
 *   [H,W,3] by Eq. 7, times mod [H,W,3] if mod is not NULL (the
 *   remodulation, for the finest level).  out must not alias fine.
 * H and W even; device pointers. */
wskp_status_t wskp_pool2(wskp_handle_t h, void *stream, int H, int W, const float *in, float *out);
wskp_status_t wskp_mr_blend(wskp_handle_t h, void *stream, int H, int W, const float *fine,
                            const float *coarse, const float *alpha, const float *mod, float *out);

/* The whole multi-resolution reconstruction in one call: L levels (1..6),
 * H and W multiples of 2^(L-1).  heads: host array of L device pointers,
 * heads[l] the activated head record of level l, [H>>l, W>>l, 2M]
 * interleaved (as wskp_decode takes it); c [H,W,3] the irradiance; alphas:
 * host array of L-1 device pointers, alphas[l] [H>>l, W>>l] the Eq. 7 blend
 * weight of level l; mod [H,W,3] or NULL; out [H,W,3].  Pools c L-1 times,
 * filters every level, blends from the coarsest and remodulates the finest
 * result: the same launches, in the same order, as the composition of
 * wskp_pool2, wskp_decode and wskp_mr_blend.  ws: device workspace of at
 * least wskp_mr_workspace_size bytes (the pooled irradiance of levels
 * 1..L-1, every level's filtered image, the intermediate blends). */
wskp_status_t wskp_mr_workspace_size(wskp_handle_t h, int L, int H, int W, size_t *bytes);
wskp_status_t wskp_mr_reconstruct(wskp_handle_t h, void *stream, int L, int H, int W,
                                  const float *const *heads, const float *c, const float *const *alphas,
                                  const float *mod, float *out, void *ws, size_t ws_bytes);

/* Temporal accumulation before denoising (Sec. 4.1, last paragraph): the
 * previous frame's accumulated radiance is reprojected to this frame with
 * the motion vectors and, where the geometry agrees, blended with this
 * frame's noisy radiance; elsewhere the noisy radiance is kept.  Its output
 * is the radiance input of wskp_denoise for this frame and the history of
 * the next one.
 *   radiance, normal, wpos [H,W,3]   this frame (noisy radiance, shading
 *                                    normal, world position)
 *   motion [H,W,2]                   per pixel, the offset (x, y) in pixels
 *                                    to where its surface point was in the
 *                                    previous frame
 *   prev_radiance [H,W,3], prev_length [H,W]   the previous call's outputs;
 *   prev_normal, prev_wpos [H,W,3]   the previous frame's geometry
 *   out_radiance [H,W,3], out_length [H,W]     (must not alias the inputs)
 * With prev_radiance == NULL (first frame, or a cut) out = radiance and
 * length 1, and only radiance is read.  Otherwise, per pixel p with
 * q = p + motion(p): of the four pixels around q (bilinear weights), those
 * inside the image whose world position lies within pos_tol of p's and
 * whose normal has a dot product >= normal_tol with p's count; S is their
 * weight.  If S > 0, with h and L the S-normalised weighted means of their
 * accumulated radiance and length, alpha = max(1/(L+1), alpha_min):
 * out = (1 - alpha) h + alpha radiance, length L + 1; if S = 0: out =
 * radiance, length 1.  (The paper gives no blend factor or tolerances;
 * alpha_min = 0.2, pos_tol = 0.02 world units, normal_tol = 0.9 are the
 * values the tests and benchmark use.)  The tap tests are evaluated in
 * double precision.  All pointers are device pointers; H x W <= 2^28. */
wskp_status_t wskp_temporal(wskp_handle_t h, void *stream, int H, int W, const float *radiance,
                            const float *normal, const float *wpos, const float *motion,
                            const float *prev_radiance, const float *prev_length,
                            const float *prev_normal, const float *prev_wpos, float alpha_min,
                            float pos_tol, float normal_tol, float *out_radiance, float *out_length);

/* Explicit kernel-map reconstruction, the baseline of the memory and time
 * comparison in Sec. 5.3 (a kernel-prediction network without weight
 * sharing predicts every pixel's full k_i x k_i kernel).  Not part of the
 * denoising path; for benchmarks and checks.
 * wskp_kp_map_bytes: size of the maps for one H x W frame:
 *   4 * H * W * sum_i k_i^2 bytes (1280 x 720 with k = 3..13: 1.67 GB).
 * wskp_kp_expand: fills the maps from a head record [1,H,W,2M] in the
 *   layout of wskp_decode: the weight of neighbour q in the kernel of
 *   centre p is W_i(q), 0 outside the image; planar per size and tap,
 *   maps[i][t][H][W] with t = (dy + r_i) k_i + (dx + r_i).
 * wskp_kp_decode: Eq. 4-5 and the remodulation from explicit maps: for each
 *   centre and size, the map-weighted sum of c over the window divided by
 *   max(sum of the weights, eps_norm), softmax-blended with the head's
 *   logits, times mod (NULL = 1).  With maps from wskp_kp_expand the result
 *   equals wskp_decode's up to rounding.  All pointers are device pointers,
 *   H x W at most 2^26 pixels. */
wskp_status_t wskp_kp_map_bytes(wskp_handle_t h, int H, int W, size_t *bytes);
wskp_status_t wskp_kp_expand(wskp_handle_t h, void *stream, int H, int W, const float *head, float *maps,
                             size_t map_bytes);
wskp_status_t wskp_kp_decode(wskp_handle_t h, void *stream, int H, int W, const float *maps,
                             size_t map_bytes, const float *head, const float *c, const float *mod,
                             float *out);

/* Location of an intermediate tensor of frame `frame` inside the workspace
 * of the last-planned batch layout for frames of sizes H[i] x W[i]: which =
 * 0..L-1 for encoder output e_l, 100 + l for decoder output u_l (shape
 * th x tw x tc = H_l x W_l x C_l), 200 for the head record (planar: th x
 * tw x tc = 2M x H x W), and (bf16 handles whose encoders pass on 2x2
 * means) 300 + l for the pooled copy of e_l, l < L-1.  Returns byte offset,
 * shape and element size (4 = fp32, 2 = bf16).  For debugging and
 * layer-by-layer checks. */
wskp_status_t wskp_workspace_tensor(wskp_handle_t h, int n, const int *H, const int *W, int frame,
                                    int which, size_t *offset, int *th, int *tw, int *tc,
                                    int *elem_bytes);

/* Launch timing, for benchmarks.  wskp_timing_enable(h, k) makes the next
 * k calls of wskp_denoise / wskp_denoise_batch record a HIP event on the
 * call's stream before the first launch and after each launch (k = 0 turns
 * it off and frees the events).  wskp_timing_read waits for those events and
 * returns in ms_sum[i] the elapsed milliseconds of launch i summed over the
 * recorded calls, the number of launches per call and the number of calls.
 * Launch i is named by wskp_launch_name(h, i): "enc0".."enc5",
 * "dec0".."dec5", "head", "decode". */
wskp_status_t wskp_timing_enable(wskp_handle_t h, int max_calls);
wskp_status_t wskp_timing_read(wskp_handle_t h, int max, float *ms_sum, int *n_launches,
                               int *n_calls);
const char *wskp_launch_name(wskp_handle_t h, int i);

/* Round-to-nearest-even conversion of n floats to OCP e4m3 bytes with
 * saturation at +-448 (the encoding the FP8 form uses for weights). */
void wskp_fp8_e4m3_encode(const float *x, uint8_t *out, size_t n);

/* Static text for a status code. */
const char *wskp_status_string(wskp_status_t s);

/* Thread-local detail of the last failing call on this thread ("" if none). */
const char *wskp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WSKP_H */
