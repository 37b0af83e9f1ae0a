// C ABI of libwskp: argument validation, weight packing, workspace layout
// and the launch sequence of one denoising pass.  Every arithmetic step of
// the path runs in the HIP kernels (conv3x3.hip, decode.hip); this file
// only plans and launches.
#include "wskp.h"
#include "wskp_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace wskp;

namespace {

thread_local std::string g_last_error;

wskp_status_t fail(wskp_status_t s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

wskp_status_t hip_fail(hipError_t e, const char *what, wskp_status_t s = WSKP_E_DEVICE)
{
    return fail(s, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct LayerPlan {
    ConvLayer L;
    int mode;
    int epi;
    int Cin;
    size_t w_off, b_off;  // byte offsets into the device weight buffer
    size_t q_off;         // fp8: per-channel dequantisation factors (0 = none)
};

// Host round-to-nearest-even to bf16 (the usual bit-level method).
uint16_t host_bf16(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Host round-to-nearest-even to OCP e4m3 (1 sign, 4 exponent bits with bias
// 7, 3 mantissa bits; largest finite 448, smallest subnormal 2^-9), with
// saturation at +-448.  Works on the exact binary value of x.
uint8_t host_e4m3(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    const uint8_t sign = (uint8_t)((u >> 24) & 0x80);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7f;            // NaN
    float a = std::fabs(x);
    if (a >= 448.f) return sign | 0x7e;                           // saturate
    int e;
    const float m = std::frexp(a, &e);                            // a = m * 2^e, m in [0.5, 1)
    if (a == 0.f) return sign;
    // exponent of the leading bit: E = e - 1; normal range E >= -6
    int E = e - 1;
    double q;      // value in units of the last mantissa bit
    int ulp_exp;
    if (E < -6) { ulp_exp = -9; }                                 // subnormal spacing 2^-9
    else { ulp_exp = E - 3; }
    q = std::ldexp((double)a, -ulp_exp);                          // exact in double
    double fl = std::floor(q);
    double rem = q - fl;
    uint32_t n = (uint32_t)fl;
    if (rem > 0.5 || (rem == 0.5 && (n & 1u))) ++n;
    (void)m;
    // n counts ulps of 2^ulp_exp: encode
    if (ulp_exp == -9) {
        // subnormal (n <= 8; n == 8 is the smallest normal 2^-6, encoding 0x08)
        return sign | (uint8_t)n;
    }
    // normal: n in [8, 16]; 16 means the next binade
    int be = E + 7;
    if (n >= 16) { n >>= 1; ++be; }
    if (be > 15 || (be == 15 && (n & 7u) == 7u)) return sign | 0x7e;
    return sign | (uint8_t)(be << 3) | (uint8_t)(n & 7u);
}

}  // namespace

extern "C" void wskp_fp8_e4m3_encode(const float *x, uint8_t *out, size_t n)
{
    for (size_t i = 0; i < n; ++i) out[i] = host_e4m3(x[i]);
}

struct wskp_ctx {
    wskp_config_t cfg;
    int device = 0;
    int prec = 0;
    int act_bytes = 4;
    bool pooled = false;   // encoder epilogues write 2x2 means p_l; enc_{l+1} reads them plainly
    std::vector<LayerPlan> layers;
    void *dweights = nullptr;
    float *dmaster = nullptr;     // fp32 handles: the weight blob (OIHW + bias, blob order), for training
    std::vector<size_t> blob_off; // offset of each conv's weights in the blob
    DecodeCfg dc{};
    // pinned host staging for batch frame tables: per slot a header (the
    // frame count) and up to kMaxBatch descriptors
    std::mutex mu;
    char *ring = nullptr;
    std::vector<hipEvent_t> ring_ev;
    int ring_next = 0;
    // graph replay of batches (WSKP_BATCH_GRAPH): one executable graph per
    // (stream, capacity bucket), each reading its own device frame table
    struct BatchGraph {
        hipStream_t s;
        bool reverse;
        std::vector<int> caps;   // workgroups of each launch
        hipGraphExec_t exec;
        char *tab;               // device: header + descriptors
    };
    std::vector<BatchGraph> graphs;
    hipStream_t cap_stream = nullptr;
    // launch timing (diagnostics): events recorded around every launch
    std::vector<hipEvent_t> tev;
    int t_max_calls = 0, t_calls = 0;
};

// ---------------------------------------------------------------------------
// Device-resident scratch of wskp_denoise_static: the workspace of one frame
// for callers that cannot allocate.  Each device the library runs on holds
// its own copy until the process ends.  Host code never passes the array's
// name to a kernel or a copy (on the host it is only a stand-in): it uses
// the device address that hipGetSymbolAddress returns, looked up once per
// device in wskp_create with that device current.
static constexpr size_t kStaticScratchBytes = WSKP_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static constexpr int kRingSlots = 8;
static constexpr int kMaxBatch = 1024;
static constexpr size_t kTableHeader = 256;   // frame count, tile count of each launch; padded
static constexpr size_t kSlotBytes = kTableHeader + sizeof(FrameDesc) * kMaxBatch;
static constexpr size_t kMaxGraphs = 256;
static_assert(kTableHeader >= sizeof(int) * (2 + 2 * WSKP_MAX_LEVELS), "header holds n and every launch's tiles");

// ---------------------------------------------------------------------------
static wskp_status_t check_config(const wskp_config_t *c)
{
    if (!c) return fail(WSKP_E_INVALID_ARG, "config is NULL");
    if (c->struct_size != sizeof(wskp_config_t))
        return fail(WSKP_E_INVALID_ARG, "config.struct_size != sizeof(wskp_config_t)");
    if (c->levels < 1 || c->levels > WSKP_MAX_LEVELS)
        return fail(WSKP_E_INVALID_ARG, "levels must be in 1..6");
    for (int l = 0; l < c->levels; ++l)
        if (c->channels[l] < 16 || c->channels[l] > 256 || c->channels[l] % 16)
            return fail(WSKP_E_INVALID_ARG, "channels[l] must be a multiple of 16 in 16..256");
    if (c->num_kernels < 1 || c->num_kernels > WSKP_MAX_KERNELS)
        return fail(WSKP_E_INVALID_ARG, "num_kernels must be in 1..8");
    for (int i = 0; i < c->num_kernels; ++i) {
        const int k = c->kernel_sizes[i];
        if (k < 1 || k > WSKP_MAX_KERNEL_SIZE || k % 2 == 0)
            return fail(WSKP_E_INVALID_ARG, "kernel sizes must be odd, 1..15");
    }
    if (c->precision < WSKP_PREC_FP32 || c->precision > WSKP_PREC_FP8_E4M3)
        return fail(WSKP_E_INVALID_ARG, "unknown precision");
    if (c->weight_act != WSKP_ACT_SOFTPLUS && c->weight_act != WSKP_ACT_EXP)
        return fail(WSKP_E_INVALID_ARG, "unknown weight activation");
    if (!(c->eps_norm > 0.f) || !(c->eps_albedo >= 0.f) || !(c->gamma > 0.f) ||
        !(c->depth_far > c->depth_near))
        return fail(WSKP_E_INVALID_ARG, "eps_norm > 0, eps_albedo >= 0, gamma > 0, far > near");
    if (c->conv_size != 3 && c->conv_size != 5)
        return fail(WSKP_E_INVALID_ARG, "conv_size must be 3 or 5");
    return WSKP_OK;
}

// (Cin, Cout) of each conv in blob order.
static void conv_dims(const wskp_config_t *c, std::vector<std::pair<int, int>> &d)
{
    const int L = c->levels;
    d.clear();
    d.push_back({10, c->channels[0]});
    for (int l = 1; l < L; ++l) d.push_back({c->channels[l - 1], c->channels[l]});
    for (int l = L - 2; l >= 0; --l) d.push_back({c->channels[l + 1] + c->channels[l], c->channels[l]});
    d.push_back({c->channels[0], 2 * c->num_kernels});
}

extern "C" size_t wskp_num_weights(const wskp_config_t *cfg)
{
    if (check_config(cfg) != WSKP_OK) return 0;
    std::vector<std::pair<int, int>> d;
    conv_dims(cfg, d);
    size_t n = 0;
    const size_t k2 = (size_t)cfg->conv_size * cfg->conv_size;
    for (auto &p : d) n += (size_t)p.second * p.first * k2 + p.second;
    return n;
}

// Packs OIHW fp32 weights into the order the kernels read (see conv3x3.hip).
// fp8: per output channel, w is divided by s_w[co] = max|w_co| / 448 before
// rounding; dq[co] receives s_in * s_w[co], the factor that turns the
// fp8 accumulator back into the layer's pre-bias output.
static void pack_layer(int prec, const LayerPlan &lp, const float *w, std::vector<char> &out,
                       float s_in = 1.f, std::vector<float> *dq = nullptr)
{
    const ConvLayer &L = lp.L;
    const int CK = L.CK, nch = L.Cin_pad / CK, Cin = lp.Cin, Cout = L.Cout;
    const int T = L.ks * L.ks;   // taps
    auto W = [&](int co, int ci, int tap) -> float {
        if (co >= Cout || ci >= Cin) return 0.f;
        return w[((size_t)co * Cin + ci) * T + tap];
    };
    if (prec == WSKP_PREC_FP8_E4M3) {
        // [chunk][Cout_pad][NK*128] bytes, K = tap*CK + c, zero padded
        const int NR = T * CK / 32, NK = (NR + 3) / 4, KR = NK * 128;
        std::vector<float> sw(L.Cout_pad, 1.f);
        for (int co = 0; co < Cout; ++co) {
            float mx = 0.f;
            for (int ci = 0; ci < Cin; ++ci)
                for (int t = 0; t < T; ++t) mx = std::max(mx, std::fabs(W(co, ci, t)));
            sw[co] = mx > 0.f ? mx / 448.f : 1.f;
        }
        out.assign((size_t)nch * L.Cout_pad * KR, 0);
        uint8_t *o = reinterpret_cast<uint8_t *>(out.data());
        for (int cc = 0; cc < nch; ++cc)
            for (int co = 0; co < L.Cout_pad; ++co)
                for (int k = 0; k < T * CK; ++k) {
                    const int tap = k / CK, c = k % CK;
                    o[((size_t)cc * L.Cout_pad + co) * KR + k] = host_e4m3(W(co, cc * CK + c, tap) / sw[co]);
                }
        if (dq) {
            dq->assign(L.Cout_pad, 0.f);
            for (int co = 0; co < Cout; ++co) (*dq)[co] = s_in * sw[co];
        }
    } else if (prec == WSKP_PREC_FP32) {
        // [chunk][tap][c][Cout_pad]
        out.assign((size_t)nch * T * CK * L.Cout_pad * 4, 0);
        float *o = reinterpret_cast<float *>(out.data());
        for (int cc = 0; cc < nch; ++cc)
            for (int tap = 0; tap < T; ++tap)
                for (int c = 0; c < CK; ++c)
                    for (int co = 0; co < L.Cout_pad; ++co)
                        o[(((size_t)cc * T + tap) * CK + c) * L.Cout_pad + co] = W(co, cc * CK + c, tap);
    } else {
        // [chunk][Cout_pad][KR], K = tap*CK + c, zero padded; the kernels
        // copy a group's rows as one contiguous block.  Register-staged
        // kernels: KR = NK*32 + 8 (the 8 extra elements make the row stride
        // in LDS bank-friendly).  Direct-to-LDS kernel: KR = NK*32, and in
        // row co the 8-element groups are stored at position g ^ (2 * ((co
        // >> 2) & 1)), the bank-conflict-free order that kernel reads.
        const bool direct = conv_uses_direct(prec, lp.mode, CK, L.ks);
        const int NK = (T * CK + 31) / 32, KR = direct ? NK * 32 : NK * 32 + 8;
        out.assign((size_t)nch * L.Cout_pad * KR * 2, 0);
        uint16_t *o = reinterpret_cast<uint16_t *>(out.data());
        for (int cc = 0; cc < nch; ++cc)
            for (int co = 0; co < L.Cout_pad; ++co)
                for (int k = 0; k < T * CK; ++k) {
                    const int tap = k / CK, c = k % CK;
                    const int pos = direct ? ((((k >> 3) ^ (((co >> 2) & 1) << 1))) << 3) | (k & 7) : k;
                    o[((size_t)cc * L.Cout_pad + co) * KR + pos] = host_bf16(W(co, cc * CK + c, tap));
                }
    }
}

// RepVGG re-parameterisation (Sec. 4.1, prediction phase): the 1x1, 3x3 and
// 5x5 branch kernels are added into the centre of one 5x5 kernel, the
// identity becomes a unit centre tap of (c, c), and the biases add up.  The
// sum of the branch outputs is the output of that conv because convolution
// is linear in its kernel and each branch's zero padding is the 5x5 kernel's
// zero border around it.
extern "C" wskp_status_t wskp_repvgg_merge(int cin, int cout, const float *w1, const float *b1,
                                           const float *w3, const float *b3, const float *w5,
                                           const float *b5, int identity, float *w_out, float *b_out)
{
    if (cin < 1 || cout < 1) return fail(WSKP_E_INVALID_ARG, "cin and cout must be >= 1");
    if (!w_out || !b_out) return fail(WSKP_E_INVALID_ARG, "output pointer is NULL");
    if (identity && cin != cout) return fail(WSKP_E_INVALID_ARG, "the identity branch needs cin == cout");
    if (!w1 != !b1 || !w3 != !b3 || !w5 != !b5)
        return fail(WSKP_E_INVALID_ARG, "a branch needs both its weights and its bias (or neither)");
    const size_t n = (size_t)cout * cin * 25;
    std::fill(w_out, w_out + n, 0.f);
    std::fill(b_out, b_out + cout, 0.f);
    const float *ws[3] = {w1, w3, w5}, *bs[3] = {b1, b3, b5};
    const int ksz[3] = {1, 3, 5};
    for (int i = 0; i < 3; ++i) {
        if (!ws[i] || !bs[i]) continue;
        const int k = ksz[i], o = (5 - k) / 2;
        for (int co = 0; co < cout; ++co) {
            for (int ci = 0; ci < cin; ++ci)
                for (int y = 0; y < k; ++y)
                    for (int x = 0; x < k; ++x)
                        w_out[(((size_t)co * cin + ci) * 5 + y + o) * 5 + x + o] +=
                            ws[i][(((size_t)co * cin + ci) * k + y) * k + x];
            b_out[co] += bs[i][co];
        }
    }
    if (identity)
        for (int c = 0; c < cout; ++c) w_out[(((size_t)c * cin + c) * 5 + 2) * 5 + 2] += 1.f;
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_create(const wskp_config_t *cfg, const float *host_weights,
                                     size_t n_weights, const float *host_act_scales, int device,
                                     wskp_handle_t *out)
{
    if (!out) return fail(WSKP_E_INVALID_ARG, "out handle pointer is NULL");
    *out = nullptr;
    wskp_status_t st = check_config(cfg);
    if (st != WSKP_OK) return st;
    if (cfg->precision == WSKP_PREC_FP8_E4M3) {
        if (!host_act_scales)
            return fail(WSKP_E_INVALID_ARG, "FP8 needs one activation scale per conv (host_act_scales)");
        for (int l = 0; l < cfg->levels; ++l)
            if (cfg->channels[l] % 32)
                return fail(WSKP_E_UNSUPPORTED, "FP8 needs every level width to be a multiple of 32");
        if (cfg->conv_size != 3) return fail(WSKP_E_UNSUPPORTED, "FP8 runs 3x3 convs only");
    }
    if (!host_weights) return fail(WSKP_E_INVALID_ARG, "weights pointer is NULL");
    if (n_weights != wskp_num_weights(cfg))
        return fail(WSKP_E_INVALID_ARG, "weight count does not match wskp_num_weights(cfg)");

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(WSKP_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(WSKP_E_DEVICE, "device index out of range");
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess)
        return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(WSKP_E_DEVICE, std::string("device is ") + prop.gcnArchName + ", need gfx950");
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (device >= kMaxDevices) return fail(WSKP_E_DEVICE, "device index beyond the library's table");
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            void *p = nullptr;
            if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess || !p)
                return hip_fail(e, "hipGetSymbolAddress(static scratch)");
            g_scratch_ptr[device] = p;
        }
    }

    wskp_ctx *h = new wskp_ctx();
    h->cfg = *cfg;
    h->device = device;
    h->prec = cfg->precision;
    h->act_bytes = h->prec == WSKP_PREC_FP32 ? 4 : 2;   // bf16 activations for bf16 and fp8

    // ---- layer plan
    const int L = cfg->levels, M = cfg->num_kernels, ks = cfg->conv_size;
    std::vector<std::pair<int, int>> dims;
    conv_dims(cfg, dims);
    auto add = [&](int mode, int level, int s0kind, int s0, int s1, int C0, int C1, int Cin, int Cout,
                   int okind, int oidx, int pool_idx) {
        LayerPlan lp{};
        ConvLayer &c = lp.L;
        c.level = level;
        c.src0_kind = s0kind;
        c.src0_idx = s0;
        c.src1_idx = s1;
        c.C0 = C0;
        c.C1 = C1;
        c.ks = ks;
        c.CK = conv_chunk(h->prec, mode, Cin, C0);
        c.Cin_pad = (Cin + c.CK - 1) / c.CK * c.CK;
        c.Cout = Cout;
        const int nblk = (Cout + 15) / 16;
        c.NB = conv_blocks_per_group(h->prec, mode, c.CK, nblk, level, ks);
        c.groups = nblk / c.NB;
        c.th = conv_tile_rows(h->prec, mode, c.CK, level, pool_idx >= 0, ks);
        c.pool_idx = pool_idx;
        c.Cout_pad = nblk * 16;
        c.out_kind = okind;
        c.out_idx = oidx;
        c.M = M;
        c.inv_gamma = 1.f / cfg->gamma;
        c.dnear = cfg->depth_near;
        c.dinv = 1.f / (cfg->depth_far - cfg->depth_near);
        lp.mode = mode;
        lp.epi = okind == 2 ? (cfg->weight_act == WSKP_ACT_EXP ? EPI_HEAD_EXP : EPI_HEAD_SOFTPLUS)
                            : EPI_RELU;
        lp.Cin = Cin;
        h->layers.push_back(lp);
    };
    const int *ch = cfg->channels;
    // bf16: each encoder epilogue (a workgroup owning whole row pairs) also
    // writes the 2x2 means of its output, and the next encoder reads those
    // with the direct-load kernel (32-channel chunks)
    h->pooled = h->prec == WSKP_PREC_BF16 && L > 1 && conv_tile_rows(h->prec, CONV_PACK, 16, 0, true, ks) >= 8 &&
                conv_tile_rows(h->prec, CONV_PLAIN, 32, 1, true, ks) >= 8;
    for (int l = 0; l + 1 < L && h->pooled; ++l)
        if (ch[l] % 32) h->pooled = false;
    if (h->pooled) {
        add(CONV_PACK, 0, 0, 0, 0, 10, 0, 10, ch[0], 0, 0, 0);
        for (int l = 1; l < L; ++l)
            add(CONV_PLAIN, l, 2, l - 1, 0, ch[l - 1], 0, ch[l - 1], ch[l], 0, l, l + 1 < L ? l : -1);
    } else {
        add(CONV_PACK, 0, 0, 0, 0, 10, 0, 10, ch[0], 0, 0, -1);
        for (int l = 1; l < L; ++l)
            add(CONV_POOL, l, 0, l - 1, 0, ch[l - 1], 0, ch[l - 1], ch[l], 0, l, -1);
    }
    for (int l = L - 2; l >= 0; --l)
        add(CONV_CAT, l, 1, l + 1, l, ch[l + 1], ch[l], ch[l + 1] + ch[l], ch[l], 1, l, -1);
    add(CONV_PLAIN, 0, 1, 0, 0, ch[0], 0, ch[0], 2 * M, 2, 0, -1);

    // ---- pack weights into one device buffer
    std::vector<char> blob;
    size_t src = 0;
    for (size_t i = 0; i < h->layers.size(); ++i) {
        LayerPlan &lp = h->layers[i];
        const int Cin = dims[i].first, Cout = dims[i].second;
        std::vector<char> pk;
        std::vector<float> dq;
        const bool f8 = h->prec == WSKP_PREC_FP8_E4M3;
        if (f8 && !(host_act_scales[i] > 0.f)) {
            delete h;
            return fail(WSKP_E_INVALID_ARG, "FP8 activation scales must be > 0");
        }
        const float s_in = f8 ? host_act_scales[i] : 1.f;
        pack_layer(h->prec, lp, host_weights + src, pk, s_in, f8 ? &dq : nullptr);
        lp.L.in_qscale = 1.f / s_in;
        src += (size_t)Cout * Cin * ks * ks;
        lp.w_off = align_up(blob.size());
        blob.resize(lp.w_off + pk.size());
        std::memcpy(blob.data() + lp.w_off, pk.data(), pk.size());
        lp.q_off = 0;
        if (f8) {
            lp.q_off = align_up(blob.size());
            blob.resize(lp.q_off + dq.size() * 4);
            std::memcpy(blob.data() + lp.q_off, dq.data(), dq.size() * 4);
        }
        lp.b_off = align_up(blob.size());
        blob.resize(lp.b_off + (size_t)Cout * 4);
        std::memcpy(blob.data() + lp.b_off, host_weights + src, (size_t)Cout * 4);
        src += Cout;
    }
    if ((e = hipMalloc(&h->dweights, blob.size())) != hipSuccess) {
        delete h;
        return hip_fail(e, "hipMalloc(weights)", WSKP_E_OOM);
    }
    if ((e = hipMemcpy(h->dweights, blob.data(), blob.size(), hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(h->dweights);
        delete h;
        return hip_fail(e, "hipMemcpy(weights)");
    }
    {
        size_t o = 0;
        for (auto &d : dims) {
            h->blob_off.push_back(o);
            o += (size_t)d.first * d.second * ks * ks + d.second;
        }
    }
    if (h->prec == WSKP_PREC_FP32) {
        const size_t nb = n_weights * sizeof(float);
        if ((e = hipMalloc(reinterpret_cast<void **>(&h->dmaster), nb)) != hipSuccess ||
            (e = hipMemcpy(h->dmaster, host_weights, nb, hipMemcpyHostToDevice)) != hipSuccess) {
            if (h->dmaster) (void)hipFree(h->dmaster);
            (void)hipFree(h->dweights);
            delete h;
            return hip_fail(e, "master weights", WSKP_E_OOM);
        }
    }
    for (auto &lp : h->layers) {
        lp.L.w = static_cast<char *>(h->dweights) + lp.w_off;
        lp.L.bias = reinterpret_cast<const float *>(static_cast<char *>(h->dweights) + lp.b_off);
        lp.L.out_scale = lp.q_off ? reinterpret_cast<const float *>(static_cast<char *>(h->dweights) +
                                                                    lp.q_off)
                                  : nullptr;
    }

    // ---- decode configuration
    h->dc.M = M;
    h->dc.R = 0;
    for (int i = 0; i < M; ++i) {
        h->dc.radius[i] = (cfg->kernel_sizes[i] - 1) / 2;
        if (h->dc.radius[i] > h->dc.R) h->dc.R = h->dc.radius[i];
    }
    h->dc.eps_norm = cfg->eps_norm;
    h->dc.eps_albedo = cfg->eps_albedo;
    // with exp weights the head conv stores the raw pre-activations and the
    // decode exponentiates them with a per-tile shift
    h->dc.exp_weights = cfg->weight_act == WSKP_ACT_EXP ? 1 : 0;
    decode_tile_shape(h->dc);
    *out = h;
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_destroy(wskp_handle_t h)
{
    if (!h) return fail(WSKP_E_INVALID_ARG, "handle is NULL");
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    for (auto ev : h->ring_ev) (void)hipEventDestroy(ev);
    for (auto ev : h->tev) (void)hipEventDestroy(ev);
    for (auto &g : h->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipFree(g.tab);
    }
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->ring) (void)hipHostFree(h->ring);
    if (h->dweights) (void)hipFree(h->dweights);
    if (h->dmaster) (void)hipFree(h->dmaster);
    delete h;
    return WSKP_OK;
}

// ---------------------------------------------------------------------------
// Workspace: [frame table][frame 0][frame 1]...; per frame e_0..e_{L-1},
// u_0..u_{L-2}, (pooled plan) p_0..p_{L-2}, head, each 256-byte aligned.
static size_t frame_bytes(const wskp_ctx *h, int H, int W, size_t *off_e, size_t *off_u,
                          size_t *off_head, size_t *off_p = nullptr)
{
    const int L = h->cfg.levels;
    size_t o = 0;
    for (int l = 0; l < L; ++l) {
        if (off_e) off_e[l] = o;
        o += align_up((size_t)(H >> l) * (W >> l) * h->cfg.channels[l] * h->act_bytes);
    }
    for (int l = 0; l < L - 1; ++l) {
        if (off_u) off_u[l] = o;
        o += align_up((size_t)(H >> l) * (W >> l) * h->cfg.channels[l] * h->act_bytes);
    }
    for (int l = 0; l < L - 1 && h->pooled; ++l) {
        if (off_p) off_p[l] = o;
        o += align_up((size_t)(H >> (l + 1)) * (W >> (l + 1)) * h->cfg.channels[l] * h->act_bytes);
    }
    if (off_head) *off_head = o;
    o += align_up((size_t)H * W * 2 * h->cfg.num_kernels * 4);
    return o;
}

static size_t table_bytes(int n) { return align_up((size_t)n * sizeof(FrameDesc)); }

static wskp_status_t check_frame_size(const wskp_ctx *h, int H, int W)
{
    const int a = 1 << (h->cfg.levels - 1);
    if (H < 1 || W < 1) return fail(WSKP_E_SHAPE, "H and W must be >= 1");
    if (H % a || W % a)
        return fail(WSKP_E_SHAPE, "H and W must be multiples of 2^(levels-1) = " + std::to_string(a));
    if ((long)H * W > (1L << 28) || H > 16384 || W > 16384)
        return fail(WSKP_E_SHAPE, "frame too large (H, W <= 16384)");
    // the conv kernels address activation maps with 32-bit byte offsets
    for (int l = 0; l < h->cfg.levels; ++l) {
        const long bytes = (long)(H >> l) * (W >> l) * h->cfg.channels[l] * 4;
        if (bytes >= (1L << 31) - (1L << 16))
            return fail(WSKP_E_SHAPE, "frame too large: an activation map would exceed 2 GiB");
    }
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_workspace_size(wskp_handle_t h, int n, const int *H, const int *W,
                                             size_t *bytes)
{
    if (!h || !H || !W || !bytes) return fail(WSKP_E_INVALID_ARG, "NULL argument");
    if (n < 1 || n > kMaxBatch) return fail(WSKP_E_INVALID_ARG, "n must be in 1..1024");
    size_t tot = table_bytes(n);
    for (int i = 0; i < n; ++i) {
        wskp_status_t st = check_frame_size(h, H[i], W[i]);
        if (st != WSKP_OK) return st;
        tot += frame_bytes(h, H[i], W[i], nullptr, nullptr, nullptr);
    }
    *bytes = tot;
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_workspace_tensor(wskp_handle_t h, int n, const int *H, const int *W,
                                               int frame, int which, size_t *offset, int *th,
                                               int *tw, int *tc, int *elem_bytes)
{
    if (!h || !H || !W || !offset) return fail(WSKP_E_INVALID_ARG, "NULL argument");
    if (n < 1 || frame < 0 || frame >= n) return fail(WSKP_E_INVALID_ARG, "frame out of range");
    const int L = h->cfg.levels;
    size_t base = table_bytes(n);
    for (int i = 0; i < frame; ++i) base += frame_bytes(h, H[i], W[i], nullptr, nullptr, nullptr);
    size_t oe[kMaxLevels], ou[kMaxLevels], op[kMaxLevels], oh;
    frame_bytes(h, H[frame], W[frame], oe, ou, &oh, op);
    int l, c, eb = h->act_bytes;
    size_t o;
    if (which >= 0 && which < L) {
        l = which; o = oe[l]; c = h->cfg.channels[l];
    } else if (which >= 100 && which < 100 + L) {
        l = which - 100;
        o = (l == L - 1) ? oe[l] : ou[l];
        c = h->cfg.channels[l];
    } else if (which == 200) {
        // planar [2M][H][W]
        *offset = base + oh;
        if (th) *th = 2 * h->cfg.num_kernels;
        if (tw) *tw = H[frame];
        if (tc) *tc = W[frame];
        if (elem_bytes) *elem_bytes = 4;
        return WSKP_OK;
    } else if (h->pooled && which >= 300 && which < 300 + L - 1) {
        o = op[which - 300]; c = h->cfg.channels[which - 300]; l = which - 300 + 1;
    } else {
        return fail(WSKP_E_INVALID_ARG, "unknown tensor id");
    }
    *offset = base + o;
    if (th) *th = H[frame] >> l;
    if (tw) *tw = W[frame] >> l;
    if (tc) *tc = c;
    if (elem_bytes) *elem_bytes = eb;
    return WSKP_OK;
}

static void fill_frame(const wskp_ctx *h, FrameDesc &fd, char *fbase, const wskp_frame_t &f)
{
    size_t oe[kMaxLevels], ou[kMaxLevels], op[kMaxLevels], oh;
    frame_bytes(h, f.H, f.W, oe, ou, &oh, op);
    const int L = h->cfg.levels;
    std::memset(&fd, 0, sizeof(fd));
    fd.H = f.H;
    fd.W = f.W;
    fd.r = f.radiance;
    fd.a = f.albedo;
    fd.n = f.normal;
    fd.d = f.depth;
    fd.out = f.out;
    for (int l = 0; l < L; ++l) fd.e[l] = fbase + oe[l];
    for (int l = 0; l < L - 1; ++l) fd.u[l] = fbase + ou[l];
    fd.u[L - 1] = fd.e[L - 1];
    for (int l = 0; l < L - 1 && h->pooled; ++l) fd.p[l] = fbase + op[l];
    fd.head = reinterpret_cast<float *>(fbase + oh);
}

static wskp_status_t set_device(const wskp_ctx *h)
{
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != h->device) {
        hipError_t e = hipSetDevice(h->device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    }
    return WSKP_OK;
}

static int n_launches(const wskp_ctx *h) { return (int)h->layers.size() + 1; }

// Queues the whole network and the decode for the frames of `fa`.
static wskp_status_t run_frames(wskp_ctx *h, const FrameArg &fa, int n, const int *Hs, const int *Ws,
                                hipStream_t s)
{
    hipEvent_t *ev = nullptr;
    if (h->t_max_calls > 0 && h->t_calls < h->t_max_calls)
        ev = h->tev.data() + (size_t)h->t_calls++ * (n_launches(h) + 1);
    int k = 0;
    if (ev) (void)hipEventRecord(ev[k], s);
    for (const LayerPlan &lp : h->layers) {
        const int blocks = conv_grid(lp.L, n, Hs, Ws);
        hipError_t e = launch_conv(lp.L, lp.mode, lp.epi, h->prec, fa, blocks, s);
        if (e != hipSuccess) return hip_fail(e, "conv launch", WSKP_E_LAUNCH);
        if (ev) (void)hipEventRecord(ev[++k], s);
    }
    hipError_t e = launch_decode_frames(h->dc, fa, decode_grid(h->dc, n, Hs, Ws), s);
    if (e != hipSuccess) return hip_fail(e, "decode launch", WSKP_E_LAUNCH);
    if (ev) (void)hipEventRecord(ev[++k], s);
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_timing_enable(wskp_handle_t h, int max_calls)
{
    if (!h || max_calls < 0) return fail(WSKP_E_INVALID_ARG, "bad argument");
    wskp_status_t st = set_device(h);
    if (st != WSKP_OK) return st;
    (void)hipDeviceSynchronize();
    for (auto ev : h->tev) (void)hipEventDestroy(ev);
    h->tev.clear();
    h->t_calls = 0;
    h->t_max_calls = 0;
    if (max_calls == 0) return WSKP_OK;
    h->tev.resize((size_t)max_calls * (n_launches(h) + 1));
    for (auto &ev : h->tev) {
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    h->t_max_calls = max_calls;
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_timing_read(wskp_handle_t h, int max, float *ms_sum, int *n_launch,
                                          int *n_calls)
{
    if (!h || !ms_sum || !n_launch || !n_calls) return fail(WSKP_E_INVALID_ARG, "NULL argument");
    const int nl = n_launches(h);
    if (max < nl) return fail(WSKP_E_INVALID_ARG, "ms_sum too short");
    for (int i = 0; i < nl; ++i) ms_sum[i] = 0.f;
    for (int c = 0; c < h->t_calls; ++c) {
        hipEvent_t *ev = h->tev.data() + (size_t)c * (nl + 1);
        hipError_t e = hipEventSynchronize(ev[nl]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        for (int i = 0; i < nl; ++i) {
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, ev[i], ev[i + 1])) != hipSuccess)
                return hip_fail(e, "hipEventElapsedTime");
            ms_sum[i] += ms;
        }
    }
    *n_launch = nl;
    *n_calls = h->t_calls;
    return WSKP_OK;
}

extern "C" const char *wskp_launch_name(wskp_handle_t h, int i)
{
    static const char *enc[] = {"enc0", "enc1", "enc2", "enc3", "enc4", "enc5"};
    static const char *dec[] = {"dec0", "dec1", "dec2", "dec3", "dec4", "dec5"};
    if (!h || i < 0 || i > (int)h->layers.size()) return "";
    if (i == (int)h->layers.size()) return "decode";
    const LayerPlan &lp = h->layers[i];
    if (lp.L.out_kind == 2) return "head";
    return lp.L.out_kind == 0 ? enc[lp.L.out_idx] : dec[lp.L.out_idx];
}

extern "C" wskp_status_t wskp_denoise(wskp_handle_t h, void *stream, int H, int W,
                                      const float *radiance, const float *albedo,
                                      const float *normal, const float *depth, float *out,
                                      void *ws, size_t ws_bytes)
{
    if (!h) return fail(WSKP_E_INVALID_ARG, "handle is NULL");
    if (!radiance || !albedo || !normal || !depth || !out || !ws)
        return fail(WSKP_E_INVALID_ARG, "NULL tensor or workspace pointer");
    wskp_status_t st = check_frame_size(h, H, W);
    if (st != WSKP_OK) return st;
    const size_t need = table_bytes(1) + frame_bytes(h, H, W, nullptr, nullptr, nullptr);
    if (ws_bytes < need)
        return fail(WSKP_E_BUDGET, "workspace too small: need " + std::to_string(need) + " bytes");
    if ((st = set_device(h)) != WSKP_OK) return st;
    wskp_frame_t f{H, W, radiance, albedo, normal, depth, out};
    FrameArg fa{};
    fa.table = nullptr;
    fa.n = 1;
    fa.reverse = 0;
    fill_frame(h, fa.one, static_cast<char *>(ws) + table_bytes(1), f);
    return run_frames(h, fa, 1, &H, &W, static_cast<hipStream_t>(stream));
}

extern "C" size_t wskp_static_scratch_bytes(void) { return kStaticScratchBytes; }

extern "C" wskp_status_t wskp_denoise_static(wskp_handle_t h, void *stream, int H, int W,
                                             const float *radiance, const float *albedo,
                                             const float *normal, const float *depth, float *out)
{
    if (!h) return fail(WSKP_E_INVALID_ARG, "handle is NULL");
    if (!radiance || !albedo || !normal || !depth || !out)
        return fail(WSKP_E_INVALID_ARG, "NULL tensor pointer");
    wskp_status_t st = check_frame_size(h, H, W);
    if (st != WSKP_OK) return st;
    const size_t need = table_bytes(1) + frame_bytes(h, H, W, nullptr, nullptr, nullptr);
    if (need > kStaticScratchBytes)
        return fail(WSKP_E_BUDGET, "frame needs " + std::to_string(need) +
                                       " bytes of workspace; the static scratch holds " +
                                       std::to_string(kStaticScratchBytes));
    if ((st = set_device(h)) != WSKP_OK) return st;
    void *ws;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        ws = g_scratch_ptr[h->device];
    }
    if (!ws) return fail(WSKP_E_INTERNAL, "static scratch address not set up");
    // every intermediate map is written in full before it is read: nothing
    // in the scratch needs clearing
    wskp_frame_t f{H, W, radiance, albedo, normal, depth, out};
    FrameArg fa{};
    fa.table = nullptr;
    fa.n = 1;
    fa.reverse = 0;
    fill_frame(h, fa.one, static_cast<char *>(ws) + table_bytes(1), f);
    return run_frames(h, fa, 1, &H, &W, static_cast<hipStream_t>(stream));
}

static int next_pow2(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Captures the network and the decode for capacity c.caps into an
// executable graph whose launches read the frame count and the descriptors
// from the device buffer c.tab (header, then descriptors), on the handle's
// own capture stream.
static wskp_status_t capture_batch_graph(wskp_ctx *h, wskp_ctx::BatchGraph &c)
{
    hipError_t e;
    if (!h->cap_stream && (e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreate");
    if ((e = hipMalloc(reinterpret_cast<void **>(&c.tab), kSlotBytes)) != hipSuccess)
        return hip_fail(e, "hipMalloc(graph frame table)", WSKP_E_OOM);
    FrameArg fa{};
    fa.table = reinterpret_cast<const FrameDesc *>(c.tab + kTableHeader);
    fa.n = 0;
    fa.reverse = c.reverse ? 1 : 0;
    fa.dev_n = reinterpret_cast<const int *>(c.tab);
    hipStream_t cs = h->cap_stream;
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed)) != hipSuccess) {
        (void)hipFree(c.tab);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    hipError_t le = hipSuccess;
    for (size_t i = 0; i < h->layers.size() && le == hipSuccess; ++i) {
        const LayerPlan &lp = h->layers[i];
        fa.launch = (int)i;
        le = launch_conv(lp.L, lp.mode, lp.epi, h->prec, fa, c.caps[i], cs);
    }
    fa.launch = (int)h->layers.size();
    if (le == hipSuccess) le = launch_decode_frames(h->dc, fa, c.caps.back(), cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (le != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipFree(c.tab);
        return hip_fail(le != hipSuccess ? le : e, "graph capture", WSKP_E_LAUNCH);
    }
    e = hipGraphInstantiate(&c.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        (void)hipFree(c.tab);
        return hip_fail(e, "hipGraphInstantiate", WSKP_E_LAUNCH);
    }
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_denoise_batch(wskp_handle_t h, void *stream, int n,
                                            const wskp_frame_t *frames, uint32_t flags, void *ws,
                                            size_t ws_bytes)
{
    if (!h || !frames || !ws) return fail(WSKP_E_INVALID_ARG, "NULL argument");
    if (n < 1 || n > kMaxBatch) return fail(WSKP_E_INVALID_ARG, "n must be in 1..1024");
    std::vector<int> Hs(n), Ws(n);
    for (int i = 0; i < n; ++i) {
        const wskp_frame_t &f = frames[i];
        if (!f.radiance || !f.albedo || !f.normal || !f.depth || !f.out)
            return fail(WSKP_E_INVALID_ARG, "NULL tensor pointer in frame " + std::to_string(i));
        wskp_status_t st = check_frame_size(h, f.H, f.W);
        if (st != WSKP_OK) return st;
        Hs[i] = f.H;
        Ws[i] = f.W;
    }
    size_t need;
    wskp_status_t st = wskp_workspace_size(h, n, Hs.data(), Ws.data(), &need);
    if (st != WSKP_OK) return st;
    if (ws_bytes < need)
        return fail(WSKP_E_BUDGET, "workspace too small: need " + std::to_string(need) + " bytes");
    if ((st = set_device(h)) != WSKP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);

    std::lock_guard<std::mutex> lock(h->mu);
    hipError_t e;
    if (!h->ring) {
        if ((e = hipHostMalloc(reinterpret_cast<void **>(&h->ring), kSlotBytes * kRingSlots,
                               hipHostMallocDefault)) != hipSuccess)
            return hip_fail(e, "hipHostMalloc(frame table ring)", WSKP_E_OOM);
        h->ring_ev.resize(kRingSlots);
        for (auto &ev : h->ring_ev)
            if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
                return hip_fail(e, "hipEventCreate");
        for (auto &ev : h->ring_ev) (void)hipEventRecord(ev, s);
    }
    const bool reverse = (flags & WSKP_BATCH_REVERSE_TILES) != 0;
    // graph replay: the executable graph of this stream and capacity bucket
    // (launch grids rounded up to powers of two), captured on first use
    wskp_ctx::BatchGraph *g = nullptr;
    std::vector<int> tiles;
    if (flags & WSKP_BATCH_GRAPH) {
        std::vector<int> caps;
        for (const LayerPlan &lp : h->layers) tiles.push_back(conv_grid(lp.L, n, Hs.data(), Ws.data()));
        tiles.push_back(decode_grid(h->dc, n, Hs.data(), Ws.data()));
        for (int t : tiles) caps.push_back(next_pow2(t));
        for (auto &c : h->graphs)
            if (c.s == s && c.reverse == reverse && c.caps == caps) g = &c;
        if (!g && h->graphs.size() < kMaxGraphs) {
            wskp_ctx::BatchGraph c{s, reverse, caps, nullptr, nullptr};
            if ((st = capture_batch_graph(h, c)) != WSKP_OK) return st;
            h->graphs.push_back(c);
            g = &h->graphs.back();
        }
        // (a full cache falls back to direct launches)
    }
    const int slot = h->ring_next;
    h->ring_next = (h->ring_next + 1) % kRingSlots;
    // the slot's previous copy must have left host memory before it is rewritten
    if ((e = hipEventSynchronize(h->ring_ev[slot])) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    char *sbase = h->ring + kSlotBytes * slot;
    FrameDesc *tab = reinterpret_cast<FrameDesc *>(sbase + kTableHeader);
    int *hdr = reinterpret_cast<int *>(sbase);
    hdr[0] = n;
    for (size_t i = 0; i < tiles.size(); ++i) hdr[1 + i] = tiles[i];
    char *base = static_cast<char *>(ws) + table_bytes(n);
    for (int i = 0; i < n; ++i) {
        fill_frame(h, tab[i], base, frames[i]);
        base += frame_bytes(h, Hs[i], Ws[i], nullptr, nullptr, nullptr);
    }
    if (g) {
        if ((e = hipMemcpyAsync(g->tab, sbase, kTableHeader + sizeof(FrameDesc) * n, hipMemcpyHostToDevice,
                                s)) != hipSuccess)
            return hip_fail(e, "hipMemcpyAsync(frame table)");
        if ((e = hipEventRecord(h->ring_ev[slot], s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        if ((e = hipGraphLaunch(g->exec, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch", WSKP_E_LAUNCH);
        return WSKP_OK;
    }
    if ((e = hipMemcpyAsync(ws, tab, sizeof(FrameDesc) * n, hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(frame table)");
    if ((e = hipEventRecord(h->ring_ev[slot], s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    FrameArg fa{};
    fa.table = static_cast<const FrameDesc *>(ws);
    fa.n = n;
    fa.reverse = reverse ? 1 : 0;
    fa.dev_n = nullptr;
    return run_frames(h, fa, n, Hs.data(), Ws.data(), s);
}

extern "C" wskp_status_t wskp_decode(wskp_handle_t h, void *stream, int N, int H, int W,
                                     const float *head, const float *c, const float *mod, float *out)
{
    if (!h) return fail(WSKP_E_INVALID_ARG, "handle is NULL");
    if (!head || !c || !out) return fail(WSKP_E_INVALID_ARG, "NULL tensor pointer");
    if (N < 1 || H < 1 || W < 1 || (long)N * H * W > (1L << 30))
        return fail(WSKP_E_SHAPE, "N, H, W must be >= 1");
    // the kernel addresses one frame's head record with 32-bit byte offsets
    if ((long)H * W * 8 * h->cfg.num_kernels >= 0xfffffff0L)
        return fail(WSKP_E_SHAPE, "frame too large: its head record would exceed 4 GiB");
    wskp_status_t st = set_device(h);
    if (st != WSKP_OK) return st;
    hipError_t e = launch_decode_tensors(h->dc, N, H, W, head, c, mod, out,
                                         static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "decode launch", WSKP_E_LAUNCH);
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_backward_workspace_size(wskp_handle_t h, int N, int H, int W,
                                                      size_t *bytes)
{
    if (!h || !bytes) return fail(WSKP_E_INVALID_ARG, "NULL argument");
    if (N < 1 || H < 1 || W < 1) return fail(WSKP_E_SHAPE, "N, H, W must be >= 1");
    *bytes = decode_backward_scratch_bytes(h->dc, N, H, W);
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_backward(wskp_handle_t h, void *stream, int N, int H, int W,
                                       const float *head, const float *c, const float *mod,
                                       const float *grad_out, float *grad_head, float *grad_c,
                                       void *ws, size_t ws_bytes)
{
    if (!h) return fail(WSKP_E_INVALID_ARG, "handle is NULL");
    if (!head || !c || !grad_out || !grad_head || !grad_c || !ws)
        return fail(WSKP_E_INVALID_ARG, "NULL tensor or workspace pointer");
    if (N < 1 || H < 1 || W < 1 || (long)N * H * W > (1L << 30))
        return fail(WSKP_E_SHAPE, "N, H, W must be >= 1");
    const size_t need = decode_backward_scratch_bytes(h->dc, N, H, W);
    if (ws_bytes < need)
        return fail(WSKP_E_BUDGET, "workspace too small: need " + std::to_string(need) + " bytes");
    wskp_status_t st = set_device(h);
    if (st != WSKP_OK) return st;
    hipError_t e = launch_decode_backward(h->dc, N, H, W, head, c, mod, grad_out, grad_head, grad_c,
                                          ws, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "backward launch", WSKP_E_LAUNCH);
    return WSKP_OK;
}

// ---------------------------------------------------------------------------
// Training (fp32 handles with softplus weights): scratch of the backward
// pass for a group of nf frames of one size, each frame's tensors
// contiguous after the previous frame's.
struct TrainScratch {
    float *X, *head, *c, *mod, *gy, *gh, *gc, *dh, *dec, *partial, *in, *gin, *part;
    float *wpk[2 * kMaxLevels];   // packed weights of each input-gradient conv (blob order)
    float *zb;                    // zero bias
    float *ge[kMaxLevels], *gu[kMaxLevels];
    FrameDesc *tab;               // frame table of the group's input-gradient convs
    size_t bytes;
};

// row stride of the head's gradient: its 2M channels padded to the conv
// kernels' 16-channel chunk
static int head_grad_stride(int M) { return (2 * M + 15) / 16 * 16; }

static size_t train_plan(const wskp_ctx *h, int Hm, int Wm, int nf, char *base, TrainScratch *ts)
{
    const int L = h->cfg.levels, M = h->cfg.num_kernels;
    const int *ch = h->cfg.channels;
    const long P = (long)Hm * Wm;
    const size_t F = (size_t)nf;
    size_t o = 0;
    auto take = [&](size_t floats) {
        float *p = base ? reinterpret_cast<float *>(base + o) : nullptr;
        o += align_up(floats * sizeof(float));
        return p;
    };
    size_t mx_in = 10 * (size_t)P, mx_part = tr_wgrad_part_floats(P, 10, ch[0], nf);
    for (int l = 0; l < L; ++l) {
        const long Pl = (long)(Hm >> l) * (Wm >> l);
        if (l > 0) {
            mx_in = std::max(mx_in, (size_t)ch[l - 1] * Pl);
            mx_part = std::max(mx_part, tr_wgrad_part_floats(Pl, ch[l - 1], ch[l], nf));
        }
        if (l + 1 < L) {
            mx_in = std::max(mx_in, (size_t)(ch[l + 1] + ch[l]) * Pl);
            mx_part = std::max(mx_part, tr_wgrad_part_floats(Pl, ch[l + 1] + ch[l], ch[l], nf));
        }
    }
    mx_in = std::max(mx_in, (size_t)ch[0] * P);
    mx_part = std::max(mx_part, tr_wgrad_part_floats(P, ch[0], 2 * M, nf));
    const int ldh = head_grad_stride(M);
    // the input-gradient convs' packed weights (C_out of the forward conv
    // in, C_in out: encoders >= 1, decoders, the head) and the zero bias
    // come first, at offsets that do not depend on the frame size: they are
    // written once per call and serve every frame
    auto r16 = [](int c) { return (size_t)(c + 15) / 16 * 16; };
    TrainScratch t{};
    for (int l = 1; l < L; ++l) t.wpk[l] = take((size_t)ch[l] * 9 * r16(ch[l - 1]));
    for (int l = 0; l + 1 < L; ++l) t.wpk[L + (L - 2 - l)] = take((size_t)ch[l] * 9 * r16(ch[l + 1] + ch[l]));
    t.wpk[2 * L - 1] = take((size_t)ldh * 9 * r16(ch[0]));
    t.zb = take(256);
    t.X = take(F * 10 * P);
    t.head = take(F * 2 * M * P);
    t.c = take(F * 3 * P);
    t.mod = take(F * 3 * P);
    t.gy = take(F * 3 * P);
    t.gh = take(F * 2 * M * P);
    t.gc = take(F * 3 * P);
    t.dh = take(F * ldh * P);
    t.dec = take(decode_backward_scratch_bytes(h->dc, nf, Hm, Wm) / sizeof(float));
    t.partial = take((size_t)std::min(nf, kTrGroup) * tr_smape_blocks(3 * P));
    t.in = take(F * mx_in);
    t.gin = take(F * mx_in);
    t.part = take(mx_part);
    for (int l = 0; l < L; ++l) {
        const size_t n = F * ch[l] * (Hm >> l) * (Wm >> l);
        t.ge[l] = take(n);
        t.gu[l] = l + 1 < L ? take(n) : nullptr;
    }
    t.tab = reinterpret_cast<FrameDesc *>(take((F * sizeof(FrameDesc) + sizeof(float) - 1) / sizeof(float)));
    t.bytes = o;
    if (ts) *ts = t;
    return o;
}

static bool train_same_size(int n, const int *H, const int *W)
{
    for (int i = 1; i < n; ++i)
        if (H[i] != H[0] || W[i] != W[0]) return false;
    return true;
}

static wskp_status_t train_check(const wskp_ctx *h)
{
    if (h->prec != WSKP_PREC_FP32 || !h->dmaster)
        return fail(WSKP_E_UNSUPPORTED, "training needs an fp32 handle");
    if (h->cfg.weight_act != WSKP_ACT_SOFTPLUS) return fail(WSKP_E_UNSUPPORTED, "training needs softplus weights");
    if (h->cfg.conv_size != 3) return fail(WSKP_E_UNSUPPORTED, "training runs 3x3 convs only");
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_train_workspace_size(wskp_handle_t h, int n, const int *H, const int *W,
                                                   size_t *bytes)
{
    if (!h || !H || !W || !bytes) return fail(WSKP_E_INVALID_ARG, "NULL argument");
    wskp_status_t st = train_check(h);
    if (st != WSKP_OK) return st;
    size_t fwd;
    if ((st = wskp_workspace_size(h, n, H, W, &fwd)) != WSKP_OK) return st;
    long best = 0;
    int Hm = 0, Wm = 0;
    for (int i = 0; i < n; ++i)
        if ((long)H[i] * W[i] > best) {
            best = (long)H[i] * W[i];
            Hm = H[i];
            Wm = W[i];
        }
    // frames of one size run their backward pass as one group; frames of
    // mixed sizes one at a time, in scratch for the largest
    size_t mx = 0;
    if (train_same_size(n, H, W))
        mx = train_plan(h, H[0], W[0], n, nullptr, nullptr);
    else
        for (int i = 0; i < n; ++i) mx = std::max(mx, train_plan(h, H[i], W[i], 1, nullptr, nullptr));
    (void)Hm;
    (void)Wm;
    *bytes = align_up(fwd) + mx;
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_train_grads(wskp_handle_t h, void *stream, int n, const wskp_frame_t *frames,
                                          const float *const *targets, float eps_smape, float *grad, float *loss,
                                          void *ws, size_t ws_bytes)
{
    if (!h || !frames || !targets || !grad || !loss || !ws) return fail(WSKP_E_INVALID_ARG, "NULL argument");
    wskp_status_t st = train_check(h);
    if (st != WSKP_OK) return st;
    if (n < 1 || n > kMaxBatch) return fail(WSKP_E_INVALID_ARG, "n must be in 1..1024");
    std::vector<int> Hs(n), Ws(n);
    for (int i = 0; i < n; ++i) {
        if (!targets[i]) return fail(WSKP_E_INVALID_ARG, "NULL target");
        Hs[i] = frames[i].H;
        Ws[i] = frames[i].W;
    }
    size_t need, fwd;
    if ((st = wskp_train_workspace_size(h, n, Hs.data(), Ws.data(), &need)) != WSKP_OK) return st;
    if (ws_bytes < need) return fail(WSKP_E_BUDGET, "workspace too small: need " + std::to_string(need) + " bytes");
    if ((st = wskp_workspace_size(h, n, Hs.data(), Ws.data(), &fwd)) != WSKP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // forward: the batched fp32 path; its workspace keeps every layer's output
    if ((st = wskp_denoise_batch(h, stream, n, frames, 0, ws, fwd)) != WSKP_OK) return st;
    const int L = h->cfg.levels, M = h->cfg.num_kernels, ldh = head_grad_stride(M);
    const int *ch = h->cfg.channels;
    long Ptot = 0;
    for (int i = 0; i < n; ++i) Ptot += (long)Hs[i] * Ws[i];
    const float inv_n = (float)(1.0 / (3.0 * (double)Ptot));
    const size_t nw = wskp_num_weights(&h->cfg);
    const float *mw = h->dmaster;
    const size_t head_k = h->layers.size() - 1;
    auto wofs = [&](size_t k) { return mw + h->blob_off[k]; };
    auto gofs = [&](size_t k) { return grad + h->blob_off[k]; };
    auto bofs = [&](size_t k, int Ci, int Co) { return grad + h->blob_off[k] + (size_t)Ci * Co * 9; };
    hipError_t e = tr_fill((long)nw, 0.f, grad, s);
    // input gradient of conv k (Ci -> Co forward): gin = conv(gm, w flipped,
    // in and out channels swapped), on the matrix cores with the fp32
    // forward kernel on the weights packed for it; gm has ldg >= Co channels
    // (the head's 2M padded with zeros to a multiple of 16, the kernel's
    // channel chunk; Ci, a network width, is one already)
    // gradients of nf frames, frame f's at gm + f sg, into gin + f si
    auto dgrad = [&](const TrainScratch &t, size_t k, int Hl, int Wl, int Ci, int ldg, int nf, const float *gm,
                     long sg, float *gin, long si) -> hipError_t {
        ConvLayer c{};
        c.level = 0;
        c.src0_kind = 0;
        c.src0_idx = 0;
        c.src1_idx = 0;
        c.C0 = ldg;
        c.C1 = 0;
        c.ks = 3;
        c.CK = 16;
        c.Cin_pad = ldg;
        c.Cout = Ci;
        const int nblk = Ci / 16;
        c.NB = nblk % 4 == 0 ? 4 : (nblk % 2 == 0 ? 2 : 1);
        c.groups = nblk / c.NB;
        c.Cout_pad = nblk * 16;
        c.th = conv_tile_rows(WSKP_PREC_FP32, CONV_PLAIN, 16, 0, false, 3);
        c.pool_idx = -1;
        c.out_kind = 0;
        c.out_idx = 1;
        c.M = 0;
        c.in_qscale = 1.f;
        c.w = t.wpk[k];
        c.bias = t.zb;
        FrameArg fa{};
        fa.n = nf;
        if (nf == 1) {
            fa.one.H = Hl;
            fa.one.W = Wl;
            fa.one.e[0] = const_cast<float *>(gm);
            fa.one.e[1] = gin;
        } else {
            hipError_t te = tr_frame_table(t.tab, nf, Hl, Wl, gm, sg, gin, si, s);
            if (te != hipSuccess) return te;
            fa.table = t.tab;
        }
        const std::vector<int> hv(nf, Hl), wv(nf, Wl);
        return launch_conv(c, CONV_PLAIN, EPI_LINEAR, WSKP_PREC_FP32, fa, conv_grid(c, nf, hv.data(), wv.data()), s);
    };
    {
        TrainScratch t;
        train_plan(h, Hs[0], Ws[0], 1, static_cast<char *>(ws) + align_up(fwd), &t);
        if (e == hipSuccess) e = tr_fill(256, 0.f, t.zb, s);
        if (e == hipSuccess) e = tr_pack_dgrad(ch[0], 2 * M, ldh, ch[0], wofs(head_k), t.wpk[head_k], s);
        for (int l = 0; l + 1 < L && e == hipSuccess; ++l) {
            const size_t k = (size_t)L + (L - 2 - l);
            e = tr_pack_dgrad(ch[l + 1] + ch[l], ch[l], ch[l], ch[l + 1] + ch[l], wofs(k), t.wpk[k], s);
        }
        for (int l = 1; l < L && e == hipSuccess; ++l)
            e = tr_pack_dgrad(ch[l - 1], ch[l], ch[l], ch[l - 1], wofs(l), t.wpk[l], s);
    }
    // Frames of one size run the backward pass as one group, every kernel
    // over all of them (frame k's tensors at a constant stride: fs floats
    // apart in the forward workspace, one frame's size apart in the
    // scratch); frames of mixed sizes one at a time.
    const int gsz = train_same_size(n, Hs.data(), Ws.data()) ? n : 1;
    char *fbase = static_cast<char *>(ws) + table_bytes(n);
    for (int f0 = 0; f0 < n && e == hipSuccess; f0 += gsz) {
        const int nf = gsz, H = Hs[f0], W = Ws[f0];
        const long P = (long)H * W;
        const size_t fbytes = frame_bytes(h, H, W, nullptr, nullptr, nullptr);
        const long fs = (long)(fbytes / sizeof(float));
        FrameDesc fd;
        fill_frame(h, fd, fbase, frames[f0]);
        TrainScratch t;
        train_plan(h, H, W, nf, static_cast<char *>(ws) + align_up(fwd), &t);
        const float *e_[kMaxLevels], *u_[kMaxLevels];
        for (int l = 0; l < L; ++l) {
            e_[l] = static_cast<const float *>(fd.e[l]);
            u_[l] = static_cast<const float *>(fd.u[l]);
        }
        // the frames' own buffers, kTrGroup frames per launch of the
        // per-frame kernels
        auto frame_ptrs = [&](int k0, int kn) {
            TrFrames fr{};
            for (int k = 0; k < kn; ++k) {
                const wskp_frame_t &q = frames[f0 + k0 + k];
                fr.r[k] = q.radiance;
                fr.a[k] = q.albedo;
                fr.n[k] = q.normal;
                fr.d[k] = q.depth;
                fr.y[k] = q.out;
                fr.t[k] = targets[f0 + k0 + k];
            }
            return fr;
        };
        // the decode adjoint's inputs, the loss and its gradient
        for (int k0 = 0; k0 < nf && e == hipSuccess; k0 += kTrGroup) {
            const int kn = std::min(kTrGroup, nf - k0);
            const TrFrames fr = frame_ptrs(k0, kn);
            e = tr_head_prep(P, M, kn, fd.head + k0 * fs, fs, fr, h->cfg.eps_albedo, t.head + k0 * 2 * M * P,
                             t.c + k0 * 3 * P, t.mod + k0 * 3 * P, s);
            if (e == hipSuccess)
                e = tr_smape(3 * P, kn, fr, eps_smape, inv_n, t.gy + k0 * 3 * P, t.partial, loss, f0 + k0 > 0, s);
        }
        // decode adjoint over the group, then the weight activation's derivative
        if (e == hipSuccess) e = launch_decode_backward(h->dc, nf, H, W, t.head, t.c, t.mod, t.gy, t.gh, t.gc, t.dec, s);
        if (e == hipSuccess) e = tr_head_act_bwd(P, M, ldh, nf, t.gh, fd.head, fs, t.dh, s);
        // Gradients of the activations, kept as gradients of their
        // pre-activations (the ReLU mask applied by the kernel that writes
        // the last contribution): gu[l] of u_l (l < L - 1; u_{L-1} is e_{L-1},
        // whose gradient is ge[L-1]), ge[l] of e_l.  Every buffer's first
        // contribution overwrites it, so none is cleared.
        auto gu_of = [&](int l) { return l == L - 1 ? t.ge[l] : t.gu[l]; };
        auto act_of = [&](int l) { return l == L - 1 ? e_[L - 1] : u_[l]; };
        auto nel = [&](int l, int C) { return (long)C * (H >> l) * (W >> l); };   // one frame's floats
        // head conv: input u_0, output 2M channels, no ReLU; u_0's gradient
        // has one contribution, masked in place
        if (e == hipSuccess)
            e = tr_wgrad(H, W, 2 * M, ldh, nf, t.dh, ldh * P, u_[0], fs, ch[0], nullptr, 0, 0, t.part, gofs(head_k),
                         bofs(head_k, ch[0], 2 * M), s);
        if (e == hipSuccess) e = dgrad(t, head_k, H, W, ch[0], ldh, nf, t.dh, ldh * P, gu_of(0), nel(0, ch[0]));
        if (e == hipSuccess) e = tr_mask(nel(0, ch[0]), nf, gu_of(0), act_of(0), fs, gu_of(0), s);
        // decoders, finest first: dec_l is conv L + (L - 2 - l) in blob order;
        // the concatenation's adjoint writes u_{l+1}'s gradient (masked, its
        // only contribution) and the first part of e_l's
        for (int l = 0; l + 1 < L && e == hipSuccess; ++l) {
            const size_t k = (size_t)L + (L - 2 - l);
            const int Hl = H >> l, Wl = W >> l, Ci = ch[l + 1] + ch[l], Co = ch[l];
            const float *gm = t.gu[l];
            // the input [upsampled u_{l+1}, e_l] is read from its two sources
            e = tr_wgrad(Hl, Wl, Co, Co, nf, gm, nel(l, Co), e_[l], fs, ch[l], u_[l + 1], fs, ch[l + 1], t.part,
                         gofs(k), bofs(k, Ci, Co), s);
            if (e == hipSuccess) e = dgrad(t, k, Hl, Wl, Ci, Co, nf, gm, nel(l, Co), t.gin, nel(l, Ci));
            if (e == hipSuccess)
                e = tr_cat_bwd(Hl, Wl, ch[l + 1], ch[l], nf, t.gin, act_of(l + 1), fs, gu_of(l + 1), t.ge[l], s);
        }
        // encoders, coarsest first: enc_l is conv l; the 2x2 mean's adjoint
        // adds the last part of e_{l-1}'s gradient and masks it
        for (int l = L - 1; l >= 1 && e == hipSuccess; --l) {
            const int Hl = H >> l, Wl = W >> l, Ci = ch[l - 1], Co = ch[l];
            const float *gm = t.ge[l];
            e = tr_pool(H >> (l - 1), W >> (l - 1), Ci, nf, e_[l - 1], fs, t.in, s);
            if (e == hipSuccess)
                e = tr_wgrad(Hl, Wl, Co, Co, nf, gm, nel(l, Co), t.in, nel(l, Ci), Ci, nullptr, 0, 0, t.part, gofs(l),
                             bofs(l, Ci, Co), s);
            if (e == hipSuccess) e = dgrad(t, (size_t)l, Hl, Wl, Ci, Co, nf, gm, nel(l, Co), t.gin, nel(l, Ci));
            if (e == hipSuccess)
                e = tr_pool_bwd(H >> (l - 1), W >> (l - 1), Ci, nf, t.gin, e_[l - 1], fs, t.ge[l - 1], s);
        }
        // first encoder: the network input written out, weight gradient only
        for (int k0 = 0; k0 < nf && e == hipSuccess; k0 += kTrGroup) {
            const int kn = std::min(kTrGroup, nf - k0);
            e = tr_pack(P, kn, frame_ptrs(k0, kn), 1.f / h->cfg.gamma, h->cfg.depth_near,
                        1.f / (h->cfg.depth_far - h->cfg.depth_near), t.X + k0 * 10 * P, s);
        }
        if (e == hipSuccess)
            e = tr_wgrad(H, W, ch[0], ch[0], nf, t.ge[0], nel(0, ch[0]), t.X, 10 * P, 10, nullptr, 0, 0, t.part,
                         gofs(0), bofs(0, 10, ch[0]), s);
        fbase += nf * fbytes;
    }
    if (e != hipSuccess) return hip_fail(e, "training launch", WSKP_E_LAUNCH);
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_adam(wskp_handle_t h, void *stream, const float *grad, float *m, float *v, int step,
                                   float lr, float beta1, float beta2, float eps)
{
    if (!h || !grad || !m || !v) return fail(WSKP_E_INVALID_ARG, "NULL argument");
    wskp_status_t st = train_check(h);
    if (st != WSKP_OK) return st;
    if (step < 1) return fail(WSKP_E_INVALID_ARG, "step counts from 1");
    if ((st = set_device(h)) != WSKP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t nw = wskp_num_weights(&h->cfg);
    const float c1 = (float)(1.0 - std::pow((double)beta1, step)), c2 = (float)(1.0 - std::pow((double)beta2, step));
    hipError_t e = tr_adam((long)nw, h->dmaster, grad, m, v, lr, beta1, beta2, c1, c2, eps, s);
    // the conv kernels read the weights in their own layout: repack each conv
    std::vector<std::pair<int, int>> d;
    conv_dims(&h->cfg, d);
    for (size_t k = 0; k < h->layers.size() && e == hipSuccess; ++k) {
        const LayerPlan &lp = h->layers[k];
        const int nch = lp.L.Cin_pad / lp.L.CK;
        e = tr_repack(d[k].first, d[k].second, lp.L.CK, nch, lp.L.Cout_pad, h->dmaster + h->blob_off[k],
                      reinterpret_cast<float *>(static_cast<char *>(h->dweights) + lp.w_off),
                      reinterpret_cast<float *>(static_cast<char *>(h->dweights) + lp.b_off), s);
    }
    if (e != hipSuccess) return hip_fail(e, "adam launch", WSKP_E_LAUNCH);
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_get_weights(wskp_handle_t h, void *stream, float *dst)
{
    if (!h || !dst) return fail(WSKP_E_INVALID_ARG, "NULL argument");
    wskp_status_t st = train_check(h);
    if (st != WSKP_OK) return st;
    if ((st = set_device(h)) != WSKP_OK) return st;
    hipError_t e = hipMemcpyAsync(dst, h->dmaster, wskp_num_weights(&h->cfg) * sizeof(float),
                                  hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(weights)");
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_pool2(wskp_handle_t h, void *stream, int H, int W, const float *in, float *out)
{
    if (!h || !in || !out) return fail(WSKP_E_INVALID_ARG, "NULL argument");
    if (H < 2 || W < 2 || H % 2 || W % 2 || (long)H * W > (1L << 28))
        return fail(WSKP_E_SHAPE, "H and W must be even, >= 2");
    wskp_status_t st = set_device(h);
    if (st != WSKP_OK) return st;
    hipError_t e = launch_pool2(H, W, in, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "pool2 launch", WSKP_E_LAUNCH);
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_mr_blend(wskp_handle_t h, void *stream, int H, int W, const float *fine,
                                       const float *coarse, const float *alpha, const float *mod, float *out)
{
    if (!h || !fine || !coarse || !alpha || !out) return fail(WSKP_E_INVALID_ARG, "NULL argument");
    if (H < 2 || W < 2 || H % 2 || W % 2 || (long)H * W > (1L << 28))
        return fail(WSKP_E_SHAPE, "H and W must be even, >= 2");
    wskp_status_t st = set_device(h);
    if (st != WSKP_OK) return st;
    hipError_t e = launch_mr_blend(H, W, fine, coarse, alpha, mod, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mr blend launch", WSKP_E_LAUNCH);
    return WSKP_OK;
}

// Workspace of the multi-resolution reconstruction, float offsets: pooled
// irradiance cs[l] (l >= 1), filtered images f[l], blends o[l] (1 <= l <= L-2;
// level 0's blend is the caller's out).
static wskp_status_t mr_plan(const wskp_ctx *h, int L, int H, int W, size_t *cs, size_t *f, size_t *o,
                             size_t *total)
{
    if (L < 1 || L > WSKP_MAX_LEVELS) return fail(WSKP_E_INVALID_ARG, "L must be in 1..6");
    const int a = 1 << (L - 1);
    if (H < a || W < a || H % a || W % a || (long)H * W > (1L << 28))
        return fail(WSKP_E_SHAPE, "H and W must be multiples of 2^(L-1)");
    if ((long)H * W * 8 * h->cfg.num_kernels >= 0xfffffff0L)
        return fail(WSKP_E_SHAPE, "frame too large: its head record would exceed 4 GiB");
    size_t off = 0;
    auto take = [&](int l) {
        const size_t at = off;
        off += align_up((size_t)(H >> l) * (W >> l) * 3 * sizeof(float)) / sizeof(float);
        return at;
    };
    for (int l = 0; l < L; ++l) {
        cs[l] = l ? take(l) : 0;
        f[l] = take(l);
        o[l] = (l >= 1 && l + 2 <= L) ? take(l) : 0;
    }
    *total = off * sizeof(float);
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_mr_workspace_size(wskp_handle_t h, int L, int H, int W, size_t *bytes)
{
    if (!h || !bytes) return fail(WSKP_E_INVALID_ARG, "NULL argument");
    size_t cs[WSKP_MAX_LEVELS], f[WSKP_MAX_LEVELS], o[WSKP_MAX_LEVELS];
    return mr_plan(h, L, H, W, cs, f, o, bytes);
}

extern "C" wskp_status_t wskp_mr_reconstruct(wskp_handle_t h, void *stream, int L, int H, int W,
                                             const float *const *heads, const float *c,
                                             const float *const *alphas, const float *mod, float *out,
                                             void *ws, size_t ws_bytes)
{
    if (!h || !heads || !c || !out || (L > 1 && (!alphas || !ws)))
        return fail(WSKP_E_INVALID_ARG, "NULL argument");
    size_t cs[WSKP_MAX_LEVELS], f[WSKP_MAX_LEVELS], o[WSKP_MAX_LEVELS], need;
    wskp_status_t st = mr_plan(h, L, H, W, cs, f, o, &need);
    if (st != WSKP_OK) return st;
    for (int l = 0; l < L; ++l)
        if (!heads[l] || (l + 1 < L && !alphas[l])) return fail(WSKP_E_INVALID_ARG, "NULL level pointer");
    if (L > 1 && ws_bytes < need) return fail(WSKP_E_BUDGET, "workspace too small: need " + std::to_string(need) + " bytes");
    if ((st = set_device(h)) != WSKP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (L == 1) {
        e = launch_decode_tensors(h->dc, 1, H, W, heads[0], c, mod, out, s);
        if (e != hipSuccess) return hip_fail(e, "decode launch", WSKP_E_LAUNCH);
        return WSKP_OK;
    }
    float *base = static_cast<float *>(ws);
    // pooled irradiance of every coarser level
    const float *cl = c;
    for (int l = 1; l < L && e == hipSuccess; ++l) {
        e = launch_pool2(H >> (l - 1), W >> (l - 1), cl, base + cs[l], s);
        cl = base + cs[l];
    }
    // every level filtered with its own head (no remodulation)
    for (int l = 0; l < L && e == hipSuccess; ++l)
        e = launch_decode_tensors(h->dc, 1, H >> l, W >> l, heads[l], l ? base + cs[l] : c, nullptr,
                                  base + f[l], s);
    // Eq. 7 from the coarsest; the finest blend is remodulated into out
    const float *coarse = base + f[L - 1];
    for (int l = L - 2; l >= 0 && e == hipSuccess; --l) {
        float *dst = l ? base + o[l] : out;
        e = launch_mr_blend(H >> l, W >> l, base + f[l], coarse, alphas[l], l ? nullptr : mod, dst, s);
        coarse = dst;
    }
    if (e != hipSuccess) return hip_fail(e, "multi-resolution launch", WSKP_E_LAUNCH);
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_temporal(wskp_handle_t h, void *stream, int H, int W, const float *radiance,
                                       const float *normal, const float *wpos, const float *motion,
                                       const float *prev_radiance, const float *prev_length,
                                       const float *prev_normal, const float *prev_wpos, float alpha_min,
                                       float pos_tol, float normal_tol, float *out_radiance,
                                       float *out_length)
{
    if (!h) return fail(WSKP_E_INVALID_ARG, "handle is NULL");
    if (!radiance || !out_radiance || !out_length) return fail(WSKP_E_INVALID_ARG, "NULL tensor pointer");
    const bool first = !prev_radiance;
    if (!first && (!normal || !wpos || !motion || !prev_length || !prev_normal || !prev_wpos))
        return fail(WSKP_E_INVALID_ARG, "with a previous frame every geometry buffer is needed");
    if (H < 1 || W < 1 || (long)H * W > (1L << 28)) return fail(WSKP_E_SHAPE, "H, W out of range");
    if (!(alpha_min > 0.f && alpha_min <= 1.f) || !(pos_tol >= 0.f) || !(normal_tol >= -1.f && normal_tol <= 1.f))
        return fail(WSKP_E_INVALID_ARG, "alpha_min in (0, 1], pos_tol >= 0, normal_tol in [-1, 1]");
    wskp_status_t st = set_device(h);
    if (st != WSKP_OK) return st;
    hipError_t e = launch_temporal(H, W, radiance, normal, wpos, motion, prev_radiance, prev_length, prev_normal,
                                   prev_wpos, alpha_min, pos_tol, normal_tol, out_radiance, out_length,
                                   static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "temporal launch", WSKP_E_LAUNCH);
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_kp_map_bytes(wskp_handle_t h, int H, int W, size_t *bytes)
{
    if (!h || !bytes) return fail(WSKP_E_INVALID_ARG, "NULL argument");
    if (H < 1 || W < 1 || (long)H * W > (1L << 26)) return fail(WSKP_E_SHAPE, "H, W out of range");
    *bytes = kp_map_floats(h->dc, H, W) * sizeof(float);
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_kp_expand(wskp_handle_t h, void *stream, int H, int W, const float *head,
                                        float *maps, size_t map_bytes)
{
    if (!h || !head || !maps) return fail(WSKP_E_INVALID_ARG, "NULL argument");
    if (H < 1 || W < 1 || (long)H * W > (1L << 26)) return fail(WSKP_E_SHAPE, "H, W out of range");
    if (map_bytes < kp_map_floats(h->dc, H, W) * sizeof(float))
        return fail(WSKP_E_BUDGET, "kernel-map buffer too small");
    wskp_status_t st = set_device(h);
    if (st != WSKP_OK) return st;
    hipError_t e = launch_kp_expand(h->dc, H, W, head, maps, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kp expand launch", WSKP_E_LAUNCH);
    return WSKP_OK;
}

extern "C" wskp_status_t wskp_kp_decode(wskp_handle_t h, void *stream, int H, int W, const float *maps,
                                        size_t map_bytes, const float *head, const float *c,
                                        const float *mod, float *out)
{
    if (!h || !maps || !head || !c || !out) return fail(WSKP_E_INVALID_ARG, "NULL argument");
    if (H < 1 || W < 1 || (long)H * W > (1L << 26)) return fail(WSKP_E_SHAPE, "H, W out of range");
    if (map_bytes < kp_map_floats(h->dc, H, W) * sizeof(float))
        return fail(WSKP_E_BUDGET, "kernel-map buffer too small");
    wskp_status_t st = set_device(h);
    if (st != WSKP_OK) return st;
    hipError_t e = launch_kp_decode(h->dc, H, W, maps, head, c, mod, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kp decode launch", WSKP_E_LAUNCH);
    return WSKP_OK;
}

extern "C" const char *wskp_status_string(wskp_status_t s)
{
    switch (s) {
    case WSKP_OK: return "ok";
    case WSKP_E_INVALID_ARG: return "invalid argument";
    case WSKP_E_SHAPE: return "unsupported shape";
    case WSKP_E_UNSUPPORTED: return "unsupported";
    case WSKP_E_DEVICE: return "device error";
    case WSKP_E_OOM: return "out of memory";
    case WSKP_E_BUDGET: return "workspace too small";
    case WSKP_E_LAUNCH: return "kernel launch failed";
    case WSKP_E_INTERNAL: return "internal error";
    }
    return "unknown status";
}

extern "C" const char *wskp_last_error(void) { return g_last_error.c_str(); }
