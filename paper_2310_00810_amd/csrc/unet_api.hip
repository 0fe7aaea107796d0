// C ABI of the warm-start network operators (declared in lbmnn.h).
#include <stdint.h>

#include <mutex>

#include "lbm.h"
#include "lbm_error.hpp"
#include "lbmnn.h"
#include "unet_kernels.hpp"

namespace {

#define NN_TRY(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return lbm_fail(LBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

inline bool mult8(long long v) { return v >= 0 && (v & 7) == 0; }
inline bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

int check_desc(const lbmnn_conv_desc *c, bool need_out) {
    if (!c) return lbm_fail(LBM_EINVAL, "descriptor is NULL");
    if (c->dims != 2 && c->dims != 3) return lbm_fail(LBM_EINVAL, "dims must be 2 or 3");
    if (c->ks != 1 && c->ks != 3) return lbm_fail(LBM_EINVAL, "ks must be 1 or 3");
    if (c->n < 1 || c->d < 1 || c->h < 1 || c->w < 1) return lbm_fail(LBM_EINVAL, "grid must be positive");
    if (c->dims == 2 && c->d != 1) return lbm_fail(LBM_EINVAL, "d must be 1 in 2D");
    if ((long long)c->n * c->d * c->h * c->w >= (1LL << 31))
        return lbm_fail(LBM_EINVAL, "the grid must have fewer than 2^31 pixels");
    if ((c->flags & (LBMNN_S2D | LBMNN_D2S | LBMNN_S2D_G)) &&
        ((long long)c->n * c->d * c->h * c->w << c->dims) >= (1LL << 31))
        return lbm_fail(LBM_EINVAL, "the fine grid of an S2D / D2S mode must have fewer than 2^31 pixels");
    if (((c->dims == 3 ? 4LL * c->h * c->w : 0) + 2LL * c->w + 2) * c->in_cstride >= (1LL << 31))
        return lbm_fail(LBM_EINVAL, "a stencil tap's element offset must fit in 32 bits");
    if (!mult8(c->cin) || c->cin == 0) return lbm_fail(LBM_EINVAL, "cin must be a positive multiple of 8");
    if (!mult8(c->in_cstride) || !mult8(c->in_coff)) return lbm_fail(LBM_EINVAL, "input stride/offset must be multiples of 8");
    if (!c->in || !aligned16(c->in)) return lbm_fail(LBM_EINVAL, "input must be a 16-byte aligned device pointer");
    if ((c->flags & (LBMNN_S2D | LBMNN_D2S | LBMNN_S2D_G)) && c->ks != 1)
        return lbm_fail(LBM_EINVAL, "S2D / D2S modes need ks = 1");
    const int taps = (c->flags & LBMNN_S2D) ? (1 << c->dims) : (c->dims == 3 ? c->ks * c->ks * c->ks : c->ks * c->ks);
    if (!(c->flags & LBMNN_S2D) && c->in_coff + c->cin > c->in_cstride)
        return lbm_fail(LBM_EINVAL, "input channels exceed the stride");
    if ((c->flags & LBMNN_S2D) && c->in_coff + c->cin > c->in_cstride)
        return lbm_fail(LBM_EINVAL, "input channels exceed the stride");
    (void)taps;
    if (need_out) {
        if (!mult8(c->cout) || c->cout == 0) return lbm_fail(LBM_EINVAL, "cout must be a positive multiple of 8");
        if (!c->out && !c->out_f32) return lbm_fail(LBM_EINVAL, "no output");
        const int cw = (c->flags & LBMNN_D2S) ? (c->cout >> c->dims) : c->cout;
        if ((c->flags & LBMNN_D2S) && (!mult8(cw) || cw == 0)) return lbm_fail(LBM_EINVAL, "D2S needs cout / 2^dims multiple of 8");
        if (c->out_coff < 0 || c->out_coff + cw > c->out_cstride) return lbm_fail(LBM_EINVAL, "output channels exceed the stride");
    }
    return LBM_OK;
}

nn::ConvArgs to_args(const lbmnn_conv_desc *c, const void *w, const float *bias) {
    nn::ConvArgs a{};
    a.in = (const uint16_t *)c->in;
    a.in_cs = c->in_cstride;
    a.in_co = c->in_coff;
    a.wt = (const uint16_t *)w;
    a.bias = bias;
    a.out = (uint16_t *)c->out;
    a.out32 = c->out_f32;
    a.out_cs = c->out_cstride;
    a.out_co = c->out_coff;
    a.n = c->n; a.d = c->d; a.h = c->h; a.w = c->w;
    a.cin = c->cin;
    a.ncols = c->cout;
    a.ks = c->ks;
    a.dims = c->dims;
    a.flags = c->flags;
    const int taps = (c->flags & LBMNN_S2D) ? (1 << c->dims) : (c->dims == 3 ? c->ks * c->ks * c->ks : c->ks * c->ks);
    a.K = taps * c->cin;
    a.M = (long long)c->n * c->d * c->h * c->w;
    return a;
}

// Validation shared by the two weight-gradient entry points; fills the
// kernel arguments and the partials' size.
int wgrad_prepare(const lbmnn_conv_desc *c, const void *g, int g_cstride, int g_coff, int rows, const float *dw,
                  int splits, nn::ConvArgs &a, size_t &need) {
    int rc = check_desc(c, false);
    if (rc) return rc;
    if (!g || !aligned16(g) || !dw) return lbm_fail(LBM_EINVAL, "NULL or misaligned pointer");
    if (!mult8(rows) || rows == 0 || !mult8(g_cstride) || !mult8(g_coff))
        return lbm_fail(LBM_EINVAL, "rows, g stride and offset must be multiples of 8");
    if (splits < 1) return lbm_fail(LBM_EINVAL, "splits must be >= 1");
    a = to_args(c, nullptr, nullptr);
    a.flags = c->flags & ~LBMNN_S2D_G;
    if (c->flags & LBMNN_S2D_G) a.flags |= nn::FLAG_S2D_G;
    const int rcols = (c->flags & LBMNN_S2D_G) ? (rows >> c->dims) : rows;
    if ((c->flags & LBMNN_S2D_G) && (!mult8(rcols) || rcols == 0)) return lbm_fail(LBM_EINVAL, "rows / 2^dims must be a multiple of 8");
    if (g_coff + rcols > g_cstride) return lbm_fail(LBM_EINVAL, "gradient channels exceed the stride");
    need = lbmnn_wgrad_workspace_bytes(a.M, rows, a.K, splits);
    return LBM_OK;
}

// The weight-gradient partials of lbmnn_conv_wgrad_noalloc: one array per
// GPU, held until the process ends.  Host code reaches it only through the
// device address that hipGetSymbolAddress gives on each device (the array's
// name on the host side is a stand-in, not a device address).
constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) float scratch[LBMNN_NOALLOC_SCRATCH_BYTES / sizeof(float)];
std::mutex g_scratch_mu;
float *g_scratch[MAX_DEVICES] = {};

// The scratch array's device address on the current device (looked up once
// per device).
int scratch_ptr(float **out) {
    int dev = 0;
    NN_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return lbm_fail(LBM_EDEVICE, "device %d beyond the supported %d", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return lbm_fail(LBM_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch[dev] = (float *)p;
    }
    *out = g_scratch[dev];
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbmnn_conv(const lbmnn_conv_desc *c, const void *w, const float *bias, void *stream) {
    int rc = check_desc(c, true);
    if (rc) return rc;
    if (!w || !aligned16(w)) return lbm_fail(LBM_EINVAL, "weights must be a 16-byte aligned device pointer");
    NN_TRY(nn::conv(to_args(c, w, bias), (hipStream_t)stream));
    return LBM_OK;
}

size_t lbmnn_conv_workspace_bytes(const lbmnn_conv_desc *c) {
    if (check_desc(c, true)) return 0;
    const nn::ConvArgs a = to_args(c, nullptr, nullptr);
    const int S = nn::conv_splits(a);
    return S > 1 ? sizeof(float) * (size_t)S * (size_t)a.M * (size_t)a.ncols : 0;
}

int lbmnn_conv_ws(const lbmnn_conv_desc *c, const void *w, const float *bias, float *ws, size_t ws_bytes,
                  void *stream) {
    int rc = check_desc(c, true);
    if (rc) return rc;
    if (!w || !aligned16(w)) return lbm_fail(LBM_EINVAL, "weights must be a 16-byte aligned device pointer");
    const nn::ConvArgs a = to_args(c, w, bias);
    const int S = nn::conv_splits(a);
    if (S > 1) {
        const size_t need = sizeof(float) * (size_t)S * (size_t)a.M * (size_t)a.ncols;
        if (!ws) return lbm_fail(LBM_EINVAL, "workspace is NULL");
        if (ws_bytes < need) return lbm_fail(LBM_ENOMEM, "conv workspace of %zu bytes, %zu needed", ws_bytes, need);
        NN_TRY(nn::conv_split(a, ws, S, (hipStream_t)stream));
    } else {
        NN_TRY(nn::conv(a, (hipStream_t)stream));
    }
    return LBM_OK;
}

size_t lbmnn_wgrad_workspace_bytes(long long pixels, int rows, int K, int splits) {
    if (splits < 1) splits = 1;
    const long long chunk = nn::wgrad_chunk(pixels, splits);
    const long long z = chunk > 0 ? (pixels + chunk - 1) / chunk : 1;
    return sizeof(float) * (size_t)z * (size_t)rows * (size_t)K;
}

int lbmnn_conv_wgrad(const lbmnn_conv_desc *c, const void *g, int g_cstride, int g_coff, int rows, float *dw,
                     int accumulate, float *ws, size_t ws_bytes, int splits, void *stream) {
    nn::ConvArgs a;
    size_t need = 0;
    int rc = wgrad_prepare(c, g, g_cstride, g_coff, rows, dw, splits, a, need);
    if (rc) return rc;
    if (!ws) return lbm_fail(LBM_EINVAL, "workspace is NULL");
    if (ws_bytes < need) return lbm_fail(LBM_ENOMEM, "wgrad workspace of %zu bytes, %zu needed", ws_bytes, need);
    NN_TRY(nn::wgrad(a, (const uint16_t *)g, g_cstride, g_coff, rows, ws, splits, dw, accumulate,
                     (hipStream_t)stream));
    return LBM_OK;
}

int lbmnn_conv_wgrad_noalloc(const lbmnn_conv_desc *c, const void *g, int g_cstride, int g_coff, int rows,
                             float *dw, int accumulate, int splits, void *stream) {
    nn::ConvArgs a;
    size_t need = 0;
    int rc = wgrad_prepare(c, g, g_cstride, g_coff, rows, dw, splits, a, need);
    if (rc) return rc;
    if (need > (size_t)LBMNN_NOALLOC_SCRATCH_BYTES)
        return lbm_fail(LBM_ENOMEM, "the weight-gradient partials need %zu bytes, beyond the %d-byte scratch of "
                                    "lbmnn_conv_wgrad_noalloc: use fewer splits", need, LBMNN_NOALLOC_SCRATCH_BYTES);
    float *part = nullptr;
    if ((rc = scratch_ptr(&part))) return rc;
    NN_TRY(nn::wgrad(a, (const uint16_t *)g, g_cstride, g_coff, rows, part, splits, dw, accumulate,
                     (hipStream_t)stream));
    return LBM_OK;
}

int lbmnn_weight_transpose(const void *w, void *wt, int rows, int taps, int cols, int flip, void *stream) {
    if (!w || !wt || rows < 1 || taps < 1 || cols < 1) return lbm_fail(LBM_EINVAL, "bad transpose arguments");
    NN_TRY(nn::wtrans((const uint16_t *)w, (uint16_t *)wt, rows, taps, cols, flip, (hipStream_t)stream));
    return LBM_OK;
}

int lbmnn_bias_grad(const void *g, int cstride, int coff, long long pixels, int C, float *db, int accumulate,
                    float *ws, int splits, void *stream) {
    if (!g || !db || !ws || C < 1 || pixels < 1 || splits < 1 || coff + C > cstride)
        return lbm_fail(LBM_EINVAL, "bad bias-gradient arguments");
    NN_TRY(nn::bias_grad((const uint16_t *)g, cstride, coff, pixels, C, ws, splits, db, accumulate,
                         (hipStream_t)stream));
    return LBM_OK;
}

int lbmnn_relu_bwd(void *g, const void *y, int cstride, int coff, long long pixels, int C, void *stream) {
    if (!g || !y || C < 1 || coff + C > cstride) return lbm_fail(LBM_EINVAL, "bad ReLU-backward arguments");
    NN_TRY(nn::relu_bwd((uint16_t *)g, (const uint16_t *)y, cstride, coff, pixels, C, (hipStream_t)stream));
    return LBM_OK;
}

int lbmnn_relu_bwd_bias_grad(void *g, const void *y, int cstride, int coff, long long pixels, int C, float *db,
                             int accumulate, float *ws, int splits, void *stream) {
    if (!g || !y || !db || !ws || C < 1 || pixels < 1 || splits < 1 || coff + C > cstride)
        return lbm_fail(LBM_EINVAL, "bad ReLU-backward / bias-gradient arguments");
    NN_TRY(nn::relu_bwd_bias_grad((uint16_t *)g, (const uint16_t *)y, cstride, coff, pixels, C, ws, splits, db,
                                  accumulate, (hipStream_t)stream));
    return LBM_OK;
}

int lbmnn_pool_fwd(const void *in, int in_cstride, int in_coff, void *out, int out_cstride, int out_coff, int n,
                   int d, int h, int w, int C, int dims, void *stream) {
    if (!in || !out || C < 1 || (dims != 2 && dims != 3) || (dims == 2 && d != 1) || in_coff + C > in_cstride ||
        out_coff + C > out_cstride)
        return lbm_fail(LBM_EINVAL, "bad pooling arguments");
    NN_TRY(nn::pool_fwd((const uint16_t *)in, in_cstride, in_coff, (uint16_t *)out, out_cstride, out_coff, n, d, h, w,
                        C, dims, (hipStream_t)stream));
    return LBM_OK;
}

int lbmnn_pool_bwd(const void *in, int in_cstride, int in_coff, const void *gout, int g_cstride, int g_coff,
                   void *gin, int gi_cstride, int gi_coff, int n, int d, int h, int w, int C, int dims,
                   int accumulate, void *stream) {
    if (!in || !gout || !gin || C < 1 || (dims != 2 && dims != 3) || (dims == 2 && d != 1))
        return lbm_fail(LBM_EINVAL, "bad pooling arguments");
    NN_TRY(nn::pool_bwd((const uint16_t *)in, in_cstride, in_coff, (const uint16_t *)gout, g_cstride, g_coff,
                        (uint16_t *)gin, gi_cstride, gi_coff, n, d, h, w, C, dims, accumulate, (hipStream_t)stream));
    return LBM_OK;
}

int lbmnn_mse(const float *pred, int pcs, const float *tgt, const float *wpix, int creal, long long pixels,
              float scale, void *dpred, double *part, double *loss, void *stream) {
    if (!pred || !tgt || !dpred || !part || !loss || creal < 1 || creal > pcs || pixels < 1)
        return lbm_fail(LBM_EINVAL, "bad MSE arguments");
    NN_TRY(nn::mse(pred, pcs, tgt, wpix, creal, pixels, scale, (uint16_t *)dpred, part, loss, (hipStream_t)stream));
    return LBM_OK;
}

int lbmnn_adam(float *w, const float *g, float *m, float *v, void *wb, long long n, float lr, float beta1,
               float beta2, float eps, int t, void *stream) {
    if (!w || !g || !m || !v || n < 1 || t < 1) return lbm_fail(LBM_EINVAL, "bad Adam arguments");
    NN_TRY(nn::adam(w, g, m, v, (uint16_t *)wb, n, lr, beta1, beta2, eps, t, (hipStream_t)stream));
    return LBM_OK;
}

int lbmnn_to_bf16(const float *x, void *y, long long n, void *stream) {
    if (!x || !y || n < 0) return lbm_fail(LBM_EINVAL, "bad conversion arguments");
    if (n == 0) return LBM_OK;
    NN_TRY(nn::to_bf16(x, (uint16_t *)y, n, (hipStream_t)stream));
    return LBM_OK;
}

int lbmnn_features(const uint8_t *solid, const float *prm, int n, int d, int h, int w, void *out, void *stream) {
    if (!solid || !prm || !out || n < 1 || d < 1 || h < 1 || w < 1) return lbm_fail(LBM_EINVAL, "bad feature arguments");
    NN_TRY(nn::features(solid, prm, n, d, h, w, (uint16_t *)out, (hipStream_t)stream));
    return LBM_OK;
}

int lbmnn_normalize(const float *drho, const float *u, const uint8_t *solid, const float *prm, long long per_sample,
                    int D, long long pixels, float *tgt, float *wpix, void *stream) {
    if (!drho || !u || !solid || !prm || !tgt || per_sample < 1 || (D != 2 && D != 3))
        return lbm_fail(LBM_EINVAL, "bad normalisation arguments");
    NN_TRY(nn::normalize(drho, u, solid, prm, per_sample, D, pixels, tgt, wpix, (hipStream_t)stream));
    return LBM_OK;
}

int lbmnn_denormalize(const float *pred, int pcs, const uint8_t *solid, const float *prm, long long per_sample,
                      int D, long long pixels, float *drho, float *u, void *stream) {
    if (!pred || !solid || !prm || !drho || !u || per_sample < 1 || (D != 2 && D != 3) || pcs < 1 + D)
        return lbm_fail(LBM_EINVAL, "bad denormalisation arguments");
    NN_TRY(nn::denormalize(pred, pcs, solid, prm, per_sample, D, pixels, drho, u, (hipStream_t)stream));
    return LBM_OK;
}

long long lbmnn_flux_balance_workspace_bytes(int n, int d, int h, int w) {
    if (n < 1 || d < 1 || h < 1 || w < 1 || w > 2048 || (long long)d * h > 0x7fffffffLL) return 0;
    return nn::flux_balance_workspace_bytes(n, (long long)d * h, w);
}

int lbmnn_flux_balance(const uint8_t *solid, int n, int d, int h, int w, int D, float *u, void *ws,
                       long long ws_bytes, void *stream) {
    if (!solid || !u || !ws || n < 1 || n > 65535 || d < 1 || h < 1 || w < 1 || w > 2048 || (D != 2 && D != 3) ||
        (long long)d * h > 0x7fffffffLL || ((uintptr_t)ws & 7))
        return lbm_fail(LBM_EINVAL, "bad flux-balance arguments");
    if (ws_bytes < lbmnn_flux_balance_workspace_bytes(n, d, h, w))
        return lbm_fail(LBM_ENOMEM, "flux-balance workspace too small");
    NN_TRY(nn::flux_balance(solid, n, d * h, w, D, u, ws, (hipStream_t)stream));
    return LBM_OK;
}

}  // extern "C"
