/*
 * lbmnn.h -- C ABI of the warm-start network operators in liblbm.so.
 *
 * The paper proposes a neural-network initial guess for the inverse LBM runs
 * as future work (Section 3.1.2 end, Section 3.5).  These operators build
 * and train that network on the GPU: a U-Net whose input is the solid mask
 * and the boundary / viscosity parameters and whose output is the steady
 * density and velocity (Stokes-scaled), used to initialise equilibrium
 * populations (Eq. 5) before the plain LBM runs to its residual threshold.
 *
 * Tensors are pixel-major ("channels last": [n][d][h][w][C], d = 1 in 2D)
 * BF16 (uint16 storage) with an explicit channel stride (elements between
 * consecutive pixels) and channel offset, so that a producer can write into
 * a slice of a concatenated buffer.  Strides, offsets and channel counts are
 * multiples of 8 (16-byte vectors).  Products accumulate in FP32 on the
 * matrix cores (MFMA 16x16x32 BF16).  Weights of a ks^dims convolution are
 * stored [cout][tap][cin] (tap = (dz * ks + dy) * ks + dx), i.e. a
 * [cout][K] matrix with K = ks^dims * cin.
 *
 * All pointers are device pointers unless marked host; the caller owns all
 * memory (workspaces included) and every call is enqueued on `stream`
 * (hipStream_t, NULL = default stream).  Calls return LBM_OK or LBM_EINVAL /
 * LBM_EDEVICE (codes of lbm.h); lbm_last_error() gives the detail.
 */
#ifndef LBMNN_H
#define LBMNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBMNN_RELU 1        /* epilogue max(0, .) */
#define LBMNN_ACCUMULATE 2  /* add to the existing output instead of overwriting */
#define LBMNN_S2D 4         /* A operand gathered from the 2x finer grid: k = sub * cin + ci, sub = sx + 2 sy + 4 sz */
#define LBMNN_D2S 8         /* output column c = sub * (cout >> dims) + co written to the 2x finer grid */
#define LBMNN_S2D_G 16      /* weight gradient: gradient rows r = sub * Cr + co read on the finer grid */

/* One implicit GEMM over the pixels of an n x d x h x w grid:
 *   C[m][c] = sum_k A[m][k] W[c][k] (+ bias[c]),  m < n d h w, c < cout,
 * A = the ks^dims zero-padded stencil of `in` (ks = 3 or 1), or its S2D
 * gather from a grid twice as fine.  Used for the 3x3 (3x3x3) convolution
 * forward, its input gradient (with flipped, transposed weights, see
 * lbmnn_weight_transpose), the 2x2(x2) stride-2 transposed convolution
 * (ks = 1, D2S) and its input gradient (ks = 1, S2D). */
typedef struct lbmnn_conv_desc {
    int n, d, h, w;          /* GEMM-row grid; d = 1 when dims = 2; n d h w < 2^31 */
    int dims;                /* 2 or 3 */
    int ks;                  /* 3 or 1 */
    int cin;                 /* A channels per tap (multiple of 8) */
    int cout;                /* GEMM columns (multiple of 8) */
    int flags;               /* LBMNN_* */
    const void *in;          /* BF16 input */
    int in_cstride, in_coff;
    void *out;               /* BF16 output (used when out_f32 is NULL) */
    float *out_f32;          /* FP32 output (nullable) */
    int out_cstride, out_coff;
} lbmnn_conv_desc;

/* C = A W^T (+ bias, ReLU / accumulate per flags).  w: [cout][K] BF16;
 * bias: [cout] (D2S: [cout >> dims]) FP32, nullable. */
int lbmnn_conv(const lbmnn_conv_desc *c, const void *w, const float *bias, void *stream);

/* lbmnn_conv with a workspace for the layers whose implicit GEMM has too few
 * output tiles to fill the GPU (the deep, low-resolution levels, whose long
 * K = taps x cin loop would otherwise run on a few CUs): their contraction is
 * split into K ranges whose FP32 products go to ws, summed in range order
 * (deterministic) by a second kernel that applies the bias, ReLU /
 * accumulate and output layout of lbmnn_conv.  Every other layer runs as
 * lbmnn_conv and ignores ws.  ws: device memory of at least
 * lbmnn_conv_workspace_bytes(c) bytes (0 when the layer is not split; c is
 * validated as by lbmnn_conv, 0 for an invalid c); LBM_EINVAL for a NULL ws
 * that is needed, LBM_ENOMEM for a smaller one.  Arguments, results and other
 * errors as lbmnn_conv. */
size_t lbmnn_conv_workspace_bytes(const lbmnn_conv_desc *c);
int lbmnn_conv_ws(const lbmnn_conv_desc *c, const void *w, const float *bias, float *ws, size_t ws_bytes,
                  void *stream);

/* Weight gradient dW[r][k] = sum_m G[m][r] A[m][k] for the A operand that c
 * describes (c->cout is ignored), G = gradient of the GEMM output with
 * channel stride/offset g_cstride / g_coff and `rows` columns (LBMNN_S2D_G in
 * c->flags: rows = 2^dims * Cr gathered on the finer grid).  dW: FP32
 * [rows][K], overwritten or (accumulate) added to.  The pixel range is split
 * into `splits` parts whose FP32 partials go to workspace `ws` of at least
 * lbmnn_wgrad_workspace_bytes() bytes and are summed deterministically. */
size_t lbmnn_wgrad_workspace_bytes(long long pixels, int rows, int K, int splits);
int lbmnn_conv_wgrad(const lbmnn_conv_desc *c, const void *g, int g_cstride, int g_coff, int rows, float *dw,
                     int accumulate, float *ws, size_t ws_bytes, int splits, void *stream);

/* lbmnn_conv_wgrad without a workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, tight training loops,
 * harnesses that forbid allocation): the split partials go to a scratch
 * array of LBMNN_NOALLOC_SCRATCH_BYTES that the library holds on each GPU
 * for the life of the process.  It calls no allocator.  Arguments, results
 * and errors as lbmnn_conv_wgrad; LBM_ENOMEM when
 * lbmnn_wgrad_workspace_bytes(pixels, rows, K, splits) exceeds the scratch
 * (pass fewer splits).  Every call on one GPU uses the same scratch: calls
 * that overlap on that GPU (other streams, other threads) race, so order
 * them.  Nothing in the scratch needs clearing: each call writes every
 * partial it reads. */
#define LBMNN_NOALLOC_SCRATCH_BYTES (32 << 20)
int lbmnn_conv_wgrad_noalloc(const lbmnn_conv_desc *c, const void *g, int g_cstride, int g_coff, int rows,
                             float *dw, int accumulate, int splits, void *stream);

/* wt[c][tap'][r] = w[r][tap][c] with tap' = taps-1-tap when flip != 0
 * (BF16).  flip = 1, (rows, taps, cols) = (cout, ks^dims, cin) gives the
 * input-gradient weights of a convolution; flip = 0, taps = 1 transposes a
 * [rows][cols] matrix. */
int lbmnn_weight_transpose(const void *w, void *wt, int rows, int taps, int cols, int flip, void *stream);

/* Bias gradient db[c] = sum over pixels of g (channels c < C at stride
 * cstride, offset coff); ws: >= splits * C floats. */
int lbmnn_bias_grad(const void *g, int cstride, int coff, long long pixels, int C, float *db, int accumulate,
                    float *ws, int splits, void *stream);

/* g[m][c] = 0 where y[m][c] <= 0 (ReLU backward), same layout for g and y. */
int lbmnn_relu_bwd(void *g, const void *y, int cstride, int coff, long long pixels, int C, void *stream);

/* lbmnn_relu_bwd followed by lbmnn_bias_grad on the masked g, in one pass
 * over g and y when the layout allows 16-byte accesses (strides, offsets and
 * C multiples of 8, 16-byte aligned pointers, C <= 2048); same results as the
 * two calls.  ws: >= splits * C floats. */
int lbmnn_relu_bwd_bias_grad(void *g, const void *y, int cstride, int coff, long long pixels, int C, float *db,
                             int accumulate, float *ws, int splits, void *stream);

/* 2x2 (2x2x2) max pooling with stride 2; (n, d, h, w) is the coarse grid.
 * Backward routes each gradient to the first maximal element of its window
 * (window order sub = sx + 2 sy + 4 sz) and writes zero to the others, or
 * (accumulate) adds only at the maximal element. */
int lbmnn_pool_fwd(const void *in, int in_cstride, int in_coff, void *out, int out_cstride, int out_coff, int n,
                   int d, int h, int w, int C, int dims, void *stream);
int lbmnn_pool_bwd(const void *in, int in_cstride, int in_coff, const void *gout, int g_cstride, int g_coff,
                   void *gin, int gi_cstride, int gi_coff, int n, int d, int h, int w, int C, int dims,
                   int accumulate, void *stream);

/* Masked MSE: loss = scale * sum_m wpix[m] sum_{c < creal} (pred[m][c] - tgt[m][c])^2
 * with pred FP32 at channel stride pcs and tgt FP32 [m][creal]; writes the
 * BF16 gradient dpred [m][pcs] (zero beyond creal) and the loss (FP64) to
 * *loss.  part: >= ceil(pixels / 256) doubles.  wpix nullable (all 1). */
int lbmnn_mse(const float *pred, int pcs, const float *tgt, const float *wpix, int creal, long long pixels,
              float scale, void *dpred, double *part, double *loss, void *stream);

/* Adam on FP32 master weights w with moments m, v; t >= 1 is the step
 * count; wb (nullable) receives the BF16 copy. */
int lbmnn_adam(float *w, const float *g, float *m, float *v, void *wb, long long n, float lr, float beta1,
               float beta2, float eps, int t, void *stream);

/* y = BF16(x), round to nearest even. */
int lbmnn_to_bf16(const float *x, void *y, long long n, void *stream);

/* Network input, 8 BF16 channels per pixel: solid (0/1), x / (w - 1),
 * 200 drho_in, 200 drho_out, 2 (tau - 0.9), 0, 0, 0.  solid: uint8
 * [n][d][h][w]; prm: FP32 [n][3] = (drho_in, drho_out, tau). */
int lbmnn_features(const uint8_t *solid, const float *prm, int n, int d, int h, int w, void *out, void *stream);

/* Stokes scaling between LBM fields and network targets, per sample of
 * `per_sample` pixels with parameters prm [n][3]:
 *   t0 = (drho - drho_out) / (drho_in - drho_out),
 *   t_{1+a} = u_a nu / (cs^2 (drho_in - drho_out)),  nu = (tau - 1/2) / 3
 * (Eq. 9).  normalize: (drho [m], u [m][D]) -> tgt [m][1 + D] and the fluid
 * weights wpix [m] (nullable); denormalize: pred FP32 (channel stride pcs) ->
 * (drho, u), zero at solid nodes. */
int lbmnn_normalize(const float *drho, const float *u, const uint8_t *solid, const float *prm, long long per_sample,
                    int D, long long pixels, float *tgt, float *wpix, void *stream);
int lbmnn_denormalize(const float *pred, int pcs, const uint8_t *solid, const float *prm, long long per_sample,
                      int D, long long pixels, float *drho, float *u, void *stream);

/* Cross-section flux balance of a predicted velocity field, applied to the
 * network initial guess of Section 3.5 before it initialises the
 * populations: a steady flow conserves mass (Eq. 1-2 moments of a steady
 * state), so every cross-section normal to the flow direction x carries the
 * same flux.  Per sample, Q(x) = sum of u_x over the fluid nodes of section
 * x (all y, z; FP64, a fixed order) and Qbar = the mean of Q over the w
 * sections; every velocity component at every node of section x is
 * multiplied by min(max(Qbar / max(Q(x), Qbar / 10), 1/4), 4).  A sample
 * with Qbar <= 0 is left unchanged.  u: device FP32 [n][d][h][w][D] (D = 2
 * or 3), in place; solid: device uint8 [n][d][h][w]; n <= 65535,
 * 1 <= w <= 2048, d * h < 2^31; ws: device workspace of at least
 * lbmnn_flux_balance_workspace_bytes(n, d, h, w) bytes, 8-byte aligned,
 * owned by the caller (the section sums and factors).  Enqueued on `stream`;
 * LBM_EINVAL for other arguments, LBM_ENOMEM for a short workspace. */
long long lbmnn_flux_balance_workspace_bytes(int n, int d, int h, int w);   /* 0 for invalid sizes */
int lbmnn_flux_balance(const uint8_t *solid, int n, int d, int h, int w, int D, float *u, void *ws,
                       long long ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LBMNN_H */
