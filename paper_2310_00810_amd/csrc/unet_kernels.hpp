// Kernel-side arguments and launchers of the U-Net operators.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nn {

enum {
    FLAG_RELU = 1,    // max(0, .) in the epilogue
    FLAG_ACC = 2,     // add to the existing output
    FLAG_S2D = 4,     // A operand gathered from the 2x finer grid (k = sub * cin + ci)
    FLAG_D2S = 8,     // output columns c = sub * Cr + co scattered to the 2x finer grid
    FLAG_S2D_G = 16,  // weight gradient: rows r = sub * Cr + co of G read on the finer grid
};

// Implicit GEMM  C[M x ncols] = A[M x K] * W^T  over pixels m of an
// n x d x h x w grid; A is the ks^dims stencil of `in` (or its S2D gather);
// W is [ncols][K] BF16.
struct ConvArgs {
    const uint16_t *in;
    int in_cs, in_co;
    const uint16_t *wt;
    const float *bias;
    uint16_t *out;
    float *out32;
    int out_cs, out_co;
    int n, d, h, w;
    int cin, ncols, ks, dims, flags;
    int K;
    long long M;
};

hipError_t conv(const ConvArgs &a, hipStream_t s);
int conv_splits(const ConvArgs &a);
hipError_t conv_split(const ConvArgs &a, float *part, int S, hipStream_t s);
long long wgrad_chunk(long long M, int splits);
hipError_t wgrad(const ConvArgs &a, const uint16_t *g, int g_cs, int g_co, int rows, float *part, int splits,
                 float *dw, int accumulate, hipStream_t s);
hipError_t bias_grad(const uint16_t *g, int cs, int co, long long npix, int C, float *part, int splits, float *db,
                     int accumulate, hipStream_t s);
hipError_t relu_bwd(uint16_t *g, const uint16_t *y, int cs, int co, long long npix, int C, hipStream_t s);
hipError_t relu_bwd_bias_grad(uint16_t *g, const uint16_t *y, int cs, int co, long long npix, int C, float *part,
                              int splits, float *db, int accumulate, hipStream_t s);
hipError_t pool_fwd(const uint16_t *in, int in_cs, int in_co, uint16_t *out, int out_cs, int out_co, int n, int d,
                    int h, int w, int C, int dims, hipStream_t s);
hipError_t pool_bwd(const uint16_t *in, int in_cs, int in_co, const uint16_t *gout, int g_cs, int g_co,
                    uint16_t *gin, int gi_cs, int gi_co, int n, int d, int h, int w, int C, int dims, int acc,
                    hipStream_t s);
hipError_t mse(const float *pred, int pcs, const float *tgt, const float *wpix, int creal, long long npix,
               float scale, uint16_t *dpred, double *part, double *loss, hipStream_t s);
hipError_t adam(float *w, const float *g, float *m1, float *m2, uint16_t *wb, long long n, float lr, float b1,
                float b2, float eps, int t, hipStream_t s);
hipError_t to_bf16(const float *x, uint16_t *y, long long n, hipStream_t s);
hipError_t features(const uint8_t *solid, const float *prm, int n, int d, int h, int w, uint16_t *out,
                    hipStream_t s);
hipError_t normalize(const float *drho, const float *u, const uint8_t *solid, const float *prm, long long per_sample,
                     int D, long long npix, float *tgt, float *wpix, hipStream_t s);
long long flux_balance_workspace_bytes(int n, long long rows, int w);
hipError_t flux_balance(const uint8_t *solid, int n, int rows, int w, int D, float *u, void *ws, hipStream_t s);
hipError_t denormalize(const float *pred, int pcs, const uint8_t *solid, const float *prm, long long per_sample,
                       int D, long long npix, float *drho, float *u, hipStream_t s);

}  // namespace nn

namespace nn {
hipError_t wtrans(const uint16_t *w, uint16_t *wt, int rows, int taps, int cols, int flip, hipStream_t s);
}
