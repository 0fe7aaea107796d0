// Launch wrappers of the lattice Boltzmann kernels (host side).
#pragma once

#include "lbm_device.hpp"

namespace lbm {

hipError_t launch_step(int q, const Geo &G, const float *src, float *dst, const float *fin,
                       const float *fout, bool tape, hipStream_t s);
// Sets *flag = 1 if states a and b differ in any population of a fluid node.
hipError_t launch_compare(int q, const Geo &G, const float *a, const float *b, unsigned *flag, hipStream_t s);
// acc: add to the partials (the later frames of a time-windowed loss).
hipError_t launch_loss(int q, const Geo &G, const float *F, const float *roi, const float *target,
                       int kind, double *part, int acc, hipStream_t s);
hipError_t launch_adj_seed(int q, const Geo &G, const float *Fprev, float *nu_out, const float *fin,
                           const float *fout, double *gin, double *gout, const float *roi,
                           const float *target, int kind, const float *seed, hipStream_t s);
// target (nullable): the loss frame taken on g^k, whose derivative joins nu^k.
hipError_t launch_adj_step(int q, const Geo &G, const float *Fprev, const float *nu_in, float *nu_out,
                           const float *fin, const float *fout, double *gin, double *gout,
                           double *dtau_part, const float *roi, const float *target, int kind, hipStream_t s);
// Zeroes the n_dense floats of dense, then writes the fluid entries
// (F0 and the face densities serve the anti-bounce-back transpose).
hipError_t launch_adj_final(int q, const Geo &G, const float *nu_in, const float *F0, const float *fin,
                            const float *fout, float *dense, long long n_dense, hipStream_t s);
// Anti-bounce-back faces: adds dL/d(drho_b) of the closure that built g^1.
hipError_t launch_abb_grad0(int q, const Geo &G, const float *F0, const float *nu1, const float *fin,
                            const float *fout, double *gin, double *gout, hipStream_t s);
hipError_t launch_init_eq(int q, const Geo &G, float *F, const float *drho, const float *u,
                          hipStream_t s);
hipError_t launch_convert(int q, const Geo &G, float *F, float *dense, int to_state, hipStream_t s);
hipError_t launch_macro(int q, const Geo &G, const float *Fa, const float *Fb, float *drho, float *u,
                        hipStream_t s);
// Residual partials of the two-step mean of (Ft, Ft1) against the snapshot,
// which then takes that mean.
hipError_t launch_residual(int q, const Geo &G, const float *Ft, const float *Ft1, float *snap,
                           double *part, hipStream_t s);
// fluid != 0: partials per fluid tile (dtau), else per dense tile.
hipError_t launch_reduce(const InstDev *inst, int n_inst, const double *part, int stride, int fluid,
                         double *out, hipStream_t s);
hipError_t launch_fill_f64(double *p, long long n, double v, hipStream_t s);
hipError_t launch_fill_u32(unsigned *p, long long n, unsigned v, hipStream_t s);
// n16 16-byte elements from src to dst, one per lane.
hipError_t launch_copy16(const void *src, void *dst, long long n16, hipStream_t s);

}  // namespace lbm
