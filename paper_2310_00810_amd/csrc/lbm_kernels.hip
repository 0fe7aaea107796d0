// HIP kernels (gfx950) of the differentiable lattice Boltzmann method.
//
// State convention: a state buffer holds post-collision shifted populations
// F = f* - w.  One step (Section 2.1, Eq. 3-5; stage list of Section 2.2)
//   g^t = Z(S(F^{t-1}))   pull streaming with halfway bounce-back, Zou-He
//   F^t = C(g^t)          BGK collision towards the second-order equilibrium
// is one kernel launch; the loss (Eq. 7, Eq. 15) is evaluated on g^T.
//
// Reverse sweep (exact derivative of the discrete map, the function the
// paper's tape replay computes, Section 2.2):
//   nu^T = Z^T dl/dg^T                                  (seed kernel)
//   nu^k = Z^T C'(g^k)^T S^T nu^{k+1},  k = T-1 .. 1     (adjoint step kernel)
// S^T is a pull of nu from x + c_i with the mirrored bounce-back rule, so
// every output element has exactly one writer and all stores are aligned.
#include "lbm_device.hpp"
#include "lbm_kernels.hpp"

namespace lbm {

// ------------------------------------------------------------------ step --
template <int Q>
__global__ void __launch_bounds__(FT) k_step(Geo G, const float *__restrict__ src,
                                             float *__restrict__ dst,
                                             const float *__restrict__ face_in,
                                             const float *__restrict__ face_out) {
    constexpr int D = Vel<Q>::D;
    __shared__ uint2 lds[NBW];
    const FTile t = fluid_tile<D>(G, xcd_tile(blockIdx.x, gridDim.x));
    const InstDev &I = G.inst[t.b];
    if (t.staged) stage_windows<D>(G, I, t, lds);
    __syncthreads();
    const FLane n = fluid_lane(G, I, t, lds);
    if (!n.active) return;
    int nb[Q];
    neighbours<Q>(G, I, t, lds, n, nb);
    const int plane = (int)I.plane;
    float g[Q];
    gather<Q, +1>(src + I.st_off, plane, n.id, nb, g);
    if (G.bcx == BC_PRESSURE) {
        const long long f = I.face_off + (long long)n.z * I.ny + n.y;
        if (n.x == 0) zouhe<Q>(g, +1, face_in[f]);
        else if (n.x == I.nx - 1) zouhe<Q>(g, -1, face_out[f]);
    }
    const Moments m = moments<Q>(g);
    const float om = I.omega;
    float *__restrict__ out = dst + I.st_off;
#pragma unroll
    for (int i = 0; i < Q; ++i) out[i * plane + n.id] = g[i] + om * (feq_shifted<Q>(i, m) - g[i]);
}

// -------------------------------------------------------- loss functions --
// dl/du at one node for the built-in loss; returns l.
template <int D>
__device__ inline float loss_node(int kind, float wgt, const float *u, const float *t, float *dldu) {
    if (kind == LOSS_NORM) {
        float nu2 = 0.f, nt2 = 0.f;
#pragma unroll
        for (int a = 0; a < D; ++a) { nu2 += u[a] * u[a]; nt2 += t[a] * t[a]; }
        const float nu = sqrtf(nu2), nt = sqrtf(nt2);
        const float d = nu - nt;
        const float c = nu > 0.f ? 2.0f * wgt * d / nu : 0.f;
#pragma unroll
        for (int a = 0; a < D; ++a) dldu[a] = c * u[a];
        return wgt * d * d;
    }
    float l = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const float d = u[a] - t[a];
        l += d * d;
        dldu[a] = 2.0f * wgt * d;
    }
    return wgt * l;
}

template <int Q>
__device__ inline Moments load_moments(const float *__restrict__ F, const InstDev &I, int id) {
    float g[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] = F[I.st_off + (long long)i * I.plane + id];
    return moments<Q>(g);
}

// Loss on the final state (moments of F^T equal those of g^T: collision
// conserves rho and j).  part[tile] = block sum.
template <int Q>
__global__ void __launch_bounds__(BLOCK) k_loss(Geo G, const float *__restrict__ F,
                                                const float *__restrict__ roi,
                                                const float *__restrict__ target, int kind,
                                                double *__restrict__ part) {
    __shared__ double lds[4];
    constexpr int D = Vel<Q>::D;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const NodeRef n = map_node(G, tile);
    float l = 0.f;
    if (n.fluid) {
        const InstDev &I = G.inst[n.b];
        const Moments m = load_moments<Q>(F, I, n.id);
        const float u[3] = {m.ux, m.uy, m.uz};
        float t[3] = {0.f, 0.f, 0.f}, d[3];
#pragma unroll
        for (int a = 0; a < D; ++a) t[a] = target[I.poff * D + (long long)a * I.plane + n.id];
        l = loss_node<D>(kind, roi[I.poff + n.id] * I.loss_scale, u, t, d);
    }
    const double s = block_sum(l, lds);
    if (threadIdx.x == 0) part[tile] = s;
}

// -------------------------------------------------------------- adjoint --
// Seed kernel: nu^T = Z^T dl/dg^T, with g^T gathered from F^{T-1}.
// seed_du (nullable) replaces the built-in loss by a caller-given dL/du(T)
// in the dense layout [node][D].
template <int Q>
__global__ void __launch_bounds__(FT) k_adj_seed(Geo G, const float *__restrict__ Fprev,
                                                    float *__restrict__ nu_out,
                                                    const float *__restrict__ face_in,
                                                    const float *__restrict__ face_out,
                                                    double *__restrict__ grad_in,
                                                    double *__restrict__ grad_out,
                                                    const float *__restrict__ roi,
                                                    const float *__restrict__ target, int kind,
                                                    const float *__restrict__ seed_du) {
    constexpr int D = Vel<Q>::D;
    using V = Vel<Q>;
    __shared__ uint2 lds[NBW];
    const FTile t = fluid_tile<D>(G, xcd_tile(blockIdx.x, gridDim.x));
    const InstDev &I = G.inst[t.b];
    if (t.staged) stage_windows<D>(G, I, t, lds);
    __syncthreads();
    const FLane n = fluid_lane(G, I, t, lds);
    if (!n.active) return;
    int nb[Q];
    neighbours<Q>(G, I, t, lds, n, nb);
    float g[Q];
    gather<Q, +1>(Fprev + I.st_off, (int)I.plane, n.id, nb, g);
    int face = 0;
    long long f = 0;
    if (G.bcx == BC_PRESSURE) {
        f = I.face_off + (long long)n.z * I.ny + n.y;
        if (n.x == 0) { zouhe<Q>(g, +1, face_in[f]); face = 1; }
        else if (n.x == I.nx - 1) { zouhe<Q>(g, -1, face_out[f]); face = -1; }
    }
    const Moments m = moments<Q>(g);
    const float u[3] = {m.ux, m.uy, m.uz};
    float dldu[3] = {0.f, 0.f, 0.f};
    if (seed_du) {
        const long long dn = I.node_off + ((long long)n.z * I.ny + n.y) * I.nx + n.x;
#pragma unroll
        for (int a = 0; a < D; ++a) dldu[a] = seed_du[dn * D + a];
    } else {
        float t[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < D; ++a) t[a] = target[I.poff * D + (long long)a * I.plane + n.id];
        loss_node<D>(kind, roi[I.poff + n.id] * I.loss_scale, u, t, dldu);
    }
    const float inv = 1.0f / m.rho;
    float a[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i)
        a[i] = inv * (dldu[0] * (V::cx(i) - m.ux) + dldu[1] * (V::cy(i) - m.uy) +
                      (D == 3 ? dldu[2] * (V::cz(i) - m.uz) : 0.f));
    if (face == 1) grad_in[f] += (double)zouhe_adj<Q>(a, +1);
    else if (face == -1) grad_out[f] += (double)zouhe_adj<Q>(a, -1);
    float *__restrict__ out = nu_out + I.st_off;
#pragma unroll
    for (int i = 0; i < Q; ++i) out[i * (int)I.plane + n.id] = a[i];
}

// Adjoint step k: reads F^{k-1} (to rebuild g^k) and nu^{k+1}, writes nu^k;
// accumulates dL/dtau per tile and dL/d(drho_b) per face node.
template <int Q>
__global__ void __launch_bounds__(FT) k_adj_step(Geo G, const float *__restrict__ Fprev,
                                                    const float *__restrict__ nu_in,
                                                    float *__restrict__ nu_out,
                                                    const float *__restrict__ face_in,
                                                    const float *__restrict__ face_out,
                                                    double *__restrict__ grad_in,
                                                    double *__restrict__ grad_out,
                                                    double *__restrict__ dtau_part) {
    constexpr int D = Vel<Q>::D;
    __shared__ double red[4];
    __shared__ uint2 lds[NBW];
    using V = Vel<Q>;
    const FTile t = fluid_tile<D>(G, xcd_tile(blockIdx.x, gridDim.x));
    const InstDev &I = G.inst[t.b];
    if (t.staged) stage_windows<D>(G, I, t, lds);
    __syncthreads();
    const FLane n = fluid_lane(G, I, t, lds);
    float dtau = 0.f;
    if (n.active) {
        const int plane = (int)I.plane;
        int nb[Q];
        neighbours<Q>(G, I, t, lds, n, nb);
        float g[Q], lam[Q];
        gather<Q, +1>(Fprev + I.st_off, plane, n.id, nb, g);
        gather<Q, -1>(nu_in + I.st_off, plane, n.id, nb, lam);
        int face = 0;
        long long f = 0;
        if (G.bcx == BC_PRESSURE) {
            f = I.face_off + (long long)n.z * I.ny + n.y;
            if (n.x == 0) { zouhe<Q>(g, +1, face_in[f]); face = 1; }
            else if (n.x == I.nx - 1) { zouhe<Q>(g, -1, face_out[f]); face = -1; }
        }
        const Moments m = moments<Q>(g);
        const float usq = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
        // A = sum_k lam_k d feq_k / d rho,  B = sum_k lam_k d feq_k / d j
        float A = 0.f, Bx = 0.f, By = 0.f, Bz = 0.f;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const float cu = V::cx(k) * m.ux + V::cy(k) * m.uy + V::cz(k) * m.uz;
            const float wl = V::w(k) * lam[k];
            A += wl * (1.0f - 4.5f * cu * cu + 1.5f * usq);
            Bx += wl * (3.0f * V::cx(k) + 9.0f * cu * V::cx(k) - 3.0f * m.ux);
            By += wl * (3.0f * V::cy(k) + 9.0f * cu * V::cy(k) - 3.0f * m.uy);
            Bz += wl * (3.0f * V::cz(k) + 9.0f * cu * V::cz(k) - 3.0f * m.uz);
            dtau += lam[k] * (g[k] - feq_shifted<Q>(k, m));
        }
        dtau *= I.inv_tau2;
        const float om = I.omega, om1 = 1.0f - I.omega;
        float a[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i)
            a[i] = om1 * lam[i] + om * (A + Bx * V::cx(i) + By * V::cy(i) + Bz * V::cz(i));
        if (face == 1) grad_in[f] += (double)zouhe_adj<Q>(a, +1);
        else if (face == -1) grad_out[f] += (double)zouhe_adj<Q>(a, -1);
        float *__restrict__ out = nu_out + I.st_off;
#pragma unroll
        for (int i = 0; i < Q; ++i) out[i * plane + n.id] = a[i];
    }
    const double s = block_sum(dtau, red);
    if (threadIdx.x == 0) dtau_part[t.tile] += s;
}

// dL/dF^0 = S^T nu^1 in the dense layout [inst][i][nz][ny][nx], fluid nodes
// only (the caller zeroes the solid entries).
template <int Q>
__global__ void __launch_bounds__(FT) k_adj_final(Geo G, const float *__restrict__ nu_in,
                                                  float *__restrict__ dense) {
    constexpr int D = Vel<Q>::D;
    __shared__ uint2 lds[NBW];
    const FTile t = fluid_tile<D>(G, xcd_tile(blockIdx.x, gridDim.x));
    const InstDev &I = G.inst[t.b];
    if (t.staged) stage_windows<D>(G, I, t, lds);
    __syncthreads();
    const FLane n = fluid_lane(G, I, t, lds);
    if (!n.active) return;
    const long long nn = (long long)I.nx * I.ny * I.nz;
    const long long d0 = I.node_off * Q + ((long long)n.z * I.ny + n.y) * I.nx + n.x;
    int nb[Q];
    neighbours<Q>(G, I, t, lds, n, nb);
    float lam[Q];
    gather<Q, -1>(nu_in + I.st_off, (int)I.plane, n.id, nb, lam);
#pragma unroll
    for (int i = 0; i < Q; ++i) dense[d0 + i * nn] = lam[i];
}

// ------------------------------------------------------------ utilities --
// Initial state: shifted equilibrium of (drho, u) (dense arrays, nullable =
// rest) at every fluid node.
template <int Q>
__global__ void __launch_bounds__(BLOCK) k_init_eq(Geo G, float *__restrict__ F,
                                                   const float *__restrict__ drho,
                                                   const float *__restrict__ u) {
    constexpr int D = Vel<Q>::D;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const NodeRef n = map_node(G, tile);
    if (!n.fluid) return;
    const InstDev &I = G.inst[n.b];
    Moments m = {0.f, 1.f, 0.f, 0.f, 0.f};
    const long long dn = dense_index(I, n);
    if (drho) { m.drho = drho[dn]; m.rho = 1.0f + m.drho; }
    if (u) {
        m.ux = u[dn * D];
        m.uy = u[dn * D + 1];
        if (D == 3) m.uz = u[dn * D + 2];
    }
    float *__restrict__ out = F + I.st_off + n.id;
#pragma unroll
    for (int i = 0; i < Q; ++i) out[(long long)i * I.plane] = feq_shifted<Q>(i, m);
}

// dense [inst][i][nz][ny][nx] <-> compact state.  to_state: fluid nodes only;
// from state: zero at solid nodes.
template <int Q>
__global__ void __launch_bounds__(BLOCK) k_convert(Geo G, float *__restrict__ F,
                                                   float *__restrict__ dense, int to_state) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const NodeRef n = map_node(G, tile);
    if (!n.inside) return;
    const InstDev &I = G.inst[n.b];
    const long long nn = (long long)I.nx * I.ny * I.nz;
    const long long d0 = I.node_off * Q + ((long long)n.z * I.ny + n.y) * I.nx + n.x;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const long long o = I.st_off + (long long)i * I.plane + n.id;
        if (to_state) { if (n.fluid) F[o] = dense[d0 + i * nn]; }
        else dense[d0 + i * nn] = n.fluid ? F[o] : 0.f;
    }
}

// Macroscopic fields (dense): drho [node], u [node][D]; with Fb != NULL the
// mean of the two states.
template <int Q>
__global__ void __launch_bounds__(BLOCK) k_macro(Geo G, const float *__restrict__ Fa,
                                                 const float *__restrict__ Fb,
                                                 float *__restrict__ drho, float *__restrict__ u) {
    constexpr int D = Vel<Q>::D;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const NodeRef n = map_node(G, tile);
    if (!n.inside) return;
    const InstDev &I = G.inst[n.b];
    const long long dn = dense_index(I, n);
    float r = 0.f, v[3] = {0.f, 0.f, 0.f};
    if (n.fluid) {
        Moments m = load_moments<Q>(Fa, I, n.id);
        r = m.drho; v[0] = m.ux; v[1] = m.uy; v[2] = m.uz;
        if (Fb) {
            m = load_moments<Q>(Fb, I, n.id);
            r = 0.5f * (r + m.drho);
            v[0] = 0.5f * (v[0] + m.ux); v[1] = 0.5f * (v[1] + m.uy); v[2] = 0.5f * (v[2] + m.uz);
        }
    }
    if (drho) drho[dn] = r;
    if (u) {
#pragma unroll
        for (int a = 0; a < D; ++a) u[dn * D + a] = v[a];
    }
}

// Residual sums of the two-step mean velocity:
//   part[2 tile]   = sum |u(t) - u(t-2)|^2,  part[2 tile+1] = sum |u(t) + u(t-1)|^2
// u(t-2) comes from a dense velocity snapshot.
template <int Q>
__global__ void __launch_bounds__(BLOCK) k_residual(Geo G, const float *__restrict__ Ft,
                                                    const float *__restrict__ Ft1,
                                                    const float *__restrict__ u2,
                                                    double *__restrict__ part) {
    __shared__ double lds[4];
    constexpr int D = Vel<Q>::D;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const NodeRef n = map_node(G, tile);
    float num = 0.f, den = 0.f;
    if (n.fluid) {
        const InstDev &I = G.inst[n.b];
        const long long dn = dense_index(I, n);
        const Moments a = load_moments<Q>(Ft, I, n.id);
        const Moments b = load_moments<Q>(Ft1, I, n.id);
        const float ua[3] = {a.ux, a.uy, a.uz}, ub[3] = {b.ux, b.uy, b.uz};
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const float d = ua[c] - u2[dn * D + c];
            const float s = ua[c] + ub[c];
            num += d * d;
            den += s * s;
        }
    }
    const double sn = block_sum(num, lds);
    const double sd = block_sum(den, lds);
    if (threadIdx.x == 0) { part[2 * tile] = sn; part[2 * tile + 1] = sd; }
}

// Per-instance sums of per-tile partials (stride values per tile):
// out[b * stride + k] = sum over the instance's tiles of part[tile * stride + k].
// fluid != 0 sums over the instance's fluid tiles instead of its dense tiles.
__global__ void __launch_bounds__(256) k_reduce(const InstDev *inst, const double *__restrict__ part,
                                                int stride, int fluid, double *__restrict__ out) {
    __shared__ double s[256];
    const InstDev &I = inst[blockIdx.x];
    const int begin = fluid ? I.ftile_begin : I.tile_begin, count = fluid ? I.n_ftiles : I.n_tiles;
    for (int k = 0; k < stride; ++k) {
        double acc = 0.0;
        for (int t = threadIdx.x; t < count; t += 256) acc += part[(long long)(begin + t) * stride + k];
        s[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[blockIdx.x * stride + k] = s[0];
        __syncthreads();
    }
}

__global__ void k_fill_f64(double *p, long long n, double v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_f32(float *p, long long n, float v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------ launch wrappers --
static inline dim3 grid_of(const Geo &G) { return dim3((unsigned)G.n_tiles); }
static inline dim3 fgrid_of(const Geo &G) { return dim3((unsigned)G.n_ftiles); }

template <int Q>
static hipError_t launch_step_q(const Geo &G, const float *src, float *dst, const float *fin,
                                const float *fout, hipStream_t s) {
    if (G.n_ftiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_step<Q>, fgrid_of(G), dim3(FT), 0, s, G, src, dst, fin, fout);
    return hipGetLastError();
}

hipError_t launch_step(int q, const Geo &G, const float *src, float *dst, const float *fin,
                       const float *fout, hipStream_t s) {
    return q == 9 ? launch_step_q<9>(G, src, dst, fin, fout, s)
                  : launch_step_q<19>(G, src, dst, fin, fout, s);
}

hipError_t launch_loss(int q, const Geo &G, const float *F, const float *roi, const float *target,
                       int kind, double *part, hipStream_t s) {
    if (q == 9) hipLaunchKernelGGL(k_loss<9>, grid_of(G), dim3(BLOCK), 0, s, G, F, roi, target, kind, part);
    else hipLaunchKernelGGL(k_loss<19>, grid_of(G), dim3(BLOCK), 0, s, G, F, roi, target, kind, part);
    return hipGetLastError();
}

hipError_t launch_adj_seed(int q, const Geo &G, const float *Fprev, float *nu_out, const float *fin,
                           const float *fout, double *gin, double *gout, const float *roi,
                           const float *target, int kind, const float *seed, hipStream_t s) {
    if (G.n_ftiles == 0) return hipSuccess;
    if (q == 9)
        hipLaunchKernelGGL(k_adj_seed<9>, fgrid_of(G), dim3(FT), 0, s, G, Fprev, nu_out, fin, fout,
                           gin, gout, roi, target, kind, seed);
    else
        hipLaunchKernelGGL(k_adj_seed<19>, fgrid_of(G), dim3(FT), 0, s, G, Fprev, nu_out, fin, fout,
                           gin, gout, roi, target, kind, seed);
    return hipGetLastError();
}

hipError_t launch_adj_step(int q, const Geo &G, const float *Fprev, const float *nu_in, float *nu_out,
                           const float *fin, const float *fout, double *gin, double *gout,
                           double *dtau_part, hipStream_t s) {
    if (G.n_ftiles == 0) return hipSuccess;
    if (q == 9)
        hipLaunchKernelGGL(k_adj_step<9>, fgrid_of(G), dim3(FT), 0, s, G, Fprev, nu_in, nu_out, fin,
                           fout, gin, gout, dtau_part);
    else
        hipLaunchKernelGGL(k_adj_step<19>, fgrid_of(G), dim3(FT), 0, s, G, Fprev, nu_in, nu_out, fin,
                           fout, gin, gout, dtau_part);
    return hipGetLastError();
}

hipError_t launch_adj_final(int q, const Geo &G, const float *nu_in, float *dense, long long n_dense,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n_dense + 255) / 256)), dim3(256), 0, s, dense, n_dense, 0.f);
    if (G.n_ftiles == 0) return hipGetLastError();
    if (q == 9) hipLaunchKernelGGL(k_adj_final<9>, fgrid_of(G), dim3(FT), 0, s, G, nu_in, dense);
    else hipLaunchKernelGGL(k_adj_final<19>, fgrid_of(G), dim3(FT), 0, s, G, nu_in, dense);
    return hipGetLastError();
}

hipError_t launch_init_eq(int q, const Geo &G, float *F, const float *drho, const float *u,
                          hipStream_t s) {
    if (q == 9) hipLaunchKernelGGL(k_init_eq<9>, grid_of(G), dim3(BLOCK), 0, s, G, F, drho, u);
    else hipLaunchKernelGGL(k_init_eq<19>, grid_of(G), dim3(BLOCK), 0, s, G, F, drho, u);
    return hipGetLastError();
}

hipError_t launch_convert(int q, const Geo &G, float *F, float *dense, int to_state, hipStream_t s) {
    if (q == 9) hipLaunchKernelGGL(k_convert<9>, grid_of(G), dim3(BLOCK), 0, s, G, F, dense, to_state);
    else hipLaunchKernelGGL(k_convert<19>, grid_of(G), dim3(BLOCK), 0, s, G, F, dense, to_state);
    return hipGetLastError();
}

hipError_t launch_macro(int q, const Geo &G, const float *Fa, const float *Fb, float *drho, float *u,
                        hipStream_t s) {
    if (q == 9) hipLaunchKernelGGL(k_macro<9>, grid_of(G), dim3(BLOCK), 0, s, G, Fa, Fb, drho, u);
    else hipLaunchKernelGGL(k_macro<19>, grid_of(G), dim3(BLOCK), 0, s, G, Fa, Fb, drho, u);
    return hipGetLastError();
}

hipError_t launch_residual(int q, const Geo &G, const float *Ft, const float *Ft1, const float *u2,
                           double *part, hipStream_t s) {
    if (q == 9) hipLaunchKernelGGL(k_residual<9>, grid_of(G), dim3(BLOCK), 0, s, G, Ft, Ft1, u2, part);
    else hipLaunchKernelGGL(k_residual<19>, grid_of(G), dim3(BLOCK), 0, s, G, Ft, Ft1, u2, part);
    return hipGetLastError();
}

hipError_t launch_reduce(const InstDev *inst, int n_inst, const double *part, int stride, int fluid,
                         double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(n_inst), dim3(256), 0, s, inst, part, stride, fluid, out);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, long long n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace lbm
