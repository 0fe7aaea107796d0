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
#include <algorithm>

#include "lbm_device.hpp"
#include "lbm_kernels.hpp"

namespace lbm {

// ------------------------------------------------------------------ step --
// The block prologue shared by the fluid-tile kernels: stage the row
// windows, locate the lane's node.
#define FLUID_PROLOGUE()                                                    \
    constexpr int D = Vel<Q>::D;                                            \
    __shared__ TileLds L;                                                   \
    const FTile t = fluid_tile<D>(G, xcd_tile(blockIdx.x, gridDim.x));      \
    const InstDev &I = G.inst[t.b];                                         \
    if (t.staged) stage_windows<D>(G, I, t, L);                             \
    __syncthreads();                                                        \
    const FLane n = fluid_lane(G, I, t, L)

// True when some lane of the wavefront sits on an inlet or outlet face: the
// step and seed kernels skip the (branch-free) Zou-He closure in wavefronts
// without face nodes, most of them in rows much wider than a wavefront.  The
// adjoint step keeps it unconditional: with the branch it spills registers
// and ran 20 % slower.
__device__ inline bool wave_has_face(bool face) { return __builtin_amdgcn_ballot_w64(face) != 0; }

// Face density of a node on a Zou-He face (issued before the gathers).
template <int BCX>
__device__ inline float face_density(const InstDev &I, const FLane &n, bool in, bool out,
                                     const float *__restrict__ face_in, const float *__restrict__ face_out) {
    float d = 0.f;
    if (density_faces(BCX) && (in || out)) d = in ? face_in[I.face_off + n.r] : face_out[I.face_off + n.r];
    return d;
}

// Adjoints of the unknowns of g^{k+1} at a face node (its own slots of
// nu^{k+1}, zero elsewhere) for the anti-bounce-back transpose.
template <int Q>
__device__ inline void face_unknown_adjoints(__amdgpu_buffer_rsrc_t rn, int plane, unsigned own, bool in, bool out,
                                             float (&nuo)[Q]) {
    using V = Vel<Q>;
#pragma unroll
    for (int i = 0; i < Q; ++i) nuo[i] = 0.f;
#pragma unroll
    for (int i = 1; i < Q; ++i)
        if (V::cx(i) != 0 && (V::cx(i) > 0 ? in : out)) nuo[i] = bload(rn, own + (unsigned)(i * plane) * 4u);
}

// NTM: 0 default cache policy, 1 non-temporal stores (a destination that no
// later step reads while it could still be cached: a tape state, or any
// state when two exceed the Infinity Cache), 2 non-temporal gathers too
// (D3Q19 states beyond the Infinity Cache).
template <int Q, int BCX, int NTM>
__global__ void __launch_bounds__(FT) k_step(Geo G, const float *__restrict__ src,
                                             float *__restrict__ dst,
                                             const float *__restrict__ face_in,
                                             const float *__restrict__ face_out) {
    FLUID_PROLOGUE();
    if (!n.active) return;
    const bool in = density_faces(BCX) && n.x == 0, out = density_faces(BCX) && n.x == I.nx - 1;
    const float drho_b = face_density<BCX>(I, n, in, out, face_in, face_out);
    const int plane = (int)I.plane;
    const __amdgpu_buffer_rsrc_t rs = planes_rsrc(src + I.st_off, Q, I.plane);
    float rhoF = 1.0f, uF[3] = {0.f, 0.f, 0.f};
    if (BCX == BC_ABB && (in || out)) own_velocity<Q>(rs, plane, (unsigned)n.id * 4u, rhoF, uF);
    Links<Q> k;
    links<Q, BCX>(G, I, t, L, n, k);
    float g[Q];
    gather_fwd<Q, BCX, NTM == 2>(rs, plane, k, g);
    if (zouhe_faces(BCX) && wave_has_face(in || out)) zouhe<Q>(g, in, out, drho_b, BCX == BC_VELOCITY);
    if (BCX == BC_ABB) abb<Q>(g, in, out, drho_b, uF);
    const Moments m = moments<Q>(g);
    const float om = I.omega;
    const __amdgpu_buffer_rsrc_t rd = planes_rsrc(dst + I.st_off, Q, I.plane);
    const unsigned own = (unsigned)n.id * 4u;
    float feq[Q];
    feq_all<Q>(m, feq);
    if constexpr (Q == 9) {
        if (G.coll == COLL_MRT) {
            float d[9], r[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) d[i] = g[i] - feq[i];
            mrt_relax(d, G.mrt, om, r);
#pragma unroll
            for (int i = 0; i < 9; ++i) bstore<(NTM >= 1)>(rd, g[i] - r[i], own, plane_off(i, plane));
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) bstore<(NTM >= 1)>(rd, g[i] + om * (feq[i] - g[i]), own, plane_off(i, plane));
}

// Bit-for-bit comparison of two states over the fluid nodes of every
// instance: a lane whose populations differ sets *flag (the padding past each
// instance's fluid nodes is not compared).
template <int Q>
__global__ void __launch_bounds__(FT) k_compare(Geo G, const float *__restrict__ a, const float *__restrict__ b,
                                                unsigned *__restrict__ flag) {
    const FTileDesc e = G.fblk[blockIdx.x];
    const InstDev &I = G.inst[e.b];
    const int id = ((int)blockIdx.x - I.ftile_begin) * FT + (int)threadIdx.x;
    if (id >= I.n_fluid) return;
    const unsigned *pa = (const unsigned *)(a + I.st_off) + id, *pb = (const unsigned *)(b + I.st_off) + id;
    bool bad = false;
#pragma unroll
    for (int i = 0; i < Q; ++i) bad |= pa[(long long)i * I.plane] != pb[(long long)i * I.plane];
    if (bad) *flag = 1u;
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

// Loss on a state F^t (its moments equal those of g^t: collision conserves
// rho and j).  part[tile] = block sum, or += with acc (the frames of a
// time-windowed loss, added in time order).
template <int Q>
__global__ void __launch_bounds__(BLOCK) k_loss(Geo G, const float *__restrict__ F,
                                                const float *__restrict__ roi,
                                                const float *__restrict__ target, int kind,
                                                double *__restrict__ part, int acc) {
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
    if (threadIdx.x == 0) part[tile] = acc ? part[tile] + s : s;
}

// -------------------------------------------------------------- adjoint --
// Seed kernel: nu^T = Z^T dl/dg^T, with g^T gathered from F^{T-1}.
// seed_du (nullable) replaces the built-in loss by a caller-given dL/du(T)
// in the dense layout [node][D].
template <int Q, int BCX>
__global__ void __launch_bounds__(FT) k_adj_seed(Geo G, const float *__restrict__ Fprev,
                                                 float *__restrict__ nu_out,
                                                 const float *__restrict__ face_in,
                                                 const float *__restrict__ face_out,
                                                 double *__restrict__ grad_in,
                                                 double *__restrict__ grad_out,
                                                 const float *__restrict__ roi,
                                                 const float *__restrict__ target, int kind,
                                                 const float *__restrict__ seed_du) {
    using V = Vel<Q>;
    FLUID_PROLOGUE();
    if (!n.active) return;
    const bool in = density_faces(BCX) && n.x == 0, out = density_faces(BCX) && n.x == I.nx - 1;
    const float drho_b = face_density<BCX>(I, n, in, out, face_in, face_out);
    const int plane = (int)I.plane;
    const __amdgpu_buffer_rsrc_t rs = planes_rsrc(Fprev + I.st_off, Q, I.plane);
    float rhoF = 1.0f, uF[3] = {0.f, 0.f, 0.f};
    if (BCX == BC_ABB && (in || out)) own_velocity<Q>(rs, plane, (unsigned)n.id * 4u, rhoF, uF);
    Links<Q> k;
    links<Q, BCX>(G, I, t, L, n, k);
    float g[Q];
    gather_fwd<Q, BCX>(rs, plane, k, g);
    if (zouhe_faces(BCX) && wave_has_face(in || out)) zouhe<Q>(g, in, out, drho_b, BCX == BC_VELOCITY);
    if (BCX == BC_ABB) abb<Q>(g, in, out, drho_b, uF);
    const Moments m = moments<Q>(g);
    const float u[3] = {m.ux, m.uy, m.uz};
    float dldu[3] = {0.f, 0.f, 0.f};
    if (seed_du) {
        const long long dn = I.node_off + (long long)n.r * I.nx + n.x;
#pragma unroll
        for (int a = 0; a < D; ++a) dldu[a] = seed_du[dn * D + a];
    } else {
        float tg[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < D; ++a) tg[a] = target[I.poff * D + (long long)a * I.plane + n.id];
        loss_node<D>(kind, roi[I.poff + n.id] * I.loss_scale, u, tg, dldu);
    }
    const float inv = 1.0f / m.rho;
    float a[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i)
        a[i] = inv * (dldu[0] * (V::cx(i) - m.ux) + dldu[1] * (V::cy(i) - m.uy) +
                      (D == 3 ? dldu[2] * (V::cz(i) - m.uz) : 0.f));
    if (zouhe_faces(BCX) && wave_has_face(in || out)) {
        const float jb = zouhe_adj<Q>(a, in, out, g, drho_b, BCX == BC_VELOCITY);
        if (in) grad_in[I.face_off + n.r] += (double)jb;
        else if (out) grad_out[I.face_off + n.r] += (double)jb;
    }
    const __amdgpu_buffer_rsrc_t rd = planes_rsrc(nu_out + I.st_off, Q, I.plane);
    const unsigned own = (unsigned)n.id * 4u;
#pragma unroll
    for (int i = 0; i < Q; ++i) bstore(rd, a[i], own, plane_off(i, plane));
}

// Adjoint step k: reads F^{k-1} (to rebuild g^k) and nu^{k+1}, writes nu^k;
// accumulates dL/dtau per tile and dL/d(drho_b) per face node.  SEED: g^k
// carries a frame of a time-windowed loss (target), whose dl/dg^k joins the
// collision transpose's output before the boundary transpose.  With
// lam = S^T nu^{k+1} and the moments of w lam (S0, S_a, S_ab), the
// collision transpose is  a_i = (1 - omega) lam_i + omega (A + B . c_i)  with
//   A   = sum_k lam_k dfeq_k/drho = S0 (1 + 1.5 u.u) - 4.5 u.S2.u,
//   B_a = sum_k lam_k dfeq_k/dj_a = 3 S_a + 9 (S2 u)_a - 3 u_a S0.
template <int Q, int BCX, bool SEED, bool NT>
__global__ void __launch_bounds__(FT) __attribute__((amdgpu_waves_per_eu(6))) k_adj_step(Geo G, const float *__restrict__ Fprev,
                                                 const float *__restrict__ nu_in,
                                                 float *__restrict__ nu_out,
                                                 const float *__restrict__ face_in,
                                                 const float *__restrict__ face_out,
                                                 double *__restrict__ grad_in,
                                                 double *__restrict__ grad_out,
                                                 double *__restrict__ dtau_part,
                                                 const float *__restrict__ roi,
                                                 const float *__restrict__ target, int kind) {
    using V = Vel<Q>;
    __shared__ double red[4];
    FLUID_PROLOGUE();
    float dtau = 0.f;
    if (n.active) {
        const bool in = density_faces(BCX) && n.x == 0, out = density_faces(BCX) && n.x == I.nx - 1;
        const float drho_b = face_density<BCX>(I, n, in, out, face_in, face_out);
        const int plane = (int)I.plane;
        const unsigned own = (unsigned)n.id * 4u;
        const __amdgpu_buffer_rsrc_t rs = planes_rsrc(Fprev + I.st_off, Q, I.plane);
        const __amdgpu_buffer_rsrc_t rn = planes_rsrc(nu_in + I.st_off, Q, I.plane);
        float rhoF = 1.0f, uF[3] = {0.f, 0.f, 0.f};
        float nuo[Q];
        if (BCX == BC_ABB) {
#pragma unroll
            for (int i = 0; i < Q; ++i) nuo[i] = 0.f;
            if (in || out) {
                own_velocity<Q>(rs, plane, own, rhoF, uF);
                face_unknown_adjoints<Q>(rn, plane, own, in, out, nuo);
            }
        }
        Links<Q> k;
        links<Q, BCX>(G, I, t, L, n, k);
        float g[Q], lam[Q];
        gather_fwd<Q, BCX, NT && Q == 19>(rs, plane, k, g);
        gather_adj<Q, NT && Q == 19>(rn, plane, k, lam);
        if (zouhe_faces(BCX)) zouhe<Q>(g, in, out, drho_b, BCX == BC_VELOCITY);
        if (BCX == BC_ABB) abb<Q>(g, in, out, drho_b, uF);
        const Moments m = moments<Q>(g);
        if (BCX == BC_ABB) {
            // g^{k+1}'s unknowns at this face node were built from F^k, whose
            // moments are those of g^k
            const float um[3] = {m.ux, m.uy, m.uz};
            const float jb = abb_adj<Q>(lam, in, out, drho_b, m.rho, um, nuo);
            if (in) grad_in[I.face_off + n.r] += (double)jb;
            else if (out) grad_out[I.face_off + n.r] += (double)jb;
        }
        // the equilibrium part of the collision transpose acts on mu:
        // BGK mu = omega lam; MRT mu = M^-1 S M lam (the update matrix is
        // symmetric), with dL/dtau from the two stress rates only
        float mu[Q];
        bool mrt = false;
        if constexpr (Q == 9) mrt = G.coll == COLL_MRT;
        if constexpr (Q == 9) {
            if (mrt) {
                mrt_relax(lam, G.mrt, I.omega, mu);
                float y7 = 0.f, y8 = 0.f, d7 = 0.f, d8 = 0.f, feq[9];
                feq_all<Q>(m, feq);
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const float dq = g[i] - feq[i];
                    if (mrt_m(7, i)) { y7 += mrt_m(7, i) * lam[i]; d7 += mrt_m(7, i) * dq; }
                    if (mrt_m(8, i)) { y8 += mrt_m(8, i) * lam[i]; d8 += mrt_m(8, i) * dq; }
                }
                dtau = (y7 * d7 / (float)mrt_norm(7) + y8 * d8 / (float)mrt_norm(8)) * I.inv_tau2;
            }
        }
        if (!mrt) {
#pragma unroll
            for (int q = 0; q < Q; ++q) mu[q] = lam[q];
        }
        float S0 = 0.f, Sx = 0.f, Sy = 0.f, Sz = 0.f;
        float Sxx = 0.f, Syy = 0.f, Szz = 0.f, Sxy = 0.f, Sxz = 0.f, Syz = 0.f;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int cx = V::cx(q), cy = V::cy(q), cz = V::cz(q);
            const float wl = V::w(q) * mu[q];
            S0 += wl;
            if (cx) { Sx += cx * wl; Sxx += wl; }
            if (cy) { Sy += cy * wl; Syy += wl; }
            if (cz) { Sz += cz * wl; Szz += wl; }
            if (cx && cy) Sxy += cx * cy * wl;
            if (cx && cz) Sxz += cx * cz * wl;
            if (cy && cz) Syz += cy * cz * wl;
            if (!mrt) dtau += lam[q] * g[q];
        }
        const float ux = m.ux, uy = m.uy, uz = m.uz;
        const float usq = ux * ux + uy * uy + uz * uz;
        const float S2ux = Sxx * ux + Sxy * uy + Sxz * uz;
        const float S2uy = Sxy * ux + Syy * uy + Syz * uz;
        const float S2uz = Sxz * ux + Syz * uy + Szz * uz;
        const float A1 = 1.5f * usq * S0 - 4.5f * (ux * S2ux + uy * S2uy + uz * S2uz);   // A - S0
        const float A = S0 + A1;
        const float Bx = 3.0f * Sx + 9.0f * S2ux - 3.0f * ux * S0;
        const float By = 3.0f * Sy + 9.0f * S2uy - 3.0f * uy * S0;
        const float Bz = 3.0f * Sz + 9.0f * S2uz - 3.0f * uz * S0;
        // BGK: dL/dtau = (1/tau^2) sum_q lam_q (g_q - f_eq,q).  f_eq is homogeneous of degree 1 in
        // (rho, j), so sum_q lam_q f_eq,q = rho A + j.B; in shifted form, without cancelling S0:
        //   sum_q lam_q (f_eq,q - w_q) = drho S0 + rho (A - S0 + u.B)
        if (!mrt) dtau = (dtau - (m.drho * S0 + m.rho * (A1 + ux * Bx + uy * By + uz * Bz))) * I.inv_tau2;
        const float om = mrt ? 1.0f : I.omega, om1 = 1.0f - I.omega;
        float a[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const float eq = A + (V::cx(i) ? V::cx(i) * Bx : 0.f) + (V::cy(i) ? V::cy(i) * By : 0.f) +
                             (V::cz(i) ? V::cz(i) * Bz : 0.f);
            // BGK: (1 - omega) lam + omega J^T lam;  MRT: lam - mu + J^T mu
            a[i] = mrt ? lam[i] - mu[i] + eq : om1 * lam[i] + om * eq;
        }
        if constexpr (SEED) {
            const float u[3] = {ux, uy, uz};
            float tg[3] = {0.f, 0.f, 0.f}, dldu[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int d = 0; d < D; ++d) tg[d] = target[I.poff * D + (long long)d * I.plane + n.id];
            loss_node<D>(kind, roi[I.poff + n.id] * I.loss_scale, u, tg, dldu);
            const float inv = 1.0f / m.rho;
#pragma unroll
            for (int i = 0; i < Q; ++i)
                a[i] += inv * (dldu[0] * (V::cx(i) - ux) + dldu[1] * (V::cy(i) - uy) +
                               (D == 3 ? dldu[2] * (V::cz(i) - uz) : 0.f));
        }
        if (zouhe_faces(BCX)) {
            const float jb = zouhe_adj<Q>(a, in, out, g, drho_b, BCX == BC_VELOCITY);
            if (in) grad_in[I.face_off + n.r] += (double)jb;
            else if (out) grad_out[I.face_off + n.r] += (double)jb;
        }
        const __amdgpu_buffer_rsrc_t rd = planes_rsrc(nu_out + I.st_off, Q, I.plane);
#pragma unroll
        for (int i = 0; i < Q; ++i) bstore<NT>(rd, a[i], own, plane_off(i, plane));
    }
    const double sum = block_sum(dtau, red);
    if (threadIdx.x == 0) dtau_part[t.tile] += sum;
}

// dL/dF^0 = S^T nu^1 (+ the anti-bounce-back transpose at face nodes, which
// needs F^0) in the dense layout [inst][i][nz][ny][nx], fluid nodes only (the
// caller zeroes the solid entries).
template <int Q, int BCX>
__global__ void __launch_bounds__(FT) k_adj_final(Geo G, const float *__restrict__ nu_in,
                                                  const float *__restrict__ F0, const float *__restrict__ face_in,
                                                  const float *__restrict__ face_out, float *__restrict__ dense) {
    FLUID_PROLOGUE();
    if (!n.active) return;
    const long long nn = (long long)I.nx * I.ny * I.nz;
    const long long d0 = I.node_off * Q + (long long)n.r * I.nx + n.x;
    const int plane = (int)I.plane;
    Links<Q> k;
    links<Q, BCX>(G, I, t, L, n, k);
    const __amdgpu_buffer_rsrc_t rn = planes_rsrc(nu_in + I.st_off, Q, I.plane);
    float lam[Q];
    gather_adj<Q>(rn, plane, k, lam);
    if (BCX == BC_ABB) {
        const bool in = n.x == 0, out = n.x == I.nx - 1;
        if (in || out) {
            const unsigned own = (unsigned)n.id * 4u;
            float rhoF, uF[3], nuo[Q];
            own_velocity<Q>(planes_rsrc(F0 + I.st_off, Q, I.plane), plane, own, rhoF, uF);
            face_unknown_adjoints<Q>(rn, plane, own, in, out, nuo);
            abb_adj<Q>(lam, in, out, face_density<BCX>(I, n, in, out, face_in, face_out), rhoF, uF, nuo);
        }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) dense[d0 + i * nn] = lam[i];
}

// Anti-bounce-back faces: dL/d(drho_b) of the closure that built g^1 from
// F^0 (the adjoint steps cover g^2 .. g^T).
template <int Q>
__global__ void __launch_bounds__(FT) k_abb_grad0(Geo G, const float *__restrict__ F0, const float *__restrict__ nu1,
                                                  const float *__restrict__ face_in, const float *__restrict__ face_out,
                                                  double *__restrict__ grad_in, double *__restrict__ grad_out) {
    FLUID_PROLOGUE();
    if (!n.active) return;
    const bool in = n.x == 0, out = n.x == I.nx - 1;
    if (!(in || out)) return;
    const int plane = (int)I.plane;
    const unsigned own = (unsigned)n.id * 4u;
    float rhoF, uF[3], nuo[Q], lam[Q];
    own_velocity<Q>(planes_rsrc(F0 + I.st_off, Q, I.plane), plane, own, rhoF, uF);
    face_unknown_adjoints<Q>(planes_rsrc(nu1 + I.st_off, Q, I.plane), plane, own, in, out, nuo);
#pragma unroll
    for (int i = 0; i < Q; ++i) lam[i] = 0.f;
    const float jb = abb_adj<Q>(lam, in, out, face_density<BC_ABB>(I, n, in, out, face_in, face_out), rhoF, uF, nuo);
    if (in) grad_in[I.face_off + n.r] += (double)jb;
    else grad_out[I.face_off + n.r] += (double)jb;
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
    Moments m = {0.f, 1.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const long long dn = dense_index(I, n);
    if (drho) { m.drho = drho[dn]; m.rho = 1.0f + m.drho; }
    if (u) {
        m.ux = u[dn * D];
        m.uy = u[dn * D + 1];
        if (D == 3) m.uz = u[dn * D + 2];
    }
    m.jx = m.rho * m.ux; m.jy = m.rho * m.uy; m.jz = m.rho * m.uz;
    float *__restrict__ out = F + I.st_off + n.id;
    float feq[Q];
    feq_all<Q>(m, feq);
#pragma unroll
    for (int i = 0; i < Q; ++i) out[(long long)i * I.plane] = feq[i];
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

// Residual sums of the two-step mean velocity ubar(t) = (u(t) + u(t-1)) / 2
// against its snapshot from the previous check (dense [node][D]):
//   part[2 tile]   = sum |ubar(t) - snap|^2,   part[2 tile+1] = sum |ubar(t)|^2,
// then the snapshot becomes ubar(t) (each node owns its entries).
template <int Q>
__global__ void __launch_bounds__(BLOCK) k_residual(Geo G, const float *__restrict__ Ft,
                                                    const float *__restrict__ Ft1,
                                                    float *__restrict__ snap,
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
            const float m = 0.5f * (ua[c] + ub[c]);
            const float d = m - snap[dn * D + c];
            num += d * d;
            den += m * m;
            snap[dn * D + c] = m;
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

// Bandwidth calibration: one 16-byte load and store per lane (grid-stride).
__global__ void __launch_bounds__(256) k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst, long long n) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        dst[i] = src[i];
}

__global__ void k_fill_u32(unsigned *p, long long n, unsigned v) {
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

// Fluid-tile kernels take the x boundary kind as a template parameter.
#define DISPATCH_BCX(q, bcx, CALL)                                                         \
    do {                                                                                   \
        if (q == 9) {                                                                      \
            if (bcx == BC_PRESSURE) CALL(9, BC_PRESSURE);                                  \
            else if (bcx == BC_PERIODIC) CALL(9, BC_PERIODIC);                             \
            else if (bcx == BC_WALL) CALL(9, BC_WALL);                                     \
            else if (bcx == BC_ABB) CALL(9, BC_ABB);                                       \
            else CALL(9, BC_VELOCITY);                                                     \
        } else {                                                                           \
            if (bcx == BC_PRESSURE) CALL(19, BC_PRESSURE);                                 \
            else if (bcx == BC_PERIODIC) CALL(19, BC_PERIODIC);                            \
            else if (bcx == BC_WALL) CALL(19, BC_WALL);                                    \
            else if (bcx == BC_ABB) CALL(19, BC_ABB);                                      \
            else CALL(19, BC_VELOCITY);                                                    \
        }                                                                                  \
    } while (0)

hipError_t launch_step(int q, const Geo &G, const float *src, float *dst, const float *fin,
                       const float *fout, bool tape, hipStream_t s) {
    if (G.n_ftiles == 0) return hipSuccess;
    // beyond the Infinity Cache every step streams, and D3Q19 gathers read
    // non-temporal too (D2Q9 ones do not: other blocks reread their
    // neighbouring rows' lines); a step into the tape streams its stores
    const int ntm = G.nt ? (q == 19 ? 2 : 1) : (tape ? 1 : 0);
#define CALL(Q, B)                                                                                 \
    do {                                                                                           \
        if (ntm == 2) hipLaunchKernelGGL((k_step<Q, B, 2>), fgrid_of(G), dim3(FT), 0, s, G, src, dst, fin, fout); \
        else if (ntm == 1) hipLaunchKernelGGL((k_step<Q, B, 1>), fgrid_of(G), dim3(FT), 0, s, G, src, dst, fin, fout); \
        else hipLaunchKernelGGL((k_step<Q, B, 0>), fgrid_of(G), dim3(FT), 0, s, G, src, dst, fin, fout); \
    } while (0)
    DISPATCH_BCX(q, G.bcx, CALL);
#undef CALL
    return hipGetLastError();
}

hipError_t launch_compare(int q, const Geo &G, const float *a, const float *b, unsigned *flag, hipStream_t s) {
    if (G.n_ftiles == 0) return hipSuccess;
    if (q == 9) hipLaunchKernelGGL(k_compare<9>, fgrid_of(G), dim3(FT), 0, s, G, a, b, flag);
    else hipLaunchKernelGGL(k_compare<19>, fgrid_of(G), dim3(FT), 0, s, G, a, b, flag);
    return hipGetLastError();
}

hipError_t launch_loss(int q, const Geo &G, const float *F, const float *roi, const float *target,
                       int kind, double *part, int acc, hipStream_t s) {
    if (q == 9) hipLaunchKernelGGL(k_loss<9>, grid_of(G), dim3(BLOCK), 0, s, G, F, roi, target, kind, part, acc);
    else hipLaunchKernelGGL(k_loss<19>, grid_of(G), dim3(BLOCK), 0, s, G, F, roi, target, kind, part, acc);
    return hipGetLastError();
}

hipError_t launch_adj_seed(int q, const Geo &G, const float *Fprev, float *nu_out, const float *fin,
                           const float *fout, double *gin, double *gout, const float *roi,
                           const float *target, int kind, const float *seed, hipStream_t s) {
    if (G.n_ftiles == 0) return hipSuccess;
#define CALL(Q, B)                                                                                 \
    hipLaunchKernelGGL((k_adj_seed<Q, B>), fgrid_of(G), dim3(FT), 0, s, G, Fprev, nu_out, fin, fout, gin, gout, \
                       roi, target, kind, seed)
    DISPATCH_BCX(q, G.bcx, CALL);
#undef CALL
    return hipGetLastError();
}

hipError_t launch_adj_step(int q, const Geo &G, const float *Fprev, const float *nu_in, float *nu_out,
                           const float *fin, const float *fout, double *gin, double *gout,
                           double *dtau_part, const float *roi, const float *target, int kind, hipStream_t s) {
    if (G.n_ftiles == 0) return hipSuccess;
#define CALL(Q, B)                                                                                 \
    do {                                                                                           \
        if (target)                                                                                \
            hipLaunchKernelGGL((k_adj_step<Q, B, true, false>), fgrid_of(G), dim3(FT), 0, s, G, Fprev, nu_in, \
                               nu_out, fin, fout, gin, gout, dtau_part, roi, target, kind);         \
        else if (G.nt)                                                                             \
            hipLaunchKernelGGL((k_adj_step<Q, B, false, true>), fgrid_of(G), dim3(FT), 0, s, G, Fprev, nu_in, \
                               nu_out, fin, fout, gin, gout, dtau_part, roi, target, kind);         \
        else                                                                                       \
            hipLaunchKernelGGL((k_adj_step<Q, B, false, false>), fgrid_of(G), dim3(FT), 0, s, G, Fprev, nu_in, \
                               nu_out, fin, fout, gin, gout, dtau_part, roi, target, kind);         \
    } while (0)
    DISPATCH_BCX(q, G.bcx, CALL);
#undef CALL
    return hipGetLastError();
}

hipError_t launch_adj_final(int q, const Geo &G, const float *nu_in, const float *F0, const float *fin,
                            const float *fout, float *dense, long long n_dense, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n_dense + 255) / 256)), dim3(256), 0, s, dense, n_dense, 0.f);
    if (G.n_ftiles == 0) return hipGetLastError();
#define CALL(Q, B) hipLaunchKernelGGL((k_adj_final<Q, B>), fgrid_of(G), dim3(FT), 0, s, G, nu_in, F0, fin, fout, dense)
    DISPATCH_BCX(q, G.bcx, CALL);
#undef CALL
    return hipGetLastError();
}

hipError_t launch_abb_grad0(int q, const Geo &G, const float *F0, const float *nu1, const float *fin,
                            const float *fout, double *gin, double *gout, hipStream_t s) {
    if (G.n_ftiles == 0) return hipSuccess;
    if (q == 9) hipLaunchKernelGGL(k_abb_grad0<9>, fgrid_of(G), dim3(FT), 0, s, G, F0, nu1, fin, fout, gin, gout);
    else hipLaunchKernelGGL(k_abb_grad0<19>, fgrid_of(G), dim3(FT), 0, s, G, F0, nu1, fin, fout, gin, gout);
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

hipError_t launch_residual(int q, const Geo &G, const float *Ft, const float *Ft1, float *snap,
                           double *part, hipStream_t s) {
    if (q == 9) hipLaunchKernelGGL(k_residual<9>, grid_of(G), dim3(BLOCK), 0, s, G, Ft, Ft1, snap, part);
    else hipLaunchKernelGGL(k_residual<19>, grid_of(G), dim3(BLOCK), 0, s, G, Ft, Ft1, snap, part);
    return hipGetLastError();
}

hipError_t launch_reduce(const InstDev *inst, int n_inst, const double *part, int stride, int fluid,
                         double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(n_inst), dim3(256), 0, s, inst, part, stride, fluid, out);
    return hipGetLastError();
}

hipError_t launch_copy16(const void *src, void *dst, long long n16, hipStream_t s) {
    if (n16 <= 0) return hipSuccess;
    const long long blocks = std::min<long long>((n16 + 255) / 256, 1LL << 20);
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (const uint4 *)src, (uint4 *)dst, n16);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned *p, long long n, unsigned v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, long long n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace lbm
