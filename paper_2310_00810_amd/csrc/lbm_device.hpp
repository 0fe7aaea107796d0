// Device-side definitions of the MI355X lattice Boltzmann kernels: velocity
// sets, per-instance descriptors, tile mapping and the fused pull gather.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

enum { BC_PRESSURE = 0, BC_PERIODIC = 1, BC_WALL = 2 };
enum { LOSS_VEC = 0, LOSS_NORM = 1 };

constexpr int TILE_X = 64;       // one wavefront spans 64 consecutive x
constexpr int TILE_Y = 4;        // four wavefronts per block, one row each
constexpr int BLOCK = TILE_X * TILE_Y;

// ---------------------------------------------------------------------------
// Velocity sets (D2Q9, D3Q19) in the ABI ordering.  Weights: rest 4/9, axis
// 1/9, diagonal 1/36 (D2Q9); rest 1/3, axis 1/18, face diagonal 1/36 (D3Q19).
// The functions fold to constants inside fully unrolled loops.
// ---------------------------------------------------------------------------
template <int Q> struct Vel;

template <> struct Vel<9> {
    static constexpr int D = 2;
    __host__ __device__ static constexpr int cx(int i) {
        return (i == 1 || i == 5 || i == 8) ? 1 : (i == 3 || i == 6 || i == 7) ? -1 : 0;
    }
    __host__ __device__ static constexpr int cy(int i) {
        return (i == 2 || i == 5 || i == 6) ? 1 : (i == 4 || i == 7 || i == 8) ? -1 : 0;
    }
    __host__ __device__ static constexpr int cz(int) { return 0; }
    __host__ __device__ static constexpr float w(int i) {
        return i == 0 ? 4.0f / 9.0f : (i <= 4 ? 1.0f / 9.0f : 1.0f / 36.0f);
    }
    __host__ __device__ static constexpr int opp(int i) {
        return i == 0 ? 0 : (i <= 4 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5);
    }
};

template <> struct Vel<19> {
    static constexpr int D = 3;
    // rest; +x -x +y -y +z -z; (1,1,0)(-1,-1,0)(1,-1,0)(-1,1,0);
    // (1,0,1)(-1,0,-1)(1,0,-1)(-1,0,1); (0,1,1)(0,-1,-1)(0,1,-1)(0,-1,1)
    __host__ __device__ static constexpr int cx(int i) {
        return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
             : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
    }
    __host__ __device__ static constexpr int cy(int i) {
        return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
             : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
    }
    __host__ __device__ static constexpr int cz(int i) {
        return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
             : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
    }
    __host__ __device__ static constexpr float w(int i) {
        return i == 0 ? 1.0f / 3.0f : (i <= 6 ? 1.0f / 18.0f : 1.0f / 36.0f);
    }
    // pairs (1,2) (3,4) ... (17,18) are opposite
    __host__ __device__ static constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
};

// ---------------------------------------------------------------------------
// Per-instance descriptor (device copy in the workspace).
// A state buffer holds, per instance, Q planes of [nz][ny][pitch] floats of
// shifted populations f_i - w_i starting at st_off.  Masks are one bit per
// node, rows of `words` 32-bit words.  Face arrays are [nz][ny].
// ---------------------------------------------------------------------------
struct InstDev {
    int nx, ny, nz, pitch;
    int tiles_x, tiles_y, tile_begin, n_tiles;
    long long poff;        // pitched-node offset of the instance (per-node arrays)
    long long st_off;      // float offset of the instance in a state buffer = Q * poff
    long long plane;       // nz * ny * pitch
    long long node_off;    // dense node offset (ABI arrays)
    long long mask_off;    // word offset of the mask
    long long face_off;    // offset into face arrays
    int words;             // mask words per row
    int n_fluid;
    float omega;           // 1 / tau
    float inv_tau2;        // 1 / tau^2
    float loss_scale;      // 1 or 1 / n_fluid
};

struct Geo {
    const InstDev *inst;
    int n_inst;
    int n_tiles;
    int bcx, bcy, bcz;
    const uint32_t *mask;
};

// Block index -> tile index such that the blocks the hardware places on one
// XCD (block % 8 round robin) cover a contiguous range of tiles, so that the
// neighbouring rows a tile reads are mostly served by the same L2.
__device__ inline int xcd_tile(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int xcd = b & 7, k = b >> 3;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

__device__ inline int find_inst(const InstDev *inst, int n_inst, int tile) {
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (inst[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

struct NodeRef {
    int b;                 // instance
    int tile;              // global tile id
    int x, y, z;
    bool inside;           // inside the lattice
};

__device__ inline NodeRef map_node(const Geo &G, int tile) {
    NodeRef n;
    n.tile = tile;
    n.b = G.n_inst == 1 ? 0 : find_inst(G.inst, G.n_inst, tile);
    const InstDev &I = G.inst[n.b];
    int lt = tile - I.tile_begin;
    int tx = lt % I.tiles_x;
    int rest = lt / I.tiles_x;
    int ty = rest % I.tiles_y;
    n.z = rest / I.tiles_y;
    n.x = tx * TILE_X + (threadIdx.x & (TILE_X - 1));
    n.y = ty * TILE_Y + (threadIdx.x / TILE_X);
    n.inside = n.x < I.nx && n.y < I.ny;
    return n;
}

__device__ inline bool solid_at(const uint32_t *mask, const InstDev &I, int x, int y, int z) {
    const uint32_t wv = mask[I.mask_off + ((long long)z * I.ny + y) * I.words + (x >> 5)];
    return (wv >> (x & 31)) & 1u;
}

// ---------------------------------------------------------------------------
// Pull gather of one node.  For each link i it looks at the neighbour
// s = x - SGN * c_i:
//   SGN = +1 (forward streaming): g_i(x) = buf_i(s); if s is solid or lies
//     beyond a wall, halfway bounce-back gives g_i(x) = buf_opp(i)(x); if s
//     lies beyond a pressure face, the link is a Zou-He unknown and g_i is
//     left to the boundary closure (set to 0 here).
//   SGN = -1 (transpose of streaming, adjoint): the same rule on the mirrored
//     link: a link that leaves through a pressure face carries no adjoint (0).
// Bit i of the returned mask marks the pressure-face links.
// ---------------------------------------------------------------------------
template <int Q, int SGN>
__device__ inline uint32_t gather(const Geo &G, const InstDev &I, const float *__restrict__ buf,
                                  int x, int y, int z, float (&g)[Q]) {
    using V = Vel<Q>;
    const long long base = I.st_off + ((long long)z * I.ny + y) * I.pitch + x;
    uint32_t open = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int dx = -SGN * V::cx(i), dy = -SGN * V::cy(i), dz = -SGN * V::cz(i);
        int sx = x + dx, sy = y + dy, sz = z + dz;
        bool out_p = false, out_w = false;
        if (dx != 0 && (sx < 0 || sx >= I.nx)) {
            if (G.bcx == BC_PERIODIC) sx = sx < 0 ? sx + I.nx : sx - I.nx;
            else if (G.bcx == BC_PRESSURE) out_p = true;
            else out_w = true;
        }
        if (dy != 0 && (sy < 0 || sy >= I.ny)) {
            if (G.bcy == BC_PERIODIC) sy = sy < 0 ? sy + I.ny : sy - I.ny;
            else out_w = true;
        }
        if (dz != 0 && (sz < 0 || sz >= I.nz)) {
            if (G.bcz == BC_PERIODIC) sz = sz < 0 ? sz + I.nz : sz - I.nz;
            else out_w = true;
        }
        long long off;
        if (out_p) {
            off = base + (long long)i * I.plane;             // not used
            open |= 1u << i;
        } else if (out_w || (i != 0 && solid_at(G.mask, I, sx, sy, sz))) {
            off = base + (long long)V::opp(i) * I.plane;     // bounce-back
        } else {
            off = I.st_off + (long long)i * I.plane + ((long long)sz * I.ny + sy) * I.pitch + sx;
        }
        const float v = buf[off];
        g[i] = out_p ? 0.0f : v;
    }
    return open;
}

// Zou-He closure of the unknown populations at a face node (shifted form:
// with populations f - w the known sum K and the rule are unchanged except
// that the imposed density enters as a deviation).  s = +1 at the inlet
// (unknowns c_x = +1), s = -1 at the outlet.
template <int Q>
__device__ inline void zouhe(float (&g)[Q], int s, float drho_b) {
    using V = Vel<Q>;
    float K = 0.f, Ny = 0.f, Nz = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (V::cx(i) == 0) {
            K += g[i];
            Ny += 0.5f * V::cy(i) * g[i];
            Nz += 0.5f * V::cz(i) * g[i];
        } else if (V::cx(i) == -s) {
            K += 2.0f * g[i];
        }
    }
    const float J = drho_b - K;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        if (V::cx(i) == s)
            g[i] = g[V::opp(i)] + 6.0f * V::w(i) * J - V::cy(i) * Ny - V::cz(i) * Nz;
}

// Transpose of the closure above applied to an adjoint vector a (in place):
// returns dL/d(drho_b).
template <int Q>
__device__ inline float zouhe_adj(float (&a)[Q], int s) {
    using V = Vel<Q>;
    float Jb = 0.f, Nyb = 0.f, Nzb = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (V::cx(i) == s) {
            a[V::opp(i)] += a[i];
            Jb += 6.0f * V::w(i) * a[i];
            Nyb -= V::cy(i) * a[i];
            Nzb -= V::cz(i) * a[i];
            a[i] = 0.f;
        }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (V::cx(i) == 0) a[i] += -Jb + 0.5f * (V::cy(i) * Nyb + V::cz(i) * Nzb);
        else if (V::cx(i) == -s) a[i] -= 2.0f * Jb;
    }
    return Jb;
}

struct Moments {
    float drho, rho, ux, uy, uz;
};

template <int Q>
__device__ inline Moments moments(const float (&g)[Q]) {
    using V = Vel<Q>;
    float d = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        d += g[i];
        if (V::cx(i)) jx += V::cx(i) * g[i];
        if (V::cy(i)) jy += V::cy(i) * g[i];
        if (V::cz(i)) jz += V::cz(i) * g[i];
    }
    Moments m;
    m.drho = d;
    m.rho = 1.0f + d;
    const float inv = 1.0f / m.rho;
    m.ux = jx * inv; m.uy = jy * inv; m.uz = jz * inv;
    return m;
}

// Shifted equilibrium f_eq,i - w_i = w_i (drho + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)).
template <int Q>
__device__ inline float feq_shifted(int i, const Moments &m) {
    using V = Vel<Q>;
    const float cu = V::cx(i) * m.ux + V::cy(i) * m.uy + V::cz(i) * m.uz;
    const float usq = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
    return V::w(i) * (m.drho + m.rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * usq));
}

// Wavefront (64-lane) sum.
__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block (256-thread) sum into double; the result is valid in thread 0.
__device__ inline double block_sum(float v, double *lds4) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) lds4[threadIdx.x >> 6] = (double)v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
    __syncthreads();
    return s;
}

}  // namespace lbm
