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
//
// Populations are stored for fluid nodes only, numbered in (z, y, x) order:
// a state buffer holds, per instance, Q planes of `plane` floats (plane >= the
// number of fluid nodes) of shifted populations f_i - w_i, starting at st_off.
// The row-word table has one entry per 32-node word of every x row:
//   .x = solid bits of the word (bit b = node x = 32 w + b; bits past nx set),
//   .y = fluid id of the first fluid node at or after the word's first node,
// so the id of fluid node x is .y + popcount(~.x & ((1 << (x & 31)) - 1)).
// Face arrays are [nz][ny].
// ---------------------------------------------------------------------------
struct InstDev {
    int nx, ny, nz, words;
    int tiles_x, tiles_y, tile_begin, n_tiles;   // dense 64 x 4 node tiles
    int ftile_begin, n_ftiles;                   // fluid tiles of FT nodes
    long long plane;       // floats per population plane (fluid nodes, padded)
    long long poff;        // offset of the instance in per-node (fluid) arrays
    long long st_off;      // float offset of the instance in a state buffer = Q * poff
    long long node_off;    // dense node offset (ABI arrays)
    long long rw_off;      // offset of the instance's row-word table
    long long face_off;    // offset into face arrays
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
    const uint2 *rw;       // row-word tables
    int n_ftiles;
    const int2 *fblk;      // per fluid tile: instance-local row words {w0, w1}
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

__device__ inline uint2 row_word(const Geo &G, const InstDev &I, int x, int y, int z) {
    return G.rw[I.rw_off + ((long long)z * I.ny + y) * I.words + (x >> 5)];
}
__device__ inline bool solid_bit(uint2 w, int x) { return (w.x >> (x & 31)) & 1u; }
__device__ inline int fluid_id(uint2 w, int x) { return (int)w.y + __popc(~w.x & ((1u << (x & 31)) - 1u)); }

struct NodeRef {
    int b;                 // instance
    int tile;              // global tile id
    int x, y, z;
    bool inside;           // inside the lattice
    bool fluid;            // inside and fluid
    int id;                // fluid id (valid when fluid)
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
    n.fluid = false;
    n.id = 0;
    if (n.inside) {
        const uint2 w = row_word(G, I, n.x, n.y, n.z);
        n.fluid = !solid_bit(w, n.x);
        n.id = fluid_id(w, n.x);
    }
    return n;
}

// Dense (ABI) index of a node.
__device__ inline long long dense_index(const InstDev &I, const NodeRef &n) {
    return I.node_off + ((long long)n.z * I.ny + n.y) * I.nx + n.x;
}

// ---------------------------------------------------------------------------
// Fluid tiles.  The stepping kernels give every lane one fluid node: block t
// of an instance takes the fluid ids [FT t, FT t + FT), so all lanes of a
// wavefront do useful work at any porosity and every store of a block is one
// contiguous run per population plane.  The ids of a block lie in a
// contiguous range of row words [w0, w1] (fblk, built at init), i.e. in rows
// r0 .. r1 (r = z ny + y).  Their neighbours lie in rows r - 1 .. r + 1 of
// the planes z - 1, z, z + 1, which are the row windows
//   [r0 - 1 + dz ny, r1 + 1 + dz ny]  (mod ny nz)
// of the linear row order.  A block stages these windows in LDS when they
// fit (NBW words); a y link that wraps around a periodic y axis leaves the
// window and reads its row word from global memory, as does every link of a
// block whose windows do not fit.  The z wrap of a periodic z axis is exact
// in the linear order because y + dy stays inside [0, ny) there.
// ---------------------------------------------------------------------------
constexpr int FT = 256;          // fluid nodes (threads) per block
constexpr int NBW = 1024;        // staged row words per block (8 KB)

struct FTile {
    int b;                 // instance
    int tile;              // global fluid-tile index
    int id0;               // first fluid id of the block
    int w0, w1;            // instance-local row words holding ids id0 .. id0 + FT - 1
    int r0;                // row of w0
    int rows;              // rows per staged window: r1 - r0 + 3
    int cdz;               // window of the block's own plane (1 in 3D, 0 in 2D)
    bool staged;
};

template <int D>
__device__ inline FTile fluid_tile(const Geo &G, int tile) {
    FTile t;
    t.tile = tile;
    int lo = 0;
    if (G.n_inst > 1) {
        int hi = G.n_inst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (G.inst[mid].ftile_begin <= tile) lo = mid; else hi = mid - 1;
        }
    }
    t.b = lo;
    const InstDev &I = G.inst[lo];
    t.id0 = (tile - I.ftile_begin) * FT;
    const int2 wr = G.fblk[tile];
    t.w0 = wr.x;
    t.w1 = wr.y;
    t.r0 = t.w0 / I.words;
    t.rows = t.w1 / I.words - t.r0 + 3;
    t.cdz = D == 3 ? 1 : 0;
    t.staged = (D == 3 ? 3 : 1) * t.rows * I.words <= NBW;
    return t;
}

template <int D>
__device__ inline void stage_windows(const Geo &G, const InstDev &I, const FTile &t, uint2 *lds) {
    const int per = t.rows * I.words;
    const int n = (D == 3 ? 3 : 1) * per;
    const int R = I.ny * I.nz;
    for (int e = threadIdx.x; e < n; e += FT) {
        const int win = e / per, rem = e - win * per;
        const int j = rem / I.words, wi = rem - j * I.words;
        int rr = (t.r0 - 1 + j + (win - t.cdz) * I.ny) % R;
        rr += rr < 0 ? R : 0;
        lds[e] = G.rw[I.rw_off + (long long)rr * I.words + wi];
    }
}

// LDS view of the staged row words.  Reading through an address-space-3
// pointer keeps these reads ds_read instructions: with a generic pointer the
// compiler may merge an LDS read and a global read into one flat load.
typedef __attribute__((address_space(3))) const unsigned long long lds_u64;
__device__ inline uint2 lds_read(const uint2 *lds, unsigned e) {
    const unsigned long long v = ((lds_u64 *)lds)[e];
    return make_uint2((unsigned)v, (unsigned)(v >> 32));
}

// Position of the k-th (0-based) set bit of m (m has more than k set bits).
__device__ inline int kth_set_bit(uint32_t m, int k) {
    int pos = 0;
#pragma unroll
    for (int s = 16; s > 0; s >>= 1) {
        const int c = __popc(m & ((1u << s) - 1u));
        if (k >= c) { k -= c; m >>= s; pos += s; }
    }
    return pos;
}

struct FLane {
    int id, x, y, z, r;
    bool active;           // id < number of fluid nodes of the instance
};

// The lane's fluid node: the last word of [w0, w1] whose first id is <= id
// holds it; its position in the word is the matching fluid bit.  Staged
// blocks search their LDS copy of the words, the others global memory (two
// separate loops, so that each keeps its own memory instructions).
__device__ inline FLane fluid_lane(const Geo &G, const InstDev &I, const FTile &t, const uint2 *lds) {
    FLane l;
    l.id = t.id0 + (int)threadIdx.x;
    l.active = l.id < I.n_fluid;
    l.x = l.y = l.z = l.r = 0;
    if (!l.active) return l;
    int lo = t.w0, hi = t.w1;
    uint2 w;
    if (t.staged) {
        const int base = (t.cdz * t.rows + 1) * I.words - t.r0 * I.words;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((int)lds_read(lds, base + mid).y <= l.id) lo = mid; else hi = mid - 1;
        }
        w = lds_read(lds, base + lo);
    } else {
        const uint2 *own = G.rw + I.rw_off;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((int)own[mid].y <= l.id) lo = mid; else hi = mid - 1;
        }
        w = own[lo];
    }
    const int bit = kth_set_bit(~w.x, l.id - (int)w.y);
    l.r = lo / I.words;
    l.x = (lo - l.r * I.words) * 32 + bit;
    l.y = l.r % I.ny;
    l.z = l.r / I.ny;
    return l;
}

enum { NB_WALL = -1, NB_OPEN = -2 };

// A coordinate at most one step outside [0, n) wrapped back inside.
__device__ inline int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// For every link k: the fluid id of node x + c_k, NB_WALL if that node is
// solid or lies beyond a wall (halfway bounce-back), NB_OPEN if it lies
// beyond a pressure face.  nb[0] is the node's own id.  A straight-line pass
// reads every link's row word from the staged windows (index clamped into
// the LDS array, so the read is always legal); lanes with links that wrap a
// periodic y axis, and every lane of an unstaged block, then redo those
// links from the global row words.  Coordinates are wrapped for indexing
// only: the boundary kind decides what the link means.
template <int Q>
__device__ inline void neighbours(const Geo &G, const InstDev &I, const FTile &t, const uint2 *lds,
                                  const FLane &l, int (&nb)[Q]) {
    using V = Vel<Q>;
    nb[0] = l.id;
    const int W = I.words;
    const int lrow = (t.cdz * t.rows + (l.r - t.r0 + 1)) * W;
    const int wstep = t.rows * W;
#pragma unroll
    for (int k = 1; k < Q; ++k) {
        const int dx = V::cx(k), dy = V::cy(k), dz = V::cz(k);
        const int xr = l.x + dx, yr = l.y + dy, zr = l.z + dz;
        const bool xout = dx != 0 && (xr < 0 || xr >= I.nx);
        const bool yout = dy != 0 && (yr < 0 || yr >= I.ny);
        const bool zout = dz != 0 && (zr < 0 || zr >= I.nz);
        const int xs = dx != 0 ? wrap1(xr, I.nx) : xr;
        const bool open = xout && G.bcx == BC_PRESSURE;
        const bool wall = (xout && G.bcx == BC_WALL) || (yout && G.bcy != BC_PERIODIC) ||
                          (zout && G.bcz != BC_PERIODIC);
        const unsigned e = (unsigned)(lrow + dz * wstep + dy * W + (xs >> 5));
        const uint2 w = lds_read(lds, e < (unsigned)NBW ? e : 0u);
        const int id = solid_bit(w, xs) ? NB_WALL : fluid_id(w, xs);
        nb[k] = open ? NB_OPEN : (wall ? NB_WALL : id);
    }
    const bool yedge = G.bcy == BC_PERIODIC && (l.y == 0 || l.y == I.ny - 1);
    if (!t.staged || yedge) {
#pragma unroll
        for (int k = 1; k < Q; ++k) {
            const int dx = V::cx(k), dy = V::cy(k), dz = V::cz(k);
            const int xr = l.x + dx, yr = l.y + dy, zr = l.z + dz;
            const bool yout = dy != 0 && (yr < 0 || yr >= I.ny);
            if (nb[k] == NB_OPEN || (t.staged && !yout)) continue;
            if ((yout && G.bcy != BC_PERIODIC) || (dz != 0 && (zr < 0 || zr >= I.nz) && G.bcz != BC_PERIODIC) ||
                (dx != 0 && (xr < 0 || xr >= I.nx) && G.bcx == BC_WALL))
                continue;   // beyond a wall: already NB_WALL
            const int xs = dx != 0 ? wrap1(xr, I.nx) : xr;
            const int ys = dy != 0 ? wrap1(yr, I.ny) : yr, zs = dz != 0 ? wrap1(zr, I.nz) : zr;
            const uint2 w = G.rw[I.rw_off + ((long long)zs * I.ny + ys) * W + (xs >> 5)];
            nb[k] = solid_bit(w, xs) ? NB_WALL : fluid_id(w, xs);
        }
    }
}

// Pull gather over a precomputed neighbourhood.  Link i reads the node
// x - SGN c_i = x + c_k with k = opp(i) for SGN = +1 (forward streaming) and
// k = i for SGN = -1 (transpose of streaming):
//   fluid neighbour -> buf_i(neighbour);
//   solid / wall    -> buf_opp(i)(x)   (halfway bounce-back);
//   pressure face   -> 0 (forward: Zou-He unknown, filled by the closure;
//                     adjoint: the link leaves the lattice).
template <int Q, int SGN>
__device__ inline void gather(const float *__restrict__ base, int plane, int id, const int (&nb)[Q], float (&g)[Q]) {
    using V = Vel<Q>;
    g[0] = base[id];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int j = nb[SGN > 0 ? V::opp(i) : i];
        const int off = j >= 0 ? i * plane + j : (j == NB_WALL ? V::opp(i) * plane + id : i * plane + id);
        const float v = base[off];
        g[i] = j == NB_OPEN ? 0.0f : v;
    }
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

// Block (4 wavefronts) sum into double; the result is valid in thread 0.
__device__ inline double block_sum(float v, double *lds4) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) lds4[threadIdx.x >> 6] = (double)v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
    __syncthreads();
    return s;
}
static_assert(BLOCK == 256 && FT == 256, "block_sum assumes four wavefronts");

}  // namespace lbm
