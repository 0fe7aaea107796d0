// Device-side definitions of the MI355X lattice Boltzmann kernels: velocity
// sets, per-instance descriptors, fluid-tile mapping, links, the pull
// gathers and the Zou-He closure.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

enum { BC_PRESSURE = 0, BC_PERIODIC = 1, BC_WALL = 2, BC_ABB = 3, BC_VELOCITY = 4 };
enum { COLL_BGK = 0, COLL_MRT = 1 };
// x boundary kinds with inlet / outlet faces: Zou-He densities (PRESSURE),
// anti-bounce-back densities (ABB), Zou-He velocity inlet + density outlet
// (VELOCITY)
__host__ __device__ constexpr bool density_faces(int bcx) {
    return bcx == BC_PRESSURE || bcx == BC_ABB || bcx == BC_VELOCITY;
}
// x kinds whose faces use the Zou-He closure
__host__ __device__ constexpr bool zouhe_faces(int bcx) { return bcx == BC_PRESSURE || bcx == BC_VELOCITY; }
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
    // 4/9, 1/9, 1/36 as FP32 values whose exact sum over the directions is
    // 1 (each within 1.2e-7 of the rational weight): with nearest-rounded
    // weights the sum is 1 + 1.5e-8, and every collision would scale the
    // mass deviation by omega times that, a drift that grows with the steps.
    __host__ __device__ static constexpr float w(int i) {
        return i == 0 ? 0x1.c71c74p-2f : (i <= 4 ? 0x1.c71c70p-4f : 0x1.c71c70p-6f);
    }
    __host__ __device__ static constexpr int opp(int i) {
        return i == 0 ? 0 : (i <= 4 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5);
    }
    // 3 w_i (coefficient of rho c.u in f_eq) and 6 w_i (of J in the Zou-He
    // unknowns) as FP32 constants whose sums are exact: 2 (a_axis + 2 a_diag)
    // = 1 and zj_axis + 2 zj_diag = 1 (1/3 and 1/12, 2/3 and 1/6 to 1e-7).
    __host__ __device__ static constexpr float a(int i) {
        return i == 0 ? 0.0f : (i <= 4 ? 0x1.555556p-2f : 0x1.555554p-4f);
    }
    __host__ __device__ static constexpr float zj(int i) {
        return i == 0 ? 0.0f : (i <= 4 ? 0x1.555556p-1f : 0x1.555554p-3f);
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
    // 1/3, 1/18, 1/36 as FP32 values whose exact sum over the directions is 1
    // (within 1.2e-7 of the rational weights; see Vel<9>::w).
    __host__ __device__ static constexpr float w(int i) {
        return i == 0 ? 0x1.555558p-2f : (i <= 6 ? 0x1.c71c70p-5f : 0x1.c71c70p-6f);
    }
    // pairs (1,2) (3,4) ... (17,18) are opposite
    __host__ __device__ static constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
    // 3 w_i and 6 w_i as FP32 constants with exact sums: 2 (a_axis + 4 a_diag)
    // = 1 and zj_axis + 4 zj_diag = 1 (1/6 and 1/12, 1/3 and 1/6 to 1e-7).
    __host__ __device__ static constexpr float a(int i) {
        return i == 0 ? 0.0f : (i <= 6 ? 0x1.555554p-3f : 0x1.555556p-4f);
    }
    __host__ __device__ static constexpr float zj(int i) {
        return i == 0 ? 0.0f : (i <= 6 ? 0x1.555554p-2f : 0x1.555556p-3f);
    }
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

// Per fluid tile (built at init): its instance, the instance-local row words
// holding its first and last fluid id, and their rows (r = z ny + y), so a
// block reads its place with one scalar load instead of searching the
// instance table and dividing.
struct FTileDesc {
    int w0, w1, b, r0, r1, pad0, pad1, pad2;
};

struct Geo {
    const InstDev *inst;
    int n_inst;
    int n_tiles;
    int bcx, bcy, bcz;
    const uint2 *rw;       // row-word tables
    int n_ftiles;
    const FTileDesc *fblk; // per fluid tile
    int coll;              // COLL_BGK or COLL_MRT (D2Q9)
    float mrt[9];          // MRT rates of the D2Q9 moments; stress entries unused (1/tau)
    int nt;                // step and adjoint stores non-temporal (two states exceed the Infinity Cache)
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
//   [r0 - 1 + dz ny, r1 + 1 + dz ny]        dz = -1, 0, 1 (3D), 0 (2D)
// of the linear row order.  A block stages these windows in LDS when they
// fit (NBW words).  Staging wraps a window row around a periodic z axis and
// replaces it by an all-solid word beyond a z wall, so that a lane reads the
// row word of every link from LDS without any z test: the linear order is
// exact for every neighbour with y + dy inside [0, ny).  Lanes on the first
// or last y row, and all lanes of a block whose windows do not fit, take
// their links from the global row words instead.
// ---------------------------------------------------------------------------
constexpr int FT = 256;          // fluid nodes (threads) per block
constexpr int NBW = 1024;        // staged row words per block (8 KB)
constexpr int X_BITS = 20;       // lane position word: (own row << X_BITS) | x
constexpr int SCATTER_WORDS = 64;

struct TileLds {
    uint2 word[NBW];             // staged row windows
    int pos[FT];                 // per lane: position of its fluid node
    unsigned char yedge[NBW];    // per centre-window row: first or last y row
};

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
    const FTileDesc e = G.fblk[tile];
    t.b = e.b;
    const InstDev &I = G.inst[e.b];
    t.id0 = (tile - I.ftile_begin) * FT;
    t.w0 = e.w0;
    t.w1 = e.w1;
    t.r0 = e.r0;
    t.rows = e.r1 - e.r0 + 3;
    t.cdz = D == 3 ? 1 : 0;
    t.staged = (D == 3 ? 3 : 1) * t.rows * I.words <= NBW;
    return t;
}

// floor(a / d) for 0 <= a < 2^20, given inv = 1 / d: the float estimate of
// (a + 1/2) / d is within 1/(4d) of the exact value, which lies at least
// 1/(2d) from an integer.
__device__ inline int small_div(int a, float inv) { return (int)(((float)a + 0.5f) * inv); }

// LDS reads of the staged row words go through an address-space-3 pointer:
// with a generic pointer the compiler may merge an LDS read and a global
// read into one flat load.
typedef __attribute__((address_space(3))) const unsigned long long lds_u64;
__device__ inline uint2 lds_read(const uint2 *lds, int e) {
    const unsigned long long v = ((lds_u64 *)lds)[e];
    return make_uint2((unsigned)v, (unsigned)(v >> 32));
}

template <int D>
__device__ inline void stage_windows(const Geo &G, const InstDev &I, const FTile &t, TileLds &L) {
    const int W = I.words, per = t.rows * W, n = (D == 3 ? 3 : 1) * per;
    const float inv_per = 1.0f / (float)per, inv_w = 1.0f / (float)W;
    const int R = I.ny * I.nz;
    const bool zwall = D == 3 && G.bcz != BC_PERIODIC;
    for (int e = threadIdx.x; e < n; e += FT) {
        const int win = D == 3 ? small_div(e, inv_per) : 0;
        const int rem = e - win * per;
        const int j = small_div(rem, inv_w);
        const int wi = rem - j * W;
        int rr = t.r0 - 1 + j + (win - t.cdz) * I.ny;
        const bool beyond = rr < 0 || rr >= R;
        rr += rr < 0 ? R : 0;
        rr += rr < 0 ? R : 0;
        rr -= rr >= R ? R : 0;
        rr -= rr >= R ? R : 0;
        L.word[e] = zwall && beyond ? make_uint2(0xffffffffu, 0u) : G.rw[I.rw_off + (long long)rr * W + wi];
        if (win == t.cdz && wi == 0) {
            const int y = rr % I.ny;
            L.yedge[j] = y == 0 || y == I.ny - 1;
        }
    }
}

// Every fluid node of the block's own words writes its position into the
// slot of its lane (staged blocks with at most SCATTER_WORDS own words).
__device__ inline void scatter_positions(const InstDev &I, const FTile &t, TileLds &L) {
    const int W = I.words;
    const float inv_w = 1.0f / (float)W;
    const int first = t.w0 - t.r0 * W;              // offset of w0 in its row
    const int obase = (t.cdz * t.rows + 1) * W;     // LDS index of the first own row
    const int nslots = (t.w1 - t.w0 + 1) * 32;
    for (int s = threadIdx.x; s < nslots; s += FT) {
        const int ow = first + (s >> 5), bit = s & 31;
        const uint2 v = lds_read(L.word, obase + ow);
        if ((v.x >> bit) & 1u) continue;
        const int k = (int)v.y + __popc(~v.x & ((1u << bit) - 1u)) - t.id0;
        if (k < 0 || k >= FT) continue;
        const int jrow = small_div(ow, inv_w);
        L.pos[k] = (jrow << X_BITS) | ((ow - jrow * W) * 32 + bit);
    }
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
    int id, x, r;          // fluid id, x, row z ny + y
    int jc;                // centre-window row of the node (staged blocks)
    bool active;           // id < number of fluid nodes of the instance
    bool yedge;            // node on the first or last y row
};

// The lane's fluid node.  Staged blocks with few own words read it from the
// scattered positions; the others search the last word of [w0, w1] whose
// first id is <= id (LDS copy or global words) and take the matching bit.
__device__ inline FLane fluid_lane(const Geo &G, const InstDev &I, const FTile &t, TileLds &L) {
    FLane l;
    l.id = t.id0 + (int)threadIdx.x;
    l.active = l.id < I.n_fluid;
    l.x = l.r = 0;
    l.jc = 1;
    l.yedge = false;
    if (t.staged && t.w1 - t.w0 < SCATTER_WORDS) {
        scatter_positions(I, t, L);
        __syncthreads();
        if (!l.active) return l;
        const int p = L.pos[threadIdx.x];
        const int jrow = p >> X_BITS;
        l.x = p & ((1 << X_BITS) - 1);
        l.r = t.r0 + jrow;
        l.jc = jrow + 1;
        l.yedge = L.yedge[l.jc];
        return l;
    }
    if (!l.active) return l;
    int lo = t.w0, hi = t.w1;
    uint2 w;
    if (t.staged) {
        const int base = (t.cdz * t.rows + 1) * I.words - t.r0 * I.words;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((int)lds_read(L.word, base + mid).y <= l.id) lo = mid; else hi = mid - 1;
        }
        w = lds_read(L.word, base + lo);
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
    l.jc = l.r - t.r0 + 1;
    const int y = l.r % I.ny;
    l.yedge = y == 0 || y == I.ny - 1;
    return l;
}

// ---------------------------------------------------------------------------
// Links.  For every link k: wall[k] if x + c_k is solid or lies beyond a wall
// (halfway bounce-back), open[k] if it lies beyond a pressure face (Zou-He
// unknown in the forward pass, a link that leaves the lattice in the
// adjoint), else fid[k] = its fluid id.  The x boundary kind is a template
// parameter; y and z kinds are read at run time (staging already applied z).
// open[k] is set for both kinds of density face.
// ---------------------------------------------------------------------------
template <int Q>
struct Links {
    int id;
    int fid[Q];
    bool wall[Q];
    bool open[Q];
};

// A coordinate at most one step outside [0, n) wrapped back inside.
__device__ inline int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

template <int Q, int BCX>
__device__ inline void links_staged(const InstDev &I, const FTile &t, const TileLds &L, const FLane &l,
                                    Links<Q> &k) {
    using V = Vel<Q>;
    const int W = I.words, per = t.rows * W;
    const int lrow = (t.cdz * t.rows + l.jc) * W;
    const bool lo_edge = l.x == 0, hi_edge = l.x == I.nx - 1;
    const int xm = lo_edge ? I.nx - 1 : l.x - 1, xp = hi_edge ? 0 : l.x + 1;
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        const int dx = V::cx(q), dy = V::cy(q), dz = V::cz(q);
        const int xs = dx < 0 ? xm : (dx > 0 ? xp : l.x);
        const uint2 w = lds_read(L.word, lrow + dz * per + dy * W + (xs >> 5));
        const bool out = BCX != BC_PERIODIC && dx != 0 && (dx < 0 ? lo_edge : hi_edge);
        k.fid[q] = fluid_id(w, xs);
        k.wall[q] = solid_bit(w, xs) || (BCX == BC_WALL && out);
        k.open[q] = density_faces(BCX) && out;
    }
}

template <int Q, int BCX>
__device__ inline void links_global(const Geo &G, const InstDev &I, const FLane &l, Links<Q> &k) {
    using V = Vel<Q>;
    const int y = l.r % I.ny, z = l.r / I.ny;
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        const int dx = V::cx(q), dy = V::cy(q), dz = V::cz(q);
        const int xr = l.x + dx, yr = y + dy, zr = z + dz;
        const bool xout = dx != 0 && (xr < 0 || xr >= I.nx);
        const bool yout = dy != 0 && (yr < 0 || yr >= I.ny);
        const bool zout = dz != 0 && (zr < 0 || zr >= I.nz);
        const int xs = dx != 0 ? wrap1(xr, I.nx) : xr;
        const int ys = dy != 0 ? wrap1(yr, I.ny) : yr, zs = dz != 0 ? wrap1(zr, I.nz) : zr;
        const uint2 w = G.rw[I.rw_off + ((long long)zs * I.ny + ys) * I.words + (xs >> 5)];
        const bool beyond = (BCX == BC_WALL && xout) || (yout && G.bcy != BC_PERIODIC) ||
                            (zout && G.bcz != BC_PERIODIC);
        k.fid[q] = fluid_id(w, xs);
        k.wall[q] = solid_bit(w, xs) || beyond;
        k.open[q] = density_faces(BCX) && xout;
    }
}

template <int Q, int BCX>
__device__ inline void links(const Geo &G, const InstDev &I, const FTile &t, const TileLds &L, const FLane &l,
                             Links<Q> &k) {
    k.id = l.id;
    if (t.staged) links_staged<Q, BCX>(I, t, L, l, k);
    if (!t.staged || l.yedge) links_global<Q, BCX>(G, I, l, k);
}

// ---------------------------------------------------------------------------
// Gathers through buffer loads: an offset past the end of the instance's
// planes (OOB) reads 0 by the hardware range check, which is what an open
// link contributes.  The planes of an accepted instance span a multiple of
// 256 B below 4 GiB, i.e. at most 2^32 - 256 B, so OOB = 2^32 - 256 lies past
// the range of every accepted size.
// ---------------------------------------------------------------------------
constexpr unsigned OOB = 0xFFFFFF00u;

// Byte range and offsets of one instance's population planes are 32-bit
// unsigned (the host rejects instances whose Q planes reach 4 GiB), so they
// are formed in unsigned arithmetic and passed on bit for bit.
__device__ inline __amdgpu_buffer_rsrc_t planes_rsrc(const float *base, int q, long long plane) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)(unsigned)(q * plane * 4), 0x00020000);
}
__device__ inline int plane_off(int i, int plane) { return (int)((unsigned)i * (unsigned)plane * 4u); }
// NT: the load carries the non-temporal cache policy (see bstore).
template <bool NT = false>
__device__ inline float bload(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, NT ? 2 : 0));
}
// NT: the store carries the non-temporal cache policy (cache-policy bit 1,
// "nt" on gfx950), for states whose ping-pong pair does not fit the
// Infinity Cache, where keeping the written lines only evicts lines the
// next step reads.
template <bool NT = false>
__device__ inline void bstore(__amdgpu_buffer_rsrc_t r, float v, unsigned voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, NT ? 2 : 0);
}
__device__ inline unsigned bload_bits(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
}

// Streaming pull: g_i(x) = F_i(x - c_i); with k = opp(i), x - c_i = x + c_k.
//   fluid -> F_i(x + c_k);  wall -> F_k(x) (bounce-back);
//   open  -> 0 for Zou-He faces (the closure fills the slot), and F_k(x), the
//            population that left through the face, for anti-bounce-back
//            faces (the closure negates and corrects it).
template <int Q, int BCX, bool NTL = false>
__device__ inline void gather_fwd(__amdgpu_buffer_rsrc_t r, int plane, const Links<Q> &k, float (&g)[Q]) {
    using V = Vel<Q>;
    const unsigned own = (unsigned)k.id * 4u;
    g[0] = bload<NTL>(r, own);
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        const int i = V::opp(q);
        const bool back = BCX == BC_ABB && V::cx(q) != 0 ? (k.wall[q] || k.open[q]) : k.wall[q];
        unsigned off = back ? own + (unsigned)(q * plane) * 4u : (unsigned)(i * plane + k.fid[q]) * 4u;
        if (zouhe_faces(BCX) && V::cx(q) != 0) off = k.open[q] ? OOB : off;
        g[i] = bload<NTL>(r, off);
    }
}

// Transpose of streaming (pull of nu from x + c_k): lam_k(x) =
//   fluid -> nu_k(x + c_k);  wall -> nu_opp(k)(x);  open -> 0.
template <int Q, bool NTL = false>
__device__ inline void gather_adj(__amdgpu_buffer_rsrc_t r, int plane, const Links<Q> &k, float (&lam)[Q]) {
    using V = Vel<Q>;
    const unsigned own = (unsigned)k.id * 4u;
    lam[0] = bload<NTL>(r, own);
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        unsigned off = k.wall[q] ? own + (unsigned)(V::opp(q) * plane) * 4u : (unsigned)(q * plane + k.fid[q]) * 4u;
        if (V::cx(q) != 0) off = k.open[q] ? OOB : off;
        lam[q] = bload<NTL>(r, off);
    }
}

// Zou-He closure of the unknown populations at a face node (shifted form:
// with populations f - w the known sum K and the rule are unchanged except
// that the imposed density enters as a deviation).  in / out select the
// inlet (unknowns c_x = +1) or outlet (c_x = -1); other nodes keep g
// exactly.  Written without branches: in a wavefront of consecutive fluid
// ids nearly every wavefront holds inlet and outlet nodes.  vin: the inlet
// imposes the normal velocity u = b instead of a density: rho = K / (1 - u)
// and J = rho - K = (Kbar + 1) u / (1 - u) (Kbar the shifted known sum).
template <int Q>
__device__ inline void zouhe(float (&g)[Q], bool in, bool out, float drho_b, bool vin = false) {
    using V = Vel<Q>;
    float K0 = 0.f, Kp = 0.f, Km = 0.f, Ny = 0.f, Nz = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (V::cx(i) == 0) {
            K0 += g[i];
            if (V::cy(i)) Ny += 0.5f * V::cy(i) * g[i];
            if (V::cz(i)) Nz += 0.5f * V::cz(i) * g[i];
        } else if (V::cx(i) > 0) {
            Kp += g[i];
        } else {
            Km += g[i];
        }
    }
    const float Kb = K0 + 2.0f * (in ? Km : Kp);
    const float J = in && vin ? (Kb + 1.0f) * drho_b / (1.0f - drho_b) : drho_b - Kb;
#pragma unroll
    for (int p = 1; p < Q; ++p) {
        if (V::cx(p) != 1) continue;
        const int m = V::opp(p);
        const float t = (V::cy(p) ? V::cy(p) * Ny : 0.f) + (V::cz(p) ? V::cz(p) * Nz : 0.f);
        const float sj = V::zj(p) * J;
        const float np = g[m] + sj - t, nm = g[p] + sj + t;
        g[p] = in ? np : g[p];
        g[m] = out ? nm : g[m];
    }
}

// Transpose of the closure above applied to an adjoint vector a (in place):
// returns dL/d(drho_b), or dL/du for a velocity inlet (0 away from the
// faces, where a is left exactly).  g: the completed populations (their
// known part gives Kbar for the velocity inlet).
template <int Q>
__device__ inline float zouhe_adj(float (&a)[Q], bool in, bool out, const float (&g)[Q], float b = 0.f,
                                  bool vin = false) {
    using V = Vel<Q>;
    float Jb = 0.f, Nyb = 0.f, Nzb = 0.f;
#pragma unroll
    for (int p = 1; p < Q; ++p) {
        if (V::cx(p) != 1) continue;
        const int m = V::opp(p);
        const float up = in ? a[p] : 0.f, um = out ? a[m] : 0.f;   // adjoints of the unknowns
        a[m] += up;
        a[p] += um;
        a[p] -= up;
        a[m] -= um;
        Jb += V::zj(p) * (up + um);
        if (V::cy(p)) Nyb -= V::cy(p) * (up - um);
        if (V::cz(p)) Nzb -= V::cz(p) * (up - um);
    }
    // dJ/dKbar: -1 for a density face, u / (1 - u) for the velocity inlet
    float dJ = -1.0f, db = 1.0f;
    if (vin && in) {
        float Kb = 0.f;
#pragma unroll
        for (int i = 0; i < Q; ++i) Kb += V::cx(i) == 0 ? g[i] : (V::cx(i) < 0 ? 2.0f * g[i] : 0.f);
        const float r = 1.0f / (1.0f - b);
        dJ = b * r;
        db = (Kb + 1.0f) * r * r;
    }
    const float Jk = dJ * Jb, Jk2 = 2.0f * Jk;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (V::cx(i) == 0) {
            a[i] += Jk + 0.5f * ((V::cy(i) ? V::cy(i) * Nyb : 0.f) + (V::cz(i) ? V::cz(i) * Nzb : 0.f));
        } else if (V::cx(i) < 0) {
            a[i] += in ? Jk2 : 0.f;
        } else {
            a[i] += out ? Jk2 : 0.f;
        }
    }
    return Jb * db;
}

struct Moments {
    float drho, rho, ux, uy, uz;
    float jx, jy, jz;      // momentum sum c g (u = j / rho)
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
    m.jx = jx; m.jy = jy; m.jz = jz;
    return m;
}

// Shifted equilibria f_eq,i - w_i = w_i (drho + rho (3 c.u + 4.5 (c.u)^2 -
// 1.5 u.u)) of all directions (Eq. 5).  The two directions of an opposite
// pair share s = w_i (drho + rho (4.5 (c.u)^2 - 1.5 u.u)) and differ in the
// sign of d = 3 w_i rho c.u = 3 w_i c.j, with 3 w_i taken from Vel::a.  The
// weights of Vel::w sum to exactly 1 and those of Vel::a give exactly j, so
// the FP32 equilibrium carries the node's mass and momentum up to unbiased
// rounding.  d is formed from the momentum sum j itself: forming it as
// rho (c.u) with u = j fl(1/rho) multiplies each node's momentum by rounding
// factors that depend only on the node's density, which over thousands of
// steps drove a systematic velocity drift (2e-4 after 8000 steps in a packed
// sphere box); from j it falls to unbiased rounding.
template <int Q>
__device__ inline void feq_all(const Moments &m, float (&feq)[Q]) {
    using V = Vel<Q>;
    const float usq15 = 1.5f * (m.ux * m.ux + m.uy * m.uy + m.uz * m.uz);
    feq[0] = V::w(0) * (m.drho - m.rho * usq15);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int o = V::opp(i);
        if (o < i) continue;
        const float cu = V::cx(i) * m.ux + V::cy(i) * m.uy + V::cz(i) * m.uz;
        const float cj = V::cx(i) * m.jx + V::cy(i) * m.jy + V::cz(i) * m.jz;
        const float sp = V::w(i) * (m.drho + m.rho * (4.5f * cu * cu - usq15)), dp = V::a(i) * cj;
        feq[i] = sp + dp;
        feq[o] = sp - dp;
    }
}

// D2Q9 moment basis of the multiple-relaxation-time collision: row r of M
// is a polynomial of the lattice velocity (rho, e, eps, jx, qx, jy, qy, pxx,
// pxy); the rows are orthogonal with squared norms mrt_norm.
__host__ __device__ constexpr int mrt_m(int r, int i) {
    using V = Vel<9>;
    const int cx = V::cx(i), cy = V::cy(i), c2 = cx * cx + cy * cy;
    return r == 0 ? 1 : r == 1 ? -4 + 3 * c2 : r == 2 ? (8 - 21 * c2 + 9 * c2 * c2) / 2 : r == 3 ? cx
         : r == 4 ? (-5 + 3 * c2) * cx : r == 5 ? cy : r == 6 ? (-5 + 3 * c2) * cy : r == 7 ? cx * cx - cy * cy
         : cx * cy;
}
__host__ __device__ constexpr int mrt_norm(int r) {
    int s = 0;
    for (int i = 0; i < 9; ++i) s += mrt_m(r, i) * mrt_m(r, i);
    return s;
}

// MRT relaxation of d = g - feq: returns M^-1 S M d in out (S: rates, the
// two stress rates being omega).
__device__ inline void mrt_relax(const float (&d)[9], const float *rates, float omega, float (&out)[9]) {
    float m[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            if (mrt_m(r, i)) acc += (float)mrt_m(r, i) * d[i];
        m[r] = acc * ((r >= 7 ? omega : rates[r]) / (float)mrt_norm(r));
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        float acc = 0.f;
#pragma unroll
        for (int r = 0; r < 9; ++r)
            if (mrt_m(r, i)) acc += (float)mrt_m(r, i) * m[r];
        out[i] = acc;
    }
}

// Moments of a node's own populations (face nodes of anti-bounce-back faces).
template <int Q>
__device__ inline void own_velocity(__amdgpu_buffer_rsrc_t r, int plane, unsigned own, float &rho, float (&u)[3]) {
    float f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = bload(r, own + (unsigned)(i * plane) * 4u);
    const Moments m = moments<Q>(f);
    rho = m.rho;
    u[0] = m.ux; u[1] = m.uy; u[2] = m.uz;
}

// Anti-bounce-back closure (Eq. 6) in shifted form.  On entry the unknown
// slots hold the outgoing post-collision populations of the node (gathered
// through the bounce-back offset); uF is the node's velocity before the
// step.  With E_i = 1 + (u.c_i)^2/(2 cs^4) - u.u/(2 cs^2) and rho_w = 1 + drho_b,
//   g_i = -F_opp(i) + 2 w_i rho_w E_i - 2 w_i = -F_opp(i) + 2 w_i (drho_b + rho_w (E_i - 1)).
// in / out select the inlet (unknowns c_x = +1) or outlet (c_x = -1).
template <int Q>
__device__ inline void abb(float (&g)[Q], bool in, bool out, float drho_b, const float (&uF)[3]) {
    using V = Vel<Q>;
    const float usq = uF[0] * uF[0] + uF[1] * uF[1] + uF[2] * uF[2];
    const float rw = 1.0f + drho_b;
#pragma unroll
    for (int p = 1; p < Q; ++p) {
        if (V::cx(p) != 1) continue;
        const int m = V::opp(p);
        const float cu = uF[0] + (V::cy(p) ? V::cy(p) * uF[1] : 0.f) + (V::cz(p) ? V::cz(p) * uF[2] : 0.f);
        const float e = 2.0f * V::w(p) * (drho_b + rw * (4.5f * cu * cu - 1.5f * usq));
        g[p] = in ? e - g[p] : g[p];
        g[m] = out ? e - g[m] : g[m];
    }
}

// Transpose of the anti-bounce-back closure that built g^{k+1} at this node
// from F^k: nu holds the node's adjoints of its unknowns at step k+1 (one per
// pair, for the active face), (rho, u) are the moments of F^k.  Adds the
// contributions to lam = dL/dF^k and returns dL/d(drho_b).
//   d g_u / d F_opp(u) = -1,
//   d g_u / d F_j      = 2 w_u rho_w (9 (u.c_u) c_u - 3 u) . (c_j - u) / rho,
//   d g_u / d drho_b   = 2 w_u E_u.
template <int Q>
__device__ inline float abb_adj(float (&lam)[Q], bool in, bool out, float drho_b, float rho, const float (&u)[3],
                                const float (&nu)[Q]) {
    using V = Vel<Q>;
    const float usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const float rw = 1.0f + drho_b;
    float gb = 0.f, Vx = 0.f, Vy = 0.f, Vz = 0.f;
#pragma unroll
    for (int p = 1; p < Q; ++p) {
        if (V::cx(p) != 1) continue;
        const int m = V::opp(p);
        const float cu = u[0] + (V::cy(p) ? V::cy(p) * u[1] : 0.f) + (V::cz(p) ? V::cz(p) * u[2] : 0.f);
        const float nu_u = in ? nu[p] : (out ? nu[m] : 0.f);
        lam[m] -= in ? nu_u : 0.f;
        lam[p] -= out ? nu_u : 0.f;
        gb += nu_u * 2.0f * V::w(p) * (1.0f + 4.5f * cu * cu - 1.5f * usq);
        const float s = nu_u * 2.0f * V::w(p) * rw;
        Vx += s * (9.0f * cu - 3.0f * u[0]);
        Vy += s * ((V::cy(p) ? 9.0f * cu * V::cy(p) : 0.f) - 3.0f * u[1]);
        Vz += s * ((V::cz(p) ? 9.0f * cu * V::cz(p) : 0.f) - 3.0f * u[2]);
    }
    const float inv = 1.0f / rho;
    const float Vu = Vx * u[0] + Vy * u[1] + Vz * u[2];
#pragma unroll
    for (int j = 0; j < Q; ++j)
        lam[j] += inv * ((V::cx(j) ? V::cx(j) * Vx : 0.f) + (V::cy(j) ? V::cy(j) * Vy : 0.f) +
                         (V::cz(j) ? V::cz(j) * Vz : 0.f) - Vu);
    return gb;
}

// Wavefront (64-lane) sum in FP64.
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block (4 wavefronts) sum of per-lane values, in FP64 from the lane value
// up (fixed order); the result is valid in thread 0.
__device__ inline double block_sum(float v, double *lds4) {
    const double w = wave_sum((double)v);
    if ((threadIdx.x & 63) == 0) lds4[threadIdx.x >> 6] = w;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
    __syncthreads();
    return s;
}
static_assert(BLOCK == 256 && FT == 256, "block_sum assumes four wavefronts");

}  // namespace lbm
