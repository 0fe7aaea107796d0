// BF16 MFMA kernels (gfx950) of the warm-start U-Net: implicit-GEMM
// convolution (3x3 / 3x3x3 / 1x1, forward and input gradient), weight
// gradient, 2x2(x2) stride-2 transposed convolution (as GEMM with a
// depth-to-space / space-to-depth operand mode), max pooling, ReLU backward,
// bias gradient, masked MSE, Adam, and the feature / normalisation maps that
// connect the network to the LBM.
//
// Activations are pixel-major ("channels last", N[D]HWC) BF16 with an
// explicit channel stride and offset so that concatenation is a layout
// choice: a producer writes straight into its slice of the concatenated
// buffer.  Products accumulate in FP32 on the matrix cores
// (v_mfma_f32_16x16x32_bf16).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "unet_kernels.hpp"

namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __host__ inline float bf2f(uint16_t v) {
    union { uint32_t u; float f; } c;
    c.u = (uint32_t)v << 16;
    return c.f;
}

// float -> bf16, round to nearest even (NaN kept quiet).
__device__ __host__ inline uint16_t f2bf(float f) {
    union { uint32_t u; float f; } c;
    c.f = f;
    if ((c.u & 0x7f800000u) == 0x7f800000u && (c.u & 0x007fffffu)) return (uint16_t)((c.u >> 16) | 0x40);
    const uint32_t r = c.u + 0x7fffu + ((c.u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}

constexpr int BM = 64, BN = 64;          // weight-gradient output tile (rows x K entries)

// Pixel index -> (b, z, y, x) on a grid of d x h x w per sample (pixel
// counts stay below 2^31: checked on the host).
struct Pix { int b, z, y, x; };
__device__ inline Pix pix_of(long long m64, int d, int h, int w) {
    unsigned m = (unsigned)m64;
    Pix p;
    unsigned q = m / (unsigned)w;
    p.x = (int)(m - q * (unsigned)w);
    m = q;
    q = m / (unsigned)h;
    p.y = (int)(m - q * (unsigned)h);
    m = q;
    q = m / (unsigned)d;
    p.z = (int)(m - q * (unsigned)d);
    p.b = (int)q;
    return p;
}

// K entry k of the implicit im2col matrix: channel ci and stencil offset
// (normal mode: k = tap * cin + ci over a ks^dims stencil centred on the
// pixel) or fine-grid sub-pixel (S2D mode: k = sub * cin + ci reads pixel
// (2z+sz, 2y+sy, 2x+sx), sub = sx + 2 sy + 4 sz).
struct Tap { int ci, dx, dy, dz; };
__device__ inline Tap tap_of(const ConvArgs &a, int k) {
    Tap t;
    const int tap = (int)((unsigned)k / (unsigned)a.cin);
    t.ci = k - tap * a.cin;
    if (a.flags & FLAG_S2D) {
        t.dx = tap & 1; t.dy = (tap >> 1) & 1; t.dz = (tap >> 2) & 1;
    } else if (a.ks == 3) {
        t.dx = tap % 3 - 1; t.dy = (tap / 3) % 3 - 1; t.dz = a.dims == 3 ? tap / 9 - 1 : 0;
    } else {
        t.dx = t.dy = t.dz = 0;
    }
    return t;
}

// The pixel of an im2col row, resolved once: its coordinates and the element
// offset of its first input channel (normal mode: the pixel itself; S2D: the
// fine-grid pixel (2z, 2y, 2x)).
struct Row { long long base; int x, y, z; bool valid; };
__device__ inline Row row_of(const ConvArgs &a, long long m) {
    Row r;
    r.valid = m < a.M;
    const Pix p = pix_of(r.valid ? m : 0, a.d, a.h, a.w);
    r.x = p.x; r.y = p.y; r.z = p.z;
    long long px;
    if (a.flags & FLAG_S2D) {
        const int fd = a.dims == 3 ? 2 * a.d : 1, fh = 2 * a.h, fw = 2 * a.w;
        px = (((long long)p.b * fd + (a.dims == 3 ? 2 * p.z : 0)) * fh + 2 * p.y) * fw + 2 * p.x;
    } else {
        px = (((long long)p.b * a.d + p.z) * a.h + p.y) * a.w + p.x;
    }
    r.base = px * a.in_cs + a.in_co;
    return r;
}

// A K entry resolved once per step: its tap offset from a row's base and the
// stencil displacement (for the zero-padding test).
struct KOff { long long delta; int dx, dy, dz; bool valid; };
__device__ inline KOff koff_of(const ConvArgs &a, int k) {
    KOff o;
    o.valid = k < a.K;
    const Tap t = tap_of(a, o.valid ? k : 0);
    o.dx = t.dx; o.dy = t.dy; o.dz = t.dz;
    long long d;
    if (a.flags & FLAG_S2D) {
        const int fh = 2 * a.h, fw = 2 * a.w;
        d = ((long long)t.dz * fh + t.dy) * fw + t.dx;
    } else {
        d = ((long long)t.dz * a.h + t.dy) * a.w + t.dx;
    }
    o.delta = d * a.in_cs + t.ci;
    return o;
}

// 16 bytes of the im2col matrix at (row, K offset), zero outside the grid.
__device__ inline uint4 im2col_load(const ConvArgs &a, const Row &r, const KOff &o) {
    bool ok = r.valid && o.valid;
    if (!(a.flags & FLAG_S2D)) {
        const unsigned xs = (unsigned)(r.x + o.dx), ys = (unsigned)(r.y + o.dy), zs = (unsigned)(r.z + o.dz);
        ok = ok && xs < (unsigned)a.w && ys < (unsigned)a.h && zs < (unsigned)a.d;
    }
    return ok ? *(const uint4 *)(a.in + r.base + o.delta) : make_uint4(0, 0, 0, 0);
}

// (b, z, y, x) of a flat pixel index kept as a mixed-radix counter: adding
// a fixed step digit by digit needs one carry per digit (each digit of the
// step is below its radix) and no division.
struct Cursor { int x, y, z, b; };
__device__ inline Cursor cursor_of(unsigned m, const ConvArgs &a) {
    const Pix p = pix_of(m, a.d, a.h, a.w);
    return Cursor{p.x, p.y, p.z, p.b};
}
__device__ inline void cursor_add(Cursor &c, const Cursor &s, const ConvArgs &a) {
    c.x += s.x;
    int k = c.x >= a.w;
    c.x -= k ? a.w : 0;
    c.y += s.y + k;
    k = c.y >= a.h;
    c.y -= k ? a.h : 0;
    c.z += s.z + k;
    k = c.z >= a.d;
    c.z -= k ? a.d : 0;
    c.b += s.b + k;
}
__device__ inline void cursor_inc(Cursor &c, const ConvArgs &a) { cursor_add(c, Cursor{1, 0, 0, 0}, a); }

__device__ inline bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// Output element of GEMM cell (m, c): returns the flat index and the bias
// channel; D2S maps column c = sub * Cr + co to the fine pixel.
__device__ inline long long out_index(const ConvArgs &a, long long m, int c, int &bias_c) {
    if (a.flags & FLAG_D2S) {
        const int cr = a.ncols >> a.dims;
        const int sub = c / cr, co = c - sub * cr;
        bias_c = co;
        const Pix p = pix_of(m, a.d, a.h, a.w);
        const int sx = sub & 1, sy = (sub >> 1) & 1, sz = (sub >> 2) & 1;
        const int fd = a.dims == 3 ? 2 * a.d : 1, fh = 2 * a.h, fw = 2 * a.w;
        const int zf = a.dims == 3 ? 2 * p.z + sz : 0;
        const long long f = (((long long)p.b * fd + zf) * fh + 2 * p.y + sy) * fw + 2 * p.x + sx;
        return f * a.out_cs + a.out_co + co;
    }
    bias_c = c;
    return m * a.out_cs + a.out_co + c;
}

// C[M x ncols] = im2col(in)[M x K] * W^T, W stored [ncols][K].
// A block computes a TBM x TBN tile with four wavefronts (2 x 2, each
// TBM/2 x TBN/2 of 16 x 16 x 32 BF16 MFMA tiles) over K steps of 64.  The
// LDS tiles are double-buffered: the next step's global loads are issued
// before the current step's MFMAs and land in the other buffer, so a step
// needs one barrier.  64 x 32 tiles serve the 32- and 8-channel layers
// without computing zero columns (and keep 5 blocks per CU).
// SPLIT: blockIdx.z takes K steps [z sper, (z + 1) sper) and the block
// stores its raw FP32 products to part[z][m][c] (k_conv_reduce adds the
// splits and applies the epilogue).
template <int TBM, int TBN, bool SPLIT = false>
__global__ void __launch_bounds__(256) k_conv(ConvArgs a, float *__restrict__ part = nullptr, int sper = 0) {
    constexpr int KB = 64, LD = KB + 8;             // LDS rows padded by 16 B
    constexpr int WM = TBM / 2, WN = TBN / 2;
    constexpr int TI = WM / 16, TJ = WN / 16;
    constexpr int AL = TBM * 8 / 256, BL = TBN * 8 / 256;   // 16-byte loads per thread
    __shared__ uint16_t As[2][TBM][LD];
    __shared__ uint16_t Bs[2][TBN][LD];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const long long m0 = (long long)blockIdx.x * TBM;
    const int n0 = blockIdx.y * TBN;
    const int kq = (t & 7) * 8;
    // rows of the im2col tile this thread loads: t / 8 + 32 l; their pixels are fixed
    Row row[AL];
#pragma unroll
    for (int l = 0; l < AL; ++l) row[l] = row_of(a, m0 + (t >> 3) + 32 * l);
    uint4 ra[AL], rb[BL];
    auto load = [&](int k0) {
        const int k = k0 + kq;
        const bool kval = k < a.K;
        const KOff ko = koff_of(a, k);
#pragma unroll
        for (int l = 0; l < AL; ++l) ra[l] = im2col_load(a, row[l], ko);
#pragma unroll
        for (int l = 0; l < BL; ++l) {
            const int n = n0 + (t >> 3) + 32 * l;
            rb[l] = n < a.ncols && kval ? *(const uint4 *)(a.wt + (long long)n * a.K + k) : make_uint4(0, 0, 0, 0);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int l = 0; l < AL; ++l) *(uint4 *)&As[buf][(t >> 3) + 32 * l][kq] = ra[l];
#pragma unroll
        for (int l = 0; l < BL; ++l) *(uint4 *)&Bs[buf][(t >> 3) + 32 * l][kq] = rb[l];
    };
    f32x4 acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int s0 = SPLIT ? (int)blockIdx.z * sper : 0;
    const int steps = SPLIT ? min((a.K + KB - 1) / KB, s0 + sper) : (a.K + KB - 1) / KB;
    load(s0 * KB);
    stash(s0 & 1);
    __syncthreads();
    for (int s = s0; s < steps; ++s) {
        const int buf = s & 1;
        if (s + 1 < steps) load((s + 1) * KB);
#pragma unroll
        for (int kh = 0; kh < KB; kh += 32) {
            const int kr = kh + (lane >> 4) * 8;
            bf16x8 fb[TJ];
#pragma unroll
            for (int j = 0; j < TJ; ++j) fb[j] = as_bf16x8(*(const uint4 *)&Bs[buf][wn * WN + j * 16 + (lane & 15)][kr]);
#pragma unroll
            for (int i = 0; i < TI; ++i) {
                const bf16x8 fa = as_bf16x8(*(const uint4 *)&As[buf][wm * WM + i * 16 + (lane & 15)][kr]);
#pragma unroll
                for (int j = 0; j < TJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb[j], acc[i][j], 0, 0, 0);
            }
        }
        if (s + 1 < steps) stash(buf ^ 1);
        __syncthreads();
    }
    if (SPLIT) {
        float *dst = part + (long long)blockIdx.z * a.M * a.ncols;
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j) {
                const int c = n0 + wn * WN + j * 16 + (lane & 15);
                if (c >= a.ncols) continue;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const long long m = m0 + wm * WM + i * 16 + (lane >> 4) * 4 + q;
                    if (m < a.M) dst[m * a.ncols + c] = acc[i][j][q];
                }
            }
        return;
    }
    const bool d2s = (a.flags & FLAG_D2S) != 0;
    const int cr = d2s ? a.ncols >> a.dims : a.ncols;      // D2S: columns sub * cr + co
    const uintptr_t base = a.out32 ? (uintptr_t)a.out32 : (uintptr_t)a.out;
    if (((a.out_cs | a.out_co) & 7) == 0 && (!d2s || (cr & 7) == 0) && (base & 15) == 0) {
        // the tile goes through LDS (the A buffers are free after the last barrier) so that each
        // thread stores 8 consecutive channels of a pixel (of the fine pixel for D2S, whose
        // 8-column groups stay inside one sub-pixel) with 16-byte writes
        constexpr int TL = TBN + 4;
        static_assert(TBM * TL * 4 <= (int)sizeof(As), "epilogue tile must fit in the A buffers");
        float *T = reinterpret_cast<float *>(&As[0][0][0]);
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j) {
                const int cl = wn * WN + j * 16 + (lane & 15), c = n0 + cl;
                const float b = a.bias && c < a.ncols ? a.bias[d2s ? c - (c / cr) * cr : c] : 0.f;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float v = acc[i][j][q] + b;
                    if (a.flags & FLAG_RELU) v = v > 0.f ? v : 0.f;
                    T[(wm * WM + i * 16 + (lane >> 4) * 4 + q) * TL + cl] = v;
                }
            }
        __syncthreads();
        constexpr int CG = TBN / 8;
        for (int e = t; e < TBM * CG; e += 256) {
            const int ml = e / CG, cl = (e - ml * CG) * 8;
            const long long m = m0 + ml;
            const int c = n0 + cl;
            if (m >= a.M || c >= a.ncols) continue;
            const float *src = &T[ml * TL + cl];
            int bc;
            const long long o = out_index(a, m, c, bc);
            if (a.out32) {
                float *dst = a.out32 + o;
                const int nk = a.ncols - c < 8 ? a.ncols - c : 8;
                if (nk == 8) {
                    float4 v0 = make_float4(src[0], src[1], src[2], src[3]);
                    float4 v1 = make_float4(src[4], src[5], src[6], src[7]);
                    if (a.flags & FLAG_ACC) {
                        const float4 o0 = *(const float4 *)dst, o1 = *(const float4 *)(dst + 4);
                        v0.x += o0.x; v0.y += o0.y; v0.z += o0.z; v0.w += o0.w;
                        v1.x += o1.x; v1.y += o1.y; v1.z += o1.z; v1.w += o1.w;
                    }
                    *(float4 *)dst = v0;
                    *(float4 *)(dst + 4) = v1;
                } else {
                    for (int k = 0; k < nk; ++k) dst[k] = (a.flags & FLAG_ACC) ? dst[k] + src[k] : src[k];
                }
                continue;
            }
            uint16_t *dst = a.out + o;
            if (c + 8 <= a.ncols) {
                float v[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) v[k] = src[k];
                if (a.flags & FLAG_ACC) {
                    const uint4 old = *(const uint4 *)dst;
                    const uint32_t ow[4] = {old.x, old.y, old.z, old.w};
#pragma unroll
                    for (int k = 0; k < 8; ++k) v[k] += bf2f((uint16_t)(ow[k >> 1] >> (16 * (k & 1))));
                }
                uint32_t pw[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) pw[k] = (uint32_t)f2bf(v[2 * k]) | ((uint32_t)f2bf(v[2 * k + 1]) << 16);
                *(uint4 *)dst = make_uint4(pw[0], pw[1], pw[2], pw[3]);
            } else {
                for (int k = 0; k < a.ncols - c; ++k) {
                    float v = src[k];
                    if (a.flags & FLAG_ACC) v += bf2f(dst[k]);
                    dst[k] = f2bf(v);
                }
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int c = n0 + wn * WN + j * 16 + (lane & 15);
            if (c >= a.ncols) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const long long m = m0 + wm * WM + i * 16 + (lane >> 4) * 4 + q;
                if (m >= a.M) continue;
                int bc;
                const long long o = out_index(a, m, c, bc);
                float v = acc[i][j][q] + (a.bias ? a.bias[bc] : 0.f);
                if (a.flags & FLAG_RELU) v = v > 0.f ? v : 0.f;
                if (a.out32) {
                    a.out32[o] = (a.flags & FLAG_ACC) ? a.out32[o] + v : v;
                } else {
                    if (a.flags & FLAG_ACC) v += bf2f(a.out[o]);
                    a.out[o] = f2bf(v);
                }
            }
        }
}

// 3 x 3 convolution of a 2D layer whose input channels come in chunks of 32
// (a last, shorter chunk is zero-filled), on tiles of 8 x 32 pixels (the
// image sizes must be multiples of those).  Per
// chunk, the tile's input patch with its one-pixel halo (10 x 34 pixels) and
// the chunk's weights of all 9 taps are staged in LDS once; the 9 taps then
// read their MFMA operands from LDS, so each input pixel crosses L2 about
// 1.3 times instead of 9.  Four wavefronts take two tile rows (64 pixels) each
// and all TN output columns.  The epilogue stages the tile in the same LDS and
// stores 8 channels of a pixel with one 16-byte write.
constexpr int HY = 8, HX = 32, HPX = HX + 2, HP = (HY + 2) * HPX;   // tile rows, columns, patch
constexpr int HC = 32;                                               // chunk channels (64-byte LDS rows)

// Half-word offset of 16-byte granule g (0..3) of LDS row `row` in the halo
// kernel's patch and weight tiles: the granules of a row are XOR-swizzled by
// (row >> 2) & 3, so the 16 consecutive rows that an MFMA operand read
// touches (one granule each) and the 4 rows x 4 granules of a staging write
// fall on 16 distinct 16-byte bank groups.
__device__ inline int hsw(int row, int g) { return row * HC + ((g ^ ((row >> 2) & 3)) << 3); }

// In 3D a block takes one 8 x 32 tile of one plane z and, per chunk, runs
// the same staging and 9 taps for each of the three input planes z - 1, z,
// z + 1 (taps dz * 9 + dy * 3 + dx), skipping planes outside the volume.
template <int TN, int DIMS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_conv3x3_halo(ConvArgs a) {
    constexpr int WNT = TN / 16;
    constexpr int PATCH = HP * HC, WTS = 9 * TN * HC;
    constexpr int TL = TN + 4;
    constexpr int ELEMS = PATCH + WTS > 2 * 256 * TL ? PATCH + WTS : 2 * 256 * TL;
    __shared__ __align__(16) uint16_t sm[ELEMS];
    uint16_t *P = sm, *Wl = sm + PATCH;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int tiles_x = a.w / HX, tiles_y = a.h / HY;
    int bt = blockIdx.x;
    const int tx = bt % tiles_x;
    bt /= tiles_x;
    const int ty = bt % tiles_y;
    bt /= tiles_y;
    const int z = DIMS == 3 ? bt % a.d : 0, b = DIMS == 3 ? bt / a.d : bt;
    const int n0 = blockIdx.y * TN, y0 = ty * HY, x0 = tx * HX;
    f32x4 acc[4][WNT];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < WNT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // Stages are (chunk, input plane) pairs; a plane outside the volume adds
    // nothing and is skipped (block-uniform).  A stage's patch and weights
    // are loaded into registers in one batch (every load in flight at once)
    // while the previous stage multiplies, then written to LDS.
    constexpr int NDZ = DIMS == 3 ? 3 : 1;
    constexpr int NPL = (HP * 4 + 255) / 256, NWL = (9 * TN * 4 + 255) / 256;
    const int nst = ((a.cin + HC - 1) / HC) * NDZ;          // a last chunk of fewer channels is zero-filled
    auto plane_ok = [&](int st) { return DIMS == 2 || (unsigned)(z + st % NDZ - 1) < (unsigned)a.d; };
    auto next_stage = [&](int st) {
        do ++st; while (st < nst && !plane_ok(st));
        return st;
    };
    uint4 pv[NPL], wv[NWL];
    auto load = [&](int st) {
        const int c0 = (st / NDZ) * HC, dz = st % NDZ;
        const int zz = DIMS == 3 ? z + dz - 1 : 0, tap0 = DIMS == 3 ? dz * 9 : 0;
#pragma unroll
        for (int k = 0; k < NPL; ++k) {
            const int e = t + 256 * k;
            const int pp = e >> 2, g8 = (e & 3) * 8;
            const int py = pp / HPX, px = pp - py * HPX;
            const int yy = y0 + py - 1, xx = x0 + px - 1;
            pv[k] = make_uint4(0, 0, 0, 0);
            if (e < HP * 4 && c0 + g8 < a.cin && (unsigned)yy < (unsigned)a.h && (unsigned)xx < (unsigned)a.w)
                pv[k] = *(const uint4 *)(a.in + ((((long long)b * a.d + zz) * a.h + yy) * a.w + xx) * a.in_cs +
                                         a.in_co + c0 + g8);
        }
#pragma unroll
        for (int k = 0; k < NWL; ++k) {
            const int e = t + 256 * k;
            const int g8 = (e & 3) * 8, r = e >> 2;
            const int tap = r / TN, n = r - tap * TN;
            wv[k] = make_uint4(0, 0, 0, 0);
            if (e < 9 * TN * 4 && c0 + g8 < a.cin && n0 + n < a.ncols)
                wv[k] = *(const uint4 *)(a.wt + (long long)(n0 + n) * a.K + (tap0 + tap) * a.cin + c0 + g8);
        }
    };
    int st = plane_ok(0) ? 0 : next_stage(0);
    if (st < nst) load(st);
    for (; st < nst;) {
        __syncthreads();                                   // the previous stage's operand reads are done
#pragma unroll
        for (int k = 0; k < NPL; ++k) {
            const int e = t + 256 * k;
            if (e < HP * 4) *(uint4 *)&P[hsw(e >> 2, e & 3)] = pv[k];
        }
#pragma unroll
        for (int k = 0; k < NWL; ++k) {
            const int e = t + 256 * k;
            if (e < 9 * TN * 4) *(uint4 *)&Wl[hsw(e >> 2, e & 3)] = wv[k];
        }
        __syncthreads();
        const int nx = next_stage(st);
        if (nx < nst) load(nx);
        st = nx;
#pragma unroll 1
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap - dy * 3;       // tap (dx - 1, dy - 1) reads patch (+dx, +dy)
            bf16x8 fb[WNT];
#pragma unroll
            for (int j = 0; j < WNT; ++j)
                fb[j] = as_bf16x8(*(const uint4 *)&Wl[hsw(tap * TN + j * 16 + (lane & 15), lane >> 4)]);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int pr = 2 * wave + (i >> 1), pc = (i & 1) * 16 + (lane & 15);
                const bf16x8 fa = as_bf16x8(*(const uint4 *)&P[hsw((pr + dy) * HPX + pc + dx, lane >> 4)]);
#pragma unroll
                for (int j = 0; j < WNT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb[j], acc[i][j], 0, 0, 0);
            }
        }
    }
    __syncthreads();                                       // the last stage's operand reads are done
    // epilogue: tile pixel p = row * 32 + column, staged as floats in the same LDS
    float *T = reinterpret_cast<float *>(sm);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < WNT; ++j) {
            const int cl = j * 16 + (lane & 15), c = n0 + cl;
            const float bias = a.bias && c < a.ncols ? a.bias[c] : 0.f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int p = (2 * wave + (i >> 1)) * HX + (i & 1) * 16 + (lane >> 4) * 4 + q;
                float v = acc[i][j][q] + bias;
                if (a.flags & FLAG_RELU) v = v > 0.f ? v : 0.f;
                T[p * TL + cl] = v;
            }
        }
    __syncthreads();
    constexpr int CG = TN / 8;
    for (int e = t; e < 256 * CG; e += 256) {
        const int p = e / CG, cl = (e - p * CG) * 8, c = n0 + cl;
        if (c >= a.ncols) continue;
        const long long m = (((long long)b * a.d + z) * a.h + y0 + p / HX) * a.w + x0 + (p % HX);
        const float *src = &T[p * TL + cl];
        const long long o = m * a.out_cs + a.out_co + c;
        const int nk = a.ncols - c < 8 ? a.ncols - c : 8;
        if (a.out32) {
            float *dst = a.out32 + o;
            for (int k = 0; k < nk; ++k) dst[k] = (a.flags & FLAG_ACC) ? dst[k] + src[k] : src[k];
            continue;
        }
        uint16_t *dst = a.out + o;
        if (nk == 8) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = src[k];
            if (a.flags & FLAG_ACC) {
                const uint4 old = *(const uint4 *)dst;
                const uint32_t ow[4] = {old.x, old.y, old.z, old.w};
#pragma unroll
                for (int k = 0; k < 8; ++k) v[k] += bf2f((uint16_t)(ow[k >> 1] >> (16 * (k & 1))));
            }
            uint32_t pw[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) pw[k] = (uint32_t)f2bf(v[2 * k]) | ((uint32_t)f2bf(v[2 * k + 1]) << 16);
            *(uint4 *)dst = make_uint4(pw[0], pw[1], pw[2], pw[3]);
        } else {
            for (int k = 0; k < nk; ++k) {
                float v = src[k];
                if (a.flags & FLAG_ACC) v += bf2f(dst[k]);
                dst[k] = f2bf(v);
            }
        }
    }
}

// Weight gradient: dW[r][k] = sum_m G[m][r] * im2col(in)[m][k], G = dout
// (S2D: r = sub * Cr + co read at the fine pixel).  blockIdx.z splits the
// pixel range; partials are summed by k_sum_splits.  The contraction runs
// over pixels, which are the slow index of both operands in memory, so each
// stage of WPB pixels is transposed on its way into LDS: a thread loads 4
// consecutive pixels x 8 channels of G and of the im2col rows, swaps them in
// registers and writes one 8-byte run of 4 pixels per channel.  The next
// stage's global loads are issued before the current stage's MFMAs.
constexpr int WPB = 128, WLD = WPB + 8;          // pixels per stage; LDS rows padded by 16 B

// Column (in halfwords) of pixel col of LDS row `row`: the 16-byte granules
// of a row are XOR-swizzled by (row >> 3) & 7.  The staging writes put 4
// pixels of 8 rows that are 8 apart; unswizzled, those rows alias onto two
// bank groups (the 272-byte row stride times 8 is a multiple of 128 banks'
// worth of bytes), swizzled they spread over all banks; the MFMA operand
// reads (16 consecutive rows, one granule) stay conflict-free.
__device__ inline int wcol(int row, int col) { return (((col >> 3) ^ ((row >> 3) & 7)) << 3) | (col & 7); }

// v[j] = 8 channels of pixel j (j = 0..3) -> o[e] = channel e of pixels 0..3.
__device__ inline void transpose_4x8(const uint4 (&v)[4], uint2 (&o)[8]) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int d = e >> 1;
        const uint32_t a0 = (&v[0].x)[d], a1 = (&v[1].x)[d], a2 = (&v[2].x)[d], a3 = (&v[3].x)[d];
        // v_perm_b32 picks bytes of {hi, lo}: 0x05040100 = low halves (lo, hi), 0x07060302 = high halves
        const uint32_t sel = (e & 1) ? 0x07060302u : 0x05040100u;
        o[e] = make_uint2(__builtin_amdgcn_perm(a1, a0, sel), __builtin_amdgcn_perm(a3, a2, sel));
    }
}

// NARROW (at most 32 rows, the 32-channel layers): a block takes 32 rows x
// 128 columns and its four wavefronts sit side by side along the columns, so
// no MFMA works on the empty rows a 64-row tile would carry; each thread then
// loads two column groups of the im2col rows, and half the threads the rows
// of G.
template <bool NARROW>
__global__ void __launch_bounds__(256) k_wgrad(ConvArgs a, const uint16_t *__restrict__ g, int g_cs,
                                               int g_co, int rows, float *__restrict__ part,
                                               long long chunk) {
    constexpr int RM = NARROW ? 32 : BM;            // rows per block
    constexpr int CN = NARROW ? 128 : BN;           // columns per block
    constexpr int NT = CN / 64;                     // column groups of 64 per thread
    __shared__ uint16_t Gs[RM][WLD];
    __shared__ uint16_t Ts[CN][WLD];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = NARROW ? 0 : (wave & 1), wn = NARROW ? wave : (wave >> 1);
    const int r0 = blockIdx.x * RM, c0 = blockIdx.y * CN;
    const long long mb = (long long)blockIdx.z * chunk;
    const long long me = mb + chunk < a.M ? mb + chunk : a.M;
    const int pg = t >> 3, cg = (t & 7) * 8;        // pixels 4 pg .. 4 pg + 3 of a stage, channels cg .. cg + 7
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bool s2d_g = (a.flags & FLAG_S2D_G) != 0, s2d = (a.flags & FLAG_S2D) != 0;
    // the thread's im2col columns (tap, channel) and G channel are fixed over
    // the pixel loop: tap displacement, 32-bit offset from the pixel's first
    // channel, and the fine-grid sub-pixel of an S2D_G row
    int dx[NT], dy[NT], dz[NT], dl[NT];
    bool kv[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        const KOff o = koff_of(a, c0 + 64 * n + cg);
        dx[n] = o.dx; dy[n] = o.dy; dz[n] = o.dz; dl[n] = (int)o.delta; kv[n] = o.valid;
    }
    const int r = r0 + cg;
    const bool g_rows = cg < RM && r < rows;        // this thread stages rows of G
    int gch = r, gsx = 0, gsy = 0, gsz = 0;
    if (s2d_g) {
        const int cr = rows >> a.dims, sub = r / cr;
        gch = r - sub * cr; gsx = sub & 1; gsy = (sub >> 1) & 1; gsz = (sub >> 2) & 1;
    }
    const int fd = a.dims == 3 ? 2 * a.d : 1, fh = 2 * a.h, fw = 2 * a.w;
    // coordinates of the thread's first pixel of the next stage; a stage
    // advances them by WPB pixels through the step's own digits
    Cursor cur = cursor_of((unsigned)(mb + 4 * pg), a);
    const Cursor step = cursor_of((unsigned)WPB, a);
    uint4 gv[4], tv[NT][4];
    auto load = [&](long long mm) {
        const long long m0 = mm + 4 * pg;
        const uint16_t *tp = a.in + a.in_co + m0 * a.in_cs;
        const uint16_t *gp = g + g_co + gch + m0 * g_cs;
        Cursor c = cur;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (j) cursor_inc(c, a);
            const bool mv = m0 + j < me;
            gv[j] = make_uint4(0, 0, 0, 0);
            if (g_rows && mv) {
                const uint16_t *src = gp + j * g_cs;
                if (s2d_g) {
                    const int zf = a.dims == 3 ? 2 * c.z + gsz : 0;
                    const int f = ((c.b * fd + zf) * fh + 2 * c.y + gsy) * fw + 2 * c.x + gsx;
                    src = g + g_co + gch + (long long)f * g_cs;
                }
                gv[j] = *(const uint4 *)src;
            }
            const uint16_t *pix = tp + j * a.in_cs;
            if (s2d) {
                const int px = ((c.b * fd + (a.dims == 3 ? 2 * c.z : 0)) * fh + 2 * c.y) * fw + 2 * c.x;
                pix = a.in + a.in_co + (long long)px * a.in_cs;
            }
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                bool ok = mv && kv[n];
                if (!s2d)
                    ok = ok && (unsigned)(c.x + dx[n]) < (unsigned)a.w && (unsigned)(c.y + dy[n]) < (unsigned)a.h &&
                         (unsigned)(c.z + dz[n]) < (unsigned)a.d;
                tv[n][j] = ok ? *(const uint4 *)(pix + dl[n]) : make_uint4(0, 0, 0, 0);
            }
        }
        cursor_add(cur, step, a);
    };
    load(mb);
    for (long long mm = mb; mm < me; mm += WPB) {
        __syncthreads();                              // the previous stage's MFMA reads are done
        {
            uint2 o[8];
            if (g_rows) {
                transpose_4x8(gv, o);
#pragma unroll
                for (int e = 0; e < 8; ++e) *(uint2 *)&Gs[cg + e][wcol(cg + e, 4 * pg)] = o[e];
            }
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                transpose_4x8(tv[n], o);
#pragma unroll
                for (int e = 0; e < 8; ++e) *(uint2 *)&Ts[64 * n + cg + e][wcol(64 * n + cg + e, 4 * pg)] = o[e];
            }
        }
        __syncthreads();
        if (mm + WPB < me) load(mm + WPB);
#pragma unroll
        for (int kh = 0; kh < WPB; kh += 32) {
            const int kr = kh + (lane >> 4) * 8;
            bf16x8 fb[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int tr = wn * 32 + j * 16 + (lane & 15);
                fb[j] = as_bf16x8(*(const uint4 *)&Ts[tr][wcol(tr, kr)]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int gr = wm * 32 + i * 16 + (lane & 15);
                const bf16x8 fa = as_bf16x8(*(const uint4 *)&Gs[gr][wcol(gr, kr)]);
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb[j], acc[i][j], 0, 0, 0);
            }
        }
    }
    float *dst = part + (long long)blockIdx.z * rows * a.K;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c = c0 + wn * 32 + j * 16 + (lane & 15);
            if (c >= a.K) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int rr = r0 + wm * 32 + i * 16 + (lane >> 4) * 4 + q;
                if (rr < rows) dst[(long long)rr * a.K + c] = acc[i][j][q];
            }
        }
}

// Weight gradient of a 2D 3 x 3 convolution from halo-staged patches.  The
// generic kernel above gathers the im2col matrix, i.e. every input pixel 9
// times, and transposes it in registers.  Here a stage is a patch of
// PH x PW = 128 pixels of one image: its G rows and its input pixels with
// the one-pixel halo are copied into LDS once, pixel-major as they lie in
// memory (16-byte chunks, no transposes), and the nine taps are LDS row
// offsets of the same halo tile.  The MFMA operands, which run over pixels
// (the contraction index), come out of LDS through the gfx950 transposing
// read ds_read_b64_tr_b16.
//
// Lane layout of that read: in each group of 16 lanes, lane 4e + c names the
// 8-byte block holding columns 4c .. 4c + 3 of row e, and lane i receives
// column i of the rows 0 .. 3.  An MFMA 16x16x32 operand (lane l: tile row
// or column l & 15, K entries 8 (l >> 4) .. + 7) is the pair of reads
// h = 0, 1 in which lane 16 G + 4 e + c names K entry 8 G + 4 h + e, column
// block c.
//
// Block: RB = 32 WR rows x CB = 16 WC input channels x all 9 taps; wavefront
// w takes 32 rows (two m tiles) x 16 channels (one n tile) x the taps of
// its group (4 / (WR WC) groups split the 9 taps).  blockIdx.z takes a
// contiguous range of `per` patches.  A layer of 8 input channels runs as a
// 16-channel tile whose upper 8 channels are staged as zeros and not stored.
typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
__device__ inline v4s lds_tr(const uint16_t *p) {
    return __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) v4s *)p);
}
__device__ inline bf16x8 tr_operand(const uint16_t *p0, const uint16_t *p1) {
    const v8s v = __builtin_shufflevector(lds_tr(p0), lds_tr(p1), 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_bit_cast(bf16x8, v);
}

// The MFMAs of one stage for taps T0 .. T1 - 1: x0 / x1 and g0 / g1 are the
// lane's read addresses (h = 0, 1) for the patch's first 32 pixels; the
// other 32-pixel chunks and the taps are constant offsets.
template <int PW, int XS, int GS, int T0, int T1, int NTAP>
__device__ inline void wgrad_halo_stage(const uint16_t *x0, const uint16_t *x1, const uint16_t *g0,
                                        const uint16_t *g1, f32x4 (&acc)[NTAP][2]) {
    constexpr int HW = PW + 2;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
        const int go = kc * 32 * GS, xo = kc * (32 / PW) * HW * XS;
        bf16x8 fa[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) fa[i] = tr_operand(g0 + go + 16 * i, g1 + go + 16 * i);
#pragma unroll
        for (int tap = T0; tap < T1; ++tap) {
            const int o = xo + ((tap / 3 - 1) * HW + tap % 3 - 1) * XS;
            const bf16x8 fb = tr_operand(x0 + o, x1 + o);
#pragma unroll
            for (int i = 0; i < 2; ++i)
                acc[tap - T0][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb, acc[tap - T0][i], 0, 0, 0);
        }
    }
}

template <int PW, int WR, int WC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_wgrad_halo(ConvArgs a, const uint16_t *__restrict__ g, int g_cs,
                                                    int g_co, int rows, float *__restrict__ part, int per,
                                                    int dz) {
    constexpr int PH = 128 / PW, HW = PW + 2, HP = (PH + 2) * HW;
    constexpr int RB = 32 * WR, CB = 16 * WC, WT = 4 / (WR * WC);
    constexpr int NTAP = (9 + WT - 1) / WT;
    constexpr int XS = CB + 8, GS = RB + 8;              // LDS row strides (halfwords), rows padded by 16 B
    constexpr int XCH = CB / 8, GCH = RB / 8;            // 16-byte chunks per pixel
    constexpr int XN = (HP * XCH + 255) / 256, GN = 128 * GCH / 256;
    static_assert(WT == 1 || WT == 2 || WT == 4, "taps split over 1, 2 or 4 wavefront groups");
    __shared__ __align__(16) uint16_t Xs[HP * XS];
    __shared__ __align__(16) uint16_t Gs[128 * GS];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wr = wave % WR, wc = (wave / WR) % WC, wt = wave / (WR * WC);
    const int r0 = blockIdx.x * RB, ci0 = blockIdx.y * CB;
    const int npx = (a.w + PW - 1) / PW, npy = (a.h + PH - 1) / PH;
    const int pb = blockIdx.z * per, pe = min(pb + per, a.n * a.d * npx * npy);
    // the lane's transposing-read addresses for the first 32 pixels
    const int G = lane >> 4, e = (lane >> 2) & 3, c = lane & 3;
    const uint16_t *xr[2], *gr[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = 8 * G + 4 * h + e;                 // pixel q of the patch (row q / PW, column q % PW)
        xr[h] = Xs + ((q / PW + 1) * HW + q % PW + 1) * XS + 16 * wc + 4 * c;
        gr[h] = Gs + q * GS + 32 * wr + 4 * c;
    }
    f32x4 acc[NTAP][2];
#pragma unroll
    for (int j = 0; j < NTAP; ++j) acc[j][0] = acc[j][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t *xin = a.in + a.in_co + ci0;
    const uint16_t *gin = g + g_co + r0;
    uint4 xv[XN], gv[GN];
    auto load = [&](int P) {
        const int px0 = (P % npx) * PW, rest = P / npx;
        const int py0 = (rest % npy) * PH, img = rest / npy;   // img = sample * d + plane
        const int base = (img * a.h + py0) * a.w + px0;  // the patch's first pixel
        // input plane z + dz (3D), zero outside the volume
        const bool zok = (unsigned)(img % a.d + dz) < (unsigned)a.d;
        const int xbase = base + dz * a.h * a.w;
#pragma unroll
        for (int i = 0; i < XN; ++i) {
            const int idx = t + 256 * i, hp = idx / XCH, cc = idx % XCH;
            const int y = py0 - 1 + hp / HW, x = px0 - 1 + hp % HW;
            const bool ok = zok && idx < HP * XCH && (unsigned)y < (unsigned)a.h && (unsigned)x < (unsigned)a.w &&
                            ci0 + 8 * cc < a.cin;
            const long long pix = xbase + (hp / HW - 1) * a.w + hp % HW - 1;
            xv[i] = ok ? *(const uint4 *)(xin + pix * a.in_cs + 8 * cc) : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < GN; ++i) {
            const int idx = t + 256 * i, p = idx / GCH, cc = idx % GCH;
            const bool ok = py0 + p / PW < a.h && px0 + p % PW < a.w;
            const long long pix = base + (p / PW) * a.w + p % PW;
            gv[i] = ok ? *(const uint4 *)(gin + pix * g_cs + 8 * cc) : make_uint4(0, 0, 0, 0);
        }
    };
    if (pb < pe) load(pb);
    for (int P = pb; P < pe; ++P) {
        __syncthreads();                                 // the previous stage's operand reads are done
#pragma unroll
        for (int i = 0; i < XN; ++i) {
            const int idx = t + 256 * i;
            if (idx < HP * XCH) *(uint4 *)&Xs[(idx / XCH) * XS + 8 * (idx % XCH)] = xv[i];
        }
#pragma unroll
        for (int i = 0; i < GN; ++i) {
            const int idx = t + 256 * i;
            *(uint4 *)&Gs[(idx / GCH) * GS + 8 * (idx % GCH)] = gv[i];
        }
        __syncthreads();
        if (P + 1 < pe) load(P + 1);
        // wavefront group wt takes taps 9 wt / WT .. 9 (wt + 1) / WT - 1
        if (WT == 1) {
            wgrad_halo_stage<PW, XS, GS, 0, 9, NTAP>(xr[0], xr[1], gr[0], gr[1], acc);
        } else if (WT == 2) {
            if (wt == 0) wgrad_halo_stage<PW, XS, GS, 0, 4, NTAP>(xr[0], xr[1], gr[0], gr[1], acc);
            else wgrad_halo_stage<PW, XS, GS, 4, 9, NTAP>(xr[0], xr[1], gr[0], gr[1], acc);
        } else {
            if (wt == 0) wgrad_halo_stage<PW, XS, GS, 0, 2, NTAP>(xr[0], xr[1], gr[0], gr[1], acc);
            else if (wt == 1) wgrad_halo_stage<PW, XS, GS, 2, 4, NTAP>(xr[0], xr[1], gr[0], gr[1], acc);
            else if (wt == 2) wgrad_halo_stage<PW, XS, GS, 4, 6, NTAP>(xr[0], xr[1], gr[0], gr[1], acc);
            else wgrad_halo_stage<PW, XS, GS, 6, 9, NTAP>(xr[0], xr[1], gr[0], gr[1], acc);
        }
    }
    // acc[j][i][q]: row r0 + 32 wr + 16 i + 4 (lane >> 4) + q, channel ci0 + 16 wc + (lane & 15), tap T0 + j
    float *dst = part + (long long)blockIdx.z * rows * a.K;
    // 3D: the launch of plane offset dz holds taps 9 (dz + 1) .. 9 (dz + 1) + 8
    const int t0 = 9 * wt / WT + (a.dims == 3 ? 9 * (dz + 1) : 0), nt = 9 * (wt + 1) / WT - 9 * wt / WT;
    const int ci = ci0 + 16 * wc + (lane & 15);
    if (ci >= a.cin) return;                              // the zero channels of a 16-channel tile over 8
#pragma unroll
    for (int j = 0; j < NTAP; ++j) {
        if (j >= nt) break;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int rr = r0 + 32 * wr + 16 * i + 4 * (lane >> 4) + q;
                if (rr < rows) dst[(long long)rr * a.K + (t0 + j) * a.cin + ci] = acc[j][i][q];
            }
    }
}

// Sum of split partials: a block takes 64 outputs, its four wavefronts the
// splits z = w, w + 4, ... (coalesced 64-float rows), combined in a fixed
// order (deterministic).
__global__ void __launch_bounds__(256) k_sum_splits(const float *__restrict__ part, int splits, long long n,
                                                    long long row, float *__restrict__ out, int accumulate) {
    __shared__ float sh[4][64];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long long i = (long long)blockIdx.x * 64 + l;
    float s = 0.f;
    if (i < n)
        for (int z = w; z < splits; z += 4) s += part[(long long)z * row + i];
    sh[w][l] = s;
    __syncthreads();
    if (w == 0 && i < n) {
        const float v = (sh[0][l] + sh[1][l]) + (sh[2][l] + sh[3][l]);
        out[i] = accumulate ? out[i] + v : v;
    }
}

// First pass of a long split sum: thread (i, c) adds the partials of splits
// c S .. c S + S - 1 of output i in order and stores the sum over split
// c S's own partial, which no other thread reads; k_sum_splits then adds
// the chunk sums (row stride S n), in order.
__global__ void __launch_bounds__(256) k_sum_split_chunks(float *__restrict__ part, int splits, long long n, int S) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int z0 = (int)blockIdx.y * S, z1 = min(z0 + S, splits);
    float s = 0.f;
#pragma unroll 8
    for (int z = z0; z < z1; ++z) s += part[(long long)z * n + i];
    part[(long long)z0 * n + i] = s;
}

// Sum of split partials when there are few outputs: one block per output,
// the threads stride over the splits, then a fixed-order tree (deterministic).
__global__ void __launch_bounds__(256) k_sum_splits_narrow(const float *__restrict__ part, int splits, long long n,
                                                           float *__restrict__ out, int accumulate) {
    __shared__ float sh[256];
    const long long i = blockIdx.x;
    float acc = 0.f;
    for (int z = threadIdx.x; z < splits; z += 256) acc += part[(long long)z * n + i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = accumulate ? out[i] + sh[0] : sh[0];
}

// Bias gradient partials with 16-byte loads (channel stride, offset and
// count multiples of 8, C <= 2048): a thread sums 8 channels of every
// (256 / (C/8))-th pixel of the split; LDS combines the pixel lanes.
// Bias gradient partials, 8 channels per thread with 16-byte loads.  RELU:
// first the ReLU backward in the same pass, g = 0 where y <= 0 (written back),
// then the masked g is summed (the same sums, in the same order, as the two
// passes one after the other).
template <bool RELU>
__global__ void __launch_bounds__(256) k_bias_grad8(uint16_t *__restrict__ g, const uint16_t *__restrict__ y,
                                                    int cs, int co, long long npix, int C, long long chunk,
                                                    float *__restrict__ part) {
    __shared__ float sh[256 * 8];
    const int tpp = C >> 3;                    // threads per pixel
    const int ppi = 256 / tpp;                 // pixels per iteration
    const int gi = threadIdx.x % tpp, pi = threadIdx.x / tpp;
    const long long mb = (long long)blockIdx.x * chunk;
    const long long me = mb + chunk < npix ? mb + chunk : npix;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (pi < ppi)
#pragma unroll 4
        for (long long m = mb + pi; m < me; m += ppi) {
            uint4 v = *(const uint4 *)(g + m * cs + co + gi * 8);
            if (RELU) {
                const uint4 yv = *(const uint4 *)(y + m * cs + co + gi * 8);
                const uint32_t y4[4] = {yv.x, yv.y, yv.z, yv.w};
                uint32_t g4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (!(bf2f((uint16_t)(y4[j] & 0xffffu)) > 0.f)) g4[j] &= 0xffff0000u;
                    if (!(bf2f((uint16_t)(y4[j] >> 16)) > 0.f)) g4[j] &= 0x0000ffffu;
                }
                v = make_uint4(g4[0], g4[1], g4[2], g4[3]);
                *(uint4 *)(g + m * cs + co + gi * 8) = v;
            }
            const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                acc[2 * j] += bf2f((uint16_t)(w4[j] & 0xffffu));
                acc[2 * j + 1] += bf2f((uint16_t)(w4[j] >> 16));
            }
        }
#pragma unroll
    for (int j = 0; j < 8; ++j) sh[threadIdx.x * 8 + j] = pi < ppi ? acc[j] : 0.f;
    __syncthreads();
    for (int c = threadIdx.x; c < C; c += 256) {
        const int gc = c >> 3, j = c & 7;
        float sum = 0.f;
        for (int p = 0; p < ppi; ++p) sum += sh[(p * tpp + gc) * 8 + j];
        part[(long long)blockIdx.x * C + c] = sum;
    }
}

// Bias gradient partials: part[split][c] = sum over the split's pixels.
__global__ void __launch_bounds__(256) k_bias_grad(const uint16_t *__restrict__ g, int cs, int co, long long npix,
                                                   int C, long long chunk, float *__restrict__ part) {
    __shared__ float s[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), pl = threadIdx.x >> 6;
    const long long mb = (long long)blockIdx.y * chunk;
    const long long me = mb + chunk < npix ? mb + chunk : npix;
    float acc = 0.f;
    if (c < C)
        for (long long m = mb + pl; m < me; m += 4) acc += bf2f(g[m * cs + co + c]);
    s[pl][threadIdx.x & 63] = acc;
    __syncthreads();
    if (pl == 0 && c < C) part[(long long)blockIdx.y * C + c] = s[0][threadIdx.x] + s[1][threadIdx.x] + s[2][threadIdx.x] + s[3][threadIdx.x];
}

__global__ void k_relu_bwd(uint16_t *__restrict__ g, const uint16_t *__restrict__ y, int cs, int co,
                           long long npix, int C) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npix * C) return;
    const long long m = i / C;
    const int c = (int)(i - m * C);
    const long long o = m * cs + co + c;
    if (!(bf2f(y[o]) > 0.f)) g[o] = 0;
}

// 2x2(x2) max pooling, stride 2; (d, h, w) is the coarse grid.
__global__ void k_pool_fwd(const uint16_t *__restrict__ in, int in_cs, int in_co, uint16_t *__restrict__ out,
                           int out_cs, int out_co, int n, int d, int h, int w, int C, int dims) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)n * d * h * w * C;
    if (i >= total) return;
    const long long m = i / C;
    const int c = (int)(i - m * C);
    const Pix p = pix_of(m, d, h, w);
    const int fd = dims == 3 ? 2 * d : 1;
    float best = -INFINITY;
    for (int sub = 0; sub < (1 << dims); ++sub) {
        const int sx = sub & 1, sy = (sub >> 1) & 1, sz = (sub >> 2) & 1;
        const int zf = dims == 3 ? 2 * p.z + sz : 0;
        const long long f = (((long long)p.b * fd + zf) * (2 * h) + 2 * p.y + sy) * (2 * w) + 2 * p.x + sx;
        best = fmaxf(best, bf2f(in[f * in_cs + in_co + c]));
    }
    out[m * out_cs + out_co + c] = f2bf(best);
}

// Routes dout to the first maximal element of each window (sub order).
__global__ void k_pool_bwd(const uint16_t *__restrict__ in, int in_cs, int in_co,
                           const uint16_t *__restrict__ gout, int g_cs, int g_co, uint16_t *__restrict__ gin,
                           int gi_cs, int gi_co, int n, int d, int h, int w, int C, int dims, int accumulate) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)n * d * h * w * C;
    if (i >= total) return;
    const long long m = i / C;
    const int c = (int)(i - m * C);
    const Pix p = pix_of(m, d, h, w);
    const int fd = dims == 3 ? 2 * d : 1;
    float best = -INFINITY;
    int arg = 0;
    long long fidx[8];
    for (int sub = 0; sub < (1 << dims); ++sub) {
        const int sx = sub & 1, sy = (sub >> 1) & 1, sz = (sub >> 2) & 1;
        const int zf = dims == 3 ? 2 * p.z + sz : 0;
        fidx[sub] = (((long long)p.b * fd + zf) * (2 * h) + 2 * p.y + sy) * (2 * w) + 2 * p.x + sx;
        const float v = bf2f(in[fidx[sub] * in_cs + in_co + c]);
        if (v > best) { best = v; arg = sub; }
    }
    const float gv = bf2f(gout[m * g_cs + g_co + c]);
    for (int sub = 0; sub < (1 << dims); ++sub) {
        const long long o = fidx[sub] * gi_cs + gi_co + c;
        const float add = sub == arg ? gv : 0.f;
        if (accumulate) { if (sub == arg) gin[o] = f2bf(bf2f(gin[o]) + add); }
        else gin[o] = f2bf(add);
    }
}

// The same two passes on 8 channels of a pixel per thread with 16-byte
// accesses (channel counts, strides and offsets multiples of 8, 16-byte
// aligned buffers); per channel the same operations in the same order.
__device__ inline void unpack8(uint4 v, float (&f)[8]) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        f[2 * k] = bf2f((uint16_t)(w[k] & 0xffffu));
        f[2 * k + 1] = bf2f((uint16_t)(w[k] >> 16));
    }
}
__device__ inline uint4 pack8(const float (&f)[8]) {
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = (uint32_t)f2bf(f[2 * k]) | ((uint32_t)f2bf(f[2 * k + 1]) << 16);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

__global__ void __launch_bounds__(256) k_pool_fwd8(const uint16_t *__restrict__ in, int in_cs, int in_co,
                                                   uint16_t *__restrict__ out, int out_cs, int out_co, int n, int d,
                                                   int h, int w, int C, int dims) {
    const int CG = C >> 3;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * d * h * w * CG) return;
    const long long m = i / CG;
    const int c = (int)(i - m * CG) * 8;
    const Pix p = pix_of(m, d, h, w);
    const int fd = dims == 3 ? 2 * d : 1;
    float best[8], v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) best[k] = -INFINITY;
    for (int sub = 0; sub < (1 << dims); ++sub) {
        const int sx = sub & 1, sy = (sub >> 1) & 1, sz = (sub >> 2) & 1;
        const int zf = dims == 3 ? 2 * p.z + sz : 0;
        const long long f = (((long long)p.b * fd + zf) * (2 * h) + 2 * p.y + sy) * (2 * w) + 2 * p.x + sx;
        unpack8(*(const uint4 *)(in + f * in_cs + in_co + c), v);
#pragma unroll
        for (int k = 0; k < 8; ++k) best[k] = fmaxf(best[k], v[k]);
    }
    *(uint4 *)(out + m * out_cs + out_co + c) = pack8(best);
}

__global__ void __launch_bounds__(256) k_pool_bwd8(const uint16_t *__restrict__ in, int in_cs, int in_co,
                                                   const uint16_t *__restrict__ gout, int g_cs, int g_co,
                                                   uint16_t *__restrict__ gin, int gi_cs, int gi_co, int n, int d,
                                                   int h, int w, int C, int dims, int accumulate) {
    const int CG = C >> 3;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * d * h * w * CG) return;
    const long long m = i / CG;
    const int c = (int)(i - m * CG) * 8;
    const Pix p = pix_of(m, d, h, w);
    const int fd = dims == 3 ? 2 * d : 1;
    float best[8], v[8], gv[8];
    int arg[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) { best[k] = -INFINITY; arg[k] = 0; }
    long long fidx[8];
    for (int sub = 0; sub < (1 << dims); ++sub) {
        const int sx = sub & 1, sy = (sub >> 1) & 1, sz = (sub >> 2) & 1;
        const int zf = dims == 3 ? 2 * p.z + sz : 0;
        fidx[sub] = (((long long)p.b * fd + zf) * (2 * h) + 2 * p.y + sy) * (2 * w) + 2 * p.x + sx;
        unpack8(*(const uint4 *)(in + fidx[sub] * in_cs + in_co + c), v);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (v[k] > best[k]) { best[k] = v[k]; arg[k] = sub; }
    }
    unpack8(*(const uint4 *)(gout + m * g_cs + g_co + c), gv);
    for (int sub = 0; sub < (1 << dims); ++sub) {
        uint16_t *o = gin + fidx[sub] * gi_cs + gi_co + c;
        float r[8];
        if (accumulate) {
            unpack8(*(const uint4 *)o, r);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (sub == arg[k]) r[k] = r[k] + gv[k];
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) r[k] = sub == arg[k] ? gv[k] : 0.f;
        }
        *(uint4 *)o = pack8(r);
    }
}

// Masked MSE over the first `creal` channels of an FP32 prediction with
// channel stride pcs: loss = scale * sum_m w_m sum_c (p - t)^2 and the BF16
// gradient (pad channels zero).  Per-block partial sums in FP64.
__global__ void __launch_bounds__(256) k_mse(const float *__restrict__ pred, int pcs, const float *__restrict__ tgt,
                                             const float *__restrict__ wpix, int creal, long long npix,
                                             float scale, uint16_t *__restrict__ dpred, double *__restrict__ part) {
    __shared__ double s[256];
    const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (m < npix) {
        const float wm = wpix ? wpix[m] : 1.f;
        for (int c = 0; c < pcs; ++c) {
            float gval = 0.f;
            if (c < creal) {
                const float d = pred[m * pcs + c] - tgt[m * creal + c];
                l += (double)(wm * d * d);
                gval = 2.f * scale * wm * d;
            }
            dpred[m * pcs + c] = f2bf(gval);
        }
    }
    s[threadIdx.x] = l * scale;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void k_sum_f64(const double *__restrict__ part, long long n, double *__restrict__ out) {
    __shared__ double s[256];
    double a = 0.0;
    for (long long i = threadIdx.x; i < n; i += 256) a += part[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// Adam on FP32 master weights with an optional BF16 mirror.
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, uint16_t *__restrict__ wb, long long n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    const float v = w[i] - lr * (a * c1) / (sqrtf(b * c2) + eps);
    w[i] = v;
    if (wb) wb[i] = f2bf(v);
}

__global__ void k_to_bf16(const float *__restrict__ x, uint16_t *__restrict__ y, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// Network input: 8 channels per pixel: solid, x / (nx - 1), 200 drho_in,
// 200 drho_out, 2 (tau - 0.9), 0, 0, 0.  prm: [n][3] = (drho_in, drho_out, tau).
__global__ void k_features(const uint8_t *__restrict__ solid, const float *__restrict__ prm, int n, int d,
                           int h, int w, uint16_t *__restrict__ out) {
    const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= (long long)n * d * h * w) return;
    const Pix p = pix_of(m, d, h, w);
    const float *q = prm + 3 * p.b;
    float f[8] = {(float)solid[m], w > 1 ? (float)p.x / (float)(w - 1) : 0.f, 200.f * q[0], 200.f * q[1],
                  2.f * (q[2] - 0.9f), 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 8; ++c) out[m * 8 + c] = f2bf(f[c]);
}

// Stokes-scaled targets from LBM fields (and back):
//   t0 = (drho - drho_out) / (drho_in - drho_out),
//   t_{1+a} = u_a nu / (cs^2 (drho_in - drho_out)),  nu = (tau - 1/2) / 3.
__global__ void k_normalize(const float *__restrict__ drho, const float *__restrict__ u, const uint8_t *__restrict__ solid,
                            const float *__restrict__ prm, long long per_sample, int D, long long npix,
                            float *__restrict__ tgt, float *__restrict__ wpix) {
    const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= npix) return;
    const float *q = prm + 3 * (m / per_sample);
    const float dr = q[0] - q[1], nu = (q[2] - 0.5f) / 3.f;
    const float su = nu / (dr / 3.f);
    const bool fl = solid[m] == 0;
    tgt[m * (1 + D)] = fl ? (drho[m] - q[1]) / dr : 0.f;
    for (int a = 0; a < D; ++a) tgt[m * (1 + D) + 1 + a] = fl ? u[m * D + a] * su : 0.f;
    if (wpix) wpix[m] = fl ? 1.f : 0.f;
}

__global__ void k_denormalize(const float *__restrict__ pred, int pcs, const uint8_t *__restrict__ solid,
                              const float *__restrict__ prm, long long per_sample, int D, long long npix,
                              float *__restrict__ drho, float *__restrict__ u) {
    const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= npix) return;
    const float *q = prm + 3 * (m / per_sample);
    const float dr = q[0] - q[1], nu = (q[2] - 0.5f) / 3.f;
    const float su = (dr / 3.f) / nu;
    const bool fl = solid[m] == 0;
    drho[m] = fl ? q[1] + dr * pred[m * pcs] : 0.f;
    for (int a = 0; a < D; ++a) u[m * D + a] = fl ? pred[m * pcs + 1 + a] * su : 0.f;
}

// Cross-section flux balance in three launches, FP64 sums in a fixed order:
// block (p, b) sums u_x over the fluid nodes of each section x within row
// chunk p of sample b (thread t of a pass over `cols` sections takes the
// rows t / cols, t / cols + groups, ... of section t % cols; the groups are
// then added in order) into part[b][p][x]; one block per sample adds the
// chunks in order to Q(x), averages Q over the sections to Qbar and writes
// the scale factors S[b][x] = clamp(Qbar / max(Q(x), Qbar / 10), 1/4, 4)
// (all 1 when Qbar <= 0); the last launch scales every value.
constexpr int FB_MAX_W = 2048, FB_MAX_CHUNKS = 64, FB_MIN_ROWS = 16;

__host__ __device__ inline int fb_chunks(long long rows) {
    const long long c = (rows + FB_MIN_ROWS - 1) / FB_MIN_ROWS;
    return (int)(c < FB_MAX_CHUNKS ? c : FB_MAX_CHUNKS);
}

__global__ void __launch_bounds__(256) k_fb_partial(const uint8_t *__restrict__ solid, const float *__restrict__ u,
                                                    int rows, int w, int D, double *__restrict__ part) {
    __shared__ double red[256];
    const int t = threadIdx.x, p = blockIdx.x, b = blockIdx.y, P = gridDim.x;
    const long long per = (long long)rows * w;
    const int r0 = (int)((long long)rows * p / P), r1 = (int)((long long)rows * (p + 1) / P);
    for (int x0 = 0; x0 < w; x0 += 256) {
        const int cols = w - x0 < 256 ? w - x0 : 256, groups = 256 / cols;
        const int x = x0 + t % cols, g = t / cols;
        double acc = 0.0;
        if (g < groups)
            for (int r = r0 + g; r < r1; r += groups) {
                const long long m = b * per + (long long)r * w + x;
                const float v = u[m * D];
                acc += solid[m] ? 0.0 : (double)v;
            }
        red[t] = acc;
        __syncthreads();
        if (t < cols) {
            double q = 0.0;
            for (int k = 0; k < groups; ++k) q += red[k * cols + t];
            part[((long long)b * P + p) * w + x0 + t] = q;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_fb_factors(const double *__restrict__ part, int P, int w,
                                                    float *__restrict__ S) {
    __shared__ double Q[FB_MAX_W];
    __shared__ double qbar;
    const int t = threadIdx.x, b = blockIdx.x;
    for (int x = t; x < w; x += 256) {
        double q = 0.0;
        for (int p = 0; p < P; ++p) q += part[((long long)b * P + p) * w + x];
        Q[x] = q;
    }
    __syncthreads();
    if (t == 0) {
        double q = 0.0;
        for (int x = 0; x < w; ++x) q += Q[x];
        qbar = q / w;
    }
    __syncthreads();
    const double qb = qbar;
    for (int x = t; x < w; x += 256) {
        double sc = 1.0;
        if (qb > 0.0) {
            sc = qb / (Q[x] > 0.1 * qb ? Q[x] : 0.1 * qb);
            sc = sc < 0.25 ? 0.25 : (sc > 4.0 ? 4.0 : sc);
        }
        S[(long long)b * w + x] = (float)sc;
    }
}

__global__ void __launch_bounds__(256) k_fb_apply(float *__restrict__ u, const float *__restrict__ S, long long n,
                                                  long long per, int w, int D) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const long long node = i / D;                      // node of the whole batch, per nodes per sample
    const long long b = node / per;
    const int x = (int)(node % w);
    u[i] *= S[b * w + x];
}

// ------------------------------------------------------------ launchers --
static inline unsigned blocks(long long n, int b) { return (unsigned)((n + b - 1) / b); }

static bool halo_ok(const ConvArgs &a) {
    const uintptr_t ob = a.out32 ? (uintptr_t)a.out32 : (uintptr_t)a.out;
    return (a.dims == 2 || a.dims == 3) && a.ks == 3 && !(a.flags & (FLAG_S2D | FLAG_D2S)) && a.cin % 8 == 0 &&
           a.h % HY == 0 &&
           a.w % HX == 0 && ((a.in_cs | a.in_co | a.out_cs | a.out_co) & 7) == 0 && ((uintptr_t)a.in & 15) == 0 &&
           (ob & 15) == 0;
}

// Sum of the K splits of a convolution, in split order, then the epilogue
// of k_conv (bias, ReLU, accumulate, FP32 or BF16 output, D2S scatter): one
// thread per output element.
__global__ void __launch_bounds__(256) k_conv_reduce(ConvArgs a, const float *__restrict__ part, int S) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= a.M * a.ncols) return;
    const long long m = e / a.ncols;
    const int c = (int)(e - m * a.ncols);
    float v = 0.f;
    for (int z = 0; z < S; ++z) v += part[(long long)z * a.M * a.ncols + e];
    int bc;
    const long long o = out_index(a, m, c, bc);
    v += a.bias ? a.bias[bc] : 0.f;
    if (a.flags & FLAG_RELU) v = v > 0.f ? v : 0.f;
    if (a.out32) {
        a.out32[o] = (a.flags & FLAG_ACC) ? a.out32[o] + v : v;
    } else {
        if (a.flags & FLAG_ACC) v += bf2f(a.out[o]);
        a.out[o] = f2bf(v);
    }
}

// K splits for a convolution whose output tiles are too few to fill the
// GPU (the deep, low-resolution layers, whose long K loop would run on a
// few CUs): enough splits for about 1024 blocks, each at least 4 K steps of
// 64; 1 when the layer has 512 tiles or more, or takes the halo kernel.
static long long conv_tiles(const ConvArgs &a) {
    return (long long)blocks(a.M, 64) * (a.ncols <= 32 ? 1 : (a.ncols + 63) / 64);
}
static bool conv_halo(const ConvArgs &a) {
    const long long tiles = halo_ok(a) ? (long long)a.n * a.d * (a.h / HY) * (a.w / HX) : 0;
    return tiles * (a.ncols <= 32 ? 1 : (a.ncols + 63) / 64) >= 512;
}
int conv_splits(const ConvArgs &a) {
    const long long tiles = conv_tiles(a);
    if (conv_halo(a) || tiles >= 512) return 1;
    const int steps = (a.K + 63) / 64;
    long long sp = (1024 + tiles - 1) / tiles;
    sp = sp < steps / 4 ? sp : steps / 4;
    if (sp < 2) return 1;
    const int sper = (int)((steps + sp - 1) / sp);
    return (steps + sper - 1) / sper;
}

hipError_t conv_split(const ConvArgs &a, float *part, int S, hipStream_t s) {
    const int steps = (a.K + 63) / 64, sper = (steps + S - 1) / S;
    if (a.ncols <= 32) {
        dim3 grid(blocks(a.M, 64), (unsigned)((a.ncols + 31) / 32), (unsigned)S);
        hipLaunchKernelGGL((k_conv<64, 32, true>), grid, dim3(256), 0, s, a, part, sper);
    } else {
        dim3 grid(blocks(a.M, 64), (unsigned)((a.ncols + 63) / 64), (unsigned)S);
        hipLaunchKernelGGL((k_conv<64, 64, true>), grid, dim3(256), 0, s, a, part, sper);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_conv_reduce, dim3(blocks(a.M * a.ncols, 256)), dim3(256), 0, s, a, part, S);
    return hipGetLastError();
}

hipError_t conv(const ConvArgs &a, hipStream_t s) {
    // the halo kernel holds 2 - 3 blocks per CU: below 512 blocks the im2col kernel fills the chip better
    const long long tiles = halo_ok(a) ? (long long)a.n * a.d * (a.h / HY) * (a.w / HX) : 0;
    if (conv_halo(a)) {
        const dim3 grid((unsigned)tiles, a.ncols <= 32 ? 1u : (unsigned)((a.ncols + 63) / 64));
        if (a.dims == 3) {
            if (a.ncols <= 32) hipLaunchKernelGGL((k_conv3x3_halo<32, 3>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((k_conv3x3_halo<64, 3>), grid, dim3(256), 0, s, a);
        } else {
            if (a.ncols <= 32) hipLaunchKernelGGL((k_conv3x3_halo<32, 2>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((k_conv3x3_halo<64, 2>), grid, dim3(256), 0, s, a);
        }
        return hipGetLastError();
    }
    if (a.ncols <= 32) {
        dim3 grid(blocks(a.M, 64), (unsigned)((a.ncols + 31) / 32));
        hipLaunchKernelGGL((k_conv<64, 32>), grid, dim3(256), 0, s, a);
    } else {
        dim3 grid(blocks(a.M, 64), (unsigned)((a.ncols + 63) / 64));
        hipLaunchKernelGGL((k_conv<64, 64>), grid, dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

long long wgrad_chunk(long long M, int splits) {
    long long c = (M + splits - 1) / splits;
    return (c + WPB - 1) / WPB * WPB;
}

// Sum of z split partials into n outputs: a block per output when there are
// few; else a thread per output and four wavefronts over the splits, after a
// first pass that adds chunks of 8 splits in place when there are more than
// 32 (each partial is added once, in split order within a chunk and in chunk
// order after; deterministic).
static hipError_t sum_splits(float *part, int z, long long n, float *out, int accumulate, hipStream_t s) {
    if (n <= 8192 && z > 16) {
        hipLaunchKernelGGL(k_sum_splits_narrow, dim3((unsigned)n), dim3(256), 0, s, part, z, n, out, accumulate);
        return hipGetLastError();
    }
    long long row = n;
    if (z > 32) {
        constexpr int S = 8;
        const int chunks = (z + S - 1) / S;
        hipLaunchKernelGGL(k_sum_split_chunks, dim3(blocks(n, 256), (unsigned)chunks), dim3(256), 0, s, part, z, n, S);
        z = chunks;
        row = S * n;
    }
    hipLaunchKernelGGL(k_sum_splits, dim3(blocks(n, 64)), dim3(256), 0, s, part, z, n, row, out, accumulate);
    return hipGetLastError();
}

// The halo kernel's block shape for a layer, or 0: (WR, WC) = (2, 2) for
// 64-row multiples, (1, 4) for 32 rows of 64-channel multiples, (1, 2) (taps
// split over two wavefront pairs) for 32 rows of 32-channel multiples, (1, 1)
// (taps split over the four wavefronts) for 32 rows of 8 channels.
static int halo_shape(const ConvArgs &a, int rows) {
    if (a.ks != 3 || (a.flags & (FLAG_S2D | FLAG_D2S | FLAG_S2D_G)) || a.w < 16) return 0;
    if (rows % 64 == 0 && a.cin % 32 == 0) return 22;
    if (rows % 32 == 0 && a.cin % 64 == 0) return 14;
    if (rows % 32 == 0 && a.cin % 32 == 0) return 12;
    if (rows % 32 == 0 && a.cin == 8) return 11;
    return 0;
}

template <int PW>
static void launch_wgrad_halo(int shape, const ConvArgs &a, const uint16_t *g, int g_cs, int g_co, int rows,
                              float *part, int z, int per, int dz, hipStream_t s) {
    const int RB = shape == 22 ? 64 : 32, CB = shape == 22 ? 32 : shape == 14 ? 64 : shape == 12 ? 32 : 16;
    const dim3 grid((unsigned)(rows / RB), (unsigned)((a.cin + CB - 1) / CB), (unsigned)z);
    if (shape == 22)
        hipLaunchKernelGGL((k_wgrad_halo<PW, 2, 2>), grid, dim3(256), 0, s, a, g, g_cs, g_co, rows, part, per, dz);
    else if (shape == 14)
        hipLaunchKernelGGL((k_wgrad_halo<PW, 1, 4>), grid, dim3(256), 0, s, a, g, g_cs, g_co, rows, part, per, dz);
    else if (shape == 12)
        hipLaunchKernelGGL((k_wgrad_halo<PW, 1, 2>), grid, dim3(256), 0, s, a, g, g_cs, g_co, rows, part, per, dz);
    else
        hipLaunchKernelGGL((k_wgrad_halo<PW, 1, 1>), grid, dim3(256), 0, s, a, g, g_cs, g_co, rows, part, per, dz);
}

hipError_t wgrad(const ConvArgs &a, const uint16_t *g, int g_cs, int g_co, int rows, float *part, int splits,
                 float *dw, int accumulate, hipStream_t s) {
    const long long chunk = wgrad_chunk(a.M, splits);
    int z = (int)((a.M + chunk - 1) / chunk);
    if (const int shape = halo_shape(a, rows)) {
        // patches of 4 x 32 (or 8 x 16 when w <= 16) pixels, split into at
        // most as many ranges as the workspace holds partials for
        // 3D: one launch per plane offset dz = -1, 0, 1, each the 9 taps of its
        // plane pair, written to disjoint columns of the same partials
        const int pw = a.w > 16 ? 32 : 16, ph = 128 / pw;
        const long long npt = (long long)a.n * a.d * ((a.h + ph - 1) / ph) * ((a.w + pw - 1) / pw);
        const int per = (int)((npt + z - 1) / z);
        z = (int)((npt + per - 1) / per);
        for (int dz = a.dims == 3 ? -1 : 0; dz <= (a.dims == 3 ? 1 : 0); ++dz) {
            if (pw == 32)
                launch_wgrad_halo<32>(shape, a, g, g_cs, g_co, rows, part, z, per, dz, s);
            else
                launch_wgrad_halo<16>(shape, a, g, g_cs, g_co, rows, part, z, per, dz, s);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return sum_splits(part, z, (long long)rows * a.K, dw, accumulate, s);
    }
    if (rows <= 32) {
        const dim3 grid(1u, (unsigned)((a.K + 127) / 128), (unsigned)z);
        hipLaunchKernelGGL(k_wgrad<true>, grid, dim3(256), 0, s, a, g, g_cs, g_co, rows, part, chunk);
    } else {
        const dim3 grid((unsigned)((rows + BM - 1) / BM), (unsigned)((a.K + BN - 1) / BN), (unsigned)z);
        hipLaunchKernelGGL(k_wgrad<false>, grid, dim3(256), 0, s, a, g, g_cs, g_co, rows, part, chunk);
    }
    const long long n = (long long)rows * a.K;
    return sum_splits(part, z, n, dw, accumulate, s);
}

bool bias_grad8_ok(const void *g, int cs, int co, int C) {
    return cs % 8 == 0 && co % 8 == 0 && C % 8 == 0 && C <= 2048 && ((uintptr_t)g & 15) == 0;
}

hipError_t relu_bwd_bias_grad(uint16_t *g, const uint16_t *y, int cs, int co, long long npix, int C, float *part,
                              int splits, float *db, int accumulate, hipStream_t s) {
    if (!bias_grad8_ok(g, cs, co, C) || ((uintptr_t)y & 15) != 0) {
        hipError_t e = relu_bwd(g, y, cs, co, npix, C, s);
        return e != hipSuccess ? e : bias_grad(g, cs, co, npix, C, part, splits, db, accumulate, s);
    }
    const long long chunk = (npix + splits - 1) / splits;
    const int z = (int)((npix + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_bias_grad8<true>, dim3((unsigned)z), dim3(256), 0, s, g, y, cs, co, npix, C, chunk, part);
    return sum_splits(part, z, (long long)C, db, accumulate, s);
}

hipError_t bias_grad(const uint16_t *g, int cs, int co, long long npix, int C, float *part, int splits, float *db,
                     int accumulate, hipStream_t s) {
    const long long chunk = (npix + splits - 1) / splits;
    const int z = (int)((npix + chunk - 1) / chunk);
    if (bias_grad8_ok(g, cs, co, C)) {
        hipLaunchKernelGGL(k_bias_grad8<false>, dim3((unsigned)z), dim3(256), 0, s, (uint16_t *)g, nullptr, cs, co,
                           npix, C, chunk, part);
    } else {
        dim3 grid((unsigned)((C + 63) / 64), (unsigned)z);
        hipLaunchKernelGGL(k_bias_grad, grid, dim3(256), 0, s, g, cs, co, npix, C, chunk, part);
    }
    return sum_splits(part, z, (long long)C, db, accumulate, s);
}

hipError_t relu_bwd(uint16_t *g, const uint16_t *y, int cs, int co, long long npix, int C, hipStream_t s) {
    hipLaunchKernelGGL(k_relu_bwd, dim3(blocks(npix * C, 256)), dim3(256), 0, s, g, y, cs, co, npix, C);
    return hipGetLastError();
}

static bool vec8(int a, int b, int c, int e, int f, const void *p, const void *q) {
    return ((a | b | c | e | f) & 7) == 0 && (((uintptr_t)p | (uintptr_t)q) & 15) == 0;
}

hipError_t pool_fwd(const uint16_t *in, int in_cs, int in_co, uint16_t *out, int out_cs, int out_co, int n, int d,
                    int h, int w, int C, int dims, hipStream_t s) {
    const long long tot = (long long)n * d * h * w * C;
    if (vec8(C, in_cs, in_co, out_cs, out_co, in, out)) {
        hipLaunchKernelGGL(k_pool_fwd8, dim3(blocks(tot / 8, 256)), dim3(256), 0, s, in, in_cs, in_co, out, out_cs,
                           out_co, n, d, h, w, C, dims);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_pool_fwd, dim3(blocks(tot, 256)), dim3(256), 0, s, in, in_cs, in_co, out, out_cs, out_co,
                       n, d, h, w, C, dims);
    return hipGetLastError();
}

hipError_t pool_bwd(const uint16_t *in, int in_cs, int in_co, const uint16_t *gout, int g_cs, int g_co,
                    uint16_t *gin, int gi_cs, int gi_co, int n, int d, int h, int w, int C, int dims, int acc,
                    hipStream_t s) {
    const long long tot = (long long)n * d * h * w * C;
    if (vec8(C, in_cs, in_co, g_cs, g_co, in, gout) && vec8(gi_cs, gi_co, 0, 0, 0, gin, nullptr)) {
        hipLaunchKernelGGL(k_pool_bwd8, dim3(blocks(tot / 8, 256)), dim3(256), 0, s, in, in_cs, in_co, gout, g_cs,
                           g_co, gin, gi_cs, gi_co, n, d, h, w, C, dims, acc);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_pool_bwd, dim3(blocks(tot, 256)), dim3(256), 0, s, in, in_cs, in_co, gout, g_cs, g_co, gin,
                       gi_cs, gi_co, n, d, h, w, C, dims, acc);
    return hipGetLastError();
}

hipError_t mse(const float *pred, int pcs, const float *tgt, const float *wpix, int creal, long long npix,
               float scale, uint16_t *dpred, double *part, double *loss, hipStream_t s) {
    const unsigned nb = blocks(npix, 256);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, pred, pcs, tgt, wpix, creal, npix, scale, dpred, part);
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, s, part, (long long)nb, loss);
    return hipGetLastError();
}

hipError_t adam(float *w, const float *g, float *m1, float *m2, uint16_t *wb, long long n, float lr, float b1,
                float b2, float eps, int t, hipStream_t s) {
    const float c1 = 1.f / (1.f - powf(b1, (float)t)), c2 = 1.f / (1.f - powf(b2, (float)t));
    hipLaunchKernelGGL(k_adam, dim3(blocks(n, 256)), dim3(256), 0, s, w, g, m1, m2, wb, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t to_bf16(const float *x, uint16_t *y, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks(n, 256)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

hipError_t features(const uint8_t *solid, const float *prm, int n, int d, int h, int w, uint16_t *out,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_features, dim3(blocks((long long)n * d * h * w, 256)), dim3(256), 0, s, solid, prm, n, d, h,
                       w, out);
    return hipGetLastError();
}

hipError_t normalize(const float *drho, const float *u, const uint8_t *solid, const float *prm, long long per_sample,
                     int D, long long npix, float *tgt, float *wpix, hipStream_t s) {
    hipLaunchKernelGGL(k_normalize, dim3(blocks(npix, 256)), dim3(256), 0, s, drho, u, solid, prm, per_sample, D, npix,
                       tgt, wpix);
    return hipGetLastError();
}

long long flux_balance_workspace_bytes(int n, long long rows, int w) {
    return (long long)n * w * (fb_chunks(rows) * (long long)sizeof(double) + (long long)sizeof(float));
}

hipError_t flux_balance(const uint8_t *solid, int n, int rows, int w, int D, float *u, void *ws, hipStream_t s) {
    const int P = fb_chunks(rows);
    double *part = (double *)ws;
    float *S = (float *)(part + (long long)n * P * w);
    hipLaunchKernelGGL(k_fb_partial, dim3((unsigned)P, (unsigned)n), dim3(256), 0, s, solid, u, rows, w, D, part);
    hipLaunchKernelGGL(k_fb_factors, dim3((unsigned)n), dim3(256), 0, s, part, P, w, S);
    const long long per = (long long)rows * w, tot = (long long)n * per * D;
    hipLaunchKernelGGL(k_fb_apply, dim3(blocks(tot, 256)), dim3(256), 0, s, u, S, tot, per, w, D);
    return hipGetLastError();
}

hipError_t denormalize(const float *pred, int pcs, const uint8_t *solid, const float *prm, long long per_sample,
                       int D, long long npix, float *drho, float *u, hipStream_t s) {
    hipLaunchKernelGGL(k_denormalize, dim3(blocks(npix, 256)), dim3(256), 0, s, pred, pcs, solid, prm, per_sample, D,
                       npix, drho, u);
    return hipGetLastError();
}

}  // namespace nn

namespace nn {

// wt[c][tap'][r] = w[r][tap][c], tap' = taps - 1 - tap when flipping (the
// input gradient of a correlation is the correlation with the flipped,
// transposed kernel).
__global__ void k_wtrans(const uint16_t *__restrict__ w, uint16_t *__restrict__ wt, int rows, int taps, int cols,
                         int flip) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)rows * taps * cols;
    if (i >= n) return;
    const int c = (int)(i % cols);
    const int tap = (int)((i / cols) % taps);
    const int r = (int)(i / ((long long)cols * taps));
    const int tp = flip ? taps - 1 - tap : tap;
    wt[((long long)c * taps + tp) * rows + r] = w[i];
}

hipError_t wtrans(const uint16_t *w, uint16_t *wt, int rows, int taps, int cols, int flip, hipStream_t s) {
    const long long n = (long long)rows * taps * cols;
    hipLaunchKernelGGL(k_wtrans, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, wt, rows, taps, cols, flip);
    return hipGetLastError();
}

}  // namespace nn
