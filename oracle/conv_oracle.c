/*
 * FP64 reference of the warm-start network layers -- TEST INFRASTRUCTURE
 * ONLY (tests, smoke check, benchmark baseline).  Shares no code with the
 * GPU path.
 *
 * Direct loops written from the definitions, channels-last tensors
 * [n][d][h][w][C] (d = 1 in 2D):
 *   convolution (zero-padded ks^dims correlation), its input gradient and its
 *   weight gradient, written as the transposes of the forward loop;
 *   2x2(x2) stride-2 transposed convolution and its gradients;
 *   2x2(x2) max pooling and its gradient (first maximum of the window).
 * Weights of a convolution: [cout][tap][cin], tap = (dz*ks + dy)*ks + dx.
 * Transposed convolution weights: [sub][cout][cin], sub = sx + 2 sy + 4 sz.
 */
#include <math.h>
#include <string.h>

static long pix(int b, int z, int y, int x, int d, int h, int w)
{
    return (((long)b * d + z) * h + y) * w + x;
}

static int taps_of(int ks, int dims) { return dims == 3 ? ks * ks * ks : ks * ks; }

static void tap_offset(int tap, int ks, int dims, int *dz, int *dy, int *dx)
{
    int r = ks / 2;
    *dx = tap % ks - r;
    *dy = (tap / ks) % ks - r;
    *dz = dims == 3 ? tap / (ks * ks) - r : 0;
}

void orc_conv_fwd(int n, int d, int h, int w, int cin, int cout, int ks, int dims, const double *x,
                  const double *wt, const double *bias, double *y)
{
    const int T = taps_of(ks, dims);
    for (int b = 0; b < n; b++)
        for (int z = 0; z < d; z++)
            for (int yy = 0; yy < h; yy++)
                for (int xx = 0; xx < w; xx++) {
                    long p = pix(b, z, yy, xx, d, h, w);
                    for (int co = 0; co < cout; co++) {
                        double acc = bias ? bias[co] : 0.0;
                        for (int t = 0; t < T; t++) {
                            int dz, dy, dx;
                            tap_offset(t, ks, dims, &dz, &dy, &dx);
                            int zs = z + dz, ys = yy + dy, xs = xx + dx;
                            if (zs < 0 || zs >= d || ys < 0 || ys >= h || xs < 0 || xs >= w) continue;
                            long q = pix(b, zs, ys, xs, d, h, w);
                            for (int ci = 0; ci < cin; ci++)
                                acc += x[q * cin + ci] * wt[((long)co * T + t) * cin + ci];
                        }
                        y[p * cout + co] = acc;
                    }
                }
}

/* dx = d<y, g>/dx for y = conv(x): every product x[q] wt that reached y[p]
 * sends g[p] wt back to q. */
void orc_conv_dgrad(int n, int d, int h, int w, int cin, int cout, int ks, int dims, const double *g,
                    const double *wt, double *dx)
{
    const int T = taps_of(ks, dims);
    memset(dx, 0, sizeof(double) * (size_t)n * d * h * w * cin);
    for (int b = 0; b < n; b++)
        for (int z = 0; z < d; z++)
            for (int yy = 0; yy < h; yy++)
                for (int xx = 0; xx < w; xx++) {
                    long p = pix(b, z, yy, xx, d, h, w);
                    for (int t = 0; t < T; t++) {
                        int dz, dy, ddx;
                        tap_offset(t, ks, dims, &dz, &dy, &ddx);
                        int zs = z + dz, ys = yy + dy, xs = xx + ddx;
                        if (zs < 0 || zs >= d || ys < 0 || ys >= h || xs < 0 || xs >= w) continue;
                        long q = pix(b, zs, ys, xs, d, h, w);
                        for (int co = 0; co < cout; co++)
                            for (int ci = 0; ci < cin; ci++)
                                dx[q * cin + ci] += g[p * cout + co] * wt[((long)co * T + t) * cin + ci];
                    }
                }
}

void orc_conv_wgrad(int n, int d, int h, int w, int cin, int cout, int ks, int dims, const double *x,
                    const double *g, double *dw, double *db)
{
    const int T = taps_of(ks, dims);
    memset(dw, 0, sizeof(double) * (size_t)cout * T * cin);
    if (db) memset(db, 0, sizeof(double) * (size_t)cout);
    for (int b = 0; b < n; b++)
        for (int z = 0; z < d; z++)
            for (int yy = 0; yy < h; yy++)
                for (int xx = 0; xx < w; xx++) {
                    long p = pix(b, z, yy, xx, d, h, w);
                    for (int co = 0; co < cout; co++) {
                        if (db) db[co] += g[p * cout + co];
                        for (int t = 0; t < T; t++) {
                            int dz, dy, dx;
                            tap_offset(t, ks, dims, &dz, &dy, &dx);
                            int zs = z + dz, ys = yy + dy, xs = xx + dx;
                            if (zs < 0 || zs >= d || ys < 0 || ys >= h || xs < 0 || xs >= w) continue;
                            long q = pix(b, zs, ys, xs, d, h, w);
                            for (int ci = 0; ci < cin; ci++)
                                dw[((long)co * T + t) * cin + ci] += g[p * cout + co] * x[q * cin + ci];
                        }
                    }
                }
}

/* fine pixel of coarse (b, z, y, x) and window position sub */
static long fine_pix(int b, int z, int y, int x, int sub, int d, int h, int w, int dims)
{
    int sx = sub & 1, sy = (sub >> 1) & 1, sz = (sub >> 2) & 1;
    int fd = dims == 3 ? 2 * d : 1;
    int zf = dims == 3 ? 2 * z + sz : 0;
    return pix(b, zf, 2 * y + sy, 2 * x + sx, fd, 2 * h, 2 * w);
}

/* y[fine(p, sub)][co] = bias[co] + sum_ci x[p][ci] wt[sub][co][ci]; (d, h, w) coarse. */
void orc_tconv_fwd(int n, int d, int h, int w, int cin, int cout, int dims, const double *x, const double *wt,
                   const double *bias, double *y)
{
    const int S = 1 << dims;
    for (int b = 0; b < n; b++)
        for (int z = 0; z < d; z++)
            for (int yy = 0; yy < h; yy++)
                for (int xx = 0; xx < w; xx++) {
                    long p = pix(b, z, yy, xx, d, h, w);
                    for (int s = 0; s < S; s++) {
                        long f = fine_pix(b, z, yy, xx, s, d, h, w, dims);
                        for (int co = 0; co < cout; co++) {
                            double acc = bias ? bias[co] : 0.0;
                            for (int ci = 0; ci < cin; ci++)
                                acc += x[p * cin + ci] * wt[((long)s * cout + co) * cin + ci];
                            y[f * cout + co] = acc;
                        }
                    }
                }
}

void orc_tconv_dgrad(int n, int d, int h, int w, int cin, int cout, int dims, const double *g, const double *wt,
                     double *dx)
{
    const int S = 1 << dims;
    for (int b = 0; b < n; b++)
        for (int z = 0; z < d; z++)
            for (int yy = 0; yy < h; yy++)
                for (int xx = 0; xx < w; xx++) {
                    long p = pix(b, z, yy, xx, d, h, w);
                    for (int ci = 0; ci < cin; ci++) dx[p * cin + ci] = 0.0;
                    for (int s = 0; s < S; s++) {
                        long f = fine_pix(b, z, yy, xx, s, d, h, w, dims);
                        for (int co = 0; co < cout; co++)
                            for (int ci = 0; ci < cin; ci++)
                                dx[p * cin + ci] += g[f * cout + co] * wt[((long)s * cout + co) * cin + ci];
                    }
                }
}

void orc_tconv_wgrad(int n, int d, int h, int w, int cin, int cout, int dims, const double *x, const double *g,
                     double *dw, double *db)
{
    const int S = 1 << dims;
    memset(dw, 0, sizeof(double) * (size_t)S * cout * cin);
    if (db) memset(db, 0, sizeof(double) * (size_t)cout);
    for (int b = 0; b < n; b++)
        for (int z = 0; z < d; z++)
            for (int yy = 0; yy < h; yy++)
                for (int xx = 0; xx < w; xx++) {
                    long p = pix(b, z, yy, xx, d, h, w);
                    for (int s = 0; s < S; s++) {
                        long f = fine_pix(b, z, yy, xx, s, d, h, w, dims);
                        for (int co = 0; co < cout; co++) {
                            if (db) db[co] += g[f * cout + co];
                            for (int ci = 0; ci < cin; ci++)
                                dw[((long)s * cout + co) * cin + ci] += g[f * cout + co] * x[p * cin + ci];
                        }
                    }
                }
}

/* (d, h, w) coarse */
void orc_pool_fwd(int n, int d, int h, int w, int C, int dims, const double *x, double *y)
{
    const int S = 1 << dims;
    for (int b = 0; b < n; b++)
        for (int z = 0; z < d; z++)
            for (int yy = 0; yy < h; yy++)
                for (int xx = 0; xx < w; xx++) {
                    long p = pix(b, z, yy, xx, d, h, w);
                    for (int c = 0; c < C; c++) {
                        double m = -INFINITY;
                        for (int s = 0; s < S; s++) {
                            double v = x[fine_pix(b, z, yy, xx, s, d, h, w, dims) * C + c];
                            if (v > m) m = v;
                        }
                        y[p * C + c] = m;
                    }
                }
}

void orc_pool_bwd(int n, int d, int h, int w, int C, int dims, const double *x, const double *g, double *dx)
{
    const int S = 1 << dims;
    const int fd = dims == 3 ? 2 * d : 1;
    memset(dx, 0, sizeof(double) * (size_t)n * fd * 2 * h * 2 * w * C);
    for (int b = 0; b < n; b++)
        for (int z = 0; z < d; z++)
            for (int yy = 0; yy < h; yy++)
                for (int xx = 0; xx < w; xx++) {
                    long p = pix(b, z, yy, xx, d, h, w);
                    for (int c = 0; c < C; c++) {
                        double m = -INFINITY;
                        int arg = 0;
                        for (int s = 0; s < S; s++) {
                            double v = x[fine_pix(b, z, yy, xx, s, d, h, w, dims) * C + c];
                            if (v > m) { m = v; arg = s; }
                        }
                        dx[fine_pix(b, z, yy, xx, arg, d, h, w, dims) * C + c] += g[p * C + c];
                    }
                }
}
