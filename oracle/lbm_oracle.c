/*
 * FP64 CPU oracle for the differentiable lattice Boltzmann method --
 * TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the package's smoke check and the benchmark's CPU-baseline
 * leg may load this library.  It shares no code with the GPU path.
 *
 * Contents
 *   - D2Q9 and D3Q19 velocity sets (textbook constants; the paper names the
 *     lattices in Section 2.1 but does not print the weights);
 *   - the forward recursion in the paper's stage order (collide, stream,
 *     boundary), real (double) and complex (double _Complex) builds, from
 *     lbm_oracle_core.h;
 *   - the reverse (adjoint) pass of every stage, written from the chain rule
 *     with explicit per-node Jacobians, and a checkpointed gradient driver
 *     (the paper obtains the same derivative with a reverse-mode tape,
 *     Section 2.2).
 *
 * Readings of the paper taken here (the paper's formulas are partly garbled):
 *   - moment sums run over i = 0..Q-1 (Eq. 1-2);
 *   - BGK relaxes towards equilibrium, Omega = -(f - feq)/tau (Eq. 4);
 *   - tau is a free parameter, nu = cs^2 (tau - 1/2), cs^2 = 1/3 (Eq. 9);
 *   - inlet/outlet densities are imposed on the x faces with Zou-He or with
 *     the paper's anti-bounce-back rule (Eq. 6, read with the opposite index
 *     on the right-hand side and u the boundary node's own velocity);
 *   - walls and grains use link-wise halfway bounce-back;
 *   - the loss is evaluated on the final state only.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define ORC_QMAX 19

enum { ORC_BC_PRESSURE = 0, ORC_BC_PERIODIC = 1, ORC_BC_WALL = 2, ORC_BC_ABB = 3, ORC_BC_VELOCITY = 4 };
enum { ORC_LOSS_VEC = 0, ORC_LOSS_NORM = 1 };
enum { ORC_LINK_NORMAL = 0, ORC_LINK_BOUNCE = 1, ORC_LINK_DROP = 2 };

typedef struct {
    int q;
    int c[ORC_QMAX][3];
    double w[ORC_QMAX];
    int opp[ORC_QMAX];
} orc_velset;

/* Geometry of one lattice.  solid may be NULL (all fluid).  mrt: NULL for
 * BGK; else the nine D2Q9 multiple-relaxation-time rates in the order of
 * the moments (rho, e, eps, jx, qx, jy, qy, pxx, pxy); the two stress rates
 * (entries 7, 8) are ignored and set to 1/tau. */
typedef struct {
    int q;                       /* 9 or 19 */
    int nx, ny, nz;              /* nz = 1 for D2Q9 */
    int bc[3];                   /* per axis, ORC_BC_*; PRESSURE, ABB and VELOCITY only on x */
    const unsigned char *solid;  /* [nz][ny][nx], nonzero = solid */
    const double *mrt;
} orc_lattice;

/* D2Q9: rest, 4 axis links, 4 diagonals; w = 4/9, 1/9, 1/36. */
static orc_velset D2Q9 = {
    9,
    {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
     {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}},
    {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36},
    {0}};

/* D3Q19: rest, 6 axis links, 12 face diagonals; w = 1/3, 1/18, 1/36. */
static orc_velset D3Q19 = {
    19,
    {{0, 0, 0},
     {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
     {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
     {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
     {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}},
    {1.0 / 3,
     1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36},
    {0}};

static void orc_fill_opposites(orc_velset *V)
{
    /* The opposite of c_i is found by search, not by a table. */
    for (int i = 0; i < V->q; i++)
        for (int k = 0; k < V->q; k++)
            if (V->c[k][0] == -V->c[i][0] && V->c[k][1] == -V->c[i][1] &&
                V->c[k][2] == -V->c[i][2])
                V->opp[i] = k;
}

static const orc_velset *orc_vel(int q)
{
    static int ready = 0;
    if (!ready) {
        orc_fill_opposites(&D2Q9);
        orc_fill_opposites(&D3Q19);
        ready = 1;
    }
    return q == 9 ? &D2Q9 : &D3Q19;
}

static long orc_nodes(const orc_lattice *L) { return (long)L->nx * L->ny * L->nz; }

/* Loss frame of the state after step t (1 <= t <= T), or -1: the frames sit
 * at T - (frames - 1 - m) * stride for m = 0 .. frames - 1, the last one at T. */
static int orc_frame_of(int t, int T, int frames, int stride)
{
    if (frames <= 1) return t == T ? 0 : -1;
    const int back = T - t;
    if (back < 0 || back % stride != 0 || back / stride > frames - 1) return -1;
    return frames - 1 - back / stride;
}

static long orc_index(const orc_lattice *L, const int x[3])
{
    return ((long)x[2] * L->ny + x[1]) * L->nx + x[0];
}

static void orc_coords(const orc_lattice *L, long k, int x[3])
{
    x[0] = (int)(k % L->nx);
    x[1] = (int)((k / L->nx) % L->ny);
    x[2] = (int)(k / ((long)L->nx * L->ny));
}

/* Fate of the link leaving x along c: lands on y (NORMAL, y filled in),
 * bounces back from a wall face (BOUNCE), or leaves through a pressure face
 * (DROP).  Solid targets are checked by the caller. */
static int orc_link_target(const orc_lattice *L, const int x[3], const int c[3], int y[3])
{
    const int n[3] = {L->nx, L->ny, L->nz};
    int outside_pressure = 0, outside_wall = 0;
    for (int a = 0; a < 3; a++) {
        y[a] = x[a] + c[a];
        if (y[a] >= 0 && y[a] < n[a]) continue;
        if (L->bc[a] == ORC_BC_PERIODIC) {
            y[a] = (y[a] + n[a]) % n[a];
        } else if (L->bc[a] == ORC_BC_PRESSURE || L->bc[a] == ORC_BC_ABB || L->bc[a] == ORC_BC_VELOCITY) {
            outside_pressure = 1;
        } else {
            outside_wall = 1;
        }
    }
    /* A link that leaves through a pressure face is reconstructed at the
     * receiving face node even when it also crosses a wall (corner links). */
    if (outside_pressure) return ORC_LINK_DROP;
    if (outside_wall) return ORC_LINK_BOUNCE;
    return ORC_LINK_NORMAL;
}

/* ---- D2Q9 moment basis for the multiple-relaxation-time collision -------
 * (Section 3.4, after Lallemand & Luo): rows are polynomials of the lattice
 * velocity, evaluated on the D2Q9 set:
 *   rho: 1,  e: -4 + 3|c|^2,  eps: 4 - 21/2 |c|^2 + 9/2 |c|^4,
 *   jx: c_x,  qx: (-5 + 3|c|^2) c_x,  jy: c_y,  qy: (-5 + 3|c|^2) c_y,
 *   pxx: c_x^2 - c_y^2,  pxy: c_x c_y.
 * The rows are mutually orthogonal, so M^-1 = M^T diag(1 / |row|^2). */
static double ORC_M[9][9], ORC_MNORM[9];
static void orc_mrt_basis(void)
{
    static int ready = 0;
    if (ready) return;
    const orc_velset *V = orc_vel(9);
    for (int i = 0; i < 9; i++) {
        const double cx = V->c[i][0], cy = V->c[i][1], c2 = cx * cx + cy * cy;
        ORC_M[0][i] = 1;
        ORC_M[1][i] = -4 + 3 * c2;
        ORC_M[2][i] = 4 - 10.5 * c2 + 4.5 * c2 * c2;
        ORC_M[3][i] = cx;
        ORC_M[4][i] = (-5 + 3 * c2) * cx;
        ORC_M[5][i] = cy;
        ORC_M[6][i] = (-5 + 3 * c2) * cy;
        ORC_M[7][i] = cx * cx - cy * cy;
        ORC_M[8][i] = cx * cy;
    }
    for (int r = 0; r < 9; r++) {
        ORC_MNORM[r] = 0;
        for (int i = 0; i < 9; i++) ORC_MNORM[r] += ORC_M[r][i] * ORC_M[r][i];
    }
    ready = 1;
}

void orc_mrt_matrix(double *m)
{
    orc_mrt_basis();
    for (int r = 0; r < 9; r++)
        for (int i = 0; i < 9; i++) m[r * 9 + i] = ORC_M[r][i];
}

/* ---------------- real and complex builds of the forward map ------------- */
#define R double
#define FN(name) orc_##name##_d
#define csqrt_or_sqrt sqrt
#include "lbm_oracle_core.h"
#undef R
#undef FN
#undef csqrt_or_sqrt

#define R double _Complex
#define FN(name) orc_##name##_z
#define csqrt_or_sqrt csqrt
#include "lbm_oracle_core.h"
#undef R
#undef FN
#undef csqrt_or_sqrt

/* ---------------- exported forward entry points (real) ------------------- */
static void orc_make(orc_lattice *L, int q, int nx, int ny, int nz, const int *bc,
                     const unsigned char *solid, const double *mrt)
{
    L->q = q; L->nx = nx; L->ny = ny; L->nz = nz;
    L->bc[0] = bc[0]; L->bc[1] = bc[1]; L->bc[2] = bc[2];
    L->solid = solid;
    L->mrt = q == 9 ? mrt : NULL;
    orc_mrt_basis();
}

#define ORC_ARGS int q, int nx, int ny, int nz, const int *bc, const unsigned char *solid, const double *mrt
#define ORC_MAKE orc_lattice L; orc_make(&L, q, nx, ny, nz, bc, solid, mrt)
#define ORC_PASS q, nx, ny, nz, bc, solid, mrt

void orc_equilibrium(int q, double rho, const double *u, double *feq)
{
    orc_equilibrium_d(q, rho, u, feq);
}

void orc_init_eq(ORC_ARGS, const double *rho, const double *u, double *f)
{
    ORC_MAKE;
    orc_init_eq_d(&L, rho, u, f);
}

void orc_collide(ORC_ARGS, double tau, double *f)
{
    ORC_MAKE;
    orc_collide_d(&L, tau, f);
}

void orc_stream(ORC_ARGS, const double *fs, double *g)
{
    ORC_MAKE;
    orc_stream_d(&L, fs, g);
}

void orc_zouhe(ORC_ARGS, const double *rho_in, const double *rho_out, double *g)
{
    ORC_MAKE;
    orc_zouhe_d(&L, rho_in, rho_out, g);
}

void orc_abb(ORC_ARGS, const double *rho_in, const double *rho_out, const double *fs, double *g)
{
    ORC_MAKE;
    orc_abb_d(&L, rho_in, rho_out, fs, g);
}

void orc_run(ORC_ARGS, double tau, const double *rho_in, const double *rho_out,
             double *f, int T)
{
    ORC_MAKE;
    orc_run_loss_d(&L, tau, rho_in, rho_out, f, T, NULL, NULL, 0, 1.0, 1, 1);
}

void orc_macro(ORC_ARGS, const double *f, double *rho, double *u)
{
    ORC_MAKE;
    orc_macro_d(&L, f, rho, u);
}

double orc_loss(ORC_ARGS, const double *f, const double *target_u, const double *weight,
                int kind, double scale)
{
    ORC_MAKE;
    return orc_loss_d(&L, f, target_u, weight, kind, scale);
}

/* Complex-step forward.  Parameters are given as real part + imaginary part;
 * f0 is real.  Returns real and imaginary parts of the loss. */
void orc_run_loss_cs(ORC_ARGS, double tau_re, double tau_im,
                     const double *rho_in_re, const double *rho_in_im,
                     const double *rho_out_re, const double *rho_out_im,
                     const double *f0, int T, const double *target_u,
                     const double *weight, int kind, double scale, int frames, int stride,
                     double *loss_re_im)
{
    ORC_MAKE;
    const long n = orc_nodes(&L);
    const long nf = (long)ny * nz;
    double _Complex *f = malloc(sizeof(double _Complex) * (size_t)(n * q));
    double _Complex *ri = malloc(sizeof(double _Complex) * (size_t)nf);
    double _Complex *ro = malloc(sizeof(double _Complex) * (size_t)nf);
    for (long k = 0; k < n * q; k++) f[k] = f0[k];
    for (long k = 0; k < nf; k++) {
        ri[k] = rho_in_re[k] + I * rho_in_im[k];
        ro[k] = rho_out_re[k] + I * rho_out_im[k];
    }
    double _Complex l = orc_run_loss_z(&L, tau_re + I * tau_im, ri, ro, f, T, target_u,
                                       weight, kind, scale, frames, stride);
    loss_re_im[0] = creal(l);
    loss_re_im[1] = cimag(l);
    free(f); free(ri); free(ro);
}

/* ---------------- reverse (adjoint) passes, real only -------------------- */

/* Transpose of the collision at one node.  With f the pre-collision state,
 * f*_k = f_k - (f_k - feq_k(f)) / tau, and fsbar = dL/df*, this returns
 * fbar_i = sum_k fsbar_k d f*_k / d f_i and adds sum_k fsbar_k d f*_k / d tau
 * to *dtau.  The Jacobian is formed entry by entry from Eq. 5 with
 * rho = sum f and u = (sum f c) / rho, so that
 *   d rho / d f_i = 1,    d u / d f_i = (c_i - u) / rho. */
static void orc_collide_adj_node(int q, double tau, const double *f, const double *fsbar,
                                 double *fbar, double *dtau)
{
    const orc_velset *V = orc_vel(q);
    const double cs2 = 1.0 / 3.0;
    double rho = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < q; i++) {
        rho += f[i];
        for (int a = 0; a < 3; a++) j[a] += f[i] * V->c[i][a];
    }
    double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    double feq[ORC_QMAX];
    orc_equilibrium_d(q, rho, u, feq);
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < q; i++) fbar[i] = 0;
    for (int k = 0; k < q; k++) {
        double uc = u[0] * V->c[k][0] + u[1] * V->c[k][1] + u[2] * V->c[k][2];
        /* d feq_k / d rho at fixed u, and d feq_k / d u_a at fixed rho */
        double dfeq_drho = V->w[k] * (1.0 + uc / cs2 + uc * uc / (2 * cs2 * cs2) - uu / (2 * cs2));
        double dfeq_du[3];
        for (int a = 0; a < 3; a++)
            dfeq_du[a] = V->w[k] * rho *
                         (V->c[k][a] / cs2 + uc * V->c[k][a] / (cs2 * cs2) - u[a] / cs2);
        for (int i = 0; i < q; i++) {
            double dfeq_dfi = dfeq_drho;
            for (int a = 0; a < 3; a++) dfeq_dfi += dfeq_du[a] * (V->c[i][a] - u[a]) / rho;
            double jac = (k == i ? 1.0 - 1.0 / tau : 0.0) + dfeq_dfi / tau;
            fbar[i] += fsbar[k] * jac;
        }
        *dtau += fsbar[k] * (f[k] - feq[k]) / (tau * tau);
    }
}

/* Transpose of the MRT collision at one node.  With A = M^-1 S M and J the
 * Jacobian of feq(f), fs = f - A (f - feq) has the Jacobian I - A (I - J), so
 *   fbar = fsbar - mu + J^T mu,   mu = A^T fsbar = M^T S M^-T fsbar,
 * and only the stress rates depend on tau (d s / d tau = -1/tau^2):
 *   d L / d tau = sum_{r stress} (M^-T fsbar)_r (M (f - feq))_r / tau^2. */
static void orc_collide_adj_node_mrt(const double *rates, double tau, const double *f, const double *fsbar,
                                     double *fbar, double *dtau)
{
    const orc_velset *V = orc_vel(9);
    const double cs2 = 1.0 / 3.0;
    double rho = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < 9; i++) {
        rho += f[i];
        for (int a = 0; a < 3; a++) j[a] += f[i] * V->c[i][a];
    }
    double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    double feq[9];
    orc_equilibrium_d(9, rho, u, feq);
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double y[9], mu[9], md[9];
    for (int r = 0; r < 9; r++) {                 /* y = M^-T fsbar, md = M (f - feq) */
        double a = 0, b = 0;
        for (int i = 0; i < 9; i++) {
            a += ORC_M[r][i] * fsbar[i];
            b += ORC_M[r][i] * (f[i] - feq[i]);
        }
        y[r] = a / ORC_MNORM[r];
        md[r] = b;
    }
    for (int r = 7; r < 9; r++) *dtau += y[r] * md[r] / (tau * tau);
    for (int i = 0; i < 9; i++) {                 /* mu = M^T S y */
        double a = 0;
        for (int r = 0; r < 9; r++) a += ORC_M[r][i] * (r >= 7 ? 1.0 / tau : rates[r]) * y[r];
        mu[i] = a;
    }
    for (int i = 0; i < 9; i++) fbar[i] = fsbar[i] - mu[i];
    for (int k = 0; k < 9; k++) {                 /* + J^T mu, J_ki = d feq_k / d f_i */
        double uc = u[0] * V->c[k][0] + u[1] * V->c[k][1];
        double dfeq_drho = V->w[k] * (1.0 + uc / cs2 + uc * uc / (2 * cs2 * cs2) - uu / (2 * cs2));
        double dfeq_du[3];
        for (int a = 0; a < 3; a++)
            dfeq_du[a] = V->w[k] * rho * (V->c[k][a] / cs2 + uc * V->c[k][a] / (cs2 * cs2) - u[a] / cs2);
        for (int i = 0; i < 9; i++) {
            double d = dfeq_drho;
            for (int a = 0; a < 3; a++) d += dfeq_du[a] * (V->c[i][a] - u[a]) / rho;
            fbar[i] += mu[k] * d;
        }
    }
}

void orc_collide_adj(ORC_ARGS, double tau, const double *f, const double *fsbar,
                     double *fbar, double *dtau)
{
    ORC_MAKE;
    const long n = orc_nodes(&L);
    /* each node's d/dtau term is formed on its own (nodes in parallel); the
     * node terms are then summed in node order, so the result does not
     * depend on the thread count */
    double *part = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; k++) {
        part[k] = 0;
        if (solid && solid[k]) {
            for (int i = 0; i < q; i++) fbar[k * q + i] = 0;
            continue;
        }
        if (L.mrt)
            orc_collide_adj_node_mrt(L.mrt, tau, &f[k * q], &fsbar[k * q], &fbar[k * q], &part[k]);
        else
            orc_collide_adj_node(q, tau, &f[k * q], &fsbar[k * q], &fbar[k * q], &part[k]);
    }
    double acc = 0;
    for (long k = 0; k < n; k++) acc += part[k];
    free(part);
    *dtau += acc;
}

/* Transpose of the streaming pass: fsbar_i(x) is the adjoint of wherever the
 * push sent f*_i(x). */
void orc_stream_adj(ORC_ARGS, const double *gbar, double *fsbar)
{
    ORC_MAKE;
    const orc_velset *V = orc_vel(q);
    const long n = orc_nodes(&L);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; k++) {
        int x[3];
        orc_coords(&L, k, x);
        for (int i = 0; i < q; i++) {
            fsbar[k * q + i] = 0;
            if (solid && solid[k]) continue;
            int y[3];
            int fate = orc_link_target(&L, x, V->c[i], y);
            if (fate == ORC_LINK_DROP) continue;
            if (fate == ORC_LINK_BOUNCE) {
                fsbar[k * q + i] = gbar[k * q + V->opp[i]];
                continue;
            }
            long ky = orc_index(&L, y);
            if (solid && solid[ky])
                fsbar[k * q + i] = gbar[k * q + V->opp[i]];
            else
                fsbar[k * q + i] = gbar[ky * q + i];
        }
    }
}

/* Transpose of one Zou-He face (in place on gbar).  The forward pass reads
 * the known populations and overwrites the unknown ones with
 *   g_u = g_opp(u) + 2 w_u J / cs^2 - sum_t c_ut N_t,
 *   J = rho_b - K(g),  N_t = 1/2 sum_{c_x=0} g c_t,
 * so the adjoint of each unknown flows to its opposite population, to J (and
 * from J to rho_b with +1 and to the known populations with -1 or -2), and
 * to the tangential sums. The unknowns' incoming values were overwritten,
 * so their adjoint is zero afterwards. */
static void orc_zouhe_face_adj(const orc_lattice *L, int face_x, int s, const double *g,
                               const double *rho_b, double *gbar, double *drho_b, int velocity)
{
    const orc_velset *V = orc_vel(L->q);
    const int q = L->q;
    const double cs2 = 1.0 / 3.0;
    for (int z = 0; z < L->nz; z++) {
        for (int y = 0; y < L->ny; y++) {
            int xc[3] = {face_x, y, z};
            long k = orc_index(L, xc);
            if (L->solid && L->solid[k]) continue;
            double *gb = &gbar[k * q];
            double Jbar = 0, Nybar = 0, Nzbar = 0;
            for (int i = 0; i < q; i++) {
                if (V->c[i][0] != s) continue;
                gb[V->opp[i]] += gb[i];
                Jbar += 2.0 * V->w[i] / cs2 * gb[i];
                Nybar -= V->c[i][1] * gb[i];
                Nzbar -= V->c[i][2] * gb[i];
                gb[i] = 0;
            }
            /* J = rho_b - K (density), or J = K u / (1 - u) (velocity) */
            double dJdK = -1.0;
            if (velocity) {
                double K = 0;
                for (int i = 0; i < q; i++) {
                    if (V->c[i][0] == 0) K += g[k * q + i];
                    else if (V->c[i][0] == -s) K += 2.0 * g[k * q + i];
                }
                const double ub = rho_b[z * L->ny + y];
                dJdK = ub / (1.0 - ub);
                drho_b[z * L->ny + y] += Jbar * K / ((1.0 - ub) * (1.0 - ub));
            } else {
                drho_b[z * L->ny + y] += Jbar;
            }
            for (int i = 0; i < q; i++) {
                if (V->c[i][0] == 0) {
                    gb[i] += dJdK * Jbar + 0.5 * V->c[i][1] * Nybar + 0.5 * V->c[i][2] * Nzbar;
                } else if (V->c[i][0] == -s) {
                    gb[i] += 2.0 * dJdK * Jbar;
                }
            }
        }
    }
}

/* g: the state the closure completed (its known populations are read by the
 * velocity face; may be NULL for density faces); rho_in: the inlet values. */
void orc_zouhe_adj(ORC_ARGS, const double *g, const double *rho_in, double *gbar, double *drho_in,
                   double *drho_out)
{
    ORC_MAKE;
    if (L.bc[0] != ORC_BC_PRESSURE && L.bc[0] != ORC_BC_VELOCITY) return;
    /* reverse order of the forward pass (inlet, then outlet) */
    orc_zouhe_face_adj(&L, nx - 1, -1, g, NULL, gbar, drho_out, 0);
    orc_zouhe_face_adj(&L, 0, +1, g, rho_in, gbar, drho_in, L.bc[0] == ORC_BC_VELOCITY);
}

/* Transpose of one anti-bounce-back face.  The forward pass wrote
 *   g_i = -fs_opp(i) + 2 w_i rho_b E_i(u),  E_i = 1 + (u.c_i)^2/(2 cs^4) - u.u/(2 cs^2),
 * into the unknown slots (c_x = s), with u = j(fs)/rho(fs) at the node, so
 *   d g_i / d fs_m   = -[m = opp(i)] + 2 w_i rho_b sum_a dE_i/du_a (c_ma - u_a)/rho,
 *   dE_i/du_a        = (u.c_i) c_ia / cs^4 - u_a / cs^2,
 *   d g_i / d rho_b  = 2 w_i E_i.
 * The adjoint of each unknown is added to fsbar and to drho_b, and the
 * unknown slot's own adjoint is cleared (its streamed value was dropped). */
static void orc_abb_face_adj(const orc_lattice *L, int face_x, int s, const double *rho_b,
                             const double *fs, double *gbar, double *fsbar, double *drho_b)
{
    const orc_velset *V = orc_vel(L->q);
    const int q = L->q;
    const double cs2 = 1.0 / 3.0;
    for (int z = 0; z < L->nz; z++) {
        for (int y = 0; y < L->ny; y++) {
            int xc[3] = {face_x, y, z};
            long k = orc_index(L, xc);
            if (L->solid && L->solid[k]) continue;
            double rho, j[3];
            orc_moments_d(L, &fs[k * q], &rho, j);
            double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
            double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            double rb = rho_b[z * L->ny + y];
            double ubar[3] = {0, 0, 0};
            for (int i = 0; i < q; i++) {
                if (V->c[i][0] != s) continue;
                double gb = gbar[k * q + i];
                double uc = u[0] * V->c[i][0] + u[1] * V->c[i][1] + u[2] * V->c[i][2];
                fsbar[k * q + V->opp[i]] -= gb;
                drho_b[z * L->ny + y] += gb * 2.0 * V->w[i] *
                                         (1.0 + uc * uc / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
                for (int a = 0; a < 3; a++)
                    ubar[a] += gb * 2.0 * V->w[i] * rb * (uc * V->c[i][a] / (cs2 * cs2) - u[a] / cs2);
                gbar[k * q + i] = 0;
            }
            for (int m = 0; m < q; m++)
                for (int a = 0; a < 3; a++) fsbar[k * q + m] += ubar[a] * (V->c[m][a] - u[a]) / rho;
        }
    }
}

/* gbar: adjoint of the state after the boundary pass (unknown slots are
 * cleared); fsbar receives the boundary pass's contribution to dL/dfs. */
void orc_abb_adj(ORC_ARGS, const double *rho_in, const double *rho_out, const double *fs,
                 double *gbar, double *fsbar, double *drho_in, double *drho_out)
{
    ORC_MAKE;
    if (L.bc[0] != ORC_BC_ABB) return;
    orc_abb_face_adj(&L, nx - 1, -1, rho_out, fs, gbar, fsbar, drho_out);
    orc_abb_face_adj(&L, 0, +1, rho_in, fs, gbar, fsbar, drho_in);
}

/* dL/df at the final state for the loss defined in orc_loss.  For NORM the
 * derivative of |u| is taken as zero where u = 0. */
void orc_loss_seed(ORC_ARGS, const double *f, const double *target_u, const double *weight,
                   int kind, double scale, double *fbar)
{
    ORC_MAKE;
    const orc_velset *V = orc_vel(q);
    const long n = orc_nodes(&L);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; k++) {
        for (int i = 0; i < q; i++) fbar[k * q + i] = 0;
        if (solid && solid[k]) continue;
        double rho, j[3];
        orc_moments_d(&L, &f[k * q], &rho, j);
        double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
        const double *t = &target_u[3 * k];
        double wgt = (weight ? weight[k] : 1.0) * scale;
        double dldu[3];
        if (kind == ORC_LOSS_NORM) {
            double nu = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            double nt = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
            for (int a = 0; a < 3; a++)
                dldu[a] = nu > 0 ? wgt * 2.0 * (nu - nt) * u[a] / nu : 0.0;
        } else {
            for (int a = 0; a < 3; a++) dldu[a] = wgt * 2.0 * (u[a] - t[a]);
        }
        for (int i = 0; i < q; i++) {
            double s = 0;
            for (int a = 0; a < 3; a++) s += dldu[a] * (V->c[i][a] - u[a]) / rho;
            fbar[k * q + i] = s;
        }
    }
}

/* Reverse-mode gradient of the loss after T steps from f0 with respect to
 * the inlet densities (per face node), the outlet densities (per face node)
 * and tau.  States f^{cK} are kept for c = 0, 1, ...; each segment is
 * recomputed from its checkpoint in reverse order and then swept backwards
 * stage by stage: boundary transpose (Zou-He, or anti-bounce-back whose
 * contribution joins the streaming transpose's), streaming transpose,
 * collision transpose.  With several loss frames (see orc_run_loss), the
 * derivative of a frame's loss with respect to the state it is taken on
 * joins dL/df^t before that step's transposes.  fbar0 (nullable) receives
 * dL/df^0.  Returns the loss. */
double orc_grad(ORC_ARGS, double tau, const double *rho_in, const double *rho_out,
                const double *f0, int T, int K, const double *target_u,
                const double *weight, int kind, double scale, int frames, int stride,
                double *drho_in, double *drho_out, double *dtau, double *fbar0)
{
    ORC_MAKE;
    const long nq = orc_nodes(&L) * q;
    const long nf = (long)ny * nz;
    if (K <= 0) K = T > 0 ? T : 1;
    const int nseg = T > 0 ? (T + K - 1) / K : 0;
    double *ckpt = malloc(sizeof(double) * (size_t)(nq * (nseg > 0 ? nseg : 1)));
    double *seg = malloc(sizeof(double) * (size_t)(nq * K));
    double *f = malloc(sizeof(double) * (size_t)nq);
    double *scratch = malloc(sizeof(double) * (size_t)nq);
    double *a = malloc(sizeof(double) * (size_t)nq);
    double *b = malloc(sizeof(double) * (size_t)nq);
    double *fsb = malloc(sizeof(double) * (size_t)nq);
    const long n = orc_nodes(&L);
    if (frames < 1) frames = 1;
    memcpy(f, f0, sizeof(double) * (size_t)nq);
    double loss = 0;
    for (int t = 0; t < T; t++) {
        if (t % K == 0) memcpy(&ckpt[(t / K) * nq], f, sizeof(double) * (size_t)nq);
        orc_step_d(&L, tau, rho_in, rho_out, f, scratch);
        const int m = orc_frame_of(t + 1, T, frames, stride);
        if (m >= 0) loss += orc_loss_d(&L, f, target_u + 3 * n * (long)m, weight, kind, scale);
    }
    for (long k = 0; k < nf; k++) drho_in[k] = drho_out[k] = 0;
    *dtau = 0;
    orc_loss_seed(ORC_PASS, f, target_u + 3 * n * (long)(frames - 1), weight, kind, scale, a);
    for (int c = nseg - 1; c >= 0; c--) {
        int t0 = c * K, t1 = (c + 1) * K < T ? (c + 1) * K : T;
        memcpy(&seg[0], &ckpt[c * nq], sizeof(double) * (size_t)nq);
        for (int t = t0 + 1; t < t1; t++) {
            memcpy(&seg[(t - t0) * nq], &seg[(t - t0 - 1) * nq], sizeof(double) * (size_t)nq);
            orc_step_d(&L, tau, rho_in, rho_out, &seg[(t - t0) * nq], scratch);
        }
        for (int t = t1; t > t0; t--) {
            /* a = dL/df^t  ->  a = dL/df^{t-1} */
            const double *fprev = &seg[(t - 1 - t0) * nq];
            const int m = t < T ? orc_frame_of(t, T, frames, stride) : -1;
            if (m >= 0) {
                /* the frame's loss on f^t: f^t is the next segment's checkpoint at t1 */
                const double *ft = t == t1 ? &ckpt[(c + 1) * nq] : &seg[(t - t0) * nq];
                orc_loss_seed(ORC_PASS, ft, target_u + 3 * n * (long)m, weight, kind, scale, fsb);
                for (long k = 0; k < nq; k++) a[k] += fsb[k];
            }
            if (L.bc[0] == ORC_BC_ABB) {
                /* the boundary pass read the post-collision state of step t-1 */
                memcpy(scratch, fprev, sizeof(double) * (size_t)nq);
                orc_collide_d(&L, tau, scratch);
                for (long k = 0; k < nq; k++) fsb[k] = 0;
                orc_abb_adj(ORC_PASS, rho_in, rho_out, scratch, a, fsb, drho_in, drho_out);
                orc_stream_adj(ORC_PASS, a, b);
                for (long k = 0; k < nq; k++) b[k] += fsb[k];
            } else {
                const double *gt = NULL;
                if (L.bc[0] == ORC_BC_VELOCITY) {
                    /* the closure's known populations at step t */
                    memcpy(scratch, fprev, sizeof(double) * (size_t)nq);
                    orc_collide_d(&L, tau, scratch);
                    orc_stream_d(&L, scratch, fsb);
                    gt = fsb;
                }
                orc_zouhe_adj(ORC_PASS, gt, rho_in, a, drho_in, drho_out);
                orc_stream_adj(ORC_PASS, a, b);
            }
            orc_collide_adj(ORC_PASS, tau, fprev, b, a, dtau);
        }
    }
    if (fbar0) memcpy(fbar0, a, sizeof(double) * (size_t)nq);
    free(ckpt); free(seg); free(f); free(scratch); free(a); free(b); free(fsb);
    return loss;
}

/* ---------------- helpers for the pins ----------------------------------- */

/* Threads of the per-node loops (the results do not depend on them). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }

/* Copies the velocity set (c as [q][3] ints, w as [q] doubles) and the
 * opposite-direction table. */
void orc_velset_get(int q, int *c, double *w, int *opp)
{
    const orc_velset *V = orc_vel(q);
    for (int i = 0; i < V->q; i++) {
        for (int a = 0; a < 3; a++) c[3 * i + a] = V->c[i][a];
        w[i] = V->w[i];
        opp[i] = V->opp[i];
    }
}

/* T complex steps from a complex state (given as real and imaginary parts,
 * overwritten with the result).  With f = f0 + i h v this yields the
 * Jacobian-vector product of the T-step map in the imaginary part. */
void orc_run_cs(ORC_ARGS, double tau, const double *rho_in, const double *rho_out,
                double *f_re, double *f_im, int T)
{
    ORC_MAKE;
    const long nq = orc_nodes(&L) * q;
    const long nf = (long)ny * nz;
    double _Complex *f = malloc(sizeof(double _Complex) * (size_t)nq);
    double _Complex *s = malloc(sizeof(double _Complex) * (size_t)nq);
    double _Complex *ri = malloc(sizeof(double _Complex) * (size_t)nf);
    double _Complex *ro = malloc(sizeof(double _Complex) * (size_t)nf);
    for (long k = 0; k < nq; k++) f[k] = f_re[k] + I * f_im[k];
    for (long k = 0; k < nf; k++) { ri[k] = rho_in[k]; ro[k] = rho_out[k]; }
    for (int t = 0; t < T; t++) orc_step_z(&L, tau, ri, ro, f, s);
    for (long k = 0; k < nq; k++) { f_re[k] = creal(f[k]); f_im[k] = cimag(f[k]); }
    free(f); free(s); free(ri); free(ro);
}
