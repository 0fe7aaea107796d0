/*
 * FP64 reference lattice Boltzmann forward map -- TEST INFRASTRUCTURE ONLY.
 *
 * Nothing in the product path may call this code.  It exists so that the
 * tests, the smoke check and the CPU-baseline leg of the benchmark can compare
 * the GPU kernels against a plain, slow, obviously correct implementation.
 *
 * This file is included twice by lbm_oracle.c: once with R = double (names
 * suffixed _d) and once with R = double _Complex (names suffixed _z).  The
 * complex build runs the very same forward recursion with complex parameters;
 * Im(L(p + i h v)) / h is then the directional derivative of the loss along v
 * to machine precision (complex-step differentiation), an independent check of
 * the hand-written reverse pass.  Every operation used below is analytic
 * (polynomials, division, sqrt of a value with positive real part), so the
 * complex build is exact in that sense.
 *
 * Structure follows the paper's stage split (Section 2.2: separate collision,
 * streaming and boundary kernels) and its push formulation of streaming
 * (Section 2.1, Eq. 3), on an array-of-structures layout f[node][i] with
 * node = (z * ny + y) * nx + x.  Solid nodes carry no populations (zeros).
 */

/* ---- moments, Eq. 1 and Eq. 2 ------------------------------------------ */
static void FN(moments)(const orc_lattice *L, const R *fn, R *rho, R j[3])
{
    const orc_velset *V = orc_vel(L->q);
    R s = 0, jx = 0, jy = 0, jz = 0;
    for (int i = 0; i < V->q; i++) {
        s += fn[i];
        jx += fn[i] * V->c[i][0];
        jy += fn[i] * V->c[i][1];
        jz += fn[i] * V->c[i][2];
    }
    *rho = s;
    j[0] = jx; j[1] = jy; j[2] = jz;
}

/* ---- second-order equilibrium, Eq. 5 with cs^2 = 1/3 -------------------- */
static void FN(equilibrium)(int q, R rho, const R u[3], R *feq)
{
    const orc_velset *V = orc_vel(q);
    const double cs2 = 1.0 / 3.0;
    R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < V->q; i++) {
        R uc = u[0] * V->c[i][0] + u[1] * V->c[i][1] + u[2] * V->c[i][2];
        feq[i] = V->w[i] * rho *
                 (1.0 + uc / cs2 + (uc * uc) / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
    }
}

/* Equilibrium initial state at every fluid node from given rho and u fields
 * (u stored as [node][3]); solid nodes are zeroed. */
static void FN(init_eq)(const orc_lattice *L, const R *rho, const R *u, R *f)
{
    const int q = L->q;
    const long n = orc_nodes(L);
    for (long k = 0; k < n; k++) {
        if (L->solid && L->solid[k]) {
            for (int i = 0; i < q; i++) f[k * q + i] = 0;
            continue;
        }
        FN(equilibrium)(q, rho[k], &u[3 * k], &f[k * q]);
    }
}

/* ---- collision ----------------------------------------------------------
 * BGK, Eq. 4 with the relaxing sign:  f* = f - (f - feq)/tau.
 * MRT (D2Q9, Section 3.4):  f* = f - M^-1 S M (f - feq), with m_eq = M feq,
 * S = diag(rates) and the two stress rates equal to 1/tau. */
static void FN(collide)(const orc_lattice *L, R tau, R *f)
{
    const int q = L->q;
    const long n = orc_nodes(L);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; k++) {
        if (L->solid && L->solid[k]) continue;
        R rho, j[3], u[3], feq[ORC_QMAX];
        FN(moments)(L, &f[k * q], &rho, j);
        u[0] = j[0] / rho; u[1] = j[1] / rho; u[2] = j[2] / rho;
        FN(equilibrium)(q, rho, u, feq);
        if (L->mrt) {
            R m[9];
            for (int r = 0; r < 9; r++) {
                R acc = 0;
                for (int i = 0; i < 9; i++) acc += ORC_M[r][i] * (f[k * q + i] - feq[i]);
                m[r] = acc * (r >= 7 ? 1.0 / tau : (R)L->mrt[r]);
            }
            for (int i = 0; i < 9; i++) {
                R acc = 0;
                for (int r = 0; r < 9; r++) acc += ORC_M[r][i] * m[r] / ORC_MNORM[r];
                f[k * q + i] -= acc;
            }
            continue;
        }
        for (int i = 0; i < q; i++)
            f[k * q + i] = f[k * q + i] - (f[k * q + i] - feq[i]) / tau;
    }
}

/* ---- streaming (push, Eq. 3) with link-wise halfway bounce-back ---------
 * Every fluid node x pushes f*_i(x) to y = x + c_i:
 *   - y leaves the lattice through a pressure (x) face: the value is dropped;
 *     the receiving boundary node reconstructs it (Zou-He pass);
 *   - y leaves through a periodic face: wrapped;
 *   - y leaves through a wall face, or y is solid: the value returns to x in
 *     the opposite direction (halfway bounce-back, wall half a link outside);
 *   - otherwise it lands in g_i(y).
 * g must not alias fs. */
static void FN(stream)(const orc_lattice *L, const R *fs, R *g)
{
    const orc_velset *V = orc_vel(L->q);
    const int q = L->q;
    const long n = orc_nodes(L);
    for (long k = 0; k < n * q; k++) g[k] = 0;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < n; k++) {
        if (L->solid && L->solid[k]) continue;
        int x[3];
        orc_coords(L, k, x);
        for (int i = 0; i < q; i++) {
            int y[3];
            int fate = orc_link_target(L, x, V->c[i], y);
            if (fate == ORC_LINK_DROP) continue;
            if (fate == ORC_LINK_BOUNCE) {
                g[k * q + V->opp[i]] = fs[k * q + i];
                continue;
            }
            long ky = orc_index(L, y);
            if (L->solid && L->solid[ky]) {
                g[k * q + V->opp[i]] = fs[k * q + i];
                continue;
            }
            g[ky * q + i] = fs[k * q + i];
        }
    }
}

/* ---- Zou-He density boundaries on the x faces ---------------------------
 * At a fluid node of the face x = 0 (s = +1) or x = nx-1 (s = -1) the
 * populations with c_x = s arrived from outside the lattice and are unknown.
 * They are fixed by three conditions: the density equals the prescribed
 * rho_b, the tangential velocity is zero, and the non-equilibrium part of the
 * normal population bounces back.  With
 *   K   = sum_{c_x = 0} g + 2 sum_{c_x = -s} g        (known populations)
 *   J   = rho_b - K                                   (= s * rho_b * u_x)
 *   N_t = 1/2 sum_{c_x = 0} g c_t                     (t = y, z)
 * every unknown population is
 *   g_i = g_opp(i) + 2 w_i J / cs^2 - sum_t c_it N_t.
 * rho_b holds one value per (z, y) face node.  With velocity != 0 the face
 * imposes the normal velocity u = rho_b[..] instead of the density (Zou-He
 * velocity inlet, s = +1): rho = K / (1 - u) and J = rho - K. */
static void FN(zouhe_face)(const orc_lattice *L, int face_x, int s, const R *rho_b, R *g, int velocity)
{
    const orc_velset *V = orc_vel(L->q);
    const int q = L->q;
    const double cs2 = 1.0 / 3.0;
    for (int z = 0; z < L->nz; z++) {
        for (int y = 0; y < L->ny; y++) {
            int xc[3] = {face_x, y, z};
            long k = orc_index(L, xc);
            if (L->solid && L->solid[k]) continue;
            R *gk = &g[k * q];
            R K = 0, Ny = 0, Nz = 0;
            for (int i = 0; i < q; i++) {
                if (V->c[i][0] == 0) {
                    K += gk[i];
                    Ny += 0.5 * gk[i] * V->c[i][1];
                    Nz += 0.5 * gk[i] * V->c[i][2];
                } else if (V->c[i][0] == -s) {
                    K += 2.0 * gk[i];
                }
            }
            R J = velocity ? K / (1.0 - rho_b[z * L->ny + y]) - K : rho_b[z * L->ny + y] - K;
            for (int i = 0; i < q; i++) {
                if (V->c[i][0] != s) continue;
                gk[i] = gk[V->opp[i]] + 2.0 * V->w[i] * J / cs2
                        - V->c[i][1] * Ny - V->c[i][2] * Nz;
            }
        }
    }
}

/* x faces: PRESSURE imposes both densities; VELOCITY imposes the inlet's
 * normal velocity (rho_in holds it) and the outlet's density. */
static void FN(zouhe)(const orc_lattice *L, const R *rho_in, const R *rho_out, R *g)
{
    if (L->bc[0] != ORC_BC_PRESSURE && L->bc[0] != ORC_BC_VELOCITY) return;
    FN(zouhe_face)(L, 0, +1, rho_in, g, L->bc[0] == ORC_BC_VELOCITY);
    FN(zouhe_face)(L, L->nx - 1, -1, rho_out, g, 0);
}

/* ---- anti-bounce-back density boundaries on the x faces (Eq. 6) ---------
 * At a fluid node x_b of the face x = 0 (s = +1) or x = nx-1 (s = -1) the
 * populations with c_x = s have no upstream node.  Each is the negated
 * post-collision population that left x_b through the face, plus twice the
 * even part of the equilibrium at the boundary density rho_b:
 *   g_i(x_b) = -f*_opp(i)(x_b) + 2 w_i rho_b (1 + (u.c_i)^2/(2 cs^4) - u.u/(2 cs^2)),
 * with u the velocity of x_b at the same time level (moments of f*(x_b),
 * equal to those before collision).  fs = post-collision state, g = streamed. */
static void FN(abb_face)(const orc_lattice *L, int face_x, int s, const R *rho_b, const R *fs, R *g)
{
    const orc_velset *V = orc_vel(L->q);
    const int q = L->q;
    const double cs2 = 1.0 / 3.0;
    for (int z = 0; z < L->nz; z++) {
        for (int y = 0; y < L->ny; y++) {
            int xc[3] = {face_x, y, z};
            long k = orc_index(L, xc);
            if (L->solid && L->solid[k]) continue;
            R rho, j[3];
            FN(moments)(L, &fs[k * q], &rho, j);
            R u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
            R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            R rb = rho_b[z * L->ny + y];
            for (int i = 0; i < q; i++) {
                if (V->c[i][0] != s) continue;
                R uc = u[0] * V->c[i][0] + u[1] * V->c[i][1] + u[2] * V->c[i][2];
                g[k * q + i] = -fs[k * q + V->opp[i]] +
                               2.0 * V->w[i] * rb * (1.0 + uc * uc / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
            }
        }
    }
}

static void FN(abb)(const orc_lattice *L, const R *rho_in, const R *rho_out, const R *fs, R *g)
{
    if (L->bc[0] != ORC_BC_ABB) return;
    FN(abb_face)(L, 0, +1, rho_in, fs, g);
    FN(abb_face)(L, L->nx - 1, -1, rho_out, fs, g);
}

/* One time step of the paper's stage order: collide, stream, boundary. */
static void FN(step)(const orc_lattice *L, R tau, const R *rho_in, const R *rho_out,
                     R *f, R *scratch)
{
    const long nq = orc_nodes(L) * L->q;
    FN(collide)(L, tau, f);
    FN(stream)(L, f, scratch);
    FN(zouhe)(L, rho_in, rho_out, scratch);
    FN(abb)(L, rho_in, rho_out, f, scratch);
    for (long k = 0; k < nq; k++) f[k] = scratch[k];
}

/* rho and u = j / rho at every fluid node (zeros at solid nodes). */
static void FN(macro)(const orc_lattice *L, const R *f, R *rho, R *u)
{
    const long n = orc_nodes(L);
    for (long k = 0; k < n; k++) {
        if (L->solid && L->solid[k]) {
            rho[k] = 0; u[3 * k] = u[3 * k + 1] = u[3 * k + 2] = 0;
            continue;
        }
        R r, j[3];
        FN(moments)(L, &f[k * L->q], &r, j);
        rho[k] = r;
        u[3 * k] = j[0] / r; u[3 * k + 1] = j[1] / r; u[3 * k + 2] = j[2] / r;
    }
}

/* Velocity-mismatch loss at the final state (Section 2.2 listing, Eq. 7,
 * Eq. 15):  L = scale * sum_fluid weight(x) * l(u(x), u_t(x)) with
 *   VEC : l = |u - u_t|^2
 *   NORM: l = (|u| - |u_t|)^2
 * target_u is [node][3]; weight may be NULL (all ones).  The sum runs in
 * node order, serially. */
static R FN(loss)(const orc_lattice *L, const R *f, const double *target_u,
                  const double *weight, int kind, double scale)
{
    const long n = orc_nodes(L);
    R acc = 0;
    for (long k = 0; k < n; k++) {
        if (L->solid && L->solid[k]) continue;
        R r, j[3];
        FN(moments)(L, &f[k * L->q], &r, j);
        R u0 = j[0] / r, u1 = j[1] / r, u2 = j[2] / r;
        const double *t = &target_u[3 * k];
        double wgt = weight ? weight[k] : 1.0;
        R l;
        if (kind == ORC_LOSS_NORM) {
            R nu = csqrt_or_sqrt(u0 * u0 + u1 * u1 + u2 * u2);
            double nt = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
            l = (nu - nt) * (nu - nt);
        } else {
            l = (u0 - t[0]) * (u0 - t[0]) + (u1 - t[1]) * (u1 - t[1]) +
                (u2 - t[2]) * (u2 - t[2]);
        }
        acc += wgt * l;
    }
    return scale * acc;
}

/* Runs T steps from f (in place) and returns the loss: with frames <= 1 the
 * loss of the final state; otherwise the sum over the states after steps
 * T - (frames - 1 - m) * stride, m = 0 .. frames - 1, each against its own
 * target frame (target_u is [frames][node][3]), added in time order. */
static R FN(run_loss)(const orc_lattice *L, R tau, const R *rho_in, const R *rho_out,
                      R *f, int T, const double *target_u, const double *weight,
                      int kind, double scale, int frames, int stride)
{
    const long n = orc_nodes(L), nq = n * L->q;
    R *scratch = (R *)malloc(sizeof(R) * (size_t)nq);
    R acc = 0;
    if (frames < 1) frames = 1;
    for (int t = 1; t <= T; t++) {
        FN(step)(L, tau, rho_in, rho_out, f, scratch);
        const int m = orc_frame_of(t, T, frames, stride);
        if (target_u && m >= 0) acc += FN(loss)(L, f, target_u + 3 * n * (long)m, weight, kind, scale);
    }
    free(scratch);
    return acc;
}
