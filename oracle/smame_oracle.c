/*
 * Plain FP64 CPU oracle for the SMAME step of arXiv 2012.03525.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the library.  Single thread,
 * built with -O2 -ffp-contract=off so every product and sum is rounded as
 * written.
 *
 * What is computed, in the paper's order (Sec. 2):
 *   1. ghost values of the level-n fields (boundary rules below);
 *   2. rho^{n+1} everywhere from the simplified continuity update, Eq. (2.10),
 *      with the centred gradient (2.12) and the 5/7-point Laplacian (2.13);
 *   3. ghost values of rho^{n+1};
 *   4. (rho u)^{n+1} everywhere from the simplified momentum update, Eq. (2.11),
 *      plus the body force delta_t rho^{n+1} g (Sec. 2, after Table-1 text)
 *      and, for two-phase flow, the surface-tension force -delta_t phi d mu;
 *   5. u^{n+1} = (rho u)^{n+1} / rho^{n+1};
 *   6. two-phase flow: Cahn-Hilliard equation (2.14) advanced by Heun's
 *      second-order Runge-Kutta method with isotropic stencils, using u^n.
 *
 * Readings where the paper is silent (each listed with its reason in the
 * design notes of the repository):
 *   - the flux d_b(rho u_a u_b) is the centred difference of the per-node
 *     product (conservative form);
 *   - the pressure term d_a(rho c_s^2) is c_s^2 times the centred difference
 *     of drho (the constant rho0 c_s^2 drops out of a difference);
 *   - walls sit halfway between nodes: ghost drho = mirror value, ghost
 *     velocity = 2 u_wall - mirror value; a symmetry plane mirrors every
 *     field and flips the normal velocity; mu is mirrored (no flux); phi
 *     obeys the wetting condition of Sec. 2 across a wall (mirrored when the
 *     contact angle is 90 degrees or at a symmetry plane); the rules are
 *     applied to the level-n fields, to rho^{n+1} and to every intermediate
 *     phase-field quantity, face by face in the order x, y, z;
 *   - the wetting condition d_n phi = -(2/W) cos(theta) (1 - phi_w^2) is
 *     taken across the halfway wall, (phi_m - phi_g)/dx, with phi_w the
 *     wall value (phi_g + phi_m)/2, and solved for the ghost exactly;
 *   - isotropic stencils are the D2Q9-weighted ones in 2D and the
 *     D3Q19-weighted ones in 3D;
 *   - Heun's method; both stages use u^n.
 */
#include "smame_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* padded grid: one ghost layer on every side of every active axis      */
/* ------------------------------------------------------------------ */
typedef struct {
    int dim, nx, ny, nz;
    int px, py, pz;   /* padded extents */
    int oz;           /* 1 in 3D, 0 in 2D */
} pgrid;

static pgrid make_grid(const orc_params* p)
{
    pgrid g;
    g.dim = p->dim;
    g.nx = p->nx;
    g.ny = p->ny;
    g.nz = (p->dim == 3) ? p->nz : 1;
    g.px = g.nx + 2;
    g.py = g.ny + 2;
    g.pz = (p->dim == 3) ? g.nz + 2 : 1;
    g.oz = (p->dim == 3) ? 1 : 0;
    return g;
}

/* padded index of node (i,j,k); i in [-1,nx], j in [-1,ny], k in [-1,nz] (3D) */
static long P(const pgrid* g, int i, int j, int k)
{
    return ((long)(k + g->oz) * g->py + (j + 1)) * g->px + (i + 1);
}

/* dense index of interior node */
static long D(const pgrid* g, int i, int j, int k)
{
    return ((long)k * g->ny + j) * g->nx + i;
}

/* Map a coordinate that may lie one layer outside [0,n) to its source node.
 * *face is set to the face crossed (lo/hi) or -1. */
static int map_axis(int i, int n, int bc_lo, int bc_hi, int face_lo, int* face)
{
    *face = -1;
    if (i < 0) {
        *face = face_lo;
        return (bc_lo == ORC_PERIODIC) ? i + n : -1 - i;
    }
    if (i >= n) {
        *face = face_lo + 1;
        return (bc_hi == ORC_PERIODIC) ? i - n : 2 * n - 1 - i;
    }
    return i;
}

static int is_ghost(const pgrid* g, int i, int j, int k)
{
    if (i < 0 || i >= g->nx || j < 0 || j >= g->ny) return 1;
    if (g->dim == 3 && (k < 0 || k >= g->nz)) return 1;
    return 0;
}

/* Fill the ghost layer of a scalar field: periodic wrap or mirror. */
static void fill_scalar(const orc_params* p, const pgrid* g, double* f)
{
    int kl = (g->dim == 3) ? -1 : 0, kh = (g->dim == 3) ? g->nz : 0;
    for (int k = kl; k <= kh; ++k)
        for (int j = -1; j <= g->ny; ++j)
            for (int i = -1; i <= g->nx; ++i) {
                if (!is_ghost(g, i, j, k)) continue;
                int fx, fy, fz;
                int si = map_axis(i, g->nx, p->bc[0], p->bc[1], 0, &fx);
                int sj = map_axis(j, g->ny, p->bc[2], p->bc[3], 2, &fy);
                int sk = (g->dim == 3) ? map_axis(k, g->nz, p->bc[4], p->bc[5], 4, &fz) : 0;
                f[P(g, i, j, k)] = f[P(g, si, sj, sk)];
            }
}

/* Ghost order parameter across a wall face (Sec. 2 wetting condition):
 * (phi_m - phi_g)/dx = -(2/W) cos(theta) (1 - phi_w^2), phi_w = (phi_g + phi_m)/2.
 * With b = dx (2/W) cos(theta) and s = phi_w this is b s^2 + 2 s - (2 phi_m + b) = 0,
 * whose root that tends to phi_m as b -> 0 is s = (2 phi_m + b) / (1 + sqrt(1 + b (2 phi_m + b))),
 * and phi_g = 2 s - phi_m = phi_m + 2 (s - phi_m).
 * The factor 1 - phi_w^2 is built on the bulk values +-1: the offset s - phi_m
 * is taken at phi_m clamped to [-1, 1] (it vanishes at +-1), so the ghost of a
 * value beyond +-1 is its mirror, b = 0 mirrors every value, and the root
 * stays real for |b| <= 1 (W >= 2 dx) where an overshoot of phi past 1 next to
 * a wall with cos(theta) near -1 would otherwise leave the quadratic without
 * a real root. */
static double wet_ghost(double m, double b)
{
    double mc = m > 1.0 ? 1.0 : (m < -1.0 ? -1.0 : m);
    double s = (2.0 * mc + b) / (1.0 + sqrt(1.0 + b * (2.0 * mc + b)));
    return m + 2.0 * (s - mc);
}

/* Fill the ghost layer of the order parameter: periodic wrap or mirror,
 * then the wetting rule of each crossed wall face (x, y, z order). */
static void fill_phi(const orc_params* p, const pgrid* g, double* f)
{
    int kl = (g->dim == 3) ? -1 : 0, kh = (g->dim == 3) ? g->nz : 0;
    for (int k = kl; k <= kh; ++k)
        for (int j = -1; j <= g->ny; ++j)
            for (int i = -1; i <= g->nx; ++i) {
                if (!is_ghost(g, i, j, k)) continue;
                int fc[3] = {-1, -1, -1};
                int si = map_axis(i, g->nx, p->bc[0], p->bc[1], 0, &fc[0]);
                int sj = map_axis(j, g->ny, p->bc[2], p->bc[3], 2, &fc[1]);
                int sk = (g->dim == 3) ? map_axis(k, g->nz, p->bc[4], p->bc[5], 4, &fc[2]) : 0;
                double val = f[P(g, si, sj, sk)];
                for (int a = 0; a < 3; ++a) {
                    int face = fc[a];
                    if (face >= 0 && p->bc[face] == ORC_WALL)
                        val = wet_ghost(val, p->dx * (2.0 / p->width) * p->wet_cos[face]);
                }
                f[P(g, i, j, k)] = val;
            }
}

/* Velocity rule when a face is crossed: wall -> 2 u_w - u (every component),
 * symmetry -> normal component negated. */
static void apply_face(const orc_params* p, int face, double* uvw)
{
    if (face < 0) return;
    int t = p->bc[face];
    if (t == ORC_WALL) {
        for (int c = 0; c < 3; ++c) uvw[c] = 2.0 * p->wall_u[face][c] - uvw[c];
    } else if (t == ORC_SYMMETRY) {
        int axis = face / 2;
        uvw[axis] = -uvw[axis];
    }
}

/* Fill ghost velocity (faces applied in the order x, y, z). */
static void fill_velocity(const orc_params* p, const pgrid* g, double* u, double* v, double* w)
{
    int kl = (g->dim == 3) ? -1 : 0, kh = (g->dim == 3) ? g->nz : 0;
    for (int k = kl; k <= kh; ++k)
        for (int j = -1; j <= g->ny; ++j)
            for (int i = -1; i <= g->nx; ++i) {
                if (!is_ghost(g, i, j, k)) continue;
                int fx, fy, fz = -1;
                int si = map_axis(i, g->nx, p->bc[0], p->bc[1], 0, &fx);
                int sj = map_axis(j, g->ny, p->bc[2], p->bc[3], 2, &fy);
                int sk = (g->dim == 3) ? map_axis(k, g->nz, p->bc[4], p->bc[5], 4, &fz) : 0;
                long s = P(g, si, sj, sk);
                double q[3];
                q[0] = u[s];
                q[1] = v[s];
                q[2] = (g->dim == 3) ? w[s] : 0.0;
                apply_face(p, fx, q);
                apply_face(p, fy, q);
                if (g->dim == 3) apply_face(p, fz, q);
                long d = P(g, i, j, k);
                u[d] = q[0];
                v[d] = q[1];
                if (g->dim == 3) w[d] = q[2];
            }
}

static void to_padded(const pgrid* g, const double* src, double* dst)
{
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) dst[P(g, i, j, k)] = src[D(g, i, j, k)];
}

static int check_params(const orc_params* p)
{
    if (!p) return -1;
    if (p->dim != 2 && p->dim != 3) return -1;
    if (p->nx < 2 || p->ny < 2) return -1;
    if (p->dim == 3 && p->nz < 2) return -1;
    if (p->two_phase && !(p->width > 0.0)) return -1;
    if (p->axisym && (p->dim != 2 || p->bc[2] != ORC_SYMMETRY)) return -1;
    int nf = (p->dim == 3) ? 6 : 4;
    for (int a = 0; a < nf; a += 2) {
        int lo = p->bc[a], hi = p->bc[a + 1];
        if ((lo == ORC_PERIODIC) != (hi == ORC_PERIODIC)) return -1;
        if (lo < 0 || lo > 2 || hi < 0 || hi > 2) return -1;
    }
    return 0;
}

/* offsets of the axis neighbours in the padded array */
static void axis_strides(const pgrid* g, long s[3])
{
    s[0] = 1;
    s[1] = g->px;
    s[2] = (long)g->px * g->py;
}

/* ------------------------------------------------------------------ */
/* isotropic stencils: D2Q9 weights in 2D, D3Q19 weights in 3D           */
/* (Sec. 2: "second-order isotropic schemes"; the weights w_i of the      */
/* lattice give d_a f = 3 sum_i w_i e_ia f_i / dx and                     */
/* d_aa f = 6 sum_i w_i (f_i - f_0) / dx^2)                               */
/* ------------------------------------------------------------------ */
/* gradient along axis a:
 *   2D: [4 (f_{+a} - f_{-a}) + sum_{+-b} (f_{+a+-b} - f_{-a+-b})] / (12 dx)
 *   3D: [2 (f_{+a} - f_{-a}) + sum_{b != a} sum_{+-b} (f_{+a+-b} - f_{-a+-b})] / (12 dx) */
static double giso(const orc_params* p, const double* f, long c, const long st[3], int a)
{
    double face = f[c + st[a]] - f[c - st[a]];
    double edge = 0.0;
    for (int b = 0; b < p->dim; ++b) {
        if (b == a) continue;
        edge += (f[c + st[a] + st[b]] + f[c + st[a] - st[b]]) - (f[c - st[a] + st[b]] + f[c - st[a] - st[b]]);
    }
    double wf = (p->dim == 2) ? 4.0 : 2.0;
    return (wf * face + edge) / (12.0 * p->dx);
}

/* Laplacian:
 *   2D: [4 (sum of the 4 axis neighbours) + (sum of the 4 diagonal ones) - 20 f] / (6 dx^2)
 *   3D: [2 (sum of the 6 face neighbours) + (sum of the 12 edge ones) - 24 f] / (6 dx^2) */
static double liso(const orc_params* p, const double* f, long c, const long st[3])
{
    double ax = 0.0, ed = 0.0;
    for (int a = 0; a < p->dim; ++a) {
        ax += f[c + st[a]] + f[c - st[a]];
        for (int b = a + 1; b < p->dim; ++b)
            ed += (f[c + st[a] + st[b]] + f[c + st[a] - st[b]]) + (f[c - st[a] + st[b]] + f[c - st[a] - st[b]]);
    }
    double wa = (p->dim == 2) ? 4.0 : 2.0, w0 = (p->dim == 2) ? 20.0 : 24.0;
    return (wa * ax + ed - w0 * f[c]) / (6.0 * p->dx * p->dx);
}

/* axisymmetric runs: (1/r) G_iso,r f, the extra part of the cylindrical
 * Laplacian (1/r) d_r(r d_r f) = d_rr f + (1/r) d_r f, with the radius of
 * the node (row j at r = (j + 1/2) dx); 0 for planar runs */
static double axi_lap_extra(const orc_params* p, const pgrid* g, const double* f, long c, const long st[3])
{
    if (!p->axisym) return 0.0;
    int j = (int)((c / g->px) % g->py) - 1;
    return giso(p, f, c, st, 1) / ((j + 0.5) * p->dx);
}

/* mu = 4 a phi (phi^2 - 1) - kappa L_iso phi on interior nodes of padded arrays,
 * a = 3 sigma / (4 W), kappa = 3 sigma W / 8 (Sec. 2); axisymmetric runs
 * take the cylindrical Laplacian L_iso phi + (1/r) G_iso,r phi */
static void chem_pot(const orc_params* p, const pgrid* g, const double* phi, double* mu)
{
    double a = 3.0 * p->sigma / (4.0 * p->width);
    double kappa = 3.0 * p->sigma * p->width / 8.0;
    long st[3];
    axis_strides(g, st);
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                long c = P(g, i, j, k);
                double f = phi[c];
                mu[c] = 4.0 * a * f * (f * f - 1.0) - kappa * (liso(p, phi, c, st) + axi_lap_extra(p, g, phi, c, st));
            }
}

/* CHE right-hand side (2.14): R = M L_iso mu - u_a G_iso,a phi (cylindrical
 * Laplacian in axisymmetric runs; the advection u . grad phi has no extra
 * term) */
static double che_rhs(const orc_params* p, const pgrid* g, const double* phi, const double* mu,
                      double* const uu[3], long c)
{
    long st[3];
    axis_strides(g, st);
    double diff = p->mobility * (liso(p, mu, c, st) + axi_lap_extra(p, g, mu, c, st));
    double adv = 0.0;
    for (int a = 0; a < p->dim; ++a) adv += uu[a][c] * giso(p, phi, c, st, a);
    return diff - adv;
}

/* ------------------------------------------------------------------ */
/* one step                                                             */
/* ------------------------------------------------------------------ */
int orc_step(const orc_params* p, const double* force_x_row,
             const double* drho, const double* u, const double* v,
             const double* w, const double* phi,
             double* out_drho, double* out_u, double* out_v,
             double* out_w, double* out_phi)
{
    if (check_params(p)) return -1;
    if (p->dim == 3 && (!w || !out_w)) return -1;
    if (p->two_phase && (!phi || !out_phi)) return -1;
    pgrid g = make_grid(p);
    long np = (long)g.px * g.py * g.pz;
    int nv = p->dim;
    /* padded arrays: drho, u, v, w, m0, m1, m2, drho_new, phi, mu, phis, mus */
    double* buf = (double*)calloc((size_t)np * 12, sizeof(double));
    if (!buf) return -2;
    double* r = buf;
    double* uu[3] = {buf + np, buf + 2 * np, buf + 3 * np};
    double* m[3] = {buf + 4 * np, buf + 5 * np, buf + 6 * np};
    double* rn = buf + 7 * np;
    double* ph = buf + 8 * np;
    double* mu = buf + 9 * np;
    double* phs = buf + 10 * np;
    double* mus = buf + 11 * np;

    /* 1. level-n fields with ghosts */
    to_padded(&g, drho, r);
    to_padded(&g, u, uu[0]);
    to_padded(&g, v, uu[1]);
    if (nv == 3) to_padded(&g, w, uu[2]);
    fill_scalar(p, &g, r);
    fill_velocity(p, &g, uu[0], uu[1], uu[2]);
    for (long q = 0; q < np; ++q) {
        double rho = p->rho0 + r[q];
        for (int a = 0; a < nv; ++a) m[a][q] = rho * uu[a][q];
    }
    if (p->two_phase) {
        to_padded(&g, phi, ph);
        fill_phi(p, &g, ph);
        chem_pot(p, &g, ph, mu);
        fill_scalar(p, &g, mu);
    }

    long st[3];
    axis_strides(&g, st);
    const double dx = p->dx, dt = p->dt, cs2 = p->cs * p->cs, nu = p->nu;

    /* 2. continuity, Eq. (2.10):
     *    rho' = rho - dt d_a(rho u_a) + 1/2 cs^2 dt^2 d_aa rho
     * Axisymmetric runs (y = radius r, axis on the -y face) take the
     * cylindrical divergence (1/r) d_r(r f) and Laplacian (1/r) d_r(r d_r f)
     * in flux form with face radii r -+ dx/2: the face value of f is the
     * mean of its two nodes, which is the centred difference (2.12) away
     * from the axis and makes sum(r drho) exact with the axis and wall
     * ghosts. */
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i < g.nx; ++i) {
                long c = P(&g, i, j, k);
                double div = 0.0, lap = 0.0;
                for (int a = 0; a < nv; ++a) {
                    if (p->axisym && a == 1) {
                        const double rc = j + 0.5, rp = j + 1.0, rm = j;  /* radii in units of dx */
                        long cp = c + st[1], cm = c - st[1];
                        div += (rp * (m[1][c] + m[1][cp]) - rm * (m[1][cm] + m[1][c])) / (2.0 * dx * rc);
                        lap += (rp * (r[cp] - r[c]) - rm * (r[c] - r[cm])) / (dx * dx * rc);
                        continue;
                    }
                    div += (m[a][c + st[a]] - m[a][c - st[a]]) / (2.0 * dx);
                    lap += (r[c + st[a]] + r[c - st[a]] - 2.0 * r[c]) / (dx * dx);
                }
                rn[c] = r[c] - dt * div + p->sat_rho * 0.5 * cs2 * dt * dt * lap;
            }
    /* 3. ghosts of rho^{n+1} */
    fill_scalar(p, &g, rn);

    /* 4-5. momentum, Eq. (2.11), then u = m / rho */
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i < g.nx; ++i) {
                long c = P(&g, i, j, k);
                long d = D(&g, i, j, k);
                double rho_new = p->rho0 + rn[c];
                double mn[3];
                for (int a = 0; a < nv; ++a) {
                    double flux = 0.0, visc = 0.0;
                    for (int b = 0; b < nv; ++b) {
                        long cp = c + st[b], cm = c - st[b];
                        /* Pi_ab = rho u_a u_b + cs^2 drho delta_ab */
                        double pip = m[a][cp] * uu[b][cp];
                        double pim = m[a][cm] * uu[b][cm];
                        if (a == b) {
                            pip += cs2 * r[cp];
                            pim += cs2 * r[cm];
                        }
                        if (p->axisym && b == 1) {  /* (1/r) d_r(r Pi_ar), (1/r) d_r(r d_r m_a) */
                            const double rc = j + 0.5, rp = j + 1.0, rm = j;
                            double pic = m[a][c] * uu[b][c] + (a == b ? cs2 * r[c] : 0.0);
                            flux += (rp * (pic + pip) - rm * (pim + pic)) / (2.0 * dx * rc);
                            visc += (rp * (m[a][cp] - m[a][c]) - rm * (m[a][c] - m[a][cm])) / (dx * dx * rc);
                            continue;
                        }
                        flux += (pip - pim) / (2.0 * dx);
                        visc += (m[a][cp] + m[a][cm] - 2.0 * m[a][c]) / (dx * dx);
                    }
                    if (p->axisym && a == 1) {
                        /* radial component: hoop term -Pi_thth / r of the
                         * divergence (Pi_thth = cs^2 drho without swirl) and
                         * -m_r / r^2 of the vector Laplacian */
                        const double rr = (j + 0.5) * dx;
                        flux -= cs2 * r[c] / rr;
                        visc -= m[1][c] / (rr * rr);
                    }
                    long ap = c + st[a], am = c - st[a];
                    double grad_new = (rn[ap] - rn[am]) / (2.0 * dx);
                    double grad_old = (r[ap] - r[am]) / (2.0 * dx);
                    double sat = (nu + 0.5 * cs2 * dt) * (grad_new - grad_old);
                    double ga = p->g[a];
                    if (a == 0 && force_x_row) ga += force_x_row[j];
                    mn[a] = m[a][c] - dt * flux + nu * dt * visc - p->sat_mom * sat + dt * rho_new * ga;
                }
                if (p->two_phase)  /* surface tension -dt phi G_iso mu (Sec. 2) */
                    for (int a = 0; a < nv; ++a) mn[a] -= dt * ph[c] * giso(p, mu, c, st, a);
                out_drho[d] = rn[c];
                out_u[d] = mn[0] / rho_new;
                out_v[d] = mn[1] / rho_new;
                if (nv == 3) out_w[d] = mn[2] / rho_new;
            }

    /* 6. Cahn-Hilliard (2.14) by Heun's method with u^n */
    if (p->two_phase) {
        for (int k = 0; k < g.nz; ++k)
            for (int j = 0; j < g.ny; ++j)
                for (int i = 0; i < g.nx; ++i) {
                    long c = P(&g, i, j, k);
                    phs[c] = ph[c] + dt * che_rhs(p, &g, ph, mu, uu, c);
                }
        fill_phi(p, &g, phs);
        chem_pot(p, &g, phs, mus);
        fill_scalar(p, &g, mus);
        for (int k = 0; k < g.nz; ++k)
            for (int j = 0; j < g.ny; ++j)
                for (int i = 0; i < g.nx; ++i) {
                    long c = P(&g, i, j, k);
                    double r2 = che_rhs(p, &g, phs, mus, uu, c);
                    out_phi[D(&g, i, j, k)] = 0.5 * (ph[c] + phs[c] + dt * r2);
                }
    }
    free(buf);
    return 0;
}

int orc_run(const orc_params* p, const double* force_x_row, long nsteps,
            double* drho, double* u, double* v, double* w, double* phi)
{
    if (check_params(p)) return -1;
    pgrid g = make_grid(p);
    long n = (long)g.nx * g.ny * g.nz;
    double* t = (double*)malloc((size_t)n * 5 * sizeof(double));
    if (!t) return -2;
    double *a[5] = {drho, u, v, w, phi};
    double *b[5] = {t, t + n, t + 2 * n, t + 3 * n, t + 4 * n};
    for (long s = 0; s < nsteps; ++s) {
        int rc = orc_step(p, force_x_row, a[0], a[1], a[2], a[3], a[4],
                          b[0], b[1], b[2], (p->dim == 3) ? b[3] : NULL,
                          p->two_phase ? b[4] : NULL);
        if (rc) {
            free(t);
            return rc;
        }
        for (int f = 0; f < 5; ++f) {
            double* x = a[f];
            a[f] = b[f];
            b[f] = x;
        }
    }
    /* the newest state is in a[]; copy it back into the caller arrays */
    if (nsteps % 2 == 1) {
        memcpy(drho, a[0], (size_t)n * sizeof(double));
        memcpy(u, a[1], (size_t)n * sizeof(double));
        memcpy(v, a[2], (size_t)n * sizeof(double));
        if (p->dim == 3) memcpy(w, a[3], (size_t)n * sizeof(double));
        if (p->two_phase) memcpy(phi, a[4], (size_t)n * sizeof(double));
    }
    free(t);
    return 0;
}

int orc_chemical_potential(const orc_params* p, const double* phi, double* out)
{
    if (check_params(p)) return -1;
    pgrid g = make_grid(p);
    long np = (long)g.px * g.py * g.pz;
    double* ph = (double*)calloc((size_t)np * 2, sizeof(double));
    if (!ph) return -2;
    double* mu = ph + np;
    to_padded(&g, phi, ph);
    fill_phi(p, &g, ph);
    chem_pot(p, &g, ph, mu);
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i < g.nx; ++i) out[D(&g, i, j, k)] = mu[P(&g, i, j, k)];
    free(ph);
    return 0;
}

/* ------------------------------------------------------------------ */
/* diagnostics                                                          */
/* ------------------------------------------------------------------ */
int orc_diag(const orc_params* p, const double* drho, const double* u,
             const double* v, const double* w, const double* phi,
             const double* prev_u, const double* prev_v, const double* prev_w,
             double* out)
{
    if (check_params(p)) return -1;
    pgrid g = make_grid(p);
    long np = (long)g.px * g.py * g.pz;
    int nv = p->dim;
    double* buf = (double*)calloc((size_t)np * 3, sizeof(double));
    if (!buf) return -2;
    double* uu[3] = {buf, buf + np, buf + 2 * np};
    to_padded(&g, u, uu[0]);
    to_padded(&g, v, uu[1]);
    if (nv == 3) to_padded(&g, w, uu[2]);
    fill_velocity(p, &g, uu[0], uu[1], uu[2]);
    long st[3];
    axis_strides(&g, st);
    /* axisymmetric runs weight every node by its cell volume 2 pi r dx^2
     * (row j at r = (j + 1/2) dx): sums (mass, momentum, kinetic energy,
     * sum phi) are volume integrals and the means (enstrophy, energy, rms
     * divergence) are volume averages; planar runs weight nodes by 1 and
     * scale the sums by dx^D */
    const double PI = 3.14159265358979323846;
    double dxd = (nv == 3) ? p->dx * p->dx * p->dx : p->dx * p->dx;
    double vol = 0;
    double mass = 0, mom[3] = {0, 0, 0}, ke = 0, dumax = 0, umax = 0, ens = 0;
    double div2 = 0, divmax = 0, phisum = 0;
    int bad = 0;
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i < g.nx; ++i) {
                long c = P(&g, i, j, k);
                long d = D(&g, i, j, k);
                const double cv = p->axisym ? 2.0 * PI * (j + 0.5) * p->dx * dxd : 1.0;
                vol += cv;
                double rho = p->rho0 + drho[d];
                double q2 = 0;
                for (int a = 0; a < nv; ++a) {
                    mom[a] += rho * uu[a][c] * cv;
                    q2 += uu[a][c] * uu[a][c];
                }
                mass += drho[d] * cv;
                ke += q2 * cv;
                double mag = sqrt(q2);
                if (mag > umax) umax = mag;
                if (prev_u) {
                    double pq = prev_u[d] * prev_u[d] + prev_v[d] * prev_v[d];
                    if (nv == 3) pq += prev_w[d] * prev_w[d];
                    double dm = fabs(mag - sqrt(pq));
                    if (dm > dumax) dumax = dm;
                }
                /* centred derivatives d_b u_a */
                double du[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
                for (int a = 0; a < nv; ++a)
                    for (int b = 0; b < nv; ++b)
                        du[a][b] = (uu[a][c + st[b]] - uu[a][c - st[b]]) / (2.0 * p->dx);
                double om2;
                if (nv == 2) {
                    double oz = du[1][0] - du[0][1];
                    om2 = oz * oz;
                } else {
                    double ox = du[2][1] - du[1][2];
                    double oy = du[0][2] - du[2][0];
                    double oz = du[1][0] - du[0][1];
                    om2 = ox * ox + oy * oy + oz * oz;
                }
                ens += om2 * cv;
                double dv = 0;
                for (int a = 0; a < nv; ++a) dv += du[a][a];
                if (p->axisym) {  /* (1/r) d_r(r u_r) in the face form of the step */
                    const double rc = j + 0.5, rp = j + 1.0, rm = j;
                    dv = du[0][0] + (rp * (uu[1][c] + uu[1][c + st[1]]) - rm * (uu[1][c - st[1]] + uu[1][c])) /
                                        (2.0 * p->dx * rc);
                }
                div2 += dv * dv * cv;
                if (fabs(dv) > divmax) divmax = fabs(dv);
                if (p->two_phase && phi) phisum += phi[d] * cv;
                double vals[5] = {drho[d], u[d], v[d], (nv == 3) ? w[d] : 0.0,
                                  (p->two_phase && phi) ? phi[d] : 0.0};
                for (int f = 0; f < 5; ++f)
                    if (!isfinite(vals[f])) bad = 1;
            }
    const double sc = p->axisym ? 1.0 : dxd;  /* planar sums are node sums times dx^D */
    out[0] = mass * sc;
    out[1] = mom[0] * sc;
    out[2] = mom[1] * sc;
    out[3] = mom[2] * sc;
    out[4] = 0.5 * ke * sc;
    out[5] = dumax;
    out[6] = umax;
    out[7] = ens / (2.0 * vol);
    out[8] = ke / (2.0 * vol);
    out[9] = sqrt(div2 / vol);
    out[10] = divmax;
    out[11] = phisum;
    out[12] = bad ? 1.0 : 0.0;
    free(buf);
    return 0;
}
