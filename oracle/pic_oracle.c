/*
 * pic_oracle.c -- plain, serial, double-precision CPU reference of the
 * charge-conserving particle-in-cell step with alternating-order field
 * interpolation (Sokolov, "Alternating-Order Interpolation in a
 * Charge-Conserving Scheme for Particle-In-Cell Simulations",
 * arXiv:1101.0809).
 *
 * TEST INFRASTRUCTURE.  This file is the independent checker of the GPU
 * library.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it; the product never does.  It shares no code, header,
 * table or constant with the GPU path.  Everything is evaluated the slow,
 * obvious way: shape functions are written as functions of the distance to
 * the particle (their definition), interpolation sums run over a superset of
 * the support, and the current is the six-box-path average written in its
 * one-sixth form.
 *
 * Conventions (paper Section 2):
 *   - positions are normalised, x/dx, y/dy, z/dz ("cell units"); time step
 *     dt; speed of light c; Courant numbers cx = c dt/dx, cy, cz; V = dx dy dz.
 *   - grid functions are stored [k][j][i], i fastest, on a periodic box:
 *       Ex[k][j][i] = E^x at (i, j+1/2, k+1/2), Ey at (i+1/2, j, k+1/2),
 *       Ez at (i+1/2, j+1/2, k)                        (face centres)
 *       Bx[k][j][i] = B^x at (i+1/2, j, k), By at (i, j+1/2, k),
 *       Bz at (i, j, k+1/2)                            (edge midpoints)
 *       J is stored like E; rho[k][j][i] sits at (i+1/2, j+1/2, k+1/2).
 *   - the field buffer holds 9 planes of nx*ny*nz doubles in the order
 *     Ex Ey Ez Bx By Bz Jx Jy Jz.
 *   - state at the start of a step: E^n, B^{n-1/2}, x^n, w^{n-1/2}, where w
 *     is momentum over mass (gamma * v).
 */
#include "pic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double PI = 3.14159265358979323846;

/* ---------------------------------------------------------------------------
 * Form-factor family (Section 3.1).  f^(0) is the unit cap of width one,
 * f^(l+1)(r) is the integral of f^(l) over [r-1/2, r+1/2].  The closed forms
 * below are those integrals carried out; the tests check them against a
 * numerical convolution of the cap.  r is the distance x - x_p in cells.
 * ------------------------------------------------------------------------- */
double orc_shape(int l, double r)
{
    double a = fabs(r);
    switch (l) {
    case 0:
        return a <= 0.5 ? 1.0 : 0.0;
    case 1:
        return a < 1.0 ? 1.0 - a : 0.0;
    case 2:
        if (a <= 0.5) return 0.75 - a * a;
        if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
        return 0.0;
    case 3:
        if (a <= 1.0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
        if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
        return 0.0;
    default:
        return NAN;
    }
}

/* Integral of f^(1) from -infinity to s: the cumulative form factor F_i of
 * Section 3.1 with s = i - x_p. */
double orc_cumulative1(double s)
{
    if (s <= -1.0) return 0.0;
    if (s <= 0.0) return 0.5 * (1.0 + s) * (1.0 + s);
    if (s < 1.0) return 1.0 - 0.5 * (1.0 - s) * (1.0 - s);
    return 1.0;
}

/* Integral of f^(2) from -infinity to s (the cumulative form factor of order
 * 2, for the order-2 1/2 current). */
double orc_cumulative2(double s)
{
    if (s <= -1.5) return 0.0;
    if (s <= -0.5) return (1.5 + s) * (1.5 + s) * (1.5 + s) / 6.0;
    if (s <= 0.5) return 1.0 / 6.0 + 0.75 * (s + 0.5) - (s * s * s + 0.125) / 3.0;
    if (s < 1.5) return 1.0 - (1.5 - s) * (1.5 - s) * (1.5 - s) / 6.0;
    return 1.0;
}

/* Alternating form factor of order l + 1/2 (Section 4.5), l = g->order: at
 * an integer point (node) n it is f^(l)(n - x_p); at a half-integer point
 * (cell centre c+1/2) it is Delta F_{c+1/2}(x_p) = f^(l+1)(c + 1/2 - x_p);
 * the current uses the cumulative F_n of f^(l) (Section 3.1). */
static int order_of(const orc_grid* g) { return g->order == 2 ? 2 : 1; }
static double node_w(const orc_grid* g, long n, double xp) { return orc_shape(order_of(g), (double)n - xp); }
static double cell_w(const orc_grid* g, long c, double xp)
{
    return orc_shape(order_of(g) + 1, (double)c + 0.5 - xp);
}
static double cumul(const orc_grid* g, long n, double xp)
{
    return order_of(g) == 2 ? orc_cumulative2((double)n - xp) : orc_cumulative1((double)n - xp);
}

static long wrap(long i, long n)
{
    long r = i % n;
    return r < 0 ? r + n : r;
}

static size_t idx(const orc_grid* g, long i, long j, long k)
{
    return ((size_t)wrap(k, g->nz) * (size_t)g->ny + (size_t)wrap(j, g->ny)) * (size_t)g->nx
           + (size_t)wrap(i, g->nx);
}

static size_t ncell(const orc_grid* g) { return (size_t)g->nx * g->ny * g->nz; }

/* ---------------------------------------------------------------------------
 * Field interpolation (Section 4.1, Eq. alphax; Section 4.2, Eq. betax).
 *   alpha^x_{i,j+1/2,k+1/2} = f_i(x) dF_{j+1/2}(y) dF_{k+1/2}(z), cyclic;
 *   beta^x_{i+1/2,j,k}      = dF_{i+1/2}(x) f_j(y) f_k(z),       cyclic.
 * The sums run over a box around the particle that contains the support of
 * every weight; weights outside the support are exactly zero.
 * ------------------------------------------------------------------------- */
/* Summation boxes: offsets -BOX_LO .. +BOX_HI from floor(x_p) contain every
 * node with a non-zero f_i (order 1 1/2: offsets 0, 1; order 2 1/2: -1..2)
 * and every cell with a non-zero Delta F (-1..1; -2..2); the extra entries
 * get exactly zero weight.  For the current the box runs from floor of the
 * lower end point to floor of the upper one, widened the same way, which
 * holds every node whose cumulative F changes (F_n(x) is constant outside
 * |n - x| < 1 resp. 3/2). */
#define BOX_LO 2
#define BOX_HI 2

/* Weight of a component at node n along one of its node axes: f_n(x_p) for
 * the alternating form factor; for the conventional interpolation of Eq.
 * wrong1 the mean of the cell factors of the two cells that share the node,
 * (Delta F_{n-1/2} + Delta F_{n+1/2}) / 2. */
static double node_gather_w(const orc_grid* g, long n, double xp)
{
    if (g->interp == 1) return 0.5 * (cell_w(g, n - 1, xp) + cell_w(g, n, xp));
    return node_w(g, n, xp);
}

void orc_gather(const orc_grid* g, const double* fields, const double xp[3], double Ep[3],
                double Bp[3])
{
    const size_t nc = ncell(g);
    const double* F[6];
    for (int c = 0; c < 6; ++c) F[c] = fields + (size_t)c * nc;
    long base[3];
    for (int a = 0; a < 3; ++a) base[a] = (long)floor(xp[a]);

    /* one-dimensional factors, indexed by offset o = index - base + BOX_LO */
    double nw[3][BOX_LO + BOX_HI + 1], cw[3][BOX_LO + BOX_HI + 1];
    for (int a = 0; a < 3; ++a)
        for (int o = 0; o <= BOX_LO + BOX_HI; ++o) {
            long n = base[a] + o - BOX_LO;
            nw[a][o] = node_gather_w(g, n, xp[a]);
            cw[a][o] = cell_w(g, n, xp[a]);
        }

    for (int c = 0; c < 3; ++c) Ep[c] = Bp[c] = 0.0;
    for (int ok = 0; ok <= BOX_LO + BOX_HI; ++ok)
        for (int oj = 0; oj <= BOX_LO + BOX_HI; ++oj)
            for (int oi = 0; oi <= BOX_LO + BOX_HI; ++oi) {
                long i = base[0] + oi - BOX_LO, j = base[1] + oj - BOX_LO, k = base[2] + ok - BOX_LO;
                size_t p = idx(g, i, j, k);
                double ax = nw[0][oi] * cw[1][oj] * cw[2][ok];
                double ay = cw[0][oi] * nw[1][oj] * cw[2][ok];
                double az = cw[0][oi] * cw[1][oj] * nw[2][ok];
                double bx = cw[0][oi] * nw[1][oj] * nw[2][ok];
                double by = nw[0][oi] * cw[1][oj] * nw[2][ok];
                double bz = nw[0][oi] * nw[1][oj] * cw[2][ok];
                Ep[0] += ax * F[0][p];
                Ep[1] += ay * F[1][p];
                Ep[2] += az * F[2][p];
                Bp[0] += bx * F[3][p];
                Bp[1] += by * F[4][p];
                Bp[2] += bz * F[5][p];
            }
    for (int c = 0; c < 3; ++c) Bp[c] += g->bext[c];
}

/* ---------------------------------------------------------------------------
 * Momentum advance (Appendix; equation of motion Eq. (1)):
 *   e = q dt E / (2m);  w~ = w + e;  b = q dt B / (2 m sqrt(w~^2 + c^2));
 *   w' = w~ + w~ x b;   w_new = w~ + e + 2 (w' x b) / (1 + b^2).
 * ------------------------------------------------------------------------- */
static void cross(const double a[3], const double b[3], double r[3])
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

void orc_push(double q_over_m, double dt, double c, const double Ep[3], const double Bp[3],
              double w[3])
{
    double e[3], wt[3], b[3], wp[3], t[3];
    for (int a = 0; a < 3; ++a) e[a] = 0.5 * q_over_m * dt * Ep[a];
    for (int a = 0; a < 3; ++a) wt[a] = w[a] + e[a];
    double g = sqrt(wt[0] * wt[0] + wt[1] * wt[1] + wt[2] * wt[2] + c * c);
    for (int a = 0; a < 3; ++a) b[a] = 0.5 * q_over_m * dt * Bp[a] / g;
    cross(wt, b, t);
    for (int a = 0; a < 3; ++a) wp[a] = wt[a] + t[a];
    double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    cross(wp, b, t);
    for (int a = 0; a < 3; ++a) w[a] = wt[a] + e[a] + 2.0 * t[a] / (1.0 + b2);
}

/* Velocity over c and the displacement in cell units (Eq. coordscheme). */
void orc_displacement(const orc_grid* g, const double w[3], double dxp[3])
{
    double gam = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + g->c * g->c);
    const double h[3] = {g->dx, g->dy, g->dz};
    for (int a = 0; a < 3; ++a) dxp[a] = (w[a] / gam) * (g->c * g->dt / h[a]);
}

/* ---------------------------------------------------------------------------
 * Charge-conserving current of one particle moving from x0 to x1 (both in
 * cell units, x1 not wrapped), Section 3.2: the average of the six box paths
 * (edges parallel to the axes), in the one-sixth form
 *   xi^x_{i,j+1/2,k+1/2} = -(1/6)(dx/dt)[F_i(x1) - F_i(x0)]
 *        * { 2[dF_j(y1)dF_k(z1) + dF_j(y0)dF_k(z0)] + dF_j(y1)dF_k(z0) + dF_j(y0)dF_k(z1) }
 * and cyclic.  Adds (q/V) xi into J (Eq. xi).
 * ------------------------------------------------------------------------- */
void orc_deposit(const orc_grid* g, const double x0[3], const double x1[3], double charge,
                 double* J)
{
    const size_t nc = ncell(g);
    double* Jc[3] = {J, J + nc, J + 2 * nc};
    const double V = g->dx * g->dy * g->dz;
    const double h[3] = {g->dx, g->dy, g->dz};
    long lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        double m = x0[a] < x1[a] ? x0[a] : x1[a];
        double M = x0[a] < x1[a] ? x1[a] : x0[a];
        lo[a] = (long)floor(m) - BOX_LO;
        hi[a] = (long)floor(M) + BOX_HI;
    }
    for (int comp = 0; comp < 3; ++comp) {
        int t1 = (comp + 1) % 3, t2 = (comp + 2) % 3; /* transverse axes */
        double pref = -(1.0 / 6.0) * (h[comp] / g->dt) * charge / V;
        for (long a = lo[comp]; a <= hi[comp]; ++a) {
            double dF = cumul(g, a, x1[comp]) - cumul(g, a, x0[comp]);
            if (dF == 0.0) continue;
            for (long b = lo[t1]; b <= hi[t1]; ++b) {
                double s0b = cell_w(g, b, x0[t1]), s1b = cell_w(g, b, x1[t1]);
                if (s0b == 0.0 && s1b == 0.0) continue;
                for (long cc = lo[t2]; cc <= hi[t2]; ++cc) {
                    double s0c = cell_w(g, cc, x0[t2]), s1c = cell_w(g, cc, x1[t2]);
                    double brace = 2.0 * (s1b * s1c + s0b * s0c) + s1b * s0c + s0b * s1c;
                    if (brace == 0.0) continue;
                    long ijk[3];
                    ijk[comp] = a;
                    ijk[t1] = b;
                    ijk[t2] = cc;
                    Jc[comp][idx(g, ijk[0], ijk[1], ijk[2])] += pref * dF * brace;
                }
            }
        }
    }
}

/* The same current in the one-quarter form of Eq. current, with the
 * cumulative difference obtained from partial sums of dF^- over cells left of
 * the face, as the paper's recursive formula states.  Used by the tests to
 * check that the two printed forms agree. */
void orc_deposit_quarter(const orc_grid* g, const double x0[3], const double x1[3],
                         double charge, double* J)
{
    const size_t nc = ncell(g);
    double* Jc[3] = {J, J + nc, J + 2 * nc};
    const double V = g->dx * g->dy * g->dz;
    const double h[3] = {g->dx, g->dy, g->dz};
    long lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        double m = x0[a] < x1[a] ? x0[a] : x1[a];
        double M = x0[a] < x1[a] ? x1[a] : x0[a];
        lo[a] = (long)floor(m) - BOX_LO;
        hi[a] = (long)floor(M) + BOX_HI;
    }
    for (int comp = 0; comp < 3; ++comp) {
        int t1 = (comp + 1) % 3, t2 = (comp + 2) % 3;
        double pref = -0.25 * (h[comp] / g->dt) * charge / V;
        double partial = 0.0; /* sum over cells c < a of dF^-_{c+1/2} */
        for (long a = lo[comp]; a <= hi[comp]; ++a) {
            if (a > lo[comp])
                partial += cell_w(g, a - 1, x1[comp]) - cell_w(g, a - 1, x0[comp]);
            if (partial == 0.0) continue;
            for (long b = lo[t1]; b <= hi[t1]; ++b) {
                double pb = cell_w(g, b, x1[t1]) + cell_w(g, b, x0[t1]);
                double mb = cell_w(g, b, x1[t1]) - cell_w(g, b, x0[t1]);
                for (long cc = lo[t2]; cc <= hi[t2]; ++cc) {
                    double pc = cell_w(g, cc, x1[t2]) + cell_w(g, cc, x0[t2]);
                    double mc = cell_w(g, cc, x1[t2]) - cell_w(g, cc, x0[t2]);
                    double tr = pb * pc + mb * mc / 3.0;
                    if (tr == 0.0) continue;
                    long ijk[3];
                    ijk[comp] = a;
                    ijk[t1] = b;
                    ijk[t2] = cc;
                    Jc[comp][idx(g, ijk[0], ijk[1], ijk[2])] += pref * partial * tr;
                }
            }
        }
    }
}

/* Charge density of Eq. rho: (1/V) sum_p q_p dF_{i+1/2}(x) dF_{j+1/2}(y) dF_{k+1/2}(z). */
void orc_rho_add(const orc_grid* g, const double xp[3], double charge, double* rho)
{
    const double V = g->dx * g->dy * g->dz;
    long base[3];
    for (int a = 0; a < 3; ++a) base[a] = (long)floor(xp[a]);
    for (long k = base[2] - BOX_LO; k <= base[2] + BOX_HI; ++k) {
        double wk = cell_w(g, k, xp[2]);
        if (wk == 0.0) continue;
        for (long j = base[1] - BOX_LO; j <= base[1] + BOX_HI; ++j) {
            double wj = cell_w(g, j, xp[1]);
            if (wj == 0.0) continue;
            for (long i = base[0] - BOX_LO; i <= base[0] + BOX_HI; ++i) {
                double wi = cell_w(g, i, xp[0]);
                if (wi == 0.0) continue;
                rho[idx(g, i, j, k)] += charge / V * wi * wj * wk;
            }
        }
    }
}

void orc_rho(const orc_grid* g, int nsp, const orc_species* sp, double* rho)
{
    memset(rho, 0, ncell(g) * sizeof(double));
    for (int s = 0; s < nsp; ++s)
        for (int64_t p = 0; p < sp[s].n; ++p) {
            double xp[3] = {sp[s].x[p], sp[s].x[sp[s].n + p], sp[s].x[2 * sp[s].n + p]};
            orc_rho_add(g, xp, sp[s].q * sp[s].weight[p], rho);
        }
}

/* ---------------------------------------------------------------------------
 * Field solver on the staggered grid (Appendix, Eqs. updateB and escheme).
 * ------------------------------------------------------------------------- */
void orc_half_b(const orc_grid* g, double* fields)
{
    const size_t nc = ncell(g);
    const double *Ex = fields, *Ey = fields + nc, *Ez = fields + 2 * nc;
    double *Bx = fields + 3 * nc, *By = fields + 4 * nc, *Bz = fields + 5 * nc;
    const double cx = g->c * g->dt / g->dx, cy = g->c * g->dt / g->dy, cz = g->c * g->dt / g->dz;
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                size_t p = idx(g, i, j, k);
                /* B^x at (i+1/2, j, k): E^z at j+-1/2, E^y at k+-1/2 */
                Bx[p] = Bx[p] - 0.5 * cy * (Ez[p] - Ez[idx(g, i, j - 1, k)])
                        + 0.5 * cz * (Ey[p] - Ey[idx(g, i, j, k - 1)]);
                /* B^y at (i, j+1/2, k): E^x at k+-1/2, E^z at i+-1/2 */
                By[p] = By[p] - 0.5 * cz * (Ex[p] - Ex[idx(g, i, j, k - 1)])
                        + 0.5 * cx * (Ez[p] - Ez[idx(g, i - 1, j, k)]);
                /* B^z at (i, j, k+1/2): E^y at i+-1/2, E^x at j+-1/2 */
                Bz[p] = Bz[p] - 0.5 * cx * (Ey[p] - Ey[idx(g, i - 1, j, k)])
                        + 0.5 * cy * (Ex[p] - Ex[idx(g, i, j - 1, k)]);
            }
}

void orc_update_e(const orc_grid* g, double* fields)
{
    const size_t nc = ncell(g);
    double *Ex = fields, *Ey = fields + nc, *Ez = fields + 2 * nc;
    const double *Bx = fields + 3 * nc, *By = fields + 4 * nc, *Bz = fields + 5 * nc;
    const double *Jx = fields + 6 * nc, *Jy = fields + 7 * nc, *Jz = fields + 8 * nc;
    const double cx = g->c * g->dt / g->dx, cy = g->c * g->dt / g->dy, cz = g->c * g->dt / g->dz;
    const double fourpidt = 4.0 * PI * g->dt;
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                size_t p = idx(g, i, j, k);
                /* E^x at (i, j+1/2, k+1/2): B^z at j, j+1; B^y at k, k+1 */
                Ex[p] = Ex[p] - fourpidt * Jx[p] + cy * (Bz[idx(g, i, j + 1, k)] - Bz[p])
                        - cz * (By[idx(g, i, j, k + 1)] - By[p]);
                Ey[p] = Ey[p] - fourpidt * Jy[p] + cz * (Bx[idx(g, i, j, k + 1)] - Bx[p])
                        - cx * (Bz[idx(g, i + 1, j, k)] - Bz[p]);
                Ez[p] = Ez[p] - fourpidt * Jz[p] + cx * (By[idx(g, i + 1, j, k)] - By[p])
                        - cy * (Bx[idx(g, i, j + 1, k)] - Bx[p]);
            }
}

/* ---------------------------------------------------------------------------
 * Plane-wave source (not part of the paper's method: the laser of the slab
 * workload).  The incident wave lives on an auxiliary 1D line with the same
 * staggered operators as the grid restricted to x (E^y at faces, B^z at
 * nodes), so a plane wave uniform in y and z evolves identically on both and
 * the correction terms below inject it without leakage into x < plane.
 * Aux index a sits at grid index src_plane - 2 + a.  Parity unpinned: the
 * waveform's phase (a sine from t = 0) is this source's convention; the
 * workload fixes only its amplitude and wavelength, which the pins check.
 * ------------------------------------------------------------------------- */
static double src_wave(const orc_grid* g, double t)
{
    double ramp = 1.0;
    if (t < g->src_ramp) {
        double s = sin(0.5 * PI * t / g->src_ramp);
        ramp = s * s;
    }
    return g->src_amp * ramp * sin(g->src_omega * t);
}

static void aux_half_b(const orc_grid* g, double* aux)
{
    double *ey = aux, *bz = aux + ORC_AUX;
    const double hc = 0.5 * g->c * g->dt / g->dx;
    for (int a = 1; a < ORC_AUX; ++a) bz[a] = bz[a] - hc * (ey[a] - ey[a - 1]);
}

static void aux_update_e(const orc_grid* g, double* aux, double t_new)
{
    double *ey = aux, *bz = aux + ORC_AUX;
    const double cx = g->c * g->dt / g->dx;
    for (int a = 1; a < ORC_AUX - 1; ++a) ey[a] = ey[a] - cx * (bz[a + 1] - bz[a]);
    ey[0] = src_wave(g, t_new);
}

/* grid corrections at the plane: B^z at node i0 sees the incident E^y at
 * face i0 + 1/2 removed; E^y at face i0 + 1/2 sees the incident B^z at node
 * i0 added. */
static void src_fix_b(const orc_grid* g, double* fields, const double* aux)
{
    const size_t nc = ncell(g);
    double* Bz = fields + 5 * nc;
    const double v = 0.5 * (g->c * g->dt / g->dx) * aux[2];
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j) Bz[idx(g, g->src_plane, j, k)] += v;
}

static void src_fix_e(const orc_grid* g, double* fields, const double* aux)
{
    const size_t nc = ncell(g);
    double* Ey = fields + nc;
    const double v = (g->c * g->dt / g->dx) * aux[ORC_AUX + 2];
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j) Ey[idx(g, g->src_plane, j, k)] += v;
}

/* ---------------------------------------------------------------------------
 * Open x boundary (xbc = 1; not part of the paper's method, whose tests are
 * periodic boxes).  The walls are the node planes x = 0 and x = nx - 1, on
 * which B^y and B^z lie.  Their values follow Mur's first-order absorbing
 * condition (G. Mur, IEEE Trans. Electromagn. Compat. 23, 377 (1981)): the
 * one-way wave equation dB/dt = +-c dB/dx of a wave leaving the box, with
 * both derivatives taken at the midpoint between the wall and the plane one
 * cell inside and between B^{n-1/2} and B^{n+1/2}, solved for the new wall
 * value:
 *   B_wall^{n+1/2} = B_in^{n-1/2} + k (B_in^{n+1/2} - B_wall^{n-1/2}),
 *   k = (c dt - dx) / (c dt + dx).
 * Every other value is updated by the periodic operators above; the cell
 * layer between x = nx - 1 and the periodic image of x = 0 is outside the
 * box and its E^y, E^z and B^x are set to zero after each update, so that
 * nothing carries across it.
 * save: [side][wall B^y, wall B^z, inside B^y, inside B^z][ny nz], side 0 the
 * wall x = 0 (inside plane x = 1), side 1 the wall x = nx - 1 (inside plane
 * x = nx - 2).
 * ------------------------------------------------------------------------- */
static void wall_save(const orc_grid* g, const double* fields, double* save)
{
    const size_t nc = ncell(g), nyz = (size_t)g->ny * g->nz;
    const double *By = fields + 4 * nc, *Bz = fields + 5 * nc;
    for (int side = 0; side < 2; ++side) {
        const long iw = side == 0 ? 0 : g->nx - 1, in = side == 0 ? 1 : g->nx - 2;
        double* sv = save + 4 * nyz * side;
        for (long k = 0; k < g->nz; ++k)
            for (long j = 0; j < g->ny; ++j) {
                const size_t q = (size_t)k * g->ny + j;
                sv[q] = By[idx(g, iw, j, k)];
                sv[nyz + q] = Bz[idx(g, iw, j, k)];
                sv[2 * nyz + q] = By[idx(g, in, j, k)];
                sv[3 * nyz + q] = Bz[idx(g, in, j, k)];
            }
    }
}

static void wall_mur(const orc_grid* g, double* fields, const double* save)
{
    const size_t nc = ncell(g), nyz = (size_t)g->ny * g->nz;
    double *Bx = fields + 3 * nc, *By = fields + 4 * nc, *Bz = fields + 5 * nc;
    const double cdt = g->c * g->dt;
    const double kmur = (cdt - g->dx) / (cdt + g->dx);
    for (int side = 0; side < 2; ++side) {
        const long iw = side == 0 ? 0 : g->nx - 1, in = side == 0 ? 1 : g->nx - 2;
        const double* sv = save + 4 * nyz * side;
        for (long k = 0; k < g->nz; ++k)
            for (long j = 0; j < g->ny; ++j) {
                const size_t q = (size_t)k * g->ny + j;
                By[idx(g, iw, j, k)] = sv[2 * nyz + q] + kmur * (By[idx(g, in, j, k)] - sv[q]);
                Bz[idx(g, iw, j, k)] = sv[3 * nyz + q] + kmur * (Bz[idx(g, in, j, k)] - sv[nyz + q]);
            }
    }
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j) Bx[idx(g, g->nx - 1, j, k)] = 0.0;
}

static void outside_zero_e(const orc_grid* g, double* fields)
{
    const size_t nc = ncell(g);
    double *Ey = fields + nc, *Ez = fields + 2 * nc;
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j) {
            Ey[idx(g, g->nx - 1, j, k)] = 0.0;
            Ez[idx(g, g->nx - 1, j, k)] = 0.0;
        }
}

/* ---------------------------------------------------------------------------
 * One full time step in the Appendix order: B half step; for every particle,
 * in index order, form factors at x^n, gather, push, new position, current;
 * second B half step; E update.  J is cleared before the particle loop, so
 * after the step it holds J^{n+1/2}.  With an open x boundary the walls'
 * B^{n-1/2} is saved first and their B^{n+1/2} is replaced by Mur's value
 * before the E update, which reads it.
 * ------------------------------------------------------------------------- */
static void wrap_pos(double* x, long n)
{
    double N = (double)n;
    if (*x >= N) *x -= N;
    if (*x < 0.0) *x += N;
    if (*x >= N) *x -= N; /* a tiny negative value can round up to N */
}

void orc_particle_step(const orc_grid* g, const double* fields, const orc_species* s,
                       double* J)
{
    const long nn[3] = {g->nx, g->ny, g->nz};
    const double q_over_m = s->q / s->m;
    for (int64_t p = 0; p < s->n; ++p) {
        double x0[3], w[3], Ep[3], Bp[3], d[3], x1[3];
        for (int a = 0; a < 3; ++a) {
            x0[a] = s->x[a * s->n + p];
            w[a] = s->w[a * s->n + p];
        }
        orc_gather(g, fields, x0, Ep, Bp);
        orc_push(q_over_m, g->dt, g->c, Ep, Bp, w);
        orc_displacement(g, w, d);
        for (int a = 0; a < 3; ++a) x1[a] = x0[a] + d[a];
        if (s->deposit) orc_deposit(g, x0, x1, s->q * s->weight[p], J);
        for (int a = 0; a < 3; ++a) {
            wrap_pos(&x1[a], nn[a]);
            s->x[a * s->n + p] = x1[a];
            s->w[a * s->n + p] = w[a];
        }
        if (g->xbc == 1 && (x1[0] < ORC_ABSORB || x1[0] >= (double)(g->nx - 1 - ORC_ABSORB)))
            s->weight[p] = 0.0; /* absorbed: its current of this step is already on the grid */
    }
}

void orc_step_src(const orc_grid* g, double* fields, int nsp, const orc_species* sp, int nsteps,
                  double* aux, int64_t step0)
{
    const size_t nc = ncell(g);
    double* J = fields + 6 * nc;
    const int src = g->src_kind == 1 && aux != NULL;
    double* save = g->xbc == 1 ? (double*)malloc(8 * (size_t)g->ny * g->nz * sizeof(double)) : NULL;
    for (int it = 0; it < nsteps; ++it) {
        if (save) wall_save(g, fields, save);
        orc_half_b(g, fields);
        if (src) {
            src_fix_b(g, fields, aux);
            aux_half_b(g, aux);
        }
        memset(J, 0, 3 * nc * sizeof(double));
        for (int s = 0; s < nsp; ++s)
            if (sp[s].mobile) orc_particle_step(g, fields, &sp[s], J);
        orc_half_b(g, fields);
        if (src) {
            src_fix_b(g, fields, aux);
            aux_half_b(g, aux);
        }
        if (save) wall_mur(g, fields, save);
        orc_update_e(g, fields);
        if (src) {
            src_fix_e(g, fields, aux);
            aux_update_e(g, aux, (double)(step0 + it + 1) * g->dt);
        }
        if (save) outside_zero_e(g, fields);
    }
    free(save);
}

void orc_step(const orc_grid* g, double* fields, int nsp, const orc_species* sp, int nsteps)
{
    orc_step_src(g, fields, nsp, sp, nsteps, NULL, 0);
}

/* ---------------------------------------------------------------------------
 * Diagnostics.
 * ------------------------------------------------------------------------- */
/* R = div E - 4 pi rho at cell centres (the discrete Gauss law, Eq. chargelaw). */
void orc_gauss_residual(const orc_grid* g, const double* fields, const double* rho, double* R)
{
    const size_t nc = ncell(g);
    const double *Ex = fields, *Ey = fields + nc, *Ez = fields + 2 * nc;
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                size_t p = idx(g, i, j, k);
                double div = (Ex[idx(g, i + 1, j, k)] - Ex[p]) / g->dx
                             + (Ey[idx(g, i, j + 1, k)] - Ey[p]) / g->dy
                             + (Ez[idx(g, i, j, k + 1)] - Ez[p]) / g->dz;
                R[p] = div - 4.0 * PI * rho[p];
            }
}

/* div B at the grid nodes (i, j, k). */
void orc_div_b(const orc_grid* g, const double* fields, double* D)
{
    const size_t nc = ncell(g);
    const double *Bx = fields + 3 * nc, *By = fields + 4 * nc, *Bz = fields + 5 * nc;
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                size_t p = idx(g, i, j, k);
                D[p] = (Bx[p] - Bx[idx(g, i - 1, j, k)]) / g->dx
                       + (By[p] - By[idx(g, i, j - 1, k)]) / g->dy
                       + (Bz[p] - Bz[idx(g, i, j, k - 1)]) / g->dz;
            }
}

/* out[0] kinetic   sum m_p c^2 (gamma^{n-1/2} - 1)
 * out[1] half-step term sum (q_p dt / 2) u^{n-1/2} . E(x^n)   (Section 4.1)
 * out[2] electric  V/(8 pi) sum E^2
 * out[3] magnetic  V/(8 pi) sum (B^n)^2, B^n = B^{n-1/2} advanced a half step
 * External uniform B is excluded from out[3] but acts in the gather. */
void orc_energies(const orc_grid* g, const double* fields, int nsp, const orc_species* sp,
                  double out[4])
{
    const size_t nc = ncell(g);
    const double V = g->dx * g->dy * g->dz;
    double* tmp = (double*)malloc(9 * nc * sizeof(double));
    memcpy(tmp, fields, 9 * nc * sizeof(double));
    orc_half_b(g, tmp);
    double kin = 0.0, half = 0.0, fe = 0.0, fb = 0.0;
    for (int s = 0; s < nsp; ++s) {
        if (!sp[s].mobile) continue;
        for (int64_t p = 0; p < sp[s].n; ++p) {
            double w[3], xp[3], Ep[3], Bp[3];
            for (int a = 0; a < 3; ++a) {
                w[a] = sp[s].w[a * sp[s].n + p];
                xp[a] = sp[s].x[a * sp[s].n + p];
            }
            double w2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
            double gam = sqrt(1.0 + w2 / (g->c * g->c));
            double mp = sp[s].m * sp[s].weight[p], qp = sp[s].q * sp[s].weight[p];
            kin += mp * w2 / (gam + 1.0); /* = m c^2 (gamma - 1) without cancellation */
            orc_gather(g, tmp, xp, Ep, Bp);
            half += 0.5 * qp * g->dt * (Ep[0] * w[0] + Ep[1] * w[1] + Ep[2] * w[2]) / gam;
        }
    }
    for (size_t p = 0; p < 3 * nc; ++p) fe += tmp[p] * tmp[p];
    for (size_t p = 3 * nc; p < 6 * nc; ++p) fb += tmp[p] * tmp[p];
    free(tmp);
    out[0] = kin;
    out[1] = half;
    out[2] = V / (8.0 * PI) * fe;
    out[3] = V / (8.0 * PI) * fb;
}
