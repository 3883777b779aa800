/*
 * pic_oracle.h -- declarations of the double-precision CPU reference of the
 * charge-conserving PIC step (arXiv:1101.0809).  TEST INFRASTRUCTURE: only the
 * test suite, the smoke check and the benchmark's CPU baseline use it.  See
 * pic_oracle.c for the conventions (cell units, storage order, staggering).
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H

#include <stdint.h>

typedef struct orc_grid {
    int64_t nx, ny, nz;  /* cells per axis, periodic */
    double dx, dy, dz;   /* cell sizes */
    double dt;           /* time step */
    double c;            /* speed of light */
    double bext[3];      /* uniform external B added at the gather */
    /* plane-wave source (kind 1): E^y wave travelling along +x, injected at
     * the total-field / scattered-field plane between node src_plane and face
     * src_plane + 1/2; incident values from an auxiliary 1D line of ORC_AUX
     * cells whose first E^y point (x = src_plane - 2 + 1/2) is driven as
     * E0 ramp(t) sin(omega t), ramp = sin^2(pi t / (2 src_ramp)) until src_ramp */
    int64_t src_kind, src_plane;
    double src_amp, src_omega, src_ramp;
    /* alternating order l_a = order + 1/2 (Section 4.5): 1 (also when 0) or 2 */
    int64_t order;
    /* field interpolation: 0 alternating-order (Eqs. alphax, betax); 1 the
     * "conventional" uniform order of Eq. wrong1 (with order 1 only): along a
     * component's node axes the weight is the mean of the two adjacent cell
     * factors, Delta F elsewhere */
    int64_t interp;
    /* x boundary: 0 periodic; 1 open -- walls at the node planes x = 0 and
     * x = nx - 1 with Mur's first-order absorbing condition on the tangential
     * B^y, B^z, the cell layer x in [nx - 1, nx) outside the box (its E^y,
     * E^z, B^x held at zero), and particles absorbed (weight set to zero) when
     * a step ends within ORC_ABSORB cells of a wall */
    int64_t xbc;
} orc_grid;

#define ORC_ABSORB 2  /* width in cells of the particle-absorbing layer at each wall */

#define ORC_AUX 8192  /* auxiliary line length: E^y[ORC_AUX] then B^z[ORC_AUX] */

typedef struct orc_species {
    int64_t n;             /* particle count */
    double q;              /* charge per unit weight */
    double m;              /* mass per unit weight */
    int32_t mobile;        /* 0: immobile (charge only) */
    int32_t deposit;       /* 0: test particles, no current */
    double* x;             /* [3][n] positions in cell units, in [0, N) */
    double* w;             /* [3][n] momentum over mass, w^{n-1/2} */
    double* weight;        /* [n] macro-particle weight (zeroed when absorbed) */
} orc_species;

double orc_shape(int l, double r);
double orc_cumulative1(double s);
double orc_cumulative2(double s);
void orc_gather(const orc_grid* g, const double* fields, const double xp[3], double Ep[3],
                double Bp[3]);
void orc_push(double q_over_m, double dt, double c, const double Ep[3], const double Bp[3],
              double w[3]);
void orc_displacement(const orc_grid* g, const double w[3], double dxp[3]);
void orc_deposit(const orc_grid* g, const double x0[3], const double x1[3], double charge,
                 double* J);
void orc_deposit_quarter(const orc_grid* g, const double x0[3], const double x1[3],
                         double charge, double* J);
void orc_rho_add(const orc_grid* g, const double xp[3], double charge, double* rho);
void orc_rho(const orc_grid* g, int nsp, const orc_species* sp, double* rho);
void orc_half_b(const orc_grid* g, double* fields);
void orc_update_e(const orc_grid* g, double* fields);
void orc_particle_step(const orc_grid* g, const double* fields, const orc_species* s,
                       double* J);
void orc_step(const orc_grid* g, double* fields, int nsp, const orc_species* sp, int nsteps);
/* same, with the source's auxiliary line state aux[2 * ORC_AUX] and the step
 * index of the first step (the source time is counted from step 0) */
void orc_step_src(const orc_grid* g, double* fields, int nsp, const orc_species* sp, int nsteps,
                  double* aux, int64_t step0);
void orc_gauss_residual(const orc_grid* g, const double* fields, const double* rho, double* R);
void orc_div_b(const orc_grid* g, const double* fields, double* D);
void orc_energies(const orc_grid* g, const double* fields, int nsp, const orc_species* sp,
                  double out[4]);

#endif
