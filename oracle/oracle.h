/*
 * Plain FP64 CPU oracle of the electromagnetic PIC timestep (λPIC, arXiv 2607.13507).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP product path; only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * What it computes follows the paper:
 *   - Maxwell's equations in the Yee discretisation, each field advance split into two
 *     half steps (Sec. 3.2, Eqs. 1-4), in normalised units c = eps0 = 1;
 *   - the per-step order of Algorithm 1 (Sec. 3.3): E half, B half, per species
 *     {position half push, interpolation, Boris momentum push, position half push,
 *     Esirkepov deposit}, then B half, E half; the deposited path is the trajectory over
 *     one dt centred on the end of the step (Sec. 3.1 and the time levels of Eq. 3);
 *   - the relativistic Boris push with u = gamma v (Sec. 3.1);
 *   - staggering-aware interpolation with a B-spline shape of order 1 (CIC) or 2
 *     (quadratic) (Sec. 3.1);
 *   - Esirkepov's charge-conserving current deposition (Sec. 3.1, Esirkepov 2001).
 * Positions are absolute FP64 coordinates.  Every boundary is periodic.
 *
 * Grid layout: one array per component, ncell = nx*ny*nz entries (nz = 1 in 2D), index
 * (k*ny + j)*nx + i, no guard cells (periodicity by index wrap).  Staggering of the array
 * entry [i,j,k] (in units of the cell size, 2D drops z):
 *   Ex (i+1/2, j, k)   Ey (i, j+1/2, k)   Ez (i, j, k+1/2)   (Ez at (i,j) in 2D)
 *   Bx (i, j+1/2, k+1/2)  By (i+1/2, j, k+1/2)  Bz (i+1/2, j+1/2, k)
 *   Jx, Jy, Jz as Ex, Ey, Ez;  rho at (i, j, k).
 */
#ifndef LPIC_ORACLE_H
#define LPIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Convolutional PML at the open x ends (the absorbing layer that Sec. 3.2 attaches to the
 * boundaries of the box, after Berenger; here in the recursive-convolution form of Roden
 * and Gedney, Microw. Opt. Technol. Lett. 27, 334 (2000), with the complex frequency
 * shift a).  The first and the last `cells` (L) node columns of x form the two layers; x
 * stays circular, so the layers meet back to back across the wrap, and the Mur condition
 * below is not applied.  Inside a layer every x derivative of the curls (dBz/dx in the Ey
 * update, dBy/dx in Ez, dEz/dx in By, dEy/dx in Bz) is replaced by D/kappa + psi, where
 * psi, one value per component and location, first takes
 *     psi <- b psi + c D,   b = exp(-(sigma/kappa + a) tau),
 *                           c = sigma (b - 1) / (kappa (sigma + kappa a)),
 * tau the time step of that update (eps0 = mu0 = c = 1, so the magnetic profile equals the
 * electric one).  Profiles, with s = depth / L and depth the distance in cells of the
 * component's location from the layer's inner face (node column L on the left, nx - L on
 * the right; E-side locations are whole columns, B-side ones half columns):
 *     sigma = sigma_max s^m,  kappa = 1 + (kappa_max - 1) s^m,  a = a_max (1 - s)^ma
 * (x^0 = 1: orders 0 make a uniform layer). */
typedef struct {
  int32_t cells;         /* L >= 1, 2 L < nx */
  int32_t order;         /* grading exponent m >= 0 of sigma and kappa */
  int32_t a_order;       /* grading exponent ma >= 0 of a */
  int32_t reserved0;
  double sigma_max, kappa_max, a_max;
  double *psi;           /* 4 x (2L) x nz x ny auxiliary values, zero at the start; index
                            ((comp * 2L + slot) * nz + k) * ny + j, comp 0..3 = Ey, Ez, By,
                            Bz, slot = column i (left layer) or i - nx + 2L (right layer) */
} orc_pml;

typedef struct {
  int32_t ndim;          /* 2 or 3 */
  int32_t nx, ny, nz;    /* cells; nz = 1 when ndim == 2 */
  double dx, dy, dz, dt;
  double rho_bg;         /* fixed neutralising background charge density (added in Gauss) */
  int32_t open_x;        /* 0: periodic in x; 1: open x ends (see below) */
  const orc_pml *pml;    /* NULL, or (with open_x) the layers above instead of Mur */
} orc_grid;

/* Open x ends (the absorbing boundaries of Sec. 3.2 and the particle loss at boundaries of
 * Sec. 2.1), without a PML (pml == NULL) the first-order Mur condition:
 *   - fields: after each E update the tangential E at the first node column (i = 0) and
 *     after each B update the tangential B at the last column (i = nx-1) follow the
 *     outgoing-wave condition u_new(edge) = u_old(inner) + k (u_new(inner) - u_old(edge)),
 *     k = (c h - dx) / (c h + dx), h the time step of that update;
 *   - particles: alive only with x in [ORC_OPEN_MARGIN dx, (nx - ORC_OPEN_MARGIN) dx); a
 *     particle whose new position leaves that range is removed (x = -1) after depositing
 *     its current for the step, so no interpolation or deposit stencil ever wraps in x. */
#define ORC_OPEN_MARGIN 3

/* Laser antenna (the GaussianLaser callback of Sec. 2.2, injection from the left boundary
 * as in Sec. 4.2): a current sheet on the node column i = ia, J_pol = -2 E_inc / dx, which
 * radiates E_inc to +x (and the same to -x, absorbed by the open boundary), with
 *   E_inc(t, y, z) = a0 omega sin^2(pi (t - t0) / tau) exp(-((y-yc)^2 + (z-zc)^2) / w^2)
 *                    sin(omega (t - t0))   for 0 <= t - t0 <= tau, else 0
 * (2D drops z).  pol = 1: E along y (J_y at (ia, j+1/2)); pol = 2: E along z (J_z at
 * (ia, j) in 2D, (ia, j, k+1/2) in 3D).  The current of step n is taken at t = (n+1) dt,
 * the time level at which the E updates around the step end use J (Algorithm 1). */
typedef struct {
  int32_t pol, ia;
  double a0, omega, waist, yc, zc, t0, tau;
} orc_laser;

typedef struct {
  double *ex, *ey, *ez, *bx, *by, *bz, *jx, *jy, *jz;
  double *rho0, *rho1;   /* optional (NULL): charge at the start / end of the step */
} orc_fields;

typedef struct {
  int64_t n;             /* number of particles */
  double q, m;           /* charge and mass in units of e and m_e */
  int32_t order;         /* 1 = CIC, 2 = quadratic */
  double *x, *y, *z;     /* absolute positions; z unused (may be NULL) in 2D; x < 0 = dead */
  double *ux, *uy, *uz;  /* u = gamma v / c */
  double *w;             /* weight = density carried by the macro-particle */
} orc_species;

/* One-dimensional B-spline shape of the given order evaluated at xi (cell units). */
double orc_shape(int32_t order, double xi);

/* Relativistic Boris push of one momentum u[3] by dt in fields E, B (Sec. 3.1). */
void orc_boris(double u[3], const double E[3], const double B[3], double q, double m, double dt);

/* Interpolate the six field components at absolute position pos[] with shape `order`. */
void orc_gather(const orc_grid *g, const orc_fields *f, int32_t order, const double pos[3],
                double E[3], double B[3]);

/* Half (or any fraction) field updates, Eqs. 3-4 in normalised units. */
void orc_yee_e(const orc_grid *g, orc_fields *f, double frac);   /* E += frac*dt*(curl B - J) */
void orc_yee_b(const orc_grid *g, orc_fields *f, double frac);   /* B -= frac*dt*curl E */

/* Esirkepov deposit of one particle moving from p0 to p1 (absolute, unwrapped) during dt,
 * adding J into f.  vz_bar is the z velocity along the path, used for Jz in 2D (ignored in
 * 3D). */
void orc_deposit_particle(const orc_grid *g, orc_fields *f, int32_t order, double q, double w,
                          const double p0[3], const double p1[3], double vz_bar);

/* Add q*w*S(pos - node) into rho at the integer nodes. */
void orc_deposit_rho(const orc_grid *g, double *rho, int32_t order, double q, double w,
                     const double pos[3]);

/* Particle part of Algorithm 1 for one species: half position push, gather, Boris, half
 * position push; Esirkepov deposit into J (J is NOT zeroed here) of the path from the
 * half-step position x^{n+1/2} to x^{n+1/2} + dt v^{n+1}; optional rho0/rho1 deposits at
 * the two path ends; periodic wrap.  If xs/ys/zs are non-NULL they receive the path start
 * x^{n+1/2} of every particle (unwrapped). */
void orc_push_deposit(const orc_grid *g, orc_fields *f, orc_species *s, int32_t deposit,
                      double *xs, double *ys, double *zs);

/* Gather + push only (no deposit); positions are wrapped. */
void orc_gather_push(const orc_grid *g, const orc_fields *f, orc_species *s);

/* Adds the antenna current of `laser` at time t into J. */
void orc_laser_source(const orc_grid *g, orc_fields *f, const orc_laser *laser, double t);

/* One full timestep of Algorithm 1 over all species; with laser != NULL the antenna current
 * at t_next = (n+1) dt is added after the particles' deposit. */
void orc_step(const orc_grid *g, orc_fields *f, orc_species *sp, int32_t nspecies,
              const orc_laser *laser, double t_next);

/* orc_step with the particle loop on nthreads threads (private current arrays added in
 * thread order afterwards; timing only).  Returns the threads used, or -1 if the private
 * arrays cannot be allocated.  The current and charge arrays are overwritten. */
int32_t orc_step_threads(const orc_grid *g, orc_fields *f, orc_species *sp, int32_t nspecies,
                         const orc_laser *laser, double t_next, int32_t nthreads);

/* Diagnostics (all FP64).  dV is the cell volume (dx*dy or dx*dy*dz). */
double orc_field_energy(const orc_grid *g, const orc_fields *f);
double orc_kinetic_energy(const orc_grid *g, const orc_species *s);
/* max |rho1 - rho0 + dt div J| / max |rho1| */
double orc_continuity(const orc_grid *g, const orc_fields *f);
/* G = div E - (rho0 + rho1)/2 - rho_bg at every node, written into out[ncell]. */
void orc_gauss(const orc_grid *g, const orc_fields *f, double *out);
/* div B at the cell centres (i+1/2, j+1/2, k+1/2), written into out[ncell]. */
void orc_div_b(const orc_grid *g, const orc_fields *f, double *out);

#ifdef __cplusplus
}
#endif
#endif
