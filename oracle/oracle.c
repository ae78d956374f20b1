/*
 * Plain FP64 CPU oracle of the λPIC timestep (arXiv 2607.13507).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the benchmark's
 * CPU-baseline leg, never by the product path.  Deliberately simple: every loop visits a
 * generous window of nodes and evaluates the shape function from its piecewise definition,
 * so that each formula can be checked against the paper by eye.  Single threaded; only
 * orc_step_threads, a timing driver, runs the same particle loop on several threads.
 *
 * Each function names the passage of the paper it follows (section, equation, algorithm).
 */
#define _DEFAULT_SOURCE
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int64_t wrap(int64_t i, int64_t n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}

static int64_t nidx(const orc_grid *g, int64_t i, int64_t j, int64_t k) {
  int64_t kk = (g->ndim == 3) ? wrap(k, g->nz) : 0;
  return (kk * g->ny + wrap(j, g->ny)) * g->nx + wrap(i, g->nx);
}

static int64_t ncell(const orc_grid *g) {
  return (int64_t)g->nx * g->ny * (g->ndim == 3 ? g->nz : 1);
}

/* Sec. 3.1: B-spline shape functions.  Order 1 is the linear (CIC, "bilinear" in 2D)
 * weight, order 2 the quadratic spline named for Esirkepov's scheme. */
double orc_shape(int32_t order, double xi) {
  double a = fabs(xi);
  if (order == 1) return a < 1.0 ? 1.0 - a : 0.0;
  if (a <= 0.5) return 0.75 - a * a;
  if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
  return 0.0;
}

/* Sec. 3.1: relativistic Boris push (half electric kick, magnetic rotation, half electric
 * kick) on the momentum u = gamma v / c, normalised units (c = 1, q in e, m in m_e). */
void orc_boris(double u[3], const double E[3], const double B[3], double q, double m,
               double dt) {
  double a = q * dt / (2.0 * m);
  double um[3], t[3], s[3], up[3], upl[3];
  for (int d = 0; d < 3; ++d) um[d] = u[d] + a * E[d];
  double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  for (int d = 0; d < 3; ++d) t[d] = a * B[d] / gm;
  double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  for (int d = 0; d < 3; ++d) s[d] = 2.0 * t[d] / (1.0 + t2);
  up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
  up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
  up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
  upl[0] = um[0] + (up[1] * s[2] - up[2] * s[1]);
  upl[1] = um[1] + (up[2] * s[0] - up[0] * s[2]);
  upl[2] = um[2] + (up[0] * s[1] - up[1] * s[0]);
  for (int d = 0; d < 3; ++d) u[d] = upl[d] + a * E[d];
}

/* Staggering of each component in units of the cell size (see the header). */
static const double STAG2[6][3] = {
    {0.5, 0.0, 0.0}, {0.0, 0.5, 0.0}, {0.0, 0.0, 0.0},   /* Ex Ey Ez (2D) */
    {0.0, 0.5, 0.0}, {0.5, 0.0, 0.0}, {0.5, 0.5, 0.0}};  /* Bx By Bz (2D) */
static const double STAG3[6][3] = {
    {0.5, 0.0, 0.0}, {0.0, 0.5, 0.0}, {0.0, 0.0, 0.5},
    {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}, {0.5, 0.5, 0.0}};

/* Sec. 3.1: staggering-aware interpolation; each component is interpolated from its own
 * node locations with the particle's shape function (sum over a 5-node window per axis,
 * which contains the whole support of both shapes). */
void orc_gather(const orc_grid *g, const orc_fields *f, int32_t order, const double pos[3],
                double E[3], double B[3]) {
  const double *arr[6] = {f->ex, f->ey, f->ez, f->bx, f->by, f->bz};
  double out[6];
  double h[3] = {g->dx, g->dy, g->dz};
  int nd = g->ndim;
  for (int c = 0; c < 6; ++c) {
    const double *st = (nd == 3) ? STAG3[c] : STAG2[c];
    double X[3], w[3][5];
    int64_t base[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
      if (d < nd) {
        X[d] = pos[d] / h[d] - st[d];
        base[d] = (int64_t)floor(X[d]) - 2;
        for (int a = 0; a < 5; ++a) w[d][a] = orc_shape(order, (double)(base[d] + a) - X[d]);
      } else {
        for (int a = 0; a < 5; ++a) w[d][a] = (a == 0) ? 1.0 : 0.0;
      }
    }
    int nk = (nd == 3) ? 5 : 1;
    double sum = 0.0;
    for (int kc = 0; kc < nk; ++kc)
      for (int b = 0; b < 5; ++b)
        for (int a = 0; a < 5; ++a) {
          double wt = w[0][a] * w[1][b] * w[2][kc];
          if (wt == 0.0) continue;
          sum += wt * arr[c][nidx(g, base[0] + a, base[1] + b, base[2] + kc)];
        }
    out[c] = sum;
  }
  E[0] = out[0]; E[1] = out[1]; E[2] = out[2];
  B[0] = out[3]; B[1] = out[4]; B[2] = out[5];
}

/* First-order Mur outgoing-wave condition on one column of a field component: the edge
 * column `e` takes u_old(inner) + k (u_new(inner) - u_old(edge)) (Sec. 3.2 absorbing
 * boundary; see the header).  old_edge and old_inner hold the values before the update. */
static void mur_column(const orc_grid *g, double *u, const double *old_edge,
                       const double *old_inner, int64_t e, int64_t inner, double h) {
  double k = (h - g->dx) / (h + g->dx);
  int nz = (g->ndim == 3) ? g->nz : 1;
  for (int64_t kk = 0; kk < nz; ++kk)
    for (int64_t j = 0; j < g->ny; ++j) {
      int64_t t = kk * g->ny + j;
      u[nidx(g, e, j, kk)] = old_inner[t] + k * (u[nidx(g, inner, j, kk)] - old_edge[t]);
    }
}

/* Copy of column i of u into out[ny*nz]. */
static void save_column(const orc_grid *g, const double *u, int64_t i, double *out) {
  int nz = (g->ndim == 3) ? g->nz : 1;
  for (int64_t kk = 0; kk < nz; ++kk)
    for (int64_t j = 0; j < g->ny; ++j) out[kk * g->ny + j] = u[nidx(g, i, j, kk)];
}

/* The convolutional PML of the header: is node column i in a layer, and which slot. */
static int pml_slot(const orc_grid *g, int64_t i) {
  if (!g->open_x || !g->pml) return -1;
  int64_t L = g->pml->cells;
  if (i < L) return (int)i;
  if (i >= g->nx - L) return (int)(i - g->nx + 2 * L);
  return -1;
}

/* Depth (cells) of slot l from its layer's inner face, for a location on a whole column
 * (E side, half = 0) or half a column further in +x (B side, half = 1). */
static double pml_depth(const orc_grid *g, int l, int half) {
  double L = g->pml->cells;
  double x = (l < g->pml->cells) ? (double)l : (double)(l - g->pml->cells) + (g->nx - L);
  if (half) x += 0.5;
  return (l < g->pml->cells) ? L - x : x - (g->nx - L);
}

/* The profiles at `depth` and the recursion coefficients for an update of step tau. */
static void pml_coef(const orc_pml *p, double depth, double tau, double *b, double *c,
                     double *kappa) {
  double s = depth / p->cells;
  double sm = 1.0;
  for (int q = 0; q < p->order; ++q) sm *= s;
  double sigma = p->sigma_max * sm;
  *kappa = 1.0 + (p->kappa_max - 1.0) * sm;
  double sa = 1.0;
  for (int q = 0; q < p->a_order; ++q) sa *= 1.0 - s;
  double a = p->a_max * sa;
  *b = exp(-(sigma / *kappa + a) * tau);
  *c = (sigma == 0.0) ? 0.0 : sigma * (*b - 1.0) / (*kappa * (sigma + *kappa * a));
}

/* Replaces the x derivative D of component comp at (slot, j, k) by D/kappa + psi after the
 * recursion step of psi (header). */
static double pml_apply(const orc_grid *g, int comp, int l, int64_t j, int64_t k,
                        double depth, double tau, double D) {
  const orc_pml *p = g->pml;
  int64_t nz = (g->ndim == 3) ? g->nz : 1;
  double *psi = p->psi + ((comp * 2 * (int64_t)p->cells + l) * nz + k) * g->ny + j;
  double b, c, kappa;
  pml_coef(p, depth, tau, &b, &c, &kappa);
  *psi = b * *psi + c * D;
  return D / kappa + *psi;
}

static void yee_e_all(const orc_grid *g, orc_fields *f, double frac);

/* Sec. 3.2, Eq. 3 in normalised units: E += frac*dt*(curl B - J) on the Yee stagger; with
 * open x ends the tangential E of column 0 then follows the Mur condition, or the x
 * derivatives inside the PML layers take their convolutional form (header). */
void orc_yee_e(const orc_grid *g, orc_fields *f, double frac) {
  if (!g->open_x || g->pml) {
    yee_e_all(g, f, frac);
    return;
  }
  int64_t m = (int64_t)g->ny * ((g->ndim == 3) ? g->nz : 1);
  double *buf = (double *)malloc(sizeof(double) * 4 * m);
  save_column(g, f->ey, 0, buf);
  save_column(g, f->ey, 1, buf + m);
  save_column(g, f->ez, 0, buf + 2 * m);
  save_column(g, f->ez, 1, buf + 3 * m);
  yee_e_all(g, f, frac);
  mur_column(g, f->ey, buf, buf + m, 0, 1, frac * g->dt);
  mur_column(g, f->ez, buf + 2 * m, buf + 3 * m, 0, 1, frac * g->dt);
  free(buf);
}

static void yee_e_all(const orc_grid *g, orc_fields *f, double frac) {
  double h = frac * g->dt;
  int three = (g->ndim == 3);
  int nz = three ? g->nz : 1;
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < g->ny; ++j)
      for (int64_t i = 0; i < g->nx; ++i) {
        int64_t c = nidx(g, i, j, k);
        double dBz_dy = (f->bz[c] - f->bz[nidx(g, i, j - 1, k)]) / g->dy;
        double dBz_dx = (f->bz[c] - f->bz[nidx(g, i - 1, j, k)]) / g->dx;
        double dBy_dx = (f->by[c] - f->by[nidx(g, i - 1, j, k)]) / g->dx;
        double dBx_dy = (f->bx[c] - f->bx[nidx(g, i, j - 1, k)]) / g->dy;
        double dBy_dz = three ? (f->by[c] - f->by[nidx(g, i, j, k - 1)]) / g->dz : 0.0;
        double dBx_dz = three ? (f->bx[c] - f->bx[nidx(g, i, j, k - 1)]) / g->dz : 0.0;
        int l = pml_slot(g, i);
        if (l >= 0) {
          double depth = pml_depth(g, l, 0);
          dBz_dx = pml_apply(g, 0, l, j, k, depth, h, dBz_dx);
          dBy_dx = pml_apply(g, 1, l, j, k, depth, h, dBy_dx);
        }
        f->ex[c] += h * ((dBz_dy - dBy_dz) - f->jx[c]);
        f->ey[c] += h * ((dBx_dz - dBz_dx) - f->jy[c]);
        f->ez[c] += h * ((dBy_dx - dBx_dy) - f->jz[c]);
      }
}

static void yee_b_all(const orc_grid *g, orc_fields *f, double frac);

/* Sec. 3.2, Eq. 4: B -= frac*dt*curl E on the Yee stagger; with open x ends the tangential
 * B of the last column then follows the Mur condition, or the x derivatives inside the
 * PML layers take their convolutional form (header). */
void orc_yee_b(const orc_grid *g, orc_fields *f, double frac) {
  if (!g->open_x || g->pml) {
    yee_b_all(g, f, frac);
    return;
  }
  int64_t m = (int64_t)g->ny * ((g->ndim == 3) ? g->nz : 1);
  int64_t e = g->nx - 1;
  double *buf = (double *)malloc(sizeof(double) * 4 * m);
  save_column(g, f->by, e, buf);
  save_column(g, f->by, e - 1, buf + m);
  save_column(g, f->bz, e, buf + 2 * m);
  save_column(g, f->bz, e - 1, buf + 3 * m);
  yee_b_all(g, f, frac);
  mur_column(g, f->by, buf, buf + m, e, e - 1, frac * g->dt);
  mur_column(g, f->bz, buf + 2 * m, buf + 3 * m, e, e - 1, frac * g->dt);
  free(buf);
}

static void yee_b_all(const orc_grid *g, orc_fields *f, double frac) {
  double h = frac * g->dt;
  int three = (g->ndim == 3);
  int nz = three ? g->nz : 1;
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < g->ny; ++j)
      for (int64_t i = 0; i < g->nx; ++i) {
        int64_t c = nidx(g, i, j, k);
        double dEz_dy = (f->ez[nidx(g, i, j + 1, k)] - f->ez[c]) / g->dy;
        double dEz_dx = (f->ez[nidx(g, i + 1, j, k)] - f->ez[c]) / g->dx;
        double dEy_dx = (f->ey[nidx(g, i + 1, j, k)] - f->ey[c]) / g->dx;
        double dEx_dy = (f->ex[nidx(g, i, j + 1, k)] - f->ex[c]) / g->dy;
        double dEy_dz = three ? (f->ey[nidx(g, i, j, k + 1)] - f->ey[c]) / g->dz : 0.0;
        double dEx_dz = three ? (f->ex[nidx(g, i, j, k + 1)] - f->ex[c]) / g->dz : 0.0;
        int l = pml_slot(g, i);
        if (l >= 0) {
          double depth = pml_depth(g, l, 1);
          dEz_dx = pml_apply(g, 2, l, j, k, depth, h, dEz_dx);
          dEy_dx = pml_apply(g, 3, l, j, k, depth, h, dEy_dx);
        }
        f->bx[c] -= h * (dEz_dy - dEy_dz);
        f->by[c] -= h * (dEx_dz - dEz_dx);
        f->bz[c] -= h * (dEy_dx - dEx_dy);
      }
}

/* Sec. 3.1 (Esirkepov 2001): charge-conserving deposition.  Shape factors S0 (start) and
 * S1 (end) are evaluated on a common window of integer nodes; with dS = S1 - S0 the
 * weights are
 *   2D: Wx = dSx (S0y + dSy/2),  Wy = dSy (S0x + dSx/2),
 *       Wz = S0x S0y + dSx S0y/2 + S0x dSy/2 + dSx dSy/3;
 *   3D: Wx = dSx (S0y S0z + dSy S0z/2 + S0y dSz/2 + dSy dSz/3) and cyclically.
 * The current along an axis is the running sum of the weights along that axis times
 * -q w h/dt (h the cell size along the axis); 2D Jz is q w vz_bar Wz. */
void orc_deposit_particle(const orc_grid *g, orc_fields *f, int32_t order, double q, double w,
                          const double p0[3], const double p1[3], double vz_bar) {
  enum { NW = 16 };
  double h[3] = {g->dx, g->dy, g->dz};
  int nd = g->ndim;
  int64_t base[3] = {0, 0, 0};
  int nw[3] = {1, 1, 1};
  double S0[3][NW], dS[3][NW];
  for (int d = 0; d < nd; ++d) {
    double X0 = p0[d] / h[d], X1 = p1[d] / h[d];
    double lo = X0 < X1 ? X0 : X1, hi = X0 < X1 ? X1 : X0;
    base[d] = (int64_t)floor(lo) - 2;
    nw[d] = (int)((int64_t)floor(hi) + 2 - base[d] + 1);
    if (nw[d] > NW) abort(); /* the CFL limit keeps a displacement far below this */
    for (int a = 0; a < nw[d]; ++a) {
      double node = (double)(base[d] + a);
      double s0 = orc_shape(order, node - X0), s1 = orc_shape(order, node - X1);
      S0[d][a] = s0;
      dS[d][a] = s1 - s0;
    }
  }
  if (nd == 2) {
    double cx = -q * w * g->dx / g->dt, cy = -q * w * g->dy / g->dt, cz = q * w * vz_bar;
    for (int b = 0; b < nw[1]; ++b) {
      double acc = 0.0;
      for (int a = 0; a < nw[0]; ++a) {
        acc += dS[0][a] * (S0[1][b] + 0.5 * dS[1][b]);
        f->jx[nidx(g, base[0] + a, base[1] + b, 0)] += cx * acc;
      }
    }
    for (int a = 0; a < nw[0]; ++a) {
      double acc = 0.0;
      for (int b = 0; b < nw[1]; ++b) {
        acc += dS[1][b] * (S0[0][a] + 0.5 * dS[0][a]);
        f->jy[nidx(g, base[0] + a, base[1] + b, 0)] += cy * acc;
      }
    }
    for (int b = 0; b < nw[1]; ++b)
      for (int a = 0; a < nw[0]; ++a) {
        double wz = S0[0][a] * S0[1][b] + 0.5 * dS[0][a] * S0[1][b] +
                    0.5 * S0[0][a] * dS[1][b] + dS[0][a] * dS[1][b] / 3.0;
        f->jz[nidx(g, base[0] + a, base[1] + b, 0)] += cz * wz;
      }
    return;
  }
  double cx = -q * w * g->dx / g->dt, cy = -q * w * g->dy / g->dt, cz = -q * w * g->dz / g->dt;
  for (int c = 0; c < nw[2]; ++c)
    for (int b = 0; b < nw[1]; ++b) {
      double acc = 0.0;
      for (int a = 0; a < nw[0]; ++a) {
        acc += dS[0][a] * (S0[1][b] * S0[2][c] + 0.5 * dS[1][b] * S0[2][c] +
                           0.5 * S0[1][b] * dS[2][c] + dS[1][b] * dS[2][c] / 3.0);
        f->jx[nidx(g, base[0] + a, base[1] + b, base[2] + c)] += cx * acc;
      }
    }
  for (int c = 0; c < nw[2]; ++c)
    for (int a = 0; a < nw[0]; ++a) {
      double acc = 0.0;
      for (int b = 0; b < nw[1]; ++b) {
        acc += dS[1][b] * (S0[0][a] * S0[2][c] + 0.5 * dS[0][a] * S0[2][c] +
                           0.5 * S0[0][a] * dS[2][c] + dS[0][a] * dS[2][c] / 3.0);
        f->jy[nidx(g, base[0] + a, base[1] + b, base[2] + c)] += cy * acc;
      }
    }
  for (int b = 0; b < nw[1]; ++b)
    for (int a = 0; a < nw[0]; ++a) {
      double acc = 0.0;
      for (int c = 0; c < nw[2]; ++c) {
        acc += dS[2][c] * (S0[0][a] * S0[1][b] + 0.5 * dS[0][a] * S0[1][b] +
                           0.5 * S0[0][a] * dS[1][b] + dS[0][a] * dS[1][b] / 3.0);
        f->jz[nidx(g, base[0] + a, base[1] + b, base[2] + c)] += cz * acc;
      }
    }
}

/* Charge density at the integer nodes: rho += q w S(x - node) (Sec. 3.1). */
void orc_deposit_rho(const orc_grid *g, double *rho, int32_t order, double q, double w,
                     const double pos[3]) {
  double h[3] = {g->dx, g->dy, g->dz};
  int nd = g->ndim;
  int64_t base[3] = {0, 0, 0};
  double S[3][5];
  for (int d = 0; d < 3; ++d) {
    if (d < nd) {
      double X = pos[d] / h[d];
      base[d] = (int64_t)floor(X) - 2;
      for (int a = 0; a < 5; ++a) S[d][a] = orc_shape(order, (double)(base[d] + a) - X);
    } else {
      for (int a = 0; a < 5; ++a) S[d][a] = (a == 0) ? 1.0 : 0.0;
    }
  }
  int nk = (nd == 3) ? 5 : 1;
  for (int c = 0; c < nk; ++c)
    for (int b = 0; b < 5; ++b)
      for (int a = 0; a < 5; ++a) {
        double wt = S[0][a] * S[1][b] * S[2][c];
        if (wt == 0.0) continue;
        rho[nidx(g, base[0] + a, base[1] + b, base[2] + c)] += q * w * wt;
      }
}

static double wrap_pos(double p, double L) {
  if (p < 0.0) p += L;
  if (p >= L) p -= L;
  return p;
}

/* Algorithm 1, particle loop of one species: push positions by dt/2, interpolate E and B
 * there, Boris push of the momentum by dt, push positions by dt/2 with the new velocity.
 * The current follows Sec. 3.1 and Eq. 3: the deposit traces the trajectory over one dt
 * centred on the end of the step, i.e. the straight path from the half-step position
 * x^{n+1/2} to x^{n+1/2} + dt v^{n+1}, which gives J at the whole time level n+1 that
 * Eq. 3 pairs with E^{n+1/2} -> E^{n+3/2}.  The stored position x^{n+1} is the midpoint of
 * that path. */
static void advance_range(const orc_grid *g, orc_fields *f, orc_species *s, int64_t p_begin,
                          int64_t p_end, int32_t deposit, double *xso, double *yso,
                          double *zso) {
  int nd = g->ndim;
  double dt = g->dt;
  double L[3] = {g->nx * g->dx, g->ny * g->dy, g->nz * g->dz};
  for (int64_t p = p_begin; p < p_end; ++p) {
    if (s->x[p] < 0.0) continue; /* dead particle */
    double p0[3] = {s->x[p], s->y[p], (nd == 3) ? s->z[p] : 0.0};
    double u[3] = {s->ux[p], s->uy[p], s->uz[p]};
    double g0 = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double ph[3] = {p0[0], p0[1], p0[2]};
    for (int d = 0; d < nd; ++d) ph[d] = p0[d] + 0.5 * dt * u[d] / g0;
    double E[3], B[3];
    orc_gather(g, f, s->order, ph, E, B);
    orc_boris(u, E, B, s->q, s->m, dt);
    double g1 = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double p1[3] = {ph[0], ph[1], ph[2]};
    double pe[3] = {ph[0], ph[1], ph[2]};
    for (int d = 0; d < nd; ++d) {
      p1[d] = ph[d] + 0.5 * dt * u[d] / g1;
      pe[d] = ph[d] + dt * u[d] / g1;
    }
    if (xso) xso[p] = ph[0];
    if (yso) yso[p] = ph[1];
    if (zso) zso[p] = ph[2];
    if (deposit) {
      orc_deposit_particle(g, f, s->order, s->q, s->w[p], ph, pe, u[2] / g1);
      if (f->rho0) orc_deposit_rho(g, f->rho0, s->order, s->q, s->w[p], ph);
      if (f->rho1) orc_deposit_rho(g, f->rho1, s->order, s->q, s->w[p], pe);
    }
    s->x[p] = wrap_pos(p1[0], L[0]);
    s->y[p] = wrap_pos(p1[1], L[1]);
    if (nd == 3) s->z[p] = wrap_pos(p1[2], L[2]);
    s->ux[p] = u[0];
    s->uy[p] = u[1];
    s->uz[p] = u[2];
    if (g->open_x && (p1[0] < ORC_OPEN_MARGIN * g->dx ||
                      p1[0] >= (g->nx - ORC_OPEN_MARGIN) * g->dx))
      s->x[p] = -1.0;   /* left through an open x end */
  }
}

static void advance_species(const orc_grid *g, orc_fields *f, orc_species *s, int32_t deposit,
                            double *xso, double *yso, double *zso) {
  advance_range(g, f, s, 0, s->n, deposit, xso, yso, zso);
}

void orc_push_deposit(const orc_grid *g, orc_fields *f, orc_species *s, int32_t deposit,
                      double *xs, double *ys, double *zs) {
  advance_species(g, f, s, deposit, xs, ys, zs);
}

void orc_gather_push(const orc_grid *g, const orc_fields *f, orc_species *s) {
  advance_species(g, (orc_fields *)f, s, 0, NULL, NULL, NULL);
}

/* The antenna current of the header's definition, added into J at time t. */
void orc_laser_source(const orc_grid *g, orc_fields *f, const orc_laser *laser, double t) {
  double tau = t - laser->t0;
  if (tau < 0.0 || tau > laser->tau) return;
  double env = sin(M_PI * tau / laser->tau);
  double amp = laser->a0 * laser->omega * env * env * sin(laser->omega * tau);
  int three = (g->ndim == 3);
  int nz = three ? g->nz : 1;
  double *J = (laser->pol == 1) ? f->jy : f->jz;
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < g->ny; ++j) {
      /* position of the J component's node: J_y at (ia, j+1/2, k), J_z at (ia, j, k+1/2) */
      double y = (j + (laser->pol == 1 ? 0.5 : 0.0)) * g->dy;
      double z = three ? (k + (laser->pol == 2 ? 0.5 : 0.0)) * g->dz : laser->zc;
      double r2 = (y - laser->yc) * (y - laser->yc) + (z - laser->zc) * (z - laser->zc);
      double einc = amp * exp(-r2 / (laser->waist * laser->waist));
      J[nidx(g, laser->ia, j, k)] += -2.0 * einc / g->dx;
    }
}

/* Algorithm 1: one timestep.  The first E half uses the current still held in J (the one
 * deposited by the previous step, zero before the first step), so that together with the
 * second half of the previous step E advances by a whole dt with that J, as in Eq. 3. */
void orc_step(const orc_grid *g, orc_fields *f, orc_species *sp, int32_t nspecies,
              const orc_laser *laser, double t_next) {
  int64_t n = ncell(g);
  orc_yee_e(g, f, 0.5);
  orc_yee_b(g, f, 0.5);
  memset(f->jx, 0, sizeof(double) * n);
  memset(f->jy, 0, sizeof(double) * n);
  memset(f->jz, 0, sizeof(double) * n);
  if (f->rho0) memset(f->rho0, 0, sizeof(double) * n);
  if (f->rho1) memset(f->rho1, 0, sizeof(double) * n);
  for (int s = 0; s < nspecies; ++s) advance_species(g, f, &sp[s], 1, NULL, NULL, NULL);
  if (laser) orc_laser_source(g, f, laser, t_next);
  orc_yee_b(g, f, 0.5);
  orc_yee_e(g, f, 0.5);
}

/* The same timestep with the particle loop spread over nthreads threads, for timing the
 * oracle on all host cores.  Every particle takes exactly the arithmetic of orc_step; each
 * thread deposits into private zeroed current (and charge) arrays, which are added into the
 * shared ones afterwards in thread order, so the result differs from orc_step only in the
 * order of the current sums.  Field updates and the antenna stay single threaded.  Returns
 * the number of threads that ran the particle loop. */
int32_t orc_step_threads(const orc_grid *g, orc_fields *f, orc_species *sp, int32_t nspecies,
                         const orc_laser *laser, double t_next, int32_t nthreads) {
  int64_t n = ncell(g);
  int nt = nthreads > 0 ? nthreads : 1;
  const int nprivate = 5;
  double *priv = (double *)calloc((size_t)nt * nprivate * n, sizeof(double));
  if (!priv) return -1;
  int ran = 1;
  orc_yee_e(g, f, 0.5);
  orc_yee_b(g, f, 0.5);
#pragma omp parallel num_threads(nt)
  {
    int t = 0, tn = 1;
#ifdef _OPENMP
    t = omp_get_thread_num();
    tn = omp_get_num_threads();
#pragma omp single
    ran = tn;
#endif
    double *base = priv + (size_t)t * nprivate * n;
    orc_fields mine = *f;
    mine.jx = base;
    mine.jy = base + n;
    mine.jz = base + 2 * n;
    mine.rho0 = f->rho0 ? base + 3 * n : NULL;
    mine.rho1 = f->rho1 ? base + 4 * n : NULL;
    for (int s = 0; s < nspecies; ++s) {
      int64_t per = (sp[s].n + tn - 1) / tn;
      int64_t lo = (int64_t)t * per, hi = lo + per < sp[s].n ? lo + per : sp[s].n;
      if (lo < hi) advance_range(g, &mine, &sp[s], lo, hi, 1, NULL, NULL, NULL);
    }
#pragma omp barrier
    double *dst[5] = {f->jx, f->jy, f->jz, f->rho0, f->rho1};
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i)
      for (int c = 0; c < nprivate; ++c) {
        if (!dst[c]) continue;
        double acc = 0.0;
        for (int k = 0; k < tn; ++k) acc += priv[((size_t)k * nprivate + c) * n + i];
        dst[c][i] = acc;
      }
  }
  free(priv);
  if (laser) orc_laser_source(g, f, laser, t_next);
  orc_yee_b(g, f, 0.5);
  orc_yee_e(g, f, 0.5);
  return ran;
}

static double cell_volume(const orc_grid *g) {
  return g->dx * g->dy * (g->ndim == 3 ? g->dz : 1.0);
}

/* Electromagnetic energy: sum over all array entries of (E^2 + B^2)/2 times the cell volume
 * (the total energy recorded for the heating test of Sec. 4.1). */
double orc_field_energy(const orc_grid *g, const orc_fields *f) {
  int64_t n = ncell(g);
  double s = 0.0;
  for (int64_t c = 0; c < n; ++c)
    s += f->ex[c] * f->ex[c] + f->ey[c] * f->ey[c] + f->ez[c] * f->ez[c] +
         f->bx[c] * f->bx[c] + f->by[c] * f->by[c] + f->bz[c] * f->bz[c];
  return 0.5 * s * cell_volume(g);
}

/* Kinetic energy m (gamma - 1) per physical particle, written as m u^2 / (1 + gamma); a
 * macro-particle stands for w * dV physical particles. */
double orc_kinetic_energy(const orc_grid *g, const orc_species *s) {
  double acc = 0.0;
  for (int64_t p = 0; p < s->n; ++p) {
    if (s->x[p] < 0.0) continue;
    double u2 = s->ux[p] * s->ux[p] + s->uy[p] * s->uy[p] + s->uz[p] * s->uz[p];
    acc += s->w[p] * s->m * u2 / (1.0 + sqrt(1.0 + u2));
  }
  return acc * cell_volume(g);
}

static double div_at_node(const orc_grid *g, const double *ax, const double *ay,
                          const double *az, int64_t i, int64_t j, int64_t k) {
  int64_t c = nidx(g, i, j, k);
  double d = (ax[c] - ax[nidx(g, i - 1, j, k)]) / g->dx + (ay[c] - ay[nidx(g, i, j - 1, k)]) / g->dy;
  if (g->ndim == 3) d += (az[c] - az[nidx(g, i, j, k - 1)]) / g->dz;
  return d;
}

/* Discrete continuity (Sec. 3.1): (rho1 - rho0)/dt + div J = 0 at every node, with rho0 and
 * rho1 the charge at the two ends of the deposited paths. */
double orc_continuity(const orc_grid *g, const orc_fields *f) {
  int nz = (g->ndim == 3) ? g->nz : 1;
  double rmax = 0.0, qmax = 0.0;
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < g->ny; ++j)
      for (int64_t i = 0; i < g->nx; ++i) {
        int64_t c = nidx(g, i, j, k);
        double r = f->rho1[c] - f->rho0[c] + g->dt * div_at_node(g, f->jx, f->jy, f->jz, i, j, k);
        if (fabs(r) > rmax) rmax = fabs(r);
        if (fabs(f->rho1[c]) > qmax) qmax = fabs(f->rho1[c]);
      }
  return qmax > 0.0 ? rmax / qmax : rmax;
}

void orc_gauss(const orc_grid *g, const orc_fields *f, double *out) {
  int nz = (g->ndim == 3) ? g->nz : 1;
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < g->ny; ++j)
      for (int64_t i = 0; i < g->nx; ++i) {
        int64_t c = nidx(g, i, j, k);
        out[c] = div_at_node(g, f->ex, f->ey, f->ez, i, j, k) - 0.5 * (f->rho0[c] + f->rho1[c]) -
                 g->rho_bg;
      }
}

void orc_div_b(const orc_grid *g, const orc_fields *f, double *out) {
  int nz = (g->ndim == 3) ? g->nz : 1;
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < g->ny; ++j)
      for (int64_t i = 0; i < g->nx; ++i) {
        int64_t c = nidx(g, i, j, k);
        double d = (f->bx[nidx(g, i + 1, j, k)] - f->bx[c]) / g->dx +
                   (f->by[nidx(g, i, j + 1, k)] - f->by[c]) / g->dy;
        if (g->ndim == 3) d += (f->bz[nidx(g, i, j, k + 1)] - f->bz[c]) / g->dz;
        out[c] = d;
      }
}
