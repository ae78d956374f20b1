/* QED event Monte-Carlo of Sec. 3.4 -- TEST INFRASTRUCTURE ONLY (see qed.h).
 * Every function evaluates its defining integral with an adaptive Simpson rule in FP64. */
#include "qed.h"

#include <math.h>
#include <stddef.h>

#define ORC_ALPHA 7.2973525693e-3 /* fine-structure constant (CODATA 2018) */
#define ORC_PI 3.14159265358979323846

/* ---- adaptive Simpson ------------------------------------------------------------------ */
typedef double (*orc_fn)(double t, const void *ctx);

static double simpson_rec(orc_fn f, const void *c, double a, double b, double fa, double fm,
                          double fb, double whole, double eps, int depth) {
  double m = 0.5 * (a + b), lm = 0.5 * (a + m), rm = 0.5 * (m + b);
  double flm = f(lm, c), frm = f(rm, c);
  double left = (m - a) / 6.0 * (fa + 4.0 * flm + fm);
  double right = (b - m) / 6.0 * (fm + 4.0 * frm + fb);
  double diff = left + right - whole;
  if (depth <= 0 || fabs(diff) <= 15.0 * eps) return left + right + diff / 15.0;
  return simpson_rec(f, c, a, m, fa, flm, fm, left, 0.5 * eps, depth - 1) +
         simpson_rec(f, c, m, b, fm, frm, fb, right, 0.5 * eps, depth - 1);
}

/* int_a^b f to a relative accuracy of about rel: P panels set the scale, then each panel
 * is refined adaptively. */
static double integrate_p(orc_fn f, const void *c, double a, double b, double rel, int P,
                          double abs_tol) {
  if (!(b > a)) return 0.0;
  double h = (b - a) / P, fx[2 * 64 + 1], coarse = 0.0;
  for (int i = 0; i <= 2 * P; ++i) fx[i] = f(a + 0.5 * h * i, c);
  for (int i = 0; i < P; ++i) coarse += h / 6.0 * (fx[2 * i] + 4.0 * fx[2 * i + 1] + fx[2 * i + 2]);
  /* below 1e-250 (and near the subnormal range) no refinement can improve anything */
  double eps = fmax(rel * fabs(coarse), abs_tol) / P;
  if (fabs(coarse) < 1e-250 || eps == 0.0) return coarse;
  double s = 0.0;
  for (int i = 0; i < P; ++i) {
    double pa = a + h * i, pb = pa + h;
    double whole = h / 6.0 * (fx[2 * i] + 4.0 * fx[2 * i + 1] + fx[2 * i + 2]);
    s += simpson_rec(f, c, pa, pb, fx[2 * i], fx[2 * i + 1], fx[2 * i + 2], whole, eps, 40);
  }
  return s;
}

static double integrate(orc_fn f, const void *c, double a, double b, double rel) {
  return integrate_p(f, c, a, b, rel, 64, 0.0);
}

/* ---- Bessel functions from their integral representations ----------------------------
 * The integrands below are even, analytic and fall off like exp(-x e^t / 2), so the
 * trapezoid rule over [0, T] (half weight at t = 0) converges faster than any power of
 * the step: the step is halved until two successive sums agree to 1e-14. */
static double k_integrand(double nu, double x, int tail, double t) {
  double ch = cosh(t);
  double v = exp(-x * ch) * cosh(nu * t);
  return tail ? v / ch : v;
}

static double bessel_int(double nu, double x, int tail) {
  if (!(x > 0.0)) return INFINITY;
  if (x > 745.0) return 0.0;               /* exp(-x) underflows */
  /* beyond T the integrand is below exp(-750) */
  double T = acosh(750.0 / x > 1.0 ? 750.0 / x : 1.0);
  double h = 0.5 / (x > 1.0 ? sqrt(x) : 1.0);
  int n = (int)ceil(T / h);
  if (n < 8) n = 8;
  h = T / n;
  double sum = 0.5 * k_integrand(nu, x, tail, 0.0);
  for (int i = 1; i <= n; ++i) sum += k_integrand(nu, x, tail, i * h);
  double prev = sum * h;
  for (int level = 0; level < 20; ++level) {
    for (int i = 0; i < n; ++i) sum += k_integrand(nu, x, tail, (i + 0.5) * h);
    n *= 2;
    h *= 0.5;
    double cur = sum * h;
    if (fabs(cur - prev) <= 1e-14 * fabs(cur)) return cur;
    prev = cur;
  }
  return prev;
}

double orc_bessel_k(double nu, double x) { return bessel_int(nu, x, 0); }
double orc_bessel_k_tail(double nu, double x) { return bessel_int(nu, x, 1); }

/* ---- nonlinear Compton ----------------------------------------------------------------- */
double orc_compton_spectrum(double chi, double xi) {
  if (!(chi > 0.0) || !(xi > 0.0) || !(xi < 1.0)) return 0.0;
  double y = 2.0 * xi / (3.0 * chi * (1.0 - xi));
  if (y > 745.0) return 0.0;
  double a = (1.0 - xi + 1.0 / (1.0 - xi)) * orc_bessel_k(2.0 / 3.0, y);
  return (a - orc_bessel_k_tail(1.0 / 3.0, y)) / (sqrt(3.0) * ORC_PI);
}

/* F has an integrable xi^(-2/3) singularity at 0: integrate over s = xi^(1/3). */
typedef struct { double chi; int moment; int bw; } sctx;

static double compton_s(double s, const void *c) {
  const sctx *k = (const sctx *)c;
  double xi = s * s * s;
  double v = 3.0 * s * s * orc_compton_spectrum(k->chi, xi);
  return k->moment ? xi * v : v;
}

double orc_compton_cdf(double chi, double xi) {
  if (!(chi > 0.0) || !(xi > 0.0)) return 0.0;
  sctx c = {chi, 0, 0};
  return integrate(compton_s, &c, 0.0, cbrt(xi < 1.0 ? xi : 1.0), 1e-10);
}

double orc_compton_rate(double chi) { return orc_compton_cdf(chi, 1.0); }

double orc_compton_moment(double chi) {
  if (!(chi > 0.0)) return 0.0;
  sctx c = {chi, 1, 0};
  return integrate(compton_s, &c, 0.0, 1.0, 1e-10);
}

/* ---- Breit-Wheeler --------------------------------------------------------------------- */
double orc_bw_spectrum(double chi, double xi) {
  if (!(chi > 0.0) || !(xi > 0.0) || !(xi < 1.0)) return 0.0;
  double y = 2.0 / (3.0 * chi * xi * (1.0 - xi));
  if (y > 745.0) return 0.0;
  double a = (xi / (1.0 - xi) + (1.0 - xi) / xi) * orc_bessel_k(2.0 / 3.0, y);
  return (a + orc_bessel_k_tail(1.0 / 3.0, y)) / (sqrt(3.0) * ORC_PI);
}

static double bw_xi(double xi, const void *c) {
  return orc_bw_spectrum(((const sctx *)c)->chi, xi);
}

double orc_bw_cdf(double chi, double xi) {
  if (!(chi > 0.0) || !(xi > 0.0)) return 0.0;
  sctx c = {chi, 0, 1};
  return integrate(bw_xi, &c, 0.0, xi < 1.0 ? xi : 1.0, 1e-10);
}

double orc_bw_rate(double chi) { return orc_bw_cdf(chi, 1.0); }

/* ---- inverse-transform sampling --------------------------------------------------------
 * Bisection for the point where the cdf reaches r times the total; each step integrates
 * only the piece between the bracket's lower end and its midpoint. */
static double sample(orc_fn f, const void *c, double lo, double hi, double total, double r) {
  double target = r * total, flo = 0.0;
  for (int it = 0; it < 60 && hi - lo > 1e-14 * hi; ++it) {
    double mid = 0.5 * (lo + hi);
    /* pieces far out in a tail need no more than an absolute accuracy of the total's */
    double fm = flo + integrate_p(f, c, lo, mid, 1e-10, 4, 1e-13 * total);
    if (fm < target) { lo = mid; flo = fm; } else { hi = mid; }
  }
  return 0.5 * (lo + hi);
}

double orc_compton_sample(double chi, double r) {
  sctx c = {chi, 0, 0};
  double s = sample(compton_s, &c, 0.0, 1.0, orc_compton_rate(chi), r);
  return s * s * s;
}

double orc_bw_sample(double chi, double r) {
  sctx c = {chi, 0, 1};
  return sample(bw_xi, &c, 0.0, 1.0, orc_bw_rate(chi), r);
}

/* ---- quantum parameters ---------------------------------------------------------------- */
static double chi_of(double scale, const double v[3], const double E[3], const double B[3],
                     double hbar_omega) {
  double a[3] = {scale * E[0] + v[1] * B[2] - v[2] * B[1],
                 scale * E[1] + v[2] * B[0] - v[0] * B[2],
                 scale * E[2] + v[0] * B[1] - v[1] * B[0]};
  double ve = v[0] * E[0] + v[1] * E[1] + v[2] * E[2];
  double s = a[0] * a[0] + a[1] * a[1] + a[2] * a[2] - ve * ve;
  return s > 0.0 ? hbar_omega * sqrt(s) : 0.0;
}

double orc_chi_lepton(const double u[3], const double E[3], const double B[3], double hbar_omega) {
  return chi_of(sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]), u, E, B, hbar_omega);
}

double orc_chi_photon(const double k[3], const double E[3], const double B[3], double hbar_omega) {
  return chi_of(sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]), k, E, B, hbar_omega);
}

/* ---- counter-based draws --------------------------------------------------------------- */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double orc_qed_uniform(uint64_t seed, int64_t step, int64_t slot, int32_t draw) {
  uint64_t k = ((((uint64_t)step) << 32) | (uint64_t)(uint32_t)slot) * 4u + (uint64_t)draw;
  return ((double)(orc_splitmix64(seed, k) >> 11) + 0.5) * 0x1p-53;
}

void orc_qed_init_tau(double *tau, int64_t n, uint64_t seed, int64_t step) {
  for (int64_t i = 0; i < n; ++i) tau[i] = -log(orc_qed_uniform(seed, step, i, 2));
}

/* ---- event steps ----------------------------------------------------------------------- */
static double wrap_to(double p, double L) {
  if (p < 0.0) p += L;
  if (p >= L) p -= L;
  return p;
}

static int64_t append(orc_qed_buf *b, const double pos[3], const double u[3], double w,
                      double tau, int32_t src) {
  int64_t i = b->count++;
  if (i >= b->capacity) return -1;
  b->x[i] = pos[0];
  b->y[i] = pos[1];
  if (b->z) b->z[i] = pos[2];
  b->ux[i] = u[0];
  b->uy[i] = u[1];
  b->uz[i] = u[2];
  b->w[i] = w;
  b->tau[i] = tau;
  b->src[i] = src;
  return i;
}

static int leaves_open_x(const orc_grid *g, double x) {
  return g->open_x && (x < ORC_OPEN_MARGIN * g->dx || x >= (g->nx - ORC_OPEN_MARGIN) * g->dx);
}

void orc_qed_gather_push(const orc_grid *g, const orc_fields *f, orc_species *s, double *tau,
                         const orc_qed *q, orc_qed_buf *photons) {
  int nd = g->ndim;
  double dt = g->dt;
  double L[3] = {g->nx * g->dx, g->ny * g->dy, g->nz * g->dz};
  for (int64_t p = 0; p < s->n; ++p) {
    if (s->x[p] < 0.0) continue;
    double p0[3] = {s->x[p], s->y[p], nd == 3 ? s->z[p] : 0.0};
    double u[3] = {s->ux[p], s->uy[p], s->uz[p]};
    double g0 = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double ph[3] = {p0[0], p0[1], p0[2]};
    for (int d = 0; d < nd; ++d) ph[d] = p0[d] + 0.5 * dt * u[d] / g0;
    double E[3], B[3];
    orc_gather(g, f, s->order, ph, E, B);
    /* Sec. 3.4: the event between the interpolation and the Boris push */
    double chi = orc_chi_lepton(u, E, B, q->hbar_omega);
    double t = tau[p] - ORC_ALPHA * orc_compton_rate(chi) / (g0 * q->hbar_omega) * dt;
    if (t <= 0.0) {
      double xi = orc_compton_sample(chi, orc_qed_uniform(q->seed, q->step, p, 0));
      double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      double k[3] = {0.0, 0.0, 0.0};
      if (um > 0.0)
        for (int d = 0; d < 3; ++d) k[d] = xi * g0 * u[d] / um;
      for (int d = 0; d < 3; ++d) u[d] -= k[d];
      double pos[3] = {wrap_to(ph[0], L[0]), wrap_to(ph[1], L[1]),
                       nd == 3 ? wrap_to(ph[2], L[2]) : 0.0};
      append(photons, pos, k, s->w[p], -log(orc_qed_uniform(q->seed, q->step, p, 2)),
             (int32_t)p);
      t = -log(orc_qed_uniform(q->seed, q->step, p, 1));
    }
    tau[p] = t;
    orc_boris(u, E, B, s->q, s->m, dt);
    double g1 = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double p1[3] = {ph[0], ph[1], ph[2]};
    for (int d = 0; d < nd; ++d) p1[d] = ph[d] + 0.5 * dt * u[d] / g1;
    s->x[p] = wrap_to(p1[0], L[0]);
    s->y[p] = wrap_to(p1[1], L[1]);
    if (nd == 3) s->z[p] = wrap_to(p1[2], L[2]);
    s->ux[p] = u[0];
    s->uy[p] = u[1];
    s->uz[p] = u[2];
    if (leaves_open_x(g, p1[0])) s->x[p] = -1.0;
  }
}

void orc_qed_photon_push(const orc_grid *g, const orc_fields *f, int32_t order,
                         orc_qed_buf *photons, const orc_qed *q, orc_qed_buf *pairs) {
  int nd = g->ndim;
  double dt = g->dt;
  double L[3] = {g->nx * g->dx, g->ny * g->dy, g->nz * g->dz};
  int64_t n = photons->count < photons->capacity ? photons->count : photons->capacity;
  orc_qed_buf *b = photons;
  for (int64_t p = 0; p < n; ++p) {
    if (b->x[p] < 0.0) continue;
    double k[3] = {b->ux[p], b->uy[p], b->uz[p]};
    double km = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    double v[3] = {0.0, 0.0, 0.0};
    if (km > 0.0)
      for (int d = 0; d < 3; ++d) v[d] = k[d] / km;
    double p0[3] = {b->x[p], b->y[p], nd == 3 ? b->z[p] : 0.0};
    double ph[3] = {p0[0], p0[1], p0[2]};
    for (int d = 0; d < nd; ++d) ph[d] = p0[d] + 0.5 * dt * v[d];
    double E[3], B[3];
    orc_gather(g, f, order, ph, E, B);
    double chi = orc_chi_photon(k, E, B, q->hbar_omega);
    double t = b->tau[p];
    if (km > 0.0) t -= ORC_ALPHA * orc_bw_rate(chi) / (km * q->hbar_omega) * dt;
    if (t <= 0.0) {
      double xi = orc_bw_sample(chi, orc_qed_uniform(q->seed, q->step, p, 0));
      double ge = xi * km, gp = (1.0 - xi) * km;
      double ae = ge > 1.0 ? sqrt(ge * ge - 1.0) : 0.0;
      double ap = gp > 1.0 ? sqrt(gp * gp - 1.0) : 0.0;
      double ue[3], up[3];
      for (int d = 0; d < 3; ++d) { ue[d] = ae * v[d]; up[d] = ap * v[d]; }
      double pos[3] = {wrap_to(ph[0], L[0]), wrap_to(ph[1], L[1]),
                       nd == 3 ? wrap_to(ph[2], L[2]) : 0.0};
      append(pairs, pos, ue, b->w[p], -log(orc_qed_uniform(q->seed, q->step, p, 2)), (int32_t)p);
      append(pairs, pos, up, b->w[p], -log(orc_qed_uniform(q->seed, q->step, p, 3)), (int32_t)p);
      b->tau[p] = t;
      b->x[p] = -1.0;
      continue;
    }
    b->tau[p] = t;
    double p1[3] = {ph[0], ph[1], ph[2]};
    for (int d = 0; d < nd; ++d) p1[d] = ph[d] + 0.5 * dt * v[d];
    b->x[p] = wrap_to(p1[0], L[0]);
    b->y[p] = wrap_to(p1[1], L[1]);
    if (nd == 3) b->z[p] = wrap_to(p1[2], L[2]);
    if (leaves_open_x(g, p1[0])) b->x[p] = -1.0;
  }
}
