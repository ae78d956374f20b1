/* QED event Monte-Carlo of Sec. 3.4 (nonlinear Compton emission and Breit-Wheeler pair
 * creation in the locally-constant-field approximation, one event per particle and step
 * triggered when the optical depth crosses zero).
 *
 * TEST INFRASTRUCTURE ONLY: part of the oracle; only the test suite, the smoke entry point
 * and the CPU-baseline leg of the benchmark may call it.  Plain FP64, single threaded,
 * every quantity from its defining integral; shares no code with the HIP library.
 *
 * Units are those of the rest of the oracle: c = m_e = e = 1, time in 1/w_r, fields in
 * m_e c w_r / e, momenta in m_e c.  hbar_omega = hbar w_r / (m_e c^2) fixes the Schwinger
 * field, E_S = 1 / hbar_omega in these units. */
#ifndef LPIC_ORACLE_QED_H
#define LPIC_ORACLE_QED_H

#include <stdint.h>

#include "oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Modified Bessel function K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt, x > 0. */
double orc_bessel_k(double nu, double x);
/* int_x^inf K_nu(s) ds = int_0^inf exp(-x cosh t) cosh(nu t) / cosh t dt, x > 0. */
double orc_bessel_k_tail(double nu, double x);

/* Photon emission spectrum per unit photon energy fraction xi = e_photon / (gamma m c^2),
 * in units of alpha m c^2 / (hbar gamma):
 *   F(chi, xi) = [ (1 - xi + 1/(1 - xi)) K_{2/3}(y) - int_y^inf K_{1/3} ] / (sqrt(3) pi),
 *   y = 2 xi / (3 chi (1 - xi)),   0 < xi < 1 (zero outside). */
double orc_compton_spectrum(double chi, double xi);
/* int_0^xi F(chi, .) ; the total h(chi) at xi = 1; the first moment int_0^1 xi F. */
double orc_compton_cdf(double chi, double xi);
double orc_compton_rate(double chi);
double orc_compton_moment(double chi);
/* The xi whose cdf is r h(chi), 0 < r < 1 (bisection). */
double orc_compton_sample(double chi, double r);

/* Pair creation spectrum per unit electron energy fraction xi = e_electron / e_photon, in
 * units of alpha (m c^2)^2 / (hbar e_photon):
 *   G(chi, xi) = [ (xi/(1 - xi) + (1 - xi)/xi) K_{2/3}(y) + int_y^inf K_{1/3} ] / (sqrt(3) pi),
 *   y = 2 / (3 chi xi (1 - xi)). */
double orc_bw_spectrum(double chi, double xi);
double orc_bw_cdf(double chi, double xi);
double orc_bw_rate(double chi);
double orc_bw_sample(double chi, double r);

/* Quantum parameters from the field tensor (Sec. 3.4):
 *   lepton  chi_e = hbar_omega sqrt((gamma E + u x B)^2 - (u . E)^2),
 *   photon  chi_g = hbar_omega sqrt((|k| E + k x B)^2 - (k . E)^2). */
double orc_chi_lepton(const double u[3], const double E[3], const double B[3], double hbar_omega);
double orc_chi_photon(const double k[3], const double E[3], const double B[3], double hbar_omega);

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the k-th output (k = 0, 1, ...) of the
 * generator seeded with `seed`. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k);
/* The uniform draw in (0, 1) of one particle: counter k = ((step << 32) | slot) * 4 + draw,
 * value ((z >> 11) + 1/2) 2^-53. */
double orc_qed_uniform(uint64_t seed, int64_t step, int64_t slot, int32_t draw);

typedef struct {
  double hbar_omega;
  uint64_t seed;
  int64_t step;
} orc_qed;

/* Records created by events: photons (from emission) or leptons (from pairs: electron at
 * an even index, positron at the next).  count grows past capacity without writing. */
typedef struct {
  int64_t capacity, count;
  double *x, *y, *z, *ux, *uy, *uz, *w, *tau;
  int32_t *src;
} orc_qed_buf;

/* Optical depths of a fresh population: tau[i] = -ln(U(seed, step, i, 2)). */
void orc_qed_init_tau(double *tau, int64_t n, uint64_t seed, int64_t step);

/* The particle part of Algorithm 1 for a lepton species with nonlinear Compton emission:
 * half position push, gather at x^{n+1/2}, the emission event with the momentum u^n (the
 * optical depth drops by W dt, W = alpha h(chi_e) / (gamma hbar_omega); where it reaches
 * zero or below: xi from draw 0, a photon of momentum xi gamma u/|u| leaves, the lepton
 * keeps u - xi gamma u/|u|, a new depth -ln(draw 1)), Boris, half position push.  The
 * photon is recorded at x^{n+1/2} (wrapped) with the lepton's weight, depth -ln(draw 2)
 * and src = the lepton's index.  Open x ends remove a lepton as orc_gather_push does. */
void orc_qed_gather_push(const orc_grid *g, const orc_fields *f, orc_species *s, double *tau,
                         const orc_qed *q, orc_qed_buf *photons);

/* One step of the photons [0, photons->count) (shape order `order` for the gather): they
 * move at c along k; at x^{n+1/2} the optical depth drops by W dt, W = alpha T(chi_g) /
 * (|k| hbar_omega); where it reaches zero or below the photon turns into a pair at
 * x^{n+1/2}: xi from draw 0, electron energy xi |k|, positron (1 - xi) |k|, momenta along
 * k (|u| = sqrt(gamma^2 - 1), zero below gamma = 1), the photon's weight, depths -ln(draw
 * 2) and -ln(draw 3), src = the photon's index; the photon is removed (x = -1).  Photons
 * leaving through an open x end are removed. */
void orc_qed_photon_push(const orc_grid *g, const orc_fields *f, int32_t order,
                         orc_qed_buf *photons, const orc_qed *q, orc_qed_buf *pairs);

#ifdef __cplusplus
}
#endif
#endif
