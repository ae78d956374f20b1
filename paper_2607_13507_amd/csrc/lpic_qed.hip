// QED event Monte-Carlo of Sec. 3.4: nonlinear Compton emission by leptons and
// Breit-Wheeler pair creation by photons in the locally-constant-field approximation, with
// one event per particle and step where its optical depth reaches zero.
//
// The rates and the inverse cumulative distributions of both spectra are tabulated once on
// the host and interpolated in the kernels:
//   rates    ln h(chi) (emission) and ln T(chi) + 8/(3 chi) (pairs; the added term removes
//            the exp(-8/(3 chi)) fall of the pair rate at small chi) at 40 points per decade
//            of chi, linear in ln chi;
//   samples  v = ln(xi / (1 - xi)) at z = ln(r / (1 - r)) in [-20, 20] (161 points) for every
//            tabulated chi, cubic in z and linear in ln chi: near r = 0 the emission
//            quantile goes like r^3 (v linear in z), near r = 1 like -ln(1 - r) (v like ln z).
// The table builder evaluates K_{2/3}(y) and int_y^inf K_{1/3} with the trapezoid rule on
// their integral representations (even, analytic, double-exponentially decaying
// integrands), integrates each spectrum over v with Simpson's rule, and inverts the
// cumulative sums with a cubic solve inside each interval.
#include <math.h>

#include <algorithm>
#include <mutex>
#include <thread>
#include <vector>

#include "lpic_internal.hpp"

namespace lpic {

namespace {

constexpr double kAlpha = 7.2973525693e-3;     // fine-structure constant (CODATA 2018)
constexpr double kPi = 3.14159265358979323846;

// ---- spectra on the host ---------------------------------------------------------------
// K_{2/3}(y) and int_y^inf K_{1/3}(s) ds: int_0^inf exp(-y cosh t) cosh(2t/3) dt and
// int_0^inf exp(-y cosh t) cosh(t/3) / cosh t dt in one trapezoid sum over [0, T], where
// the integrand has fallen below exp(-760).
void bessel_pair(double y, double& k23, double& ik13) {
  k23 = ik13 = 0.0;
  if (y > 740.0) return;
  const double T = acosh(std::max(760.0 / y, 1.0));
  double h = y > 1.0 ? 0.08 / sqrt(y) : 0.08;
  const int n = std::max(16, (int)ceil(T / h));
  h = T / n;
  double a = 0.0, b = 0.0;
  for (int i = 0; i <= n; ++i) {
    const double t = i * h, ch = cosh(t);
    const double e = exp(-y * ch) * (i == 0 ? 0.5 : 1.0);
    a += e * cosh(t * (2.0 / 3.0));
    b += e * cosh(t * (1.0 / 3.0)) / ch;
  }
  k23 = a * h;
  ik13 = b * h;
}

// The spectra as densities in v = ln(xi / (1 - xi)): F(chi, xi) xi (1 - xi) and the same
// for G.  With om = 1 - xi: 1 - xi + 1/(1 - xi) = om + 1/om, xi/(1 - xi) = e^v.
double emit_density(double chi, double v) {
  const double y = 2.0 / (3.0 * chi) * exp(v);
  if (y > 740.0) return 0.0;
  const double xi = 1.0 / (1.0 + exp(-v)), om = 1.0 / (1.0 + exp(v));
  double k23, ik13;
  bessel_pair(y, k23, ik13);
  return ((om + 1.0 / om) * k23 - ik13) / (sqrt(3.0) * kPi) * xi * om;
}

double pair_density(double chi, double v) {
  const double y = 4.0 / (3.0 * chi) * (1.0 + cosh(v));   // 2 / (3 chi xi (1 - xi))
  if (y > 740.0) return 0.0;
  const double xi = 1.0 / (1.0 + exp(-v)), om = 1.0 / (1.0 + exp(v));
  double k23, ik13;
  bessel_pair(y, k23, ik13);
  return ((exp(v) + exp(-v)) * k23 + ik13) / (sqrt(3.0) * kPi) * xi * om;
}

// One tabulated chi: the density on a uniform v grid (nodes and midpoints), its running
// Simpson integral, the total, and the v of every quantile level of the z grid.
// `below` is the mass under the grid's first node (emission: the xi^(-2/3) law there).
void build_row(double (*dens)(double, double), double chi, double vlo, double vhi, double dv,
               bool power_below, double* total, double* vrow) {
  const int n = std::max(2, (int)ceil((vhi - vlo) / dv));
  dv = (vhi - vlo) / n;
  std::vector<double> p(n + 1), m(n), C(n + 1);
  for (int k = 0; k <= n; ++k) p[k] = dens(chi, vlo + k * dv);
  for (int k = 0; k < n; ++k) m[k] = dens(chi, vlo + (k + 0.5) * dv);
  // below the first node F ~ A xi^(-2/3), so int_0^xi0 F = 3 xi0 F(xi0) = 3 p0 / (1 - xi0)
  C[0] = power_below ? 3.0 * p[0] * (1.0 + exp(vlo)) : 0.0;
  for (int k = 0; k < n; ++k) C[k + 1] = C[k] + dv / 6.0 * (p[k] + 4.0 * m[k] + p[k + 1]);
  *total = C[n];
  for (int j = 0; j < QED_NZ; ++j) {
    const double z = QED_Z0 + QED_DZ * j;
    const double r = 1.0 / (1.0 + exp(-z));
    const double target = r * C[n];
    if (target <= C[0]) {            // inside the power law below the grid: xi ~ (C/C0)^3
      vrow[j] = C[0] > 0.0 ? vlo + 3.0 * log(target / C[0]) : vlo;
      continue;
    }
    const int k = std::min<int>(n - 1, (int)(std::upper_bound(C.begin(), C.end(), target) -
                                             C.begin()) - 1);
    // inside [v_k, v_k + dv] the density is the parabola through p_k, m_k, p_k+1; solve
    // C_k + int_0^s P = target for s by Newton steps from the linear guess
    const double a0 = p[k], a1 = (4.0 * m[k] - 3.0 * p[k] - p[k + 1]) / dv,
                 a2 = 2.0 * (p[k] + p[k + 1] - 2.0 * m[k]) / (dv * dv);
    const double need = target - C[k];
    double s = C[k + 1] > C[k] ? dv * need / (C[k + 1] - C[k]) : 0.0;
    for (int it = 0; it < 4; ++it) {
      const double f = a0 * s + a1 * s * s / 2.0 + a2 * s * s * s / 3.0 - need;
      const double d = a0 + a1 * s + a2 * s * s;
      if (d > 0.0) s -= f / d;
      s = std::min(std::max(s, 0.0), dv);
    }
    vrow[j] = vlo + k * dv + s;
  }
}

std::vector<double> g_host;
std::once_flag g_once;

void build_tables() {
  g_host.assign(qed_table_doubles(), 0.0);
  double* er = g_host.data();
  double* pr = er + QED_NE;
  double* ei = pr + QED_NP;
  double* pinv = ei + (size_t)QED_NE * QED_NZ;
  const int rows = QED_NE + QED_NP;
  auto work = [&](int first, int stride) {
    for (int i = first; i < rows; i += stride) {
      double total;
      if (i < QED_NE) {
        const double lc = QED_E_L0 + QED_E_DL * i, chi = exp(lc);
        build_row(emit_density, chi, lc - 75.0, 40.0, 0.08, true, &total,
                  ei + (size_t)i * QED_NZ);
        er[i] = log(total);
      } else {
        const int b = i - QED_NE;
        const double lc = QED_P_L0 + QED_P_DL * b, chi = exp(lc);
        // the pair density is a narrow peak at v = 0 for small chi (width ~ sqrt(chi))
        const double dv = std::min(0.08, 0.1 * sqrt(3.0 * chi / 4.0));
        build_row(pair_density, chi, -40.0, 40.0, dv, false, &total, pinv + (size_t)b * QED_NZ);
        pr[b] = log(total) + 8.0 / (3.0 * chi);
      }
    }
  };
  // rows are independent: spread them over the host threads; if no thread can be started
  // the calling thread takes the rows of the threads that are missing
  const unsigned nt = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  std::vector<int> orphan;
  for (unsigned t = 1; t < nt; ++t) {
    try {
      th.emplace_back(work, (int)t, (int)nt);
    } catch (...) {
      orphan.push_back((int)t);
    }
  }
  work(0, (int)nt);
  for (int t : orphan) work(t, (int)nt);
  for (auto& t : th) t.join();
}

// ---- kernels ----------------------------------------------------------------------------
__device__ __forceinline__ double qed_chi(double scale, const double v[3], const double E[3],
                                          const double B[3], double hw) {
  const double a0 = scale * E[0] + v[1] * B[2] - v[2] * B[1];
  const double a1 = scale * E[1] + v[2] * B[0] - v[0] * B[2];
  const double a2 = scale * E[2] + v[0] * B[1] - v[1] * B[0];
  const double ve = v[0] * E[0] + v[1] * E[1] + v[2] * E[2];
  const double s = a0 * a0 + a1 * a1 + a2 * a2 - ve * ve;
  return s > 0.0 ? hw * sqrt(s) : 0.0;
}

__device__ __forceinline__ double wrap_pos(double p, double L) {
  return p < 0.0 ? p + L : (p >= L ? p - L : p);
}

// Record slots for the threads of a workgroup that want `per` records each: one atomic add
// on the count per workgroup (same-address atomics serialise in the L2, one per wave cost
// more than the rest of the kernel), each wanting thread's first slot from its rank in the
// workgroup.  Every thread of the workgroup must call it.
constexpr int QED_BLOCK = 1024;

__device__ __forceinline__ int64_t block_slots(int32_t* count, bool want, int per) {
  __shared__ int wcount[QED_BLOCK / 64];
  __shared__ int bbase;
  const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
  const uint64_t mask = __ballot(want);
  if (lane == 0) wcount[wave] = __popcll(mask);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      const int c = wcount[w];
      wcount[w] = tot;
      tot += c;
    }
    bbase = tot ? atomicAdd(count, per * tot) : 0;
  }
  __syncthreads();
  const int rank = __popcll(mask & ((1ull << lane) - 1ull));
  return want ? (int64_t)bbase + (int64_t)per * (wcount[wave] + rank) : -1;
}

// One record's contents.
struct QedRec {
  double pos[3], u[3], w, tau;
};

// Writes one record at slot i (below capacity only).
__device__ __forceinline__ void put_record(const QedBufDesc& b, int64_t i, const double pos[3],
                                           const double u[3], double w, double tau, int src) {
  if (i >= b.cap) return;
  b.x[i] = pos[0];
  b.y[i] = pos[1];
  if (b.z) b.z[i] = pos[2];
  b.ux[i] = u[0];
  b.uy[i] = u[1];
  b.uz[i] = u[2];
  b.w[i] = w;
  b.tau[i] = tau;
  b.src[i] = src;
}

template <typename R, int DIM, int ORDER>
__device__ __forceinline__ bool qed_push_one(const SegDesc& s, const RunDesc& r, int64_t p,
                                             void* old, double* tau, const QedCall& q,
                                             QedRec& rec) {
  PState<R> ps;
  load_particle<R, DIM>(s, r, (int32_t)p, ps);
  OldState<R, DIM> os(old, s.n);
  if (!ps.alive) {
    if (os.cell) os.cell[p] = -1;
    else os.o[0][p] = R(-1);
    return false;
  }
  const GlobalAcc<R> A = global_acc<R>(r);
  const PushConst<R> k = push_const<R>(r, s);
  int pc[3];
  R po[3], xh[3], E[3], B[3];
  half_push<DIM>(ps.c, ps, k, pc, po, xh);
  gather<DIM, ORDER>(A, pc, po, E, B);
  const int n[3] = {r.nx, r.ny, r.nz};
  int wc[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < DIM; ++d) wc[d] = wrapi(pc[d], n[d]);

  // the emission event, with u^n, before the Boris push
  double u[3] = {(double)ps.u[0], (double)ps.u[1], (double)ps.u[2]};
  const double Ed[3] = {(double)E[0], (double)E[1], (double)E[2]};
  const double Bd[3] = {(double)B[0], (double)B[1], (double)B[2]};
  const double g0 = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  const double chi = qed_chi(g0, u, Ed, Bd, q.hw);
  double t = tau[p] - kAlpha * qed_emit_rate(q.tab, chi) / (g0 * q.hw) * r.dt;
  const bool fire = t <= 0.0;
  double* kk = rec.u;
  double* pos = rec.pos;
#pragma unroll
  for (int d = 0; d < 3; ++d) kk[d] = pos[d] = 0.0;
  if (fire) {
    const double xi = qed_emit_sample(q.tab, chi, qed_draw(q.seed, q.step, p, 0));
    const double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (um > 0.0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) kk[d] = xi * g0 * u[d] / um;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      u[d] -= kk[d];
      ps.u[d] = (R)u[d];
    }
    const double h[3] = {r.dx, r.dy, r.dz};
#pragma unroll
    for (int d = 0; d < DIM; ++d) pos[d] = ((double)wc[d] + (double)po[d]) * h[d];
    t = qed_neglog(qed_draw(q.seed, q.step, p, 1));
    rec.w = (double)ps.w;
    rec.tau = qed_neglog(qed_draw(q.seed, q.step, p, 2));
  }
  tau[p] = t;

  boris<R>(ps.u, E, B, k.qdt2m);
  const R ig1 = rsq<R>(R(1) + ps.u[0] * ps.u[0] + ps.u[1] * ps.u[1] + ps.u[2] * ps.u[2]);
  const R hd[3] = {k.hdx, k.hdy, k.hdz};
  if constexpr (sizeof(R) == 4) {
    os.cell[p] = pack_cell(wc, DIM);
#pragma unroll
    for (int d = 0; d < DIM; ++d) os.o[d][p] = po[d];
  } else {
    const double h[3] = {r.dx, r.dy, r.dz};
#pragma unroll
    for (int d = 0; d < DIM; ++d) os.o[d][p] = ((double)wc[d] + po[d]) * h[d];
  }
#pragma unroll
  for (int d = 0; d < DIM; ++d) advance_cell<R>(ps.c[d], ps.o[d], xh[d] + hd[d] * ps.u[d] * ig1, n[d]);
  store_particle<R, DIM>(s, r, (int32_t)p, ps);
  return fire;
}

// One species of a single run (the tables of lpic_qed_gather_push), QED_BLOCK particles per
// workgroup; every thread reaches the slot reservation.
template <typename R, int DIM>
__global__ __launch_bounds__(QED_BLOCK) void k_qed_push(Tables T, void* old, double* tau,
                                                        QedCall q) {
  const SegDesc& s = seg_of(T, 0);
  const int64_t p = (int64_t)blockIdx.x * QED_BLOCK + threadIdx.x;
  QedRec rec;
  bool fire = false;
  if (p < s.n) {
    const RunDesc& r = run_of(T, s.run);
    fire = s.order == 1 ? qed_push_one<R, DIM, 1>(s, r, p, old, tau, q, rec)
                        : qed_push_one<R, DIM, 2>(s, r, p, old, tau, q, rec);
  }
  const int64_t slot = block_slots(q.out.count, fire, 1);
  if (fire) put_record(q.out, slot, rec.pos, rec.u, rec.w, rec.tau, (int)p);
}

template <typename R, int DIM, int ORDER>
__device__ __forceinline__ bool qed_photon_one(const RunDesc& r, const QedBufDesc& ph,
                                               int64_t p, const QedCall& q, QedRec& re,
                                               QedRec& rp) {
  if (!(ph.x[p] >= 0.0)) return false;
  const double kv[3] = {ph.ux[p], ph.uy[p], ph.uz[p]};
  const double km = sqrt(kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2]);
  double v[3] = {0.0, 0.0, 0.0};
  if (km > 0.0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) v[d] = kv[d] / km;
  }
  const double h[3] = {r.dx, r.dy, r.dz};
  const double L[3] = {r.nx * r.dx, r.ny * r.dy, r.nz * r.dz};
  double pos[3] = {ph.x[p], ph.y[p], DIM == 3 ? ph.z[p] : 0.0};
#pragma unroll
  for (int d = 0; d < DIM; ++d) pos[d] += 0.5 * r.dt * v[d];
  // the gather point as (cell, offset); the cell is off the box by at most one
  int c[3] = {0, 0, 0};
  R o[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double X = pos[d] / h[d], f = floor(X);
    c[d] = (int)f;
    o[d] = (R)(X - f);
  }
  R E[3], B[3];
  gather<DIM, ORDER>(global_acc<R>(r), c, o, E, B);
  const double Ed[3] = {(double)E[0], (double)E[1], (double)E[2]};
  const double Bd[3] = {(double)B[0], (double)B[1], (double)B[2]};
  const double chi = qed_chi(km, kv, Ed, Bd, q.hw);
  double t = ph.tau[p];
  if (km > 0.0) t -= kAlpha * qed_pair_rate(q.tab, chi) / (km * q.hw) * r.dt;
  const bool fire = t <= 0.0;
  double *ue = re.u, *up = rp.u;
  if (fire) {
    const double xi = qed_pair_sample(q.tab, chi, qed_draw(q.seed, q.step, p, 0));
    const double ge = xi * km, gp = (1.0 - xi) * km;
    const double ae = ge > 1.0 ? sqrt(ge * ge - 1.0) : 0.0;
    const double ap = gp > 1.0 ? sqrt(gp * gp - 1.0) : 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      ue[d] = ae * v[d];
      up[d] = ap * v[d];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) re.pos[d] = rp.pos[d] = d < DIM ? wrap_pos(pos[d], L[d]) : 0.0;
    re.w = rp.w = ph.w[p];
    re.tau = qed_neglog(qed_draw(q.seed, q.step, p, 2));
    rp.tau = qed_neglog(qed_draw(q.seed, q.step, p, 3));
    ph.tau[p] = t;
    ph.x[p] = -1.0;
    return true;
  }
  ph.tau[p] = t;
  double x1[3];
#pragma unroll
  for (int d = 0; d < DIM; ++d) x1[d] = pos[d] + 0.5 * r.dt * v[d];
  ph.x[p] = wrap_pos(x1[0], L[0]);
  ph.y[p] = wrap_pos(x1[1], L[1]);
  if (DIM == 3) ph.z[p] = wrap_pos(x1[2], L[2]);
  if (r.open_x && (x1[0] < OPEN_MARGIN * r.dx || x1[0] >= (r.nx - OPEN_MARGIN) * r.dx))
    ph.x[p] = -1.0;
  return false;
}

template <typename R, int DIM>
__global__ __launch_bounds__(QED_BLOCK) void k_qed_photons(RunDesc r, QedBufDesc ph, int order,
                                                           QedCall q) {
  const int64_t n = min((int64_t)*ph.count, ph.cap);
  const int64_t p = (int64_t)blockIdx.x * QED_BLOCK + threadIdx.x;
  if ((int64_t)blockIdx.x * QED_BLOCK >= n) return;      // the whole workgroup
  QedRec re, rp;
  bool fire = false;
  if (p < n) {
    fire = order == 1 ? qed_photon_one<R, DIM, 1>(r, ph, p, q, re, rp)
                      : qed_photon_one<R, DIM, 2>(r, ph, p, q, re, rp);
  }
  const int64_t slot = block_slots(q.out.count, fire, 2);
  if (fire) {
    put_record(q.out, slot, re.pos, re.u, re.w, re.tau, (int)p);
    put_record(q.out, slot + 1, rp.pos, rp.u, rp.w, rp.tau, (int)p);
  }
}

__global__ __launch_bounds__(256) void k_qed_tau(double* tau, int64_t n, uint64_t seed,
                                                 int64_t step) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) tau[i] = qed_neglog(qed_draw(seed, step, i, 2));
}

// Stable compaction of a record buffer (the lazily deleted records, x < 0, dropped):
// per-workgroup live counts, one workgroup's exclusive scan of them, then a scatter that
// keeps the records' order.
__global__ __launch_bounds__(QED_BLOCK) void k_qed_live_counts(QedBufDesc b, int32_t* blk) {
  __shared__ int wsum[QED_BLOCK / 64];
  const int64_t n = min((int64_t)*b.count, b.cap);
  const int64_t i = (int64_t)blockIdx.x * QED_BLOCK + threadIdx.x;
  const bool live = i < n && b.x[i] >= 0.0;
  const uint64_t m = __ballot(live);
  if (__lane_id() == 0) wsum[threadIdx.x >> 6] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < QED_BLOCK / 64; ++w) t += wsum[w];
    blk[blockIdx.x] = t;
  }
}

// Exclusive scan of nblk counts in place, the total into blk[nblk]: one workgroup walks the
// counts QED_BLOCK at a time.
__global__ __launch_bounds__(QED_BLOCK) void k_qed_scan_counts(int32_t* blk, int nblk) {
  __shared__ int wsum[QED_BLOCK / 64];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
  for (int base = 0; base < nblk; base += QED_BLOCK) {
    const int i = base + (int)threadIdx.x;
    const int v = i < nblk ? blk[i] : 0;
    int x = v;   // inclusive scan inside the wave
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int before = carry;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    if (i < nblk) blk[i] = before + x - v;
    __syncthreads();
    if (threadIdx.x == QED_BLOCK - 1) carry = before + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) blk[nblk] = carry;
}

__global__ __launch_bounds__(QED_BLOCK) void k_qed_compact(QedBufDesc in, QedBufDesc out,
                                                           const int32_t* blk, int nblk) {
  __shared__ int wsum[QED_BLOCK / 64];
  const int64_t n = min((int64_t)*in.count, in.cap);
  const int64_t i = (int64_t)blockIdx.x * QED_BLOCK + threadIdx.x;
  const bool live = i < n && in.x[i] >= 0.0;
  const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
  const uint64_t m = __ballot(live);
  if (lane == 0) wsum[wave] = __popcll(m);
  __syncthreads();
  int before = blk[blockIdx.x];
  for (int w = 0; w < wave; ++w) before += wsum[w];
  const int64_t j = (int64_t)before + __popcll(m & ((1ull << lane) - 1ull));
  if (live && j < out.cap) {
    out.x[j] = in.x[i];
    out.y[j] = in.y[i];
    if (out.z && in.z) out.z[j] = in.z[i];
    out.ux[j] = in.ux[i];
    out.uy[j] = in.uy[i];
    out.uz[j] = in.uz[i];
    out.w[j] = in.w[i];
    out.tau[j] = in.tau[i];
    out.src[j] = in.src[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *out.count = blk[nblk];
}

// Records into species slots: record i of the selected parity (or every record, parity < 0)
// goes to slot first + i / 2 (or first + i); positions become the species' representation
// (FP32: wrapped cell and offset; FP64: absolute), momenta and weight its precision.
template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_qed_insert(Tables T, int64_t first, QedBufDesc b,
                                                    int parity, int32_t* dropped) {
  const SegDesc& s = seg_of(T, 0);
  const RunDesc& r = run_of(T, s.run);
  const int64_t nrec = min((int64_t)*b.count, b.cap);
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nrec || (parity >= 0 && (i & 1) != parity)) return;
  const int64_t p = first + (parity >= 0 ? i >> 1 : i);
  if (p >= s.n) {
    if (dropped) atomicAdd(dropped, 1);
    return;
  }
  const double src[3] = {b.x[i], b.y[i], DIM == 3 ? b.z[i] : 0.0};
  if constexpr (sizeof(R) == 4) {
    const double h[3] = {r.dx, r.dy, r.dz};
    const int n[3] = {r.nx, r.ny, r.nz};
    int c[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double X = src[d] / h[d];
      const double f = floor(X);
      int ci = (int)f;
      float o = (float)(X - f);
      if (o >= 1.0f) { o = 0.0f; ci += 1; }
      ci = ci >= n[d] ? ci - n[d] : (ci < 0 ? ci + n[d] : ci);
      c[d] = ci;
      ((float*)s.p[P_OX + d])[p] = o;
    }
    ((int32_t*)s.p[P_CELL])[p] = b.x[i] >= 0.0 ? pack_cell(c, DIM) : -1;
  } else {
#pragma unroll
    for (int d = 0; d < DIM; ++d) ((double*)s.p[P_X + d])[p] = src[d];
  }
  ((R*)s.p[P_UX])[p] = (R)b.ux[i];
  ((R*)s.p[P_UY])[p] = (R)b.uy[i];
  ((R*)s.p[P_UZ])[p] = (R)b.uz[i];
  ((R*)s.p[P_W])[p] = (R)b.w[i];
}

}  // namespace

size_t qed_table_doubles() {
  return (size_t)QED_NE + QED_NP + (size_t)(QED_NE + QED_NP) * QED_NZ;
}

// nullptr if the host memory for the tables could not be had
const double* qed_host_tables() {
  try {
    std::call_once(g_once, build_tables);
  } catch (...) {
    return nullptr;
  }
  return g_host.size() == qed_table_doubles() ? g_host.data() : nullptr;
}

QedTab qed_views(const double* base) {
  QedTab t;
  t.emit_rate = base;
  t.pair_rate = base + QED_NE;
  t.emit_inv = t.pair_rate + QED_NP;
  t.pair_inv = t.emit_inv + (size_t)QED_NE * QED_NZ;
  return t;
}

void launch_qed_tau(double* tau, int64_t n, uint64_t seed, int64_t step, hipStream_t st) {
  if (n <= 0) return;
  k_qed_tau<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(tau, n, seed, step);
}

void launch_qed_push(const Tables& T, int prec, int dim, int64_t n, void* old, double* tau,
                     const QedCall& q, hipStream_t st) {
  if (n <= 0) return;
  const unsigned nblocks = (unsigned)((n + QED_BLOCK - 1) / QED_BLOCK);
  LPIC_PD(prec, dim, (k_qed_push<R, D><<<nblocks, QED_BLOCK, 0, st>>>(T, old, tau, q)));
}

void launch_qed_insert(const Tables& T, int prec, int dim, int64_t first, const QedBufDesc& b,
                       int parity, int32_t* dropped, hipStream_t st) {
  if (b.cap <= 0) return;
  const unsigned nb = (unsigned)((b.cap + 255) / 256);
  LPIC_PD(prec, dim, (k_qed_insert<R, D><<<nb, 256, 0, st>>>(T, first, b, parity, dropped)));
}

int qed_compact_blocks(int64_t cap) { return (int)((cap + QED_BLOCK - 1) / QED_BLOCK); }

void launch_qed_compact(const QedBufDesc& in, const QedBufDesc& out, int32_t* blk,
                        hipStream_t st) {
  const int nb = qed_compact_blocks(in.cap);
  if (nb <= 0) return;
  k_qed_live_counts<<<nb, QED_BLOCK, 0, st>>>(in, blk);
  k_qed_scan_counts<<<1, QED_BLOCK, 0, st>>>(blk, nb);
  k_qed_compact<<<nb, QED_BLOCK, 0, st>>>(in, out, blk, nb);
}

void launch_qed_photons(const RunDesc& r, int prec, int dim, int order, const QedBufDesc& ph,
                        const QedCall& q, hipStream_t st) {
  if (ph.cap <= 0) return;
  const unsigned nb = (unsigned)((ph.cap + QED_BLOCK - 1) / QED_BLOCK);
  LPIC_PD(prec, dim, (k_qed_photons<R, D><<<nb, QED_BLOCK, 0, st>>>(r, ph, order, q)));
}

}  // namespace lpic
