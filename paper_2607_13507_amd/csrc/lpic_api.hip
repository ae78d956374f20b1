// C ABI of the PIC hot path: argument validation, descriptor set-up, launch sequencing,
// the Algorithm 1 step loop with named-stage hooks, HIP graph capture and the autotuner.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <numeric>
#include <cmath>
#include <string>
#include <vector>

#include "lpic.h"
#include "lpic_internal.hpp"

static_assert(LPIC_OPEN_MARGIN == lpic::OPEN_MARGIN, "open-end margin differs");

using namespace lpic;

namespace {

thread_local std::string g_err;

lpic_status fail(lpic_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(LPIC_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define CHK(expr)                          \
  do {                                     \
    lpic_status s_ = (expr);               \
    if (s_ != LPIC_OK) return s_;          \
  } while (0)

lpic_status last_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LPIC_EHIP, "%s launch: %s", what, hipGetErrorString(e));
  return LPIC_OK;
}

int ilog2_exact(int v) {
  if (v <= 0 || (v & (v - 1))) return -1;
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

int64_t ncells(const lpic_grid* g) {
  return (int64_t)g->nx * g->ny * (g->ndim == 3 ? g->nz : 1);
}

lpic_status check_grid(const lpic_grid* g, int prec) {
  if (!g) return fail(LPIC_EINVAL, "grid is NULL");
  if (g->ndim != 2 && g->ndim != 3) return fail(LPIC_EINVAL, "ndim must be 2 or 3 (got %d)", g->ndim);
  if (g->nx < 4 || g->ny < 4 || (g->ndim == 3 && g->nz < 4))
    return fail(LPIC_EINVAL, "every grid dimension must be >= 4 cells");
  if (g->ndim == 2 && g->nz != 1) return fail(LPIC_EINVAL, "nz must be 1 in 2D");
  if (!(g->dx > 0) || !(g->dy > 0) || (g->ndim == 3 && !(g->dz > 0)) || !(g->dt > 0))
    return fail(LPIC_EINVAL, "cell sizes and dt must be positive");
  double s = 1.0 / (g->dx * g->dx) + 1.0 / (g->dy * g->dy);
  if (g->ndim == 3) s += 1.0 / (g->dz * g->dz);
  const double cfl = 1.0 / sqrt(s);
  if (g->dt > cfl * (1.0 + 1e-12))
    return fail(LPIC_EINVAL, "dt = %g exceeds the CFL limit %g", g->dt, cfl);
  if (prec == LPIC_F32_CELLOFS) {
    if (g->ndim == 2 && (g->nx > 65536 || g->ny > 32768))
      return fail(LPIC_EINVAL, "2D cell packing needs nx <= 65536, ny <= 32768");
    if (g->ndim == 3 && (g->nx > 2048 || g->ny > 2048 || g->nz > 512))
      return fail(LPIC_EINVAL, "3D cell packing needs nx, ny <= 2048, nz <= 512");
  }
  if (ncells(g) >= (int64_t)1 << 31) return fail(LPIC_EINVAL, "grid has too many cells");
  if (g->open_x != 0 && g->open_x != 1) return fail(LPIC_EINVAL, "open_x must be 0 or 1");
  if (g->open_x && g->nx < 2 * LPIC_OPEN_MARGIN + 2)
    return fail(LPIC_EINVAL, "open x ends need nx >= %d", 2 * LPIC_OPEN_MARGIN + 2);
  if (prec != LPIC_F32_CELLOFS && prec != LPIC_F64_ABS)
    return fail(LPIC_EINVAL, "unknown precision %d", prec);
  return LPIC_OK;
}

lpic_status check_fields(const lpic_fields* f, bool need_rho) {
  if (!f) return fail(LPIC_EINVAL, "fields is NULL");
  const void* p[9] = {f->ex, f->ey, f->ez, f->bx, f->by, f->bz, f->jx, f->jy, f->jz};
  for (int i = 0; i < 9; ++i)
    if (!p[i]) return fail(LPIC_EINVAL, "field array %d is NULL", i);
  if (need_rho && (!f->rho0 || !f->rho1)) return fail(LPIC_EINVAL, "rho0/rho1 are required");
  return LPIC_OK;
}

lpic_status check_species(const lpic_species* s, int ndim, int prec) {
  if (!s) return fail(LPIC_EINVAL, "species is NULL");
  if (s->n < 0) return fail(LPIC_EINVAL, "negative particle count");
  // (kernels address a particle array with a 32-bit byte offset: slot * 8 < 2^32)
  if (s->n > ((int64_t)1 << 29)) return fail(LPIC_EINVAL, "a species holds at most 2^29 slots");
  if (s->shape_order != 1 && s->shape_order != 2)
    return fail(LPIC_EINVAL, "shape_order must be 1 or 2 (got %d)", s->shape_order);
  if (!(s->m > 0)) return fail(LPIC_EINVAL, "mass must be positive");
  if (s->n == 0) return LPIC_OK;
  if (!s->ux || !s->uy || !s->uz || !s->w) return fail(LPIC_EINVAL, "momentum/weight arrays are NULL");
  if (prec == LPIC_F32_CELLOFS) {
    if (!s->cell || !s->ox || !s->oy || (ndim == 3 && !s->oz))
      return fail(LPIC_EINVAL, "cell/offset arrays are NULL");
  } else {
    if (!s->x || !s->y || (ndim == 3 && !s->z)) return fail(LPIC_EINVAL, "position arrays are NULL");
  }
  return LPIC_OK;
}

lpic_status check_tiling(const lpic_tiling* t, const lpic_grid* g, int prec,
                         bool need_lds = true) {
  if (!t) return fail(LPIC_EINVAL, "tiling is NULL");
  const int nd = g->ndim;
  if (ilog2_exact(t->tx) < 0 || ilog2_exact(t->ty) < 0 || (nd == 3 && ilog2_exact(t->tz) < 0))
    return fail(LPIC_EINVAL, "tile edges must be powers of two");
  if (t->halo < 3) return fail(LPIC_EINVAL, "halo must be >= 3");
  if (t->halo > g->nx || t->halo > g->ny || (nd == 3 && t->halo > g->nz))
    return fail(LPIC_EINVAL, "halo larger than the grid");
  if (t->chunk < 1) return fail(LPIC_EINVAL, "chunk must be >= 1");
  if (t->flags & ~(LPIC_SORT_SPREAD | LPIC_FIELD_SEPARATE | LPIC_ESCAPE_REBIN))
    return fail(LPIC_EINVAL, "unknown tiling flags 0x%x", t->flags);
  const size_t smem = fused_smem_bytes(prec, nd, t->tx, t->ty, nd == 3 ? t->tz : 1, t->halo, 1);
  if (need_lds && smem > 160 * 1024)
    return fail(LPIC_EINVAL, "tile + halo needs %zu bytes of LDS (limit 163840)", smem);
  return LPIC_OK;
}

void tile_counts(const lpic_grid* g, const lpic_tiling* t, int& ntx, int& nty, int& ntz) {
  ntx = (g->nx + t->tx - 1) / t->tx;
  nty = (g->ny + t->ty - 1) / t->ty;
  ntz = g->ndim == 3 ? (g->nz + t->tz - 1) / t->tz : 1;
}

RunDesc make_run(const lpic_grid* g, const lpic_fields* f, const lpic_tiling* t) {
  RunDesc r;
  memset(&r, 0, sizeof(r));
  r.ndim = g->ndim;
  r.nx = g->nx;
  r.ny = g->ny;
  r.nz = g->ndim == 3 ? g->nz : 1;
  r.dx = g->dx;
  r.dy = g->dy;
  r.dz = g->ndim == 3 ? g->dz : 1.0;
  r.dt = g->dt;
  r.rho_bg = g->rho_bg;
  r.open_x = g->open_x;
  r.has_laser = 0;
  r.seg_first = 0;
  r.nseg = 1;
  r.vbase = 0;
  if (t) {
    tile_counts(g, t, r.ntx, r.nty, r.ntz);
    r.ntiles = r.ntx * r.nty * r.ntz;
  } else {
    r.ntx = r.nty = r.ntz = 1;
    r.ntiles = 1;
  }
  if (f) {
    void* p[F_NUM] = {f->ex, f->ey, f->ez, f->bx, f->by, f->bz, f->jx, f->jy, f->jz,
                      f->rho0, f->rho1};
    for (int i = 0; i < F_NUM; ++i) r.f[i] = p[i];
  }
  r.diag = nullptr;
  return r;
}

void species_ptrs(const lpic_species* s, int prec, void* out[P_NUM]) {
  for (int i = 0; i < P_NUM; ++i) out[i] = nullptr;
  if (!s) return;
  if (prec == LPIC_F32_CELLOFS) {
    out[P_CELL] = s->cell;
    out[P_OX] = s->ox;
    out[P_OY] = s->oy;
    out[P_OZ] = s->oz;
  } else {
    out[P_X] = s->x;
    out[P_Y] = s->y;
    out[P_Z] = s->z;
  }
  out[P_UX] = s->ux;
  out[P_UY] = s->uy;
  out[P_UZ] = s->uz;
  out[P_W] = s->w;
}

void set_species_ptrs(lpic_species* s, int prec, void* const in[P_NUM]) {
  if (prec == LPIC_F32_CELLOFS) {
    s->cell = (int32_t*)in[P_CELL];
    s->ox = in[P_OX];
    s->oy = in[P_OY];
    s->oz = in[P_OZ];
  } else {
    s->x = in[P_X];
    s->y = in[P_Y];
    s->z = in[P_Z];
  }
  s->ux = in[P_UX];
  s->uy = in[P_UY];
  s->uz = in[P_UZ];
  s->w = in[P_W];
}

SegDesc make_seg(const lpic_species* s, const lpic_species* alt, int run, const lpic_tiling* t,
                 int bin_base, int64_t pbase, int prec) {
  SegDesc d;
  memset(&d, 0, sizeof(d));
  d.run = run;
  d.order = s->shape_order;
  if (t) {
    d.lx = ilog2_exact(t->tx);
    d.ly = ilog2_exact(t->ty);
    d.lz = ilog2_exact(t->tz > 0 ? t->tz : 1);
    if (d.lz < 0) d.lz = 0;
    d.halo = t->halo;
  }
  d.bin_base = bin_base;
  d.n = s->n;
  d.pbase = pbase;
  d.q = s->q;
  d.m = s->m;
  species_ptrs(s, prec, d.p);
  species_ptrs(alt, prec, d.alt);
  return d;
}

Tables single_tables(const RunDesc& r, const SegDesc* s) {
  Tables T;
  memset(&T, 0, sizeof(T));
  T.nruns = 1;
  T.nsegs = 1;
  T.run0 = r;
  if (s) T.seg0 = *s;
  return T;
}

size_t old_state_bytes(int ndim, int64_t n, int prec) {
  if (prec == LPIC_F32_CELLOFS) return (size_t)n * (4 + 4 * ndim);
  return (size_t)n * 8 * ndim;
}

int64_t max_chunks_of(int64_t ntiles, int64_t n, int chunk) {
  return ntiles + (n + chunk - 1) / chunk;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Escapes per step from which a simulation with LPIC_ESCAPE_REBIN groups them by present
// tile for a second fused pass (below it, k_escape's global atomics cost less than the
// grouping's scans).
constexpr int REBIN_THRESHOLD = 4096;

// The fused kernel is persistent: XCD x (workgroups x, x+8, x+16, ...) owns the contiguous
// chunk range [x*per, (x+1)*per), per = ceil(nchunks/8), split into equal slices.  The grid
// is a multiple of 8: as many workgroups as fit on the device at once, and never more than
// there can be chunks.
int fused_grid(int64_t max_chunks, int blocks_per_cu) {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
  }
  int64_t g = (int64_t)cus * std::max(1, blocks_per_cu);
  g = std::min<int64_t>(g, std::max<int64_t>(max_chunks, 1));
  return (int)((g + 7) / 8 * 8);
}

}  // namespace

// =======================================================================================
// Stateless entry points
// =======================================================================================
extern "C" {

const char* lpic_last_error(void) { return g_err.c_str(); }
const char* lpic_version(void) { return "lpic-mi355x 0.1 (gfx950)"; }

lpic_status lpic_yee_update_EB(const lpic_grid* grid, const lpic_fields* fields, int32_t which,
                               double frac, int32_t flags, lpic_precision prec,
                               hipStream_t stream) {
  CHK(check_grid(grid, prec));
  CHK(check_fields(fields, false));
  if (which != 0 && which != 1) return fail(LPIC_EINVAL, "which must be 0 (E) or 1 (B)");
  if (!(frac > 0) || frac > 1.0) return fail(LPIC_EINVAL, "frac must be in (0, 1]");
  RunDesc r = make_run(grid, fields, nullptr);
  Tables T = single_tables(r, nullptr);
  const int64_t nb = (ncells(grid) + 255) / 256;
  launch_yee(T, prec, grid->ndim, (int)nb, which, frac, (flags & LPIC_YEE_ZERO_J) ? 1 : 0, 1,
             stream);
  return last_launch("yee");
}

lpic_status check_laser(const lpic_laser* l, const lpic_grid* g) {
  if (!l) return fail(LPIC_EINVAL, "laser is NULL");
  if (l->pol != 1 && l->pol != 2) return fail(LPIC_EINVAL, "laser pol must be 1 (y) or 2 (z)");
  if (l->ia < 0 || l->ia >= g->nx) return fail(LPIC_EINVAL, "laser column %d outside the grid", l->ia);
  if (!(l->tau > 0) || !(l->waist > 0) || !std::isfinite(l->a0) || !std::isfinite(l->omega))
    return fail(LPIC_EINVAL, "laser needs tau > 0, waist > 0 and finite a0, omega");
  return LPIC_OK;
}

LaserDesc make_laser(const lpic_laser* l) {
  LaserDesc d;
  d.pol = l->pol;
  d.ia = l->ia;
  d.e0 = l->a0 * l->omega;
  d.omega = l->omega;
  d.waist = l->waist;
  d.yc = l->yc;
  d.zc = l->zc;
  d.t0 = l->t0;
  d.tau = l->tau;
  return d;
}

int columns_bpr(const lpic_grid* g) {
  return (int)(((int64_t)g->ny * (g->ndim == 3 ? g->nz : 1) + 255) / 256);
}

lpic_status lpic_laser_source(const lpic_grid* grid, const lpic_fields* fields,
                              const lpic_laser* laser, double t, lpic_precision prec,
                              hipStream_t stream) {
  CHK(check_grid(grid, prec));
  CHK(check_fields(fields, false));
  CHK(check_laser(laser, grid));
  RunDesc r = make_run(grid, fields, nullptr);
  r.has_laser = 1;
  r.laser = make_laser(laser);
  Tables T = single_tables(r, nullptr);
  launch_laser(T, prec, grid->ndim, 1, columns_bpr(grid), t, nullptr, nullptr, stream);
  return last_launch("laser");
}

size_t lpic_old_state_bytes(int32_t ndim, int64_t n, lpic_precision prec) {
  return old_state_bytes(ndim, n, prec);
}

lpic_status lpic_gather_push(const lpic_grid* grid, const lpic_fields* fields,
                             const lpic_species* sp, void* old_state, size_t old_bytes,
                             lpic_precision prec, hipStream_t stream) {
  CHK(check_grid(grid, prec));
  CHK(check_fields(fields, false));
  CHK(check_species(sp, grid->ndim, prec));
  if (sp->n == 0) return LPIC_OK;
  if (!old_state || old_bytes < old_state_bytes(grid->ndim, sp->n, prec))
    return fail(LPIC_EINVAL, "old_state needs %zu bytes", old_state_bytes(grid->ndim, sp->n, prec));
  RunDesc r = make_run(grid, fields, nullptr);
  SegDesc s = make_seg(sp, nullptr, 0, nullptr, 0, 0, prec);
  Tables T = single_tables(r, &s);
  launch_gather_push(T, prec, grid->ndim, (int)((sp->n + 255) / 256), old_state, stream);
  return last_launch("gather_push");
}

lpic_status lpic_deposit_esirkepov(const lpic_grid* grid, const lpic_fields* fields,
                                   const lpic_species* sp, const void* old_state,
                                   size_t old_bytes, int32_t with_rho, lpic_precision prec,
                                   hipStream_t stream) {
  CHK(check_grid(grid, prec));
  CHK(check_fields(fields, with_rho != 0));
  CHK(check_species(sp, grid->ndim, prec));
  if (sp->n == 0) return LPIC_OK;
  if (!old_state || old_bytes < old_state_bytes(grid->ndim, sp->n, prec))
    return fail(LPIC_EINVAL, "old_state needs %zu bytes", old_state_bytes(grid->ndim, sp->n, prec));
  RunDesc r = make_run(grid, fields, nullptr);
  SegDesc s = make_seg(sp, nullptr, 0, nullptr, 0, 0, prec);
  Tables T = single_tables(r, &s);
  launch_deposit(T, prec, grid->ndim, (int)((sp->n + 255) / 256), old_state, with_rho, stream);
  return last_launch("deposit");
}

// ---- QED event Monte-Carlo (Sec. 3.4) -------------------------------------------------
struct lpic_qed_tables {
  QedTab host;
  QedTab dev;
  double* dev_base = nullptr;
};

static lpic_status check_qed_params(const lpic_qed_params* q) {
  if (!q) return fail(LPIC_EINVAL, "qed params are NULL");
  if (!(q->hbar_omega > 0.0) || !std::isfinite(q->hbar_omega))
    return fail(LPIC_EINVAL, "hbar_omega must be positive (got %g)", q->hbar_omega);
  if (q->step < 0 || q->step >= ((int64_t)1 << 30))
    return fail(LPIC_EINVAL, "step must be in [0, 2^30) (got %lld)", (long long)q->step);
  return LPIC_OK;
}

static lpic_status check_qed_buffer(const lpic_qed_buffer* b, int ndim, const char* what) {
  if (!b) return fail(LPIC_EINVAL, "%s buffer is NULL", what);
  if (b->capacity < 0 || b->capacity > ((int64_t)1 << 31) - 4)
    return fail(LPIC_EINVAL, "%s capacity must be in [0, 2^31 - 4]", what);
  if (!b->count) return fail(LPIC_EINVAL, "%s count is NULL", what);
  if (b->capacity > 0 && (!b->x || !b->y || (ndim == 3 && !b->z) || !b->ux || !b->uy ||
                          !b->uz || !b->w || !b->tau || !b->src))
    return fail(LPIC_EINVAL, "%s arrays must not be NULL", what);
  return LPIC_OK;
}

static QedBufDesc qed_desc(const lpic_qed_buffer* b) {
  QedBufDesc d;
  d.cap = b->capacity;
  d.count = b->count;
  d.x = b->x; d.y = b->y; d.z = b->z;
  d.ux = b->ux; d.uy = b->uy; d.uz = b->uz;
  d.w = b->w; d.tau = b->tau; d.src = b->src;
  return d;
}

lpic_status lpic_qed_tables_create(int32_t on_device, lpic_qed_tables** out) {
  if (!out) return fail(LPIC_EINVAL, "out is NULL");
  *out = nullptr;
  const double* host = qed_host_tables();
  if (!host) return fail(LPIC_ENOMEM, "QED tables: host memory");
  lpic_qed_tables* t = new (std::nothrow) lpic_qed_tables;
  if (!t) return fail(LPIC_ENOMEM, "QED tables: host memory");
  t->host = qed_views(host);
  t->dev = QedTab{nullptr, nullptr, nullptr, nullptr};
  if (on_device) {
    const size_t bytes = qed_table_doubles() * sizeof(double);
    hipError_t e = hipMalloc((void**)&t->dev_base, bytes);
    if (e == hipSuccess) e = hipMemcpy(t->dev_base, host, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      if (t->dev_base) (void)hipFree(t->dev_base);
      delete t;
      return fail(LPIC_EHIP, "QED tables: %s", hipGetErrorString(e));
    }
    t->dev = qed_views(t->dev_base);
  }
  *out = t;
  return LPIC_OK;
}

lpic_status lpic_qed_tables_destroy(lpic_qed_tables* t) {
  if (!t) return LPIC_OK;
  if (t->dev_base) HIPCHK(hipFree(t->dev_base));
  delete t;
  return LPIC_OK;
}

double lpic_qed_table_eval(const lpic_qed_tables* t, int32_t what, double chi, double r) {
  if (!t) return NAN;
  switch (what) {
    case LPIC_QED_EMIT_RATE: return qed_emit_rate(t->host, chi);
    case LPIC_QED_EMIT_SAMPLE: return qed_emit_sample(t->host, chi, r);
    case LPIC_QED_PAIR_RATE: return qed_pair_rate(t->host, chi);
    case LPIC_QED_PAIR_SAMPLE: return qed_pair_sample(t->host, chi, r);
    default: return NAN;
  }
}

lpic_status lpic_qed_init_tau(double* tau, int64_t n, uint64_t seed, int64_t step,
                              hipStream_t stream) {
  if (n < 0 || n >= ((int64_t)1 << 31)) return fail(LPIC_EINVAL, "n must be in [0, 2^31)");
  if (n > 0 && !tau) return fail(LPIC_EINVAL, "tau is NULL");
  if (step < 0 || step >= ((int64_t)1 << 30)) return fail(LPIC_EINVAL, "step must be in [0, 2^30)");
  launch_qed_tau(tau, n, seed, step, stream);
  return last_launch("qed_init_tau");
}

lpic_status lpic_qed_gather_push(const lpic_grid* grid, const lpic_fields* fields,
                                 const lpic_species* sp, double* tau,
                                 const lpic_qed_tables* tables, const lpic_qed_params* params,
                                 const lpic_qed_buffer* photons, void* old_state,
                                 size_t old_bytes, lpic_precision prec, hipStream_t stream) {
  CHK(check_grid(grid, prec));
  CHK(check_fields(fields, false));
  CHK(check_species(sp, grid->ndim, prec));
  CHK(check_qed_params(params));
  CHK(check_qed_buffer(photons, grid->ndim, "photon"));
  if (!tables || !tables->dev_base) return fail(LPIC_EINVAL, "QED tables without a device copy");
  if (sp->n == 0) return LPIC_OK;
  if (sp->n >= ((int64_t)1 << 31)) return fail(LPIC_EINVAL, "too many particles for the QED draws");
  if (!tau) return fail(LPIC_EINVAL, "tau is NULL");
  if (!old_state || old_bytes < old_state_bytes(grid->ndim, sp->n, prec))
    return fail(LPIC_EINVAL, "old_state needs %zu bytes", old_state_bytes(grid->ndim, sp->n, prec));
  RunDesc r = make_run(grid, fields, nullptr);
  SegDesc s = make_seg(sp, nullptr, 0, nullptr, 0, 0, prec);
  Tables T = single_tables(r, &s);
  QedCall q{tables->dev, params->hbar_omega, params->seed, params->step, qed_desc(photons)};
  launch_qed_push(T, prec, grid->ndim, sp->n, old_state, tau, q, stream);
  return last_launch("qed_gather_push");
}

lpic_status lpic_qed_photon_push(const lpic_grid* grid, const lpic_fields* fields,
                                 int32_t order, const lpic_qed_buffer* photons,
                                 const lpic_qed_tables* tables, const lpic_qed_params* params,
                                 const lpic_qed_buffer* pairs, lpic_precision prec,
                                 hipStream_t stream) {
  CHK(check_grid(grid, prec));
  CHK(check_fields(fields, false));
  CHK(check_qed_params(params));
  CHK(check_qed_buffer(photons, grid->ndim, "photon"));
  CHK(check_qed_buffer(pairs, grid->ndim, "pair"));
  if (order != 1 && order != 2) return fail(LPIC_EINVAL, "shape order must be 1 or 2");
  if (!tables || !tables->dev_base) return fail(LPIC_EINVAL, "QED tables without a device copy");
  if (photons->capacity == 0) return LPIC_OK;
  RunDesc r = make_run(grid, fields, nullptr);
  QedCall q{tables->dev, params->hbar_omega, params->seed, params->step, qed_desc(pairs)};
  launch_qed_photons(r, prec, grid->ndim, order, qed_desc(photons), q, stream);
  return last_launch("qed_photon_push");
}

size_t lpic_qed_compact_ws_bytes(int64_t capacity) {
  return capacity <= 0 ? 0 : sizeof(int32_t) * ((size_t)qed_compact_blocks(capacity) + 1);
}

lpic_status lpic_qed_compact(const lpic_qed_buffer* in, const lpic_qed_buffer* out, int32_t ndim,
                             void* ws, size_t ws_bytes, hipStream_t stream) {
  if (ndim != 2 && ndim != 3) return fail(LPIC_EINVAL, "ndim must be 2 or 3");
  CHK(check_qed_buffer(in, ndim, "input"));
  CHK(check_qed_buffer(out, ndim, "output"));
  if (in->capacity == 0) return LPIC_OK;
  if (out->capacity < in->capacity)
    return fail(LPIC_EINVAL, "the output buffer must hold the input's capacity");
  if (in->x == out->x) return fail(LPIC_EINVAL, "compaction is out of place");
  if (!ws || ws_bytes < lpic_qed_compact_ws_bytes(in->capacity))
    return fail(LPIC_EINVAL, "ws needs %zu bytes", lpic_qed_compact_ws_bytes(in->capacity));
  launch_qed_compact(qed_desc(in), qed_desc(out), (int32_t*)ws, stream);
  return last_launch("qed_compact");
}

lpic_status lpic_qed_insert(const lpic_grid* grid, const lpic_species* sp, int64_t first,
                            const lpic_qed_buffer* records, int32_t parity, int32_t* dropped,
                            lpic_precision prec, hipStream_t stream) {
  CHK(check_grid(grid, prec));
  CHK(check_species(sp, grid->ndim, prec));
  CHK(check_qed_buffer(records, grid->ndim, "record"));
  if (parity < -1 || parity > 1) return fail(LPIC_EINVAL, "parity must be -1, 0 or 1");
  if (first < 0) return fail(LPIC_EINVAL, "first must be >= 0");
  if (records->capacity == 0 || sp->n == 0) return LPIC_OK;
  RunDesc r = make_run(grid, nullptr, nullptr);
  SegDesc s = make_seg(sp, nullptr, 0, nullptr, 0, 0, prec);
  Tables T = single_tables(r, &s);
  launch_qed_insert(T, prec, grid->ndim, first, qed_desc(records), parity, dropped, stream);
  return last_launch("qed_insert");
}

int64_t lpic_num_tiles(const lpic_grid* grid, const lpic_tiling* tiling) {
  if (!grid || !tiling || tiling->tx <= 0 || tiling->ty <= 0) return -1;
  lpic_tiling t = *tiling;
  if (grid->ndim != 3) t.tz = 1;
  int a, b, c;
  tile_counts(grid, &t, a, b, c);
  return (int64_t)a * b * c;
}

size_t lpic_sort_ws_bytes(const lpic_grid* grid, const lpic_tiling* tiling, int64_t n) {
  (void)n;
  const int64_t nt = lpic_num_tiles(grid, tiling);
  if (nt < 0) return 0;
  return 3 * align256((size_t)(nt + 1) * 4);   // counts, cursor, placement multipliers
}

lpic_status lpic_sort_tiles(const lpic_grid* grid, lpic_species* sp, lpic_species* alt,
                            const lpic_tiling* tiling, int32_t* tile_offsets, void* ws,
                            size_t ws_bytes, lpic_precision prec, hipStream_t stream) {
  CHK(check_grid(grid, prec));
  CHK(check_species(sp, grid->ndim, prec));
  CHK(check_species(alt, grid->ndim, prec));
  CHK(check_tiling(tiling, grid, prec, false));
  if (alt->n != sp->n) return fail(LPIC_EINVAL, "alt must have as many slots as sp");
  if (!tile_offsets) return fail(LPIC_EINVAL, "tile_offsets is NULL");
  const size_t need = lpic_sort_ws_bytes(grid, tiling, sp->n);
  if (!ws || ws_bytes < need) return fail(LPIC_EINVAL, "sort workspace needs %zu bytes", need);
  lpic_tiling t = *tiling;
  if (grid->ndim != 3) t.tz = 1;
  RunDesc r = make_run(grid, nullptr, &t);
  const int nbins = r.ntiles + 1;
  int32_t* counts = (int32_t*)ws;
  int32_t* cursor = (int32_t*)((char*)ws + align256((size_t)nbins * 4));
  int32_t* mult = (int32_t*)((char*)ws + 2 * align256((size_t)nbins * 4));
  if (sp->n > 0) {
    SegDesc s = make_seg(sp, alt, 0, &t, 0, 0, prec);
    Tables T = single_tables(r, &s);
    launch_zero_u32((uint32_t*)counts, nbins, stream);
    CHK(last_launch("sort clear"));
    launch_sort(T, prec, grid->ndim, (int)((sp->n + SORT_BLOCK - 1) / SORT_BLOCK), counts,
                tile_offsets, cursor, mult, nbins, (t.flags & LPIC_SORT_SPREAD) ? 1 : 0, stream);
    CHK(last_launch("sort"));
  } else {
    launch_zero_u32((uint32_t*)tile_offsets, nbins + 1, stream);
    return last_launch("sort clear");
  }
  void* a[P_NUM];
  void* b[P_NUM];
  species_ptrs(sp, prec, a);
  species_ptrs(alt, prec, b);
  set_species_ptrs(sp, prec, b);
  set_species_ptrs(alt, prec, a);
  return LPIC_OK;
}

}  // extern "C"

// =======================================================================================
// Tile sort without allocation: the bin counts, cursors and placement multipliers live in a
// file-scope device array instead of a caller workspace.
// =======================================================================================
namespace {

constexpr size_t STATIC_SORT_ARRAY = (size_t)LPIC_SORT_STATIC_MAX_TILES + 64;   // words
__device__ __align__(256) int32_t scratch[3 * STATIC_SORT_ARRAY];

// Device address of `scratch` on each device, looked up once per device with that device
// current (in host code the symbol's name is only a stand-in for it).
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_ptr[MAX_DEVICES] = {};

lpic_status static_scratch(int32_t** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES)
    return fail(LPIC_EUNSUPPORTED, "device %d beyond the %d the library tracks", dev, MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(LPIC_EHIP, "no device address for the sort scratch array");
    g_scratch_ptr[dev] = (int32_t*)p;
  }
  *out = g_scratch_ptr[dev];
  return LPIC_OK;
}

}  // namespace

extern "C" {

lpic_status lpic_sort_tiles_static(const lpic_grid* grid, lpic_species* sp, lpic_species* alt,
                                   const lpic_tiling* tiling, int32_t* tile_offsets,
                                   lpic_precision prec, hipStream_t stream) {
  CHK(check_grid(grid, prec));
  CHK(check_species(sp, grid->ndim, prec));
  CHK(check_species(alt, grid->ndim, prec));
  CHK(check_tiling(tiling, grid, prec, false));
  if (alt->n != sp->n) return fail(LPIC_EINVAL, "alt must have as many slots as sp");
  if (!tile_offsets) return fail(LPIC_EINVAL, "tile_offsets is NULL");
  const int64_t nt = lpic_num_tiles(grid, tiling);
  if (nt < 1 || nt > LPIC_SORT_STATIC_MAX_TILES)
    return fail(LPIC_EINVAL, "%lld tiles: lpic_sort_tiles_static handles at most %d",
                (long long)nt, LPIC_SORT_STATIC_MAX_TILES);
  int32_t* base = nullptr;
  CHK(static_scratch(&base));
  lpic_tiling t = *tiling;
  if (grid->ndim != 3) t.tz = 1;
  RunDesc r = make_run(grid, nullptr, &t);
  const int nbins = r.ntiles + 1;
  int32_t* counts = base;
  int32_t* cursor = base + STATIC_SORT_ARRAY;
  int32_t* mult = base + 2 * STATIC_SORT_ARRAY;
  if (sp->n > 0) {
    SegDesc s = make_seg(sp, alt, 0, &t, 0, 0, prec);
    Tables T = single_tables(r, &s);
    // the array keeps whatever the last call left: the counts start from zero (a fill
    // kernel, no memset node)
    launch_zero_u32((uint32_t*)counts, nbins, stream);
    CHK(last_launch("static sort clear"));
    launch_sort(T, prec, grid->ndim, (int)((sp->n + SORT_BLOCK - 1) / SORT_BLOCK), counts,
                tile_offsets, cursor, mult, nbins, (t.flags & LPIC_SORT_SPREAD) ? 1 : 0, stream);
    CHK(last_launch("static sort"));
  } else {
    launch_zero_u32((uint32_t*)tile_offsets, nbins + 1, stream);
    return last_launch("static sort clear");
  }
  void* a[P_NUM];
  void* b[P_NUM];
  species_ptrs(sp, prec, a);
  species_ptrs(alt, prec, b);
  set_species_ptrs(sp, prec, b);
  set_species_ptrs(alt, prec, a);
  return LPIC_OK;
}

size_t lpic_fused_ws_bytes(const lpic_grid* grid, const lpic_tiling* tiling, int64_t n) {
  if (!tiling || tiling->chunk < 1) return 0;
  const int64_t nt = lpic_num_tiles(grid, tiling);
  if (nt < 0) return 0;
  // chunk count, escape counters and total, fixed-point shift; chunk table; escape list;
  // weight maxima
  return 256 + align256((size_t)max_chunks_of(nt, n, tiling->chunk) * sizeof(Chunk)) +
         align256((size_t)std::max<int64_t>(n, 1) * 8) + (size_t)fixed_shift_slots() * 8;
}

lpic_status lpic_push_deposit_fused(const lpic_grid* grid, const lpic_fields* fields,
                                    const lpic_species* sp, const lpic_tiling* tiling,
                                    const int32_t* tile_offsets, void* ws, size_t ws_bytes,
                                    int32_t with_rho, double* kinetic, lpic_precision prec,
                                    hipStream_t stream) {
  CHK(check_grid(grid, prec));
  if (with_rho != 0 && with_rho != 1) return fail(LPIC_EINVAL, "with_rho must be 0 or 1");
  CHK(check_fields(fields, with_rho != 0));
  CHK(check_species(sp, grid->ndim, prec));
  CHK(check_tiling(tiling, grid, prec));
  if (!tile_offsets) return fail(LPIC_EINVAL, "tile_offsets is NULL");
  if (sp->n == 0) return LPIC_OK;
  const size_t need = lpic_fused_ws_bytes(grid, tiling, sp->n);
  if (!ws || ws_bytes < need) return fail(LPIC_EINVAL, "fused workspace needs %zu bytes", need);
  lpic_tiling t = *tiling;
  if (grid->ndim != 3) t.tz = 1;
  RunDesc r = make_run(grid, fields, &t);
  SegDesc s = make_seg(sp, nullptr, 0, &t, 0, 0, prec);
  Tables T = single_tables(r, &s);
  const int64_t maxch = max_chunks_of(r.ntiles, sp->n, t.chunk);
  int32_t* nchunks = (int32_t*)ws;
  EscapeList esc;
  esc.count = (unsigned int*)((char*)ws + 64);
  esc.total = (unsigned long long*)((char*)ws + 128);
  Chunk* chunks = (Chunk*)((char*)ws + 256);
  esc.items = (unsigned long long*)((char*)chunks + align256((size_t)maxch * sizeof(Chunk)));
  esc.capacity = sp->n;
  int32_t* jshift = (int32_t*)((char*)ws + 192);
  unsigned long long* wmax = (unsigned long long*)((char*)esc.items + align256((size_t)sp->n * 8));
  launch_zero_u32((uint32_t*)ws, 64, stream);   // chunk count, escape counters
  CHK(last_launch("fused clear"));
  launch_zero_u32((uint32_t*)wmax, 2 * (int64_t)fixed_shift_slots(), stream);
  CHK(last_launch("weight max clear"));
  launch_fixed_shift(T, prec, grid->ndim, (int)((sp->n + SORT_BLOCK - 1) / SORT_BLOCK), 1, 1,
                     wmax, jshift, stream);
  CHK(last_launch("fixed-point shift"));
  launch_build_chunks(T, tile_offsets, r.ntiles, t.chunk, chunks, nchunks, stream);
  CHK(last_launch("build chunks"));
  const size_t smem = fused_smem_bytes(prec, grid->ndim, t.tx, t.ty, t.tz, t.halo, with_rho);
  const int geo = fused_geometry(grid->ndim, t.tx, t.ty, t.tz, t.halo);
  int bpc = 1;
  HIPCHK(prepare_fused(prec, grid->ndim, geo, smem, smem, &bpc));
  launch_fused(T, prec, grid->ndim, geo, fused_grid(maxch, bpc), smem, chunks, nchunks, with_rho,
               kinetic, 0, esc, jshift, stream);
  return last_launch("fused");
}

lpic_status lpic_load_positions(const lpic_grid* grid, const lpic_species* sp, const double* x,
                                const double* y, const double* z, lpic_precision prec,
                                hipStream_t stream) {
  CHK(check_grid(grid, prec));
  CHK(check_species(sp, grid->ndim, prec));
  if (sp->n == 0) return LPIC_OK;
  if (!x || !y || (grid->ndim == 3 && !z)) return fail(LPIC_EINVAL, "source arrays are NULL");
  RunDesc r = make_run(grid, nullptr, nullptr);
  SegDesc s = make_seg(sp, nullptr, 0, nullptr, 0, 0, prec);
  Tables T = single_tables(r, &s);
  launch_load_positions(T, prec, grid->ndim, (int)((sp->n + 255) / 256), x, y, z, stream);
  return last_launch("load positions");
}

lpic_status lpic_store_positions(const lpic_grid* grid, const lpic_species* sp, double* x,
                                 double* y, double* z, lpic_precision prec, hipStream_t stream) {
  CHK(check_grid(grid, prec));
  CHK(check_species(sp, grid->ndim, prec));
  if (sp->n == 0) return LPIC_OK;
  if (!x || !y || (grid->ndim == 3 && !z)) return fail(LPIC_EINVAL, "destination arrays are NULL");
  RunDesc r = make_run(grid, nullptr, nullptr);
  SegDesc s = make_seg(sp, nullptr, 0, nullptr, 0, 0, prec);
  Tables T = single_tables(r, &s);
  launch_store_positions(T, prec, grid->ndim, (int)((sp->n + 255) / 256), x, y, z, stream);
  return last_launch("store positions");
}

lpic_status lpic_reduce_fields(const lpic_grid* grid, const lpic_fields* fields,
                               int32_t with_rho, double* out, lpic_precision prec,
                               hipStream_t stream) {
  CHK(check_grid(grid, prec));
  CHK(check_fields(fields, with_rho != 0));
  if (!out) return fail(LPIC_EINVAL, "out is NULL");
  RunDesc r = make_run(grid, fields, nullptr);
  Tables T = single_tables(r, nullptr);
  launch_zero_doubles(out, 4, stream);
  CHK(last_launch("reduce clear"));
  launch_reduce_fields(T, prec, grid->ndim, (int)((ncells(grid) + 255) / 256), with_rho, out,
                       stream);
  return last_launch("reduce");
}

}  // extern "C"

// =======================================================================================
// Simulation object: Algorithm 1 over one box or an ensemble of boxes
// =======================================================================================
struct HookEntry {
  lpic_hook_fn fn;
  void* user;
};

struct lpic_sim {
  int prec = 0, ndim = 2, nruns = 0, nsegs = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  std::vector<lpic_grid> grids;
  std::vector<lpic_fields> fields;
  std::vector<lpic_species> sp, alt;          // host mirrors, current buffer in sp
  std::vector<int32_t> species_run;
  std::vector<RunDesc> runs_h;
  std::vector<SegDesc> segs_h;
  lpic_options opt{};
  // device tables and scratch
  RunDesc* runs_d = nullptr;
  SegDesc* segs_d = nullptr;
  int32_t* run_blk_d = nullptr;
  int32_t* seg_blk256_d = nullptr;
  int32_t* seg_blk_sort_d = nullptr;
  int nblk_cells = 0, nblk_p256 = 0, nblk_sort = 0;
  int32_t *counts = nullptr, *offsets = nullptr, *cursor = nullptr, *mult = nullptr;
  int nbins = 0;
  int nvirt = 0;                             // (tile, species) slots of the chunk order
  Chunk* chunks = nullptr;
  int32_t* nchunks = nullptr;
  int32_t* scan_part = nullptr;     // scratch of the many-workgroup scans
  int64_t max_chunks = 0;
  size_t smem = 0, smem_rho = 0;
  int geo = 0;
  int geo_rho = 0;                  // the geometry of diagnostic steps (charge planes)
  // Chained charge (3D FP32 with 8 x 4 x 4 tiles and halo 3): the step before a
  // diagnostic step accumulates the charge at the ends of its paths into rho0, leaving out
  // the particles that leave the box, and the diagnostic step only the charge at the ends of
  // its own paths, into rho1.  A path ends half a step past the stored position
  // (x^n + (dt/2) v^n) and the next step's path starts at the same point, so rho0 of the
  // diagnostic step is that charge; each of the two steps then carries one charge plane
  // instead of two on one step, which keeps the occupancy of the other steps (3D FP32 on an
  // unpadded geometry: two workgroups per CU).
  bool chain = false;
  int geo_chain = 0;
  size_t smem_chain = 0;
  int blocks_per_cu_chain = 1;
  double* diag = nullptr;
  unsigned long long* escapes = nullptr;     // cumulative escape count
  unsigned int* esc_count = nullptr;         // per-step escape counters
  unsigned long long* esc_items = nullptr;   // escape list (capacity: all particles)
  unsigned long long* wmax = nullptr;        // per segment: max |w| (FP64 bits)
  std::vector<int> has_laser;                // per run
  std::vector<LaserDesc> lasers;             // per run
  // convolutional PML per run (cells = 0: none) and its auxiliary values (2 halves)
  std::vector<lpic_pml> pmls;
  std::vector<void*> psi;
  // moving windows: per run the origin column and the total shift; per segment the fresh
  // particles written since the last sort; `windows` once any window has moved
  std::vector<int32_t> x0;
  std::vector<int64_t> shifted;
  std::vector<int64_t> inject_used;
  bool windows = false;
  bool offsets_valid = false;                // bin offsets of the current particle layout
  int laser_bpr = 0;                         // antenna kernel blocks per run (0: no laser)
  int64_t* step_dev = nullptr;               // steps taken, on the device (antenna time)
  unsigned int* laser_done = nullptr;        // workgroup counter of the antenna kernel
  int32_t* jshift = nullptr;                 // per run: fixed-point shift of FP32 currents
  int64_t esc_capacity = 0;
  // re-binned escape path (LPIC_ESCAPE_REBIN)
  Rebin rb{};
  bool rebin = false;
  unsigned long long* rb_items = nullptr;     // grouped escape list
  unsigned long long* esc2_items = nullptr;   // the second pass's own escape list
  void* esc_rec = nullptr;                    // escape records of the list, and grouped
  void* rb_rec = nullptr;
  int32_t* esc_keys = nullptr;                // the present bin of each escape-list entry
  unsigned int* esc2_count = nullptr;         // its counters (and a total)
  int blocks_per_cu = 1;       // fused workgroups resident per CU (without / with charge planes)
  int blocks_per_cu_rho = 1;
  // fused 2D field update between steps (launch_yee_mid); mid_tx == 0: not in use
  int mid_tx = 0, mid_ty = 0, mid_ntiles = 0;
  int32_t* mid_pfx_d = nullptr;              // nruns + 1 prefix of field tiles
  void* bands = nullptr;                     // two edge snapshots
  int64_t band_half = 0;                     // values per snapshot
  void* old_state = nullptr;
  std::vector<size_t> old_off;
  std::vector<HookEntry> hooks[LPIC_NUM_STAGES];
  // progress
  int64_t step = 0, sorts = 0, diag_step = -1;
  bool need_sort = true;
  bool need_spread = true;   // the first sort after particles are loaded spreads tiles
  // captured steps keyed by (charge mode, sort, diagnostics, first field updates already
  // done by the previous step, last field updates merged into the next step's)
  static constexpr int NGRAPHS = 64;
  hipGraphExec_t gexec[NGRAPHS] = {};
  // timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending, ev_free;
  double fused_ms = 0.0;
  int64_t fused_launches = 0;
  bool last_fused = false, last_graph = false;
};

namespace {

void free_dev(void* p) {
  if (p) (void)hipFree(p);
}

void drop_graphs(lpic_sim* s) {
  for (int i = 0; i < lpic_sim::NGRAPHS; ++i) {
    if (s->gexec[i]) (void)hipGraphExecDestroy(s->gexec[i]);
    s->gexec[i] = nullptr;
  }
}

bool intermediate_hooks(const lpic_sim* s) {
  for (int st = LPIC_STAGE_PUSH_POSITION_1; st <= LPIC_STAGE_PUSH_POSITION_2; ++st)
    if (!s->hooks[st].empty()) return true;
  return false;
}

bool any_hooks(const lpic_sim* s) {
  for (const auto& v : s->hooks)
    if (!v.empty()) return true;
  return false;
}

bool inner_hooks(const lpic_sim* s) {
  for (int st = LPIC_STAGE_MAXWELL_1; st <= LPIC_STAGE_MAXWELL_2; ++st)
    if (!s->hooks[st].empty()) return true;
  return false;
}

Tables sim_tables(const lpic_sim* s, const int32_t* seg_blk) {
  Tables T;
  memset(&T, 0, sizeof(T));
  T.runs = s->runs_d;
  T.segs = s->segs_d;
  T.run_blk = s->run_blk_d;
  T.seg_blk = seg_blk;
  T.nruns = s->nruns;
  T.nsegs = s->nsegs;
  return T;
}

lpic_status run_hooks(lpic_sim* s, int stage) {
  for (auto& h : s->hooks[stage]) {
    const int rc = h.fn(s, stage, s->step, h.user);
    if (rc != 0) return fail(LPIC_EHOOK, "hook at stage %d returned %d at step %lld", stage, rc,
                             (long long)s->step);
  }
  return LPIC_OK;
}

// (Re)build everything that depends on the options: tiling, bins, chunk tables.
// Bytes of the two halves of a run's PML auxiliary values (the coefficient table follows).
size_t pml_psi_bytes(const lpic_grid* g, int cells, int prec) {
  return (size_t)2 * 4 * g->ny * (g->ndim == 3 ? g->nz : 1) * 2 * cells *
         (prec == LPIC_F32_CELLOFS ? 4 : 8);
}

size_t lds_of_geometry(const lpic_sim* s, int g);

lpic_status configure(lpic_sim* s) {
  drop_graphs(s);
  lpic_tiling t = s->opt.tiling;
  if (s->ndim != 3) t.tz = 1;
  for (int r = 0; r < s->nruns; ++r) {
    CHK(check_tiling(&t, &s->grids[r], s->prec));
    CHK(check_fields(&s->fields[r], s->opt.diag_interval > 0));
  }
  if (s->opt.sort_interval < 1) return fail(LPIC_EINVAL, "sort_interval must be >= 1");
  if (s->opt.diag_interval < 0) return fail(LPIC_EINVAL, "diag_interval must be >= 0");
  // runs
  s->runs_h.clear();
  std::vector<int32_t> run_blk(1, 0);
  s->has_laser.resize(s->nruns, 0);
  s->lasers.resize(s->nruns);
  s->pmls.resize(s->nruns, lpic_pml{});
  s->psi.resize(s->nruns, nullptr);
  if (!s->step_dev) {
    if (hipMalloc((void**)&s->step_dev, 256) != hipSuccess)
      return fail(LPIC_ENOMEM, "device allocation of 256 bytes failed");
    s->laser_done = (unsigned int*)((char*)s->step_dev + 64);
    HIPCHK(hipMemset(s->step_dev, 0, 256));
  }
  s->x0.resize(s->nruns, 0);
  s->shifted.resize(s->nruns, 0);
  s->inject_used.resize(std::max(1, s->nsegs), 0);
  s->laser_bpr = 0;
  for (int r = 0; r < s->nruns; ++r) {
    RunDesc d = make_run(&s->grids[r], &s->fields[r], &t);
    d.diag = s->diag + (size_t)r * DIAG_NUM;
    d.has_laser = s->has_laser[r];
    d.laser = s->lasers[r];
    d.x0 = s->x0[r];
    const lpic_pml& pm = s->pmls[r];
    if (pm.cells > 0) {
      d.pml_cells = pm.cells;
      d.psi = s->psi[r];
      d.pml_tab = (const char*)s->psi[r] + pml_psi_bytes(&s->grids[r], pm.cells, s->prec);
      d.psi_parity = (const int32_t*)((char*)s->step_dev + 128);
    }
    if (d.has_laser) s->laser_bpr = std::max(s->laser_bpr, columns_bpr(&s->grids[r]));
    s->runs_h.push_back(d);
    run_blk.push_back(run_blk.back() + (int32_t)((ncells(&s->grids[r]) + 255) / 256));
  }
  // segments (current buffers first)
  s->segs_h.clear();
  std::vector<int32_t> blk256(1, 0), blks(1, 0);
  int bin = 0;
  int64_t pbase = 0, maxch = 0;
  for (int i = 0; i < s->nsegs; ++i) {
    const int r = s->species_run[i];
    SegDesc d = make_seg(&s->sp[i], &s->alt[i], r, &t, bin, pbase, s->prec);
    s->segs_h.push_back(d);
    bin += s->runs_h[r].ntiles + 1;
    pbase += s->sp[i].n;
    maxch += max_chunks_of(s->runs_h[r].ntiles, s->sp[i].n, t.chunk);
    blk256.push_back(blk256.back() + (int32_t)((s->sp[i].n + 255) / 256));
    blks.push_back(blks.back() + (int32_t)((s->sp[i].n + SORT_BLOCK - 1) / SORT_BLOCK));
  }
  if (pbase >= ((int64_t)1 << 31) - 1) return fail(LPIC_EINVAL, "too many particles in total");
  // chunk order: run by run, tile by tile, the run's species one after the other, so that
  // the chunks of all species of one tile are consecutive (one staging of the tile)
  s->nvirt = 0;
  for (int r = 0; r < s->nruns; ++r) {
    RunDesc& d = s->runs_h[r];
    d.seg_first = 0;
    d.nseg = 0;
    for (int i = 0; i < s->nsegs; ++i)
      if (s->species_run[i] == r) {
        if (d.nseg == 0) d.seg_first = i;
        ++d.nseg;
      }
    d.vbase = s->nvirt;
    s->nvirt += d.ntiles * d.nseg;
  }
  s->nblk_cells = run_blk.back();
  s->nblk_p256 = blk256.back();
  s->nblk_sort = blks.back();
  s->nbins = bin;
  s->max_chunks = maxch;
  // device tables
  free_dev(s->runs_d); free_dev(s->segs_d); free_dev(s->run_blk_d);
  free_dev(s->seg_blk256_d); free_dev(s->seg_blk_sort_d);
  free_dev(s->counts); free_dev(s->offsets); free_dev(s->cursor); free_dev(s->mult);
  free_dev(s->chunks); free_dev(s->scan_part);
  free_dev(s->rb.counts); free_dev(s->rb.offsets); free_dev(s->rb.cursor);
  free_dev(s->rb.chunks); free_dev(s->rb.nchunks);
  s->rb = Rebin{};
  s->rebin = false;
  s->mult = nullptr;
  s->runs_d = nullptr; s->segs_d = nullptr; s->run_blk_d = nullptr;
  s->seg_blk256_d = s->seg_blk_sort_d = nullptr;
  s->counts = s->offsets = s->cursor = nullptr;
  s->chunks = nullptr;
#define ALLOC(ptr, bytes)                                                            \
  do {                                                                               \
    if (hipMalloc((void**)&(ptr), std::max<size_t>(bytes, 256)) != hipSuccess)        \
      return fail(LPIC_ENOMEM, "device allocation of %zu bytes failed", (size_t)(bytes)); \
  } while (0)
  ALLOC(s->runs_d, sizeof(RunDesc) * s->nruns);
  ALLOC(s->segs_d, sizeof(SegDesc) * std::max(1, s->nsegs));
  ALLOC(s->run_blk_d, sizeof(int32_t) * run_blk.size());
  ALLOC(s->seg_blk256_d, sizeof(int32_t) * blk256.size());
  ALLOC(s->seg_blk_sort_d, sizeof(int32_t) * blks.size());
  ALLOC(s->counts, sizeof(int32_t) * (s->nbins + 1));
  ALLOC(s->offsets, sizeof(int32_t) * (s->nbins + 1));
  ALLOC(s->cursor, sizeof(int32_t) * (s->nbins + 1));
  ALLOC(s->mult, sizeof(int32_t) * (s->nbins + 1));
  ALLOC(s->chunks, sizeof(Chunk) * std::max<int64_t>(1, maxch));
  ALLOC(s->scan_part, sizeof(int32_t) * part_words(std::max(s->nbins, s->nvirt)));
  HIPCHK(hipMemcpy(s->runs_d, s->runs_h.data(), sizeof(RunDesc) * s->nruns, hipMemcpyHostToDevice));
  if (s->nsegs)
    HIPCHK(hipMemcpy(s->segs_d, s->segs_h.data(), sizeof(SegDesc) * s->nsegs, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s->run_blk_d, run_blk.data(), sizeof(int32_t) * run_blk.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s->seg_blk256_d, blk256.data(), sizeof(int32_t) * blk256.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s->seg_blk_sort_d, blks.data(), sizeof(int32_t) * blks.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemset(s->counts, 0, sizeof(int32_t) * (s->nbins + 1)));
  HIPCHK(hipMemset(s->nchunks, 0, sizeof(int32_t)));
  s->smem = fused_smem_bytes(s->prec, s->ndim, t.tx, t.ty, t.tz, t.halo, 0);
  s->geo = fused_geometry(s->ndim, t.tx, t.ty, t.tz, t.halo);
  // FP32 8 x 4 x 4 tiles with halo 3: the charge planes of diagnostic steps leave one
  // workgroup per CU, which then runs 1024 threads (geometry 9) instead of 512
  s->geo_rho = (s->prec == LPIC_F32_CELLOFS && s->geo == 7) ? 9 : s->geo;
  s->smem_rho = fused_smem_bytes(s->prec, s->ndim, t.tx, t.ty, t.tz, t.halo, 1, s->geo_rho);
  {
    // (FP32 only: FP64 positions are absolute, and the start of the next step's path,
    // found again from the stored position, rounds at the scale of the box length -- about
    // 1e-11 of a cell in a box of 65536 cells, above the FP64 continuity that the two planes
    // of one step keep.  3D only: in 2D both planes cost one workgroup of four per CU, and
    // the chained 2D steps measured no faster.)
    const bool f32_3d = s->prec == LPIC_F32_CELLOFS && s->ndim == 3;
    s->chain = f32_3d && s->geo == 7;
    s->geo_chain = f32_3d && s->geo == 7 ? 8 : s->geo;
    s->smem_chain = fused_smem_bytes(s->prec, s->ndim, t.tx, t.ty, t.tz, t.halo, 2,
                                     s->geo_chain);
  }
  HIPCHK(prepare_fused(s->prec, s->ndim, s->geo_rho, lds_of_geometry(s, s->geo_rho),
                       s->smem_rho, &s->blocks_per_cu_rho));
  HIPCHK(prepare_fused(s->prec, s->ndim, s->geo, lds_of_geometry(s, s->geo), s->smem,
                       &s->blocks_per_cu));
  if (s->chain)
    HIPCHK(prepare_fused(s->prec, s->ndim, s->geo_chain, lds_of_geometry(s, s->geo_chain),
                         s->smem_chain, &s->blocks_per_cu_chain));
  HIPCHK(hipMemcpy(s->step_dev, &s->step, sizeof(int64_t), hipMemcpyHostToDevice));
  // fused 2D field update between steps: the largest field tile dividing every box
  free_dev(s->mid_pfx_d);
  free_dev(s->bands);
  s->mid_pfx_d = nullptr;
  s->bands = nullptr;
  s->mid_tx = s->mid_ty = s->mid_ntiles = 0;
  s->band_half = 0;
  if (s->ndim == 2 && !(t.flags & LPIC_FIELD_SEPARATE) && !s->windows) {
    int tx = MID_MAX_TX, ty = MID_MAX_TY;
    for (int r = 0; r < s->nruns; ++r) {
      while (tx >= 8 && s->grids[r].nx % tx) tx >>= 1;
      while (ty >= 4 && s->grids[r].ny % ty) ty >>= 1;
    }
    if (tx >= 8 && ty >= 4) {
      std::vector<int32_t> pfx(1, 0);
      for (int r = 0; r < s->nruns; ++r)
        pfx.push_back(pfx.back() + (s->grids[r].nx / tx) * (s->grids[r].ny / ty));
      s->band_half = (int64_t)pfx.back() * band_values_per_tile(tx, ty);
      ALLOC(s->mid_pfx_d, sizeof(int32_t) * pfx.size());
      ALLOC(s->bands, 2 * (size_t)s->band_half * (s->prec == LPIC_F32_CELLOFS ? 4 : 8));
      HIPCHK(hipMemcpy(s->mid_pfx_d, pfx.data(), sizeof(int32_t) * pfx.size(),
                       hipMemcpyHostToDevice));
      s->mid_tx = tx;
      s->mid_ty = ty;
      s->mid_ntiles = pfx.back();
    }
  }
  if (!s->wmax) {
    ALLOC(s->wmax, sizeof(unsigned long long) * fixed_shift_slots() * std::max(1, s->nsegs));
    ALLOC(s->jshift, sizeof(int32_t) * std::max(1, s->nruns));
  }
  if (!s->esc_items) {
    s->esc_capacity = std::max<int64_t>(pbase, 1);
    ALLOC(s->esc_items, sizeof(unsigned long long) * s->esc_capacity);
    ALLOC(s->esc_count, 256);
    HIPCHK(hipMemset(s->esc_count, 0, 256));
  }
  if (t.flags & LPIC_ESCAPE_REBIN) {
    if (!s->rb_items) {
      ALLOC(s->rb_items, sizeof(unsigned long long) * s->esc_capacity);
      ALLOC(s->esc2_items, sizeof(unsigned long long) * s->esc_capacity);
      // escape records (3D): 8 values of the kernel precision per entry
      if (s->ndim == 3) {
        const size_t rec = 8 * (s->prec == LPIC_F32_CELLOFS ? 4 : 8);
        ALLOC(s->esc_rec, rec * s->esc_capacity);
        ALLOC(s->rb_rec, rec * s->esc_capacity);
        if (s->prec == LPIC_F32_CELLOFS) ALLOC(s->esc_keys, sizeof(int32_t) * s->esc_capacity);
      }
      ALLOC(s->esc2_count, 256);
      HIPCHK(hipMemset(s->esc2_count, 0, 256));
    }
    Rebin& rb = s->rb;
    ALLOC(rb.counts, sizeof(int32_t) * (s->nbins + 1));
    ALLOC(rb.offsets, sizeof(int32_t) * (s->nbins + 1));
    ALLOC(rb.cursor, sizeof(int32_t) * (s->nbins + 1));
    ALLOC(rb.chunks, sizeof(Chunk) * std::max<int64_t>(1, maxch));
    ALLOC(rb.nchunks, 256);
    HIPCHK(hipMemset(rb.counts, 0, sizeof(int32_t) * (s->nbins + 1)));
    HIPCHK(hipMemset(rb.nchunks, 0, 256));
    rb.threshold = REBIN_THRESHOLD;
    rb.nbins = s->nbins;
    rb.nvirt = s->nvirt;
    rb.part = s->scan_part;
    rb.chunk = t.chunk;
    rb.count_blocks = (int)std::min<int64_t>(2048, (s->esc_capacity + 2047) / 2048);
    rb.items = s->rb_items;
    rb.rec = s->rb_rec;
    rb.esc2.items = s->esc2_items;
    rb.esc2.count = s->esc2_count;
    rb.esc2.total = (unsigned long long*)((char*)s->esc2_count + 64);
    rb.esc2.capacity = s->esc_capacity;
    // second pass: the re-binned particles lie inside their present tile, so a 3D FP32
    // 8 x 4 x 4 tiling with halo 4 runs it on the halo-3 geometry, two workgroups per CU
    const bool small = s->prec == LPIC_F32_CELLOFS && s->ndim == 3 && s->geo == 5;
    rb.geo[0] = small ? fused_geometry(3, 8, 4, 4, 3) : s->geo;
    rb.geo[1] = small ? 9 : s->geo_rho;
    rb.smem[0] = small ? fused_smem_bytes(s->prec, 3, 8, 4, 4, 3, 0) : s->smem;
    rb.smem[1] = small ? fused_smem_bytes(s->prec, 3, 8, 4, 4, 3, 1, 9) : s->smem_rho;
    // (the chained-charge steps' second pass: one charge plane, as their first pass)
    rb.geo[2] = s->chain ? s->geo_chain : rb.geo[1];
    rb.smem[2] = s->chain ? s->smem_chain : rb.smem[1];
    int bpc[3] = {1, 1, 1};
    for (int k = 0; k < 3; ++k)
      HIPCHK(prepare_fused(s->prec, s->ndim, rb.geo[k], lds_of_geometry(s, rb.geo[k]),
                           rb.smem[k], &bpc[k]));
    rb.grid[0] = fused_grid(maxch, bpc[0]);
    rb.grid[1] = fused_grid(maxch, bpc[1]);
    rb.grid[2] = fused_grid(maxch, bpc[2]);
    s->rebin = true;
  }
  s->need_sort = true;
  s->offsets_valid = false;
  return LPIC_OK;
#undef ALLOC
}

void swap_host_buffers(lpic_sim* s) {
  for (int i = 0; i < s->nsegs; ++i) {
    std::swap(s->sp[i], s->alt[i]);
    for (int q = 0; q < P_NUM; ++q) std::swap(s->segs_h[i].p[q], s->segs_h[i].alt[q]);
  }
}

// Fixed-point shift of the FP32 current accumulators from the present weights.  Weights
// change only through the caller (between lpic_step calls or in hooks), so this runs at
// the start of every lpic_step call and, when hooks are registered, in every step.
lpic_status enqueue_fixed_shift(lpic_sim* s, hipStream_t st) {
  if (s->nsegs == 0 || s->prec != LPIC_F32_CELLOFS) return LPIC_OK;
  launch_zero_u32((uint32_t*)s->wmax, 2 * (int64_t)fixed_shift_slots() * s->nsegs, st);
  CHK(last_launch("weight max clear"));
  launch_fixed_shift(sim_tables(s, s->seg_blk_sort_d), s->prec, s->ndim, s->nblk_sort, s->nruns,
                     s->nsegs, s->wmax, s->jshift, st);
  return last_launch("fixed-point shift");
}

int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// The edge snapshots of the fused 2D field update; the parity word sits in the device step
// block.
FieldBands sim_bands(const lpic_sim* s) {
  FieldBands b;
  memset(&b, 0, sizeof(b));
  b.base = s->bands;
  b.half = s->band_half;
  b.tile_pfx = s->mid_pfx_d;
  b.parity = (int32_t*)((char*)s->step_dev + 128);
  b.step = s->laser_bpr > 0 ? s->step_dev : nullptr;
  b.tx = s->mid_tx;
  b.ty = s->mid_ty;
  b.lx = log2i(s->mid_tx);
  b.ly = log2i(s->mid_ty);
  return b;
}

// The device work of one step between the LOOP_START and LOOP_END hooks.  With hooks at the
// inner stages the host runs them in between (eager mode only).
// first_full: the previous step deferred its last E half (skip_last), so this step's first
// E update covers both halves at once: between them B does not change and J is the same
// array, so E + (dt/2)(curl B - J) twice is E + dt (curl B - J).  With the fused 2D field
// update the previous step already did all of it (its B half, this full E update and this
// step's first B half), and this step only clears the sources.
// rho: the charge this step accumulates (deposit's with_rho): 1 on a diagnostic step, or
// with chained charge 2 on the step before one and 3 on the diagnostic step; 0 otherwise.
lpic_status enqueue_step(lpic_sim* s, hipStream_t st, bool do_sort, bool spread, bool diag,
                         bool eager_hooks, bool capturing, bool first_full, bool skip_last,
                         int rho) {
  const Tables Tc = sim_tables(s, nullptr);
  const Tables Ts = sim_tables(s, s->seg_blk_sort_d);
  const bool mid = s->mid_tx > 0;
  const FieldBands bands = mid ? sim_bands(s) : FieldBands{};
  if (diag) {
    launch_diag_clear(Tc, s->nruns, st);
    CHK(last_launch("diag clear"));
  }
  // (the charge arrays are only written, and so only cleared, by the steps that accumulate
  // charge: both on a diagnostic step, rho0 before it and rho1 on it with chained charge)
  if (first_full && mid) {
    const int zero = rho == 1 ? 1 : (rho == 2 ? 3 : (rho == 3 ? 4 : 0));
    launch_clear_sources(Tc, s->prec, s->ndim, s->nblk_cells, zero, bands.parity,
                         s->laser_bpr > 0 ? s->step_dev : nullptr, st);
    CHK(last_launch("clear sources"));
  } else {
    // field half update t -> t + dt/2 (E first), clearing J for the deposit
    const int zero = rho == 1 ? 1 : (rho == 2 ? 3 : (rho == 3 ? 4 : 2));
    launch_yee(Tc, s->prec, s->ndim, s->nblk_cells, 0, first_full ? 1.0 : 0.5, zero,
               first_full ? 2 : 1, st);
    CHK(last_launch("yee E"));
    // a step whose last field updates go to the fused update publishes the tile edges
    launch_yee(Tc, s->prec, s->ndim, s->nblk_cells, 1, 0.5, 0, 1, st,
               (mid && skip_last) ? &bands : nullptr);
    CHK(last_launch("yee B"));
  }
  if (eager_hooks) CHK(run_hooks(s, LPIC_STAGE_MAXWELL_1));
  // sort particles (every sort_interval steps)
  if (do_sort && s->nsegs > 0) {
    launch_sort(Ts, s->prec, s->ndim, s->nblk_sort, s->counts, s->offsets, s->cursor, s->mult,
                s->nbins, spread ? 1 : 0, st, s->scan_part);
    CHK(last_launch("sort"));
    launch_swap_segments(s->segs_d, s->nsegs, st);
    CHK(last_launch("swap"));
    launch_build_chunks(Tc, s->offsets, s->nvirt, s->opt.tiling.chunk, s->chunks, s->nchunks, st,
                        s->scan_part);
    CHK(last_launch("chunks"));
    // the host mirror follows the device table at once, so that launches later in this
    // step that take descriptors by value see the sorted buffers (not while capturing: a
    // captured graph is replayed later and the caller swaps per replay)
    if (!capturing) swap_host_buffers(s);
  }
  // particle loop
  if (any_hooks(s)) CHK(enqueue_fixed_shift(s, st));
  const bool fused = !intermediate_hooks(s);
  s->last_fused = fused;
  if (s->nsegs > 0) {
    if (fused) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (s->timing) {
        if (s->ev_free.empty()) {
          HIPCHK(hipEventCreate(&e0));
          HIPCHK(hipEventCreate(&e1));
        } else {
          e0 = s->ev_free.back().first;
          e1 = s->ev_free.back().second;
          s->ev_free.pop_back();
        }
        HIPCHK(hipEventRecord(e0, st));
      }
      EscapeList esc;
      esc.items = s->esc_items;
      esc.rec = s->rebin && s->ndim == 3 ? s->esc_rec : nullptr;   // records: 3D only
      // FP32: the fused pass writes each escapee's bin (a few shifts of the packed cell),
      // so the re-binning kernels read 4 bytes per entry instead of its record
      esc.keys = esc.rec && s->prec == LPIC_F32_CELLOFS ? s->esc_keys : nullptr;
      esc.count = s->esc_count;
      esc.total = s->escapes;
      esc.capacity = s->esc_capacity;
      const int geo = rho == 0 ? s->geo : (rho == 1 ? s->geo_rho : s->geo_chain);
      const int bpc = rho == 0 ? s->blocks_per_cu
                    : (rho == 1 ? s->blocks_per_cu_rho : s->blocks_per_cu_chain);
      const size_t smem = rho == 0 ? s->smem : (rho == 1 ? s->smem_rho : s->smem_chain);
      launch_fused(Tc, s->prec, s->ndim, geo, fused_grid(s->max_chunks, bpc), smem, s->chunks,
                   s->nchunks, rho, nullptr, diag ? 1 : 0, esc, s->jshift, st,
                   s->rebin ? &s->rb : nullptr);
      CHK(last_launch("fused"));
      if (s->timing) {
        HIPCHK(hipEventRecord(e1, st));
        s->ev_pending.push_back({e0, e1});
      }
    } else {
      // split path, species by species, with the intermediate hooks in between
      char* old = (char*)s->old_state;
      for (int i = 0; i < s->nsegs; ++i) {
        const int r = s->species_run[i];
        RunDesc rd = s->runs_h[r];
        Tables T1 = single_tables(rd, &s->segs_h[i]);
        const int nb = (int)((s->sp[i].n + 255) / 256);
        if (nb == 0) continue;
        launch_gather_push(T1, s->prec, s->ndim, nb, old + s->old_off[i], st);
        CHK(last_launch("gather_push"));
        if (eager_hooks) {
          CHK(run_hooks(s, LPIC_STAGE_PUSH_POSITION_1));
          CHK(run_hooks(s, LPIC_STAGE_INTERPOLATOR));
          CHK(run_hooks(s, LPIC_STAGE_PUSH_MOMENTUM));
          CHK(run_hooks(s, LPIC_STAGE_PUSH_POSITION_2));
        }
        launch_deposit(T1, s->prec, s->ndim, nb, old + s->old_off[i], diag ? 1 : 0, st);
        CHK(last_launch("deposit"));
        if (diag) {
          launch_kinetic(T1, s->prec, s->ndim, nb, rd.diag + DIAG_UKIN, st);
          CHK(last_launch("kinetic"));
        }
      }
    }
  }
  if (s->laser_bpr > 0 && !(skip_last && mid)) {   // antenna current at t = (step + 1) dt
    // (a fused field update adds it itself)
    launch_laser(Tc, s->prec, s->ndim, s->nruns, s->laser_bpr, 0.0, s->step_dev, s->laser_done,
                 st);
    CHK(last_launch("laser"));
  }
  if (eager_hooks) {
    CHK(run_hooks(s, LPIC_STAGE_CURRENT_DEPOSITION));
    // Algorithm 1 creates photons and pairs after every species is pushed and deposited
    CHK(run_hooks(s, LPIC_STAGE_QED_CREATE));
  }
  if (skip_last && mid) {
    // this step's last field halves and the next step's first ones, fused
    Tables Tm = Tc;
    Tm.run_blk = s->mid_pfx_d;
    bool pml = false;
    for (const lpic_pml& p : s->pmls) pml = pml || p.cells > 0;
    launch_yee_mid(Tm, s->prec, s->mid_ntiles, bands, pml, st);
    CHK(last_launch("yee fused"));
  } else {
    // field half update t + dt/2 -> t + dt (B first)
    launch_yee(Tc, s->prec, s->ndim, s->nblk_cells, 1, 0.5, 0, 1, st);
    CHK(last_launch("yee B"));
    if (!skip_last) {
      launch_yee(Tc, s->prec, s->ndim, s->nblk_cells, 0, 0.5, 0, 1, st);
      CHK(last_launch("yee E"));
    }
  }
  if (eager_hooks) CHK(run_hooks(s, LPIC_STAGE_MAXWELL_2));
  if (diag) {
    launch_reduce_fields(Tc, s->prec, s->ndim, s->nblk_cells, 1, nullptr, st);
    CHK(last_launch("reduce"));
  }
  return LPIC_OK;
}

// The largest dynamic LDS that any launch of fused geometry g asks for in this simulation:
// the attribute belongs to the kernel instance, so it must cover every use of it.
size_t lds_of_geometry(const lpic_sim* s, int g) {
  size_t m = 0;
  if (g == s->geo) m = std::max(m, s->smem);
  if (g == s->geo_rho) m = std::max(m, s->smem_rho);
  if (s->chain && g == s->geo_chain) m = std::max(m, s->smem_chain);
  for (int k = 0; k < 3; ++k)
    if (s->rb.smem[k] && g == s->rb.geo[k]) m = std::max(m, s->rb.smem[k]);
  return m;
}

lpic_status ensure_old_state(lpic_sim* s) {
  if (s->old_state) return LPIC_OK;
  size_t tot = 0;
  s->old_off.clear();
  for (int i = 0; i < s->nsegs; ++i) {
    s->old_off.push_back(tot);
    tot += align256(old_state_bytes(s->ndim, s->sp[i].n, s->prec));
  }
  if (hipMalloc(&s->old_state, std::max<size_t>(tot, 256)) != hipSuccess)
    return fail(LPIC_ENOMEM, "old-state allocation of %zu bytes failed", tot);
  return LPIC_OK;
}

}  // namespace

extern "C" {

lpic_status lpic_sim_create(lpic_sim** out, int32_t nruns, const lpic_grid* grids,
                            const lpic_fields* fields, int32_t nspecies,
                            const lpic_species* species, const int32_t* species_run,
                            const lpic_species* species_alt, lpic_precision prec,
                            const lpic_options* opt, hipStream_t stream) {
  if (!out) return fail(LPIC_EINVAL, "out is NULL");
  *out = nullptr;
  if (nruns < 1 || !grids || !fields) return fail(LPIC_EINVAL, "need at least one box");
  if (nspecies < 0 || (nspecies > 0 && (!species || !species_run || !species_alt)))
    return fail(LPIC_EINVAL, "species arrays are NULL");
  if (!opt) return fail(LPIC_EINVAL, "options are NULL");
  for (int r = 0; r < nruns; ++r) {
    CHK(check_grid(&grids[r], prec));
    CHK(check_fields(&fields[r], opt->diag_interval > 0));
    if (grids[r].ndim != grids[0].ndim) return fail(LPIC_EINVAL, "all boxes must have one ndim");
  }
  for (int i = 0; i < nspecies; ++i) {
    if (species_run[i] < 0 || species_run[i] >= nruns)
      return fail(LPIC_EINVAL, "species %d names box %d", i, species_run[i]);
    if (i > 0 && species_run[i] < species_run[i - 1])
      return fail(LPIC_EINVAL, "species must be listed in box order");
    CHK(check_species(&species[i], grids[0].ndim, prec));
    CHK(check_species(&species_alt[i], grids[0].ndim, prec));
    if (species_alt[i].n != species[i].n) return fail(LPIC_EINVAL, "alt size mismatch");
  }
  lpic_sim* s = new lpic_sim();
  s->prec = prec;
  s->ndim = grids[0].ndim;
  s->nruns = nruns;
  s->nsegs = nspecies;
  s->stream = stream;
  s->grids.assign(grids, grids + nruns);
  s->fields.assign(fields, fields + nruns);
  if (nspecies) {
    s->sp.assign(species, species + nspecies);
    s->alt.assign(species_alt, species_alt + nspecies);
    s->species_run.assign(species_run, species_run + nspecies);
  }
  s->opt = *opt;
  if (hipMalloc((void**)&s->diag, sizeof(double) * DIAG_NUM * nruns) != hipSuccess ||
      hipMalloc((void**)&s->nchunks, 256) != hipSuccess ||
      hipMalloc((void**)&s->escapes, 256) != hipSuccess) {
    lpic_sim_destroy(s);
    return fail(LPIC_ENOMEM, "device allocation failed");
  }
  if (hipMemset(s->diag, 0, sizeof(double) * DIAG_NUM * nruns) != hipSuccess ||
      hipMemset(s->escapes, 0, 256) != hipSuccess) {
    lpic_sim_destroy(s);
    return fail(LPIC_EHIP, "hipMemset failed");
  }
  if (hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    lpic_sim_destroy(s);
    return fail(LPIC_EHIP, "stream creation failed");
  }
  lpic_status st = configure(s);
  if (st != LPIC_OK) {
    std::string keep = g_err;
    lpic_sim_destroy(s);
    g_err = keep;
    return st;
  }
  *out = s;
  return LPIC_OK;
}

void lpic_sim_destroy(lpic_sim* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  drop_graphs(s);
  for (auto& e : s->ev_pending) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  for (auto& e : s->ev_free) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  free_dev(s->runs_d); free_dev(s->segs_d); free_dev(s->run_blk_d);
  free_dev(s->seg_blk256_d); free_dev(s->seg_blk_sort_d);
  free_dev(s->counts); free_dev(s->offsets); free_dev(s->cursor); free_dev(s->mult);
  free_dev(s->chunks); free_dev(s->nchunks); free_dev(s->diag); free_dev(s->escapes);
  free_dev(s->scan_part);
  free_dev(s->esc_items); free_dev(s->esc_count);
  free_dev(s->rb.counts); free_dev(s->rb.offsets); free_dev(s->rb.cursor);
  free_dev(s->rb.chunks); free_dev(s->rb.nchunks);
  free_dev(s->rb_items); free_dev(s->esc2_items); free_dev(s->esc2_count);
  free_dev(s->esc_rec); free_dev(s->rb_rec); free_dev(s->esc_keys);
  free_dev(s->wmax); free_dev(s->jshift); free_dev(s->step_dev);
  free_dev(s->mid_pfx_d); free_dev(s->bands);
  free_dev(s->old_state);
  for (void* p : s->psi) free_dev(p);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  delete s;
}

lpic_status lpic_register_hook(lpic_sim* s, int32_t stage, lpic_hook_fn fn, void* user) {
  if (!s || !fn) return fail(LPIC_EINVAL, "sim or hook is NULL");
  if (stage < 0 || stage >= LPIC_NUM_STAGES) return fail(LPIC_EINVAL, "bad stage %d", stage);
  s->hooks[stage].push_back({fn, user});
  drop_graphs(s);
  return LPIC_OK;
}

lpic_status lpic_clear_hooks(lpic_sim* s) {
  if (!s) return fail(LPIC_EINVAL, "sim is NULL");
  for (auto& v : s->hooks) v.clear();
  drop_graphs(s);
  return LPIC_OK;
}

lpic_status lpic_step(lpic_sim* s, int32_t nsteps) {
  if (!s) return fail(LPIC_EINVAL, "sim is NULL");
  if (nsteps < 0) return fail(LPIC_EINVAL, "nsteps must be >= 0");
  const bool split = intermediate_hooks(s);
  if (split) CHK(ensure_old_state(s));
  const bool use_graph = s->opt.use_graph && !s->timing && !inner_hooks(s);
  s->last_graph = use_graph;
  CHK(run_hooks(s, LPIC_STAGE_START));
  if (nsteps > 0) CHK(enqueue_fixed_shift(s, s->stream));
  const bool hooks = any_hooks(s);
  // chained charge inside this call (no hooks, so nothing looks at or moves the particles
  // between the two steps of a chain)
  const bool chain = s->chain && !hooks && !split && s->opt.diag_interval >= 2;
  int prev_rho = 0;
  bool e_half_pending = false;
  for (int n = 0; n < nsteps; ++n) {
    CHK(run_hooks(s, LPIC_STAGE_LOOP_START));
    const bool do_sort = s->need_sort || (s->step % s->opt.sort_interval) == 0;
    const bool always_spread = (s->opt.tiling.flags & LPIC_SORT_SPREAD) != 0;
    const bool spread = do_sort && (s->need_spread || always_spread);
    const bool diag = s->opt.diag_interval > 0 && ((s->step + 1) % s->opt.diag_interval) == 0;
    const bool pre_diag = chain && n + 1 < nsteps && ((s->step + 2) % s->opt.diag_interval) == 0;
    const int rho = diag ? (prev_rho == 2 ? 3 : 1) : (pre_diag ? 2 : 0);
    prev_rho = rho;
    // inside one call, with no hooks that could look at the fields between steps, a step
    // that ends without diagnostics leaves its last E half to the next step
    const bool first_full = e_half_pending;
    const bool skip_last = !hooks && !diag && n + 1 < nsteps;
    e_half_pending = skip_last;
    // the one-off spreading sort runs eagerly; captured sort steps use the plain sort unless
    // every sort spreads
    if (use_graph && (!spread || always_spread)) {
      const int gi = rho * 16 + (do_sort ? 8 : 0) + (diag ? 4 : 0) + (first_full ? 2 : 0) +
                     (skip_last ? 1 : 0);
      if (!s->gexec[gi]) {
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
        lpic_status st = enqueue_step(s, s->cap_stream, do_sort, spread, diag, false, true,
                                      first_full, skip_last, rho);
        hipError_t ee = hipStreamEndCapture(s->cap_stream, &g);
        if (st != LPIC_OK) { if (g) (void)hipGraphDestroy(g); return st; }
        if (ee != hipSuccess) return fail(LPIC_EHIP, "graph capture: %s", hipGetErrorString(ee));
        hipError_t ie = hipGraphInstantiate(&s->gexec[gi], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return fail(LPIC_EHIP, "graph instantiate: %s", hipGetErrorString(ie));
      }
      HIPCHK(hipGraphLaunch(s->gexec[gi], s->stream));
      if (do_sort && s->nsegs > 0) swap_host_buffers(s);
    } else {
      CHK(enqueue_step(s, s->stream, do_sort, spread, diag, true, false, first_full, skip_last,
                       rho));
    }
    if (do_sort && s->nsegs > 0) {
      ++s->sorts;
      s->need_sort = false;
      s->need_spread = false;
      std::fill(s->inject_used.begin(), s->inject_used.end(), 0);
      s->offsets_valid = true;
    }
    if (diag) s->diag_step = s->step + 1;
    ++s->step;
    CHK(run_hooks(s, LPIC_STAGE_LOOP_END));
  }
  CHK(run_hooks(s, LPIC_STAGE_FINISH));
  return LPIC_OK;
}

lpic_status lpic_get_species(lpic_sim* s, int32_t i, lpic_species* out) {
  if (!s || !out) return fail(LPIC_EINVAL, "NULL argument");
  if (i < 0 || i >= s->nsegs) return fail(LPIC_EINVAL, "species index %d out of range", i);
  *out = s->sp[i];
  return LPIC_OK;
}

lpic_status lpic_get_stats(lpic_sim* s, lpic_stats* out) {
  if (!s || !out) return fail(LPIC_EINVAL, "NULL argument");
  for (auto& e : s->ev_pending) {
    HIPCHK(hipEventSynchronize(e.second));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e.first, e.second));
    s->fused_ms += ms;
    ++s->fused_launches;
    s->ev_free.push_back(e);
  }
  s->ev_pending.clear();
  out->steps = s->step;
  out->sorts = s->sorts;
  out->fused = s->last_fused ? 1 : 0;
  out->graph = s->last_graph ? 1 : 0;
  out->fused_ms = s->fused_ms;
  out->fused_launches = s->fused_launches;
  unsigned long long esc = 0;
  HIPCHK(hipStreamSynchronize(s->stream));
  HIPCHK(hipMemcpy(&esc, s->escapes, sizeof(esc), hipMemcpyDeviceToHost));
  out->halo_escapes = (int64_t)esc;
  out->field_tile[0] = s->mid_tx;
  out->field_tile[1] = s->mid_ty;
  return LPIC_OK;
}

lpic_status lpic_get_diagnostics(lpic_sim* s, int32_t r, double out[5]) {
  if (!s || !out) return fail(LPIC_EINVAL, "NULL argument");
  if (r < 0 || r >= s->nruns) return fail(LPIC_EINVAL, "box index %d out of range", r);
  HIPCHK(hipStreamSynchronize(s->stream));
  double d[DIAG_NUM];
  HIPCHK(hipMemcpy(d, s->diag + (size_t)r * DIAG_NUM, sizeof(d), hipMemcpyDeviceToHost));
  const lpic_grid& g = s->grids[r];
  const double dV = g.dx * g.dy * (g.ndim == 3 ? g.dz : 1.0);
  out[0] = d[DIAG_UFIELD];
  out[1] = d[DIAG_UKIN] * dV;
  out[2] = d[DIAG_RHOMAX] > 0 ? d[DIAG_RES] / d[DIAG_RHOMAX] : d[DIAG_RES];
  out[3] = d[DIAG_GAUSS];
  out[4] = (double)s->diag_step;
  for (int i = 0; i < 4; ++i)
    if (!isfinite(out[i])) return fail(LPIC_ENUMERIC, "diagnostic %d of box %d is not finite", i, r);
  return LPIC_OK;
}

lpic_status lpic_set_timing(lpic_sim* s, int32_t on) {
  if (!s) return fail(LPIC_EINVAL, "sim is NULL");
  s->timing = on != 0;
  if (!s->timing) {
    lpic_stats tmp;
    CHK(lpic_get_stats(s, &tmp));
  }
  s->fused_ms = 0.0;
  s->fused_launches = 0;
  return LPIC_OK;
}

lpic_status lpic_set_options(lpic_sim* s, const lpic_options* opt) {
  if (!s || !opt) return fail(LPIC_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(s->stream));
  // the device segment table is rebuilt from the host mirror, which tracks the buffers
  lpic_options keep = s->opt;
  s->opt = *opt;
  lpic_status st = configure(s);
  if (st != LPIC_OK) {
    s->opt = keep;
    std::string err = g_err;
    (void)configure(s);
    g_err = err;
  }
  return st;
}

lpic_status lpic_set_laser(lpic_sim* s, int32_t r, const lpic_laser* laser) {
  if (!s) return fail(LPIC_EINVAL, "sim is NULL");
  if (r < 0 || r >= s->nruns) return fail(LPIC_EINVAL, "run index %d out of range", r);
  if (laser) {
    CHK(check_laser(laser, &s->grids[r]));
    s->lasers[r] = make_laser(laser);
  }
  s->has_laser[r] = laser ? 1 : 0;
  return configure(s);   // rebuilds the device tables and the step counter, drops graphs
}

lpic_status lpic_set_pml(lpic_sim* s, int32_t r, const lpic_pml* pml) {
  if (!s) return fail(LPIC_EINVAL, "sim is NULL");
  if (r < 0 || r >= s->nruns) return fail(LPIC_EINVAL, "run index %d out of range", r);
  const lpic_grid& g = s->grids[r];
  s->pmls.resize(s->nruns, lpic_pml{});
  s->psi.resize(s->nruns, nullptr);
  if (pml) {
    if (!g.open_x) return fail(LPIC_EINVAL, "a PML needs open x ends (grid.open_x)");
    if (s->x0.size() > (size_t)r && s->shifted[r] != 0)
      return fail(LPIC_EUNSUPPORTED, "box %d has moved its window", r);
    if (pml->cells < 1 || 2 * pml->cells > g.nx - 8)
      return fail(LPIC_EINVAL, "PML of %d cells in a box of %d", pml->cells, g.nx);
    if (pml->order < 0 || pml->order > 8 || pml->a_order < 0 || pml->a_order > 8)
      return fail(LPIC_EINVAL, "PML grading orders %d, %d outside [0, 8]", pml->order,
                  pml->a_order);
    if (!std::isfinite(pml->sigma_max) || !std::isfinite(pml->kappa_max) ||
        !std::isfinite(pml->a_max) || !(pml->kappa_max >= 1.0) || !(pml->a_max >= 0.0))
      return fail(LPIC_EINVAL, "PML needs finite sigma_max, kappa_max >= 1 and a_max >= 0");
    if (pml->reserved0 != 0) return fail(LPIC_EINVAL, "lpic_pml.reserved0 must be 0");
  }
  free_dev(s->psi[r]);
  s->psi[r] = nullptr;
  s->pmls[r] = lpic_pml{};
  if (pml) {
    lpic_pml p = *pml;
    if (p.sigma_max < 0.0) p.sigma_max = 0.8 * (p.order + 1) / g.dx;
    // recursion coefficients per slot for a half step dt/2 (every field update of a
    // simulation is made of such halves): E side, then B side, each {b, c, 1/kappa}
    const int L = p.cells;
    std::vector<double> tab;
    for (int side = 0; side < 2; ++side)
      for (int slot = 0; slot < 2 * L; ++slot) {
        const double half = side ? 0.5 : 0.0;
        const double depth = slot < L ? (L - slot) - half : (slot - L) + half;
        const double sd = depth / L;
        double sm = 1.0, sa = 1.0;
        for (int q = 0; q < p.order; ++q) sm *= sd;
        for (int q = 0; q < p.a_order; ++q) sa *= 1.0 - sd;
        const double sigma = p.sigma_max * sm, kappa = 1.0 + (p.kappa_max - 1.0) * sm;
        const double a = p.a_max * sa;
        const double b = std::exp(-(sigma / kappa + a) * 0.5 * g.dt);
        tab.push_back(b);
        tab.push_back(sigma > 0.0 ? sigma * (b - 1.0) / (kappa * (sigma + kappa * a)) : 0.0);
        tab.push_back(1.0 / kappa);
      }
    const size_t psi_bytes = pml_psi_bytes(&g, L, s->prec);
    const bool f32 = s->prec == LPIC_F32_CELLOFS;
    std::vector<float> tabf(tab.begin(), tab.end());
    const size_t tab_bytes = tab.size() * (f32 ? 4 : 8);
    if (hipMalloc(&s->psi[r], psi_bytes + tab_bytes) != hipSuccess)
      return fail(LPIC_ENOMEM, "PML allocation of %zu bytes failed", psi_bytes + tab_bytes);
    HIPCHK(hipMemset(s->psi[r], 0, psi_bytes));
    HIPCHK(hipMemcpy((char*)s->psi[r] + psi_bytes, f32 ? (const void*)tabf.data()
                                                      : (const void*)tab.data(),
                     tab_bytes, hipMemcpyHostToDevice));
    s->pmls[r] = p;
  }
  return configure(s);   // device tables (and the field update path), drops graphs
}

lpic_status lpic_window_shift(lpic_sim* s, int32_t r, int32_t m, const lpic_plasma* plasma) {
  if (!s) return fail(LPIC_EINVAL, "sim is NULL");
  if (r < 0 || r >= s->nruns) return fail(LPIC_EINVAL, "run index %d out of range", r);
  const lpic_grid& g = s->grids[r];
  if (!g.open_x) return fail(LPIC_EINVAL, "a moving window needs open x ends");
  if (s->pmls.size() > (size_t)r && s->pmls[r].cells > 0)
    return fail(LPIC_EUNSUPPORTED, "box %d has PML layers (moving windows use Mur ends)", r);
  if (s->ndim != 2) return fail(LPIC_EUNSUPPORTED, "moving windows are 2D only");
  if (m < 1 || m > g.nx - 2 * LPIC_OPEN_MARGIN - 1)
    return fail(LPIC_EINVAL, "shift %d outside [1, nx - 7]", m);
  if (!s->offsets_valid) return fail(LPIC_EINVAL, "take a step before moving the window");
  int seg = -1;
  if (plasma) {
    seg = plasma->species;
    if (seg < 0 || seg >= s->nsegs || s->species_run[seg] != r)
      return fail(LPIC_EINVAL, "species %d is not a species of box %d", seg, r);
    if (plasma->ppc_x < 1 || plasma->ppc_y < 1 || plasma->ppc_x * plasma->ppc_y > 4096)
      return fail(LPIC_EINVAL, "plasma lattice %d x %d", plasma->ppc_x, plasma->ppc_y);
    if (!(plasma->density >= 0.0) || !std::isfinite(plasma->ux) || !std::isfinite(plasma->uy) ||
        !std::isfinite(plasma->uz))
      return fail(LPIC_EINVAL, "bad plasma density or momentum");
  }
  if (!s->windows) {   // the fused field update assumes the origin at column 0
    s->windows = true;
    s->mid_tx = s->mid_ty = s->mid_ntiles = 0;
    drop_graphs(s);
  }
  Tables T = sim_tables(s, s->seg_blk256_d);
  launch_window_shift(T, s->prec, s->ndim, r, m, (int64_t)g.ny, s->nblk_p256, s->stream);
  CHK(last_launch("window shift"));
  s->x0[r] = (s->x0[r] + m) % g.nx;
  s->runs_h[r].x0 = s->x0[r];
  s->shifted[r] += m;
  if (plasma) {
    const int64_t count = (int64_t)m * g.ny * plasma->ppc_x * plasma->ppc_y;
    const double w = plasma->density / (plasma->ppc_x * plasma->ppc_y);
    launch_window_inject(T, s->prec, s->ndim, seg, m, count, plasma->ppc_x, plasma->ppc_y, w,
                         plasma->ux, plasma->uy, plasma->uz, s->offsets, s->inject_used[seg],
                         (unsigned long long*)((char*)s->step_dev + 192), s->stream);
    CHK(last_launch("window inject"));
    s->inject_used[seg] += count;
  }
  s->need_sort = true;
  return LPIC_OK;
}

lpic_status lpic_window_info(lpic_sim* s, int32_t r, int64_t* shifted, int64_t* dropped) {
  if (!s) return fail(LPIC_EINVAL, "sim is NULL");
  if (r < 0 || r >= s->nruns) return fail(LPIC_EINVAL, "run index %d out of range", r);
  if (shifted) *shifted = s->shifted[r];
  if (dropped) {
    unsigned long long v = 0;
    HIPCHK(hipStreamSynchronize(s->stream));
    HIPCHK(hipMemcpy(&v, (char*)s->step_dev + 192, sizeof(v), hipMemcpyDeviceToHost));
    *dropped = (int64_t)v;
  }
  return LPIC_OK;
}

}  // extern "C"

namespace {

// One autotuner trial: the options set (false: infeasible), an untimed warm-up of whole
// periods of its sort and diagnostics intervals (sorts, graph captures), then as many steps
// timed with events on the simulation's stream.
lpic_status time_trial(lpic_sim* s, const lpic_options& o, int32_t steps_each, bool* feasible,
                       double* ms_per_step) {
  *feasible = false;
  if (lpic_set_options(s, &o) != LPIC_OK) return LPIC_OK;
  *feasible = true;
  const int k = std::max(1, o.sort_interval), d = std::max(1, o.diag_interval);
  const int period = k / std::gcd(k, d) * d;
  const int n = (std::max(1, steps_each) + period - 1) / period * period;
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  lpic_status st = lpic_step(s, n);
  if (st == LPIC_OK && hipEventRecord(a, s->stream) != hipSuccess) st = fail(LPIC_EHIP, "event");
  if (st == LPIC_OK) st = lpic_step(s, n);
  if (st == LPIC_OK && (hipEventRecord(b, s->stream) != hipSuccess ||
                        hipEventSynchronize(b) != hipSuccess))
    st = fail(LPIC_EHIP, "event");
  float ms = 0.f;
  if (st == LPIC_OK && hipEventElapsedTime(&ms, a, b) != hipSuccess) st = fail(LPIC_EHIP, "event");
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms_per_step = (double)ms / n;
  return st;
}

int pow2_floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}
int pow2_ceil(int v) {
  int p = 1;
  while (p < v) p *= 2;
  return p;
}

}  // namespace

extern "C" {

lpic_status lpic_autotune(lpic_sim* s, const lpic_options* cand, int32_t ncand,
                          int32_t steps_each, lpic_options* best) {
  if (!s || !cand || ncand < 1 || steps_each < 1) return fail(LPIC_EINVAL, "bad autotune arguments");
  double best_ms = 1e300;
  int best_i = -1;
  for (int i = 0; i < ncand; ++i) {
    bool ok = false;
    double ms = 0.0;
    CHK(time_trial(s, cand[i], steps_each, &ok, &ms));
    if (ok && ms < best_ms) { best_ms = ms; best_i = i; }
  }
  if (best_i < 0) return fail(LPIC_EINVAL, "no feasible candidate");
  CHK(lpic_set_options(s, &cand[best_i]));
  if (best) *best = cand[best_i];
  return LPIC_OK;
}

lpic_status lpic_autotune_search(lpic_sim* s, const lpic_tune_space* sp, lpic_options* best,
                                 lpic_tune_report* report) {
  if (!s || !sp) return fail(LPIC_EINVAL, "sim or search space is NULL");
  if (sp->steps_each < 1) return fail(LPIC_EINVAL, "steps_each must be >= 1");
  const int nd = s->ndim;
  // parameter p: 0..2 tile edges, 3 halo, 4 chunk, 5 sort interval, 6 the re-binned
  // escape path (0 / 1); lo/hi per parameter
  constexpr int NP = 7;
  int lo[NP], hi[NP];
  for (int d = 0; d < 3; ++d) {
    lo[d] = pow2_ceil(std::max(1, sp->tile_min[d]));
    hi[d] = pow2_floor(std::max(1, sp->tile_max[d]));
  }
  if (nd != 3) lo[2] = hi[2] = 1;
  lo[3] = std::max(3, sp->halo_min);
  hi[3] = sp->halo_max;
  lo[4] = pow2_ceil(std::max(1, sp->chunk_min));
  hi[4] = pow2_floor(std::max(1, sp->chunk_max));
  lo[5] = std::max(1, sp->sort_min);
  hi[5] = sp->sort_max;
  lo[6] = sp->rebin == 1 ? 1 : 0;
  hi[6] = sp->rebin == 0 ? 0 : 1;
  for (int p = 0; p < NP; ++p)
    if (lo[p] > hi[p]) return fail(LPIC_EINVAL, "empty search range for parameter %d", p);
  const int budget = std::min(LPIC_TUNE_MAX_TRIALS,
                              sp->max_trials > 0 ? sp->max_trials : LPIC_TUNE_MAX_TRIALS);
  const lpic_options base = s->opt;
  auto get = [&](const lpic_options& o, int p) {
    switch (p) {
      case 0: return o.tiling.tx;
      case 1: return o.tiling.ty;
      case 2: return o.tiling.tz;
      case 3: return o.tiling.halo;
      case 4: return o.tiling.chunk;
      case 5: return o.sort_interval;
      default: return (o.tiling.flags & LPIC_ESCAPE_REBIN) ? 1 : 0;
    }
  };
  auto put = [&](lpic_options& o, int p, int v) {
    switch (p) {
      case 0: o.tiling.tx = v; break;
      case 1: o.tiling.ty = v; break;
      case 2: o.tiling.tz = v; break;
      case 3: o.tiling.halo = v; break;
      case 4: o.tiling.chunk = v; break;
      case 5: o.sort_interval = v; break;
      default:
        o.tiling.flags = v ? (o.tiling.flags | LPIC_ESCAPE_REBIN) : (o.tiling.flags & ~LPIC_ESCAPE_REBIN);
        break;
    }
  };
  // the starting point: the present options clamped into the space
  lpic_options cur = base;
  if (nd != 3) cur.tiling.tz = 1;
  for (int p = 0; p < NP; ++p) {
    int v = get(cur, p);
    if (p <= 2 || p == 4) v = pow2_floor(std::max(1, v));
    put(cur, p, std::min(hi[p], std::max(lo[p], v)));
  }
  std::vector<lpic_options> tried;
  std::vector<double> times;
  auto same = [](const lpic_options& a, const lpic_options& b) {
    return a.tiling.tx == b.tiling.tx && a.tiling.ty == b.tiling.ty &&
           a.tiling.tz == b.tiling.tz && a.tiling.halo == b.tiling.halo &&
           a.tiling.chunk == b.tiling.chunk && a.sort_interval == b.sort_interval &&
           a.tiling.flags == b.tiling.flags;
  };
  // time of an option set (cached); < 0 infeasible; budget exhausted: +inf, not recorded
  auto trial = [&](const lpic_options& o, double* ms) -> lpic_status {
    for (size_t i = 0; i < tried.size(); ++i)
      if (same(tried[i], o)) { *ms = times[i]; return LPIC_OK; }
    if ((int)tried.size() >= budget) { *ms = 1e300; return LPIC_OK; }
    bool ok = false;
    double t = 0.0;
    CHK(time_trial(s, o, sp->steps_each, &ok, &t));
    tried.push_back(o);
    times.push_back(ok ? t : -1.0);
    *ms = ok ? t : -1.0;
    return LPIC_OK;
  };
  auto better = [](double a, double b) { return a >= 0.0 && (b < 0.0 || a < b); };
  double cur_ms = 0.0;
  CHK(trial(cur, &cur_ms));
  bool moved = true;
  while (moved && (int)tried.size() < budget) {
    moved = false;
    for (int p = 0; p < NP; ++p) {
      if (lo[p] == hi[p]) continue;
      for (int dir = +1; dir >= -1; dir -= 2) {
        for (;;) {
          const int v = get(cur, p);
          // halo: one cell more or less; sizes and the sort interval: twice or half; the
          // re-binned path: on or off
          const int nv = (p == 3 || p == 6) ? v + dir : (dir > 0 ? v * 2 : v / 2);
          if (nv < lo[p] || nv > hi[p] || nv == v) break;
          lpic_options o = cur;
          put(o, p, nv);
          double ms = 0.0;
          CHK(trial(o, &ms));
          if (!better(ms, cur_ms) || ms >= 1e299) break;
          cur = o;
          cur_ms = ms;
          moved = true;
        }
      }
    }
  }
  int bi = -1;
  for (size_t i = 0; i < tried.size(); ++i)
    if (times[i] >= 0.0 && (bi < 0 || times[i] < times[bi])) bi = (int)i;
  if (bi < 0) {
    (void)lpic_set_options(s, &base);
    return fail(LPIC_EINVAL, "no feasible option set in the search space");
  }
  CHK(lpic_set_options(s, &tried[bi]));
  if (best) *best = tried[bi];
  if (report) {
    memset(report, 0, sizeof(*report));
    report->ntrials = (int32_t)tried.size();
    report->best = bi;
    for (size_t i = 0; i < tried.size(); ++i) {
      report->trial[i] = tried[i];
      report->ms_per_step[i] = times[i];
    }
  }
  return LPIC_OK;
}

}  // extern "C"
