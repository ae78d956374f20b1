// Internal interface between the C ABI (lpic_api.hip) and the kernels (lpic_kernels.hip,
// lpic_fused.hip).
#pragma once

#include "lpic_device.hpp"

namespace lpic {

// Split particle path: the start of each particle's deposit path (x^{n+1/2}), written by
// the gather-push kernels and read by the deposit:
//   FP32  cell[n] (packed, wrapped) o0[n] o1[n] (o2[n])     FP64  x[n] y[n] (z[n]) (wrapped)
template <typename R, int DIM>
struct OldState {
  int32_t* cell;
  R* o[3];
  __device__ __forceinline__ OldState(void* base, int64_t n) {
    char* b = (char*)base;
    if (sizeof(R) == 4) {
      cell = (int32_t*)b;
      b += 4 * n;
    } else {
      cell = nullptr;
    }
    for (int d = 0; d < 3; ++d) {
      if (d < DIM) { o[d] = (R*)b; b += sizeof(R) * n; } else { o[d] = nullptr; }
    }
  }
};


// Instantiate `call` with R (float / double) and D (2 / 3) from runtime values.
#define LPIC_PD(prec, dim, call)                                  \
  do {                                                            \
    if (prec == 0) {                                              \
      if (dim == 2) { using R = float; constexpr int D = 2; call; } \
      else { using R = float; constexpr int D = 3; call; }        \
    } else {                                                      \
      if (dim == 2) { using R = double; constexpr int D = 2; call; } \
      else { using R = double; constexpr int D = 3; call; }       \
    }                                                             \
  } while (0)

constexpr int SORT_BLOCK = 2048;   // particles per workgroup of the sort kernels

// Snapshot of the tile edges for the fused 2D field update (launch_yee_mid): the domain is
// cut into field tiles of tx x ty cells, and every tile publishes, per field component
// (Ex Ey Ez Bx By Bz), the values of its first two and its last column (3 ty values) and
// of its first two and its last row (3 tx values).  Two buffers of `half` values: the
// word *parity names the one holding the present fields.
struct FieldBands {
  void* base;
  int64_t half;
  const int32_t* tile_pfx;     // nruns + 1 prefix of field tiles (one workgroup per tile)
  int32_t* parity;
  const int64_t* step;         // antenna clock (steps taken); NULL: no run has an antenna
  int32_t tx, ty;              // powers of two, tx <= MID_MAX_TX, ty <= MID_MAX_TY
  int32_t lx, ly;              // their log2
};
constexpr int MID_MAX_TX = 64, MID_MAX_TY = 16;
inline int64_t band_values_per_tile(int tx, int ty) { return 6 * 3 * (int64_t)(tx + ty); }

// which = 0: E update (zero_j = 1 also clears J and rho, 2 J only, 3 J and rho0, 4 J and
// rho1), 1: B update.  halves = 2: the E
// update stands for two equal half updates (open x ends apply their condition twice).
// bands (B update in 2D only, may be NULL): also publish E and the new B of the tile edges
// into the snapshot buffer named by *parity, for a fused update that follows.
void launch_yee(const Tables& T, int prec, int dim, int nblocks, int which, double frac,
                int zero_j, int halves, hipStream_t st, const FieldBands* bands = nullptr);
// The three field updates between two particle pushes of 2D steps, fused: B by dt/2, E by
// dt (two merged halves, with the J in place), B by dt/2 -- the last half update of one
// step and the first two of the next.  T.run_blk must be the tile prefix (one workgroup
// per field tile).  Reads the snapshot named by *parity and writes the other one; J is
// only read.  Runs with an antenna get its current of this step (t = (*step + 1) dt) added
// in the E update instead of through the array, so the antenna kernel is not launched for
// the step.  The next launch on the stream must be launch_clear_sources with
// flip = bands.parity and clock = bands.step: it clears J for the next deposit, names the
// new snapshot and advances the antenna clock.  pml: some run has PML layers (their psi
// follow the same two-half scheme, with the same parity word); false selects kernels
// without that code.
void launch_yee_mid(const Tables& T, int prec, int ntiles, const FieldBands& bands, bool pml,
                    hipStream_t st);
// J := 0 (and the charge arrays when with_rho) over every cell of every run (nblocks: the
// 256-cell blocks of T.run_blk).  flip != NULL: also *flip ^= 1 and, clock != NULL,
// *clock += 1 (one thread).
// with_rho: 1 also clears both charge arrays, 3 rho0 only, 4 rho1 only.
void launch_clear_sources(const Tables& T, int prec, int dim, int nblocks, int with_rho,
                          int32_t* flip, int64_t* clock, hipStream_t st);
// Laser antennas of the runs that have one (bpr workgroups of 256 (j, k) cells per run).
// step != NULL: t = (*step + 1) dt, and the launch advances *step (done: a zeroed counter).
void launch_laser(const Tables& T, int prec, int dim, int nruns, int bpr, double t,
                  int64_t* step, unsigned int* done, hipStream_t st);
void launch_gather_push(const Tables& T, int prec, int dim, int nblocks, void* old,
                        hipStream_t st);
void launch_deposit(const Tables& T, int prec, int dim, int nblocks, const void* old,
                    int with_rho, hipStream_t st);
void launch_zero_u32(uint32_t* p, int64_t n, hipStream_t st);
// part: scan scratch of part_words(nbins) words (NULL: the one-workgroup scan).
void launch_sort(const Tables& T, int prec, int dim, int nblocks, int32_t* counts,
                 int32_t* offsets, int32_t* cursor, int32_t* mult, int nbins, int spread,
                 hipStream_t st, int32_t* part = nullptr);
// Words of scan scratch for n bins or chunk-order slots.
int part_words(int n);
void launch_swap_segments(SegDesc* segs, int nsegs, hipStream_t st);
// Work list of the fused kernel: every (tile, species) particle range cut into chunks, run
// by run, tile by tile, the run's species consecutive (nvirt = sum over runs of tiles x
// species; RunDesc seg_first / nseg / vbase describe the order).
// part (NULL: one workgroup): scratch of part_words(nvirt) words for the many-workgroup
// version.
void launch_build_chunks(const Tables& T, const int32_t* offsets, int nvirt, int chunk,
                         Chunk* out, int32_t* nchunks, hipStream_t st, int32_t* part = nullptr);
// Particles whose stencils leave the staged region of their home tile: the fused kernel
// records them here and a second kernel pushes them through global memory (or, re-binned, a
// second fused pass); the escape kernel's last workgroup
// clears the list (count[0] entries, count[1] workgroups done) for the next step.
struct EscapeList {
  unsigned long long* items;   // (segment << 32) | particle
  unsigned int* count;         // two counters, zero between steps
  unsigned long long* total;   // cumulative number of escapes
  int64_t capacity;
  void* rec = nullptr;         // with the re-binned path: entry k's particle words as an
                               // escape record (EscRec, 8 values of the kernel precision)
  int32_t* keys = nullptr;     // with records: entry k's (segment, tile) bin by the tile its
                               // particle is in, written with the record
};
constexpr int ESCAPE_BLOCKS = 128;

// The re-binned escape path (tiling flag LPIC_ESCAPE_REBIN): when a step's escape list
// holds at least `threshold` particles, they are grouped by the tile they are in now (bins
// in the sort's layout: segment s owns [bin_base, bin_base + ntiles]) and pushed by a
// second fused pass against the staged regions of those tiles; below the threshold
// k_escape pushes them through global memory as without the flag.
struct Rebin {
  int threshold;
  int nbins;                   // bins of all segments
  int nvirt, chunk;            // the chunk order of the fused kernel (launch_build_chunks)
  int32_t* part;               // scan scratch (part_words(max(nbins, nvirt)) words)
  int count_blocks;            // workgroups of the count and scatter kernels
  int32_t *counts, *offsets, *cursor;   // nbins + 1 each; counts zero between steps
  unsigned long long* items;   // the escape list grouped by bin (capacity of the list)
  void* rec;                   // their escape records in the same order
  Chunk* chunks;
  int32_t* nchunks;
  EscapeList esc2;             // particles the second pass finds outside its regions
  int geo[3];                  // the second pass's geometry (fused_geometry()), grid and
  int grid[3];                 // dynamic LDS without charge, with both charge planes, and
  size_t smem[3];              // with one (the with_rho modes of the first pass)
};

// geometry: 0 = runtime strides, else a compiled (tile, halo) shape (fused_geometry()).
int fused_geometry(int dim, int tx, int ty, int tz, int halo);
// Launches the fused kernel (persistent grid of nblocks, a multiple of 8) and then the
// escape kernel on the same stream.
// jshift[run]: the fixed-point shift S of the FP32 current accumulators (launch_fixed_shift).
// rebin != NULL: the re-binned escape path follows the first pass (see Rebin).
void launch_fused(const Tables& T, int prec, int dim, int geo, int nblocks, size_t smem,
                  const Chunk* chunks, const int32_t* nchunks, int with_rho, double* kinetic,
                  int ke_to_diag, const EscapeList& esc, const int32_t* jshift,
                  hipStream_t st, const Rebin* rebin = nullptr);
// Escape-list entries to (segment, present tile) bins and their grouped list (the first
// three kernels of the re-binned path), then the chunk list over those bins.
void launch_rebin(const Tables& T, int prec, int dim, const EscapeList& esc, const Rebin& rb,
                  hipStream_t st);
// Per run, the shift S for the fixed-point current accumulators of the fused kernel, from
// the largest |q w| of its species (wmax: fixed_shift_slots() 8-byte words per segment,
// zeroed by the caller; nblocks workgroups of SORT_BLOCK particles as for the sort) and its
// particle count.
int fixed_shift_slots();
void launch_fixed_shift(const Tables& T, int prec, int dim, int nblocks, int nruns, int nsegs,
                        unsigned long long* wmax, int32_t* jshift, hipStream_t st);
// Sets the dynamic LDS limit to smem and returns how many workgroups of the kernel fit on a
// CU when each uses smem_occ bytes.
hipError_t prepare_fused(int prec, int dim, int geo, size_t smem, size_t smem_occ,
                         int* blocks_per_cu);
void launch_reduce_fields(const Tables& T, int prec, int dim, int nblocks, int with_rho,
                          double* out, hipStream_t st);
void launch_kinetic(const Tables& T, int prec, int dim, int nblocks, double* out,
                    hipStream_t st);
void launch_zero_doubles(double* p, int n, hipStream_t st);
void launch_diag_clear(const Tables& T, int nruns, hipStream_t st);
// Moving window of run `run` (open x ends): clear the fields of its first m box columns,
// remove the particles there (nblk_part: 256-particle blocks of all segments, T.seg_blk the
// matching prefix), then advance the run's origin x0 by m on the device.
void launch_window_shift(const Tables& T, int prec, int dim, int run, int m, int64_t rows,
                         int nblk_part, hipStream_t st);
// Fresh plasma for the m box columns inside the right-hand margin of segment seg's run (after
// launch_window_shift): count = m * ny * px * py particles on a px x py lattice per cell,
// written after the segment's alive particles of the last sort (offsets) plus `used`.
void launch_window_inject(const Tables& T, int prec, int dim, int seg, int m, int64_t count,
                          int px, int py, double w, double ux, double uy, double uz,
                          const int32_t* offsets, int64_t used, unsigned long long* dropped,
                          hipStream_t st);
void launch_load_positions(const Tables& T, int prec, int dim, int nblocks, const double* x,
                           const double* y, const double* z, hipStream_t st);
void launch_store_positions(const Tables& T, int prec, int dim, int nblocks, double* x,
                            double* y, double* z, hipStream_t st);
// geo >= 0: the LDS of that geometry's launch (its workgroup size), else the tiling's own
size_t fused_smem_bytes(int prec, int dim, int tx, int ty, int tz, int halo, int with_rho,
                        int geo = -1);

// ---- QED event Monte-Carlo (Sec. 3.4) ------------------------------------------------------
// Table geometry: emission rows at ln chi = QED_E_L0 + i QED_E_DL (chi from 1e-4, 40 per
// decade, to 1e3), pair rows from chi = 1e-2 likewise, QED_NZ quantile levels z = QED_Z0 +
// j QED_DZ, r = 1 / (1 + e^-z).  Layout of one table block (doubles): emission ln h[NE],
// pair ln T + 8/(3 chi)[NP], emission v[NE][NZ], pair v[NP][NZ], v = ln(xi / (1 - xi)).
constexpr int QED_NE = 281, QED_NP = 201, QED_NZ = 161;
constexpr double QED_E_L0 = -9.210340371976184;    // ln 1e-4
constexpr double QED_P_L0 = -4.605170185988091;    // ln 1e-2
constexpr double QED_E_DL = 0.05756462732485115;   // ln 10 / 40
constexpr double QED_P_DL = 0.05756462732485115;
constexpr double QED_Z0 = -20.0, QED_DZ = 0.25;

struct QedTab {
  const double *emit_rate, *pair_rate, *emit_inv, *pair_inv;
};

struct QedBufDesc {
  int64_t cap;
  int32_t* count;
  double *x, *y, *z, *ux, *uy, *uz, *w, *tau;
  int32_t* src;
};

struct QedCall {
  QedTab tab;
  double hw;
  uint64_t seed;
  int64_t step;
  QedBufDesc out;
};

size_t qed_table_doubles();
const double* qed_host_tables();          // built once per process, on all host threads
QedTab qed_views(const double* base);

// Counter-based SplitMix64 draw in (0, 1): output number ((step << 32) | slot) * 4 + draw of
// the generator seeded with `seed`.
__host__ __device__ inline double qed_draw(uint64_t seed, int64_t step, int64_t slot,
                                           int draw) {
  const uint64_t k = ((((uint64_t)step) << 32) | (uint64_t)(uint32_t)slot) * 4u + (uint64_t)draw;
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return ((double)(z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// Row interpolation at quantile position fz = (z - Z0) / DZ: cubic through the four nearest
// levels inside the table, linear with the end slopes beyond it.
__host__ __device__ inline double qed_row(const double* row, double fz) {
  if (fz < 0.0) return row[0] + fz * (row[1] - row[0]);
  if (fz > QED_NZ - 1) return row[QED_NZ - 1] + (fz - (QED_NZ - 1)) * (row[QED_NZ - 1] - row[QED_NZ - 2]);
  int j = (int)floor(fz);
  j = j < 1 ? 1 : (j > QED_NZ - 3 ? QED_NZ - 3 : j);
  const double t = fz - j;
  const double wm = -t * (t - 1.0) * (t - 2.0) / 6.0, w0 = (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0;
  const double w1 = -(t + 1.0) * t * (t - 2.0) / 2.0, w2 = (t + 1.0) * t * (t - 1.0) / 6.0;
  return wm * row[j - 1] + w0 * row[j] + w1 * row[j + 1] + w2 * row[j + 2];
}

// The table lookups take their logarithms and exponentials in FP32 (a few instructions
// against the long software sequences of FP64 ones): an index or weight off by 1e-7 and a value
// off by 1e-7 relative are far below the tables' own 1e-4.  The decisions themselves
// (optical depth minus rate x dt) stay in FP64.
__host__ __device__ inline double qed_exp(double a) {
  return a > -80.0 ? (double)expf((float)a) : exp(a);
}

// -ln u for a draw u in (0, 1) to 1e-7 relative: above 1/2 through log1p of 1 - u (exact in
// FP64), so depths near zero keep their relative accuracy.
__host__ __device__ inline double qed_neglog(double u) {
  return u > 0.5 ? -(double)log1pf(-(float)(1.0 - u)) : -(double)logf((float)u);
}

__host__ __device__ inline double qed_emit_rate(const QedTab& t, double chi) {
  if (!(chi > 0.0)) return 0.0;
  const double f = ((double)logf((float)chi) - QED_E_L0) / QED_E_DL;
  if (f <= 0.0) return qed_exp(t.emit_rate[0] + f * QED_E_DL);   // classical: h ~ chi
  const int i = f < QED_NE - 2 ? (int)f : QED_NE - 2;
  return qed_exp(t.emit_rate[i] + (f - i) * (t.emit_rate[i + 1] - t.emit_rate[i]));
}

__host__ __device__ inline double qed_pair_rate(const QedTab& t, double chi) {
  if (!(chi >= 1e-2)) return 0.0;
  const double f = ((double)logf((float)chi) - QED_P_L0) / QED_P_DL;
  const int i = f < QED_NP - 2 ? (int)f : QED_NP - 2;
  return qed_exp(t.pair_rate[i] + (f - i) * (t.pair_rate[i + 1] - t.pair_rate[i]) -
                 8.0 / (3.0 * chi));
}

__host__ __device__ inline double qed_sample(const double* inv, int nrows, double l0,
                                             double dl, double chi, double r, double& scale) {
  const double z = (double)(logf((float)r) - logf((float)(1.0 - r)));
  const double fz = (z - QED_Z0) / QED_DZ;
  double f = ((double)logf((float)chi) - l0) / dl;
  scale = 1.0;
  if (f < 0.0) {            // below the first row
    scale = qed_exp(f * dl);
    f = 0.0;
  }
  int i = (int)f;
  i = i > nrows - 2 ? nrows - 2 : i;
  double a = f - i;
  a = a > 1.0 ? 1.0 : a;    // beyond the last row: the last row
  const double v = (1.0 - a) * qed_row(inv + (size_t)i * QED_NZ, fz) +
                   a * qed_row(inv + (size_t)(i + 1) * QED_NZ, fz);
  return v < -80.0 ? exp(v) : 1.0 / (1.0 + qed_exp(-v));
}

// Emission: below the first row the spectrum is the classical one, a function of xi / chi.
__host__ __device__ inline double qed_emit_sample(const QedTab& t, double chi, double r) {
  double scale;
  const double xi = qed_sample(t.emit_inv, QED_NE, QED_E_L0, QED_E_DL, chi, r, scale);
  return xi * scale;
}

__host__ __device__ inline double qed_pair_sample(const QedTab& t, double chi, double r) {
  double scale;
  return qed_sample(t.pair_inv, QED_NP, QED_P_L0, QED_P_DL, chi < 1e-2 ? 1e-2 : chi, r, scale);
}

void launch_qed_tau(double* tau, int64_t n, uint64_t seed, int64_t step, hipStream_t st);
void launch_qed_push(const Tables& T, int prec, int dim, int64_t n, void* old, double* tau,
                     const QedCall& q, hipStream_t st);
void launch_qed_photons(const RunDesc& r, int prec, int dim, int order, const QedBufDesc& ph,
                        const QedCall& q, hipStream_t st);
int qed_compact_blocks(int64_t cap);
void launch_qed_compact(const QedBufDesc& in, const QedBufDesc& out, int32_t* blk,
                        hipStream_t st);
void launch_qed_insert(const Tables& T, int prec, int dim, int64_t first, const QedBufDesc& b,
                       int parity, int32_t* dropped, hipStream_t st);

}  // namespace lpic
