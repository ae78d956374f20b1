// HIP kernels of the PIC hot path (gfx950, wave64).  No matrix cores: nothing here is a
// dense contraction.  The particle stream is structure-of-arrays and read/written once per
// step with unit stride; field tiles are staged in LDS for the gather and the current of a
// tile is accumulated in LDS, then flushed with one global atomic per non-zero cell.
#include "lpic_internal.hpp"

namespace lpic {

// =======================================================================================
// Small utilities
// =======================================================================================
__device__ __forceinline__ const RunDesc& run_of(const Tables& T, int r) {
  return T.runs ? T.runs[r] : T.run0;
}
__device__ __forceinline__ const SegDesc& seg_of(const Tables& T, int s) {
  return T.segs ? T.segs[s] : T.seg0;
}

// Block -> (run, block within run) for kernels over grid cells.
__device__ __forceinline__ int cell_block(const Tables& T, int& blk) {
  blk = blockIdx.x;
  if (!T.runs) return 0;
  const int r = uniform(find_owner(T.run_blk, T.nruns, blk));
  blk = uniform(blk - T.run_blk[r]);
  return r;
}
// Block -> (segment, block within segment) for kernels over particles.
__device__ __forceinline__ int part_block(const Tables& T, int& blk) {
  blk = blockIdx.x;
  if (!T.segs) return 0;
  const int s = uniform(find_owner(T.seg_blk, T.nsegs, blk));
  blk = uniform(blk - T.seg_blk[s]);
  return s;
}

// Full periodic wrap (the staged region may be wider than a small box).
__device__ __forceinline__ int wrapm(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

__global__ void k_fill_zero_u32(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// =======================================================================================
// Yee field half updates (Sec. 3.2, Eqs. 3-4), periodic by index wrap.
// =======================================================================================
struct CellIdx {
  int64_t c, cim, cip, cjm, cjp, ckm, ckp;
};

__device__ __forceinline__ bool cell_index(const RunDesc& r, int blk, int dim, CellIdx& x) {
  const int64_t plane = (int64_t)r.nx * r.ny;
  const int64_t ncell = plane * (dim == 3 ? r.nz : 1);
  const int64_t c = (int64_t)blk * 256 + threadIdx.x;
  if (c >= ncell) return false;
  const int i = (int)(c % r.nx);
  const int64_t rest = c / r.nx;
  const int j = (int)(rest % r.ny);
  const int k = (int)(rest / r.ny);
  x.c = c;
  x.cim = c + (i == 0 ? r.nx - 1 : -1);
  x.cip = c + (i == r.nx - 1 ? 1 - r.nx : 1);
  x.cjm = c + (j == 0 ? (int64_t)(r.ny - 1) * r.nx : -(int64_t)r.nx);
  x.cjp = c + (j == r.ny - 1 ? -(int64_t)(r.ny - 1) * r.nx : (int64_t)r.nx);
  if (dim == 3) {
    x.ckm = c + (k == 0 ? (int64_t)(r.nz - 1) * plane : -plane);
    x.ckp = c + (k == r.nz - 1 ? -(int64_t)(r.nz - 1) * plane : plane);
  } else {
    x.ckm = x.ckp = c;
  }
  return true;
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_yee_e(Tables T, double frac, int zero_j) {
  int blk;
  const RunDesc& r = run_of(T, cell_block(T, blk));
  CellIdx x;
  if (!cell_index(r, blk, DIM, x)) return;
  gptr<R> f[F_NUM];
#pragma unroll
  for (int c = 0; c < F_NUM; ++c) f[c] = gp((R*)r.f[c]);
  const double h = frac * r.dt;
  const R hx = R(h / r.dx), hy = R(h / r.dy), hz = R(DIM == 3 ? h / r.dz : 0.0), hh = R(h);
  const R bx = f[F_BX][x.c], by = f[F_BY][x.c], bz = f[F_BZ][x.c];
  const R jx = f[F_JX][x.c], jy = f[F_JY][x.c], jz = f[F_JZ][x.c];
  R dex = hy * (bz - f[F_BZ][x.cjm]) - hh * jx;
  R dey = -hx * (bz - f[F_BZ][x.cim]) - hh * jy;
  R dez = hx * (by - f[F_BY][x.cim]) - hy * (bx - f[F_BX][x.cjm]) - hh * jz;
  if (DIM == 3) {
    dex -= hz * (by - f[F_BY][x.ckm]);
    dey += hz * (bx - f[F_BX][x.ckm]);
  }
  f[F_EX][x.c] += dex;
  f[F_EY][x.c] += dey;
  f[F_EZ][x.c] += dez;
  if (zero_j) {
    f[F_JX][x.c] = R(0);
    f[F_JY][x.c] = R(0);
    f[F_JZ][x.c] = R(0);
    if (f[F_R0]) f[F_R0][x.c] = R(0);
    if (f[F_R1]) f[F_R1][x.c] = R(0);
  }
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_yee_b(Tables T, double frac) {
  int blk;
  const RunDesc& r = run_of(T, cell_block(T, blk));
  CellIdx x;
  if (!cell_index(r, blk, DIM, x)) return;
  gptr<R> f[F_NUM];
#pragma unroll
  for (int c = 0; c < F_NUM; ++c) f[c] = gp((R*)r.f[c]);
  const double h = frac * r.dt;
  const R hx = R(h / r.dx), hy = R(h / r.dy), hz = R(DIM == 3 ? h / r.dz : 0.0);
  const R ex = f[F_EX][x.c], ey = f[F_EY][x.c], ez = f[F_EZ][x.c];
  R dbx = -hy * (f[F_EZ][x.cjp] - ez);
  R dby = hx * (f[F_EZ][x.cip] - ez);
  R dbz = -hx * (f[F_EY][x.cip] - ey) + hy * (f[F_EX][x.cjp] - ex);
  if (DIM == 3) {
    dbx += hz * (f[F_EY][x.ckp] - ey);
    dby -= hz * (f[F_EX][x.ckp] - ex);
  }
  f[F_BX][x.c] += dbx;
  f[F_BY][x.c] += dby;
  f[F_BZ][x.c] += dbz;
}

// =======================================================================================
// Split particle path: gather + push, then deposit (used when a hook sits between them).
// The old state holds the start of each particle's deposit path, the half-step position:
//   FP32  cell[n] (packed, wrapped) o0[n] o1[n] (o2[n])     FP64  x[n] y[n] (z[n]) (wrapped)
// =======================================================================================
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

template <typename R>
__device__ __forceinline__ GlobalAcc<R> global_acc(const RunDesc& r) {
  GlobalAcc<R> A;
#pragma unroll
  for (int c = 0; c < F_NUM; ++c) A.f[c] = gp((R*)r.f[c]);
  A.nx = r.nx; A.ny = r.ny; A.nz = r.nz;
  return A;
}

template <typename R, int DIM, int ORDER>
__device__ __forceinline__ void gather_push_one(const SegDesc& s, const RunDesc& r, int64_t p,
                                                void* old) {
  PState<R> ps;
  load_particle<R, DIM>(s, r, p, ps);
  OldState<R, DIM> os(old, s.n);
  if (!ps.alive) {
    if (os.cell) os.cell[p] = -1;
    else os.o[0][p] = R(-1);
    return;
  }
  const GlobalAcc<R> A = global_acc<R>(r);
  const PushConst<R> k = push_const<R>(r, s);
  int pc[3];
  R po[3], pe[3], x1[3], vz1, g1;
  push<DIM, ORDER>(A, ps.c, ps, k, pc, po, pe, x1, vz1, g1);
  const int n[3] = {r.nx, r.ny, r.nz};
  int wc[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < DIM; ++d) wc[d] = wrapi(pc[d], n[d]);
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
  for (int d = 0; d < DIM; ++d) advance_cell<R>(ps.c[d], ps.o[d], x1[d], n[d]);
  store_particle<R, DIM>(s, r, p, ps);
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_gather_push(Tables T, void* old) {
  int blk;
  const SegDesc& s = seg_of(T, part_block(T, blk));
  const int64_t p = (int64_t)blk * 256 + threadIdx.x;
  if (p >= s.n) return;
  const RunDesc& r = run_of(T, s.run);
  if (s.order == 1) gather_push_one<R, DIM, 1>(s, r, p, old);
  else gather_push_one<R, DIM, 2>(s, r, p, old);
}

template <typename R, int DIM, int ORDER>
__device__ __forceinline__ void deposit_one(const SegDesc& s, const RunDesc& r, int64_t p,
                                            const void* old, bool with_rho) {
  OldState<R, DIM> os((void*)old, s.n);
  PState<R> now;
  load_particle<R, DIM>(s, r, p, now);
  if (!now.alive) return;
  const int n[3] = {r.nx, r.ny, r.nz};
  int c0[3];
  R o0[3], pe[3];
  if constexpr (sizeof(R) == 4) {
    const int32_t cell0 = os.cell[p];
    if (cell0 < 0) return;
    unpack_cell(cell0, DIM, c0);
    if (c0[0] >= n[0] || c0[1] >= n[1] || (DIM == 3 && c0[2] >= n[2])) return;
#pragma unroll
    for (int d = 0; d < 3; ++d) o0[d] = d < DIM ? os.o[d][p] : R(0);
  } else {
    if (!(os.o[0][p] >= 0.0)) return;
    const double h[3] = {r.dx, r.dy, r.dz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d < DIM) {
        const double X = os.o[d][p] / h[d];
        if (!(X >= 0.0 && X <= (double)n[d])) return;
        const double f = floor(X);
        int ci = (int)f;
        o0[d] = X - f;
        c0[d] = ci >= n[d] ? ci - n[d] : ci;
      } else {
        c0[d] = 0; o0[d] = 0.0;
      }
    }
  }
  // path end: the start plus dt v^{n+1}, from the momentum the push left behind
  const PushConst<R> k = push_const<R>(r, s);
  const R ig1 = rsq<R>(R(1) + now.u[0] * now.u[0] + now.u[1] * now.u[1] + now.u[2] * now.u[2]);
  const R hd[3] = {k.hdx, k.hdy, k.hdz};
#pragma unroll
  for (int d = 0; d < 3; ++d) pe[d] = d < DIM ? o0[d] + R(2) * (hd[d] * now.u[d] * ig1) : R(0);
  const GlobalAcc<R> A = global_acc<R>(r);
  deposit<DIM, ORDER>(A, c0, o0, pe, now.w, now.u[2] * ig1, k, with_rho);
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_deposit(Tables T, const void* old, int with_rho) {
  int blk;
  const SegDesc& s = seg_of(T, part_block(T, blk));
  const int64_t p = (int64_t)blk * 256 + threadIdx.x;
  if (p >= s.n) return;
  const RunDesc& r = run_of(T, s.run);
  if (s.order == 1) deposit_one<R, DIM, 1>(s, r, p, old, with_rho != 0);
  else deposit_one<R, DIM, 2>(s, r, p, old, with_rho != 0);
}

// =======================================================================================
// Tile counting sort: count -> scan -> scatter.  Keys are global bins: segment s owns bins
// [bin_base, bin_base + ntiles] (the last one collects dead particles).  Consecutive lanes
// of a wave that share a key are merged into one atomic (particles are mostly in tile
// order already, so a wave usually touches one or two bins).
// =======================================================================================
constexpr int SORT_ITEMS = 8;   // particles per thread per block: 2048 per block

template <typename R, int DIM>
__device__ __forceinline__ int particle_bin(const SegDesc& s, const RunDesc& r, int64_t p) {
  int c[3];
  if constexpr (sizeof(R) == 4) {
    const int32_t cell = ((const int32_t*)s.p[P_CELL])[p];
    if (cell < 0) return s.bin_base + r.ntiles;
    unpack_cell(cell, DIM, c);
    if (c[0] >= r.nx || c[1] >= r.ny || (DIM == 3 && c[2] >= r.nz)) return s.bin_base + r.ntiles;
  } else {
    const double h[3] = {r.dx, r.dy, r.dz};
    const int n[3] = {r.nx, r.ny, r.nz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d < DIM) {
        const double X = ((const double*)s.p[P_X + d])[p] / h[d];
        if (!(X >= 0.0 && X <= (double)n[d])) return s.bin_base + r.ntiles;   // dead
        int ci = (int)floor(X);
        c[d] = ci >= n[d] ? ci - n[d] : ci;
      } else {
        c[d] = 0;
      }
    }
  }
  const int t = (((c[2] >> s.lz) * r.nty) + (c[1] >> s.ly)) * r.ntx + (c[0] >> s.lx);
  return s.bin_base + t;
}

// Run-length grouping of equal keys inside a wave.  Returns true for the first lane of each
// run, with `len` the run length; `head` is the first lane of this lane's run.
__device__ __forceinline__ bool wave_runs(int key, bool valid, int& len, int& head) {
  const int lane = __lane_id();
  const int prev = __shfl_up(key, 1, 64);
  const bool is_head = valid && (lane == 0 || prev != key);
  const uint64_t heads = __ballot(is_head) | ~__ballot(valid);
  const uint64_t above = heads & ~((2ull << lane) - 1ull);
  len = (above ? __ffsll((unsigned long long)above) - 1 : 64) - lane;
  const uint64_t upto = heads & ((2ull << lane) - 1ull);
  head = 63 - __clzll((unsigned long long)upto);
  return is_head;
}

// Keys of the SORT_ITEMS particles a thread handles (loads issued together); -1 past the end.
template <typename R, int DIM>
__device__ __forceinline__ void block_keys(const SegDesc& s, const RunDesc& r, int blk,
                                           int key[SORT_ITEMS], int64_t p[SORT_ITEMS]) {
  const int64_t beg = (int64_t)blk * 256 * SORT_ITEMS;
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    p[it] = beg + it * 256 + threadIdx.x;
    key[it] = p[it] < s.n ? particle_bin<R, DIM>(s, r, p[it]) : -1;
  }
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_sort_count(Tables T, int32_t* counts) {
  int blk;
  const SegDesc s = seg_of(T, part_block(T, blk));
  const RunDesc r = run_of(T, s.run);
  int key[SORT_ITEMS];
  int64_t p[SORT_ITEMS];
  block_keys<R, DIM>(s, r, blk, key, p);
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    int len, head;
    if (wave_runs(key[it], key[it] >= 0, len, head)) atomicAdd(&counts[key[it]], len);
  }
}

// Spread placement inside a bin (on request): the particle of rank r (arrival order,
// roughly the previous order, e.g. grouped by cell as loaded) goes to slot r*P mod N with P
// the inverse of Q mod N and Q ~ N/64 coprime to N.  Slot s then holds rank s*Q mod N, so
// the 64 particles a wavefront reads together come from 64 different stretches of the bin
// -- different cells -- and their current goes to different LDS addresses.  Without the
// request P = 1: ranks are slots and writes stay contiguous.
__device__ __forceinline__ int64_t gcd64(int64_t a, int64_t b) {
  while (b) { const int64_t t = a % b; a = b; b = t; }
  return a;
}
__device__ __forceinline__ int32_t spread_multiplier(int32_t n) {
  if (n <= 64) return 1;
  int64_t q = n >> 6;
  while (gcd64(q, n) != 1) ++q;
  // inverse of q modulo n (extended Euclid)
  int64_t t0 = 0, t1 = 1, r0 = n, r1 = q;
  while (r1) {
    const int64_t k = r0 / r1;
    int64_t t = t0 - k * t1; t0 = t1; t1 = t;
    t = r0 - k * r1; r0 = r1; r1 = t;
  }
  if (t0 < 0) t0 += n;
  return (int32_t)t0;
}

// Exclusive scan of the bin counts by one workgroup; clears the counts for the next sort
// and records each bin's placement multiplier.
__global__ __launch_bounds__(1024) void k_scan_bins(int32_t* counts, int32_t* offsets,
                                                    int32_t* cursor, int32_t* mult, int nbins,
                                                    int spread) {
  __shared__ int32_t wsum[16];
  const int tid = threadIdx.x;
  const int per = (nbins + 1023) / 1024;
  const int b0 = tid * per, b1 = min(nbins, b0 + per);
  int32_t local = 0;
  for (int b = b0; b < b1; ++b) local += counts[b];
  // block exclusive scan of `local`
  const int lane = tid & 63, wid = tid >> 6;
  int32_t incl = local;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int32_t o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  if (tid < 64) {
    int32_t v = tid < 16 ? wsum[tid] : 0;
    int32_t vi = v;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      int32_t o = __shfl_up(vi, off, 64);
      if (lane >= off) vi += o;
    }
    if (tid < 16) wsum[tid] = vi - v;
  }
  __syncthreads();
  int32_t run = wsum[wid] + incl - local;
  for (int b = b0; b < b1; ++b) {
    const int32_t c = counts[b];
    offsets[b] = run;
    cursor[b] = run;
    mult[b] = spread ? spread_multiplier(c) : 1;
    counts[b] = 0;
    run += c;
  }
  if (tid == 1023) offsets[nbins] = run;
}

template <class V>
__device__ __forceinline__ void move_items(const int64_t p[SORT_ITEMS],
                                           const int64_t dst[SORT_ITEMS], const V* from, V* to) {
  V v[SORT_ITEMS];
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it)
    if (dst[it] >= 0) v[it] = gp(from)[p[it]];
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it)
    if (dst[it] >= 0) gp(to)[dst[it]] = v[it];
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_sort_scatter(Tables T, int32_t* cursor,
                                                      const int32_t* offsets,
                                                      const int32_t* mult, int spread) {
  int blk;
  const SegDesc s = seg_of(T, part_block(T, blk));
  const RunDesc r = run_of(T, s.run);
  int key[SORT_ITEMS];
  int64_t p[SORT_ITEMS];
  block_keys<R, DIM>(s, r, blk, key, p);
  // destinations: one cursor atomic per run of equal keys in a wave
  int64_t dst[SORT_ITEMS];
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    int len, head;
    int base = 0;
    if (wave_runs(key[it], key[it] >= 0, len, head)) base = atomicAdd(&cursor[key[it]], len);
    base = __shfl(base, head, 64);
    dst[it] = -1;
    if (key[it] >= 0) {
      const int64_t slot = (int64_t)base + (__lane_id() - head);
      if (spread) {
        const int32_t b0 = offsets[key[it]], nb = offsets[key[it] + 1] - b0;
        dst[it] = b0 + ((slot - b0) * mult[key[it]]) % nb - s.pbase;
      } else {
        dst[it] = slot - s.pbase;
      }
    }
  }
  // move the particle arrays, one array at a time for all items (loads issued together)
  if constexpr (sizeof(R) == 4) {
    move_items(p, dst, (const int32_t*)s.p[P_CELL], (int32_t*)s.alt[P_CELL]);
#pragma unroll
    for (int d = 0; d < DIM; ++d) move_items(p, dst, (const float*)s.p[P_OX + d], (float*)s.alt[P_OX + d]);
  } else {
#pragma unroll
    for (int d = 0; d < DIM; ++d) move_items(p, dst, (const double*)s.p[P_X + d], (double*)s.alt[P_X + d]);
  }
#pragma unroll
  for (int q = P_UX; q <= P_W; ++q) move_items(p, dst, (const R*)s.p[q], (R*)s.alt[q]);
}

// After a sort inside a simulation, the device segment table points at the sorted buffers.
__global__ void k_swap_segments(SegDesc* segs, int nsegs) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsegs) return;
  for (int q = 0; q < P_NUM; ++q) {
    void* t = segs[s].p[q];
    segs[s].p[q] = segs[s].alt[q];
    segs[s].alt[q] = t;
  }
}

// Work list of the fused kernel: every tile's particle range cut into chunks.
__device__ __forceinline__ int seg_of_bin(const Tables& T, int bin) {
  if (!T.segs) return 0;
  int lo = 0, hi = T.nsegs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (T.segs[mid].bin_base <= bin) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(1024) void k_build_chunks(Tables T, const int32_t* offsets,
                                                       int nbins, int chunk, Chunk* out,
                                                       int32_t* nchunks) {
  __shared__ int32_t wsum[16];
  const int tid = threadIdx.x;
  const int per = (nbins + 1023) / 1024;
  const int b0 = tid * per, b1 = min(nbins, b0 + per);
  int32_t local = 0;
  for (int b = b0; b < b1; ++b) {
    const SegDesc& s = seg_of(T, seg_of_bin(T, b));
    const int tile = b - s.bin_base;
    if (tile >= run_of(T, s.run).ntiles) continue;   // dead bin
    const int32_t cnt = offsets[b + 1] - offsets[b];
    local += (cnt + chunk - 1) / chunk;
  }
  const int lane = tid & 63, wid = tid >> 6;
  int32_t incl = local;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int32_t o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  if (tid < 64) {
    int32_t v = tid < 16 ? wsum[tid] : 0;
    int32_t vi = v;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      int32_t o = __shfl_up(vi, off, 64);
      if (lane >= off) vi += o;
    }
    if (tid < 16) wsum[tid] = vi - v;
  }
  __syncthreads();
  int32_t pos = wsum[wid] + incl - local;
  for (int b = b0; b < b1; ++b) {
    const int si = seg_of_bin(T, b);
    const SegDesc& s = seg_of(T, si);
    const int tile = b - s.bin_base;
    if (tile >= run_of(T, s.run).ntiles) continue;
    const int32_t o0 = offsets[b] - (int32_t)s.pbase, o1 = offsets[b + 1] - (int32_t)s.pbase;
    for (int32_t a = o0; a < o1; a += chunk) {
      Chunk c;
      c.seg = si;
      c.tile = tile;
      c.beg = a;
      c.end = min(o1, a + chunk);
      out[pos++] = c;
    }
  }
  if (tid == 1023) *nchunks = pos;
}

// =======================================================================================
// Fused gather + push + deposit (unified pusher).  One workgroup per chunk; the chunk's
// field tile (tile + halo) is staged in LDS, the current accumulates in LDS and is flushed
// once.  Workgroups are mapped to chunks so that each XCD (every 8th workgroup) walks a
// contiguous range of chunks: neighbouring tiles share that XCD's L2.
// =======================================================================================
// Region geometries compiled with constant strides: (tile x, y, z, halo).  Geometry 0 is the
// runtime-stride kernel used for every other tiling.
struct GeoFix { int tx, ty, tz, halo; };
__host__ __device__ constexpr GeoFix geo_table(int g) {
  return g == 1 ? GeoFix{16, 16, 1, 5} : g == 2 ? GeoFix{8, 8, 1, 5} : g == 3 ? GeoFix{32, 32, 1, 5}
       : g == 4 ? GeoFix{16, 16, 1, 4} : g == 5 ? GeoFix{8, 8, 8, 4} : g == 6 ? GeoFix{8, 8, 4, 4}
       : GeoFix{0, 0, 0, 0};
}
constexpr int NUM_GEO = 7;

template <int DIM, int G>
struct GeoStrides {
  static constexpr GeoFix f = geo_table(G);
  using type = FixStrides<f.tx + 2 * f.halo, f.ty + 2 * f.halo, DIM == 3 ? f.tz + 2 * f.halo : 1>;
};
template <int DIM>
struct GeoStrides<DIM, 0> {
  using type = DynStrides;
};

// One staged region: the home tile of a run plus `halo` cells, in LDS.
struct Region {
  int r0[3];     // global origin (may be negative: periodic)
  int rw[3];     // extent
};

template <int DIM>
__device__ __forceinline__ Region region_of(const RunDesc& r, const SegDesc& s, int tile) {
  Region g;
  const int TXs[3] = {1 << s.lx, 1 << s.ly, DIM == 3 ? (1 << s.lz) : 1};
  int tc[3];
  tc[0] = tile % r.ntx; tile /= r.ntx;
  tc[1] = tile % r.nty;
  tc[2] = tile / r.nty;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d < DIM) { g.r0[d] = tc[d] * TXs[d] - s.halo; g.rw[d] = TXs[d] + 2 * s.halo; }
    else { g.r0[d] = 0; g.rw[d] = 1; }
  }
  return g;
}

__device__ __forceinline__ int64_t region_global(const RunDesc& r, const Region& g, int e) {
  const int lx = e % g.rw[0];
  const int rest = e / g.rw[0];
  const int ly = rest % g.rw[1];
  const int lz = rest / g.rw[1];
  return ((int64_t)wrapm(g.r0[2] + lz, r.nz) * r.ny + wrapm(g.r0[1] + ly, r.ny)) * r.nx +
         wrapm(g.r0[0] + lx, r.nx);
}

// Stage E and B of the region, clear its current (and charge) planes.
template <typename R>
__device__ __forceinline__ void stage_region(const RunDesc& r, const Region& g, int plane,
                                             int njplanes, R* sm, double* jm) {
  gptr<R> F[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) F[c] = gp((R*)r.f[c]);
  for (int e = threadIdx.x; e < plane; e += blockDim.x) {
    const int64_t gi = region_global(r, g, e);
#pragma unroll
    for (int c = 0; c < 6; ++c) sm[c * plane + e] = F[c][gi];
    for (int c = 0; c < njplanes; ++c) jm[c * plane + e] = 0.0;
  }
}

// Add the region's current (and charge) into the global arrays: one atomic per non-zero
// entry, converted to the field precision.
template <typename R>
__device__ __forceinline__ void flush_region(const RunDesc& r, const Region& g, int plane,
                                             int njplanes, const double* jm) {
  gptr<R> F[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) F[c] = gp((R*)r.f[F_JX + c]);
  for (int e = threadIdx.x; e < plane; e += blockDim.x) {
    const int64_t gi = region_global(r, g, e);
    for (int c = 0; c < njplanes; ++c) {
      const double v = jm[c * plane + e];
      if (v != 0.0) atomic_add_global(F[c] + gi, R(v));
    }
  }
}

__device__ __forceinline__ void escape_append(const EscapeList& esc, bool want, int seg,
                                              int32_t p) {
  const uint64_t mask = __ballot(want);
  if (!mask) return;
  const int lane = __lane_id();
  const int leader = __ffsll((unsigned long long)mask) - 1;
  unsigned int base = 0;
  if (lane == leader) base = atomicAdd(esc.count, (unsigned int)__popcll(mask));
  base = __shfl(base, leader, 64);
  if (want) {
    const unsigned int k = base + (unsigned int)__popcll(mask & ((1ull << lane) - 1ull));
    if ((int64_t)k < esc.capacity) esc.items[k] = ((unsigned long long)seg << 32) | (unsigned long long)p;
  }
}

// The particles of one chunk against the staged region, in rounds: each thread first
// issues the loads of BATCH particles (256 apart, so every load instruction reads 64
// consecutive particles) and then pushes them one by one, so HBM latency is paid once per
// round rather than once per particle.  Returns the summed w m u^2/(1+gamma).
constexpr int BATCH = 4;

template <typename R, int DIM, int ORDER, class ST>
__device__ __forceinline__ double process_chunk(const RunDesc& r, const SegDesc& s, int seg,
                                                const Chunk& ch, const Region& g,
                                                const LdsAcc<R, ST>& L, int with_rho,
                                                bool want_ke, const EscapeList& esc) {
  const int n[3] = {r.nx, r.ny, r.nz};
  const PushConst<R> k = push_const<R>(r, s);
  const PartPtrs<R> q = part_ptrs<R>(s, r);
  double ke = 0.0;
  const int32_t span = (int32_t)blockDim.x * BATCH;
  for (int32_t base = ch.beg; base < ch.end; base += span) {
    PState<R> ps[BATCH];
    int32_t pi[BATCH];
    bool ok[BATCH];
#pragma unroll
    for (int b = 0; b < BATCH; ++b) {
      pi[b] = base + b * (int32_t)blockDim.x + (int32_t)threadIdx.x;
      ok[b] = pi[b] < ch.end;
      if (ok[b]) load_particle<R, DIM>(q, pi[b], ps[b]);
    }
#pragma unroll
    for (int b = 0; b < BATCH; ++b) {
      bool inside = ok[b] && ps[b].alive;
      int a[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (d < DIM) {
          // local start cell; gather and deposit touch cells [a-3, a+4] per axis
          int v = ps[b].c[d] - g.r0[d];
          v = v < 0 ? v + n[d] : (v >= n[d] ? v - n[d] : v);
          a[d] = v;
          inside = inside && v >= 3 && v <= g.rw[d] - 5;
        } else {
          a[d] = 0;
        }
      }
      escape_append(esc, ok[b] && ps[b].alive && !inside, seg, pi[b]);
      if (!inside) continue;
      int pcell[3];
      R po[3], pe[3], x1[3], vz1, g1;
      push<DIM, ORDER>(L, a, ps[b], k, pcell, po, pe, x1, vz1, g1);
      deposit<DIM, ORDER>(L, pcell, po, pe, ps[b].w, vz1, k, with_rho != 0);
#pragma unroll
      for (int d = 0; d < DIM; ++d) advance_cell<R>(ps[b].c[d], ps[b].o[d], x1[d], n[d]);
      store_particle<R, DIM>(q, pi[b], ps[b]);
      if (want_ke) {   // diagnostic steps only
        const double u2 = (double)ps[b].u[0] * ps[b].u[0] + (double)ps[b].u[1] * ps[b].u[1] +
                          (double)ps[b].u[2] * ps[b].u[2];
        ke += (double)ps[b].w * u2 / (1.0 + (double)g1);
      }
    }
  }
  return ke * s.m;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  T t = T(0);
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  return t;
}

// Fused gather + push + deposit over the chunk table, persistent: the grid is a multiple of
// 8 and XCD x (workgroups x, x+8, ...) owns the contiguous chunk range [x*per, (x+1)*per),
// split into equal contiguous slices per workgroup.  Consecutive chunks of one tile (and of
// the other species of the same box, which follow in the table) reuse the staged region;
// the region is flushed when the tile changes.
template <typename R, int DIM, int G>
__global__ __launch_bounds__(256) void k_fused(Tables T, const Chunk* chunks,
                                               const int32_t* nchunks, int with_rho,
                                               double* kinetic, int ke_to_diag,
                                               EscapeList esc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[4];
  R* sm = (R*)smem_raw;
  const int nch = uniform(*nchunks);
  const int nb8 = gridDim.x >> 3;
  const int per = (nch + 7) >> 3;
  const int q = (per + nb8 - 1) / nb8;
  const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
  const int lo = xcd * per + j * q;
  const int hi = min(min(lo + q, (xcd + 1) * per), nch);
  if (lo >= hi) return;

  using ST = typename GeoStrides<DIM, G>::type;
  const SegDesc& s0 = seg_of(T, uniform(chunks[lo].seg));
  ST st;
  if constexpr (G == 0) {
    const int rw = (1 << s0.lx) + 2 * s0.halo, rh = (1 << s0.ly) + 2 * s0.halo;
    const int rd = DIM == 3 ? (1 << s0.lz) + 2 * s0.halo : 1;
    st.sy_ = rw;
    st.sz_ = rw * rh;
    st.plane_ = rw * rh * rd;
  }
  const int plane = st.plane();
  const int njplanes = 3 + (with_rho ? 2 : 0);
  double* jm = (double*)(sm + 6 * plane + (plane & 1));   // 8-byte aligned after the fields
  LdsAcc<R, ST> L;
  L.fbase = sm;
  L.jbase = jm;
  L.st = st;

  int cur_run = -1, cur_tile = -1;
  Region g;
  double ke = 0.0;
  for (int c = lo; c < hi; ++c) {
    Chunk ch = chunks[c];
    ch.seg = uniform(ch.seg);
    ch.tile = uniform(ch.tile);
    ch.beg = uniform(ch.beg);
    ch.end = uniform(ch.end);
    const SegDesc s = seg_of(T, ch.seg);
    if (s.run != cur_run || ch.tile != cur_tile) {
      if (cur_run >= 0) {
        const RunDesc& rp = run_of(T, cur_run);
        __syncthreads();
        flush_region<R>(rp, g, plane, njplanes, jm);
        if (kinetic || ke_to_diag) {
          const double t = block_sum(ke, red);
          if (threadIdx.x == 0) atomic_add_global(ke_to_diag ? rp.diag + DIAG_UKIN : kinetic, t);
          ke = 0.0;
        }
      }
      const RunDesc rn = run_of(T, s.run);
      g = region_of<DIM>(rn, s, ch.tile);
      __syncthreads();
      stage_region<R>(rn, g, plane, njplanes, sm, jm);
      __syncthreads();
      cur_run = s.run;
      cur_tile = ch.tile;
    }
    const RunDesc r = run_of(T, s.run);
    const bool want_ke = kinetic || ke_to_diag;
    ke += s.order == 1 ? process_chunk<R, DIM, 1>(r, s, ch.seg, ch, g, L, with_rho, want_ke, esc)
                       : process_chunk<R, DIM, 2>(r, s, ch.seg, ch, g, L, with_rho, want_ke, esc);
  }
  const RunDesc& rl = run_of(T, cur_run);
  __syncthreads();
  flush_region<R>(rl, g, plane, njplanes, jm);
  if (kinetic || ke_to_diag) {
    const double t = block_sum(ke, red);
    if (threadIdx.x == 0) atomic_add_global(ke_to_diag ? rl.diag + DIAG_UKIN : kinetic, t);
  }
}

// Escaped particles: the same push and deposit through global memory.  The last workgroup
// to finish clears the list for the next step.
template <typename R, int DIM, int ORDER>
__device__ __forceinline__ double escape_one(const RunDesc& r, const SegDesc& s, int64_t p,
                                             int with_rho) {
  PState<R> ps;
  load_particle<R, DIM>(s, r, p, ps);
  if (!ps.alive) return 0.0;
  const GlobalAcc<R> G = global_acc<R>(r);
  const PushConst<R> k = push_const<R>(r, s);
  int pcell[3];
  R po[3], pe[3], x1[3], vz1, g1;
  push<DIM, ORDER>(G, ps.c, ps, k, pcell, po, pe, x1, vz1, g1);
  deposit<DIM, ORDER>(G, pcell, po, pe, ps.w, vz1, k, with_rho != 0);
  const int n[3] = {r.nx, r.ny, r.nz};
#pragma unroll
  for (int d = 0; d < DIM; ++d) advance_cell<R>(ps.c[d], ps.o[d], x1[d], n[d]);
  store_particle<R, DIM>(s, r, p, ps);
  const double u2 = (double)ps.u[0] * ps.u[0] + (double)ps.u[1] * ps.u[1] + (double)ps.u[2] * ps.u[2];
  return (double)ps.w * s.m * u2 / (1.0 + (double)g1);
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_escape(Tables T, int with_rho, double* kinetic,
                                                int ke_to_diag, EscapeList esc) {
  const unsigned int cnt = min((int64_t)esc.count[0], esc.capacity);
  for (unsigned int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += gridDim.x * blockDim.x) {
    const unsigned long long v = esc.items[i];
    const int seg = (int)(v >> 32);
    const int64_t p = (int64_t)(v & 0xffffffffull);
    const SegDesc& s = seg_of(T, seg);
    const RunDesc& r = run_of(T, s.run);
    const double ke = s.order == 1 ? escape_one<R, DIM, 1>(r, s, p, with_rho)
                                   : escape_one<R, DIM, 2>(r, s, p, with_rho);
    if (kinetic || ke_to_diag) atomic_add_global(ke_to_diag ? r.diag + DIAG_UKIN : kinetic, ke);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned int done = atomicAdd(esc.count + 1, 1u);
    if (done == gridDim.x - 1) {
      atomicAdd(esc.total, (unsigned long long)esc.count[0]);
      atomicExch(esc.count, 0u);
      atomicExch(esc.count + 1, 0u);
    }
  }
}

// =======================================================================================
// FP64 diagnostics: field energy, continuity and Gauss residuals (max over cells).
// =======================================================================================
__device__ __forceinline__ void atomic_max_nonneg(double* p, double v) {
  atomicMax((unsigned long long*)p, (unsigned long long)__double_as_longlong(v));
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_reduce_fields(Tables T, int with_rho, double* out) {
  int blk;
  const int ri = cell_block(T, blk);
  const RunDesc& r = run_of(T, ri);
  double* o = out ? out : r.diag;
  CellIdx x;
  double en = 0.0, res = 0.0, rm = 0.0, ga = 0.0;
  if (cell_index(r, blk, DIM, x)) {
    gptr<R> f[F_NUM];
#pragma unroll
    for (int c = 0; c < F_NUM; ++c) f[c] = gp((R*)r.f[c]);
    for (int c = 0; c < 6; ++c) {
      const double v = (double)f[c][x.c];
      en += v * v;
    }
    if (with_rho) {
      const double r0 = (double)f[F_R0][x.c], r1 = (double)f[F_R1][x.c];
      double divj = ((double)f[F_JX][x.c] - (double)f[F_JX][x.cim]) / r.dx +
                    ((double)f[F_JY][x.c] - (double)f[F_JY][x.cjm]) / r.dy;
      double dive = ((double)f[F_EX][x.c] - (double)f[F_EX][x.cim]) / r.dx +
                    ((double)f[F_EY][x.c] - (double)f[F_EY][x.cjm]) / r.dy;
      if (DIM == 3) {
        divj += ((double)f[F_JZ][x.c] - (double)f[F_JZ][x.ckm]) / r.dz;
        dive += ((double)f[F_EZ][x.c] - (double)f[F_EZ][x.ckm]) / r.dz;
      }
      res = fabs(r1 - r0 + r.dt * divj);
      rm = fabs(r1);
      ga = fabs(dive - 0.5 * (r0 + r1) - r.rho_bg);
    }
  }
  __shared__ double red[4][4];
  en = wave_sum(en);
  res = wave_max(res);
  rm = wave_max(rm);
  ga = wave_max(ga);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { red[0][w] = en; red[1][w] = res; red[2][w] = rm; red[3][w] = ga; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0, c = 0, d = 0;
    for (int i = 0; i < 4; ++i) {
      a += red[0][i];
      b = fmax(b, red[1][i]);
      c = fmax(c, red[2][i]);
      d = fmax(d, red[3][i]);
    }
    const double dV = r.dx * r.dy * (DIM == 3 ? r.dz : 1.0);
    atomic_add_global(o + (out ? 0 : DIAG_UFIELD), 0.5 * a * dV);
    if (with_rho) {
      atomic_max_nonneg(o + (out ? 1 : DIAG_RES), b);
      atomic_max_nonneg(o + (out ? 2 : DIAG_RHOMAX), c);
      atomic_max_nonneg(o + (out ? 3 : DIAG_GAUSS), d);
    }
  }
}

__global__ void k_zero_doubles(double* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void k_diag_clear(Tables T) {
  const int r = blockIdx.x;
  const RunDesc& rd = run_of(T, r);
  if (threadIdx.x < DIAG_NUM && rd.diag) rd.diag[threadIdx.x] = 0.0;
}

// =======================================================================================
// Position representation <-> absolute FP64 coordinates.
// =======================================================================================
template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_load_positions(Tables T, const double* x,
                                                        const double* y, const double* z) {
  int blk;
  const SegDesc& s = seg_of(T, part_block(T, blk));
  const RunDesc& r = run_of(T, s.run);
  const int64_t p = (int64_t)blk * 256 + threadIdx.x;
  if (p >= s.n) return;
  const double* src[3] = {x, y, z};
  if constexpr (sizeof(R) == 4) {
    if (!(x[p] >= 0.0)) {
      ((int32_t*)s.p[P_CELL])[p] = -1;
      return;
    }
    const double h[3] = {r.dx, r.dy, r.dz};
    const int n[3] = {r.nx, r.ny, r.nz};
    int c[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) {
      const double X = src[d][p] / h[d];
      if (!(X >= 0.0 && X <= (double)n[d])) {    // outside the box: dead slot
        ((int32_t*)s.p[P_CELL])[p] = -1;
        return;
      }
      const double f = floor(X);
      int ci = (int)f;
      float o = (float)(X - f);
      if (o >= 1.0f) { o = 0.0f; ci += 1; }
      ci = ci >= n[d] ? ci - n[d] : ci;
      c[d] = ci;
      ((float*)s.p[P_OX + d])[p] = o;
    }
    ((int32_t*)s.p[P_CELL])[p] = pack_cell(c, DIM);
  } else {
    for (int d = 0; d < DIM; ++d) ((double*)s.p[P_X + d])[p] = src[d][p];
  }
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_store_positions(Tables T, double* x, double* y,
                                                         double* z) {
  int blk;
  const SegDesc& s = seg_of(T, part_block(T, blk));
  const RunDesc& r = run_of(T, s.run);
  const int64_t p = (int64_t)blk * 256 + threadIdx.x;
  if (p >= s.n) return;
  double* dst[3] = {x, y, z};
  if constexpr (sizeof(R) == 4) {
    const int32_t cell = ((const int32_t*)s.p[P_CELL])[p];
    if (cell < 0) {
      for (int d = 0; d < DIM; ++d) dst[d][p] = -1.0;
      return;
    }
    int c[3];
    unpack_cell(cell, DIM, c);
    const double h[3] = {r.dx, r.dy, r.dz};
    for (int d = 0; d < DIM; ++d)
      dst[d][p] = ((double)c[d] + (double)((const float*)s.p[P_OX + d])[p]) * h[d];
  } else {
    for (int d = 0; d < DIM; ++d) dst[d][p] = ((const double*)s.p[P_X + d])[p];
  }
}

// =======================================================================================
// Host-side launchers
// =======================================================================================
template <typename R, int DIM>
static void launch_yee_t(const Tables& T, int nblocks, int which, double frac, int zero_j,
                         hipStream_t st) {
  if (which == 0) k_yee_e<R, DIM><<<nblocks, 256, 0, st>>>(T, frac, zero_j);
  else k_yee_b<R, DIM><<<nblocks, 256, 0, st>>>(T, frac);
}

void launch_yee(const Tables& T, int prec, int dim, int nblocks, int which, double frac,
                int zero_j, hipStream_t st) {
  if (prec == 0) {
    if (dim == 2) launch_yee_t<float, 2>(T, nblocks, which, frac, zero_j, st);
    else launch_yee_t<float, 3>(T, nblocks, which, frac, zero_j, st);
  } else {
    if (dim == 2) launch_yee_t<double, 2>(T, nblocks, which, frac, zero_j, st);
    else launch_yee_t<double, 3>(T, nblocks, which, frac, zero_j, st);
  }
}

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

void launch_gather_push(const Tables& T, int prec, int dim, int nblocks, void* old,
                        hipStream_t st) {
  LPIC_PD(prec, dim, (k_gather_push<R, D><<<nblocks, 256, 0, st>>>(T, old)));
}

void launch_deposit(const Tables& T, int prec, int dim, int nblocks, const void* old,
                    int with_rho, hipStream_t st) {
  LPIC_PD(prec, dim, (k_deposit<R, D><<<nblocks, 256, 0, st>>>(T, old, with_rho)));
}

void launch_zero_u32(uint32_t* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  k_fill_zero_u32<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n);
}

void launch_sort(const Tables& T, int prec, int dim, int nblocks, int32_t* counts,
                 int32_t* offsets, int32_t* cursor, int32_t* mult, int nbins, int spread,
                 hipStream_t st) {
  LPIC_PD(prec, dim, (k_sort_count<R, D><<<nblocks, 256, 0, st>>>(T, counts)));
  k_scan_bins<<<1, 1024, 0, st>>>(counts, offsets, cursor, mult, nbins, spread);
  LPIC_PD(prec, dim, (k_sort_scatter<R, D><<<nblocks, 256, 0, st>>>(T, cursor, offsets, mult,
                                                                     spread)));
}

void launch_swap_segments(SegDesc* segs, int nsegs, hipStream_t st) {
  k_swap_segments<<<(nsegs + 63) / 64, 64, 0, st>>>(segs, nsegs);
}

void launch_build_chunks(const Tables& T, const int32_t* offsets, int nbins, int chunk,
                         Chunk* out, int32_t* nchunks, hipStream_t st) {
  k_build_chunks<<<1, 1024, 0, st>>>(T, offsets, nbins, chunk, out, nchunks);
}

int fused_geometry(int dim, int tx, int ty, int tz, int halo) {
  for (int g = 1; g < NUM_GEO; ++g) {
    const GeoFix f = geo_table(g);
    if (dim == 2 && f.tz == 1 && f.tx == tx && f.ty == ty && f.halo == halo) return g;
    if (dim == 3 && f.tz > 1 && f.tx == tx && f.ty == ty && f.tz == tz && f.halo == halo) return g;
  }
  return 0;
}

template <typename R, int D, int G>
static void launch_fused_g(const Tables& T, int nblocks, size_t smem, const Chunk* chunks,
                           const int32_t* nchunks, int with_rho, double* kinetic, int ke_to_diag,
                           const EscapeList& esc, hipStream_t st) {
  k_fused<R, D, G><<<nblocks, 256, smem, st>>>(T, chunks, nchunks, with_rho, kinetic,
                                               ke_to_diag, esc);
}

template <typename R, int D>
static void launch_fused_d(int geo, const Tables& T, int nblocks, size_t smem,
                           const Chunk* chunks, const int32_t* nchunks, int with_rho,
                           double* kinetic, int ke_to_diag, const EscapeList& esc,
                           hipStream_t st) {
#define LPIC_GEO(g) launch_fused_g<R, D, g>(T, nblocks, smem, chunks, nchunks, with_rho, kinetic, ke_to_diag, esc, st)
  if constexpr (D == 2) {
    switch (geo) {
      case 1: LPIC_GEO(1); return;
      case 2: LPIC_GEO(2); return;
      case 3: LPIC_GEO(3); return;
      case 4: LPIC_GEO(4); return;
      default: LPIC_GEO(0); return;
    }
  } else {
    switch (geo) {
      case 5: LPIC_GEO(5); return;
      case 6: LPIC_GEO(6); return;
      default: LPIC_GEO(0); return;
    }
  }
#undef LPIC_GEO
}

void launch_fused(const Tables& T, int prec, int dim, int geo, int nblocks, size_t smem,
                  const Chunk* chunks, const int32_t* nchunks, int with_rho, double* kinetic,
                  int ke_to_diag, const EscapeList& esc, hipStream_t st) {
  LPIC_PD(prec, dim, (launch_fused_d<R, D>(geo, T, nblocks, smem, chunks, nchunks, with_rho,
                                           kinetic, ke_to_diag, esc, st)));
  LPIC_PD(prec, dim, (k_escape<R, D><<<ESCAPE_BLOCKS, 256, 0, st>>>(T, with_rho, kinetic,
                                                                    ke_to_diag, esc)));
}

template <typename R, int D, int G>
static hipError_t set_smem(size_t smem, int* blocks_per_cu) {
  hipError_t e = hipFuncSetAttribute((const void*)k_fused<R, D, G>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_fused<R, D, G>, 256, smem);
}

hipError_t prepare_fused(int prec, int dim, int geo, size_t smem, int* blocks_per_cu) {
  hipError_t e = hipSuccess;
  int* b = blocks_per_cu;
  if (dim == 2) {
    switch (geo) {
      case 1: e = prec == 0 ? set_smem<float, 2, 1>(smem, b) : set_smem<double, 2, 1>(smem, b); break;
      case 2: e = prec == 0 ? set_smem<float, 2, 2>(smem, b) : set_smem<double, 2, 2>(smem, b); break;
      case 3: e = prec == 0 ? set_smem<float, 2, 3>(smem, b) : set_smem<double, 2, 3>(smem, b); break;
      case 4: e = prec == 0 ? set_smem<float, 2, 4>(smem, b) : set_smem<double, 2, 4>(smem, b); break;
      default: e = prec == 0 ? set_smem<float, 2, 0>(smem, b) : set_smem<double, 2, 0>(smem, b); break;
    }
  } else {
    switch (geo) {
      case 5: e = prec == 0 ? set_smem<float, 3, 5>(smem, b) : set_smem<double, 3, 5>(smem, b); break;
      case 6: e = prec == 0 ? set_smem<float, 3, 6>(smem, b) : set_smem<double, 3, 6>(smem, b); break;
      default: e = prec == 0 ? set_smem<float, 3, 0>(smem, b) : set_smem<double, 3, 0>(smem, b); break;
    }
  }
  return e;
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_kinetic(Tables T, double* out) {
  int blk;
  const SegDesc& s = seg_of(T, part_block(T, blk));
  const RunDesc& r = run_of(T, s.run);
  const int64_t p = (int64_t)blk * 256 + threadIdx.x;
  double ke = 0.0;
  if (p < s.n) {
    PState<R> ps;
    load_particle<R, DIM>(s, r, p, ps);
    if (ps.alive) {
      const double u2 = (double)ps.u[0] * ps.u[0] + (double)ps.u[1] * ps.u[1] +
                        (double)ps.u[2] * ps.u[2];
      ke = (double)ps.w * s.m * u2 / (1.0 + sqrt(1.0 + u2));
    }
  }
  __shared__ double red[4];
  ke = wave_sum(ke);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ke;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = red[0] + red[1] + red[2] + red[3];
    atomic_add_global(out ? out : r.diag + DIAG_UKIN, t);
  }
}

void launch_kinetic(const Tables& T, int prec, int dim, int nblocks, double* out,
                    hipStream_t st) {
  LPIC_PD(prec, dim, (k_kinetic<R, D><<<nblocks, 256, 0, st>>>(T, out)));
}

void launch_reduce_fields(const Tables& T, int prec, int dim, int nblocks, int with_rho,
                          double* out, hipStream_t st) {
  LPIC_PD(prec, dim, (k_reduce_fields<R, D><<<nblocks, 256, 0, st>>>(T, with_rho, out)));
}

void launch_zero_doubles(double* p, int n, hipStream_t st) {
  k_zero_doubles<<<(n + 255) / 256, 256, 0, st>>>(p, n);
}

void launch_diag_clear(const Tables& T, int nruns, hipStream_t st) {
  k_diag_clear<<<nruns, 64, 0, st>>>(T);
}

void launch_load_positions(const Tables& T, int prec, int dim, int nblocks, const double* x,
                           const double* y, const double* z, hipStream_t st) {
  LPIC_PD(prec, dim, (k_load_positions<R, D><<<nblocks, 256, 0, st>>>(T, x, y, z)));
}

void launch_store_positions(const Tables& T, int prec, int dim, int nblocks, double* x,
                            double* y, double* z, hipStream_t st) {
  LPIC_PD(prec, dim, (k_store_positions<R, D><<<nblocks, 256, 0, st>>>(T, x, y, z)));
}

size_t fused_smem_bytes(int prec, int dim, int tx, int ty, int tz, int halo, int with_rho) {
  const size_t plane = (size_t)(tx + 2 * halo) * (ty + 2 * halo) * (dim == 3 ? (tz + 2 * halo) : 1);
  // six field planes in the kernel precision (padded to 8 bytes), then FP64 current planes
  return (plane * 6 + (plane & 1)) * (prec == 0 ? 4 : 8) + plane * (3 + (with_rho ? 2 : 0)) * 8;
}

}  // namespace lpic
