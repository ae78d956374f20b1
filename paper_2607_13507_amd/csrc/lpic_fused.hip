// The fused particle kernel of the PIC hot path (gfx950, wave64): gather + relativistic
// Boris push + Esirkepov deposit in one pass over a tile-sorted particle stream, with the
// field tile staged in LDS and the tile's current accumulated in LDS (64-bit fixed point on
// the FP32 path, FP64 on the FP64 path) before one global atomic flush per non-zero entry;
// plus the kernel that handles, through global memory, the particles whose stencils have
// left the staged region of their tile.
#include "lpic_internal.hpp"

namespace lpic {

// =======================================================================================
// Fused gather + push + deposit (unified pusher).  Persistent workgroups walk the chunk
// table; for each tile the field region (tile + halo) is staged in LDS once, the current
// accumulates in LDS and is flushed when the tile changes.  Workgroups are mapped to chunks
// so that each XCD (every 8th workgroup) walks a contiguous range of chunks: neighbouring
// tiles share that XCD's L2.
// =======================================================================================
// Region geometries compiled with constant strides: (tile x, y, z, halo, z-layer pad).
// Geometry 0 is the runtime-stride kernel used for every other tiling.  The 3D pads put
// consecutive z layers 4 (8 x 4 x 4 tiles: a 16 x 12 layer is 192 entries, 3 x 64) or 8
// (8 x 8 x 4 tiles: 256 entries) banks apart; the 8 x 4 x 4 pad is also the largest whose
// region, charge planes included, still fits the LDS.  Geometry 7 (8 x 4 x 4 tiles, halo 3)
// runs 512-thread workgroups, two per CU: it is also the second pass of the re-binned
// escape path for 8 x 4 x 4 tilings with halo 4 (its particles lie inside their present
// tile, so a halo of 3 always holds their stencils).  Geometry 8 is the same region without
// the layer pad, for the FP32 steps that carry one charge plane (chained charge, see
// k_fused): it still fits two 512-thread workgroups per CU (80.7 KB each).  Geometry 9 is
// the padded region with 1024-thread workgroups, for FP32 steps with both charge planes:
// they leave room for one workgroup per CU, which then brings all sixteen waves by itself.
struct GeoFix { int tx, ty, tz, halo, pz; };
__host__ __device__ constexpr GeoFix geo_table(int g) {
  return g == 1 ? GeoFix{16, 16, 1, 5, 0} : g == 2 ? GeoFix{8, 8, 1, 5, 0}
       : g == 3 ? GeoFix{32, 32, 1, 5, 0} : g == 4 ? GeoFix{16, 16, 1, 4, 0}
       : g == 5 ? GeoFix{8, 4, 4, 4, 4} : g == 6 ? GeoFix{8, 8, 4, 4, 8}
       : g == 7 ? GeoFix{8, 4, 4, 3, 8} : g == 8 ? GeoFix{8, 4, 4, 3, 0}
       : g == 9 ? GeoFix{8, 4, 4, 3, 8} : GeoFix{0, 0, 0, 0, 0};
}
constexpr int NUM_GEO = 10;   // fused_geometry() returns the first match: 7, never 8 or 9

template <int DIM, int G>
struct GeoStrides {
  static constexpr GeoFix f = geo_table(G);
  using type = FixStrides<f.tx + 2 * f.halo, f.ty + 2 * f.halo, DIM == 3 ? f.tz + 2 * f.halo : 1,
                          DIM == 3 ? f.pz : 0>;
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
__device__ __forceinline__ Region region_of(const RunDesc& r, const SegDesc& s, int tile,
                                            int halo) {
  Region g;
  const int TXs[3] = {1 << s.lx, 1 << s.ly, DIM == 3 ? (1 << s.lz) : 1};
  int tc[3];
  tc[0] = tile % r.ntx; tile /= r.ntx;
  tc[1] = tile % r.nty;
  tc[2] = tile / r.nty;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d < DIM) { g.r0[d] = tc[d] * TXs[d] - halo; g.rw[d] = TXs[d] + 2 * halo; }
    else { g.r0[d] = 0; g.rw[d] = 1; }
  }
  return g;
}

// The periodic wrap of a staged region (uniform per tile): the wrapped origin per axis,
// and whether some extent exceeds its box's (then a full modulo per cell, else one
// conditional subtraction).
struct RegionWrap {
  int o[3], n[3];
  bool wide;
};

__device__ __forceinline__ RegionWrap region_wrap(const RunDesc& r, const Region& g) {
  RegionWrap w;
  w.n[0] = r.nx; w.n[1] = r.ny; w.n[2] = r.nz;
  w.wide = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    w.o[d] = wrapm(g.r0[d], w.n[d]);
    w.wide = w.wide || g.rw[d] > w.n[d];
  }
  return w;
}

// Region cell e (x fastest over the region's extents): its global index, and its LDS entry
// li under the strides S (which may pad the z layers).  With the extents of a fixed
// geometry the decomposition divides by constants.
template <class S>
__device__ __forceinline__ int64_t region_cell(const RegionWrap& w, const S& st, int e,
                                               int& li) {
  const int lx = e % st.ex();
  const int rest = e / st.ex();
  const int ly = rest % st.ey();
  const int lz = rest / st.ey();
  li = lx + ly * st.sy() + lz * st.sz();
  int gx = w.o[0] + lx, gy = w.o[1] + ly, gz = w.o[2] + lz;
  if (w.wide) {
    gx %= w.n[0]; gy %= w.n[1]; gz %= w.n[2];
  } else {
    gx -= gx >= w.n[0] ? w.n[0] : 0;
    gy -= gy >= w.n[1] ? w.n[1] : 0;
    gz -= gz >= w.n[2] ? w.n[2] : 0;
  }
  return ((int64_t)gz * w.n[1] + gy) * w.n[0] + gx;
}

// Stage E and B of the region, clear its current (and charge) planes.  Each thread takes
// up to STAGE_BATCH region cells per pass and issues all their loads before the first LDS
// write, so a tile change costs about one memory latency rather than one per cell (a 3D
// region of 2304 cells is 2.25 cells per thread of a 1024-thread workgroup).
constexpr int STAGE_BATCH = 4;

template <typename R, class S>
__device__ __forceinline__ void stage_region(const RunDesc& r, const Region& g, const S& st,
                                             int njplanes, R* sm, double* jm, bool paired) {
  gptr<R> F[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) F[c] = gp((R*)r.f[c]);
  const int bd = (int)blockDim.x;
  const int plane = st.plane();
  const int ncell = g.rw[0] * g.rw[1] * g.rw[2];
  const RegionWrap w = region_wrap(r, g);
  for (int e0 = threadIdx.x; e0 < ncell; e0 += STAGE_BATCH * bd) {
    R v[STAGE_BATCH][6];
    int li[STAGE_BATCH];
#pragma unroll
    for (int k = 0; k < STAGE_BATCH; ++k) {
      const int e = e0 + k * bd;
      if (e < ncell) {
        const int64_t gi = region_cell(w, st, e, li[k]);
#pragma unroll
        for (int c = 0; c < 6; ++c) v[k][c] = F[c][gi];
      }
    }
#pragma unroll
    for (int k = 0; k < STAGE_BATCH; ++k) {
      if (e0 + k * bd < ncell) {
        const int e = li[k];
        if (paired) {   // 2D: (Ex,By) pairs, (Ey,Bx) pairs, Ez, Bz
          sm[2 * e] = v[k][F_EX];
          sm[2 * e + 1] = v[k][F_BY];
          sm[2 * (plane + e)] = v[k][F_EY];
          sm[2 * (plane + e) + 1] = v[k][F_BX];
          sm[4 * plane + e] = v[k][F_EZ];
          sm[5 * plane + e] = v[k][F_BZ];
        } else {
#pragma unroll
          for (int c = 0; c < 6; ++c) sm[c * plane + e] = v[k][c];
        }
        for (int c = 0; c < njplanes; ++c) jm[c * plane + e] = 0.0;
      }
    }
  }
}

// Add the region's current (and charge) into the global arrays: one atomic per non-zero
// entry, converted to the field precision (FP32 path: from fixed point, times 2^-S).  With
// a single charge plane (with_rho 2 or 3) it goes to rho0 or rho1.
template <typename R, class S>
__device__ __forceinline__ void flush_region(const RunDesc& r, const Region& g, const S& st,
                                             int njplanes, const double* jm, double unscale,
                                             int with_rho) {
  gptr<R> F[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) F[c] = gp((R*)r.f[F_JX + c]);
  if (with_rho == 3) F[3] = gp((R*)r.f[F_R1]);
  const int plane = st.plane();
  const int ncell = g.rw[0] * g.rw[1] * g.rw[2];
  const RegionWrap w = region_wrap(r, g);
  for (int i = threadIdx.x; i < ncell; i += blockDim.x) {
    int e;
    const int64_t gi = region_cell(w, st, i, e);
    for (int c = 0; c < njplanes; ++c) {
      double v;
      if constexpr (sizeof(R) == 4) v = (double)((const long long*)jm)[c * plane + e] * unscale;
      else v = jm[c * plane + e];
      if (v != 0.0) atomic_add_global(F[c] + gi, R(v));
    }
  }
}

// The second pass of the re-binned escape path: its chunk ranges index `list` (entries
// segment << 32 | slot) and, when set, `rec` (the same particles' escape records in the same
// order, read contiguously instead of the particles' scattered slots).
struct PassList {
  const unsigned long long* list;
  const void* rec;
};

// Append the lanes that want it to the escape list (one reservation per wave), with their
// escape records when the list keeps them (3D only: the 2D body has no registers to spare
// for the record's words, and 2D particles rarely leave their regions).
// Entry k of the escape list: the particle's record and the bin of the tile it is in.
template <typename R, int DIM>
__device__ __forceinline__ void escape_record(const EscapeList& esc, int64_t k,
                                              const RunDesc& r, const SegDesc& s,
                                              const PartPtrs<R>& q, int32_t p) {
  const PWords<R> x = load_words<R, DIM>(q, p);
  store_rec<R>(esc.rec, k, rec_of(x));
  if (!esc.keys) return;   // (the list may carry records without keys)
  int c[3];
  esc.keys[k] = decode_cell<R, DIM>(q, x.cell, x.pos, c)
                    ? s.bin_base + (((c[2] >> s.lz) * r.nty) + (c[1] >> s.ly)) * r.ntx + (c[0] >> s.lx)
                    : s.bin_base + r.ntiles;
}

template <typename R, int DIM>
__device__ __forceinline__ void escape_append(const EscapeList& esc, bool want, int seg,
                                              int32_t p, const PartPtrs<R>& q,
                                              const RunDesc& r, const SegDesc& s) {
  const uint64_t mask = __ballot(want);
  if (!mask) return;
  const int lane = __lane_id();
  const int leader = __ffsll((unsigned long long)mask) - 1;
  unsigned int base = 0;
  if (lane == leader) base = atomicAdd(esc.count, (unsigned int)__popcll(mask));
  base = __shfl(base, leader, 64);
  if (want) {
    const unsigned int k = base + (unsigned int)__popcll(mask & ((1ull << lane) - 1ull));
    if ((int64_t)k < esc.capacity) {
      esc.items[k] = ((unsigned long long)seg << 32) | (unsigned long long)p;
      if constexpr (DIM == 3)
        if (esc.rec) escape_record<R, DIM>(esc, k, r, s, q, p);
    }
  }
}

// The particles of one chunk against the staged region, in rounds: each thread first
// issues the loads of BATCH particles (a workgroup apart, so every load instruction reads 64
// consecutive particles) and then pushes them one by one, so HBM latency is paid once per
// round rather than once per particle.  Returns the summed w m u^2/(1+gamma).
// In 3D one particle per thread per round: the unrolled body of four 3D particles is too
// large for the compiler to keep their states in registers (it put them in scratch memory,
// read and written for every particle), and a 3D workgroup brings 16 waves per CU anyway.
// In 2D FP64 one as well: a second FP64 state takes the registers of a third wave per SIMD
// (169 VGPRs with two, two waves; 154 with one, three waves and a 10% faster launch).
template <typename R, int DIM>
constexpr int batch_of() { return DIM == 3 ? 1 : (sizeof(R) == 4 ? 4 : 1); }
// Waves per SIMD the fused kernel's register budget is set for: 2D FP32 and the two-per-CU
// 3D FP32 geometry fit 4 (at most 128 VGPRs), the others keep the compiler's choice.
template <typename R, int DIM, int G>
constexpr int fused_waves() {
  return (sizeof(R) == 4 && (DIM == 2 || G >= 7)) ? 4 : 1;
}

// Threads per workgroup: a 3D region (tile + halo on three axes) fills most of a CU's LDS,
// so one workgroup per CU must bring enough waves by itself: 16 (four per SIMD) in FP32, whose
// quadratic particle loop fits 128 VGPRs; 8 in FP64, which needs more registers per lane.
// The smaller regions of geometries 7 and 8 let two 512-thread workgroups share a CU.
template <typename R, int DIM, int G>
constexpr int fused_block() {
  return DIM == 2 ? 256 : (sizeof(R) == 8 || G == 7 || G == 8 ? 512 : 1024);
}

// pl.list != NULL (the second pass of the re-binned escape path): the chunk's range indexes
// pl.list, whose entries name the particles (segment << 32 | slot), and pl.rec when set.
// Local start cell a of a particle in the staged region, and whether it can be on chip: a
// particle that stays in its cell for the half push and keeps its nearest node reads and
// adds cells [a-1, a+2] per axis, so a must lie in [1, rw-3].  The exact test follows once
// the particle's own half-step position and path are known (gather_fits, deposit_fits): a
// fast particle near the edge of the region may still need the cells beyond.
template <int DIM>
__device__ __forceinline__ bool on_chip(const int c[3], const Region& g, const int n[3],
                                        int a[3]) {
  bool inside = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d < DIM) {
      int v = c[d] - g.r0[d];
      v = v < 0 ? v + n[d] : (v >= n[d] ? v - n[d] : v);
      a[d] = v;
      inside = inside && v >= 1 && v <= g.rw[d] - 3;
    } else {
      a[d] = 0;
    }
  }
  return inside;
}

// Whether start cell a lies at least two cells inside the staged region on every axis:
// then, whatever the particle's momentum, its gather stencil and deposit window fit (with
// dt below the CFL step a particle moves less than half a cell per axis in a half push, so
// the stencil lies in [a-2, a+2] and the window in [a-2, a+3]), and the exact tests can be
// skipped for a wave whose particles all start there.
template <int DIM>
__device__ __forceinline__ bool deep_inside(const int a[3], const Region& g) {
  bool deep = true;
#pragma unroll
  for (int d = 0; d < DIM; ++d) deep = deep && a[d] >= 2 && a[d] <= g.rw[d] - 4;
  return deep;
}

// Push and deposit one particle against the staged region if its gather stencil and its
// deposit window both lie inside it (the particle is stored); false otherwise (nothing is
// written and the particle's stored state is unchanged: it escapes to a later pass).
// check: false when every particle of the wave starts deep inside the region (a uniform
// value, so the tests are branched over rather than evaluated).
template <typename R, int DIM, int ORDER, class LA>
__device__ __forceinline__ bool push_on_chip(const RunDesc& r, const Region& g, const LA& L,
                                             const int n[3], const int a[3], PState<R>& ps,
                                             const PushConst<R>& k, const PartPtrs<R>& q,
                                             int32_t slot, int with_rho, bool want_ke,
                                             double& ke, bool check) {
  const int lim[3] = {g.rw[0] - 1, g.rw[1] - 1, g.rw[2] - 1};
  int pcell[3];
  R po[3], xh[3];
  half_push<DIM>(a, ps, k, pcell, po, xh);
  bool fit = true;
  if (check) fit = gather_fits<DIM, ORDER>(pcell, po, lim);
  if (!fit) return false;
  R pe[3], x1[3], vz1, g1;
  push_rest<DIM, ORDER>(L, pcell, po, xh, ps, k, pe, x1, vz1, g1);
  if (check) fit = deposit_fits<DIM, ORDER>(pcell, po, pe, lim);
  if (!fit) return false;
#pragma unroll
  for (int d = 0; d < DIM; ++d) advance_cell<R>(ps.c[d], ps.o[d], x1[d], n[d]);
  if (leaves_box(r, ps.c[0])) ps.alive = false;
  // (with_rho 2: the charge where the next step's paths start; a particle leaving the box
  // has none there)
  deposit<DIM, ORDER>(L, pcell, po, pe, ps.w, vz1, k, with_rho == 2 && !ps.alive ? 0 : with_rho);
  store_particle<R, DIM>(q, slot, ps);
  if (want_ke && ps.alive) {   // diagnostic steps only
    const double u2 = (double)ps.u[0] * ps.u[0] + (double)ps.u[1] * ps.u[1] +
                      (double)ps.u[2] * ps.u[2];
    ke += (double)ps.w * u2 / (1.0 + (double)g1);
  }
  return true;
}

// 3D rounds with compaction (one particle per thread per round): each thread first reads
// only its particle's cell and classifies it (on chip / escaped / none); the on-chip
// particles of the workgroup are then packed into the first threads (their slots pass
// through LDS) and pushed there, so no wave carries idle lanes for escaped particles; the
// escaped ones are appended to the escape list with one global reservation per round.
// cbuf: blockDim + 64 words of LDS.
template <typename R, int DIM, int ORDER, class LA>
__device__ __forceinline__ double process_chunk_compact(
    const RunDesc& r, const SegDesc& s, int seg, const Chunk& ch, const Region& g, const LA& L,
    int with_rho, bool want_ke, const EscapeList& esc, const PassList& pl, int32_t* cbuf) {
  const int n[3] = {r.nx, r.ny, r.nz};
  const PushConst<R> k = push_const<R>(r, s);
  const PartPtrs<R> q = part_ptrs<R>(s, r);
  const int bd = (int)blockDim.x, tid = (int)threadIdx.x;
  const int lane = __lane_id(), wv = tid >> 6, nw = bd >> 6;
  // one list of bd entries: the on-chip particles (slots; list indexes when their records
  // are read) packed from the front, the slots of the escaped ones from the back
  int32_t* cin = cbuf;
  int32_t* wsum = cbuf + bd;           // per wave: on-chip and escaped counts -> bases;
                                       // [2 nw], [2 nw + 1]: totals; [2 nw + 2]: list base
  double ke = 0.0;
  for (int32_t base = ch.beg; base < ch.end; base += bd) {
    const int32_t lp = base + tid;
    const bool ok = lp < ch.end;
    int32_t slot = lp;
    if (pl.list && ok) slot = (int32_t)(gp(pl.list)[lp] & 0xffffffffull);
    bool alive = false;
    int c[3] = {0, 0, 0};
    if (ok) alive = pl.rec ? rec_cell<R, DIM>(q, pl.rec, lp, c) : load_cell<R, DIM>(q, slot, c);
    int a[3];
    const bool inside = alive && on_chip<DIM>(c, g, n, a);
    const bool gone = alive && !inside;
    const uint64_t mi = __ballot(inside), me = __ballot(gone);
    const uint64_t below = (1ull << lane) - 1ull;
    __syncthreads();                   // the previous round has read the list and wsum
    if (lane == 0) {
      wsum[wv] = __popcll(mi);
      wsum[nw + wv] = __popcll(me);
    }
    __syncthreads();
    if (tid == 0) {
      int ti = 0, te = 0;
      for (int w = 0; w < nw; ++w) {
        const int vi = wsum[w], ve = wsum[nw + w];
        wsum[w] = ti;
        wsum[nw + w] = te;
        ti += vi;
        te += ve;
      }
      wsum[2 * nw] = ti;
      wsum[2 * nw + 1] = te;
      wsum[2 * nw + 2] = te ? (int32_t)atomicAdd(esc.count, (unsigned int)te) : 0;
    }
    __syncthreads();
    if (inside) cin[wsum[wv] + __popcll(mi & below)] = pl.rec ? lp : slot;
    if (gone) cbuf[bd - 1 - (wsum[nw + wv] + __popcll(me & below))] = slot;
    __syncthreads();
    const int n_in = wsum[2 * nw], n_esc = wsum[2 * nw + 1];
    const int64_t ebase = (int64_t)(uint32_t)wsum[2 * nw + 2];
    for (int e = tid; e < n_esc; e += bd)
      if (ebase + e < esc.capacity) {
        const int32_t es = cbuf[bd - 1 - e];
        esc.items[ebase + e] = ((unsigned long long)seg << 32) | (unsigned long long)(uint32_t)es;
        if (esc.rec) escape_record<R, DIM>(esc, ebase + e, r, s, q, es);
      }
    bool late = false;                 // on chip by its cell, not by its own path
    int32_t p = 0;
    if (tid < n_in) {
      const int32_t src = cin[tid];
      PState<R> ps;
      if (pl.rec) {
        p = (int32_t)(gp(pl.list)[src] & 0xffffffffull);
        decode_particle<R, DIM>(q, words_of(load_rec<R>(pl.rec, src)), ps);
      } else {
        p = src;
        load_particle<R, DIM>(q, p, ps);
      }
      int b[3];
      (void)on_chip<DIM>(ps.c, g, n, b);
      // always tested: skipping the tests for deep waves costs the 3D body a spilled register
      late = !push_on_chip<R, DIM, ORDER>(r, g, L, n, b, ps, k, q, p, with_rho, want_ke, ke,
                                          true);
    }
    escape_append<R, DIM>(esc, late, seg, p, q, r, s);
  }
  return ke * s.m;
}

template <typename R, int DIM, int ORDER, bool DIRECT, class LA>
__device__ __forceinline__ double process_chunk(const RunDesc& r, const SegDesc& s, int seg,
                                                const Chunk& ch, const Region& g,
                                                const LA& L, int with_rho,
                                                bool want_ke, const EscapeList& esc,
                                                const PassList& pl, int32_t* cbuf) {
  // 3D: compacted rounds, except for the second pass of the re-binned path on the two-per-CU
  // geometry (DIRECT), whose particles lie inside their present tile (nearly all on chip):
  // there the records are loaded directly, one memory latency and no barriers per round
  if constexpr (DIM == 3)
    if (!(DIRECT && pl.rec))
      return process_chunk_compact<R, DIM, ORDER>(r, s, seg, ch, g, L, with_rho, want_ke, esc,
                                                  pl, cbuf);
  (void)cbuf;
  const int n[3] = {r.nx, r.ny, r.nz};
  const PushConst<R> k = push_const<R>(r, s);
  const PartPtrs<R> q = part_ptrs<R>(s, r);
  double ke = 0.0;
  constexpr int BATCH = batch_of<R, DIM>();
  const int32_t span = (int32_t)blockDim.x * BATCH;
  for (int32_t base = ch.beg; base < ch.end; base += span) {
    PState<R> ps[BATCH];
    int32_t pi[BATCH];
    bool ok[BATCH];
#pragma unroll
    for (int b = 0; b < BATCH; ++b) {
      const int32_t lp = base + b * (int32_t)blockDim.x + (int32_t)threadIdx.x;
      ok[b] = lp < ch.end;
      pi[b] = lp;
      if (pl.list && ok[b]) pi[b] = (int32_t)(gp(pl.list)[lp] & 0xffffffffull);
      if (ok[b]) {
        if constexpr (DIM == 3) {
          if (pl.rec) decode_particle<R, DIM>(q, words_of(load_rec<R>(pl.rec, lp)), ps[b]);
          else load_particle<R, DIM>(q, pi[b], ps[b]);
        } else {
          load_particle<R, DIM>(q, pi[b], ps[b]);   // 2D lists carry no records
        }
      }
    }
#pragma unroll
    for (int b = 0; b < BATCH; ++b) {
      int a[3];
      const bool live = ok[b] && ps[b].alive;
      const bool in = live && on_chip<DIM>(ps[b].c, g, n, a);
      const bool check = __ballot(in && !deep_inside<DIM>(a, g)) != 0;
      bool done = false;
      if (in)
        done = push_on_chip<R, DIM, ORDER>(r, g, L, n, a, ps[b], k, q, pi[b], with_rho,
                                           want_ke, ke, check);
      escape_append<R, DIM>(esc, live && !done, seg, pi[b], q, r, s);
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

// A descriptor copied into wavefront-uniform registers word by word.  Every lane holds the
// same descriptor, but loaded through a generic reference (the device table, or the copy in
// the kernel arguments) its words land in vector registers; with the particle loop's
// registers at the limit of four waves per SIMD they were spilled to scratch memory around
// every chunk, which raised the kernel's memory traffic about 40% above the bytes its
// particles and fields need.
template <typename D>
__device__ __forceinline__ D uniform_copy(const D& src) {
  static_assert(sizeof(D) % 4 == 0, "descriptor of whole words");
  D out;
  const uint32_t* w = (const uint32_t*)&src;
  uint32_t* o = (uint32_t*)&out;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(D) / 4); ++i) o[i] = __builtin_amdgcn_readfirstlane(w[i]);
  return out;
}

// Fused gather + push + deposit over the chunk table, persistent: the grid is a multiple of
// 8 and XCD x (workgroups x, x+8, ...) owns the contiguous chunk range [x*per, (x+1)*per),
// split into equal contiguous slices per workgroup.  Consecutive chunks of one tile (and of
// the other species of the same box, which follow in the table) reuse the staged region;
// the region is flushed when the tile changes.
template <typename R, int DIM, int G>
__global__ __launch_bounds__((fused_block<R, DIM, G>())) __attribute__((amdgpu_waves_per_eu(fused_waves<R, DIM, G>()))) void k_fused(Tables T, const Chunk* chunks,
                                               const int32_t* nchunks, int with_rho,
                                               double* kinetic, int ke_to_diag,
                                               EscapeList esc, const int32_t* jshift,
                                               PassList pl) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[fused_block<R, DIM, G>() / 64];
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
    st.ey_ = rh;
  }
  const int plane = st.plane();
  const int njplanes = 3 + charge_planes(with_rho);
  // the current planes follow the six field planes; 6 plane values of 4 or 8 bytes end on an
  // 8-byte boundary, as the 64-bit LDS atomics need
  double* jm = (double*)(sm + 6 * plane);
  // 3D: the round compaction's slot list after the current (and charge) planes
  int32_t* cbuf = (int32_t*)(jm + (size_t)njplanes * plane);
  LdsAcc<R, ST, DIM == 2> L;
  L.fbase = sm;
  L.jbase = jm;
  L.st = st;
  L.jfold = 1.0f;

  int cur_run = -1, cur_tile = -1;
  Region g;
  double ke = 0.0;
  double unscale = 1.0;
  for (int c = lo; c < hi; ++c) {
    Chunk ch = chunks[c];
    ch.seg = uniform(ch.seg);
    ch.tile = uniform(ch.tile);
    ch.beg = uniform(ch.beg);
    ch.end = uniform(ch.end);
    const SegDesc s = uniform_copy(seg_of(T, ch.seg));
    if (s.run != cur_run || ch.tile != cur_tile) {
      if (cur_run >= 0) {
        const RunDesc& rp = run_of(T, cur_run);
        __syncthreads();
        flush_region<R>(rp, g, st, njplanes, jm, unscale, with_rho);
        if (kinetic || ke_to_diag) {
          const double t = block_sum(ke, red);
          if (threadIdx.x == 0) atomic_add_global(ke_to_diag ? rp.diag + DIAG_UKIN : kinetic, t);
          ke = 0.0;
        }
      }
      if constexpr (sizeof(R) == 4) {
        const int sh = uniform(jshift[s.run]);
        L.jfold = ldexpf(1.0f, sh);
        unscale = ldexp(1.0, -sh);
      }
      const RunDesc rn = run_of(T, s.run);
      g = region_of<DIM>(rn, s, ch.tile, G ? geo_table(G).halo : s.halo);
      __syncthreads();
      stage_region<R>(rn, g, st, njplanes, sm, jm, DIM == 2);
      __syncthreads();
      cur_run = s.run;
      cur_tile = ch.tile;
    }
    const RunDesc r = run_of(T, s.run);
    const bool want_ke = kinetic || ke_to_diag;
    ke += s.order == 1
              ? process_chunk<R, DIM, 1, (G >= 7)>(r, s, ch.seg, ch, g, L, with_rho, want_ke, esc, pl, cbuf)
              : process_chunk<R, DIM, 2, (G >= 7)>(r, s, ch.seg, ch, g, L, with_rho, want_ke, esc, pl, cbuf);
  }
  const RunDesc& rl = run_of(T, cur_run);
  __syncthreads();
  flush_region<R>(rl, g, st, njplanes, jm, unscale, with_rho);
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
  const int n[3] = {r.nx, r.ny, r.nz};
#pragma unroll
  for (int d = 0; d < DIM; ++d) advance_cell<R>(ps.c[d], ps.o[d], x1[d], n[d]);
  if (leaves_box(r, ps.c[0])) ps.alive = false;
  deposit<DIM, ORDER>(G, pcell, po, pe, ps.w, vz1, k, with_rho == 2 && !ps.alive ? 0 : with_rho);
  store_particle<R, DIM>(s, r, p, ps);
  if (!ps.alive) return 0.0;
  const double u2 = (double)ps.u[0] * ps.u[0] + (double)ps.u[1] * ps.u[1] + (double)ps.u[2] * ps.u[2];
  return (double)ps.w * s.m * u2 / (1.0 + (double)g1);
}

// skip_at: a list of at least this many entries was taken by the re-binned path; only the
// clearing is left to do.
template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_escape(Tables T, int with_rho, double* kinetic,
                                                int ke_to_diag, EscapeList esc, int skip_at) {
  unsigned int cnt = min((int64_t)esc.count[0], esc.capacity);
  if ((int)min(esc.count[0], 0x7fffffffu) >= skip_at) cnt = 0;
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
  // the last workgroup to finish clears the list (every workgroup has read the count by
  // then; no fence: nothing this launch wrote is read before the launch ends)
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int done = atomicAdd(esc.count + 1, 1u);
    if (done == gridDim.x - 1) {
      atomicAdd(esc.total, (unsigned long long)esc.count[0]);
      atomicExch(esc.count, 0u);
      atomicExch(esc.count + 1, 0u);
    }
  }
}

// ---------------------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------------------
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
                           const EscapeList& esc, const int32_t* jshift, PassList pl,
                           hipStream_t st) {
  k_fused<R, D, G><<<nblocks, fused_block<R, D, G>(), smem, st>>>(T, chunks, nchunks, with_rho, kinetic,
                                               ke_to_diag, esc, jshift, pl);
}

template <typename R, int D>
static void launch_fused_d(int geo, const Tables& T, int nblocks, size_t smem,
                           const Chunk* chunks, const int32_t* nchunks, int with_rho,
                           double* kinetic, int ke_to_diag, const EscapeList& esc,
                           const int32_t* jshift, PassList pl, hipStream_t st) {
#define LPIC_GEO(g) launch_fused_g<R, D, g>(T, nblocks, smem, chunks, nchunks, with_rho, kinetic, ke_to_diag, esc, jshift, pl, st)
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
      case 7: LPIC_GEO(7); return;
      case 8: LPIC_GEO(8); return;
      case 9: LPIC_GEO(9); return;
      default: LPIC_GEO(0); return;
    }
  }
#undef LPIC_GEO
}

void launch_fused(const Tables& T, int prec, int dim, int geo, int nblocks, size_t smem,
                  const Chunk* chunks, const int32_t* nchunks, int with_rho, double* kinetic,
                  int ke_to_diag, const EscapeList& esc, const int32_t* jshift,
                  hipStream_t st, const Rebin* rb) {
  LPIC_PD(prec, dim, (launch_fused_d<R, D>(geo, T, nblocks, smem, chunks, nchunks, with_rho,
                                           kinetic, ke_to_diag, esc, jshift,
                                           PassList{nullptr, nullptr}, st)));
  if (rb) {
    // escapees by present tile, a second pass over them, then whatever that pass could not
    // place (normally nothing) through global memory
    launch_rebin(T, prec, dim, esc, *rb, st);
    const int k = with_rho == 0 ? 0 : (with_rho == 1 ? 1 : 2);
    LPIC_PD(prec, dim, (launch_fused_d<R, D>(rb->geo[k], T, rb->grid[k], rb->smem[k], rb->chunks,
                                             rb->nchunks, with_rho, kinetic, ke_to_diag,
                                             rb->esc2, jshift,
                                             PassList{rb->items, esc.rec ? rb->rec : nullptr},
                                             st)));
    LPIC_PD(prec, dim, (k_escape<R, D><<<ESCAPE_BLOCKS, 256, 0, st>>>(
                           T, with_rho, kinetic, ke_to_diag, esc, rb->threshold)));
    LPIC_PD(prec, dim, (k_escape<R, D><<<ESCAPE_BLOCKS, 256, 0, st>>>(
                           T, with_rho, kinetic, ke_to_diag, rb->esc2, 0x7fffffff)));
  } else {
    LPIC_PD(prec, dim, (k_escape<R, D><<<ESCAPE_BLOCKS, 256, 0, st>>>(
                           T, with_rho, kinetic, ke_to_diag, esc, 0x7fffffff)));
  }
}

template <typename R, int D, int G>
static hipError_t set_smem(size_t smem, size_t smem_occ, int* blocks_per_cu) {
  hipError_t e = hipFuncSetAttribute((const void*)k_fused<R, D, G>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_fused<R, D, G>,
                                                      fused_block<R, D, G>(),
                                                      smem_occ);
}

hipError_t prepare_fused(int prec, int dim, int geo, size_t smem, size_t smem_occ,
                         int* blocks_per_cu) {
  hipError_t e = hipSuccess;
  int* b = blocks_per_cu;
  if (dim == 2) {
    switch (geo) {
      case 1: e = prec == 0 ? set_smem<float, 2, 1>(smem, smem_occ, b) : set_smem<double, 2, 1>(smem, smem_occ, b); break;
      case 2: e = prec == 0 ? set_smem<float, 2, 2>(smem, smem_occ, b) : set_smem<double, 2, 2>(smem, smem_occ, b); break;
      case 3: e = prec == 0 ? set_smem<float, 2, 3>(smem, smem_occ, b) : set_smem<double, 2, 3>(smem, smem_occ, b); break;
      case 4: e = prec == 0 ? set_smem<float, 2, 4>(smem, smem_occ, b) : set_smem<double, 2, 4>(smem, smem_occ, b); break;
      default: e = prec == 0 ? set_smem<float, 2, 0>(smem, smem_occ, b) : set_smem<double, 2, 0>(smem, smem_occ, b); break;
    }
  } else {
    switch (geo) {
      case 5: e = prec == 0 ? set_smem<float, 3, 5>(smem, smem_occ, b) : set_smem<double, 3, 5>(smem, smem_occ, b); break;
      case 6: e = prec == 0 ? set_smem<float, 3, 6>(smem, smem_occ, b) : set_smem<double, 3, 6>(smem, smem_occ, b); break;
      case 7: e = prec == 0 ? set_smem<float, 3, 7>(smem, smem_occ, b) : set_smem<double, 3, 7>(smem, smem_occ, b); break;
      case 8: e = prec == 0 ? set_smem<float, 3, 8>(smem, smem_occ, b) : set_smem<double, 3, 8>(smem, smem_occ, b); break;
      case 9: e = prec == 0 ? set_smem<float, 3, 9>(smem, smem_occ, b) : set_smem<double, 3, 9>(smem, smem_occ, b); break;
      default: e = prec == 0 ? set_smem<float, 3, 0>(smem, smem_occ, b) : set_smem<double, 3, 0>(smem, smem_occ, b); break;
    }
  }
  return e;
}

size_t fused_smem_bytes(int prec, int dim, int tx, int ty, int tz, int halo, int with_rho,
                        int geo) {
  // the z layers of a fixed 3D geometry are padded (GeoFix::pz)
  if (geo < 0) geo = fused_geometry(dim, tx, ty, tz, halo);
  const int pz = dim == 3 ? geo_table(geo).pz : 0;
  const size_t plane = ((size_t)(tx + 2 * halo) * (ty + 2 * halo) + pz) *
                       (dim == 3 ? (tz + 2 * halo) : 1);
  // six field planes in the kernel precision (24 or 48 bytes per cell: the current planes
  // after them start 8-byte aligned), then 8-byte current planes (and, on diagnostic steps,
  // two charge planes)
  const int jplanes = 3 + charge_planes(with_rho);
  static_assert((6 * sizeof(float)) % 8 == 0, "current planes must start 8-byte aligned");
  // 3D: the round compaction's slot list and wave sums (process_chunk_compact), sized for
  // the workgroup of this precision and geometry
  const int block = geo == 7 || geo == 8
                        ? (prec == 0 ? fused_block<float, 3, 7>() : fused_block<double, 3, 7>())
                        : (prec == 0 ? fused_block<float, 3, 0>() : fused_block<double, 3, 0>());
  const size_t compact = dim == 3 ? ((size_t)block + 64) * 4 : 0;
  return plane * 6 * (prec == 0 ? 4 : 8) + plane * jplanes * 8 + compact;
}

}  // namespace lpic
