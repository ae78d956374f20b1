// Device-side building blocks of the PIC hot path for gfx950.
//
// The particle math follows lambda-PIC (arXiv 2607.13507): Algorithm 1 (half position push,
// interpolation, Boris momentum push, half position push, deposit), the relativistic Boris
// scheme of Sec. 3.1, staggering-aware B-spline interpolation (Sec. 3.1) and Esirkepov's
// charge-conserving deposition (Sec. 3.1, Esirkepov 2001).  Everything here is written for
// 64-wide wavefronts: no warp-size assumptions other than wave64 ballots in the sort.
//
// Positions inside kernels are always (integer cell, offset in [0,1)) per axis, in cell
// units.  In the FP32 mode this is the stored representation; in the FP64 mode it is
// derived from the absolute coordinate on load.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpic {

enum FieldSlot { F_EX = 0, F_EY, F_EZ, F_BX, F_BY, F_BZ, F_JX, F_JY, F_JZ, F_R0, F_R1, F_NUM };

// Particle array slots.  FP32: cell(int32) ox oy oz ux uy uz w;  FP64: x y z - ux uy uz w.
enum PartSlot { P_CELL = 0, P_X = 0, P_OX = 1, P_Y = 1, P_OY = 2, P_Z = 2, P_OZ = 3,
                P_UX = 4, P_UY = 5, P_UZ = 6, P_W = 7, P_NUM = 8 };

enum { DIAG_UFIELD = 0, DIAG_UKIN = 1, DIAG_RES = 2, DIAG_RHOMAX = 3, DIAG_GAUSS = 4,
       DIAG_NUM = 8 };

// Laser antenna of a box: E_inc amplitude e0 = a0 omega (see lpic_laser).
struct LaserDesc {
  int32_t pol, ia;
  double e0, omega, waist, yc, zc, t0, tau;
};

// Cells at each open x end in which particles do not live.
constexpr int OPEN_MARGIN = 3;

// One simulation box.
struct RunDesc {
  int32_t ndim, nx, ny, nz;
  int32_t ntx, nty, ntz, ntiles;   // tiles per axis of the current tiling
  int32_t open_x, has_laser;       // open x ends; laser antenna present
  int32_t seg_first, nseg;         // the run's species: segments [seg_first, seg_first + nseg)
  int32_t vbase;                   // first (tile, species) slot of the run in the chunk order
  int32_t x0;                      // array column of the box's column 0 (a moving window's
                                   // origin; 0 otherwise): x is circular in the arrays
  double dx, dy, dz, dt, rho_bg;
  void* f[F_NUM];
  double* diag;                    // DIAG_NUM device accumulators
  LaserDesc laser;
  // convolutional PML at the open x ends (pml_cells = 0: Mur condition instead)
  int32_t pml_cells, pad1;
  void* psi;                       // 2 halves x 4 components x rows x 2 pml_cells values
  const void* pml_tab;             // b, c, 1/kappa per slot for a half step dt/2: E side
                                   // (2 pml_cells slots), then B side
  const int32_t* psi_parity;       // which half is current (the fused field update's parity)
};

// Box column of array column i, and back (x0: the moving window's origin).
__device__ __forceinline__ int box_x(const RunDesc& r, int i) {
  const int p = i - r.x0;
  return p < 0 ? p + r.nx : p;
}
__device__ __forceinline__ int array_x(const RunDesc& r, int p) {
  const int i = p + r.x0;
  return i >= r.nx ? i - r.nx : i;
}

// A particle whose cell column is inside the margin of an open x end leaves the box.
__device__ __forceinline__ bool leaves_box(const RunDesc& r, int cx) {
  const int p = box_x(r, cx);
  return r.open_x && (p < OPEN_MARGIN || p >= r.nx - OPEN_MARGIN);
}

// One species of one box (a "segment" of the global particle key space).
struct SegDesc {
  int32_t run, order;
  int32_t lx, ly, lz, halo;        // log2 of the tile edges, halo cells
  int32_t bin_base;                // global bin of tile 0; the dead bin is bin_base + ntiles
  int32_t pad0;
  int64_t n;                       // slots
  int64_t pbase;                   // position of slot 0 in the concatenation of all segments
  double q, m;
  void* p[P_NUM];                  // current arrays
  void* alt[P_NUM];                // second buffer of the sort
};

struct Chunk {
  int32_t seg, tile, beg, end;     // particles [beg, end) of segment `seg`, home tile `tile`
};

// Descriptor access: either device tables (simulations, ensembles) or one run / one
// segment passed by value (single-box entry points).
struct Tables {
  const RunDesc* runs;
  const SegDesc* segs;
  const int32_t* run_blk;          // nruns + 1 block prefix for cell kernels
  const int32_t* seg_blk;          // nsegs + 1 block prefix for particle kernels
  int32_t nruns, nsegs;
  RunDesc run0;
  SegDesc seg0;
};

__device__ __forceinline__ int find_owner(const int32_t* prefix, int count, int b) {
  int lo = 0, hi = count - 1;  // largest i with prefix[i] <= b
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------------------
// precision helpers
// ---------------------------------------------------------------------------------------
template <typename R> __device__ __forceinline__ R rsq(R x);
template <> __device__ __forceinline__ float rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ __forceinline__ double rsq<double>(double x) { return 1.0 / sqrt(x); }
template <typename R> __device__ __forceinline__ R rcp(R x);
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }
template <typename R> __device__ __forceinline__ R ffloor(R x) { return floor(x); }
template <> __device__ __forceinline__ float ffloor<float>(float x) { return floorf(x); }

// Global-memory pointers.  Arrays reached through descriptor tables would otherwise be
// generic (flat) pointers: flat accesses count against the LDS wait counter too, so every
// LDS wait would also wait for all in-flight particle loads.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> gp(T* p) {
  return (gptr<T>)p;
}
template <typename T>
__device__ __forceinline__ T uniform(T v) {   // wavefront-uniform value (scalar register)
  return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ void atomic_add_lds(float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void atomic_add_lds(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void atomic_add_global(float* p, float v) {
  __hip_atomic_fetch_add(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_add_global(double* p, double v) {
  __hip_atomic_fetch_add(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_add_global(gptr<float> p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_add_global(gptr<double> p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// floor(x) limited to [lo, hi]; NaN maps to lo.  Every cell index derived from a particle
// offset goes through this, so no input can produce an access outside the stencil window.
template <typename R>
__device__ __forceinline__ R floor_clamped(R x, R lo, R hi) {
  return fmin(fmax(floor(x), lo), hi);
}
template <>
__device__ __forceinline__ float floor_clamped<float>(float x, float lo, float hi) {
  return fminf(fmaxf(floorf(x), lo), hi);
}

__device__ __forceinline__ int wrapi(int i, int n) {  // |i| small compared to n
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

// ---------------------------------------------------------------------------------------
// Shape weights (Sec. 3.1).  For a particle at cell `c` with offset o in [0,1] the weights
// of the ORDER+1 nodes that can be non-zero are returned with the index of the first one,
// for the integer lattice (nodes at i) and the half lattice (nodes at i+1/2, index i).
//   CIC       S(x) = 1 - |x|
//   quadratic S(x) = 3/4 - x^2 (|x| <= 1/2),  (3/2 - |x|)^2 / 2 (1/2 < |x| < 3/2)
// ---------------------------------------------------------------------------------------
template <int ORDER, typename R>
__device__ __forceinline__ void weights_int(R o, int c, int& base, R w[ORDER + 1]) {
  if constexpr (ORDER == 1) {
    base = c;
    w[0] = R(1) - o;
    w[1] = o;
  } else {
    const int up = o >= R(0.5);
    const R d = o - R(up);                // offset from the nearest node, in [-1/2, 1/2)
    base = c + up - 1;
    const R a = R(0.5) - d, b = R(0.5) + d;
    w[0] = R(0.5) * a * a;
    w[1] = R(0.75) - d * d;
    w[2] = R(0.5) * b * b;
  }
}

template <int ORDER, typename R>
__device__ __forceinline__ void weights_half(R o, int c, int& base, R w[ORDER + 1]) {
  if constexpr (ORDER == 1) {
    const int up = o >= R(0.5);
    const R t = o + R(0.5) - R(up);       // distance past the half node at index base
    base = c - 1 + up;
    w[0] = R(1) - t;
    w[1] = t;
  } else {
    const R d = o - R(0.5);               // the nearest half node is c + 1/2
    base = c - 1;
    const R a = R(0.5) - d, b = R(0.5) + d;
    w[0] = R(0.5) * a * a;
    w[1] = R(0.75) - d * d;
    w[2] = R(0.5) * b * b;
  }
}

// ---------------------------------------------------------------------------------------
// Field / current accessors.  Coordinates are in the accessor's frame: global (wrapped)
// for the global accessor, tile-local for the on-chip one.  xo/yo/zo turn a coordinate into
// an element offset so a stencil's offsets are computed once and reused by every component.
// ---------------------------------------------------------------------------------------
template <typename R>
struct GlobalAcc {
  static constexpr bool kPaired = false;
  static constexpr bool kLinear = false;   // offsets wrap: one per node
  gptr<R> f[F_NUM];
  int nx, ny, nz;
  __device__ __forceinline__ int xo(int x) const { return wrapi(x, nx); }
  __device__ __forceinline__ int yo(int y) const { return wrapi(y, ny) * nx; }
  __device__ __forceinline__ int zo(int z) const { return wrapi(z, nz) * nx * ny; }
  __device__ __forceinline__ R get(int comp, int off) const { return f[comp][off]; }
  // current values arrive unscaled; exact zeros are skipped (a global atomic each)
  __device__ __forceinline__ R fold() const { return R(1); }
  __device__ __forceinline__ void add(int comp, int off, R v) const {
    if (v != R(0)) atomic_add_global(f[comp] + off, v);
  }
  __device__ __forceinline__ void add_core(int comp, int off, R v) const { add(comp, off, v); }
};

// Strides of the staged region (tile + halo).  Fixed strides are compile-time constants, so
// every stencil offset folds into the immediate offset of the LDS instruction; dynamic
// strides serve any other tiling.  PZ pads each z layer: with RW * RH a multiple of the LDS
// bank count, every z layer of a 3D region maps onto the same banks, and the 64 lanes of a
// wave (particles spread over one tile) fall on a fraction of them; a pad of a few entries
// spreads the layers over the banks.
template <int RW, int RH, int RD, int PZ = 0>
struct FixStrides {
  static constexpr int kSy = RW, kSz = RW * RH + PZ, kPlane = (RW * RH + PZ) * RD;
  __device__ __forceinline__ constexpr int sy() const { return kSy; }
  __device__ __forceinline__ constexpr int sz() const { return kSz; }
  __device__ __forceinline__ constexpr int plane() const { return kPlane; }
  // region extents along x and y (cells)
  __device__ __forceinline__ constexpr int ex() const { return RW; }
  __device__ __forceinline__ constexpr int ey() const { return RH; }
};
struct DynStrides {
  int sy_, sz_, plane_, ey_;
  __device__ __forceinline__ int sy() const { return sy_; }
  __device__ __forceinline__ int sz() const { return sz_; }
  __device__ __forceinline__ int plane() const { return plane_; }
  __device__ __forceinline__ int ex() const { return sy_; }
  __device__ __forceinline__ int ey() const { return ey_; }
};

// LDS accessor of a staged region: the six field planes in the kernel's precision, and the
// current (and charge) planes: signed 64-bit fixed point on the FP32 path (see add()), FP64
// on the FP64 path.  PAIR (2D): components that share a staggering are
// interleaved so that one 8-byte (FP32) / 16-byte (FP64) read fetches both at a node:
// planes [ (Ex,By) pairs | (Ey,Bx) pairs | Ez | Bz ]; otherwise planes Ex Ey Ez Bx By Bz.
template <typename R, class S, bool PAIR = false>
struct LdsAcc {
  static constexpr bool kPaired = PAIR;
  // offsets are linear in the node index: one base per window, the nodes at compile-time
  // offsets from it (immediates of the LDS instructions when the strides are fixed)
  static constexpr bool kLinear = true;
  R* fbase;       // the six field components, laid out as above
  double* jbase;  // planes Jx Jy Jz, then rho0 rho1 (FP32 path: int64 fixed point)
  S st;
  float jfold;    // FP32 path: 2^S, the fixed-point scale of the current accumulators
  __device__ __forceinline__ int xo(int x) const { return x; }
  __device__ __forceinline__ int yo(int y) const { return y * st.sy(); }
  __device__ __forceinline__ int zo(int z) const { return z * st.sz(); }
  __device__ __forceinline__ R get(int comp, int off) const {
    return fbase[comp * st.plane() + off];
  }
  // PAIR layout: pair 0 = (Ex, By), pair 1 = (Ey, Bx); single 4 = Ez, 5 = Bz.
  typedef R R2 __attribute__((ext_vector_type(2)));
  __device__ __forceinline__ R2 get2(int pair, int off) const {
    return *(const R2*)(fbase + 2 * (pair * st.plane() + off));
  }
  __device__ __forceinline__ R get1(int plane_idx, int off) const {
    return fbase[plane_idx * st.plane() + off];
  }
  __device__ __forceinline__ const R2* pair_ptr(int pair, int off) const {
    return (const R2*)(fbase + 2 * (pair * st.plane() + off));
  }
  __device__ __forceinline__ const R* plane_ptr(int plane_idx, int off) const {
    return fbase + plane_idx * st.plane() + off;
  }
  // The factor the deposit folds into its per-particle current constants, so that every
  // value reaching add() is already in accumulator units.  FP32 path: the accumulators are
  // signed 64-bit fixed point with 2^-S resolution (integer LDS atomics run about twice as
  // fast as FP64 ones on gfx950 and their sums do not depend on the order of the adds; FP32
  // LDS atomics take a slow path there), and the scale 2^S is chosen per run (fixed_shift)
  // so that every single contribution stays below 2^29 in these units: it rounds to a
  // 32-bit integer (half-up) that is sign-extended into the 64-bit add, and no sum of a
  // run's contributions can overflow.
  __device__ __forceinline__ R fold() const {
    if constexpr (sizeof(R) == 4) return jfold;
    else return R(1);
  }
  __device__ __forceinline__ void add_core(int comp, int off, R v) const {
    double* p = jbase + (comp - F_JX) * st.plane() + off;
    if constexpr (sizeof(R) == 4) {
      int k;
      asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(k) : "v"(v));
      __hip_atomic_fetch_add((long long*)p, (long long)k, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
      atomic_add_lds(p, (double)v);
    }
  }
  // Entries that are exactly zero for most particles (the window's last node, which only a
  // path that changes its nearest node reaches) skip the add: a lane masked off costs the
  // LDS nothing.  The other entries (add_core) are added unconditionally.
  __device__ __forceinline__ void add(int comp, int off, R v) const {
    if (v != R(0)) add_core(comp, off, v);
  }
};

// The charge planes a fused pass accumulates for a with_rho mode (see deposit).
__host__ __device__ constexpr int charge_planes(int with_rho) {
  return with_rho == 1 ? 2 : (with_rho >= 2 ? 1 : 0);
}

// ---------------------------------------------------------------------------------------
// Interpolation (Sec. 3.1): every component from its own staggered nodes.
// 2D:  Ex (h,i)  Ey (i,h)  Ez (i,i)  Bx (i,h)  By (h,i)  Bz (h,h)
// 3D:  Ex (h,i,i) Ey (i,h,i) Ez (i,i,h) Bx (i,h,h) By (h,i,h) Bz (h,h,i)
// ---------------------------------------------------------------------------------------
template <int N, typename R, class Acc>
__device__ __forceinline__ R interp2(const Acc& A, int comp, const int* xo, const R* wx,
                                     const int* yo, const R* wy) {
  R s = R(0);
#pragma unroll
  for (int b = 0; b < N; ++b) {
    R r = R(0);
#pragma unroll
    for (int a = 0; a < N; ++a) r += wx[a] * A.get(comp, yo[b] + xo[a]);
    s += wy[b] * r;
  }
  return s;
}

template <int N, typename R, class Acc>
__device__ __forceinline__ R interp3(const Acc& A, int comp, const int* xo, const R* wx,
                                     const int* yo, const R* wy, const int* zo, const R* wz) {
  R s = R(0);
#pragma unroll
  for (int c = 0; c < N; ++c) {
    R t = R(0);
#pragma unroll
    for (int b = 0; b < N; ++b) {
      R r = R(0);
#pragma unroll
      for (int a = 0; a < N; ++a) r += wx[a] * A.get(comp, zo[c] + yo[b] + xo[a]);
      t += wy[b] * r;
    }
    s += wz[c] * t;
  }
  return s;
}

// Two components with the same staggering from the paired layout: one read per node.
template <int N, typename R, class Acc>
__device__ __forceinline__ void interp2_pair(const Acc& A, int pair, const int* xo, const R* wx,
                                             const int* yo, const R* wy, R& s0, R& s1) {
  s0 = R(0);
  s1 = R(0);
#pragma unroll
  for (int b = 0; b < N; ++b) {
    R r0 = R(0), r1 = R(0);
#pragma unroll
    for (int a = 0; a < N; ++a) {
      const auto v = A.get2(pair, yo[b] + xo[a]);
      r0 += wx[a] * v.x;
      r1 += wx[a] * v.y;
    }
    s0 += wy[b] * r0;
    s1 += wy[b] * r1;
  }
}

template <int N, typename R, class Acc>
__device__ __forceinline__ R interp2_single(const Acc& A, int plane_idx, const int* xo,
                                            const R* wx, const int* yo, const R* wy) {
  R s = R(0);
#pragma unroll
  for (int b = 0; b < N; ++b) {
    R r = R(0);
#pragma unroll
    for (int a = 0; a < N; ++a) r += wx[a] * A.get1(plane_idx, yo[b] + xo[a]);
    s += wy[b] * r;
  }
  return s;
}

template <int ORDER, typename R, class Acc>
__device__ __forceinline__ void stencil_axis(const Acc& A, int axis, int c, R o, int* oi,
                                             R* wi, int* oh, R* wh) {
  constexpr int N = ORDER + 1;
  int bi, bh;
  weights_int<ORDER>(o, c, bi, wi);
  weights_half<ORDER>(o, c, bh, wh);
#pragma unroll
  for (int a = 0; a < N; ++a) {
    if (axis == 0) { oi[a] = A.xo(bi + a); oh[a] = A.xo(bh + a); }
    else if (axis == 1) { oi[a] = A.yo(bi + a); oh[a] = A.yo(bh + a); }
    else { oi[a] = A.zo(bi + a); oh[a] = A.zo(bh + a); }
  }
}

// 2D gather from the paired LDS layout: one base address per staggering, every node of
// the (ORDER+1)^2 stencil a compile-time offset from it (an immediate of the LDS read when
// the region's strides are fixed).
template <int ORDER, typename R, class Acc>
__device__ __forceinline__ void gather2_paired(const Acc& A, const int* c, const R* o, R E[3],
                                               R B[3]) {
  constexpr int N = ORDER + 1;
  int bix, bhx, biy, bhy;
  R wxi[N], wxh[N], wyi[N], wyh[N];
  weights_int<ORDER>(o[0], c[0], bix, wxi);
  weights_half<ORDER>(o[0], c[0], bhx, wxh);
  weights_int<ORDER>(o[1], c[1], biy, wyi);
  weights_half<ORDER>(o[1], c[1], bhy, wyh);
  const int sy = A.st.sy();
  const auto* p0 = A.pair_ptr(0, biy * sy + bhx);   // (h,i): Ex, By
  const auto* p1 = A.pair_ptr(1, bhy * sy + bix);   // (i,h): Ey, Bx
  const R* pz = A.plane_ptr(4, biy * sy + bix);     // (i,i): Ez
  const R* pb = A.plane_ptr(5, bhy * sy + bhx);     // (h,h): Bz
  R ex = R(0), by = R(0), ey = R(0), bx = R(0), ez = R(0), bz = R(0);
#pragma unroll
  for (int b = 0; b < N; ++b) {
    R r0 = R(0), r1 = R(0), r2 = R(0), r3 = R(0), r4 = R(0), r5 = R(0);
#pragma unroll
    for (int a = 0; a < N; ++a) {
      const int off = b * sy + a;
      const auto v0 = p0[off];
      const auto v1 = p1[off];
      r0 += wxh[a] * v0.x;
      r1 += wxh[a] * v0.y;
      r2 += wxi[a] * v1.x;
      r3 += wxi[a] * v1.y;
      r4 += wxi[a] * pz[off];
      r5 += wxh[a] * pb[off];
    }
    ex += wyi[b] * r0;
    by += wyi[b] * r1;
    ey += wyh[b] * r2;
    bx += wyh[b] * r3;
    ez += wyi[b] * r4;
    bz += wyh[b] * r5;
  }
  E[0] = ex; E[1] = ey; E[2] = ez;
  B[0] = bx; B[1] = by; B[2] = bz;
}

// One 3D component from a linear LDS layout: p at the stencil's first node.
template <int N, typename R, class Acc>
__device__ __forceinline__ R interp3_lin(const Acc& A, const R* p, const R* wx, const R* wy,
                                         const R* wz) {
  const int sy = A.st.sy(), sz = A.st.sz();
  R s = R(0);
#pragma unroll
  for (int c = 0; c < N; ++c) {
    R t = R(0);
#pragma unroll
    for (int b = 0; b < N; ++b) {
      R r = R(0);
#pragma unroll
      for (int a = 0; a < N; ++a) r += wx[a] * p[c * sz + b * sy + a];
      t += wy[b] * r;
    }
    s += wz[c] * t;
  }
  return s;
}

// 3D gather from the LDS planes Ex Ey Ez Bx By Bz: one base address per component (its
// staggering), every node a compile-time offset from it when the strides are fixed.
template <int ORDER, typename R, class Acc>
__device__ __forceinline__ void gather3_linear(const Acc& A, const int* c, const R* o, R E[3],
                                               R B[3]) {
  constexpr int N = ORDER + 1;
  int ix, hx, iy, hy, iz, hz;
  R wxi[N], wxh[N], wyi[N], wyh[N], wzi[N], wzh[N];
  weights_int<ORDER>(o[0], c[0], ix, wxi);
  weights_half<ORDER>(o[0], c[0], hx, wxh);
  weights_int<ORDER>(o[1], c[1], iy, wyi);
  weights_half<ORDER>(o[1], c[1], hy, wyh);
  weights_int<ORDER>(o[2], c[2], iz, wzi);
  weights_half<ORDER>(o[2], c[2], hz, wzh);
  const int sy = A.st.sy(), sz = A.st.sz();
  E[0] = interp3_lin<N>(A, A.plane_ptr(F_EX, iz * sz + iy * sy + hx), wxh, wyi, wzi);
  E[1] = interp3_lin<N>(A, A.plane_ptr(F_EY, iz * sz + hy * sy + ix), wxi, wyh, wzi);
  E[2] = interp3_lin<N>(A, A.plane_ptr(F_EZ, hz * sz + iy * sy + ix), wxi, wyi, wzh);
  B[0] = interp3_lin<N>(A, A.plane_ptr(F_BX, hz * sz + hy * sy + ix), wxi, wyh, wzh);
  B[1] = interp3_lin<N>(A, A.plane_ptr(F_BY, hz * sz + iy * sy + hx), wxh, wyi, wzh);
  B[2] = interp3_lin<N>(A, A.plane_ptr(F_BZ, iz * sz + hy * sy + hx), wxh, wyh, wzi);
}

template <int DIM, int ORDER, typename R, class Acc>
__device__ __forceinline__ void gather(const Acc& A, const int* c, const R* o, R E[3], R B[3]) {
  if constexpr (DIM == 2 && Acc::kPaired) {
    gather2_paired<ORDER>(A, c, o, E, B);
    return;
  } else if constexpr (DIM == 3 && Acc::kLinear) {
    gather3_linear<ORDER>(A, c, o, E, B);
    return;
  }
  constexpr int N = ORDER + 1;
  int xi[N], xh[N], yi[N], yh[N];
  R wxi[N], wxh[N], wyi[N], wyh[N];
  stencil_axis<ORDER>(A, 0, c[0], o[0], xi, wxi, xh, wxh);
  stencil_axis<ORDER>(A, 1, c[1], o[1], yi, wyi, yh, wyh);
  if constexpr (DIM == 2 && Acc::kPaired) {
  } else if constexpr (DIM == 2) {
    E[0] = interp2<N>(A, F_EX, xh, wxh, yi, wyi);
    E[1] = interp2<N>(A, F_EY, xi, wxi, yh, wyh);
    E[2] = interp2<N>(A, F_EZ, xi, wxi, yi, wyi);
    B[0] = interp2<N>(A, F_BX, xi, wxi, yh, wyh);
    B[1] = interp2<N>(A, F_BY, xh, wxh, yi, wyi);
    B[2] = interp2<N>(A, F_BZ, xh, wxh, yh, wyh);
  } else {
    int zi[N], zh[N];
    R wzi[N], wzh[N];
    stencil_axis<ORDER>(A, 2, c[2], o[2], zi, wzi, zh, wzh);
    E[0] = interp3<N>(A, F_EX, xh, wxh, yi, wyi, zi, wzi);
    E[1] = interp3<N>(A, F_EY, xi, wxi, yh, wyh, zi, wzi);
    E[2] = interp3<N>(A, F_EZ, xi, wxi, yi, wyi, zh, wzh);
    B[0] = interp3<N>(A, F_BX, xi, wxi, yh, wyh, zh, wzh);
    B[1] = interp3<N>(A, F_BY, xh, wxh, yi, wyi, zh, wzh);
    B[2] = interp3<N>(A, F_BZ, xh, wxh, yh, wyh, zi, wzi);
  }
}

// ---------------------------------------------------------------------------------------
// Relativistic Boris push (Sec. 3.1): half electric kick, rotation, half electric kick.
// ---------------------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void boris(R u[3], const R E[3], const R B[3], R qdt2m) {
  const R umx = u[0] + qdt2m * E[0], umy = u[1] + qdt2m * E[1], umz = u[2] + qdt2m * E[2];
  const R f = qdt2m * rsq<R>(R(1) + umx * umx + umy * umy + umz * umz);
  const R tx = f * B[0], ty = f * B[1], tz = f * B[2];
  const R s = R(2) * rcp<R>(R(1) + tx * tx + ty * ty + tz * tz);
  const R sx = s * tx, sy = s * ty, sz = s * tz;
  const R upx = umx + (umy * tz - umz * ty);
  const R upy = umy + (umz * tx - umx * tz);
  const R upz = umz + (umx * ty - umy * tx);
  u[0] = umx + (upy * sz - upz * sy) + qdt2m * E[0];
  u[1] = umy + (upz * sx - upx * sz) + qdt2m * E[1];
  u[2] = umz + (upx * sy - upy * sx) + qdt2m * E[2];
}

// ---------------------------------------------------------------------------------------
// Esirkepov window along one axis.  x0 in [0,1) is the start offset and x1 in (-1,2) the
// end offset, both relative to the start cell.  Fills S0 and S1 on a window of W = ORDER+2
// integer nodes starting at start_cell + base.
// ---------------------------------------------------------------------------------------
template <int ORDER, typename R>
__device__ __forceinline__ void esk_axis(R x0, R x1, int& base, R S0[ORDER + 2], R S1[ORDER + 2]) {
  if constexpr (ORDER == 1) {
    const R f1 = floor_clamped<R>(x1, R(-1), R(1));
    const int c1 = (int)f1;                      // -1, 0 or 1
    const R d1 = x1 - f1;
    base = c1 < 0 ? c1 : 0;
    const int s0 = -base, s1 = c1 - base;        // 0 or 1 each
    const R a0 = R(1) - x0, a1 = x0, b0 = R(1) - d1, b1 = d1;
    S0[0] = s0 ? R(0) : a0;
    S0[1] = s0 ? a0 : a1;
    S0[2] = s0 ? a1 : R(0);
    S1[0] = s1 ? R(0) : b0;
    S1[1] = s1 ? b0 : b1;
    S1[2] = s1 ? b1 : R(0);
  } else {
    const int c0 = x0 >= R(0.5);
    const R fc1 = floor_clamped<R>(x1 + R(0.5), R(-1), R(2));
    const int c1 = (int)fc1;                     // -1 .. 2
    const R d0 = x0 - R(c0), d1 = x1 - fc1;
    base = (c0 < c1 ? c0 : c1) - 1;
    const int s0 = c0 - 1 - base, s1 = c1 - 1 - base;   // 0 or 1 each
    R a[3], b[3];
    {
      const R p = R(0.5) - d0, q = R(0.5) + d0;
      a[0] = R(0.5) * p * p; a[1] = R(0.75) - d0 * d0; a[2] = R(0.5) * q * q;
    }
    {
      const R p = R(0.5) - d1, q = R(0.5) + d1;
      b[0] = R(0.5) * p * p; b[1] = R(0.75) - d1 * d1; b[2] = R(0.5) * q * q;
    }
    S0[0] = s0 ? R(0) : a[0];
    S0[1] = s0 ? a[0] : a[1];
    S0[2] = s0 ? a[1] : a[2];
    S0[3] = s0 ? a[2] : R(0);
    S1[0] = s1 ? R(0) : b[0];
    S1[1] = s1 ? b[0] : b[1];
    S1[2] = s1 ? b[1] : b[2];
    S1[3] = s1 ? b[2] : R(0);
  }
}

// Per-segment constants in the kernel's precision.
template <typename R>
struct PushConst {
  R hdx, hdy, hdz;      // dt / (2 h): half-step displacement in cells per unit velocity
  R qdt2m;              // q dt / (2 m)
  R jx, jy, jz;         // -q h / dt per axis (Esirkepov current factor, times w)
  R q;                  // charge (2D Jz and rho, times w)
};

template <typename R>
__device__ __forceinline__ PushConst<R> push_const(const RunDesc& r, const SegDesc& s) {
  PushConst<R> c;
  c.hdx = R(0.5 * r.dt / r.dx);
  c.hdy = R(0.5 * r.dt / r.dy);
  c.hdz = R(0.5 * r.dt / r.dz);
  c.qdt2m = R(s.q * r.dt / (2.0 * s.m));
  c.jx = R(-s.q * r.dx / r.dt);
  c.jy = R(-s.q * r.dy / r.dt);
  c.jz = R(-s.q * r.dz / r.dt);
  c.q = R(s.q);
  return c;
}

// Esirkepov deposit of one particle (2D3V or 3D3V) through accessor A, whose frame places
// the start cell at c[] (accessor coordinates).  x0/x1 per axis as in esk_axis.
//   2D: Wx = dSx (S0y + S1y)/2 summed along x, Wy likewise, and
//       Wz = (S0x (2 S0y + S1y) + S1x (S0y + 2 S1y)) / 6   (= S0 S0 + dS S0/2 + S0 dS/2 + dS dS/3)
//   3D: Wx = dSx (S0y (2 S0z + S1z) + S1y (S0z + 2 S1z)) / 6 summed along x, cyclic.
// The accessor's scale (A.fold()) is folded into the per-particle factors.  Entries on the
// first W-1 nodes of every axis (and, along a running sum, before its last node) are the
// ones a path that keeps its nearest node fills: they go through add_core; the others are
// exactly zero for such a path and go through add, which skips zeros.
// with_rho: 0 no charge; 1 the charge at both ends of the path (rho0 at x0, rho1 at x1);
// 2 or 3 only the charge at the path's end, into rho0 (2) or rho1 (3) -- through the
// on-chip accessor into its single charge plane, which sits in rho0's place (charge_planes).
template <int DIM, int ORDER, typename R, class Acc>
__device__ __forceinline__ void deposit(const Acc& A, const int* c, const R* x0, const R* x1,
                                        R w, R vz_bar, const PushConst<R>& k, int with_rho) {
  constexpr int W = ORDER + 2;
  R S0x[W], S1x[W], S0y[W], S1y[W], S0z[W], S1z[W];
  int bx, by, bz = 0;
  esk_axis<ORDER>(x0[0], x1[0], bx, S0x, S1x);
  esk_axis<ORDER>(x0[1], x1[1], by, S0y, S1y);
  if constexpr (DIM == 3) esk_axis<ORDER>(x0[2], x1[2], bz, S0z, S1z);
  // The last node of an axis' window carries weight only for a path that changes its
  // nearest node along that axis.  When no lane of the wave has such a path, every entry
  // on that node is an exact zero and the wave skips it (a uniform branch).
  const bool lx = __ballot(S0x[W - 1] != R(0) || S1x[W - 1] != R(0)) != 0;
  const bool ly = __ballot(S0y[W - 1] != R(0) || S1y[W - 1] != R(0)) != 0;
  // A lane whose path keeps its nearest node along an axis has both shapes on the first W-1
  // nodes; each shape sums to 1 there, so the running sum of the current along that axis is
  // exactly zero at node W-2: the lane adds nothing there rather than the rounding residue.
  const bool xs = S0x[W - 1] == R(0) && S1x[W - 1] == R(0);
  const bool ys = S0y[W - 1] == R(0) && S1y[W - 1] == R(0);
  int xo[W], yo[W];
  if constexpr (Acc::kLinear) {
    // one base per particle (the window's first node, z included in 3D); every entry is a
    // compile-time offset from it
    const int wb = (DIM == 3 ? A.zo(c[2] + bz) : 0) + A.yo(c[1] + by) + A.xo(c[0] + bx);
#pragma unroll
    for (int a = 0; a < W; ++a) { xo[a] = wb + a; yo[a] = A.yo(a); }
  } else {
#pragma unroll
    for (int a = 0; a < W; ++a) { xo[a] = A.xo(c[0] + bx + a); yo[a] = A.yo(c[1] + by + a); }
  }
  const R fw = A.fold() * w;
  const R cx = k.jx * fw, cy = k.jy * fw;
  R dSx[W], dSy[W];
#pragma unroll
  for (int a = 0; a < W; ++a) { dSx[a] = S1x[a] - S0x[a]; dSy[a] = S1y[a] - S0y[a]; }
  if constexpr (DIM == 2) {
    const R cz = k.q * fw * vz_bar * R(1.0 / 6.0);
#pragma unroll
    for (int b = 0; b < W; ++b) {
      if (b == W - 1 && !ly) continue;
      const R hy = cx * R(0.5) * (S0y[b] + S1y[b]);
      R acc = R(0);
#pragma unroll
      for (int a = 0; a < W - 1; ++a) {
        acc += dSx[a] * hy;
        if (b < W - 1 && a < W - 2) A.add_core(F_JX, yo[b] + xo[a], acc);
        else A.add(F_JX, yo[b] + xo[a], a == W - 2 && xs ? R(0) : acc);
      }
    }
#pragma unroll
    for (int a = 0; a < W; ++a) {
      if (a == W - 1 && !lx) continue;
      const R hx = cy * R(0.5) * (S0x[a] + S1x[a]);
      R acc = R(0);
#pragma unroll
      for (int b = 0; b < W - 1; ++b) {
        acc += dSy[b] * hx;
        if (a < W - 1 && b < W - 2) A.add_core(F_JY, yo[b] + xo[a], acc);
        else A.add(F_JY, yo[b] + xo[a], b == W - 2 && ys ? R(0) : acc);
      }
    }
    R p0[W], p1[W];
#pragma unroll
    for (int a = 0; a < W; ++a) { p0[a] = cz * S0x[a]; p1[a] = cz * S1x[a]; }
#pragma unroll
    for (int b = 0; b < W; ++b) {
      if (b == W - 1 && !ly) continue;
      const R ay = R(2) * S0y[b] + S1y[b], by2 = S0y[b] + R(2) * S1y[b];
#pragma unroll
      for (int a = 0; a < W; ++a) {
        if (a == W - 1 && !lx) continue;
        const R v = p0[a] * ay + p1[a] * by2;
        if (a < W - 1 && b < W - 1) A.add_core(F_JZ, yo[b] + xo[a], v);
        else A.add(F_JZ, yo[b] + xo[a], v);
      }
    }
    if (with_rho) {
      const R qw = k.q * fw;
      if constexpr (Acc::kLinear) {
        // each shape on its own ORDER + 1 nodes (as in 3D below)
        constexpr int N = ORDER + 1;
        const int s0x = S0x[0] == R(0), s0y = S0y[0] == R(0);
        const int s1x = S1x[0] == R(0), s1y = S1y[0] == R(0);
        R a0[N], b0[N], a1[N], b1[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
          a0[i] = s0x ? S0x[i + 1] : S0x[i]; b0[i] = s0y ? S0y[i + 1] : S0y[i];
          a1[i] = s1x ? S1x[i + 1] : S1x[i]; b1[i] = s1y ? S1y[i + 1] : S1y[i];
        }
        const int o0 = xo[0] + s0x + A.yo(s0y), o1 = xo[0] + s1x + A.yo(s1y);
        const bool both = with_rho == 1;
#pragma unroll
        for (int b = 0; b < N; ++b)
#pragma unroll
          for (int a = 0; a < N; ++a) {
            if (both) A.add_core(F_R0, o0 + A.yo(b) + a, qw * a0[a] * b0[b]);
            A.add_core(both ? F_R1 : F_R0, o1 + A.yo(b) + a, qw * a1[a] * b1[b]);
          }
      } else {
        const int end = with_rho == 2 ? F_R0 : F_R1;
#pragma unroll
        for (int b = 0; b < W; ++b)
#pragma unroll
          for (int a = 0; a < W; ++a) {
            if ((a == W - 1 && !lx) || (b == W - 1 && !ly)) continue;
            if (with_rho == 1) A.add(F_R0, yo[b] + xo[a], qw * S0x[a] * S0y[b]);
            A.add(end, yo[b] + xo[a], qw * S1x[a] * S1y[b]);
          }
      }
    }
  } else {
    const bool lz = __ballot(S0z[W - 1] != R(0) || S1z[W - 1] != R(0)) != 0;
    const bool zs = S0z[W - 1] == R(0) && S1z[W - 1] == R(0);
    int zo[W];
    R dSz[W];
#pragma unroll
    for (int a = 0; a < W; ++a) {
      zo[a] = Acc::kLinear ? A.zo(a) : A.zo(c[2] + bz + a);   // (linear: base in xo)
      dSz[a] = S1z[a] - S0z[a];
    }
    const R cz = k.jz * fw;
    const R sixth = R(1.0 / 6.0);
    // Jx: running sum along x of dSx * Ryz
#pragma unroll
    for (int cc = 0; cc < W; ++cc)
#pragma unroll
      for (int b = 0; b < W; ++b) {
        if ((b == W - 1 && !ly) || (cc == W - 1 && !lz)) continue;
        const R ryz = cx * sixth * (S0y[b] * (R(2) * S0z[cc] + S1z[cc]) +
                                    S1y[b] * (S0z[cc] + R(2) * S1z[cc]));
        R acc = R(0);
#pragma unroll
        for (int a = 0; a < W - 1; ++a) {
          acc += dSx[a] * ryz;
          if (b < W - 1 && cc < W - 1 && a < W - 2) A.add_core(F_JX, zo[cc] + yo[b] + xo[a], acc);
          else A.add(F_JX, zo[cc] + yo[b] + xo[a], a == W - 2 && xs ? R(0) : acc);
        }
      }
#pragma unroll
    for (int cc = 0; cc < W; ++cc)
#pragma unroll
      for (int a = 0; a < W; ++a) {
        if ((a == W - 1 && !lx) || (cc == W - 1 && !lz)) continue;
        const R rxz = cy * sixth * (S0x[a] * (R(2) * S0z[cc] + S1z[cc]) +
                                    S1x[a] * (S0z[cc] + R(2) * S1z[cc]));
        R acc = R(0);
#pragma unroll
        for (int b = 0; b < W - 1; ++b) {
          acc += dSy[b] * rxz;
          if (a < W - 1 && cc < W - 1 && b < W - 2) A.add_core(F_JY, zo[cc] + yo[b] + xo[a], acc);
          else A.add(F_JY, zo[cc] + yo[b] + xo[a], b == W - 2 && ys ? R(0) : acc);
        }
      }
#pragma unroll
    for (int b = 0; b < W; ++b)
#pragma unroll
      for (int a = 0; a < W; ++a) {
        if ((a == W - 1 && !lx) || (b == W - 1 && !ly)) continue;
        const R rxy = cz * sixth * (S0x[a] * (R(2) * S0y[b] + S1y[b]) +
                                    S1x[a] * (S0y[b] + R(2) * S1y[b]));
        R acc = R(0);
#pragma unroll
        for (int cc = 0; cc < W - 1; ++cc) {
          acc += dSz[cc] * rxy;
          if (a < W - 1 && b < W - 1 && cc < W - 2) A.add_core(F_JZ, zo[cc] + yo[b] + xo[a], acc);
          else A.add(F_JZ, zo[cc] + yo[b] + xo[a], cc == W - 2 && zs ? R(0) : acc);
        }
      }
    if (with_rho) {
      const R qw = k.q * fw;
      if constexpr (Acc::kLinear) {
        // each shape is non-zero on ORDER + 1 consecutive nodes of the window, from node 0
        // or node 1 (the first node of a shape is never zero when it is in use): a base per
        // shape and lane, and (ORDER + 1)^3 unconditional adds at fixed offsets from it
        // instead of W^3 conditional ones
        constexpr int N = ORDER + 1;
        const int s0x = S0x[0] == R(0), s0y = S0y[0] == R(0), s0z = S0z[0] == R(0);
        const int s1x = S1x[0] == R(0), s1y = S1y[0] == R(0), s1z = S1z[0] == R(0);
        R a0[N], b0[N], c0[N], a1[N], b1[N], c1[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
          a0[i] = s0x ? S0x[i + 1] : S0x[i]; b0[i] = s0y ? S0y[i + 1] : S0y[i];
          c0[i] = s0z ? S0z[i + 1] : S0z[i]; a1[i] = s1x ? S1x[i + 1] : S1x[i];
          b1[i] = s1y ? S1y[i + 1] : S1y[i]; c1[i] = s1z ? S1z[i + 1] : S1z[i];
        }
        const int o0 = xo[0] + s0x + A.yo(s0y) + A.zo(s0z);
        const int o1 = xo[0] + s1x + A.yo(s1y) + A.zo(s1z);
        const bool both = with_rho == 1;
#pragma unroll
        for (int cc = 0; cc < N; ++cc)
#pragma unroll
          for (int b = 0; b < N; ++b)
#pragma unroll
            for (int a = 0; a < N; ++a) {
              const int off = A.zo(cc) + A.yo(b) + a;
              if (both) A.add_core(F_R0, o0 + off, qw * a0[a] * b0[b] * c0[cc]);
              A.add_core(both ? F_R1 : F_R0, o1 + off, qw * a1[a] * b1[b] * c1[cc]);
            }
      } else {
        const int end = with_rho == 2 ? F_R0 : F_R1;
#pragma unroll
        for (int cc = 0; cc < W; ++cc)
#pragma unroll
          for (int b = 0; b < W; ++b)
#pragma unroll
            for (int a = 0; a < W; ++a) {
              if ((a == W - 1 && !lx) || (b == W - 1 && !ly) || (cc == W - 1 && !lz)) continue;
              const int off = zo[cc] + yo[b] + xo[a];
              if (with_rho == 1) A.add(F_R0, off, qw * S0x[a] * S0y[b] * S0z[cc]);
              A.add(end, off, qw * S1x[a] * S1y[b] * S1z[cc]);
            }
      }
    }
  }
}


// ---------------------------------------------------------------------------------------
// Particle state in (cell, offset) form.
// ---------------------------------------------------------------------------------------
template <typename R>
struct PState {
  int c[3];      // global cell
  R o[3];        // offsets in [0,1)
  R u[3];
  R w;
  bool alive;
};

__device__ __forceinline__ void unpack_cell(int32_t cell, int dim, int c[3]) {
  if (dim == 2) {
    c[0] = cell & 0xFFFF;
    c[1] = cell >> 16;
    c[2] = 0;
  } else {
    c[0] = cell & 0x7FF;
    c[1] = (cell >> 11) & 0x7FF;
    c[2] = cell >> 22;
  }
}
__device__ __forceinline__ int32_t pack_cell(const int c[3], int dim) {
  return dim == 2 ? (c[1] << 16) | c[0] : (c[2] << 22) | (c[1] << 11) | c[0];
}

// The arrays of one species as global pointers, copied out of the descriptor once (they stay
// in scalar registers instead of being re-read after every store).
template <typename R>
struct PartPtrs {
  gptr<int32_t> cell;   // FP32: packed cells
  gptr<R> pos[3];       // FP32: float offsets; FP64: absolute double positions
  gptr<R> u[3];
  gptr<R> w;
  int nx, ny, nz;
  double dx, dy, dz;
};

template <typename R>
__device__ __forceinline__ PartPtrs<R> part_ptrs(const SegDesc& s, const RunDesc& r, bool alt = false) {
  void* const* a = alt ? s.alt : s.p;
  PartPtrs<R> q;
  q.cell = gp((int32_t*)a[P_CELL]);
  if (sizeof(R) == 4) {
    for (int d = 0; d < 3; ++d) q.pos[d] = gp((R*)a[P_OX + d]);
  } else {
    for (int d = 0; d < 3; ++d) q.pos[d] = gp((R*)a[P_X + d]);
  }
  for (int d = 0; d < 3; ++d) q.u[d] = gp((R*)a[P_UX + d]);
  q.w = gp((R*)a[P_W]);
  q.nx = r.nx; q.ny = r.ny; q.nz = r.nz;
  q.dx = r.dx; q.dy = r.dy; q.dz = r.dz;
  return q;
}

// Element p of a particle array through a 32-bit byte offset from the array's (uniform)
// base: the load or store can then take the base from scalar registers and one 32-bit
// offset per lane, shared by every array of the same element size, instead of a 64-bit
// address per array.  Slots are below 2^29 (check_species), so p * 8 fits.
template <typename T>
__device__ __forceinline__ gptr<T> at_byte(gptr<T> base, uint32_t off) {
  return (gptr<T>)((__attribute__((address_space(1))) char*)base + off);
}

// A particle's array words as stored: FP32 the packed cell and the offsets, FP64 the
// absolute positions (cell unused); then the momenta and the weight.  Every load of a
// particle, from its slot or from an escape record, decodes these words the same way.
template <typename R>
struct PWords {
  int32_t cell;
  R pos[3];
  R u[3];
  R w;
};

// The cell of a particle from its words (FP32: the packed cell; FP64: from the absolute
// position); false for a dead or invalid slot (as decode_particle's alive).
template <typename R, int DIM>
__device__ __forceinline__ bool decode_cell(const PartPtrs<R>& q, int32_t cell, const R* pos,
                                            int c[3]) {
  if constexpr (sizeof(R) == 4) {
    (void)pos;
    unpack_cell(cell < 0 ? 0 : cell, DIM, c);
    return cell >= 0 && c[0] < q.nx && c[1] < q.ny && (DIM == 2 || c[2] < q.nz);
  } else {
    (void)cell;
    const double h[3] = {q.dx, q.dy, q.dz};
    const int n[3] = {q.nx, q.ny, q.nz};
    bool alive = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d < DIM) {
        const double X = pos[d] / h[d];
        if (!(X >= 0.0 && X <= (double)n[d])) alive = false;
        int ci = (int)floor_clamped<double>(X, 0.0, (double)n[d]);
        c[d] = ci >= n[d] ? ci - n[d] : ci;
      } else {
        c[d] = 0;
      }
    }
    return alive;
  }
}

template <typename R, int DIM>
__device__ __forceinline__ void decode_particle(const PartPtrs<R>& q, const PWords<R>& x,
                                                PState<R>& ps) {
  if constexpr (sizeof(R) == 4) {
    unpack_cell(x.cell < 0 ? 0 : x.cell, DIM, ps.c);
    // a cell outside the box cannot come from the library; treat it like a dead slot
    ps.alive = x.cell >= 0 && ps.c[0] < q.nx && ps.c[1] < q.ny && (DIM == 2 || ps.c[2] < q.nz);
    ps.o[0] = x.pos[0];
    ps.o[1] = x.pos[1];
    ps.o[2] = DIM == 3 ? x.pos[2] : 0.f;
  } else {
    const double h[3] = {q.dx, q.dy, q.dz};
    const int n[3] = {q.nx, q.ny, q.nz};
    ps.alive = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d < DIM) {
        const double X = x.pos[d] / h[d];
        // positions outside [0, L] (or NaN) cannot come from the library: dead slot
        if (!(X >= 0.0 && X <= (double)n[d])) ps.alive = false;
        const double f = floor_clamped<double>(X, 0.0, (double)n[d]);
        int ci = (int)f;
        ps.o[d] = X - f;
        ci = ci >= n[d] ? ci - n[d] : ci;
        ps.c[d] = ci;
      } else {
        ps.c[d] = 0;
        ps.o[d] = 0.0;
      }
    }
  }
  ps.u[0] = x.u[0];
  ps.u[1] = x.u[1];
  ps.u[2] = x.u[2];
  ps.w = x.w;
}

// The words of slot p from the species' arrays.
template <typename R, int DIM>
__device__ __forceinline__ PWords<R> load_words(const PartPtrs<R>& q, int32_t p) {
  const uint32_t o4 = (uint32_t)p * 4u, oR = (uint32_t)p * (uint32_t)sizeof(R);
  PWords<R> x;
  x.cell = sizeof(R) == 4 ? *at_byte(q.cell, o4) : 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) x.pos[d] = d < DIM ? *at_byte(q.pos[d], oR) : R(0);
#pragma unroll
  for (int d = 0; d < 3; ++d) x.u[d] = *at_byte(q.u[d], oR);
  x.w = *at_byte(q.w, oR);
  return x;
}

// The cell of particle p only; false for a dead or invalid slot.
template <typename R, int DIM>
__device__ __forceinline__ bool load_cell(const PartPtrs<R>& q, int32_t p, int c[3]) {
  R pos[3] = {R(0), R(0), R(0)};
  int32_t cell = 0;
  if constexpr (sizeof(R) == 4) {
    cell = *at_byte(q.cell, (uint32_t)p * 4u);
  } else {
#pragma unroll
    for (int d = 0; d < DIM; ++d) pos[d] = *at_byte(q.pos[d], (uint32_t)p * 8u);
  }
  return decode_cell<R, DIM>(q, cell, pos, c);
}

template <typename R, int DIM>
__device__ __forceinline__ void load_particle(const PartPtrs<R>& q, int32_t p, PState<R>& ps) {
  decode_particle<R, DIM>(q, load_words<R, DIM>(q, p), ps);
}

// Escape records: the words of an escaped particle in eight consecutive slots of the kernel's
// precision (FP32: the packed cell's bits, three offsets, three momenta, the weight; FP64:
// three positions, three momenta, the weight, one unused slot), so that the re-binned pass
// reads each particle as one contiguous 32- or 64-byte record instead of eight scattered
// words.  Unused position slots (2D) hold zero.
template <typename R>
struct alignas(8 * sizeof(R)) EscRec {
  R v[8];
};

template <typename R>
__device__ __forceinline__ EscRec<R> rec_of(const PWords<R>& x) {
  EscRec<R> e;
  if constexpr (sizeof(R) == 4) {
    e.v[0] = __int_as_float(x.cell);
    e.v[1] = x.pos[0]; e.v[2] = x.pos[1]; e.v[3] = x.pos[2];
  } else {
    e.v[0] = x.pos[0]; e.v[1] = x.pos[1]; e.v[2] = x.pos[2]; e.v[3] = R(0);
  }
  e.v[4] = x.u[0]; e.v[5] = x.u[1]; e.v[6] = x.u[2]; e.v[7] = x.w;
  return e;
}

template <typename R>
__device__ __forceinline__ PWords<R> words_of(const EscRec<R>& e) {
  PWords<R> x;
  if constexpr (sizeof(R) == 4) {
    x.cell = __float_as_int(e.v[0]);
    x.pos[0] = e.v[1]; x.pos[1] = e.v[2]; x.pos[2] = e.v[3];
  } else {
    x.cell = 0;
    x.pos[0] = e.v[0]; x.pos[1] = e.v[1]; x.pos[2] = e.v[2];
  }
  x.u[0] = e.v[4]; x.u[1] = e.v[5]; x.u[2] = e.v[6]; x.w = e.v[7];
  return x;
}

// Records move as 16-byte vectors (two per FP32 record, four per FP64 record).
template <typename R>
using Rec16 = R __attribute__((ext_vector_type(16 / sizeof(R))));

template <typename R>
__device__ __forceinline__ void store_rec(void* base, int64_t k, const EscRec<R>& e) {
  constexpr int NV = (int)(sizeof(EscRec<R>) / 16), L = (int)(16 / sizeof(R));
  gptr<Rec16<R>> b = gp((Rec16<R>*)base) + k * NV;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    Rec16<R> v;
#pragma unroll
    for (int j = 0; j < L; ++j) v[j] = e.v[i * L + j];
    b[i] = v;
  }
}

template <typename R>
__device__ __forceinline__ EscRec<R> load_rec(const void* base, int64_t k) {
  constexpr int NV = (int)(sizeof(EscRec<R>) / 16), L = (int)(16 / sizeof(R));
  gptr<const Rec16<R>> b = gp((const Rec16<R>*)base) + k * NV;
  EscRec<R> e;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const Rec16<R> v = b[i];
#pragma unroll
    for (int j = 0; j < L; ++j) e.v[i * L + j] = v[j];
  }
  return e;
}

// The cell from a record only (the first slot in FP32; the positions in FP64).
template <typename R, int DIM>
__device__ __forceinline__ bool rec_cell(const PartPtrs<R>& q, const void* base, int64_t k,
                                         int c[3]) {
  const R* e = ((const EscRec<R>*)base)[k].v;
  if constexpr (sizeof(R) == 4) {
    const R pos[3] = {0.f, 0.f, 0.f};
    return decode_cell<R, DIM>(q, __float_as_int(*gp(e)), pos, c);
  } else {
    R pos[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) pos[d] = gp(e)[d];
    return decode_cell<R, DIM>(q, 0, pos, c);
  }
}

template <typename R, int DIM>
__device__ __forceinline__ void load_particle(const SegDesc& s, const RunDesc& r, int32_t p,
                                              PState<R>& ps) {
  load_particle<R, DIM>(part_ptrs<R>(s, r), p, ps);
}

// New cell and offset from the end offset x1 (relative to the start cell).  If the offset
// rounds up to 1 (x1 a tiny negative number) the particle is put at the start of the cell
// it came from instead; the error is below half an ulp of 1.
template <typename R>
__device__ __forceinline__ void advance_cell(int& c, R& o, R x1, int n) {
  const R f = floor_clamped<R>(x1, R(-1), R(1));
  int k = (int)f;
  R on = x1 - f;
  if (on >= R(1)) { on = R(0); k += 1; }
  c = wrapi(c + k, n);
  o = on;
}

template <typename R, int DIM>
__device__ __forceinline__ void store_particle(const PartPtrs<R>& q, int32_t p,
                                               const PState<R>& ps) {
  const uint32_t o4 = (uint32_t)p * 4u, oR = (uint32_t)p * (uint32_t)sizeof(R);
  // a particle removed during this step gets the dead marker (cell -1 / x = -1) in place of
  // its position; the other words are written either way (no branch around the stores)
  if constexpr (sizeof(R) == 4) {
    *at_byte(q.cell, o4) = ps.alive ? pack_cell(ps.c, DIM) : -1;
    *at_byte(q.pos[0], oR) = ps.o[0];
    *at_byte(q.pos[1], oR) = ps.o[1];
    if (DIM == 3) *at_byte(q.pos[2], oR) = ps.o[2];
  } else {
    const double h[3] = {q.dx, q.dy, q.dz};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double x = ((double)ps.c[d] + ps.o[d]) * h[d];
      *at_byte(q.pos[d], oR) = (d == 0 && !ps.alive) ? -1.0 : x;
    }
  }
  *at_byte(q.u[0], oR) = ps.u[0];
  *at_byte(q.u[1], oR) = ps.u[1];
  *at_byte(q.u[2], oR) = ps.u[2];
}

template <typename R, int DIM>
__device__ __forceinline__ void store_particle(const SegDesc& s, const RunDesc& r, int32_t p,
                                               const PState<R>& ps) {
  store_particle<R, DIM>(part_ptrs<R>(s, r), p, ps);
}

// The particle part of Algorithm 1 for one particle: half push, gather at the half position,
// Boris, second half push.  Fields come through accessor A whose frame has the particle's
// start cell at a[].  Outputs, per axis:
//   pc, po  the half-step position x^{n+1/2} as (cell in A's frame, offset in [0,1)): the
//           gather point and the start of the deposited path;
//   pe      the path end x^{n+1/2} + dt v^{n+1}, as an offset relative to pc;
//   x1      the new position x^{n+1} (the path midpoint), relative to the start cell.
// The deposited path is the trajectory over one dt centred on the end of the step
// (Sec. 3.1 with the time levels of Eq. 3), so vz1 = v_z^{n+1} is the 2D Jz velocity.
// The first half push: xh = x^{n+1/2} relative to the start cell, and the same point as
// (cell pc in the frame whose start cell is a[], offset po in [0,1)).
template <int DIM, typename R>
__device__ __forceinline__ void half_push(const int* a, const PState<R>& ps,
                                          const PushConst<R>& k, int pc[3], R po[3],
                                          R xh[3]) {
  const R ig0 = rsq<R>(R(1) + ps.u[0] * ps.u[0] + ps.u[1] * ps.u[1] + ps.u[2] * ps.u[2]);
  const R hd[3] = {k.hdx, k.hdy, k.hdz};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d < DIM) {
      xh[d] = ps.o[d] + hd[d] * ps.u[d] * ig0;
      const R f = floor_clamped<R>(xh[d], R(-1), R(1));
      pc[d] = a[d] + (int)f;
      po[d] = xh[d] - f;
    } else {
      xh[d] = R(0); pc[d] = 0; po[d] = R(0);
    }
  }
}

// Whether every node the gather at (pc, po) reads lies in [0, lim] on every axis.  Per axis
// the integer-lattice weights sit on [pc + up - 1, pc + up + 1] (quadratic) or [pc, pc + 1]
// (CIC), the half-lattice ones on [pc - 1, pc + 1] or [pc - 1 + up, pc + up], up = (po >=
// 1/2); the union is [pc - 1, pc + 1 + up] or [pc - 1 + up, pc + 1].
template <int DIM, int ORDER, typename R>
__device__ __forceinline__ bool gather_fits(const int* pc, const R* po, const int* lim) {
  bool fit = true;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int up = po[d] >= R(0.5);
    const int lo = ORDER == 2 ? pc[d] - 1 : pc[d] - 1 + up;
    const int hi = ORDER == 2 ? pc[d] + 1 + up : pc[d] + 1;
    fit = fit && lo >= 0 && hi <= lim[d];
  }
  return fit;
}

// Whether every node the deposit of the path po -> pe (offsets relative to cell pc) touches
// lies in [0, lim] on every axis.  The window of esk_axis starts at pc + base; its last node
// (W - 1) carries weight only for a path that changes its nearest node, and deposit() adds
// nothing there otherwise (exact zeros are skipped), so the nodes touched are
// [pc + base, pc + base + W - 2 + cross].
template <int DIM, int ORDER, typename R>
__device__ __forceinline__ bool deposit_fits(const int* pc, const R* po, const R* pe,
                                             const int* lim) {
  bool fit = true;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    int base, cross;
    if constexpr (ORDER == 1) {
      const int c1 = (int)floor_clamped<R>(pe[d], R(-1), R(1));
      base = c1 < 0 ? c1 : 0;
      cross = c1 != 0;
    } else {
      const int c0 = po[d] >= R(0.5);
      const int c1 = (int)floor_clamped<R>(pe[d] + R(0.5), R(-1), R(2));
      base = (c0 < c1 ? c0 : c1) - 1;
      cross = c0 != c1;
    }
    const int lo = pc[d] + base, hi = pc[d] + base + ORDER + cross;   // W - 2 = ORDER
    fit = fit && lo >= 0 && hi <= lim[d];
  }
  return fit;
}

// The rest of the particle push after half_push: gather at (pc, po), Boris, second half.
template <int DIM, int ORDER, typename R, class Acc>
__device__ __forceinline__ void push_rest(const Acc& A, const int* pc, const R* po,
                                          const R* xh, PState<R>& ps, const PushConst<R>& k,
                                          R pe[3], R x1[3], R& vz1, R& gamma1) {
  const R hd[3] = {k.hdx, k.hdy, k.hdz};
  R E[3], B[3];
  gather<DIM, ORDER>(A, pc, po, E, B);
  boris<R>(ps.u, E, B, k.qdt2m);
  const R u2 = ps.u[0] * ps.u[0] + ps.u[1] * ps.u[1] + ps.u[2] * ps.u[2];
  const R ig1 = rsq<R>(R(1) + u2);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const R half = d < DIM ? hd[d] * ps.u[d] * ig1 : R(0);
    x1[d] = xh[d] + half;
    pe[d] = po[d] + R(2) * half;
  }
  vz1 = ps.u[2] * ig1;
  gamma1 = R(1) / ig1;
}

template <int DIM, int ORDER, typename R, class Acc>
__device__ __forceinline__ void push(const Acc& A, const int* a, PState<R>& ps,
                                     const PushConst<R>& k, int pc[3], R po[3], R pe[3],
                                     R x1[3], R& vz1, R& gamma1) {
  R xh[3];
  half_push<DIM>(a, ps, k, pc, po, xh);
  push_rest<DIM, ORDER>(A, pc, po, xh, ps, k, pe, x1, vz1, gamma1);
}

// Global-memory accumulator over a run's field arrays.
template <typename R>
__device__ __forceinline__ GlobalAcc<R> global_acc(const RunDesc& r) {
  GlobalAcc<R> A;
#pragma unroll
  for (int c = 0; c < F_NUM; ++c) A.f[c] = gp((R*)r.f[c]);
  A.nx = r.nx; A.ny = r.ny; A.nz = r.nz;
  return A;
}

// =======================================================================================
// Descriptor lookup and wave/block utilities shared by the kernels
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

}  // namespace lpic
