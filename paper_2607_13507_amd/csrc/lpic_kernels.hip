// HIP kernels of the PIC hot path (gfx950, wave64).  No matrix cores: nothing here is a
// dense contraction.  The particle stream is structure-of-arrays and read/written once per
// step with unit stride; field tiles are staged in LDS for the gather and the current of a
// tile is accumulated in LDS, then flushed with one global atomic per non-zero cell.
#include <cstring>

#include "lpic_internal.hpp"

namespace lpic {

__global__ void k_fill_zero_u32(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// =======================================================================================
// Yee field half updates (Sec. 3.2, Eqs. 3-4), periodic by index wrap.
// =======================================================================================
struct CellIdx {
  int64_t c, cim, cip, cjm, cjp, ckm, ckp;
  int64_t row;   // k ny + j
  int i;         // x index
};

__device__ __forceinline__ bool cell_index(const RunDesc& r, int blk, int dim, CellIdx& x) {
  const int64_t plane = (int64_t)r.nx * r.ny;
  const int64_t ncell = plane * (dim == 3 ? r.nz : 1);
  const int64_t c = (int64_t)blk * 256 + threadIdx.x;
  if (c >= ncell) return false;
  int i, j, k;
  if (ncell <= 0x7fffffff) {   // 32-bit index arithmetic (no 64-bit division)
    const uint32_t cc = (uint32_t)c, rest = cc / (uint32_t)r.nx;
    i = (int)(cc - rest * (uint32_t)r.nx);
    j = (int)(rest % (uint32_t)r.ny);
    k = (int)(rest / (uint32_t)r.ny);
  } else {
    const int64_t rest = c / r.nx;
    i = (int)(c - rest * r.nx);
    j = (int)(rest % r.ny);
    k = (int)(rest / r.ny);
  }
  x.i = i;
  x.c = c;
  x.row = (int64_t)k * r.ny + j;
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

// E += h (curl B - J) at one cell: the increments (shared by the edge kernel).
template <typename R, int DIM>
__device__ __forceinline__ void yee_e_delta(const gptr<R>* f, const CellIdx& x, R hx, R hy,
                                            R hz, R hh, R& dex, R& dey, R& dez) {
  const R bx = f[F_BX][x.c], by = f[F_BY][x.c], bz = f[F_BZ][x.c];
  const R jx = f[F_JX][x.c], jy = f[F_JY][x.c], jz = f[F_JZ][x.c];
  dex = hy * (bz - f[F_BZ][x.cjm]) - hh * jx;
  dey = -hx * (bz - f[F_BZ][x.cim]) - hh * jy;
  dez = hx * (by - f[F_BY][x.cim]) - hy * (bx - f[F_BX][x.cjm]) - hh * jz;
  if (DIM == 3) {
    dex -= hz * (by - f[F_BY][x.ckm]);
    dey += hz * (bx - f[F_BX][x.ckm]);
  }
}

// B -= h curl E at one cell: the increments.
template <typename R, int DIM>
__device__ __forceinline__ void yee_b_delta(const gptr<R>* f, const CellIdx& x, R hx, R hy,
                                            R hz, R& dbx, R& dby, R& dbz) {
  const R ex = f[F_EX][x.c], ey = f[F_EY][x.c], ez = f[F_EZ][x.c];
  dbx = -hy * (f[F_EZ][x.cjp] - ez);
  dby = hx * (f[F_EZ][x.cip] - ez);
  dbz = -hx * (f[F_EY][x.cip] - ey) + hy * (f[F_EX][x.cjp] - ex);
  if (DIM == 3) {
    dbx += hz * (f[F_EY][x.ckp] - ey);
    dby -= hz * (f[F_EX][x.ckp] - ex);
  }
}

// Open x ends, first-order Mur condition on a tangential component u of the edge column:
// u_new(edge) = u_old(inner) + k (u_new(inner) - u_old(edge)), k = (h - dx)/(h + dx).  The
// thread of the inner column applies it (it knows u_old and u_new there, and the edge
// column's own thread leaves u alone), so no thread reads a value another one writes.
// halves = 2: the update is two equal half updates of step h/2 merged into one (the inner
// increment is d = 2 d_half), and the condition is applied twice.
template <typename R>
__device__ __forceinline__ R mur_edge(R u_edge_old, R u_in_old, R d, double h, double dx,
                                      int halves) {
  if (halves == 2) {
    const R k = R((0.5 * h - dx) / (0.5 * h + dx));
    const R u_in_mid = u_in_old + R(0.5) * d;
    const R u_edge_mid = u_in_old + k * (u_in_mid - u_edge_old);
    return u_in_mid + k * ((u_in_old + d) - u_edge_mid);
  }
  const R k = R((h - dx) / (h + dx));
  return u_in_old + k * ((u_in_old + d) - u_edge_old);
}

// ---------------------------------------------------------------------------------------
// Convolutional PML at the open x ends (lpic_set_pml).  The auxiliary values psi are held
// in units of a difference (psi * dx), so that a stretched difference is D/kappa + psi with
// D the plain difference of two neighbouring values.  Every field update of a simulation
// is made of half steps dt/2 (an E update of a whole dt between two steps is two merged
// halves), so the recursion coefficients are a per-slot table for that step.
// ---------------------------------------------------------------------------------------
// Slot of array column i in the auxiliary arrays: 0 .. L-1 the left layer, L .. 2L-1 the
// right one, -1 outside both.
__device__ __forceinline__ int pml_slot(const RunDesc& r, int i) {
  const int L = r.pml_cells;
  if (L == 0) return -1;
  const int p = box_x(r, i);
  return p < L ? p : (p >= r.nx - L ? p - r.nx + 2 * L : -1);
}

// Recursion coefficients b, c and 1/kappa at slot `slot` (B-side locations lie half a
// column further in +x than the E-side ones).
template <typename R>
__device__ __forceinline__ void pml_coef(const RunDesc& r, bool bside, int slot, R& b, R& c,
                                         R& ik) {
  const R* t = (const R*)r.pml_tab + ((bside ? 2 * r.pml_cells : 0) + slot) * 3;
  b = t[0];
  c = t[1];
  ik = t[2];
}

// Index of psi for component comp (0 Ey, 1 Ez, 2 By, 3 Bz) at (row, slot) in half `half`.
__device__ __forceinline__ int64_t pml_index(const RunDesc& r, int half, int comp, int64_t row,
                                             int slot) {
  const int64_t rows = (int64_t)r.ny * r.nz;
  return ((int64_t)(half * 4 + comp) * rows + row) * (2 * r.pml_cells) + slot;
}

__device__ __forceinline__ int pml_half(const RunDesc& r) {
  return r.psi_parity ? (*r.psi_parity & 1) : 0;
}

// One stretched x difference of component comp at (row, slot), in place in the current
// half: advances psi over `steps` half-step updates with the same plain difference D (an E
// update of a whole dt made of two merged halves takes steps = 2 and returns the mean of
// the two stretched differences) and returns the stretched difference.
template <typename R>
__device__ __forceinline__ R pml_stretch(const RunDesc& r, int comp, int64_t row, int slot,
                                         int steps, R D) {
  R b, c, ik;
  pml_coef<R>(r, comp >= 2, slot, b, c, ik);
  R* psi = (R*)r.psi + pml_index(r, pml_half(r), comp, row, slot);
  const R p1 = b * *psi + c * D;
  if (steps == 1) {
    *psi = p1;
    return D * ik + p1;
  }
  const R p2 = b * p1 + c * D;
  *psi = p2;
  return D * ik + R(0.5) * (p1 + p2);
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_yee_e(Tables T, double frac, int zero_j, int halves) {
  int blk;
  const RunDesc& r = run_of(T, cell_block(T, blk));
  CellIdx x;
  if (!cell_index(r, blk, DIM, x)) return;
  gptr<R> f[F_NUM];
#pragma unroll
  for (int c = 0; c < F_NUM; ++c) f[c] = gp((R*)r.f[c]);
  const double h = frac * r.dt;
  const R hx = R(h / r.dx), hy = R(h / r.dy), hz = R(DIM == 3 ? h / r.dz : 0.0), hh = R(h);
  R dex, dey, dez;
  yee_e_delta<R, DIM>(f, x, hx, hy, hz, hh, dex, dey, dez);
  const int ps = pml_slot(r, x.i);
  if (ps >= 0) {   // in a PML layer: the x differences of Bz and By are stretched
    const R dbz = f[F_BZ][x.c] - f[F_BZ][x.cim], dby = f[F_BY][x.c] - f[F_BY][x.cim];
    const int64_t row = x.row;
    dey += hx * (dbz - pml_stretch<R>(r, 0, row, ps, halves, dbz));
    dez -= hx * (dby - pml_stretch<R>(r, 1, row, ps, halves, dby));
  }
  f[F_EX][x.c] += dex;
  const int bxi = box_x(r, x.i);   // box column (a moving window shifts the arrays' origin)
  const bool mur = r.open_x && r.pml_cells == 0;
  if (mur && bxi == 1) {   // Mur for column 0 (same j, k)
    const R ey1 = f[F_EY][x.c], ez1 = f[F_EZ][x.c];
    f[F_EY][x.cim] = mur_edge<R>(f[F_EY][x.cim], ey1, dey, h, r.dx, halves);
    f[F_EZ][x.cim] = mur_edge<R>(f[F_EZ][x.cim], ez1, dez, h, r.dx, halves);
  }
  if (!(mur && bxi == 0)) {   // column 0 of an open end: set by the thread of column 1
    f[F_EY][x.c] += dey;
    f[F_EZ][x.c] += dez;
  }
  if (zero_j) {   // 1: clear J and the charge arrays (when given); 2: J only; 3: J and
                  // rho0; 4: J and rho1
    f[F_JX][x.c] = R(0);
    f[F_JY][x.c] = R(0);
    f[F_JZ][x.c] = R(0);
    if ((zero_j == 1 || zero_j == 3) && f[F_R0]) f[F_R0][x.c] = R(0);
    if ((zero_j == 1 || zero_j == 4) && f[F_R1]) f[F_R1][x.c] = R(0);
  }
}

// Antenna current on node (j, k) of column ia at time t (the current component is Jy for
// pol 1, Jz for pol 2); false outside the pulse envelope.
template <int DIM>
__device__ __forceinline__ bool antenna_current(const RunDesc& r, double t_abs, int j, int k,
                                                double& jant) {
  const LaserDesc& L = r.laser;
  const double t = t_abs - L.t0;
  if (!(t >= 0.0 && t <= L.tau)) return false;
  const double y = (j + (L.pol == 1 ? 0.5 : 0.0)) * r.dy;
  const double z = DIM == 3 ? (k + (L.pol == 2 ? 0.5 : 0.0)) * r.dz : L.zc;
  const double env = sin(M_PI * t / L.tau);
  const double r2 = (y - L.yc) * (y - L.yc) + (z - L.zc) * (z - L.zc);
  const double einc = L.e0 * env * env * sin(L.omega * t) * exp(-r2 / (L.waist * L.waist));
  jant = -2.0 * einc / r.dx;
  return true;
}

// ---------------------------------------------------------------------------------------
// Tile-edge snapshot of the fused 2D field update (FieldBands).  Cell (i, j) of a run lies
// in field tile (i >> lx, j >> ly) at (li, lj); the tile's slice of component k starts at
// ((tile0 + tile) * 6 + k) * 3 (tx + ty) and holds columns li = 0, 1, tx-1 (ty values
// each), then rows lj = 0, 1, ty-1 (tx values each).  A corner cell is in both.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int band_col(int li, int tx) { return li <= 1 ? li : (li == tx - 1 ? 2 : -1); }

// Snapshot index of cell (i, j), component k; the cell must lie on an edge band.
__device__ __forceinline__ int64_t band_at(const FieldBands& Bd, int ntx, int64_t tile0, int i,
                                          int j, int k) {
  const int ti = i >> Bd.lx, tj = j >> Bd.ly;
  const int li = i - (ti << Bd.lx), lj = j - (tj << Bd.ly);
  const int64_t base = ((tile0 + (int64_t)tj * ntx + ti) * 6 + k) * (3 * (Bd.tx + Bd.ty));
  const int cb = band_col(li, Bd.tx);
  if (cb >= 0) return base + cb * Bd.ty + lj;
  return base + 3 * Bd.ty + band_col(lj, Bd.ty) * Bd.tx + li;
}

// Publishes value v of a cell at (li, lj) of a tile whose slice of component 0 starts at
// `base` (stride 3 (tx + ty) per component).
template <typename R>
__device__ __forceinline__ void band_put(R* out, const FieldBands& Bd, int64_t base, int li,
                                         int lj, int k, R v) {
  const int64_t b = base + (int64_t)k * (3 * (Bd.tx + Bd.ty));
  const int cb = band_col(li, Bd.tx), rb = band_col(lj, Bd.ty);
  if (cb >= 0) out[b + cb * Bd.ty + lj] = v;
  if (rb >= 0) out[b + 3 * Bd.ty + rb * Bd.tx + li] = v;
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_yee_b(Tables T, double frac, FieldBands Bd) {
  int blk;
  const int ri = cell_block(T, blk);
  const RunDesc& r = run_of(T, ri);
  CellIdx x;
  if (!cell_index(r, blk, DIM, x)) return;
  gptr<R> f[F_NUM];
#pragma unroll
  for (int c = 0; c < F_NUM; ++c) f[c] = gp((R*)r.f[c]);
  const double h = frac * r.dt;
  const R hx = R(h / r.dx), hy = R(h / r.dy), hz = R(DIM == 3 ? h / r.dz : 0.0);
  R dbx, dby, dbz;
  yee_b_delta<R, DIM>(f, x, hx, hy, hz, dbx, dby, dbz);
  const int ps = pml_slot(r, x.i);
  if (ps >= 0) {   // in a PML layer: the x differences of Ez and Ey are stretched
    const R dez = f[F_EZ][x.cip] - f[F_EZ][x.c], dey = f[F_EY][x.cip] - f[F_EY][x.c];
    const int64_t row = x.row;
    dby -= hx * (dez - pml_stretch<R>(r, 2, row, ps, 1, dez));
    dbz += hx * (dey - pml_stretch<R>(r, 3, row, ps, 1, dey));
  }
  const R bx = f[F_BX][x.c] + dbx;
  f[F_BX][x.c] = bx;
  const int bxi = box_x(r, x.i);   // box column (a moving window shifts the arrays' origin)
  const bool mur = r.open_x && r.pml_cells == 0;
  const bool edge_in = mur && bxi == r.nx - 2;
  const bool edge = mur && bxi == r.nx - 1;
  R by_e = R(0), bz_e = R(0);
  if (edge_in) {   // Mur for column nx-1 (same j, k)
    const R by1 = f[F_BY][x.c], bz1 = f[F_BZ][x.c];
    by_e = mur_edge<R>(f[F_BY][x.cip], by1, dby, h, r.dx, 1);
    bz_e = mur_edge<R>(f[F_BZ][x.cip], bz1, dbz, h, r.dx, 1);
    f[F_BY][x.cip] = by_e;
    f[F_BZ][x.cip] = bz_e;
  }
  R by = R(0), bz = R(0);
  if (!edge) {   // last column of an open end: set by column nx-2
    by = f[F_BY][x.c] + dby;
    bz = f[F_BZ][x.c] + dbz;
    f[F_BY][x.c] = by;
    f[F_BZ][x.c] = bz;
  }
  if (DIM == 2 && Bd.base) {
    const int j = (int)(x.c / r.nx);
    const int ti = x.i >> Bd.lx, tj = j >> Bd.ly;
    const int li = x.i - (ti << Bd.lx), lj = j - (tj << Bd.ly);
    const int ntx = r.nx >> Bd.lx;
    R* out = (R*)Bd.base + (int64_t)(*Bd.parity & 1) * Bd.half;
    const int64_t base = (Bd.tile_pfx[ri] + (int64_t)tj * ntx + ti) * 6 * (3 * (Bd.tx + Bd.ty));
    if (band_col(li, Bd.tx) >= 0 || band_col(lj, Bd.ty) >= 0) {
      band_put(out, Bd, base, li, lj, 0, (R)f[F_EX][x.c]);
      band_put(out, Bd, base, li, lj, 1, (R)f[F_EY][x.c]);
      band_put(out, Bd, base, li, lj, 2, (R)f[F_EZ][x.c]);
      band_put(out, Bd, base, li, lj, 3, bx);
      if (!edge) {
        band_put(out, Bd, base, li, lj, 4, by);
        band_put(out, Bd, base, li, lj, 5, bz);
      }
    }
    if (edge_in) {   // column nx-1: the last column of this thread's tile (tx divides nx)
      band_put(out, Bd, base, li + 1, lj, 4, by_e);
      band_put(out, Bd, base, li + 1, lj, 5, bz_e);
    }
  }
}

// ---------------------------------------------------------------------------------------
// The field updates between the particle pushes of two 2D steps in one pass per tile:
// B += (dt/2) (-curl E), E += dt (curl B - J), B += (dt/2) (-curl E) -- the same arithmetic,
// cell by cell, as k_yee_b, k_yee_e (two merged halves) and k_yee_b in sequence.  The output
// tile [a, a+tx) x [c, c+ty) needs E on [a-1, a+tx+2) x [c-1, c+ty+2) and B on
// [a-1, a+tx+1) x [c-1, c+ty+1); its own cells come from the field arrays, the others from
// the neighbours' edge snapshot (never from the arrays, which the neighbours overwrite during
// this launch).  Cells outside the output tile are recomputed redundantly.  With open x
// ends, values computed for a wrapped image of column 0 or nx-1 only feed components that
// the open-end condition replaces, so they are left as computed.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int wrap_once(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

template <int N> struct Log2 { static constexpr int v = 1 + Log2<N / 2>::v; };
template <> struct Log2<1> { static constexpr int v = 0; };

// Cell h of the halo ring of a region (TX + 1 + HI) x (TY + 1 + HI) whose interior TX x TY
// starts at (1, 1): first the 1 + HI full rows (v = 0, TY + 1, ..), then the 1 + HI columns
// (u = 0, TX + 1, ..) of the interior rows.
template <int TX, int TY, int HI>
__device__ __forceinline__ void ring_cell(int h, int& u, int& v) {
  constexpr int W = TX + 1 + HI;
  if (h < (1 + HI) * W) {
    const int r = h / W;
    u = h - r * W;
    v = r == 0 ? 0 : TY + r;
  } else {
    h -= (1 + HI) * W;
    const int r = h / TY;
    v = 1 + h - r * TY;
    u = r == 0 ? 0 : TX + r;
  }
}

template <typename R, int TX, int TY, bool PML>
__global__ __launch_bounds__(256) void k_yee_mid(Tables T, FieldBands Bd) {
  constexpr int EW = TX + 3, EH = TY + 3, BW = TX + 2, BH = TY + 2, NC = TX * TY;
  constexpr int LX = Log2<TX>::v;
  constexpr int PER = (NC + 255) / 256;                    // interior cells per thread
  constexpr int ER = EW * EH - NC, BR = BW * BH - NC;      // halo rings of E and B
  constexpr int JR = TX + TY + 1;                          // J outside the tile that E needs
  constexpr int NER = (ER + 255) / 256, NBR = (BR + 255) / 256, NJR = (JR + 255) / 256;
  static_assert(TX <= MID_MAX_TX && TY <= MID_MAX_TY, "field tile too large");
  __shared__ R sE[3][EW * EH];
  __shared__ R sB[3][BW * BH];
  int blk;
  const int ri = cell_block(T, blk);   // blk: tile of the run (T.run_blk is the tile prefix)
  const RunDesc& r = run_of(T, ri);
  const int nx = r.nx, ny = r.ny;
  const int ntx = nx / TX;
  int tj = blk / ntx, ti = blk - tj * ntx;
  if (PML && r.pml_cells > 0) {
    // the tile columns that reach into a layer (ke at each end) come first, so that their
    // longer work overlaps the interior tiles instead of trailing them
    const int ke = (r.pml_cells + TX) / TX, nty = ny / TY;
    if (2 * ke < ntx) {
      if (blk < 2 * ke * nty) {
        const int col = blk / nty;
        tj = blk - col * nty;
        ti = col < ke ? col : ntx - 2 * ke + col;
      } else {
        const int rest = blk - 2 * ke * nty, ncol = ntx - 2 * ke;
        tj = rest / ncol;
        ti = ke + rest - tj * ncol;
      }
    }
  }
  const int tile = tj * ntx + ti;
  const int a = ti * TX, c = tj * TY;
  const int64_t tile0 = Bd.tile_pfx[ri];
  const int cur = *Bd.parity & 1;
  const R* bin = (const R*)Bd.base + (int64_t)cur * Bd.half;
  R* bout = (R*)Bd.base + (int64_t)(cur ^ 1) * Bd.half;
  gptr<R> f[F_NUM];
#pragma unroll
  for (int k = 0; k < F_NUM; ++k) f[k] = gp((R*)r.f[k]);
  const int tid = threadIdx.x;
  // the antenna current of this step where a run has one, added to J in the E update
  // exactly as the antenna kernel would have added it to the array (that kernel does not
  // run before a fused update; the clock advances in the launch that follows).  Column ia
  // is local column u_ant of the E-update range [a, a + TX] (maybe as the wrapped image of
  // column 0); it is computed first, per row, while nothing else is live.
  __shared__ R sAnt[MID_MAX_TY + 2];
  int u_ant = -1;
  if (r.has_laser && Bd.step) {
    const int ia = array_x(r, r.laser.ia);
    const int ua = ia >= a && ia <= a + TX ? ia - a + 1 : (ia == 0 && a + TX == nx ? TX + 1 : -1);
    double jant;
    const double t_ant = (double)(*Bd.step + 1) * r.dt;
    if (ua > 0 && antenna_current<2>(r, t_ant, 0, 0, jant)) {   // inside the envelope
      u_ant = ua;
      if (tid < TY + 1) {
        antenna_current<2>(r, t_ant, wrap_once(c + tid, ny), 0, jant);
        sAnt[1 + tid] = R(jant);
      }
    }
  }
  // every load of the workgroup is issued before the first is used: the tile's own E, B
  // and J, the halo rings from the snapshot, and the J of the column and row past the tile
  R e[PER][3], b[PER][3], jv[PER][3], er[NER][3], br[NBR][3], je[NJR][3];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int q = tid + p * 256;
    if (NC % 256 == 0 || q < NC) {
      const int64_t g = (int64_t)(c + (q >> LX)) * nx + a + (q & (TX - 1));
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        e[p][k] = f[F_EX + k][g];
        b[p][k] = f[F_BX + k][g];
        jv[p][k] = f[F_JX + k][g];
      }
    }
  }
#pragma unroll
  for (int p = 0; p < NER; ++p) {
    const int h = tid + p * 256;
    if (h < ER) {
      int u, v;
      ring_cell<TX, TY, 2>(h, u, v);
      const int i = wrap_once(a - 1 + u, nx), j = wrap_once(c - 1 + v, ny);
#pragma unroll
      for (int k = 0; k < 3; ++k) er[p][k] = bin[band_at(Bd, ntx, tile0, i, j, k)];
    }
  }
#pragma unroll
  for (int p = 0; p < NBR; ++p) {
    const int h = tid + p * 256;
    if (h < BR) {
      int u, v;
      ring_cell<TX, TY, 1>(h, u, v);
      const int i = wrap_once(a - 1 + u, nx), j = wrap_once(c - 1 + v, ny);
#pragma unroll
      for (int k = 0; k < 3; ++k) br[p][k] = bin[band_at(Bd, ntx, tile0, i, j, 3 + k)];
    }
  }
#pragma unroll
  for (int p = 0; p < NJR; ++p) {
    const int h = tid + p * 256;
    if (h < JR) {   // column u = TX + 1 (v = 1 .. TY + 1), then row v = TY + 1 (u = 1 .. TX)
      const int u = h <= TY ? TX + 1 : h - TY, v = h <= TY ? 1 + h : TY + 1;
      const int64_t g = (int64_t)wrap_once(c - 1 + v, ny) * nx + wrap_once(a - 1 + u, nx);
#pragma unroll
      for (int k = 0; k < 3; ++k) je[p][k] = f[F_JX + k][g];
    }
  }
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int q = tid + p * 256;
    if (NC % 256 == 0 || q < NC) {
      const int v = (q >> LX) + 1, u = (q & (TX - 1)) + 1;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sE[k][v * EW + u] = e[p][k];
        sB[k][v * BW + u] = b[p][k];
      }
    }
  }
#pragma unroll
  for (int p = 0; p < NER; ++p) {
    const int h = tid + p * 256;
    if (h < ER) {
      int u, v;
      ring_cell<TX, TY, 2>(h, u, v);
#pragma unroll
      for (int k = 0; k < 3; ++k) sE[k][v * EW + u] = er[p][k];
    }
  }
#pragma unroll
  for (int p = 0; p < NBR; ++p) {
    const int h = tid + p * 256;
    if (h < BR) {
      int u, v;
      ring_cell<TX, TY, 1>(h, u, v);
#pragma unroll
      for (int k = 0; k < 3; ++k) sB[k][v * BW + u] = br[p][k];
    }
  }
  __syncthreads();
  const double h1 = 0.5 * r.dt, h2 = r.dt;
  const R hx1 = R(h1 / r.dx), hy1 = R(h1 / r.dy);
  const R hx2 = R(h2 / r.dx), hy2 = R(h2 / r.dy), hh2 = R(h2);
  const bool mur = r.open_x != 0 && r.pml_cells == 0;
  // PML layers (lpic_set_pml) in reach of this tile: psi is read from the current half
  // and, for the tile's own cells, written to the other half (the neighbours recompute
  // this tile's edge values from the current half during this launch)
  const int PL = r.pml_cells;
  const bool pml_tile = PML && PL > 0 && (a - 1 < PL || a + TX + 1 > nx - PL);
  const int hcur = pml_tile ? pml_half(r) : 0;
  R* psi = (R*)r.psi;
  // 1. B half update on the whole B region (reads E only): the tile's cells (their psi
  // parked in the other half, where the same thread picks it up for the second B half),
  // then the ring around it
  auto b_first = [&](int u, int v, bool own) {
    const int ie = v * EW + u, q = v * BW + u, gu = a - 1 + u;
    const R ex = sE[0][ie], ey = sE[1][ie], ez = sE[2][ie];
    const R dbx = -hy1 * (sE[2][ie + EW] - ez);
    R dby = hx1 * (sE[2][ie + 1] - ez);
    R dbz = -hx1 * (sE[1][ie + 1] - ey) + hy1 * (sE[0][ie + EW] - ex);
    if (pml_tile) {
      const int sl = pml_slot(r, wrap_once(gu, nx));
      if (sl >= 0) {
        const int64_t row = wrap_once(c - 1 + v, ny);
        R pb, pc, ik;
        pml_coef<R>(r, true, sl, pb, pc, ik);
        const R Dz = sE[2][ie + 1] - ez, Dy = sE[1][ie + 1] - ey;
        const R p2 = pb * psi[pml_index(r, hcur, 2, row, sl)] + pc * Dz;
        const R p3 = pb * psi[pml_index(r, hcur, 3, row, sl)] + pc * Dy;
        dby = hx1 * (Dz * ik + p2);
        dbz = -hx1 * (Dy * ik + p3) + hy1 * (sE[0][ie + EW] - ex);
        if (own) {
          psi[pml_index(r, hcur ^ 1, 2, row, sl)] = p2;
          psi[pml_index(r, hcur ^ 1, 3, row, sl)] = p3;
        }
      }
    }
    sB[0][q] += dbx;
    if (mur && gu == nx - 2 && u + 1 < BW) {   // Mur for column nx-1
      sB[1][q + 1] = mur_edge<R>(sB[1][q + 1], sB[1][q], dby, h1, r.dx, 1);
      sB[2][q + 1] = mur_edge<R>(sB[2][q + 1], sB[2][q], dbz, h1, r.dx, 1);
    }
    if (!(mur && gu == nx - 1 && u >= 1)) {
      sB[1][q] += dby;
      sB[2][q] += dbz;
    }
  };
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int q = tid + p * 256;
    if (NC % 256 == 0 || q < NC) b_first((q & (TX - 1)) + 1, (q >> LX) + 1, true);
  }
#pragma unroll
  for (int p = 0; p < NBR; ++p) {
    const int h = tid + p * 256;
    if (h < BR) {
      int u, v;
      ring_cell<TX, TY, 1>(h, u, v);
      b_first(u, v, false);
    }
  }
  __syncthreads();
  // 2. E full update on [a, a+TX+1) x [c, c+TY+1) (reads B): the tile's cells with the J
  // held by their threads, then the column and row past the tile
  auto e_update = [&](int u, int v, R jx, R jy, R jz, bool own) {
    const int ib = v * BW + u, ie = v * EW + u, gu = a - 1 + u;
    if (u == u_ant) {
      if (r.laser.pol == 1) jy += sAnt[v];
      else jz += sAnt[v];
    }
    const R bx = sB[0][ib], by = sB[1][ib], bz = sB[2][ib];
    const R dex = hy2 * (bz - sB[2][ib - BW]) - hh2 * jx;
    R dey = -hx2 * (bz - sB[2][ib - 1]) - hh2 * jy;
    R dez = hx2 * (by - sB[1][ib - 1]) - hy2 * (bx - sB[0][ib - BW]) - hh2 * jz;
    if (pml_tile) {   // two merged halves of dt/2: the recursion runs twice
      const int sl = pml_slot(r, wrap_once(gu, nx));
      if (sl >= 0) {
        const int64_t row = wrap_once(c - 1 + v, ny);
        R pb, pc, ik;
        pml_coef<R>(r, false, sl, pb, pc, ik);
        const R Dz = bz - sB[2][ib - 1], Dy = by - sB[1][ib - 1];
        const R q0 = pb * psi[pml_index(r, hcur, 0, row, sl)] + pc * Dz, q0b = pb * q0 + pc * Dz;
        const R q1 = pb * psi[pml_index(r, hcur, 1, row, sl)] + pc * Dy, q1b = pb * q1 + pc * Dy;
        dey = -hx2 * (Dz * ik + R(0.5) * (q0 + q0b)) - hh2 * jy;
        dez = hx2 * (Dy * ik + R(0.5) * (q1 + q1b)) - hy2 * (bx - sB[0][ib - BW]) - hh2 * jz;
        if (own) {
          psi[pml_index(r, hcur ^ 1, 0, row, sl)] = q0b;
          psi[pml_index(r, hcur ^ 1, 1, row, sl)] = q1b;
        }
      }
    }
    sE[0][ie] += dex;
    if (mur && gu == 1 && u >= 2) {   // Mur for column 0
      sE[1][ie - 1] = mur_edge<R>(sE[1][ie - 1], sE[1][ie], dey, h2, r.dx, 2);
      sE[2][ie - 1] = mur_edge<R>(sE[2][ie - 1], sE[2][ie], dez, h2, r.dx, 2);
    }
    if (!(mur && gu == 0)) {
      sE[1][ie] += dey;
      sE[2][ie] += dez;
    }
  };
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int q = tid + p * 256;
    if (NC % 256 == 0 || q < NC)
      e_update((q & (TX - 1)) + 1, (q >> LX) + 1, jv[p][0], jv[p][1], jv[p][2], true);
  }
#pragma unroll
  for (int p = 0; p < NJR; ++p) {
    const int h = tid + p * 256;
    if (h < JR)
      e_update(h <= TY ? TX + 1 : h - TY, h <= TY ? 1 + h : TY + 1, je[p][0], je[p][1],
               je[p][2], false);
  }
  __syncthreads();
  // 3. B half update on the output tile (reads E only)
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int q = tid + p * 256;
    if (NC % 256 == 0 || q < NC) {
      const int v = (q >> LX) + 1, u = (q & (TX - 1)) + 1;
      const int ie = v * EW + u, ib = v * BW + u, gu = a - 1 + u;
      const R ex = sE[0][ie], ey = sE[1][ie], ez = sE[2][ie];
      const R dbx = -hy1 * (sE[2][ie + EW] - ez);
      R dby = hx1 * (sE[2][ie + 1] - ez);
      R dbz = -hx1 * (sE[1][ie + 1] - ey) + hy1 * (sE[0][ie + EW] - ex);
      if (pml_tile) {
        const int sl = pml_slot(r, wrap_once(gu, nx));
        if (sl >= 0) {
          const int64_t row = c - 1 + v;
          R pb, pc, ik;
          pml_coef<R>(r, true, sl, pb, pc, ik);
          const R Dz = sE[2][ie + 1] - ez, Dy = sE[1][ie + 1] - ey;
          R* q2 = psi + pml_index(r, hcur ^ 1, 2, row, sl);
          R* q3 = psi + pml_index(r, hcur ^ 1, 3, row, sl);
          const R p2 = pb * *q2 + pc * Dz, p3 = pb * *q3 + pc * Dy;
          dby = hx1 * (Dz * ik + p2);
          dbz = -hx1 * (Dy * ik + p3) + hy1 * (sE[0][ie + EW] - ex);
          *q2 = p2;
          *q3 = p3;
        }
      }
      sB[0][ib] += dbx;
      if (mur && gu == nx - 2 && u + 1 <= TX) {   // Mur for column nx-1
        sB[1][ib + 1] = mur_edge<R>(sB[1][ib + 1], sB[1][ib], dby, h1, r.dx, 1);
        sB[2][ib + 1] = mur_edge<R>(sB[2][ib + 1], sB[2][ib], dbz, h1, r.dx, 1);
      }
      if (!(mur && gu == nx - 1 && u >= 2)) {
        sB[1][ib] += dby;
        sB[2][ib] += dbz;
      }
    }
  }
  __syncthreads();
  // 4. the tile's E and B to the arrays, its edges to the other snapshot
  const int64_t bbase = (tile0 + tile) * 6 * (3 * (TX + TY));
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int q = tid + p * 256;
    if (NC % 256 == 0 || q < NC) {
      const int lj = q >> LX, li = q & (TX - 1);
      const int ie = (lj + 1) * EW + li + 1, ib = (lj + 1) * BW + li + 1;
      const int64_t g = (int64_t)(c + lj) * nx + a + li;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        f[F_EX + k][g] = sE[k][ie];
        f[F_BX + k][g] = sB[k][ib];
      }
      if (band_col(li, TX) >= 0 || band_col(lj, TY) >= 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          band_put(bout, Bd, bbase, li, lj, k, sE[k][ie]);
          band_put(bout, Bd, bbase, li, lj, 3 + k, sB[k][ib]);
        }
      }
    }
  }
}

// J := 0 (and the charge arrays when asked and present), four cells per thread, 256 cells
// per wave, four waves per workgroup.  flip != NULL: the launch follows a fused field update; its first
// thread makes the snapshot that update wrote the present one and, with clock != NULL,
// advances the antenna clock as the antenna kernel would have.
template <typename R>
__device__ __forceinline__ void zero4(R* p, int64_t c, int64_t n) {
  if (c + 3 < n && ((uintptr_t)p & 15) == 0) {
    if constexpr (sizeof(R) == 4) {
      *(float4*)(p + c) = make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
      *(double2*)(p + c) = make_double2(0.0, 0.0);
      *(double2*)(p + c + 2) = make_double2(0.0, 0.0);
    }
  } else {
    for (int64_t i = c; i < n && i < c + 4; ++i) p[i] = R(0);
  }
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_clear_sources(Tables T, int nblk, int with_rho,
                                                       int32_t* flip, int64_t* clock) {
  if (flip && blockIdx.x == 0 && threadIdx.x == 0) {
    *flip ^= 1;
    if (clock) *clock += 1;
  }
  // each wave clears one 256-cell block of the cell-block prefix (four per workgroup)
  const int vb = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (vb >= nblk) return;
  int blk = vb, ri = 0;
  if (T.runs) {
    ri = uniform(find_owner(T.run_blk, T.nruns, vb));
    blk = uniform(vb - T.run_blk[ri]);
  }
  const RunDesc& r = run_of(T, ri);
  const int64_t n = (int64_t)r.nx * r.ny * (DIM == 3 ? r.nz : 1);
  const int64_t c = (int64_t)blk * 256 + 4 * (threadIdx.x & 63);
  if (c >= n) return;
  zero4((R*)r.f[F_JX], c, n);
  zero4((R*)r.f[F_JY], c, n);
  zero4((R*)r.f[F_JZ], c, n);
  // with_rho: 1 both charge arrays, 3 rho0 only, 4 rho1 only (as k_yee_e's zero_j)
  if ((with_rho == 1 || with_rho == 3) && r.f[F_R0]) zero4((R*)r.f[F_R0], c, n);
  if ((with_rho == 1 || with_rho == 4) && r.f[F_R1]) zero4((R*)r.f[F_R1], c, n);
}

// ---------------------------------------------------------------------------------------
// Laser antenna: J_pol += -2 E_inc(t) / dx on node column ia (see lpic_laser).  With a
// device step counter, t = (step + 1) dt and the last workgroup advances the counter (one
// launch per step); otherwise t is the argument.
// ---------------------------------------------------------------------------------------
template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_laser(Tables T, int nruns, int bpr, double t_arg,
                                               int64_t* step, unsigned int* done) {
  const int ri = blockIdx.x / bpr;
  if (ri < nruns) {
    const RunDesc& r = run_of(T, ri);
    const int64_t m = (int64_t)r.ny * (DIM == 3 ? r.nz : 1);
    const int64_t tcell = (int64_t)(blockIdx.x % bpr) * 256 + threadIdx.x;
    if (r.has_laser && tcell < m) {
      const int j = (int)(tcell % r.ny), k = (int)(tcell / r.ny);
      double jant;
      if (antenna_current<DIM>(r, step ? (double)(*step + 1) * r.dt : t_arg, j, k, jant)) {
        const int64_t c = ((int64_t)k * r.ny + j) * r.nx + array_x(r, r.laser.ia);
        gptr<R> J = gp((R*)r.f[r.laser.pol == 1 ? F_JY : F_JZ]);
        J[c] += R(jant);
      }
    }
  }
  if (step) {   // the last workgroup advances the clock (all have read it by then)
    __syncthreads();
    if (threadIdx.x == 0) {
      if (atomicAdd(done, 1u) == gridDim.x - 1) {
        *step += 1;
        *done = 0u;
      }
    }
  }
}

// =======================================================================================
// Split particle path: gather + push, then deposit (used when a hook sits between them).
// The old state (OldState) holds the start of each particle's deposit path, x^{n+1/2}.
// =======================================================================================
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
  deposit<DIM, ORDER>(A, c0, o0, pe, now.w, now.u[2] * ig1, k, with_rho ? 1 : 0);
  if (leaves_box(r, now.c[0])) {   // its new position is in an open end's margin
    now.alive = false;
    store_particle<R, DIM>(s, r, (int32_t)p, now);
  }
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

// Groups the lanes of a wave by key: the mask of the lanes holding this lane's key (0 for an
// invalid lane).  One pass per distinct key in the wave, so a wave whose particles sit in a
// few tiles, in any lane order, costs a few passes.
__device__ __forceinline__ uint64_t wave_match(int key, bool valid) {
  uint64_t todo = __ballot(valid);
  uint64_t mine = 0;
  while (todo) {
    const int k = __shfl(key, __ffsll((unsigned long long)todo) - 1, 64);
    const uint64_t m = __ballot(valid && key == k);
    if (valid && key == k) mine = m;
    todo &= ~m;
  }
  return mine;
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

// Per-workgroup key cache in LDS: the 2048 particles of a workgroup come from a handful of
// tiles (their home tile and its neighbours), so the counts of a workgroup are summed in LDS
// and reach the global bins with one atomic per distinct key.  A key whose cache slot is
// taken by another key falls back to global atomics.
constexpr int SORT_SLOTS = 256;

struct SortCache {
  int32_t tag[SORT_SLOTS];
  int32_t cnt[SORT_SLOTS];
  int32_t base[SORT_SLOTS];
};

__device__ __forceinline__ void sort_cache_clear(SortCache& C) {
  for (int i = threadIdx.x; i < SORT_SLOTS; i += blockDim.x) {
    C.tag[i] = -1;
    C.cnt[i] = 0;
  }
}

// Claims the cache slot of `key`; true if the slot holds this key.
__device__ __forceinline__ bool sort_cache_claim(SortCache& C, int key) {
  const int slot = key & (SORT_SLOTS - 1);
  int t = C.tag[slot];
  if (t == -1) {
    t = atomicCAS(&C.tag[slot], -1, key);
    if (t == -1) t = key;
  }
  return t == key;
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_sort_count(Tables T, int32_t* counts) {
  __shared__ SortCache C;
  int blk;
  const SegDesc s = seg_of(T, part_block(T, blk));
  const RunDesc r = run_of(T, s.run);
  sort_cache_clear(C);
  int key[SORT_ITEMS];
  int64_t p[SORT_ITEMS];
  block_keys<R, DIM>(s, r, blk, key, p);
  __syncthreads();
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    const uint64_t m = wave_match(key[it], key[it] >= 0);
    if (m && __lane_id() == __ffsll((unsigned long long)m) - 1) {   // first lane of its key
      const int len = __popcll(m);
      if (sort_cache_claim(C, key[it])) atomicAdd(&C.cnt[key[it] & (SORT_SLOTS - 1)], len);
      else atomicAdd(&counts[key[it]], len);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < SORT_SLOTS; i += blockDim.x)
    if (C.tag[i] >= 0 && C.cnt[i] > 0) atomicAdd(&counts[C.tag[i]], C.cnt[i]);
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

// Exclusive scan over the 1024 threads of a workgroup (wsum: 17 shared words); *total gets
// the sum.  Contains barriers: every thread must call it.
__device__ __forceinline__ int32_t block_exscan1024(int32_t local, int32_t* wsum,
                                                    int32_t* total) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  int32_t incl = local;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  __syncthreads();   // wsum may still be read from a previous call
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  if (tid < 64) {
    const int32_t v = tid < 16 ? wsum[tid] : 0;
    int32_t vi = v;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      const int32_t o = __shfl_up(vi, off, 64);
      if (lane >= off) vi += o;
    }
    if (tid < 16) wsum[tid] = vi - v;
    if (tid == 15) wsum[16] = vi;
  }
  __syncthreads();
  *total = wsum[16];
  return wsum[wid] + incl - local;
}

// Bins per thread and pass of the one-workgroup kernels over all bins: a thread loads its
// run of bins at once (one memory latency per pass rather than one per bin).
constexpr int SCAN_PER = 16;

// Exclusive scan of the bin counts by one workgroup; clears the counts for the next sort
// and records each bin's placement multiplier.
// gate != NULL: only when *gate >= threshold (the re-binned escape path); mult may be NULL.
__global__ __launch_bounds__(1024) void k_scan_bins(int32_t* counts, int32_t* offsets,
                                                    int32_t* cursor, int32_t* mult, int nbins,
                                                    int spread, const unsigned int* gate,
                                                    int threshold) {
  if (gate && (int)min(gate[0], 0x7fffffffu) < threshold) return;
  __shared__ int32_t wsum[17];
  int32_t base = 0;
  for (int pass = 0; pass < nbins; pass += 1024 * SCAN_PER) {
    const int b0 = pass + threadIdx.x * SCAN_PER;
    int32_t v[SCAN_PER];
    int32_t local = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER; ++k) {
      v[k] = b0 + k < nbins ? counts[b0 + k] : 0;
      local += v[k];
    }
    int32_t total;
    int32_t run = base + block_exscan1024(local, wsum, &total);
#pragma unroll
    for (int k = 0; k < SCAN_PER; ++k) {
      const int b = b0 + k;
      if (b < nbins) {
        offsets[b] = run;
        cursor[b] = run;
        if (mult) mult[b] = spread ? spread_multiplier(v[k]) : 1;
        counts[b] = 0;
      }
      run += v[k];
    }
    base += total;
  }
  if (threadIdx.x == 0) offsets[nbins] = base;
}

// The same scan over many workgroups (a sum per workgroup of SCAN_TILE bins, a scan of those
// sums, then each workgroup's bins from its base): one memory latency per phase instead of
// one per SCAN_TILE bins, for the many-bin scans of every step (3D re-binned escapes).
constexpr int SCAN_TILE = 1024 * SCAN_PER;

__device__ __forceinline__ bool gate_closed(const unsigned int* gate, int threshold) {
  return gate && (int)min(gate[0], 0x7fffffffu) < threshold;
}

__global__ __launch_bounds__(1024) void k_scan_sums(const int32_t* counts, int nbins,
                                                    int32_t* part, const unsigned int* gate,
                                                    int threshold) {
  if (gate_closed(gate, threshold)) return;
  __shared__ int32_t wsum[17];
  const int b0 = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER;
  int32_t local = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) local += b0 + k < nbins ? counts[b0 + k] : 0;
  int32_t total;
  (void)block_exscan1024(local, wsum, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Exclusive scan of the nparts workgroup sums in place (one workgroup); the grand total to
// *total_out.
__global__ __launch_bounds__(1024) void k_scan_parts(int32_t* part, int nparts,
                                                     int32_t* total_out,
                                                     const unsigned int* gate, int threshold,
                                                     int zero_if_closed) {
  if (gate_closed(gate, threshold)) {
    if (zero_if_closed && threadIdx.x == 0) *total_out = 0;
    return;
  }
  __shared__ int32_t wsum[17];
  int32_t base = 0;
  for (int pass = 0; pass < nparts; pass += 1024) {
    const int i = pass + threadIdx.x;
    const int32_t v = i < nparts ? part[i] : 0;
    int32_t total;
    const int32_t ex = block_exscan1024(v, wsum, &total);
    if (i < nparts) part[i] = base + ex;
    base += total;
  }
  if (threadIdx.x == 0) *total_out = base;
}

__global__ __launch_bounds__(1024) void k_scan_apply(int32_t* counts, int32_t* offsets,
                                                     int32_t* cursor, int32_t* mult, int nbins,
                                                     int spread, const int32_t* part,
                                                     const unsigned int* gate, int threshold) {
  if (gate_closed(gate, threshold)) return;
  __shared__ int32_t wsum[17];
  const int b0 = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER;
  int32_t v[SCAN_PER];
  int32_t local = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    v[k] = b0 + k < nbins ? counts[b0 + k] : 0;
    local += v[k];
  }
  int32_t total;
  int32_t run = part[blockIdx.x] + block_exscan1024(local, wsum, &total);
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    const int b = b0 + k;
    if (b < nbins) {
      offsets[b] = run;
      cursor[b] = run;
      if (mult) mult[b] = spread ? spread_multiplier(v[k]) : 1;
      counts[b] = 0;
    }
    run += v[k];
  }
}

int part_words(int n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

void launch_scan(int32_t* counts, int32_t* offsets, int32_t* cursor, int32_t* mult, int nbins,
                 int spread, const unsigned int* gate, int threshold, int32_t* part,
                 hipStream_t st) {
  const int nparts = (nbins + SCAN_TILE - 1) / SCAN_TILE;
  if (!part || nparts <= 1) {
    k_scan_bins<<<1, 1024, 0, st>>>(counts, offsets, cursor, mult, nbins, spread, gate,
                                    threshold);
    return;
  }
  k_scan_sums<<<nparts, 1024, 0, st>>>(counts, nbins, part, gate, threshold);
  k_scan_parts<<<1, 1024, 0, st>>>(part, nparts, offsets + nbins, gate, threshold, 0);
  k_scan_apply<<<nparts, 1024, 0, st>>>(counts, offsets, cursor, mult, nbins, spread, part,
                                        gate, threshold);
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_sort_scatter(Tables T, int32_t* cursor,
                                                      const int32_t* offsets,
                                                      const int32_t* mult, int spread) {
  __shared__ SortCache C;
  int blk;
  const SegDesc s = seg_of(T, part_block(T, blk));
  const RunDesc r = run_of(T, s.run);
  sort_cache_clear(C);
  int key[SORT_ITEMS];
  int64_t p[SORT_ITEMS];
  block_keys<R, DIM>(s, r, blk, key, p);
  __syncthreads();
  // ranks: inside the workgroup for cached keys, straight from the bin cursor otherwise
  int32_t rank[SORT_ITEMS];
  bool cached[SORT_ITEMS];
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    // lanes of one key take consecutive ranks in lane order after the first lane's reservation
    const uint64_t m = wave_match(key[it], key[it] >= 0);
    const int lane = __lane_id();
    const int head = m ? __ffsll((unsigned long long)m) - 1 : lane;
    int base = 0, hit = 0;
    if (m && lane == head) {
      const int len = __popcll(m);
      hit = sort_cache_claim(C, key[it]);
      base = hit ? atomicAdd(&C.cnt[key[it] & (SORT_SLOTS - 1)], len)
                 : atomicAdd(&cursor[key[it]], len);
    }
    base = __shfl(base, head, 64);
    hit = __shfl(hit, head, 64);
    rank[it] = base + __popcll(m & ((1ull << lane) - 1ull));
    cached[it] = hit != 0;
  }
  __syncthreads();
  // one cursor reservation per cached key
  for (int i = threadIdx.x; i < SORT_SLOTS; i += blockDim.x)
    if (C.tag[i] >= 0 && C.cnt[i] > 0) C.base[i] = atomicAdd(&cursor[C.tag[i]], C.cnt[i]);
  __syncthreads();
  int64_t dst[SORT_ITEMS];
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    dst[it] = -1;
    if (key[it] < 0) continue;
    const int64_t slot = (cached[it] ? (int64_t)C.base[key[it] & (SORT_SLOTS - 1)] : 0) + rank[it];
    if (spread) {
      const int32_t b0 = offsets[key[it]], nb = offsets[key[it] + 1] - b0;
      dst[it] = b0 + ((slot - b0) * mult[key[it]]) % nb - s.pbase;
    } else {
      dst[it] = slot - s.pbase;
    }
  }
  // move the particle arrays: every item's words of every array are loaded before the first
  // store, so the workgroup waits for memory once rather than once per array
  constexpr int NA = (sizeof(R) == 4 ? 1 + DIM : DIM) + 4;   // arrays per particle
  constexpr int WPA = sizeof(R) / 4;                          // 32-bit words per entry
  int map[NA];
  {
    int k = 0;
    if constexpr (sizeof(R) == 4) {
      map[k++] = P_CELL;
      for (int d = 0; d < DIM; ++d) map[k++] = P_OX + d;
    } else {
      for (int d = 0; d < DIM; ++d) map[k++] = P_X + d;
    }
    for (int q = P_UX; q <= P_W; ++q) map[k++] = q;
  }
  uint32_t v[NA][SORT_ITEMS][WPA];
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    const uint32_t* from = (const uint32_t*)s.p[map[a]];
#pragma unroll
    for (int it = 0; it < SORT_ITEMS; ++it)
      if (dst[it] >= 0)
#pragma unroll
        for (int w = 0; w < WPA; ++w) v[a][it][w] = gp(from)[p[it] * WPA + w];
  }
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    uint32_t* to = (uint32_t*)s.alt[map[a]];
#pragma unroll
    for (int it = 0; it < SORT_ITEMS; ++it)
      if (dst[it] >= 0)
#pragma unroll
        for (int w = 0; w < WPA; ++w) gp(to)[dst[it] * WPA + w] = v[a][it][w];
  }
}

// =======================================================================================
// Fixed-point scale of the FP32 current accumulators.  A deposit contribution is bounded
// by |q w| max(1, h/dt) (the Esirkepov running sums and shape products are at most 1 and
// |v| < c), so with cmax = 2 max|q w| max(1, h/dt) and n particles in a run:
//   |v| 2^S < 2^29 for every contribution (it rounds to a 32-bit integer, sign-extended
//   into the 64-bit accumulator), and
//   |any accumulated sum| <= n cmax 2^S < 2^61 (no 64-bit overflow, whatever the order).
// S stays within [-120, 120] so that 2^S is a normal FP32 number.
// =======================================================================================
constexpr int WMAX_SPAN = 4;    // sort-sized particle blocks per workgroup
// Each segment's maximum is spread over WMAX_SLOTS words (workgroup b uses slot b mod
// WMAX_SLOTS) so that the workgroups' atomics do not all queue on one address.
constexpr int WMAX_SLOTS = 64;

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_wmax(Tables T, int nvblk, unsigned long long* wmax) {
  __shared__ double red[4];
  double m = 0.0;
  int cur = -1;
  for (int k = 0; k < WMAX_SPAN; ++k) {
    const int vb = blockIdx.x * WMAX_SPAN + k;
    if (vb >= nvblk) break;
    int blk = vb, si = 0;
    if (T.segs) {
      si = uniform(find_owner(T.seg_blk, T.nsegs, vb));
      blk = uniform(vb - T.seg_blk[si]);
    }
    if (si != cur) {
      if (cur >= 0) {
        m = wave_max(m);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0)
          atomicMax(&wmax[cur * WMAX_SLOTS + (blockIdx.x & (WMAX_SLOTS - 1))],
                    (unsigned long long)__double_as_longlong(
                        fmax(fmax(red[0], red[1]), fmax(red[2], red[3]))));
      }
      m = 0.0;
      cur = si;
    }
    const SegDesc& s = seg_of(T, si);
    const gptr<const R> w = gp((const R*)s.p[P_W]);
    const int64_t beg = (int64_t)blk * 256 * SORT_ITEMS;
#pragma unroll
    for (int it = 0; it < SORT_ITEMS; ++it) {
      const int64_t p = beg + it * 256 + threadIdx.x;
      if (p < s.n) m = fmax(m, fabs((double)w[p]));
    }
  }
  if (cur >= 0) {
    m = wave_max(m);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
      atomicMax(&wmax[cur * WMAX_SLOTS + (blockIdx.x & (WMAX_SLOTS - 1))],
                (unsigned long long)__double_as_longlong(
                    fmax(fmax(red[0], red[1]), fmax(red[2], red[3]))));   // >= 0
  }
}

__global__ void k_fixed_shift(Tables T, int nruns, int nsegs, const unsigned long long* wmax,
                              int32_t* jshift) {
  const int ri = blockIdx.x * blockDim.x + threadIdx.x;
  if (ri >= nruns) return;
  const RunDesc r = run_of(T, ri);
  double h = fmax(1.0, fmax(r.dx, r.dy) / r.dt);
  if (r.ndim == 3) h = fmax(h, r.dz / r.dt);
  double cmax = 0.0, n = 0.0;
  for (int i = 0; i < nsegs; ++i) {
    const SegDesc& s = seg_of(T, i);
    if (s.run != ri) continue;
    double wm = 0.0;
    for (int k = 0; k < WMAX_SLOTS; ++k)
      wm = fmax(wm, __longlong_as_double((long long)wmax[i * WMAX_SLOTS + k]));
    cmax = fmax(cmax, fabs(s.q) * wm);
    n += (double)s.n;
  }
  cmax *= 2.0 * h;
  int sh = 32;
  if (cmax > 0.0 && n > 0.0) {
    int e1, e2;
    frexp(cmax, &e1);       // cmax < 2^e1
    frexp(n * cmax, &e2);   // n cmax < 2^e2
    sh = min(30 - e1, 61 - e2);
    sh = max(-120, min(120, sh));
  }
  jshift[ri] = sh;
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

// Slot v of the chunk order (run by run, tile by tile, species by species): its segment,
// tile and bin.
struct VSlot {
  int run, vbase, vend, nseg, seg_first;
};
__device__ __forceinline__ VSlot vslot_run(const Tables& T, int v) {
  int lo = 0, hi = T.runs ? T.nruns - 1 : 0;   // last run with vbase <= v
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (T.runs[mid].vbase <= v) lo = mid; else hi = mid - 1;
  }
  const RunDesc& r = run_of(T, lo);
  VSlot q;
  q.run = lo;
  q.vbase = r.vbase;
  q.nseg = r.nseg;
  q.seg_first = r.seg_first;
  q.vend = r.vbase + r.ntiles * r.nseg;
  return q;
}

// absolute: chunk ranges are positions in the list the offsets describe (the re-binned
// escape list) instead of slots relative to the segment.  gate != NULL: only when
// *gate >= threshold; otherwise the chunk count is set to zero.
// The particle ranges of SCAN_PER consecutive slots from v0: segment (-1: none), tile and
// range (relative to the segment, or absolute).
__device__ __forceinline__ void slot_ranges(const Tables& T, const int32_t* offsets, int nvirt,
                                            int v0, int absolute, int sg[SCAN_PER],
                                            int tl[SCAN_PER], int32_t o0[SCAN_PER],
                                            int32_t o1[SCAN_PER]) {
  VSlot q = vslot_run(T, min(v0, nvirt - 1));
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    const int v = v0 + k;
    sg[k] = -1;
    tl[k] = 0;
    o0[k] = o1[k] = 0;
    if (v < nvirt) {
      while (v >= q.vend) q = vslot_run(T, v);   // runs without species span no slots
      const int w = v - q.vbase;
      tl[k] = w / q.nseg;
      sg[k] = q.seg_first + (w - tl[k] * q.nseg);
      const SegDesc& s = seg_of(T, sg[k]);
      const int b = s.bin_base + tl[k];
      const int32_t rel = absolute ? 0 : (int32_t)s.pbase;
      o0[k] = offsets[b] - rel;
      o1[k] = offsets[b + 1] - rel;
    }
  }
}

__device__ __forceinline__ void write_chunks(Chunk* out, int32_t pos, int chunk,
                                             const int sg[SCAN_PER], const int tl[SCAN_PER],
                                             const int32_t o0[SCAN_PER],
                                             const int32_t o1[SCAN_PER]) {
  for (int k = 0; k < SCAN_PER; ++k) {
    if (sg[k] < 0) continue;
    for (int32_t a = o0[k]; a < o1[k]; a += chunk) {
      Chunk c;
      c.seg = sg[k];
      c.tile = tl[k];
      c.beg = a;
      c.end = min(o1[k], a + chunk);
      out[pos++] = c;
    }
  }
}

__device__ __forceinline__ int32_t chunk_count(int chunk, const int sg[SCAN_PER],
                                               const int32_t o0[SCAN_PER],
                                               const int32_t o1[SCAN_PER]) {
  int32_t n = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k)
    if (sg[k] >= 0) n += (o1[k] - o0[k] + chunk - 1) / chunk;
  return n;
}

__global__ __launch_bounds__(1024) void k_build_chunks(Tables T, const int32_t* offsets,
                                                       int nvirt, int chunk, Chunk* out,
                                                       int32_t* nchunks, int absolute,
                                                       const unsigned int* gate,
                                                       int threshold) {
  if (gate_closed(gate, threshold)) {
    if (threadIdx.x == 0) *nchunks = 0;
    return;
  }
  __shared__ int32_t wsum[17];
  int32_t cbase = 0;
  for (int pass = 0; pass < nvirt; pass += 1024 * SCAN_PER) {
    int sg[SCAN_PER], tl[SCAN_PER];
    int32_t o0[SCAN_PER], o1[SCAN_PER];
    slot_ranges(T, offsets, nvirt, pass + threadIdx.x * SCAN_PER, absolute, sg, tl, o0, o1);
    int32_t total;
    const int32_t pos = cbase + block_exscan1024(chunk_count(chunk, sg, o0, o1), wsum, &total);
    write_chunks(out, pos, chunk, sg, tl, o0, o1);
    cbase += total;
  }
  if (threadIdx.x == 0) *nchunks = cbase;
}

// The chunk list over many workgroups (counts per workgroup of SCAN_TILE slots, their scan,
// then each workgroup's chunks from its base), as the bin scan above.
__global__ __launch_bounds__(1024) void k_chunk_sums(Tables T, const int32_t* offsets,
                                                     int nvirt, int chunk, int32_t* part,
                                                     int absolute, const unsigned int* gate,
                                                     int threshold) {
  if (gate_closed(gate, threshold)) return;
  __shared__ int32_t wsum[17];
  int sg[SCAN_PER], tl[SCAN_PER];
  int32_t o0[SCAN_PER], o1[SCAN_PER];
  slot_ranges(T, offsets, nvirt, blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER, absolute,
              sg, tl, o0, o1);
  int32_t total;
  (void)block_exscan1024(chunk_count(chunk, sg, o0, o1), wsum, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_chunk_apply(Tables T, const int32_t* offsets,
                                                      int nvirt, int chunk, Chunk* out,
                                                      const int32_t* part, int absolute,
                                                      const unsigned int* gate,
                                                      int threshold) {
  if (gate_closed(gate, threshold)) return;
  __shared__ int32_t wsum[17];
  int sg[SCAN_PER], tl[SCAN_PER];
  int32_t o0[SCAN_PER], o1[SCAN_PER];
  slot_ranges(T, offsets, nvirt, blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_PER, absolute,
              sg, tl, o0, o1);
  int32_t total;
  const int32_t pos = part[blockIdx.x] +
                      block_exscan1024(chunk_count(chunk, sg, o0, o1), wsum, &total);
  write_chunks(out, pos, chunk, sg, tl, o0, o1);
}

static void build_chunks(const Tables& T, const int32_t* offsets, int nvirt, int chunk,
                         Chunk* out, int32_t* nchunks, int absolute, const unsigned int* gate,
                         int threshold, int32_t* part, hipStream_t st) {
  const int nparts = (nvirt + SCAN_TILE - 1) / SCAN_TILE;
  if (!part || nparts <= 1) {
    k_build_chunks<<<1, 1024, 0, st>>>(T, offsets, nvirt, chunk, out, nchunks, absolute, gate,
                                       threshold);
    return;
  }
  k_chunk_sums<<<nparts, 1024, 0, st>>>(T, offsets, nvirt, chunk, part, absolute, gate,
                                        threshold);
  k_scan_parts<<<1, 1024, 0, st>>>(part, nparts, nchunks, gate, threshold, 1);
  k_chunk_apply<<<nparts, 1024, 0, st>>>(T, offsets, nvirt, chunk, out, part, absolute, gate,
                                         threshold);
}

// =======================================================================================
// Re-binned escapes.  Particles whose stencils have left the staged region of their home
// tile since the last sort (the fused kernel's escape list) are grouped by the tile they
// are in now:
// count per (segment, tile) bin, scan, scatter of the list entries, a chunk list over those
// bins; a second fused pass then pushes them against the staged regions of their present
// tiles, where they are always inside.  Every kernel of the path first reads the escape
// count and does nothing below `threshold` (the step then leaves the escapees to k_escape),
// so the path can sit in a captured graph.
// =======================================================================================
__device__ __forceinline__ bool rebin_on(const unsigned int* esc_count, int threshold) {
  return (int)min(esc_count[0], 0x7fffffffu) >= threshold;
}

// The bin of escape-list entry i: from its escape record when the list carries them (one
// contiguous read), else from the particle's slot.
template <typename R, int DIM>
__device__ __forceinline__ int escapee_bin(const Tables& T, const EscapeList& esc, int64_t i,
                                           unsigned long long item) {
  if (esc.keys) return esc.keys[i];   // written by the fused pass with the record
  const int seg = (int)(item >> 32);
  const int64_t p = (int64_t)(item & 0xffffffffull);
  const SegDesc& s = seg_of(T, seg);
  const RunDesc& r = run_of(T, s.run);
  if (!esc.rec) return particle_bin<R, DIM>(s, r, p);
  int c[3];
  if (!rec_cell<R, DIM>(part_ptrs<R>(s, r), esc.rec, i, c)) return s.bin_base + r.ntiles;
  return s.bin_base + (((c[2] >> s.lz) * r.nty) + (c[1] >> s.ly)) * r.ntx + (c[0] >> s.lx);
}

// ESC_ITEMS escape-list entries per thread: 2048 per workgroup of 256, as for the sort.
constexpr int ESC_ITEMS = SORT_ITEMS;

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_rebin_count(Tables T, EscapeList esc, int threshold,
                                                     int32_t* counts) {
  if (!rebin_on(esc.count, threshold)) return;
  const int64_t n = min((int64_t)esc.count[0], esc.capacity);
  __shared__ SortCache C;
  sort_cache_clear(C);
  __syncthreads();
  for (int64_t beg = (int64_t)blockIdx.x * 256 * ESC_ITEMS; beg < n;
       beg += (int64_t)gridDim.x * 256 * ESC_ITEMS) {
    int key[ESC_ITEMS];
#pragma unroll
    for (int it = 0; it < ESC_ITEMS; ++it) {
      const int64_t i = beg + it * 256 + threadIdx.x;
      key[it] = i < n ? escapee_bin<R, DIM>(T, esc, i, esc.keys ? 0ull : esc.items[i]) : -1;
    }
#pragma unroll
    for (int it = 0; it < ESC_ITEMS; ++it) {
      const uint64_t m = wave_match(key[it], key[it] >= 0);
      if (m && __lane_id() == __ffsll((unsigned long long)m) - 1) {
        const int len = __popcll(m);
        if (sort_cache_claim(C, key[it])) atomicAdd(&C.cnt[key[it] & (SORT_SLOTS - 1)], len);
        else atomicAdd(&counts[key[it]], len);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < SORT_SLOTS; i += blockDim.x)
    if (C.tag[i] >= 0 && C.cnt[i] > 0) atomicAdd(&counts[C.tag[i]], C.cnt[i]);
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_rebin_scatter(Tables T, EscapeList esc, int threshold,
                                                       int32_t* cursor,
                                                       unsigned long long* out, void* out_rec) {
  if (!rebin_on(esc.count, threshold)) return;
  const int64_t n = min((int64_t)esc.count[0], esc.capacity);
  __shared__ SortCache C;
  for (int64_t beg = (int64_t)blockIdx.x * 256 * ESC_ITEMS; beg < n;
       beg += (int64_t)gridDim.x * 256 * ESC_ITEMS) {
    sort_cache_clear(C);
    __syncthreads();
    int key[ESC_ITEMS];
    unsigned long long item[ESC_ITEMS];
    EscRec<R> rec[ESC_ITEMS];   // (loaded with the entries: one memory latency per batch)
#pragma unroll
    for (int it = 0; it < ESC_ITEMS; ++it) {
      const int64_t i = beg + it * 256 + threadIdx.x;
      item[it] = i < n ? esc.items[i] : 0ull;
      key[it] = i < n ? escapee_bin<R, DIM>(T, esc, i, item[it]) : -1;
      if (esc.rec && i < n) rec[it] = load_rec<R>(esc.rec, i);
    }
    // ranks inside the workgroup for cached keys, straight from the bin cursor otherwise
    int32_t rank[ESC_ITEMS];
    bool cached[ESC_ITEMS];
#pragma unroll
    for (int it = 0; it < ESC_ITEMS; ++it) {
      const uint64_t m = wave_match(key[it], key[it] >= 0);
      const int lane = __lane_id();
      const int head = m ? __ffsll((unsigned long long)m) - 1 : lane;
      int base = 0, hit = 0;
      if (m && lane == head) {
        const int len = __popcll(m);
        hit = sort_cache_claim(C, key[it]);
        base = hit ? atomicAdd(&C.cnt[key[it] & (SORT_SLOTS - 1)], len)
                   : atomicAdd(&cursor[key[it]], len);
      }
      base = __shfl(base, head, 64);
      hit = __shfl(hit, head, 64);
      rank[it] = base + __popcll(m & ((1ull << lane) - 1ull));
      cached[it] = hit != 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < SORT_SLOTS; i += blockDim.x)
      if (C.tag[i] >= 0 && C.cnt[i] > 0) C.base[i] = atomicAdd(&cursor[C.tag[i]], C.cnt[i]);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ESC_ITEMS; ++it) {
      if (key[it] < 0) continue;
      const int64_t slot =
          (cached[it] ? (int64_t)C.base[key[it] & (SORT_SLOTS - 1)] : 0) + rank[it];
      out[slot] = item[it];
      if (esc.rec)
        store_rec<R>(out_rec, slot, rec[it]);
    }
    __syncthreads();   // the cache is cleared for the next batch
  }
}

// =======================================================================================
// FP64 diagnostics: field energy, continuity and Gauss residuals (max over cells).
// =======================================================================================
__device__ __forceinline__ void atomic_max_nonneg(double* p, double v) {
  atomicMax((unsigned long long*)p, (unsigned long long)__double_as_longlong(v));
}

// Each workgroup walks REDUCE_SPAN consecutive 256-cell blocks of the cell-block space (all
// runs end to end) and flushes its partial sums once per run it touched: one set of global
// atomics per workgroup rather than per 256 cells.
constexpr int REDUCE_SPAN = 16;

template <int DIM>
__device__ __forceinline__ void reduce_flush(const RunDesc& r, double* out, int with_rho,
                                             double en, double res, double rm, double ga,
                                             double (*red)[4]) {
  en = wave_sum(en);
  res = wave_max(res);
  rm = wave_max(rm);
  ga = wave_max(ga);
  const int w = threadIdx.x >> 6;
  __syncthreads();   // red[] may still be read by the previous flush
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
    double* o = out ? out : r.diag;
    const double dV = r.dx * r.dy * (DIM == 3 ? r.dz : 1.0);
    atomic_add_global(o + (out ? 0 : DIAG_UFIELD), 0.5 * a * dV);
    if (with_rho) {
      atomic_max_nonneg(o + (out ? 1 : DIAG_RES), b);
      atomic_max_nonneg(o + (out ? 2 : DIAG_RHOMAX), c);
      atomic_max_nonneg(o + (out ? 3 : DIAG_GAUSS), d);
    }
  }
}

// One cell's terms: field energy density (sum of squares), and with the charge arrays the
// continuity residual, max |rho1| and the Gauss residual.
template <typename R, int DIM>
__device__ __forceinline__ void reduce_cell(const RunDesc& r, const CellIdx& x, int with_rho,
                                            double& en, double& res, double& rm, double& ga) {
  gptr<R> f[F_NUM];
#pragma unroll
  for (int c = 0; c < F_NUM; ++c) f[c] = gp((R*)r.f[c]);
#pragma unroll
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
    rm = fmax(rm, fabs(r1));
    // a laser antenna's current is prescribed, not carried by charges (its transverse
    // profile has a divergence): its node column is left out of both residuals
    if (!(r.has_laser && box_x(r, x.i) == r.laser.ia)) {
      res = fmax(res, fabs(r1 - r0 + r.dt * divj));
      ga = fmax(ga, fabs(dive - 0.5 * (r0 + r1) - r.rho_bg));
    }
  }
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_reduce_fields(Tables T, int ncellblk, int with_rho,
                                                       double* out) {
  __shared__ double red[4][4];
  double en = 0.0, res = 0.0, rm = 0.0, ga = 0.0;
  const int vb0 = blockIdx.x * REDUCE_SPAN;
  const int vb1 = min(vb0 + REDUCE_SPAN, ncellblk) - 1;
  int r0 = 0, r1 = 0;
  if (T.runs) {
    r0 = uniform(find_owner(T.run_blk, T.nruns, vb0));
    r1 = uniform(find_owner(T.run_blk, T.nruns, vb1));
  }
  if (r0 == r1) {
    // all blocks in one run: no flush inside the loop, so the loads of several blocks can
    // be in flight together
    const RunDesc r = run_of(T, r0);
    const int blk0 = vb0 - (T.runs ? T.run_blk[r0] : 0);
#pragma unroll 4
    for (int k = 0; k < REDUCE_SPAN; ++k) {
      CellIdx x;
      if (vb0 + k <= vb1 && cell_index(r, blk0 + k, DIM, x))
        reduce_cell<R, DIM>(r, x, with_rho, en, res, rm, ga);
    }
    reduce_flush<DIM>(r, out, with_rho, en, res, rm, ga, red);
    return;
  }
  int cur = -1;
  RunDesc r;
  for (int k = 0; k < REDUCE_SPAN; ++k) {
    const int vb = vb0 + k;
    if (vb >= ncellblk) break;
    int blk = vb, ri = 0;
    if (T.runs) {
      ri = uniform(find_owner(T.run_blk, T.nruns, vb));
      blk = uniform(vb - T.run_blk[ri]);
    }
    if (ri != cur) {
      if (cur >= 0) reduce_flush<DIM>(r, out, with_rho, en, res, rm, ga, red);
      en = res = rm = ga = 0.0;
      cur = ri;
      r = run_of(T, ri);
    }
    CellIdx x;
    if (!cell_index(r, blk, DIM, x)) continue;
    reduce_cell<R, DIM>(r, x, with_rho, en, res, rm, ga);
  }
  if (cur >= 0) reduce_flush<DIM>(r, out, with_rho, en, res, rm, ga, red);
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
// Moving window (open x ends): the box moves m cells in +x between two steps.  x is circular
// in the arrays, so only the box's origin column x0 moves: the m array columns that held the
// box's first columns become its last ones, so their fields are cleared and their particles
// removed, and fresh plasma fills the m columns just inside the right-hand margin.
// =======================================================================================
template <typename R>
__global__ __launch_bounds__(256) void k_window_clear(Tables T, int run, int m) {
  const RunDesc& r = run_of(T, run);
  const int64_t rows = (int64_t)r.ny * (r.ndim == 3 ? r.nz : 1);
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * m) return;
  const int col = (int)(e / rows);
  const int64_t c = (e - col * rows) * r.nx + array_x(r, col);   // box column col < m
#pragma unroll
  for (int k = 0; k < F_NUM; ++k)
    if (r.f[k]) gp((R*)r.f[k])[c] = R(0);
}

template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_window_kill(Tables T, int run, int m) {
  int blk;
  const SegDesc& s = seg_of(T, part_block(T, blk));
  if (s.run != run) return;
  const RunDesc& r = run_of(T, s.run);
  const int64_t p = (int64_t)blk * 256 + threadIdx.x;
  if (p >= s.n) return;
  if constexpr (sizeof(R) == 4) {
    gptr<int32_t> cell = gp((int32_t*)s.p[P_CELL]);
    const int32_t cv = cell[p];
    if (cv < 0) return;
    int c[3];
    unpack_cell(cv, DIM, c);
    if (box_x(r, c[0]) < m) cell[p] = -1;
  } else {
    gptr<double> x = gp((double*)s.p[P_X]);
    const double X = x[p] / r.dx;
    if (!(X >= 0.0 && X <= (double)r.nx)) return;   // dead already
    int ci = (int)floor(X);
    ci = ci >= r.nx ? ci - r.nx : ci;
    if (box_x(r, ci) < m) x[p] = -1.0;
  }
}

__global__ void k_window_advance(Tables T, int run, int m) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    RunDesc* r = const_cast<RunDesc*>(&T.runs[run]);
    const int x0 = r->x0 + m;
    r->x0 = x0 >= r->nx ? x0 - r->nx : x0;
  }
}

// Fresh plasma: particle k of the m * ny * px * py new ones sits in box column
// nx - OPEN_MARGIN - m + k / (ny px py), row (k / (px py)) mod ny, at lattice point
// ((l mod px) + 1/2) / px, ((l / px) + 1/2) / py of its cell (l = k mod px py).  It takes slot
// n_alive + used + k of the segment, n_alive being the start of the dead particles after the
// last sort; slots past the segment's end are not written and are counted in *dropped.
template <typename R, int DIM>
__global__ __launch_bounds__(256) void k_window_inject(Tables T, int seg, int m, int px,
                                                       int py, double w, double ux, double uy,
                                                       double uz, const int32_t* offsets,
                                                       int64_t used,
                                                       unsigned long long* dropped) {
  const SegDesc& s = seg_of(T, seg);
  const RunDesc& r = run_of(T, s.run);
  const int ppc = px * py;
  const int64_t per_col = (int64_t)r.ny * ppc;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= per_col * m) return;
  const int col = (int)(k / per_col);
  const int64_t rem = k - col * per_col;
  const int j = (int)(rem / ppc), l = (int)(rem - (int64_t)j * ppc);
  const int lx = l % px, ly = l / px;
  const int i = array_x(r, r.nx - OPEN_MARGIN - m + col);
  const double ox = (2.0 * lx + 1.0) / (2.0 * px), oy = (2.0 * ly + 1.0) / (2.0 * py);
  const int64_t slot = (int64_t)offsets[s.bin_base + r.ntiles] - s.pbase + used + k;
  if (slot < 0 || slot >= s.n) {
    atomicAdd(dropped, 1ull);
    return;
  }
  if constexpr (sizeof(R) == 4) {
    const int c[3] = {i, j, 0};
    gp((int32_t*)s.p[P_CELL])[slot] = pack_cell(c, DIM);
    gp((float*)s.p[P_OX])[slot] = (float)ox;
    gp((float*)s.p[P_OY])[slot] = (float)oy;
  } else {
    gp((double*)s.p[P_X])[slot] = (i + ox) * r.dx;
    gp((double*)s.p[P_Y])[slot] = (j + oy) * r.dy;
  }
  gp((R*)s.p[P_UX])[slot] = R(ux);
  gp((R*)s.p[P_UY])[slot] = R(uy);
  gp((R*)s.p[P_UZ])[slot] = R(uz);
  gp((R*)s.p[P_W])[slot] = R(w);
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
      c[d] = d == 0 ? array_x(r, ci) : ci;
      ((float*)s.p[P_OX + d])[p] = o;
    }
    ((int32_t*)s.p[P_CELL])[p] = pack_cell(c, DIM);
  } else {
    for (int d = 0; d < DIM; ++d) ((double*)s.p[P_X + d])[p] = src[d][p];
    if (r.x0 != 0 && src[0][p] >= 0.0) {   // array frame of a moved window
      const double L = r.nx * r.dx;
      double xa = src[0][p] + r.x0 * r.dx;
      ((double*)s.p[P_X])[p] = xa >= L ? xa - L : xa;
    }
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
    c[0] = box_x(r, c[0]);
    const double h[3] = {r.dx, r.dy, r.dz};
    for (int d = 0; d < DIM; ++d)
      dst[d][p] = ((double)c[d] + (double)((const float*)s.p[P_OX + d])[p]) * h[d];
  } else {
    for (int d = 0; d < DIM; ++d) dst[d][p] = ((const double*)s.p[P_X + d])[p];
    if (r.x0 != 0 && dst[0][p] >= 0.0) {   // box frame of a moved window
      const double xb = dst[0][p] - r.x0 * r.dx;
      dst[0][p] = xb < 0.0 ? xb + r.nx * r.dx : xb;
    }
  }
}

// =======================================================================================
// Host-side launchers
// =======================================================================================
template <typename R, int DIM>
static void launch_yee_t(const Tables& T, int nblocks, int which, double frac, int zero_j,
                         int halves, hipStream_t st, const FieldBands& bands) {
  if (which == 0) k_yee_e<R, DIM><<<nblocks, 256, 0, st>>>(T, frac, zero_j, halves);
  else k_yee_b<R, DIM><<<nblocks, 256, 0, st>>>(T, frac, bands);
}

void launch_yee(const Tables& T, int prec, int dim, int nblocks, int which, double frac,
                int zero_j, int halves, hipStream_t st, const FieldBands* bands) {
  FieldBands nb;
  memset(&nb, 0, sizeof(nb));
  const FieldBands& b = (bands && dim == 2) ? *bands : nb;
  if (prec == 0) {
    if (dim == 2) launch_yee_t<float, 2>(T, nblocks, which, frac, zero_j, halves, st, b);
    else launch_yee_t<float, 3>(T, nblocks, which, frac, zero_j, halves, st, b);
  } else {
    if (dim == 2) launch_yee_t<double, 2>(T, nblocks, which, frac, zero_j, halves, st, b);
    else launch_yee_t<double, 3>(T, nblocks, which, frac, zero_j, halves, st, b);
  }
}

template <typename R, int TX, bool PML>
static void launch_yee_mid_t(const Tables& T, int ntiles, const FieldBands& b, hipStream_t st) {
  if (b.ty == 16) k_yee_mid<R, TX, 16, PML><<<ntiles, 256, 0, st>>>(T, b);
  else if (b.ty == 8) k_yee_mid<R, TX, 8, PML><<<ntiles, 256, 0, st>>>(T, b);
  else k_yee_mid<R, TX, 4, PML><<<ntiles, 256, 0, st>>>(T, b);
}

template <typename R, bool PML>
static void launch_yee_mid_r(const Tables& T, int ntiles, const FieldBands& b, hipStream_t st) {
  if (b.tx == 64) launch_yee_mid_t<R, 64, PML>(T, ntiles, b, st);
  else if (b.tx == 32) launch_yee_mid_t<R, 32, PML>(T, ntiles, b, st);
  else if (b.tx == 16) launch_yee_mid_t<R, 16, PML>(T, ntiles, b, st);
  else launch_yee_mid_t<R, 8, PML>(T, ntiles, b, st);
}

void launch_yee_mid(const Tables& T, int prec, int ntiles, const FieldBands& bands, bool pml,
                    hipStream_t st) {
  if (ntiles <= 0) return;
  if (prec == 0) {
    if (pml) launch_yee_mid_r<float, true>(T, ntiles, bands, st);
    else launch_yee_mid_r<float, false>(T, ntiles, bands, st);
  } else {
    if (pml) launch_yee_mid_r<double, true>(T, ntiles, bands, st);
    else launch_yee_mid_r<double, false>(T, ntiles, bands, st);
  }
}

void launch_clear_sources(const Tables& T, int prec, int dim, int nblocks, int with_rho,
                          int32_t* flip, int64_t* clock, hipStream_t st) {
  LPIC_PD(prec, dim, (k_clear_sources<R, D><<<(nblocks + 3) / 4, 256, 0, st>>>(T, nblocks, with_rho,
                                                                              flip, clock)));
}

void launch_laser(const Tables& T, int prec, int dim, int nruns, int bpr, double t,
                  int64_t* step, unsigned int* done, hipStream_t st) {
  LPIC_PD(prec, dim, (k_laser<R, D><<<nruns * bpr, 256, 0, st>>>(T, nruns, bpr, t, step, done)));
}


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
                 hipStream_t st, int32_t* part) {
  LPIC_PD(prec, dim, (k_sort_count<R, D><<<nblocks, 256, 0, st>>>(T, counts)));
  launch_scan(counts, offsets, cursor, mult, nbins, spread, nullptr, 0, part, st);
  LPIC_PD(prec, dim, (k_sort_scatter<R, D><<<nblocks, 256, 0, st>>>(T, cursor, offsets, mult,
                                                                     spread)));
}

int fixed_shift_slots() { return WMAX_SLOTS; }

void launch_fixed_shift(const Tables& T, int prec, int dim, int nblocks, int nruns, int nsegs,
                        unsigned long long* wmax, int32_t* jshift, hipStream_t st) {
  if (nblocks > 0) {
    const int grid = (nblocks + WMAX_SPAN - 1) / WMAX_SPAN;
    LPIC_PD(prec, dim, (k_wmax<R, D><<<grid, 256, 0, st>>>(T, nblocks, wmax)));
  }
  k_fixed_shift<<<(nruns + 63) / 64, 64, 0, st>>>(T, nruns, nsegs, wmax, jshift);
}

void launch_swap_segments(SegDesc* segs, int nsegs, hipStream_t st) {
  k_swap_segments<<<(nsegs + 63) / 64, 64, 0, st>>>(segs, nsegs);
}

void launch_build_chunks(const Tables& T, const int32_t* offsets, int nvirt, int chunk,
                         Chunk* out, int32_t* nchunks, hipStream_t st, int32_t* part) {
  build_chunks(T, offsets, nvirt, chunk, out, nchunks, 0, nullptr, 0, part, st);
}

void launch_rebin(const Tables& T, int prec, int dim, const EscapeList& esc, const Rebin& rb,
                  hipStream_t st) {
  LPIC_PD(prec, dim, (k_rebin_count<R, D><<<rb.count_blocks, 256, 0, st>>>(T, esc, rb.threshold,
                                                                          rb.counts)));
  launch_scan(rb.counts, rb.offsets, rb.cursor, nullptr, rb.nbins, 0, esc.count, rb.threshold,
              rb.part, st);
  LPIC_PD(prec, dim, (k_rebin_scatter<R, D><<<rb.count_blocks, 256, 0, st>>>(
                         T, esc, rb.threshold, rb.cursor, rb.items, rb.rec)));
  build_chunks(T, rb.offsets, rb.nvirt, rb.chunk, rb.chunks, rb.nchunks, 1, esc.count,
               rb.threshold, rb.part, st);
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
  const int grid = (nblocks + REDUCE_SPAN - 1) / REDUCE_SPAN;
  LPIC_PD(prec, dim, (k_reduce_fields<R, D><<<grid, 256, 0, st>>>(T, nblocks, with_rho, out)));
}

void launch_zero_doubles(double* p, int n, hipStream_t st) {
  k_zero_doubles<<<(n + 255) / 256, 256, 0, st>>>(p, n);
}

void launch_diag_clear(const Tables& T, int nruns, hipStream_t st) {
  k_diag_clear<<<nruns, 64, 0, st>>>(T);
}

void launch_window_shift(const Tables& T, int prec, int dim, int run, int m, int64_t rows,
                         int nblk_part, hipStream_t st) {
  const unsigned nb = (unsigned)((rows * m + 255) / 256);
  if (prec == 0) k_window_clear<float><<<nb, 256, 0, st>>>(T, run, m);
  else k_window_clear<double><<<nb, 256, 0, st>>>(T, run, m);
  if (nblk_part > 0)
    LPIC_PD(prec, dim, (k_window_kill<R, D><<<nblk_part, 256, 0, st>>>(T, run, m)));
  k_window_advance<<<1, 64, 0, st>>>(T, run, m);
}

void launch_window_inject(const Tables& T, int prec, int dim, int seg, int m, int64_t count,
                          int px, int py, double w, double ux, double uy, double uz,
                          const int32_t* offsets, int64_t used, unsigned long long* dropped,
                          hipStream_t st) {
  const unsigned nb = (unsigned)((count + 255) / 256);
  if (nb == 0) return;
  LPIC_PD(prec, dim, (k_window_inject<R, D><<<nb, 256, 0, st>>>(T, seg, m, px, py, w, ux, uy,
                                                                 uz, offsets, used, dropped)));
}

void launch_load_positions(const Tables& T, int prec, int dim, int nblocks, const double* x,
                           const double* y, const double* z, hipStream_t st) {
  LPIC_PD(prec, dim, (k_load_positions<R, D><<<nblocks, 256, 0, st>>>(T, x, y, z)));
}

void launch_store_positions(const Tables& T, int prec, int dim, int nblocks, double* x,
                            double* y, double* z, hipStream_t st) {
  LPIC_PD(prec, dim, (k_store_positions<R, D><<<nblocks, 256, 0, st>>>(T, x, y, z)));
}


}  // namespace lpic
