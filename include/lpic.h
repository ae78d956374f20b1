/*
 * lpic.h -- C ABI of the MI355X (gfx950) electromagnetic PIC hot path.
 *
 * The library advances the particle-in-cell timestep of lambda-PIC (arXiv 2607.13507):
 * field half updates on the Yee grid, and per species a position half push, staggered
 * field interpolation, a relativistic Boris momentum push, a second position half push and
 * Esirkepov's charge-conserving current deposition (Sec. 3.1-3.3, Algorithm 1), with the
 * per-tile particle sort that keeps the particle stream local to the field tiles.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units are normalised: c = eps0 = 1, charge in e, mass in m_e, u = gamma v / c, so the
 * Maxwell system of Sec. 3.2 reads dE/dt = curl B - J, dB/dt = -curl E.  A macro-particle
 * carries a weight w that is the density it contributes, so rho = sum q w S.
 *
 * Grid arrays: one array per component, ncell = nx*ny*nz entries (nz = 1 in 2D), index
 * (k*ny + j)*nx + i, x fastest, NO guard cells: every boundary is periodic and is realised
 * by wrapping indices inside the kernels (the guard fill after each field half and the
 * guard fold of J after deposition of Algorithm 1 are therefore implicit).  Staggering of
 * entry [i,j,k] in cell units: Ex (i+1/2,j,k), Ey (i,j+1/2,k), Ez (i,j,k+1/2) (2D: (i,j)),
 * Bx (i,j+1/2,k+1/2), By (i+1/2,j,k+1/2), Bz (i+1/2,j+1/2,k); J as E; rho at (i,j,k).
 *
 * Precision:
 *   LPIC_F32_CELLOFS  fields float; particles hold a packed int32 cell coordinate and FP32
 *                     offsets in [0,1) inside that cell, FP32 momenta and weights.  Cell
 *                     packing: 2D  cell = iy<<16 | ix          (nx <= 65536, ny <= 32768)
 *                                 3D  cell = iz<<22 | iy<<11 | ix (nx, ny <= 2048, nz <= 512)
 *                     A dead particle has cell = -1.
 *   LPIC_F64_ABS      fields double; particles hold absolute FP64 positions (as the paper's
 *                     particle arrays do, Sec. 2.1), FP64 momenta and weights.  A dead
 *                     particle has x < 0.
 * FP64 is also used, in both modes, for the global energy and continuity reductions.
 *
 * Memory: every pointer in the structs below is a DEVICE pointer owned by the caller
 * (normally a PyTorch tensor); the library never frees it.  Entry points taking a
 * hipStream_t only enqueue work on that stream and return; errors detectable on the host
 * (bad sizes, null pointers, unsupported options) are reported before anything is
 * enqueued.  Functions return an lpic_status; lpic_last_error() gives a thread-local
 * message for the last failure.  No entry point aborts or throws.
 */
#ifndef LPIC_H
#define LPIC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LPIC_OK = 0,
  LPIC_EINVAL = -1,       /* invalid argument (null pointer, bad size, dt above CFL, ...) */
  LPIC_EHIP = -2,         /* a HIP runtime call failed; lpic_last_error() has the text */
  LPIC_ENOMEM = -3,       /* device allocation of library scratch failed */
  LPIC_EUNSUPPORTED = -4, /* valid request the build does not support */
  LPIC_EHOOK = -5,        /* a registered hook returned non-zero; the step stopped there */
  LPIC_ENUMERIC = -6      /* NaN or Inf found by a diagnostic reduction */
} lpic_status;

typedef enum { LPIC_F32_CELLOFS = 0, LPIC_F64_ABS = 1 } lpic_precision;

/* One simulation box (Sec. 3.2).  dt must satisfy the CFL bound
 * dt <= 1 / sqrt(dx^-2 + dy^-2 [+ dz^-2]).
 * open_x = 1 makes both x ends open (the absorbing boundaries of Sec. 3.2, where the paper
 * uses a CPML layer; here the first-order Mur outgoing-wave condition):
 *   - after every E update the tangential E of the first node column (Ey, Ez at i = 0), and
 *     after every B update the tangential B of the last column (By, Bz at i = nx-1), take
 *     u_new(edge) = u_old(inner) + k (u_new(inner) - u_old(edge)), k = (h - dx)/(h + dx),
 *     h the time step of that update (c = 1);
 *   - particles live only with x in [LPIC_OPEN_MARGIN dx, (nx - LPIC_OPEN_MARGIN) dx): a
 *     particle whose new position leaves that range is marked dead after depositing the
 *     current of that step (particles lost at boundaries, Sec. 2.1), so no interpolation
 *     or deposit stencil reaches across an open end.
 * y and z stay periodic. */
#define LPIC_OPEN_MARGIN 3
typedef struct {
  int32_t ndim;              /* 2 or 3 */
  int32_t nx, ny, nz;        /* cells; nz = 1 for ndim == 2 */
  double dx, dy, dz, dt;     /* dz ignored in 2D */
  double rho_bg;             /* fixed uniform background charge density (Gauss diagnostic) */
  int32_t open_x;            /* 0: periodic in x; 1: open x ends (above) */
  int32_t reserved0;         /* 0 */
} lpic_grid;

/* Laser antenna: the GaussianLaser callback of Sec. 2.2, injecting from the left boundary
 * as in the laser-plasma setup of Sec. 4.2.  A current sheet on node column ia,
 * J_pol += -2 E_inc / dx, radiates E_inc towards +x (and the same towards -x, which an
 * open left end absorbs), with
 *   E_inc(t, y, z) = a0 omega sin^2(pi (t - t0)/tau) exp(-((y - yc)^2 + (z - zc)^2)/waist^2)
 *                    sin(omega (t - t0))    for 0 <= t - t0 <= tau, else 0
 * (2D drops z; a0 is the normalised vector potential, omega the laser frequency, tau the
 * full duration of the sin^2 envelope).  pol = 1: E along y (J_y at (ia, j+1/2, k));
 * pol = 2: E along z (J_z at (ia, j) in 2D, (ia, j, k+1/2) in 3D).  Within a step the
 * antenna current is taken at t = (n+1) dt, the time level at which the E updates around
 * the end of step n use J (Algorithm 1). */
typedef struct {
  int32_t pol;               /* 1 or 2 */
  int32_t ia;                /* antenna node column, 0 <= ia < nx */
  double a0, omega, waist, yc, zc, t0, tau;
} lpic_laser;

/* Field arrays of one box, each ncell elements of float (F32) or double (F64). */
typedef struct {
  void *ex, *ey, *ez, *bx, *by, *bz;
  void *jx, *jy, *jz;
  void *rho0, *rho1;         /* optional charge at the start / end of the deposited paths
                                (may be NULL unless a call asks for it) */
} lpic_fields;

/* Particle arrays of one species (Sec. 2.1, structure of arrays), n slots each. */
typedef struct {
  int64_t n;                 /* number of slots (alive + dead), at most 2^29 */
  double q, m;               /* charge [e] and mass [m_e] */
  int32_t shape_order;       /* 1 = CIC (linear), 2 = quadratic spline */
  int32_t reserved0;
  int32_t *cell;             /* F32_CELLOFS: packed cell coordinate */
  void *ox, *oy, *oz;        /* F32_CELLOFS: float offsets; oz unused in 2D */
  void *x, *y, *z;           /* F64_ABS: double absolute positions; z unused in 2D */
  void *ux, *uy, *uz, *w;    /* float (F32) or double (F64) */
} lpic_species;

/* Tiling used by the sort and the fused particle kernel.  Tile edges are powers of two;
 * the field tile staged in on-chip memory is the tile plus `halo` cells on each side, and
 * a tile's particles are processed in chunks of at most `chunk` particles per workgroup.
 * A particle's gather and deposit touch cells up to 2 below and 3 above its cell, so with
 * halo h a particle may drift h - 2 cells below and h - 3 cells above its tile since the
 * last sort and stay on chip; particles beyond that are still handled exactly, through
 * global memory (counted in lpic_stats.halo_escapes).  halo must be >= 3.
 * flags: LPIC_SORT_SPREAD makes every sort spread each tile's particles over the tile's
 * range (see lpic_sort_tiles); without it only a simulation's first sort after particles
 * are loaded does.  LPIC_FIELD_SEPARATE (lpic_step in 2D): run the three field updates
 * between two particle pushes of consecutive steps (B by dt/2, E by dt, B by dt/2; Sec. 3.3,
 * Algorithm 1) as three grid-wide kernels; without it they run as one kernel over field
 * tiles of up to 64 x 16 cells whenever every box's nx and ny are multiples of a tile edge
 * (>= 8 and >= 4), which computes the same values with one pass over the arrays.
 * LPIC_ESCAPE_REBIN (lpic_step): when a step finds many particles (at least 4096) whose
 * gather stencil or deposit window leaves the staged region of the tile they were sorted
 * into, group them by the tile they are in now (a count, a scan and a scatter of their
 * indices; in 3D with each particle's words copied into a contiguous escape record) and push
 * them in a second pass of the fused kernel against the staged regions of those tiles,
 * instead of through global memory; the sort itself still runs every sort_interval steps.
 * Device memory, allocated when the flag is first set: two 8-byte entries per particle slot
 * beyond the escape list's own, and in 3D two escape records of 32 (FP32) or 64 (FP64)
 * bytes per slot. */
#define LPIC_SORT_SPREAD 1
#define LPIC_FIELD_SEPARATE 2
#define LPIC_ESCAPE_REBIN 4
typedef struct {
  int32_t tx, ty, tz;        /* tz ignored in 2D */
  int32_t halo;
  int32_t chunk;
  int32_t flags;             /* LPIC_SORT_SPREAD | LPIC_FIELD_SEPARATE | LPIC_ESCAPE_REBIN;
                                other bits must be 0 */
} lpic_tiling;

/* ---------------------------------------------------------------------------------------
 * Field solver -- Sec. 3.2 Eqs. 3-4, split into halves as in Algorithm 1.
 * which = 0: E += frac*dt*(curl B - J);  which = 1: B -= frac*dt*curl E.
 * flags LPIC_YEE_ZERO_J (which = 0 only): after J has been read, set J (and rho0/rho1 when
 * non-NULL) to zero, so that a following deposit starts from a clean array.
 * ------------------------------------------------------------------------------------- */
#define LPIC_YEE_ZERO_J 1
lpic_status lpic_yee_update_EB(const lpic_grid *grid, const lpic_fields *fields,
                               int32_t which, double frac, int32_t flags,
                               lpic_precision prec, hipStream_t stream);

/* ---------------------------------------------------------------------------------------
 * Gather + push -- Sec. 3.1 and the particle part of Algorithm 1 up to (not including) the
 * deposit: half position push to x^{n+1/2}, interpolation of E and B there, Boris push of
 * u by dt, second half position push to x^{n+1}, periodic wrap.  The half-step position
 * x^{n+1/2} of every particle -- the start of the path the deposit traces -- is written
 * into `old_state` (lpic_old_state_bytes() bytes, caller-owned device memory, layout private
 * to the library) for lpic_deposit_esirkepov.  Fields are read from global memory; no sort
 * is needed.
 * ------------------------------------------------------------------------------------- */
size_t lpic_old_state_bytes(int32_t ndim, int64_t n, lpic_precision prec);
lpic_status lpic_gather_push(const lpic_grid *grid, const lpic_fields *fields,
                             const lpic_species *sp, void *old_state, size_t old_bytes,
                             lpic_precision prec, hipStream_t stream);

/* ---------------------------------------------------------------------------------------
 * Esirkepov deposit -- Sec. 3.1 (Esirkepov 2001): adds into jx, jy, jz (NOT cleared) the
 * current of every particle's straight path over one dt centred on the end of the step:
 * from x^{n+1/2} (old_state) to x^{n+1/2} + dt v^{n+1} (v from the present momentum).  This
 * is the trajectory "from t - dt/2 to t + dt/2" of Sec. 3.1 around the whole time level at
 * which Eq. 3 applies J; x^{n+1} is the midpoint of the path.  In 2D, Jz uses v_z^{n+1}.
 * with_rho != 0 also adds q w S at the path start (rho0) and end (rho1), so that
 * rho1 - rho0 + dt div J = 0 holds node by node.
 * ------------------------------------------------------------------------------------- */
lpic_status lpic_deposit_esirkepov(const lpic_grid *grid, const lpic_fields *fields,
                                   const lpic_species *sp, const void *old_state,
                                   size_t old_bytes, int32_t with_rho, lpic_precision prec,
                                   hipStream_t stream);

/* ---------------------------------------------------------------------------------------
 * Tile sort -- Algorithm 1 sorts particles by cell before the push; here particles are
 * grouped by tile with a counting sort (histogram, scan, scatter) so that each workgroup
 * of the fused kernel reads one field tile.  Order inside a tile is not specified: by
 * default a tile keeps roughly the order its particles had; with LPIC_SORT_SPREAD in
 * tiling->flags the particle of rank r in a tile of N goes to slot r*P mod N (P coprime to
 * N, about N/64 stretches apart), so that particles that sat together -- typically in one
 * cell, as loaded -- end up in different wavefronts.  Spreading costs scattered writes
 * (several times a plain sort); once spread, the order stays mixed under later plain
 * sorts.  Dead particles go to the end.  The sorted arrays are written into `alt` (same sizes as `sp`),
 * then the array pointers of *sp and *alt are exchanged, so *sp describes the sorted data.
 * tile_offsets (device, int32, ntiles + 2 entries): start of every tile, then the start of
 * the dead block, then n.  ws: caller-owned device scratch of lpic_sort_ws_bytes() bytes.
 * ------------------------------------------------------------------------------------- */
size_t lpic_sort_ws_bytes(const lpic_grid *grid, const lpic_tiling *tiling, int64_t n);
int64_t lpic_num_tiles(const lpic_grid *grid, const lpic_tiling *tiling);
lpic_status lpic_sort_tiles(const lpic_grid *grid, lpic_species *sp, lpic_species *alt,
                            const lpic_tiling *tiling, int32_t *tile_offsets, void *ws,
                            size_t ws_bytes, lpic_precision prec, hipStream_t stream);

/* ---------------------------------------------------------------------------------------
 * lpic_sort_tiles for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same sort, argument
 * for argument, except that the bin counts, cursors and placement multipliers live in a
 * device array inside the library (3 x (LPIC_SORT_STATIC_MAX_TILES + 64) 32-bit words, about
 * 3 MiB, held on every device the library runs on until the process ends) instead of a
 * caller workspace.  It allocates nothing (no hipMalloc, hipFree or allocating library
 * routine) and enqueues only kernels.  At most LPIC_SORT_STATIC_MAX_TILES tiles: a larger
 * tiling returns LPIC_EINVAL.  Every call on one device shares that array, so calls that
 * overlap on one device (different streams, or host threads) race and must be serialised
 * by the caller; consecutive calls on one stream are fine (each clears the counts first).
 * ------------------------------------------------------------------------------------- */
#define LPIC_SORT_STATIC_MAX_TILES 262144
lpic_status lpic_sort_tiles_static(const lpic_grid *grid, lpic_species *sp, lpic_species *alt,
                                   const lpic_tiling *tiling, int32_t *tile_offsets,
                                   lpic_precision prec, hipStream_t stream);

/* ---------------------------------------------------------------------------------------
 * Fused gather + push + deposit -- the unified pusher of Sec. 2.3 / Sec. 3.3: one pass
 * over the particles of a species that does everything lpic_gather_push and
 * lpic_deposit_esirkepov do, with the field tile staged on chip and the current of a tile
 * accumulated on chip before one atomic flush.  Requires the particle order produced by
 * lpic_sort_tiles with the same tiling (tile_offsets from that call); particles that have
 * since left their tile are still handled exactly.  with_rho as in the deposit.
 * FP32: a tile's current is summed on chip in signed 64-bit fixed point, 2^-S per unit,
 * with S chosen per call from the particle count and the largest |q w| so that no sum can
 * overflow (S = 36 for 16.8M particles of |q w| ~ 0.6 and dx/dt ~ 1.5); the flush rounds
 * to FP32 once.  Such sums do not depend on the order of the adds.
 * kinetic (device double, may be NULL): adds sum w m u^2/(1+gamma) over the pushed
 * particles (new momenta, not multiplied by the cell volume).
 * ------------------------------------------------------------------------------------- */
size_t lpic_fused_ws_bytes(const lpic_grid *grid, const lpic_tiling *tiling, int64_t n);
lpic_status lpic_push_deposit_fused(const lpic_grid *grid, const lpic_fields *fields,
                                    const lpic_species *sp, const lpic_tiling *tiling,
                                    const int32_t *tile_offsets, void *ws, size_t ws_bytes,
                                    int32_t with_rho, double *kinetic, lpic_precision prec,
                                    hipStream_t stream);

/* ---------------------------------------------------------------------------------------
 * Position representation (input/output plumbing, not part of the step): convert absolute
 * FP64 positions (device arrays x, y, z) into the species' representation and back.
 * ------------------------------------------------------------------------------------- */
lpic_status lpic_load_positions(const lpic_grid *grid, const lpic_species *sp,
                                const double *x, const double *y, const double *z,
                                lpic_precision prec, hipStream_t stream);
lpic_status lpic_store_positions(const lpic_grid *grid, const lpic_species *sp, double *x,
                                 double *y, double *z, lpic_precision prec,
                                 hipStream_t stream);

/* ---------------------------------------------------------------------------------------
 * Laser antenna (struct lpic_laser above): adds the antenna current at time t into the
 * J component of `laser->pol` of `fields` (device arrays of the grid's size).
 * ------------------------------------------------------------------------------------- */
lpic_status lpic_laser_source(const lpic_grid *grid, const lpic_fields *fields,
                              const lpic_laser *laser, double t, lpic_precision prec,
                              hipStream_t stream);

/* ---------------------------------------------------------------------------------------
 * FP64 field diagnostics (energy of Sec. 4.1, continuity of Sec. 3.1).  Writes into
 * out (device, 4 doubles, overwritten):
 *   out[0] = sum (E^2 + B^2)/2 * dV                 field energy
 *   out[1] = max |rho1 - rho0 + dt div J|           continuity residual (needs rho0, rho1)
 *   out[2] = max |rho1|
 *   out[3] = max |div E - (rho0 + rho1)/2 - rho_bg|  Gauss residual (needs rho0, rho1)
 * Accumulation is FP64 whatever the field precision.
 * ------------------------------------------------------------------------------------- */
lpic_status lpic_reduce_fields(const lpic_grid *grid, const lpic_fields *fields,
                               int32_t with_rho, double *out, lpic_precision prec,
                               hipStream_t stream);

/* ---------------------------------------------------------------------------------------
 * Orchestration: Algorithm 1 over one box (or an ensemble of independent boxes) with
 * named-stage hooks (Sec. 2.2, Sec. 3.3).
 * ------------------------------------------------------------------------------------- */
typedef struct lpic_sim lpic_sim;

typedef enum {
  LPIC_STAGE_START = 0,             /* once, before the first step of a call */
  LPIC_STAGE_LOOP_START = 1,        /* start of every step */
  LPIC_STAGE_MAXWELL_1 = 2,         /* after the first field half update */
  LPIC_STAGE_PUSH_POSITION_1 = 3,   /* intermediate particle stages: registering a hook at */
  LPIC_STAGE_INTERPOLATOR = 4,      /* any of these four disables the fused kernel and   */
  LPIC_STAGE_PUSH_MOMENTUM = 5,     /* graph capture (the unified-pusher rule of          */
  LPIC_STAGE_PUSH_POSITION_2 = 6,   /* Sec. 2.3); they fire per species, between the      */
                                    /* split gather-push and deposit calls                 */
  LPIC_STAGE_CURRENT_DEPOSITION = 7,/* after all species deposited */
  LPIC_STAGE_QED_CREATE = 8,        /* after the deposit stage, where Algorithm 1 creates
                                       photons and pairs (e.g. lpic_qed_insert, compact) */
  LPIC_STAGE_MAXWELL_2 = 9,         /* after the second field half update */
  LPIC_STAGE_LOOP_END = 10,         /* end of every step */
  LPIC_STAGE_FINISH = 11,           /* once, after the last step of a call */
  LPIC_NUM_STAGES = 12
} lpic_stage;

/* A hook runs on the host between enqueued kernels; it may enqueue its own work on the
 * simulation's stream and may read or change any field or particle array.  Returning
 * non-zero stops lpic_step with LPIC_EHOOK. */
typedef int (*lpic_hook_fn)(lpic_sim *sim, int32_t stage, int64_t step, void *user);

typedef struct {
  lpic_tiling tiling;        /* tile shape, halo and chunk size (all runs) */
  int32_t sort_interval;     /* re-sort every K steps (>= 1) */
  int32_t diag_interval;     /* FP64 diagnostics every D steps (0 = never) */
  int32_t use_graph;         /* capture hook-free steps in a HIP graph */
  int32_t reserved0;
} lpic_options;

typedef struct {
  int64_t steps;             /* steps completed */
  int64_t sorts;             /* sorts performed */
  int32_t fused;             /* 1 when the fused kernel is in use */
  int32_t graph;             /* 1 when steps run as a captured graph */
  double fused_ms;           /* summed fused-kernel time measured with HIP events, when
                                timing is on (lpic_set_timing) */
  int64_t fused_launches;    /* launches covered by fused_ms */
  int64_t halo_escapes;      /* particle pushes that left their tile's on-chip halo and went
                                through global memory (cumulative) */
  int32_t field_tile[2];     /* tile (x, y) of the fused field update between steps; 0 0 when
                                those updates run as separate kernels (3D, LPIC_FIELD_SEPARATE,
                                or no tile edge divides every box) */
} lpic_stats;

/* Create a simulation over nruns independent boxes.  species[s] belongs to box
 * species_run[s]; species_alt[s] holds same-sized arrays used as the sort's second buffer.
 * fields[r].rho0/rho1 must be non-NULL when diagnostics are on; they hold the charge of the
 * latest diagnostic step (other steps neither write nor clear them, except that in 3D FP32
 * with 8x4x4 tiles and halo 3 the step before a diagnostic step inside the same lpic_step
 * call writes rho0: the charge at the ends of its paths, which is where the diagnostic
 * step's paths start, so that each step carries one charge plane in on-chip memory).  All
 * arrays stay owned by
 * the caller and must outlive the simulation; the library allocates only its own scratch
 * (sort workspace, tile and chunk tables, diagnostics) and frees it in lpic_sim_destroy. */
lpic_status lpic_sim_create(lpic_sim **out, int32_t nruns, const lpic_grid *grids,
                            const lpic_fields *fields, int32_t nspecies,
                            const lpic_species *species, const int32_t *species_run,
                            const lpic_species *species_alt, lpic_precision prec,
                            const lpic_options *opt, hipStream_t stream);
void lpic_sim_destroy(lpic_sim *sim);

/* Advance nsteps steps of Algorithm 1.  Returns after enqueueing (plus host hooks). */
lpic_status lpic_step(lpic_sim *sim, int32_t nsteps);

lpic_status lpic_register_hook(lpic_sim *sim, int32_t stage, lpic_hook_fn fn, void *user);
lpic_status lpic_clear_hooks(lpic_sim *sim);

/* Current arrays of species s (the sort exchanges the two buffers). */
lpic_status lpic_get_species(lpic_sim *sim, int32_t s, lpic_species *out);
lpic_status lpic_get_stats(lpic_sim *sim, lpic_stats *out);
/* Latest diagnostics of box r, synchronous: out[0] field energy, out[1] kinetic energy,
 * out[2] continuity residual / max|rho1|, out[3] Gauss residual max, out[4] the step they
 * were taken at.  LPIC_ENUMERIC if any is NaN or Inf.  With a laser antenna the two
 * residuals leave out the antenna's node column: its current is prescribed, not carried by
 * charges, and its transverse profile has a divergence. */
lpic_status lpic_get_diagnostics(lpic_sim *sim, int32_t r, double out[5]);
/* Per-kernel timing of the fused kernel with HIP events on the simulation's stream
 * (on = 1).  Timing forces eager launches (no graph). */
lpic_status lpic_set_timing(lpic_sim *sim, int32_t on);
/* Replace the options (tiling, intervals, graph) of an existing simulation, e.g. from an
 * autotuner; the next step re-sorts. */
lpic_status lpic_set_options(lpic_sim *sim, const lpic_options *opt);
/* Attach a laser antenna to run r (laser = NULL removes it).  Every step then adds the
 * antenna current at t = (step + 1) dt after the particles' deposit (before the
 * CURRENT_DEPOSITION hooks), where step counts the steps taken so far.  (A step whose
 * field updates are fused with the next step's -- see LPIC_FIELD_SEPARATE -- adds it inside
 * the E update instead of to the J array; J is cleared before anything else reads it.) */
lpic_status lpic_set_laser(lpic_sim *sim, int32_t r, const lpic_laser *laser);

/* Convolutional PML at the open x ends of run r (the absorbing layers Sec. 3.2 attaches to
 * the boundaries of the box; recursive-convolution form of Roden and Gedney, 2000, with the
 * complex frequency shift a), replacing the Mur condition of lpic_grid.open_x for that run.
 * The first and the last `cells` (L) node columns of x are the two layers (x stays
 * circular, so they meet back to back across the wrap).  Inside a layer each x derivative
 * D of the curls (dBz/dx in the Ey update, dBy/dx in Ez, dEz/dx in By, dEy/dx in Bz)
 * becomes D/kappa + psi, where psi (one value per component and location, held by the
 * library) first takes psi <- b psi + c D over an update of step tau:
 *   b = exp(-(sigma/kappa + a) tau),  c = sigma (b - 1) / (kappa (sigma + kappa a)),
 *   sigma = sigma_max s^order, kappa = 1 + (kappa_max - 1) s^order, a = a_max (1-s)^a_order,
 * s = depth / L, depth the distance in cells of the component's location from the layer's
 * inner face (node column L on the left, nx - L on the right; E-side locations on whole
 * columns, B-side ones half a column further in +x); x^0 = 1, so orders 0 give a uniform
 * layer.  sigma_max < 0 selects 0.8 (order + 1) / dx.  An E update of a whole dt made of two
 * merged halves applies the recursion twice.  Particles keep the open-end rule of
 * lpic_grid; a laser antenna belongs outside the layers (inside one its field is damped).
 * Requirements: run r has open_x; 1 <= cells, 2 cells <= nx - 8; order, a_order in [0, 8];
 * kappa_max >= 1, a_max >= 0, all finite.  pml = NULL removes the layers (Mur again).  Every
 * call sets psi to zero, rebuilds the device tables and drops captured graphs.  A run with
 * layers cannot move a window (LPIC_EUNSUPPORTED). */
typedef struct {
  int32_t cells;             /* L: layer thickness in cells at each open x end */
  int32_t order;             /* grading exponent of sigma and kappa (3 is usual) */
  int32_t a_order;           /* grading exponent of a (1 is usual) */
  int32_t reserved0;         /* 0 */
  double sigma_max;          /* < 0: 0.8 (order + 1) / dx */
  double kappa_max;          /* >= 1 */
  double a_max;              /* >= 0, in units of the inverse time unit */
} lpic_pml;
lpic_status lpic_set_pml(lpic_sim *sim, int32_t r, const lpic_pml *pml);

/* Fresh plasma for a moving window: ppc_x x ppc_y macro-particles per cell of species
 * `species` (a global species index of the run) on a regular lattice (offsets
 * (l + 1/2)/ppc per axis), weight density / (ppc_x ppc_y), momentum (ux, uy, uz). */
typedef struct {
  int32_t species;
  int32_t ppc_x, ppc_y;
  int32_t reserved0;
  double density;
  double ux, uy, uz;
} lpic_plasma;

/* Moving window (open x ends, 2D): between two steps, move box r by m cells in +x (a window
 * that follows a laser pulse; the paper's lazy deletion of Sec. 2.1 recycles the slots).
 * Field arrays are circular in x with a moving origin, so nothing is copied: the m columns
 * that were the box's first become its last, with their fields set to zero and their
 * particles removed (marked dead); with plasma != NULL, the m columns just inside the
 * right-hand margin (box columns nx-3-m .. nx-4) receive fresh particles, written into the
 * species' dead slots that follow its alive particles as of the last sort (slots beyond the
 * arrays are dropped and counted).  The next step re-sorts.  Field arrays and particle
 * arrays are then in the array frame: box column c is array column (c + x0) mod nx with
 * x0 = (total shift) mod nx (lpic_window_info), so lpic_store_positions returns array-frame
 * x, and box x = array x - x0 dx (mod nx dx).  A simulation that has moved a window runs the
 * field updates between steps as separate kernels.  1 <= m <= nx - 2*3 - 1; at least one
 * step must have been taken (the alive/dead split of the last sort is used). */
lpic_status lpic_window_shift(lpic_sim *sim, int32_t r, int32_t m, const lpic_plasma *plasma);
/* Total cells box r has moved, and fresh particles that found no free slot. */
lpic_status lpic_window_info(lpic_sim *sim, int32_t r, int64_t *shifted, int64_t *dropped);
/* Try the listed candidate options and keep the fastest (the simulation really advances);
 * writes the winner into *best when non-NULL.  Each candidate runs n steps untimed (its
 * sort, graph captures) and then n steps timed, where n is steps_each rounded up to a
 * multiple of its sort interval and of its diagnostics interval, so that every candidate
 * pays its own sorts and diagnostics in proportion; candidates compare by time per step.
 * Infeasible candidates (e.g. an LDS demand above the limit) are skipped. */
lpic_status lpic_autotune(lpic_sim *sim, const lpic_options *candidates, int32_t ncand,
                          int32_t steps_each, lpic_options *best);

/* Search space of lpic_autotune_search.  Each pair of bounds is inclusive and equal bounds
 * fix the parameter.  Tile edges and chunk sizes are powers of two (bounds are rounded to
 * them); tile_*[2] is ignored in 2D. */
#define LPIC_TUNE_MAX_TRIALS 64
typedef struct {
  int32_t tile_min[3], tile_max[3];
  int32_t halo_min, halo_max;
  int32_t chunk_min, chunk_max;
  int32_t sort_min, sort_max;  /* sort interval in steps */
  int32_t rebin;               /* LPIC_ESCAPE_REBIN: 0 off, 1 on, 2 both tried */
  int32_t steps_each;          /* timed steps per trial, rounded up to whole periods */
  int32_t max_trials;          /* at most this many timed trials (<= LPIC_TUNE_MAX_TRIALS;
                                  0 = LPIC_TUNE_MAX_TRIALS) */
} lpic_tune_space;

/* What the search tried: options and time per step of every trial in order (infeasible
 * ones, e.g. an LDS demand above the limit, have ms_per_step < 0), and the winner. */
typedef struct {
  int32_t ntrials;
  int32_t best;                /* index of the winning trial */
  lpic_options trial[LPIC_TUNE_MAX_TRIALS];
  double ms_per_step[LPIC_TUNE_MAX_TRIALS];
} lpic_tune_report;

/* Autotuner (the options of the fused kernel and the sort): a coordinate search over the
 * space, from the simulation's present options clamped into it.  For one parameter at a
 * time (tile edge x, y, z, halo, chunk, sort interval, re-binned escape path) it times the
 * neighbouring values (twice / half the size, one more / one less halo cell, the path on /
 * off) and keeps walking in a
 * direction while the time per step falls; it passes over the parameters again until no
 * move helps or the trial budget is spent.  Every trial runs as lpic_autotune's candidates
 * do (untimed warm-up period, then the timed steps; the simulation really advances), and
 * no option set is timed twice.  Leaves the simulation on the winner, written into *best
 * when non-NULL; *report (optional) receives every trial. */
lpic_status lpic_autotune_search(lpic_sim *sim, const lpic_tune_space *space,
                                 lpic_options *best, lpic_tune_report *report);

/* =======================================================================================
 * QED event Monte-Carlo -- Sec. 3.4: nonlinear Compton emission by leptons and
 * Breit-Wheeler pair creation by photons in the locally-constant-field approximation, each
 * particle carrying an optical depth that falls by (rate x dt) every step and triggers one
 * event where it reaches zero or below (event-based Monte-Carlo).  Units as everywhere in
 * this library (c = m_e = e = 1, time in 1/w_r, fields in m_e c w_r / e, momenta in m_e c);
 * hbar_omega = hbar w_r / (m_e c^2) sets the Schwinger field 1 / hbar_omega.
 *
 *   chi_e = hbar_omega sqrt((gamma E + u x B)^2 - (u . E)^2)         (lepton, momentum u)
 *   chi_g = hbar_omega sqrt((|k| E + k x B)^2 - (k . E)^2)           (photon, momentum k)
 *   emission: rate alpha h(chi_e) / (gamma hbar_omega), photon energy fraction xi of the
 *     spectrum F(chi, xi) = [(1 - xi + 1/(1 - xi)) K_{2/3}(y) - int_y^inf K_{1/3}] /
 *     (sqrt3 pi), y = 2 xi / (3 chi (1 - xi)), h(chi) = int_0^1 F;
 *   pairs: rate alpha T(chi_g) / (|k| hbar_omega), electron energy fraction xi of
 *     G(chi, xi) = [(xi/(1 - xi) + (1 - xi)/xi) K_{2/3}(y) + int_y^inf K_{1/3}] / (sqrt3 pi),
 *     y = 2 / (3 chi xi (1 - xi)), T(chi) = int_0^1 G.
 * h, T and the inverse cumulative distributions of F and G are tabulated once per process
 * (lpic_qed_tables_create) and interpolated: rates within ~1e-4 relative for chi in
 * [1e-4, 1e3] (emission) and [1e-2, 1e3] (pairs; below 1e-2 the pair rate, under
 * exp(-266) of the emission scale, is taken as zero); beyond 1e3 the tables extend with
 * their end slope.  Every random number is a counter-based SplitMix64 draw (Steele, Lea
 * and Flood 2014): output number ((step << 32) | slot) * 4 + draw of the generator seeded
 * with `seed`, mapped to ((z >> 11) + 1/2) 2^-53 in (0, 1); results depend on the slot
 * order, never on scheduling.  In both precisions the quantum parameters, rates x dt,
 * optical depths, decisions and records are FP64; the table lookups and -ln(draw) take
 * their logarithms and exponentials in FP32 (1e-7 relative, against the tables' 1e-4).
 * ======================================================================================= */
typedef struct lpic_qed_tables lpic_qed_tables;

/* Builds the tables on the host (a fraction of a second, on all host threads) and, with
 * on_device != 0, copies them to the current device.  The same tables serve every later
 * call; destroy releases both copies. */
lpic_status lpic_qed_tables_create(int32_t on_device, lpic_qed_tables **out);
lpic_status lpic_qed_tables_destroy(lpic_qed_tables *t);

/* Host evaluation of the tabulated quantities with the device's interpolation (for
 * checks): what = LPIC_QED_EMIT_RATE h(chi), LPIC_QED_EMIT_SAMPLE xi(chi, r),
 * LPIC_QED_PAIR_RATE T(chi), LPIC_QED_PAIR_SAMPLE xi(chi, r); NaN for a bad `what`. */
enum { LPIC_QED_EMIT_RATE = 0, LPIC_QED_EMIT_SAMPLE = 1, LPIC_QED_PAIR_RATE = 2,
       LPIC_QED_PAIR_SAMPLE = 3 };
double lpic_qed_table_eval(const lpic_qed_tables *t, int32_t what, double chi, double r);

typedef struct {
  double hbar_omega;     /* hbar w_r / (m_e c^2) > 0 */
  uint64_t seed;
  int64_t step;          /* the step number, part of every draw's counter (0 <= step < 2^30) */
} lpic_qed_params;

/* Event records, caller-owned device memory, FP64 absolute positions (z may be NULL in
 * 2D) and momenta: photons (from emission; the photon population itself) or leptons (from
 * pairs: the electron at an even index, the positron at the next).  *count (device) is the
 * number of records; a call that creates records advances it atomically and writes a
 * record only below capacity, so *count > capacity after a call reports an overflow (the
 * records beyond capacity are lost).  tau is the record's optical depth, src the index of
 * the particle or photon it came from.  A removed photon has x = -1.  The order of the
 * records a call appends is not specified (each workgroup of 1024 particles reserves one
 * contiguous range with a single atomic add; the ranges follow the workgroups' finishing
 * order); match records by src. */
typedef struct {
  int64_t capacity;
  int32_t *count;
  double *x, *y, *z, *ux, *uy, *uz, *w, *tau;
  int32_t *src;
} lpic_qed_buffer;

/* tau[i] = -ln U(seed, step, i, draw 2) for i < n: the optical depths of a fresh
 * population (device array). */
lpic_status lpic_qed_init_tau(double *tau, int64_t n, uint64_t seed, int64_t step,
                              hipStream_t stream);

/* lpic_gather_push with nonlinear Compton emission between the interpolation and the Boris
 * push, as Algorithm 1 places the QED step: for every live lepton, x^{n+1/2} from u^n, E
 * and B there, chi_e from u^n; tau (device, n doubles) falls by the emission rate x dt;
 * where it reaches zero or below, xi = the inverse-cdf sample at draw 0, a photon of
 * momentum xi gamma u/|u| is recorded in *photons at x^{n+1/2} (wrapped) with the lepton's
 * weight, depth -ln(draw 2) and src = the lepton's slot, the lepton keeps u - xi gamma
 * u/|u| and a new depth -ln(draw 1).  The rest (Boris, second half push, old_state for
 * lpic_deposit_esirkepov) is lpic_gather_push's.  Photons created here are part of the
 * next step's photon push (Algorithm 1 creates them after all species are pushed).
 * tau is indexed by slot, and lpic_sort_tiles does not move it: after a sort, draw the
 * depths afresh (lpic_qed_init_tau with a step number not used before).  That leaves the
 * event statistics unchanged, since a depth drawn as -ln U is exponential and so
 * memoryless: the remaining depth of a particle that has not fired is again -ln U. */
lpic_status lpic_qed_gather_push(const lpic_grid *grid, const lpic_fields *fields,
                                 const lpic_species *sp, double *tau,
                                 const lpic_qed_tables *tables, const lpic_qed_params *params,
                                 const lpic_qed_buffer *photons, void *old_state,
                                 size_t old_bytes, lpic_precision prec, hipStream_t stream);

/* One step of the photons in *photons (records [0, min(*count, capacity)) as *count stands
 * when the kernel starts; call it before the step's lpic_qed_gather_push): a photon moves
 * at c along k; at x^{n+1/2} (shape `order` gather from the fields, precision prec) tau
 * falls by the pair rate x dt; where it reaches zero or below, xi = the inverse-cdf sample
 * at draw 0 and two records go to *pairs at x^{n+1/2}: the electron with energy xi |k|,
 * the positron with (1 - xi) |k|, momenta along k (|u| = sqrt(gamma^2 - 1), zero below
 * gamma = 1), the photon's weight, depths -ln(draw 2) and -ln(draw 3), src = the photon's
 * index; the photon is removed (x = -1).  With open x ends a photon leaving
 * [LPIC_OPEN_MARGIN dx, (nx - LPIC_OPEN_MARGIN) dx) is removed. */
lpic_status lpic_qed_photon_push(const lpic_grid *grid, const lpic_fields *fields,
                                 int32_t order, const lpic_qed_buffer *photons,
                                 const lpic_qed_tables *tables, const lpic_qed_params *params,
                                 const lpic_qed_buffer *pairs, lpic_precision prec,
                                 hipStream_t stream);

/* Stable compaction of a record buffer, out of place: the records of *in (i < min(*count,
 * capacity)) that are alive (x >= 0; a converted photon is removed lazily by x = -1) are
 * copied to the front of *out in their order and *out->count is set to their number.
 * out->capacity >= in->capacity; ws: caller-owned device scratch of
 * lpic_qed_compact_ws_bytes(in->capacity) bytes.  The compacted records keep their src;
 * their slots (the counters of later photon draws) change. */
size_t lpic_qed_compact_ws_bytes(int64_t capacity);
lpic_status lpic_qed_compact(const lpic_qed_buffer *in, const lpic_qed_buffer *out, int32_t ndim,
                             void *ws, size_t ws_bytes, hipStream_t stream);

/* Inserts event records into a species (Sec. 3.4: the new particles of a pair go into the
 * species arrays; Algorithm 1 does it after all species are pushed): record i of *records
 * (i < min(*count, capacity) as the kernel starts) with i % 2 == parity (0: the electrons
 * of a pair buffer, 1: the positrons), or every record with parity = -1, is written into
 * slot first + i / 2 (first + i with parity -1) of *sp: its position in the species'
 * representation (a record with x < 0 becomes a dead slot), momentum and weight.  Slots
 * at or beyond sp->n are not written and counted in *dropped (device int32, may be NULL).
 * The caller chooses `first`, e.g. the start of the dead block that lpic_sort_tiles
 * reports (tile_offsets[ntiles]); what the slots held before is overwritten. */
lpic_status lpic_qed_insert(const lpic_grid *grid, const lpic_species *sp, int64_t first,
                            const lpic_qed_buffer *records, int32_t parity, int32_t *dropped,
                            lpic_precision prec, hipStream_t stream);

const char *lpic_last_error(void);
const char *lpic_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LPIC_H */
