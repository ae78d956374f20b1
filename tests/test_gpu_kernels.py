"""Per-kernel parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (relative to the largest magnitude of the compared quantity):
  FP64 path  1e-11  -- only rounding order differs from the oracle (atomics, FMA)
  FP32 path  2e-5   -- single-precision arithmetic: each quantity passes through O(10-100)
                       FP32 operations with unit round-off 6e-8, on inputs the oracle
                       receives already rounded to FP32
Positions are compared in cell units (periodic distance).
"""
import numpy as np
import pytest
import torch

from gpu_helpers import (FIELDS, banner, compare_fields, compare_particles, device_state,
                         periodic_diff)
from oracle import OracleSim
from paper_2607_13507_amd import lpic as L
from paper_2607_13507_amd import workloads as W
from paper_2607_13507_amd.simulation import DeviceSpecies

pytestmark = pytest.mark.gpu

PRECS = [L.F64_ABS, L.F32_CELLOFS]
PNAME = {L.F64_ABS: "f64", L.F32_CELLOFS: "f32"}


def small_2d(order, seed=5, nx=40, ny=36, ppc=6, T=0.3):
    # 40x36 cells: several 16x16 tiles and a ragged tail in both directions
    return W.thermal_2d(nx=nx, ny=ny, dx=0.1, ppc=ppc, T=T, order=order, seed=seed)


def small_3d(order, seed=6, n=20, ppc=2, T=0.3):
    return W.thermal_3d(n=n, dx=0.1, ppc=ppc, T=T, order=order, seed=seed)


@pytest.mark.parametrize("prec", PRECS, ids=PNAME.get)
@pytest.mark.parametrize("ndim", [2, 3])
def test_yee_half_updates(prec, ndim):
    banner(f"yee prec={PNAME[prec]} ndim={ndim}")
    wl = small_2d(1) if ndim == 2 else small_3d(1)
    wl.species = []
    grid, F, S, orc = device_state(wl, prec, random_fields_seed=3)
    rng = np.random.default_rng(4)
    for k in ("jx", "jy", "jz"):
        v = rng.uniform(-1, 1, wl.ncell)
        F.t[k].copy_(torch.from_numpy(v))
        orc.f[k][:] = F.t[k].double().cpu().numpy()
    L.lpic_yee_update_EB(grid, F.struct(), 0, 0.5, 0, prec)
    orc.yee_e(0.5)
    compare_fields(F, orc, prec, what="E half")
    L.lpic_yee_update_EB(grid, F.struct(), 1, 0.5, 0, prec)
    orc.yee_b(0.5)
    compare_fields(F, orc, prec, what="B half")
    L.lpic_yee_update_EB(grid, F.struct(), 0, 0.5, L.YEE_ZERO_J, prec)
    orc.yee_e(0.5)
    compare_fields(F, orc, prec, keys=("ex", "ey", "ez"), what="E half + clear")
    for k in ("jx", "jy", "jz"):
        assert torch.count_nonzero(F.t[k]).item() == 0
    assert torch.count_nonzero(F.rho0).item() == 0


@pytest.mark.parametrize("prec", PRECS, ids=PNAME.get)
@pytest.mark.parametrize("ndim,order", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_gather_push_then_deposit(prec, ndim, order):
    banner(f"split push/deposit prec={PNAME[prec]} ndim={ndim} order={order}")
    wl = small_2d(order) if ndim == 2 else small_3d(order)
    grid, F, S, orc = device_state(wl, prec, random_fields_seed=7, field_scale=0.5)
    d, o = S[0], orc.species[0]
    nbytes = L.lpic_old_state_bytes(ndim, d.n, prec)
    old = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    L.lpic_gather_push(grid, F.struct(), d.struct(), old.data_ptr(), nbytes, prec)
    L.lpic_deposit_esirkepov(grid, F.struct(), d.struct(), old.data_ptr(), nbytes, 1, prec)
    torch.cuda.synchronize()
    orc.zero_currents()
    orc.push_deposit(o)
    compare_particles(grid, d, o, prec, what="push")
    compare_fields(F, orc, prec, keys=("jx", "jy", "jz", "rho0", "rho1"), what="deposit")


def _tiling(prec, ndim, chunk):
    """Tiles that span several tiles of the small boxes with a ragged edge, and fit LDS."""
    if ndim == 2:
        return L.Tiling(16, 8, 1, 4, chunk, 0)
    if prec == L.F64_ABS:
        return L.Tiling(8, 4, 4, 3, chunk, 0)
    return L.Tiling(8, 8, 4, 3, chunk, 0)


def _sorted_state(wl, prec, tiling):
    grid, F, S, orc = device_state(wl, prec, random_fields_seed=9, field_scale=0.5)
    d = S[0]
    alt = d.like()
    nt = L.lpic_num_tiles(grid, tiling)
    offs = torch.zeros(nt + 2, dtype=torch.int32, device="cuda")
    wsb = L.lpic_sort_ws_bytes(grid, tiling, d.n)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    s_struct, a_struct = d.struct(), alt.struct()
    L.lpic_sort_tiles(grid, s_struct, a_struct, tiling, offs.data_ptr(), ws.data_ptr(), wsb, prec)
    torch.cuda.synchronize()
    return grid, F, d, alt, offs, orc


def _tile_of(grid, tiling, pos):
    tx = np.floor(pos[0] / grid.dx).astype(np.int64) // tiling.tx
    ty = np.floor(pos[1] / grid.dy).astype(np.int64) // tiling.ty
    ntx = -(-grid.nx // tiling.tx)
    nty = -(-grid.ny // tiling.ty)
    t = ty * ntx + tx
    if grid.ndim == 3:
        tz = np.floor(pos[2] / grid.dz).astype(np.int64) // tiling.tz
        t = t + tz * ntx * nty
    return t


@pytest.mark.parametrize("prec", PRECS, ids=PNAME.get)
@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("spread", [False, True], ids=["plain", "spread"])
def test_sort_is_an_exact_tile_grouping(prec, ndim, spread):
    banner(f"sort prec={PNAME[prec]} ndim={ndim} spread={spread}")
    wl = small_2d(2) if ndim == 2 else small_3d(2)
    n = wl.species[0].n
    wl.species[0].w = np.arange(1, n + 1, dtype=np.float64)   # unique tags (exact in FP32)
    # kill a few particles: they must end up after every tile
    dead = np.arange(0, n, 97)
    wl.species[0].x[dead] = -1.0
    tiling = _tiling(prec, ndim, chunk=64)
    tiling.flags = L.SORT_SPREAD if spread else 0
    grid, F, d0, alt, offs, orc = _sorted_state(wl, prec, tiling)
    # after the call the struct's pointers were exchanged: `alt` tensors hold the sorted data
    cur, before = alt, d0
    tags_before = before.numpy("w")
    tags_after = cur.numpy("w")
    assert sorted(tags_after.tolist()) == sorted(tags_before.tolist())
    order = np.argsort(tags_before)
    inv = order[np.searchsorted(tags_before[order], tags_after)]
    for k in cur.a:
        np.testing.assert_array_equal(cur.numpy(k), before.numpy(k)[inv])   # bit-exact payload
    o = offs.cpu().numpy()
    nt = L.lpic_num_tiles(grid, tiling)
    assert o[0] == 0 and o[-1] == n and np.all(np.diff(o) >= 0)
    assert o[nt + 1] - o[nt] == len(dead)
    pos = cur.positions(grid)
    alive = pos[0] >= 0
    assert np.all(~alive[o[nt]:]) and np.all(alive[:o[nt]])
    tiles = _tile_of(grid, tiling, pos)[: o[nt]]
    expect = np.repeat(np.arange(nt), np.diff(o[: nt + 1]))
    np.testing.assert_array_equal(tiles, expect)


@pytest.mark.parametrize("prec", PRECS, ids=PNAME.get)
@pytest.mark.parametrize("ndim,order", [(2, 1), (2, 2), (3, 1), (3, 2)])
@pytest.mark.parametrize("displaced", [False, True], ids=["in_tile", "escaped"])
def test_fused_matches_oracle(prec, ndim, order, displaced):
    banner(f"fused prec={PNAME[prec]} ndim={ndim} order={order} displaced={displaced}")
    wl = small_2d(order) if ndim == 2 else small_3d(order)
    tiling = _tiling(prec, ndim, chunk=97)    # odd chunk size: ragged chunks
    grid, F, d0, cur, offs, orc = _sorted_state(wl, prec, tiling)
    o = orc.species[0]
    # the oracle follows the sorted order
    pos = cur.positions(grid)
    o.x[:], o.y[:] = pos[0], pos[1]
    if ndim == 3:
        o.z[:] = pos[2]
    for k in ("ux", "uy", "uz", "w"):
        getattr(o, k)[:] = cur.numpy(k)
    if displaced:
        # move every particle by up to 6 cells without re-sorting: most leave the on-chip
        # halo of their home tile and must take the global-memory path
        rng = np.random.default_rng(1)
        shift = [rng.integers(-6, 7, cur.n) * h for h in (grid.dx, grid.dy, grid.dz)]
        Ls = (grid.nx * grid.dx, grid.ny * grid.dy, grid.nz * grid.dz)
        new = [np.mod(pos[dd] + shift[dd], Ls[dd]) for dd in range(ndim)]
        cur.load_positions(grid, *new, *([None] * (3 - ndim)))
        pos = cur.positions(grid)
        o.x[:], o.y[:] = pos[0], pos[1]
        if ndim == 3:
            o.z[:] = pos[2]
    ke = torch.zeros(1, dtype=torch.float64, device="cuda")
    wsb = L.lpic_fused_ws_bytes(grid, tiling, cur.n)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    L.lpic_push_deposit_fused(grid, F.struct(), cur.struct(), tiling, offs.data_ptr(),
                              ws.data_ptr(), wsb, 1, ke.data_ptr(), prec)
    torch.cuda.synchronize()
    orc.zero_currents()
    orc.push_deposit(o)
    compare_particles(grid, cur, o, prec, what="fused push")
    compare_fields(F, orc, prec, keys=("jx", "jy", "jz", "rho0", "rho1"), what="fused deposit")
    dV = grid.dx * grid.dy * (grid.dz if ndim == 3 else 1.0)
    assert ke.item() * dV == pytest.approx(orc.kinetic_energy(), rel=1e-11 if prec == L.F64_ABS else 1e-5)


@pytest.mark.parametrize("prec", PRECS, ids=PNAME.get)
def test_reduce_fields_matches_oracle(prec):
    banner(f"reduce prec={PNAME[prec]}")
    wl = small_2d(2)
    grid, F, S, orc = device_state(wl, prec, random_fields_seed=11)
    d, o = S[0], orc.species[0]
    nbytes = L.lpic_old_state_bytes(2, d.n, prec)
    old = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    for k in ("jx", "jy", "jz"):
        F.t[k].zero_()
    F.rho0.zero_()
    F.rho1.zero_()
    L.lpic_gather_push(grid, F.struct(), d.struct(), old.data_ptr(), nbytes, prec)
    L.lpic_deposit_esirkepov(grid, F.struct(), d.struct(), old.data_ptr(), nbytes, 1, prec)
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    L.lpic_reduce_fields(grid, F.struct(), 1, out.data_ptr(), prec)
    torch.cuda.synchronize()
    r = out.cpu().numpy()
    # reference values from the GPU's own arrays, summed in FP64 on the host
    g = F.numpy()
    ref = OracleSim(2, wl.nx, wl.ny, 1, wl.dx, wl.dy, 1.0, wl.dt, wl.rho_bg, [],
                    {k: g[k] for k in FIELDS})
    ref.rho0[:] = g["rho0"]
    ref.rho1[:] = g["rho1"]
    assert r[0] == pytest.approx(ref.field_energy(), rel=1e-12)
    assert r[1] / r[2] == pytest.approx(ref.continuity(), rel=1e-6, abs=1e-15)
    assert r[3] == pytest.approx(np.abs(ref.gauss()).max(), rel=1e-12)
    assert r[1] / r[2] < (1e-13 if prec == L.F64_ABS else 1e-5)


@pytest.mark.parametrize("prec", PRECS, ids=PNAME.get)
def test_empty_and_dead_species(prec):
    banner(f"empty/dead prec={PNAME[prec]}")
    wl = small_2d(1, ppc=1)
    n = wl.species[0].n
    wl.species[0].x[:] = -1.0          # every particle dead
    grid, F, S, orc = device_state(wl, prec, random_fields_seed=2)
    d = S[0]
    nbytes = L.lpic_old_state_bytes(2, d.n, prec)
    old = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    before = {k: d.numpy(k).copy() for k in d.a}
    L.lpic_gather_push(grid, F.struct(), d.struct(), old.data_ptr(), nbytes, prec)
    L.lpic_deposit_esirkepov(grid, F.struct(), d.struct(), old.data_ptr(), nbytes, 1, prec)
    torch.cuda.synchronize()
    for k in d.a:
        np.testing.assert_array_equal(d.numpy(k), before[k])
    for k in ("jx", "jy", "jz"):
        assert torch.count_nonzero(F.t[k]).item() == 0
    empty = DeviceSpecies(2, 0, -1.0, 1.0, 2, prec)
    L.lpic_gather_push(grid, F.struct(), empty.struct(), None, 0, prec)
    tiling = L.Tiling(16, 16, 1, 4, 256, 0)
    offs = torch.full((L.lpic_num_tiles(grid, tiling) + 2,), 7, dtype=torch.int32, device="cuda")
    ws = torch.empty(L.lpic_sort_ws_bytes(grid, tiling, 0), dtype=torch.uint8, device="cuda")
    L.lpic_sort_tiles(grid, empty.struct(), empty.like().struct(), tiling, offs.data_ptr(),
                      ws.data_ptr(), ws.numel(), prec)
    torch.cuda.synchronize()
    assert torch.count_nonzero(offs).item() == 0


def test_cell_offset_precision_independent_of_position():
    """FP32 cell + offset: a slow particle far from the origin moves exactly like one near
    it (absolute FP32 would have an ulp of 2^-11 cell at x = 8190 cells)."""
    banner("cell+offset precision")
    nx = 8192
    wl = W.thermal_2d(nx=nx, ny=8, dx=0.1, ppc=1, T=0.0, order=2, seed=1)
    sp = wl.species[0]
    sel = np.array([0, 1])
    for k in ("x", "y", "ux", "uy", "uz", "w"):
        setattr(sp, k, getattr(sp, k)[sel].copy())
    sp.x[:] = np.array([2.3, 8190.3]) * 0.1
    sp.y[:] = 0.45
    sp.ux[:] = 1e-4
    sp.w[:] = 0.0
    grid, F, S, orc = device_state(wl, L.F32_CELLOFS)
    F.t["ex"].fill_(1e-3)
    d = S[0]
    nbytes = L.lpic_old_state_bytes(2, d.n, L.F32_CELLOFS)
    old = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    for _ in range(200):
        L.lpic_gather_push(grid, F.struct(), d.struct(), old.data_ptr(), nbytes, L.F32_CELLOFS)
    torch.cuda.synchronize()
    ox = d.numpy("ox")
    cell = d.numpy("cell") & 0xFFFF
    assert ox[0] == ox[1]                       # bitwise identical offsets
    assert cell[1] - cell[0] == 8188
    assert d.numpy("ux")[0] == d.numpy("ux")[1]


def test_offset_rounding_edge():
    """A particle a hair left of a cell edge lands on the edge, never at offset 1.0."""
    banner("offset rounding edge")
    wl = W.thermal_2d(nx=16, ny=16, dx=0.1, ppc=1, T=0.0, order=1, seed=1)
    sp = wl.species[0]
    m = 64
    for k in ("x", "y", "ux", "uy", "uz", "w"):
        setattr(sp, k, getattr(sp, k)[:m].copy())
    rng = np.random.default_rng(3)
    sp.x[:] = (np.arange(m) % 16 + 1e-9 * rng.random(m)) * 0.1
    sp.ux[:] = -1e-7 * (1 + rng.random(m))        # moves left by ~1e-8 cells: crosses
    sp.w[:] = 0.0
    grid, F, S, orc = device_state(wl, L.F32_CELLOFS)
    d = S[0]
    nbytes = L.lpic_old_state_bytes(2, d.n, L.F32_CELLOFS)
    old = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    L.lpic_gather_push(grid, F.struct(), d.struct(), old.data_ptr(), nbytes, L.F32_CELLOFS)
    torch.cuda.synchronize()
    ox = d.numpy("ox")
    assert np.all(ox >= 0.0) and np.all(ox < 1.0)
    pos = d.positions(grid)[0]
    exp = np.mod(sp.x - 1e-7 * 0.5 * wl.dt, 1.6)
    assert np.abs(periodic_diff(pos, sp.x, 1.6)).max() < 1e-7


@pytest.mark.parametrize("prec", PRECS, ids=PNAME.get)
@pytest.mark.parametrize("n", [540, 577, 1000])
def test_fused_covers_every_chunk(prec, n):
    """One tile holding every particle: the chunk count (9, 10, 16 for chunk 64) is close to
    the launch bound, so each of the eight XCD ranges must still be covered by workgroups."""
    banner(f"fused chunk coverage prec={PNAME[prec]} n={n}")
    wl = W.thermal_2d(nx=16, ny=16, dx=0.1, ppc=4, T=0.1, order=2, seed=n)
    sp = wl.species[0]
    for k in ("x", "y", "ux", "uy", "uz", "w"):
        setattr(sp, k, getattr(sp, k)[:n].copy())
    tiling = L.Tiling(16, 16, 1, 4, 64, 0)
    grid, F, d0, cur, offs, orc = _sorted_state(wl, prec, tiling)
    o = orc.species[0]
    pos = cur.positions(grid)
    o.x[:], o.y[:] = pos[0], pos[1]
    for k in ("ux", "uy", "uz", "w"):
        getattr(o, k)[:] = cur.numpy(k)
    wsb = L.lpic_fused_ws_bytes(grid, tiling, cur.n)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    L.lpic_push_deposit_fused(grid, F.struct(), cur.struct(), tiling, offs.data_ptr(),
                              ws.data_ptr(), wsb, 1, None, prec)
    torch.cuda.synchronize()
    orc.zero_currents()
    orc.push_deposit(o)
    compare_particles(grid, cur, o, prec, what="fused push")
    compare_fields(F, orc, prec, keys=("jx", "jy", "jz", "rho0", "rho1"), what="fused deposit")


@pytest.mark.parametrize("prec", PRECS, ids=PNAME.get)
@pytest.mark.parametrize("ndim,order", [(2, 1), (2, 2), (3, 2)])
@pytest.mark.parametrize("halo", [3, 4])
def test_fused_window_edges(prec, ndim, order, halo):
    """Particles moved after the sort to the farthest cells that still count as on chip
    (h - 2 below their tile, h - 3 above it), moving outwards at 0.99 c along every axis at
    once: their gather and deposit windows reach the edges of the staged region, and the
    results must equal the oracle's."""
    banner(f"fused window edges prec={PNAME[prec]} ndim={ndim} order={order} halo={halo}")
    if prec == L.F64_ABS and ndim == 3 and halo == 4:
        pytest.skip("FP64 3D region with halo 4 does not fit the LDS at this tile")
    wl = small_2d(order) if ndim == 2 else small_3d(order)
    T = (16, 8, 1) if ndim == 2 else (8, 4, 4)
    tiling = L.Tiling(*T, halo, 61, 0)
    grid, F, d0, cur, offs, orc = _sorted_state(wl, prec, tiling)
    o = orc.species[0]
    pos = cur.positions(grid)
    h = (grid.dx, grid.dy, grid.dz)
    n = (grid.nx, grid.ny, grid.nz)
    rng = np.random.default_rng(7)
    side = rng.integers(0, 2, (ndim, cur.n))            # 0: low edge, 1: high edge, per axis
    new, u = [], []
    for a in range(ndim):
        cell = np.floor(pos[a] / h[a]).astype(np.int64)
        t0 = (cell // T[a]) * T[a]                        # the home tile's first cell
        lo = t0 - (halo - 2)
        hi = t0 + T[a] - 1 + (halo - 3)
        c = np.where(side[a] == 0, lo, hi)
        frac = np.where(side[a] == 0, 0.01, 0.99)
        new.append(np.mod((c + frac) * h[a], n[a] * h[a]))
        u.append(np.where(side[a] == 0, -7.0, 7.0))
    cur.load_positions(grid, *new, *([None] * (3 - ndim)))
    for a, k in enumerate(("ux", "uy", "uz")[:ndim]):
        cur.a[k].copy_(torch.from_numpy(u[a]).to(cur.a[k].dtype))
    pos = cur.positions(grid)
    o.x[:], o.y[:] = pos[0], pos[1]
    if ndim == 3:
        o.z[:] = pos[2]
    for k in ("ux", "uy", "uz", "w"):
        getattr(o, k)[:] = cur.numpy(k)
    wsb = L.lpic_fused_ws_bytes(grid, tiling, cur.n)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    L.lpic_push_deposit_fused(grid, F.struct(), cur.struct(), tiling, offs.data_ptr(),
                              ws.data_ptr(), wsb, 1, None, prec)
    torch.cuda.synchronize()
    orc.zero_currents()
    orc.push_deposit(o)
    compare_particles(grid, cur, o, prec, what="edge push")
    compare_fields(F, orc, prec, keys=("jx", "jy", "jz", "rho0", "rho1"), what="edge deposit")


@pytest.mark.parametrize("halo", [3, 4])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("prec", [L.F64_ABS, L.F32_CELLOFS], ids=["f64", "f32"])
def test_fused_exact_fit_edges(prec, ndim, order, halo):
    """Particles placed after the sort on the first and last cells a particle can start from
    and still be on chip (h - 1 below its tile, h - 2 above it: region cells 1 and rw - 3),
    at random offsets, with momenta from slow (|u| ~ 0.01) to ultra-relativistic (|u| ~ 20)
    along every axis: the slow ones stay on chip, the fast ones' gather stencil or deposit
    window leaves the staged region and they escape to the global-memory path; either way
    the results must equal the oracle's (and nothing outside the region is touched)."""
    banner(f"fused exact fit edges prec={PNAME[prec]} ndim={ndim} order={order} halo={halo}")
    if prec == L.F64_ABS and ndim == 3 and halo == 4:
        pytest.skip("FP64 3D region with halo 4 does not fit the LDS at this tile")
    wl = small_2d(order) if ndim == 2 else small_3d(order)
    T = (16, 8, 1) if ndim == 2 else (8, 4, 4)
    tiling = L.Tiling(*T, halo, 61, 0)
    grid, F, d0, cur, offs, orc = _sorted_state(wl, prec, tiling)
    o = orc.species[0]
    pos = cur.positions(grid)
    h = (grid.dx, grid.dy, grid.dz)
    n = (grid.nx, grid.ny, grid.nz)
    rng = np.random.default_rng(11 + halo + 3 * order + 7 * ndim)
    side = rng.integers(0, 2, (ndim, cur.n))
    speed = 10.0 ** rng.uniform(-2, 1.3, cur.n)        # |u| from 0.01 to 20
    new, u = [], []
    for a in range(ndim):
        cell = np.floor(pos[a] / h[a]).astype(np.int64)
        t0 = (cell // T[a]) * T[a]
        c = np.where(side[a] == 0, t0 - (halo - 1), t0 + T[a] - 1 + (halo - 2))
        new.append(np.mod((c + rng.random(cur.n)) * h[a], n[a] * h[a]))
        u.append(speed * rng.uniform(-1, 1, cur.n))
    cur.load_positions(grid, *new, *([None] * (3 - ndim)))
    for a, k in enumerate(("ux", "uy", "uz")[:ndim]):
        cur.a[k].copy_(torch.from_numpy(u[a]).to(cur.a[k].dtype))
    pos = cur.positions(grid)
    o.x[:], o.y[:] = pos[0], pos[1]
    if ndim == 3:
        o.z[:] = pos[2]
    for k in ("ux", "uy", "uz", "w"):
        getattr(o, k)[:] = cur.numpy(k)
    wsb = L.lpic_fused_ws_bytes(grid, tiling, cur.n)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    L.lpic_push_deposit_fused(grid, F.struct(), cur.struct(), tiling, offs.data_ptr(),
                              ws.data_ptr(), wsb, 1, None, prec)
    torch.cuda.synchronize()
    orc.zero_currents()
    orc.push_deposit(o)
    compare_particles(grid, cur, o, prec, what="exact-fit edge push")
    compare_fields(F, orc, prec, keys=("jx", "jy", "jz", "rho0", "rho1"),
                   what="exact-fit edge deposit")
