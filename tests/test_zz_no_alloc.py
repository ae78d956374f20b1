"""lpic_sort_tiles_static (the tile sort for callers that cannot allocate: its scratch is a
device array inside the library) against lpic_sort_tiles with a caller workspace, through
the C ABI: two calls in a row on the same device, the second with a smaller input (fewer
particles and fewer tiles), each compared element by element with the workspace variant
(bit-exact permutation of the particle records and identical tile offsets); and the size
limit is refused before anything is enqueued."""
import numpy as np
import pytest
import torch

from paper_2607_13507_amd import lpic as L
from paper_2607_13507_amd import workloads as W
from paper_2607_13507_amd.simulation import DeviceSpecies, grid_struct

pytestmark = pytest.mark.gpu

KEYS = ("cell", "ox", "oy", "ux", "uy", "uz", "w")


def _sorted_both(wl, tiling, kill_every):
    grid = grid_struct(wl)
    s = wl.species[0]
    d = DeviceSpecies.from_init(grid, s, L.F32_CELLOFS)
    d.a["cell"][::kill_every] = -1              # dead particles go to the dead bin
    nt = L.lpic_num_tiles(grid, tiling)
    # reference: the workspace variant
    ref_in = {k: v.clone() for k, v in d.a.items()}
    ref = d.like()
    ref.a = ref_in
    ref_out = d.like()
    offs_ref = torch.full((nt + 2,), -7, dtype=torch.int32, device="cuda")
    wsb = L.lpic_sort_ws_bytes(grid, tiling, d.n)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    L.lpic_sort_tiles(grid, ref.struct(), ref_out.struct(), tiling, offs_ref.data_ptr(),
                      ws.data_ptr(), wsb, L.F32_CELLOFS)
    # the static variant on the same input
    out = d.like()
    offs = torch.full((nt + 2,), -7, dtype=torch.int32, device="cuda")
    L.lpic_sort_tiles_static(grid, d.struct(), out.struct(), tiling, offs.data_ptr(),
                             L.F32_CELLOFS)
    torch.cuda.synchronize()
    return nt, offs, offs_ref, out, ref_out


def test_static_sort_matches_workspace_sort_twice():
    # first call: 96 x 80 box, 8 ppc, tiles 8 x 8 (120 tiles); second: 40 x 24, 3 ppc,
    # tiles 16 x 8 (9 tiles) -- fewer particles and fewer bins than the first left behind
    cases = [(W.thermal_2d(nx=96, ny=80, ppc=8, order=2, seed=21), L.Tiling(8, 8, 1, 4, 256, 0), 97),
             (W.thermal_2d(nx=40, ny=24, ppc=3, order=1, seed=22), L.Tiling(16, 8, 1, 4, 256, 0), 13)]
    for wl, tiling, kill in cases:
        nt, offs, offs_ref, out, ref_out = _sorted_both(wl, tiling, kill)
        np.testing.assert_array_equal(offs.cpu().numpy(), offs_ref.cpu().numpy())
        o = offs.cpu().numpy().astype(np.int64)
        assert o[0] == 0 and o[nt + 1] == out.n
        # the order inside a tile comes from atomics and is not unique: every tile (and the
        # dead block) holds the same records, compared as sorted raw 32-bit rows
        ra = np.stack([out.numpy(k).view(np.int32) for k in KEYS], axis=1)
        rb = np.stack([ref_out.numpy(k).view(np.int32) for k in KEYS], axis=1)
        for b in range(nt + 1):
            x, y = ra[o[b]:o[b + 1]], rb[o[b]:o[b + 1]]
            np.testing.assert_array_equal(x[np.lexsort(x.T[::-1])], y[np.lexsort(y.T[::-1])],
                                          err_msg=f"bin {b}")
        # and every record sits in the tile of its cell
        cell = ra[:o[nt], 0]
        tx, ty = tiling.tx, tiling.ty
        ntx = (wl.nx + tx - 1) // tx
        tiles = ((cell >> 16) // ty) * ntx + (cell & 0xFFFF) // tx
        np.testing.assert_array_equal(tiles, np.repeat(np.arange(nt), np.diff(o[:nt + 1])))
        assert np.all(ra[o[nt]:, 0] < 0)


def test_static_sort_refuses_too_many_tiles():
    wl = W.Workload("tiles", 2, 4096, 2048, 1, 0.05, 0.05, 1.0, W.cfl_dt(0.95, 0.05, 0.05),
                    0.0, [])
    grid = grid_struct(wl)
    tiling = L.Tiling(4, 4, 1, 3, 256, 0)     # 524,288 tiles > LPIC_SORT_STATIC_MAX_TILES
    assert L.lpic_num_tiles(grid, tiling) > L.SORT_STATIC_MAX_TILES
    d = DeviceSpecies(2, 0, -1.0, 1.0, 1, L.F32_CELLOFS)
    offs = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(L.LpicError) as e:
        L.lpic_sort_tiles_static(grid, d.struct(), d.like().struct(), tiling, offs.data_ptr(),
                                 L.F32_CELLOFS)
    assert e.value.status == -1 and "at most" in str(e.value)   # LPIC_EINVAL
