"""The C-ABI library loads on a machine without a GPU and exports every symbol that
include/lpic.h declares (no compute calls here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lpic.h")
SO = os.path.join(ROOT, "paper_2607_13507_amd", "liblpic.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(lpic_[a-z0-9_A-Z]+)\s*\(", text)
    return sorted(set(n for n in names if n != "lpic_hook_fn"))


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (bind to torch's HIP runtime, as the binding does)
    if not os.path.exists(SO):
        from paper_2607_13507_amd import build
        build.build()
    return ctypes.CDLL(SO)


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ("lpic_gather_push", "lpic_deposit_esirkepov", "lpic_yee_update_EB",
              "lpic_sort_tiles", "lpic_step"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_exports_are_plain_c(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", SO], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    for n in declared_functions():
        assert n in exported, n          # unmangled C names


def test_binding_covers_the_header():
    from paper_2607_13507_amd import lpic
    assert set(declared_functions()) <= set(lpic.EXPORTS)


def test_error_path_without_gpu(lib):
    """Argument validation happens on the host, before any GPU call."""
    from paper_2607_13507_amd import lpic as L
    L.lib()
    g = L.Grid(2, 16, 16, 1, 0.1, 0.1, 1.0, 1.0, 0.0)     # dt far above the CFL limit
    f = L.Fields(*([1] * 9), None, None)
    with pytest.raises(L.LpicError) as e:
        L.lpic_yee_update_EB(g, f, 0, 0.5, 0, L.F32_CELLOFS, stream=0)
    assert e.value.status == -1 and "CFL" in str(e.value)
    g = L.Grid(4, 16, 16, 1, 0.1, 0.1, 1.0, 0.05, 0.0)
    with pytest.raises(L.LpicError):
        L.lpic_yee_update_EB(g, f, 0, 0.5, 0, L.F32_CELLOFS, stream=0)
    g = L.Grid(2, 16, 16, 1, 0.1, 0.1, 1.0, 0.05, 0.0)
    s = L.Species(10, -1.0, 1.0, 3, 0, *([1] * 11))
    with pytest.raises(L.LpicError) as e:
        L.lpic_gather_push(g, f, s, 1, 1 << 20, L.F32_CELLOFS, stream=0)
    assert "shape_order" in str(e.value)
    t = L.Tiling(12, 16, 1, 4, 256, 0)
    assert L.lpic_num_tiles(g, L.Tiling(8, 8, 1, 4, 256, 0)) == 4
    s = L.Species(10, -1.0, 1.0, 2, 0, *([1] * 11))
    with pytest.raises(L.LpicError) as e:
        L.lpic_sort_tiles(g, s, s, t, 1, 1, 1 << 20, L.F32_CELLOFS, stream=0)
    assert "power" in str(e.value)
    t = L.Tiling(16, 16, 1, 4, 256, 8)   # no such flag
    with pytest.raises(L.LpicError) as e:
        L.lpic_sort_tiles(g, s, s, t, 1, 1, 1 << 20, L.F32_CELLOFS, stream=0)
    assert "flags" in str(e.value)
    # the defined flags pass the tiling check (the call then stops at the workspace size)
    t = L.Tiling(16, 16, 1, 4, 256, L.SORT_SPREAD | L.FIELD_SEPARATE | L.ESCAPE_REBIN)
    with pytest.raises(L.LpicError) as e:
        L.lpic_sort_tiles(g, s, s, t, 1, 1, 0, L.F32_CELLOFS, stream=0)
    assert "workspace" in str(e.value)
    # the single fused call takes no charge mode but none (0) and both ends (1)
    t = L.Tiling(16, 16, 1, 4, 256, 0)
    for mode in (2, 3, -1):
        with pytest.raises(L.LpicError) as e:
            L.lpic_push_deposit_fused(g, f, s, t, 1, 1, 1 << 20, mode, None, L.F32_CELLOFS,
                                      stream=0)
        assert "with_rho" in str(e.value)
