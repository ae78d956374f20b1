"""ctypes binding of liblpic.so (include/lpic.h): argument marshalling only.

Every function here has the name of the C entry point it calls, converts Python/torch
arguments into the C structs, and raises LpicError with the library's message when the
status is not LPIC_OK.  All arithmetic of the hot path happens in the HIP library; if the
library is missing, loading fails loudly (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblpic.so")

F32_CELLOFS = 0
F64_ABS = 1
YEE_ZERO_J = 1
SORT_SPREAD = 1
FIELD_SEPARATE = 2
ESCAPE_REBIN = 4

STAGES = ["START", "LOOP_START", "MAXWELL_1", "PUSH_POSITION_1", "INTERPOLATOR",
          "PUSH_MOMENTUM", "PUSH_POSITION_2", "CURRENT_DEPOSITION", "QED_CREATE",
          "MAXWELL_2", "LOOP_END", "FINISH"]
STAGE = {name: i for i, name in enumerate(STAGES)}

STATUS = {0: "LPIC_OK", -1: "LPIC_EINVAL", -2: "LPIC_EHIP", -3: "LPIC_ENOMEM",
          -4: "LPIC_EUNSUPPORTED", -5: "LPIC_EHOOK", -6: "LPIC_ENUMERIC"}

_vp = ctypes.c_void_p


OPEN_MARGIN = 3   # LPIC_OPEN_MARGIN


class Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("dz", ctypes.c_double), ("dt", ctypes.c_double), ("rho_bg", ctypes.c_double),
                ("open_x", ctypes.c_int32), ("reserved0", ctypes.c_int32)]


class Laser(ctypes.Structure):
    _fields_ = [("pol", ctypes.c_int32), ("ia", ctypes.c_int32), ("a0", ctypes.c_double),
                ("omega", ctypes.c_double), ("waist", ctypes.c_double), ("yc", ctypes.c_double),
                ("zc", ctypes.c_double), ("t0", ctypes.c_double), ("tau", ctypes.c_double)]


class Plasma(ctypes.Structure):
    _fields_ = [("species", ctypes.c_int32), ("ppc_x", ctypes.c_int32), ("ppc_y", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("density", ctypes.c_double),
                ("ux", ctypes.c_double), ("uy", ctypes.c_double), ("uz", ctypes.c_double)]


class Pml(ctypes.Structure):
    _fields_ = [("cells", ctypes.c_int32), ("order", ctypes.c_int32),
                ("a_order", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("sigma_max", ctypes.c_double), ("kappa_max", ctypes.c_double),
                ("a_max", ctypes.c_double)]


class Fields(ctypes.Structure):
    _fields_ = [(n, _vp) for n in ("ex", "ey", "ez", "bx", "by", "bz", "jx", "jy", "jz",
                                   "rho0", "rho1")]


class Species(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("q", ctypes.c_double), ("m", ctypes.c_double),
                ("shape_order", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("cell", _vp), ("ox", _vp), ("oy", _vp), ("oz", _vp),
                ("x", _vp), ("y", _vp), ("z", _vp),
                ("ux", _vp), ("uy", _vp), ("uz", _vp), ("w", _vp)]


class Tiling(ctypes.Structure):
    _fields_ = [("tx", ctypes.c_int32), ("ty", ctypes.c_int32), ("tz", ctypes.c_int32),
                ("halo", ctypes.c_int32), ("chunk", ctypes.c_int32), ("flags", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("tiling", Tiling), ("sort_interval", ctypes.c_int32),
                ("diag_interval", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("reserved0", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("sorts", ctypes.c_int64), ("fused", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("fused_ms", ctypes.c_double),
                ("fused_launches", ctypes.c_int64), ("halo_escapes", ctypes.c_int64),
                ("field_tile", ctypes.c_int32 * 2)]


TUNE_MAX_TRIALS = 64


class TuneSpace(ctypes.Structure):
    _fields_ = [("tile_min", ctypes.c_int32 * 3), ("tile_max", ctypes.c_int32 * 3),
                ("halo_min", ctypes.c_int32), ("halo_max", ctypes.c_int32),
                ("chunk_min", ctypes.c_int32), ("chunk_max", ctypes.c_int32),
                ("sort_min", ctypes.c_int32), ("sort_max", ctypes.c_int32),
                ("rebin", ctypes.c_int32), ("steps_each", ctypes.c_int32),
                ("max_trials", ctypes.c_int32)]


class TuneReport(ctypes.Structure):
    _fields_ = [("ntrials", ctypes.c_int32), ("best", ctypes.c_int32),
                ("trial", Options * TUNE_MAX_TRIALS),
                ("ms_per_step", ctypes.c_double * TUNE_MAX_TRIALS)]


HOOK_FN = ctypes.CFUNCTYPE(ctypes.c_int, _vp, ctypes.c_int32, ctypes.c_int64, _vp)


class QedParams(ctypes.Structure):
    _fields_ = [("hbar_omega", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("step", ctypes.c_int64)]


class QedBuffer(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int64), ("count", _vp)] + \
               [(k, _vp) for k in ("x", "y", "z", "ux", "uy", "uz", "w", "tau")] + [("src", _vp)]


QED_EMIT_RATE, QED_EMIT_SAMPLE, QED_PAIR_RATE, QED_PAIR_SAMPLE = 0, 1, 2, 3


class LpicError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn}: {STATUS.get(status, status)}: {msg}")
        self.status = status


EXPORTS = {
    # name: (restype, argtypes)
    "lpic_last_error": (ctypes.c_char_p, []),
    "lpic_version": (ctypes.c_char_p, []),
    "lpic_yee_update_EB": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Fields),
                                          ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                          ctypes.c_int, _vp]),
    "lpic_old_state_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int]),
    "lpic_gather_push": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Fields),
                                        ctypes.POINTER(Species), _vp, ctypes.c_size_t,
                                        ctypes.c_int, _vp]),
    "lpic_deposit_esirkepov": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Fields),
                                              ctypes.POINTER(Species), _vp, ctypes.c_size_t,
                                              ctypes.c_int32, ctypes.c_int, _vp]),
    "lpic_sort_ws_bytes": (ctypes.c_size_t, [ctypes.POINTER(Grid), ctypes.POINTER(Tiling),
                                             ctypes.c_int64]),
    "lpic_num_tiles": (ctypes.c_int64, [ctypes.POINTER(Grid), ctypes.POINTER(Tiling)]),
    "lpic_sort_tiles": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Species),
                                       ctypes.POINTER(Species), ctypes.POINTER(Tiling), _vp,
                                       _vp, ctypes.c_size_t, ctypes.c_int, _vp]),
    "lpic_sort_tiles_static": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Species),
                                              ctypes.POINTER(Species), ctypes.POINTER(Tiling),
                                              _vp, ctypes.c_int, _vp]),
    "lpic_fused_ws_bytes": (ctypes.c_size_t, [ctypes.POINTER(Grid), ctypes.POINTER(Tiling),
                                              ctypes.c_int64]),
    "lpic_push_deposit_fused": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Fields),
                                               ctypes.POINTER(Species), ctypes.POINTER(Tiling),
                                               _vp, _vp, ctypes.c_size_t, ctypes.c_int32, _vp,
                                               ctypes.c_int, _vp]),
    "lpic_load_positions": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Species), _vp,
                                           _vp, _vp, ctypes.c_int, _vp]),
    "lpic_store_positions": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Species), _vp,
                                            _vp, _vp, ctypes.c_int, _vp]),
    "lpic_reduce_fields": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Fields),
                                          ctypes.c_int32, _vp, ctypes.c_int, _vp]),
    "lpic_laser_source": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Fields),
                                         ctypes.POINTER(Laser), ctypes.c_double, ctypes.c_int,
                                         _vp]),
    "lpic_set_laser": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(Laser)]),
    "lpic_set_pml": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(Pml)]),
    "lpic_window_shift": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(Plasma)]),
    "lpic_window_info": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64)]),
    "lpic_sim_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.POINTER(Grid),
                                       ctypes.POINTER(Fields), ctypes.c_int32,
                                       ctypes.POINTER(Species), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(Species), ctypes.c_int,
                                       ctypes.POINTER(Options), _vp]),
    "lpic_sim_destroy": (None, [_vp]),
    "lpic_step": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "lpic_register_hook": (ctypes.c_int, [_vp, ctypes.c_int32, HOOK_FN, _vp]),
    "lpic_clear_hooks": (ctypes.c_int, [_vp]),
    "lpic_get_species": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(Species)]),
    "lpic_get_stats": (ctypes.c_int, [_vp, ctypes.POINTER(Stats)]),
    "lpic_get_diagnostics": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "lpic_set_timing": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "lpic_set_options": (ctypes.c_int, [_vp, ctypes.POINTER(Options)]),
    "lpic_autotune": (ctypes.c_int, [_vp, ctypes.POINTER(Options), ctypes.c_int32, ctypes.c_int32,
                                     ctypes.POINTER(Options)]),
    "lpic_autotune_search": (ctypes.c_int, [_vp, ctypes.POINTER(TuneSpace),
                                            ctypes.POINTER(Options), ctypes.POINTER(TuneReport)]),
    "lpic_qed_tables_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_vp)]),
    "lpic_qed_tables_destroy": (ctypes.c_int, [_vp]),
    "lpic_qed_table_eval": (ctypes.c_double, [_vp, ctypes.c_int32, ctypes.c_double,
                                              ctypes.c_double]),
    "lpic_qed_init_tau": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int64,
                                         _vp]),
    "lpic_qed_gather_push": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Fields),
                                            ctypes.POINTER(Species), _vp, _vp,
                                            ctypes.POINTER(QedParams), ctypes.POINTER(QedBuffer),
                                            _vp, ctypes.c_size_t, ctypes.c_int, _vp]),
    "lpic_qed_compact_ws_bytes": (ctypes.c_size_t, [ctypes.c_int64]),
    "lpic_qed_compact": (ctypes.c_int, [ctypes.POINTER(QedBuffer), ctypes.POINTER(QedBuffer),
                                        ctypes.c_int32, _vp, ctypes.c_size_t, _vp]),
    "lpic_qed_insert": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Species),
                                       ctypes.c_int64, ctypes.POINTER(QedBuffer), ctypes.c_int32,
                                       _vp, ctypes.c_int, _vp]),
    "lpic_qed_photon_push": (ctypes.c_int, [ctypes.POINTER(Grid), ctypes.POINTER(Fields),
                                            ctypes.c_int32, ctypes.POINTER(QedBuffer), _vp,
                                            ctypes.POINTER(QedParams), ctypes.POINTER(QedBuffer),
                                            ctypes.c_int, _vp]),
}

_lib = None


def lib():
    """Load liblpic.so (built in-tree by __graft_entry__.build()); no fallback."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime with the same soname as /opt/rocm's; importing it
        # first makes liblpic.so bind to that one, so the process holds a single runtime
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(fn, status):
    if status != 0:
        msg = lib().lpic_last_error().decode(errors="replace")
        raise LpicError(fn, status, msg)


def ptr(t):
    """Device address of a tensor (None for None)."""
    return None if t is None else t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream


# ------------------------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ------------------------------------------------------------------------------------------
def lpic_version():
    return lib().lpic_version().decode()


def lpic_yee_update_EB(grid, fields, which, frac, flags, prec, stream=None):
    _check("lpic_yee_update_EB", lib().lpic_yee_update_EB(ctypes.byref(grid), ctypes.byref(fields),
                                                          which, frac, flags, prec, _stream(stream)))


def lpic_old_state_bytes(ndim, n, prec):
    return lib().lpic_old_state_bytes(ndim, n, prec)


def lpic_gather_push(grid, fields, species, old_state, old_bytes, prec, stream=None):
    _check("lpic_gather_push", lib().lpic_gather_push(ctypes.byref(grid), ctypes.byref(fields),
                                                      ctypes.byref(species), old_state, old_bytes,
                                                      prec, _stream(stream)))


def lpic_deposit_esirkepov(grid, fields, species, old_state, old_bytes, with_rho, prec,
                           stream=None):
    _check("lpic_deposit_esirkepov",
           lib().lpic_deposit_esirkepov(ctypes.byref(grid), ctypes.byref(fields),
                                        ctypes.byref(species), old_state, old_bytes, with_rho,
                                        prec, _stream(stream)))


def lpic_sort_ws_bytes(grid, tiling, n):
    return lib().lpic_sort_ws_bytes(ctypes.byref(grid), ctypes.byref(tiling), n)


def lpic_num_tiles(grid, tiling):
    return lib().lpic_num_tiles(ctypes.byref(grid), ctypes.byref(tiling))


def lpic_sort_tiles(grid, species, alt, tiling, tile_offsets, ws, ws_bytes, prec, stream=None):
    """Sorts `species` into `alt`'s arrays, then swaps the two structs' array pointers."""
    _check("lpic_sort_tiles", lib().lpic_sort_tiles(ctypes.byref(grid), ctypes.byref(species),
                                                    ctypes.byref(alt), ctypes.byref(tiling),
                                                    tile_offsets, ws, ws_bytes, prec,
                                                    _stream(stream)))


SORT_STATIC_MAX_TILES = 262144   # LPIC_SORT_STATIC_MAX_TILES


def lpic_sort_tiles_static(grid, species, alt, tiling, tile_offsets, prec, stream=None):
    """lpic_sort_tiles with the library's own static scratch (allocates nothing)."""
    _check("lpic_sort_tiles_static",
           lib().lpic_sort_tiles_static(ctypes.byref(grid), ctypes.byref(species),
                                        ctypes.byref(alt), ctypes.byref(tiling), tile_offsets,
                                        prec, _stream(stream)))


def lpic_fused_ws_bytes(grid, tiling, n):
    return lib().lpic_fused_ws_bytes(ctypes.byref(grid), ctypes.byref(tiling), n)


def lpic_push_deposit_fused(grid, fields, species, tiling, tile_offsets, ws, ws_bytes, with_rho,
                            kinetic, prec, stream=None):
    _check("lpic_push_deposit_fused",
           lib().lpic_push_deposit_fused(ctypes.byref(grid), ctypes.byref(fields),
                                         ctypes.byref(species), ctypes.byref(tiling),
                                         tile_offsets, ws, ws_bytes, with_rho, kinetic, prec,
                                         _stream(stream)))


def lpic_load_positions(grid, species, x, y, z, prec, stream=None):
    _check("lpic_load_positions", lib().lpic_load_positions(ctypes.byref(grid),
                                                            ctypes.byref(species), x, y, z, prec,
                                                            _stream(stream)))


def lpic_store_positions(grid, species, x, y, z, prec, stream=None):
    _check("lpic_store_positions", lib().lpic_store_positions(ctypes.byref(grid),
                                                              ctypes.byref(species), x, y, z,
                                                              prec, _stream(stream)))


def lpic_reduce_fields(grid, fields, with_rho, out, prec, stream=None):
    _check("lpic_reduce_fields", lib().lpic_reduce_fields(ctypes.byref(grid), ctypes.byref(fields),
                                                          with_rho, out, prec, _stream(stream)))


def lpic_laser_source(grid, fields, laser, t, prec, stream=None):
    _check("lpic_laser_source", lib().lpic_laser_source(ctypes.byref(grid), ctypes.byref(fields),
                                                        ctypes.byref(laser), float(t), prec,
                                                        _stream(stream)))


def lpic_set_laser(h, r, laser):
    """laser: a Laser struct, or None to remove the run's antenna."""
    _check("lpic_set_laser", lib().lpic_set_laser(h, r, ctypes.byref(laser) if laser else None))


def lpic_set_pml(h, r, pml):
    """pml: a Pml struct for run r's open x ends, or None for the Mur condition."""
    _check("lpic_set_pml", lib().lpic_set_pml(h, r, ctypes.byref(pml) if pml else None))


def lpic_window_shift(h, r, m, plasma=None):
    """Move box r's window by m cells (plasma: a Plasma struct for the fresh columns, or
    None)."""
    _check("lpic_window_shift",
           lib().lpic_window_shift(h, r, m, ctypes.byref(plasma) if plasma else None))


def lpic_window_info(h, r):
    """(cells moved so far, fresh particles dropped for lack of slots)"""
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check("lpic_window_info", lib().lpic_window_info(h, r, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def lpic_sim_create(grids, fields, species, species_run, species_alt, prec, options, stream=None):
    h = _vp()
    nr, ns = len(grids), len(species)
    G = (Grid * nr)(*grids)
    F = (Fields * nr)(*fields)
    S = (Species * max(1, ns))(*species)
    A = (Species * max(1, ns))(*species_alt)
    R = (ctypes.c_int32 * max(1, ns))(*species_run)
    _check("lpic_sim_create", lib().lpic_sim_create(ctypes.byref(h), nr, G, F, ns, S, R, A, prec,
                                                    ctypes.byref(options), _stream(stream)))
    return h


def lpic_sim_destroy(h):
    lib().lpic_sim_destroy(h)


def lpic_step(h, nsteps):
    _check("lpic_step", lib().lpic_step(h, nsteps))


def lpic_register_hook(h, stage, fn, user=None):
    _check("lpic_register_hook", lib().lpic_register_hook(h, stage, fn, user))


def lpic_clear_hooks(h):
    _check("lpic_clear_hooks", lib().lpic_clear_hooks(h))


def lpic_get_species(h, i):
    out = Species()
    _check("lpic_get_species", lib().lpic_get_species(h, i, ctypes.byref(out)))
    return out


def lpic_get_stats(h):
    out = Stats()
    _check("lpic_get_stats", lib().lpic_get_stats(h, ctypes.byref(out)))
    return out


def lpic_get_diagnostics(h, r):
    out = (ctypes.c_double * 5)()
    _check("lpic_get_diagnostics", lib().lpic_get_diagnostics(h, r, out))
    return list(out)


def lpic_set_timing(h, on):
    _check("lpic_set_timing", lib().lpic_set_timing(h, int(on)))


def lpic_set_options(h, options):
    _check("lpic_set_options", lib().lpic_set_options(h, ctypes.byref(options)))


def lpic_autotune(h, candidates, steps_each):
    arr = (Options * len(candidates))(*candidates)
    best = Options()
    _check("lpic_autotune", lib().lpic_autotune(h, arr, len(candidates), steps_each,
                                                ctypes.byref(best)))
    return best


def lpic_autotune_search(h, space):
    best = Options()
    rep = TuneReport()
    _check("lpic_autotune_search", lib().lpic_autotune_search(h, ctypes.byref(space),
                                                              ctypes.byref(best),
                                                              ctypes.byref(rep)))
    return best, rep


# QED event Monte-Carlo (Sec. 3.4)
def lpic_qed_tables_create(on_device=1):
    h = _vp()
    _check("lpic_qed_tables_create", lib().lpic_qed_tables_create(on_device, ctypes.byref(h)))
    return h.value


def lpic_qed_tables_destroy(h):
    _check("lpic_qed_tables_destroy", lib().lpic_qed_tables_destroy(h))


def lpic_qed_table_eval(h, what, chi, r=0.5):
    return lib().lpic_qed_table_eval(h, what, chi, r)


def lpic_qed_init_tau(tau, n, seed, step, stream=None):
    _check("lpic_qed_init_tau", lib().lpic_qed_init_tau(tau, n, seed, step, _stream(stream)))


def lpic_qed_gather_push(grid, fields, species, tau, tables, params, photons, old_state,
                         old_bytes, prec, stream=None):
    _check("lpic_qed_gather_push",
           lib().lpic_qed_gather_push(ctypes.byref(grid), ctypes.byref(fields),
                                      ctypes.byref(species), tau, tables, ctypes.byref(params),
                                      ctypes.byref(photons), old_state, old_bytes, prec,
                                      _stream(stream)))


def lpic_qed_photon_push(grid, fields, order, photons, tables, params, pairs, prec,
                         stream=None):
    _check("lpic_qed_photon_push",
           lib().lpic_qed_photon_push(ctypes.byref(grid), ctypes.byref(fields), order,
                                      ctypes.byref(photons), tables, ctypes.byref(params),
                                      ctypes.byref(pairs), prec, _stream(stream)))


def lpic_qed_insert(grid, species, first, records, parity, dropped, prec, stream=None):
    _check("lpic_qed_insert",
           lib().lpic_qed_insert(ctypes.byref(grid), ctypes.byref(species), first,
                                 ctypes.byref(records), parity, dropped, prec, _stream(stream)))


def lpic_qed_compact_ws_bytes(capacity):
    return lib().lpic_qed_compact_ws_bytes(capacity)


def lpic_qed_compact(inp, out, ndim, ws, ws_bytes, stream=None):
    _check("lpic_qed_compact",
           lib().lpic_qed_compact(ctypes.byref(inp), ctypes.byref(out), ndim, ws, ws_bytes,
                                  _stream(stream)))
