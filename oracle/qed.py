"""The oracle's QED event Monte-Carlo (Sec. 3.4), wrapping ``qed.c``.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test suite, the smoke
entry point and the CPU-baseline leg of the benchmark may use it.  Plain FP64 C, single
threaded; shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import Fields, Grid, OracleSim, OracleSpecies, Species, _dp, _ptr, lib as _lib

_i32p = ctypes.POINTER(ctypes.c_int32)
_ready = False


class Qed(ctypes.Structure):
    _fields_ = [("hbar_omega", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("step", ctypes.c_int64)]


class QedBufStruct(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int64), ("count", ctypes.c_int64)] + \
               [(k, _dp) for k in ("x", "y", "z", "ux", "uy", "uz", "w", "tau")] + \
               [("src", _i32p)]


def lib():
    global _ready
    L = _lib()
    if not _ready:
        d, i64, u64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32
        for name, args in (("orc_bessel_k", [d, d]), ("orc_bessel_k_tail", [d, d]),
                           ("orc_compton_spectrum", [d, d]), ("orc_compton_cdf", [d, d]),
                           ("orc_compton_rate", [d]), ("orc_compton_moment", [d]),
                           ("orc_compton_sample", [d, d]), ("orc_bw_spectrum", [d, d]),
                           ("orc_bw_cdf", [d, d]), ("orc_bw_rate", [d]),
                           ("orc_bw_sample", [d, d]), ("orc_chi_lepton", [_dp, _dp, _dp, d]),
                           ("orc_chi_photon", [_dp, _dp, _dp, d]),
                           ("orc_qed_uniform", [u64, i64, i64, i32])):
            getattr(L, name).restype = d
            getattr(L, name).argtypes = args
        L.orc_splitmix64.restype = u64
        L.orc_splitmix64.argtypes = [u64, u64]
        L.orc_qed_init_tau.argtypes = [_dp, i64, u64, i64]
        L.orc_qed_gather_push.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fields),
                                          ctypes.POINTER(Species), _dp, ctypes.POINTER(Qed),
                                          ctypes.POINTER(QedBufStruct)]
        L.orc_qed_photon_push.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Fields), i32,
                                          ctypes.POINTER(QedBufStruct), ctypes.POINTER(Qed),
                                          ctypes.POINTER(QedBufStruct)]
        _ready = True
    return L


def _f(name):
    return getattr(lib(), name)


def bessel_k(nu, x):
    return _f("orc_bessel_k")(nu, x)


def bessel_k_tail(nu, x):
    return _f("orc_bessel_k_tail")(nu, x)


def compton_spectrum(chi, xi):
    return _f("orc_compton_spectrum")(chi, xi)


def compton_cdf(chi, xi):
    return _f("orc_compton_cdf")(chi, xi)


def compton_rate(chi):
    return _f("orc_compton_rate")(chi)


def compton_moment(chi):
    return _f("orc_compton_moment")(chi)


def compton_sample(chi, r):
    return _f("orc_compton_sample")(chi, r)


def bw_spectrum(chi, xi):
    return _f("orc_bw_spectrum")(chi, xi)


def bw_cdf(chi, xi):
    return _f("orc_bw_cdf")(chi, xi)


def bw_rate(chi):
    return _f("orc_bw_rate")(chi)


def bw_sample(chi, r):
    return _f("orc_bw_sample")(chi, r)


def _vec(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def chi_lepton(u, E, B, hbar_omega):
    u, E, B = _vec(u), _vec(E), _vec(B)
    return _f("orc_chi_lepton")(_ptr(u), _ptr(E), _ptr(B), hbar_omega)


def chi_photon(k, E, B, hbar_omega):
    k, E, B = _vec(k), _vec(E), _vec(B)
    return _f("orc_chi_photon")(_ptr(k), _ptr(E), _ptr(B), hbar_omega)


def splitmix64(seed, k):
    return _f("orc_splitmix64")(seed, k)


def uniform(seed, step, slot, draw):
    return _f("orc_qed_uniform")(seed, step, slot, draw)


def init_tau(n, seed, step):
    tau = np.zeros(n)
    lib().orc_qed_init_tau(_ptr(tau), n, seed, step)
    return tau


class QedBuf:
    """Event records (photons, or leptons from pairs) as FP64 arrays with a count."""

    KEYS = ("x", "y", "z", "ux", "uy", "uz", "w", "tau")

    def __init__(self, capacity, count=0):
        self.capacity, self.count = int(capacity), int(count)
        for k in self.KEYS:
            setattr(self, k, np.zeros(self.capacity))
        self.src = np.zeros(self.capacity, dtype=np.int32)

    def struct(self):
        return QedBufStruct(self.capacity, self.count, *(_ptr(getattr(self, k)) for k in self.KEYS),
                            self.src.ctypes.data_as(_i32p))

    def valid(self):
        return min(self.count, self.capacity)


def qed_gather_push(sim: OracleSim, s: OracleSpecies, tau, hbar_omega, seed, step,
                    photons: QedBuf):
    assert tau.dtype == np.float64 and tau.flags.c_contiguous and tau.shape[0] == s.n
    fs = sim.fields_struct()
    st = s.struct()
    q = Qed(hbar_omega, seed, step)
    b = photons.struct()
    lib().orc_qed_gather_push(ctypes.byref(sim.grid), ctypes.byref(fs), ctypes.byref(st),
                              _ptr(tau), ctypes.byref(q), ctypes.byref(b))
    photons.count = b.count


def qed_photon_push(sim: OracleSim, order, photons: QedBuf, hbar_omega, seed, step,
                    pairs: QedBuf):
    fs = sim.fields_struct()
    q = Qed(hbar_omega, seed, step)
    b, pb = photons.struct(), pairs.struct()
    lib().orc_qed_photon_push(ctypes.byref(sim.grid), ctypes.byref(fs), order, ctypes.byref(b),
                              ctypes.byref(q), ctypes.byref(pb))
    pairs.count = pb.count
