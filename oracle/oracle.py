"""ctypes wrapper around the CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may use this module; the product package never imports it.
The oracle follows the paper's method step by step (Eq. 1-3, Sec. 3.1, 3.3
and 4); see rfim_oracle.c for the conventions it fixes.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = [os.path.join(_HERE, "rfim_oracle.c")]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C99, no contraction)."""
    import subprocess

    if not force and os.path.exists(LIB_PATH):
        newest = max(os.path.getmtime(p) for p in SOURCES + [os.path.join(_HERE, "rfim_oracle.h")])
        if os.path.getmtime(LIB_PATH) >= newest:
            return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-o", tmp] + SOURCES + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def timed_build(out_dir: str) -> str:
    """The same source built for timing on this host (-O3 -march=native,
    still -ffp-contract=off) into out_dir; the tested library is left as it
    is.  Returns the path of the build."""
    import subprocess

    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, "liboracle_native.so")
    tmp = path + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c99", "-O3", "-march=native", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-o", tmp] + SOURCES + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, path)
    return path


_lib = None
_lib_path = None


def use_library(path: str) -> None:
    """Load the oracle from `path` (a timed_build) instead of the tested
    build; call before the first Oracle is made."""
    global _lib, _lib_path
    _lib = None
    _lib_path = path


def lib():
    global _lib
    if _lib is None:
        if _lib_path is None:
            build()
        L = C.CDLL(_lib_path or LIB_PATH)
        vp, i32, i64, u32, u64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
        L.orc_create.restype = vp
        L.orc_create.argtypes = [i32, i32, dbl, dbl, vp, vp, u64, u32, i32, i32]
        L.orc_destroy.argtypes = [vp]
        L.orc_destroy.restype = None
        L.orc_last_error.restype = C.c_char_p
        for name in ("orc_num_replicas", "orc_field_kind"):
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = i32
        L.orc_sweep.argtypes = [vp, i64, i32]
        for name in ("orc_energies", "orc_magnetizations", "orc_temps", "orc_get_spins",
                     "orc_set_spins", "orc_get_perm", "orc_set_perm", "orc_reset_exchange_stats",
                     "orc_exchange_once"):
            getattr(L, name).restype = i32
        for name in ("orc_energies", "orc_magnetizations", "orc_temps", "orc_get_spins",
                     "orc_set_spins", "orc_get_perm", "orc_set_perm"):
            getattr(L, name).argtypes = [vp, vp]
        L.orc_reset_exchange_stats.argtypes = [vp]
        L.orc_exchange_once.argtypes = [vp]
        L.orc_components.argtypes = [vp, vp, vp, vp]
        L.orc_get_counters.argtypes = [vp, vp, vp]
        L.orc_set_counters.argtypes = [vp, u64, u64]
        L.orc_exchange_stats.argtypes = [vp, vp, vp]
        L.orc_flip_delta.argtypes = [vp, i32, i32]
        L.orc_flip_delta.restype = dbl
        L.orc_accept.argtypes = [vp, i32, i32, u32]
        L.orc_accept.restype = i32
        L.orc_fourier.argtypes = [vp, vp]
        L.orc_fourier.restype = i32
        L.orc_thresholds.argtypes = [vp, vp, vp]
        L.orc_adapt_temps.argtypes = [vp, i32, i64, i32, dbl, i32, i32]
        L.orc_adapt_temps.restype = i32
        L.orc_insert_step.argtypes = [vp, dbl, i32, i32]
        L.orc_insert_step.restype = i32
        L.orc_set_update_order.argtypes = [vp, i32, i32, i32, i32, i32]
        L.orc_set_update_order.restype = i32
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_philox4x32_10.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


class Oracle:
    """One disorder realization with R temperature replicas, on the CPU."""

    def __init__(self, L, R, J, h, fields, temps, seed=0, realization=0, field_kind=-1, R_cap=0):
        self.L = int(L)
        self.N = self.L ** 3
        f = np.ascontiguousarray(fields, dtype=np.float32).reshape(-1)
        T = np.ascontiguousarray(temps, dtype=np.float64).reshape(-1)
        if f.size != self.N or T.size != int(R):
            raise ValueError("fields must hold L^3 values and temps R values")
        self._h = lib().orc_create(self.L, int(R), float(J), float(h), _p(f), _p(T),
                                   int(seed) & 0xFFFFFFFFFFFFFFFF, int(realization), int(field_kind),
                                   int(R_cap))
        if not self._h:
            raise ValueError(lib().orc_last_error().decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    __del__ = close

    @property
    def R(self) -> int:
        return lib().orc_num_replicas(self._h)

    @property
    def field_kind(self) -> int:
        return lib().orc_field_kind(self._h)

    def _check(self, rc):
        if rc < 0:
            raise RuntimeError(lib().orc_last_error().decode())
        return rc

    def set_update_order(self, order, tiles=(0, 0, 0), hits=1):
        """order 0: plain checkerboard; order 1: double checkerboard of
        tiles (tx, ty, tz) with `hits` local sweeps per tile visit."""
        self._check(lib().orc_set_update_order(self._h, int(order), *[int(t) for t in tiles], int(hits)))

    def sweep(self, n, every=0):
        self._check(lib().orc_sweep(self._h, int(n), int(every)))

    def energies(self) -> np.ndarray:
        E = np.zeros(self.R, dtype=np.float64)
        lib().orc_energies(self._h, _p(E))
        return E

    def magnetizations(self) -> np.ndarray:
        M = np.zeros(self.R, dtype=np.int64)
        lib().orc_magnetizations(self._h, _p(M))
        return M

    def temps(self) -> np.ndarray:
        T = np.zeros(self.R, dtype=np.float64)
        lib().orc_temps(self._h, _p(T))
        return T

    def components(self):
        R = self.R
        B = np.zeros(R, dtype=np.int64)
        F = np.zeros(R, dtype=np.float64)
        M = np.zeros(R, dtype=np.int64)
        lib().orc_components(self._h, _p(B), _p(F), _p(M))
        return B, F, M

    def spins(self) -> np.ndarray:
        s = np.zeros((self.R, self.N), dtype=np.int8)
        lib().orc_get_spins(self._h, _p(s))
        return s

    def set_spins(self, s):
        a = np.ascontiguousarray(s, dtype=np.int8).reshape(self.R, self.N)
        self._check(lib().orc_set_spins(self._h, _p(a)))

    def perm(self) -> np.ndarray:
        p = np.zeros(self.R, dtype=np.int32)
        lib().orc_get_perm(self._h, _p(p))
        return p

    def set_perm(self, t2r):
        a = np.ascontiguousarray(t2r, dtype=np.int32)
        self._check(lib().orc_set_perm(self._h, _p(a)))

    def counters(self):
        t = C.c_uint64()
        k = C.c_uint64()
        lib().orc_get_counters(self._h, C.byref(t), C.byref(k))
        return t.value, k.value

    def set_counters(self, t, k):
        lib().orc_set_counters(self._h, int(t), int(k))

    def exchange_stats(self):
        n = max(self.R - 1, 0)
        att = np.zeros(max(n, 1), dtype=np.uint64)
        acc = np.zeros(max(n, 1), dtype=np.uint64)
        lib().orc_exchange_stats(self._h, _p(att), _p(acc))
        return att[:n], acc[:n]

    def reset_exchange_stats(self):
        lib().orc_reset_exchange_stats(self._h)

    def exchange_once(self):
        lib().orc_exchange_once(self._h)

    def flip_delta(self, r, i) -> float:
        return lib().orc_flip_delta(self._h, int(r), int(i))

    def fourier(self) -> np.ndarray:
        """F of the correlation length for the configuration at every slot."""
        F = np.zeros(self.R, dtype=np.float64)
        self._check(lib().orc_fourier(self._h, _p(F)))
        return F

    def accept(self, r, i, u) -> bool:
        """The sweep's decision for site i of replica r with word u."""
        return bool(self._check(lib().orc_accept(self._h, int(r), int(i), int(u) & 0xFFFFFFFF)))

    def thresholds(self):
        thr = np.zeros((self.R, 14), dtype=np.uint32)
        always = np.zeros(14, dtype=np.uint8)
        lib().orc_thresholds(self._h, _p(thr), _p(always))
        return thr, always.astype(bool)

    def insert_step(self, rate_threshold, max_insert, R_cap):
        return self._check(lib().orc_insert_step(self._h, float(rate_threshold), int(max_insert), int(R_cap)))

    def adapt_temps(self, trials, sweeps_per_trial, every, rate_threshold, max_insert_per_trial, R_cap):
        return self._check(lib().orc_adapt_temps(self._h, int(trials), int(sweeps_per_trial), int(every),
                                                 float(rate_threshold), int(max_insert_per_trial),
                                                 int(R_cap)))
