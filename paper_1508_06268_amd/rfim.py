"""Thin ctypes binding of librfim.so: the C ABI of include/rfim.h under the
same names, plus a small ``Rfim`` handle class.  Argument marshalling only;
every step of the method runs in the library's HIP kernels.

PyTorch supplies the HIP runtime and streams: it is imported before the
library is opened so that both share one runtime, and ``Rfim`` issues its
work on a ``torch.cuda`` stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librfim.so")

RFIM_OK, RFIM_EINVAL, RFIM_ENOMEM, RFIM_EDEVICE, RFIM_ESTATE, RFIM_ECAP, RFIM_EBUSY = 0, -1, -2, -3, -4, -5, -6
FIELDS_AUTO, FIELDS_BIMODAL, FIELDS_CONTINUOUS = -1, 0, 1
MEASURE_FOURIER = 1
# Batch and pool class shape (MODE_BITS, 0, 0): one bit per spin (L = 64, 128, 256)
MODE_BITS = 5

# Every symbol include/rfim.h declares (checked by the CPU tests).
EXPORTS = [
    "rfim_create", "rfim_create_ex", "rfim_sweep", "rfim_energies", "rfim_adapt_temps",
    "rfim_destroy", "rfim_last_error", "rfim_set_stream", "rfim_synchronize",
    "rfim_num_replicas", "rfim_lattice_size", "rfim_field_kind", "rfim_temps",
    "rfim_magnetizations", "rfim_components", "rfim_get_spins", "rfim_set_spins",
    "rfim_get_perm", "rfim_set_perm", "rfim_get_counters", "rfim_set_counters",
    "rfim_exchange_stats", "rfim_reset_exchange_stats", "rfim_save", "rfim_load",
    "rfim_set_launch_shape", "rfim_get_launch_shape", "rfim_set_concurrency", "rfim_get_concurrency",
    "rfim_observables", "rfim_reset_observables", "rfim_set_measure", "rfim_fourier",
    "rfim_batch_create", "rfim_batch_destroy", "rfim_batch_size", "rfim_batch_sweep",
    "rfim_batch_synchronize", "rfim_batch_item", "rfim_batch_set_shape", "rfim_batch_set_group_bytes",
    "rfim_batch_get_group_bytes",
    "rfim_pool_create", "rfim_pool_destroy", "rfim_pool_bytes_needed", "rfim_pool_admit",
    "rfim_pool_admit_job", "rfim_pool_step", "rfim_pool_poll", "rfim_pool_result",
    "rfim_pool_adapt", "rfim_pool_release", "rfim_pool_item",
    "rfim_pool_active", "rfim_pool_reserved", "rfim_pool_set_shape", "rfim_pool_synchronize",
    "rfim_energies_noalloc", "rfim_set_update_order", "rfim_get_update_order",
    "rfim_set_spin_storage", "rfim_get_spin_storage",
]
ORDER_CHECKERBOARD, ORDER_TILES = 0, 1
SPINS_BYTES, SPINS_BITS = 0, 1
NOALLOC_MAX_PARTIALS = 1 << 18


class RfimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("rfim error %d: %s" % (code, msg))
        self.code = code


class rfim_params_t(C.Structure):
    _fields_ = [("L", C.c_int), ("R", C.c_int), ("R_cap", C.c_int), ("J", C.c_double),
                ("h", C.c_double), ("fields", C.c_void_p), ("temps", C.c_void_p),
                ("seed", C.c_uint64), ("realization", C.c_uint32), ("field_kind", C.c_int)]


class rfim_job_t(C.Structure):
    _fields_ = [("params", rfim_params_t), ("trials", C.c_int), ("sweeps_per_trial", C.c_int64),
                ("rate_threshold", C.c_double), ("max_insert_per_trial", C.c_int),
                ("production_sweeps", C.c_int64)]


class rfim_result_t(C.Structure):
    _fields_ = [("R", C.c_int), ("capacity", C.c_int), ("temps", C.c_void_p), ("energies", C.c_void_p),
                ("magnetizations", C.c_void_p), ("perm", C.c_void_p), ("sweeps", C.c_uint64),
                ("exchanges", C.c_uint64), ("attempts", C.c_uint64), ("finished", C.c_int)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class rfim_alloc_t(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


def torch_allocator(stream=None) -> rfim_alloc_t:
    """A device memory provider backed by PyTorch's caching allocator (on
    `stream`, a torch.cuda.Stream, or torch's current stream).  The caller
    keeps the returned structure alive as long as the handle it serves."""
    import torch

    device = torch.cuda.current_device()

    def alloc(nbytes, _ctx):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), device, stream))
        except Exception:            # out of memory: the library reports RFIM_ENOMEM
            return None

    def free(ptr, _ctx):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:            # interpreter shutdown: nothing left to return to
            pass

    return rfim_alloc_t(ALLOC_FN(alloc), FREE_FN(free), None)


_lib = None


def load_library(path: str = LIB_PATH):
    """Open librfim.so (after torch, so that one HIP runtime serves both).
    Raises if the library has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401  (loads the HIP runtime the library binds to)
    except Exception:
        pass
    if not os.path.exists(path):
        raise RuntimeError("librfim.so not built: run python -m paper_1508_06268_amd.build")
    L = C.CDLL(path)
    vp, i32, i64, u64, dbl, sz = C.c_void_p, C.c_int, C.c_int64, C.c_uint64, C.c_double, C.c_size_t
    sig = {
        "rfim_create": (vp, [i32, i32, dbl, dbl, vp, vp, u64]),
        "rfim_create_ex": (vp, [C.POINTER(rfim_params_t), C.POINTER(rfim_alloc_t), vp]),
        "rfim_sweep": (i32, [vp, i64, i32]),
        "rfim_energies": (i32, [vp, vp]),
        "rfim_energies_noalloc": (i32, [i32, i32, dbl, dbl, vp, vp, vp, vp]),
        "rfim_set_update_order": (i32, [vp, i32, i32, i32, i32, i32]),
        "rfim_get_update_order": (i32, [vp, vp, vp, vp, vp, vp]),
        "rfim_set_spin_storage": (i32, [vp, i32]),
        "rfim_get_spin_storage": (i32, [vp]),
        "rfim_adapt_temps": (i32, [vp, i32, i64, i32, dbl, i32, i32]),
        "rfim_destroy": (None, [vp]),
        "rfim_last_error": (C.c_char_p, []),
        "rfim_set_stream": (i32, [vp, vp]),
        "rfim_synchronize": (i32, [vp]),
        "rfim_num_replicas": (i32, [vp]),
        "rfim_lattice_size": (i32, [vp]),
        "rfim_field_kind": (i32, [vp]),
        "rfim_temps": (i32, [vp, vp]),
        "rfim_magnetizations": (i32, [vp, vp]),
        "rfim_components": (i32, [vp, vp, vp, vp]),
        "rfim_get_spins": (i32, [vp, vp]),
        "rfim_set_spins": (i32, [vp, vp]),
        "rfim_get_perm": (i32, [vp, vp]),
        "rfim_set_perm": (i32, [vp, vp]),
        "rfim_get_counters": (i32, [vp, vp, vp]),
        "rfim_set_counters": (i32, [vp, u64, u64]),
        "rfim_exchange_stats": (i32, [vp, vp, vp]),
        "rfim_reset_exchange_stats": (i32, [vp]),
        "rfim_save": (i32, [vp, vp, C.POINTER(sz)]),
        "rfim_load": (vp, [vp, sz, vp]),
        "rfim_set_launch_shape": (i32, [vp, i32, i32, i32]),
        "rfim_get_launch_shape": (i32, [vp, vp, vp, vp]),
        "rfim_set_concurrency": (i32, [vp, i32]),
        "rfim_set_measure": (i32, [vp, i32]),
        "rfim_fourier": (i32, [vp, vp]),
        "rfim_get_concurrency": (i32, [vp]),
        "rfim_observables": (i32, [vp, vp]),
        "rfim_reset_observables": (i32, [vp]),
        "rfim_batch_create": (vp, [i32, vp, vp]),
        "rfim_batch_destroy": (None, [vp]),
        "rfim_batch_size": (i32, [vp]),
        "rfim_batch_sweep": (i32, [vp, i64, i32]),
        "rfim_batch_synchronize": (i32, [vp]),
        "rfim_batch_item": (vp, [vp, i32]),
        "rfim_batch_set_shape": (i32, [vp, i32, i32, i32, i32, i32]),
        "rfim_batch_set_group_bytes": (i32, [vp, i64]),
        "rfim_batch_get_group_bytes": (i64, [vp]),
        "rfim_pool_create": (vp, [sz, vp]),
        "rfim_pool_destroy": (None, [vp]),
        "rfim_pool_bytes_needed": (sz, [C.POINTER(rfim_params_t)]),
        "rfim_pool_admit": (i32, [vp, C.POINTER(rfim_params_t)]),
        "rfim_pool_admit_job": (i32, [vp, C.POINTER(rfim_job_t)]),
        "rfim_pool_step": (i32, [vp, i32, i32]),
        "rfim_pool_poll": (i32, [vp, vp, i32]),
        "rfim_pool_result": (i32, [vp, i32, C.POINTER(rfim_result_t)]),
        "rfim_pool_adapt": (i32, [vp, i32, dbl, i32, i32]),
        "rfim_pool_release": (i32, [vp, i32]),
        "rfim_pool_item": (vp, [vp, i32]),
        "rfim_pool_active": (i32, [vp]),
        "rfim_pool_reserved": (sz, [vp]),
        "rfim_pool_set_shape": (i32, [vp, i32, i32, i32, i32, i32]),
        "rfim_pool_synchronize": (i32, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    return load_library().rfim_last_error().decode()


def _check(rc):
    if rc < 0:
        raise RfimError(rc, last_error())
    return rc


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---- C ABI under the same names ---------------------------------------
def rfim_create(L, R, J, h, fields, temps, seed):
    f = np.ascontiguousarray(fields, dtype=np.float32).reshape(-1)
    T = np.ascontiguousarray(temps, dtype=np.float64).reshape(-1)
    return load_library().rfim_create(int(L), int(R), float(J), float(h), _p(f), _p(T),
                                      int(seed) & 0xFFFFFFFFFFFFFFFF)


def rfim_create_ex(L, R, J, h, fields, temps, seed=0, realization=0, field_kind=FIELDS_AUTO,
                   R_cap=0, stream=None, alloc=None):
    f = np.ascontiguousarray(fields, dtype=np.float32).reshape(-1)
    T = np.ascontiguousarray(temps, dtype=np.float64).reshape(-1)
    if f.size != int(L) ** 3 or T.size != int(R):
        raise ValueError("fields must hold L^3 values and temps R values")
    prm = rfim_params_t(int(L), int(R), int(R_cap), float(J), float(h), f.ctypes.data,
                        T.ctypes.data, int(seed) & 0xFFFFFFFFFFFFFFFF, int(realization),
                        int(field_kind))
    return load_library().rfim_create_ex(C.byref(prm), C.byref(alloc) if alloc is not None else None, stream)


def rfim_sweep(handle, n, exchange_every):
    return _check(load_library().rfim_sweep(handle, int(n), int(exchange_every)))


def rfim_energies(handle, R):
    E = np.zeros(R, dtype=np.float64)
    _check(load_library().rfim_energies(handle, _p(E)))
    return E


def rfim_energies_noalloc(L, R, J, h, d_spins, d_fields, d_E, stream=None):
    """Energies of R configurations held on the device, written to d_E on
    `stream` without allocating or synchronizing.  d_spins (int8 [R][L^3],
    +-1), d_fields (float32 [L^3]) and d_E (float64 [R]) are contiguous
    torch tensors on the current device; stream a torch.cuda.Stream or None
    (torch's current stream)."""
    import torch

    for t, dt, n in ((d_spins, torch.int8, R * L ** 3), (d_fields, torch.float32, L ** 3),
                     (d_E, torch.float64, R)):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous() and t.numel() == n):
            raise ValueError("expected a contiguous %s device tensor of %d elements" % (dt, n))
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(load_library().rfim_energies_noalloc(L, R, J, h, d_spins.data_ptr(), d_fields.data_ptr(),
                                                d_E.data_ptr(), s))


def rfim_adapt_temps(handle, trials, sweeps_per_trial, exchange_every, rate_threshold,
                     max_insert_per_trial, R_cap):
    return _check(load_library().rfim_adapt_temps(handle, int(trials), int(sweeps_per_trial),
                                                  int(exchange_every), float(rate_threshold),
                                                  int(max_insert_per_trial), int(R_cap)))


def rfim_destroy(handle):
    load_library().rfim_destroy(handle)


class Rfim:
    """One disorder realization on the GPU (owns a librfim handle)."""

    def __init__(self, L, R, J, h, fields, temps, seed=0, realization=0, field_kind=FIELDS_AUTO,
                 R_cap=0, stream=None, allocator=None):
        """allocator: None (the library's hipMalloc), "torch" (PyTorch's
        caching allocator on `stream`) or an rfim_alloc_t."""
        self.L = int(L)
        self.N = self.L ** 3
        self._torch_stream = None
        sptr = None
        if stream is not None:
            self._torch_stream = stream
            sptr = C.c_void_p(int(stream.cuda_stream))
        if allocator == "torch":
            allocator = torch_allocator(stream)
        self._alloc = allocator           # the callbacks must outlive the handle
        self._h = rfim_create_ex(L, R, J, h, fields, temps, seed, realization, field_kind, R_cap,
                                 sptr, allocator)
        if not self._h:
            raise ValueError(last_error())

    @classmethod
    def _wrap(cls, handle, L):
        obj = cls.__new__(cls)
        obj.L = int(L)
        obj.N = obj.L ** 3
        obj._torch_stream = None
        obj._h = handle
        return obj

    def close(self):
        if getattr(self, "_h", None):
            rfim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    @property
    def R(self) -> int:
        return load_library().rfim_num_replicas(self._h)

    @property
    def field_kind(self) -> int:
        return load_library().rfim_field_kind(self._h)

    def set_stream(self, stream):
        """Issue future work on a torch.cuda.Stream (None: the handle's own)."""
        self._torch_stream = stream
        ptr = C.c_void_p(int(stream.cuda_stream)) if stream is not None else None
        _check(load_library().rfim_set_stream(self._h, ptr))

    def synchronize(self):
        _check(load_library().rfim_synchronize(self._h))

    def sweep(self, n, every=0):
        rfim_sweep(self._h, n, every)

    def energies(self) -> np.ndarray:
        return rfim_energies(self._h, self.R)

    def magnetizations(self) -> np.ndarray:
        M = np.zeros(self.R, dtype=np.int64)
        _check(load_library().rfim_magnetizations(self._h, _p(M)))
        return M

    def components(self):
        R = self.R
        B = np.zeros(R, dtype=np.int64)
        F = np.zeros(R, dtype=np.float64)
        M = np.zeros(R, dtype=np.int64)
        _check(load_library().rfim_components(self._h, _p(B), _p(F), _p(M)))
        return B, F, M

    def temps(self) -> np.ndarray:
        T = np.zeros(self.R, dtype=np.float64)
        _check(load_library().rfim_temps(self._h, _p(T)))
        return T

    def spins(self) -> np.ndarray:
        s = np.zeros((self.R, self.N), dtype=np.int8)
        _check(load_library().rfim_get_spins(self._h, _p(s)))
        return s

    def set_spins(self, s):
        a = np.ascontiguousarray(s, dtype=np.int8).reshape(self.R, self.N)
        _check(load_library().rfim_set_spins(self._h, _p(a)))

    def perm(self) -> np.ndarray:
        p = np.zeros(self.R, dtype=np.int32)
        _check(load_library().rfim_get_perm(self._h, _p(p)))
        return p

    def set_perm(self, t2r):
        a = np.ascontiguousarray(t2r, dtype=np.int32)
        _check(load_library().rfim_set_perm(self._h, _p(a)))

    def counters(self):
        t = C.c_uint64()
        k = C.c_uint64()
        _check(load_library().rfim_get_counters(self._h, C.byref(t), C.byref(k)))
        return t.value, k.value

    def set_counters(self, t, k):
        _check(load_library().rfim_set_counters(self._h, int(t), int(k)))

    def exchange_stats(self):
        n = max(self.R - 1, 0)
        att = np.zeros(max(n, 1), dtype=np.uint64)
        acc = np.zeros(max(n, 1), dtype=np.uint64)
        _check(load_library().rfim_exchange_stats(self._h, _p(att), _p(acc)))
        return att[:n], acc[:n]

    def reset_exchange_stats(self):
        _check(load_library().rfim_reset_exchange_stats(self._h))

    def adapt_temps(self, trials, sweeps_per_trial, every, rate_threshold, max_insert_per_trial,
                    R_cap):
        return rfim_adapt_temps(self._h, trials, sweeps_per_trial, every, rate_threshold,
                                max_insert_per_trial, R_cap)

    def observables(self) -> np.ndarray:
        """Per slot: [count, sum E, sum E^2, sum |M|, sum M^2, sum M^4]."""
        o = np.zeros((self.R, 6), dtype=np.float64)
        _check(load_library().rfim_observables(self._h, _p(o)))
        return o

    def reset_observables(self):
        _check(load_library().rfim_reset_observables(self._h))

    def set_measure(self, flags: int):
        """MEASURE_FOURIER: also sample the correlation-length observable F
        at every exchange step (see rfim_set_measure)."""
        _check(load_library().rfim_set_measure(self._h, int(flags)))

    def fourier(self) -> np.ndarray:
        """Per slot: [count, sum F]."""
        o = np.zeros((self.R, 2), dtype=np.float64)
        _check(load_library().rfim_fourier(self._h, _p(o)))
        return o

    def launch_shape(self):
        m, nw, wg = C.c_int(), C.c_int(), C.c_int()
        _check(load_library().rfim_get_launch_shape(self._h, C.byref(m), C.byref(nw), C.byref(wg)))
        return m.value, nw.value, wg.value

    def set_launch_shape(self, mode, nw, wg):
        _check(load_library().rfim_set_launch_shape(self._h, int(mode), int(nw), int(wg)))

    def concurrency(self) -> int:
        return _check(load_library().rfim_get_concurrency(self._h))

    def set_concurrency(self, streams: int):
        """0 automatic, 1 one stream, 2 two streams (see rfim_set_concurrency)."""
        _check(load_library().rfim_set_concurrency(self._h, int(streams)))

    def set_update_order(self, order: int, tiles=(0, 0, 0), hits: int = 1):
        """ORDER_CHECKERBOARD, or ORDER_TILES with tiles (tx, ty, tz) and
        `hits` local sweeps per tile visit (see rfim_set_update_order)."""
        tx, ty, tz = (int(v) for v in tiles)
        _check(load_library().rfim_set_update_order(self._h, int(order), tx, ty, tz, int(hits)))

    def set_spin_storage(self, storage: int):
        """SPINS_BYTES or SPINS_BITS (one bit per spin, L = 64/128/256)."""
        _check(load_library().rfim_set_spin_storage(self._h, int(storage)))

    def spin_storage(self) -> int:
        return _check(load_library().rfim_get_spin_storage(self._h))

    def update_order(self):
        """(order, (tx, ty, tz), hits)."""
        v = [C.c_int(0) for _ in range(5)]
        _check(load_library().rfim_get_update_order(self._h, *[C.byref(x) for x in v]))
        return v[0].value, (v[1].value, v[2].value, v[3].value), v[4].value

    def save(self) -> bytes:
        n = C.c_size_t(0)
        _check(load_library().rfim_save(self._h, None, C.byref(n)))
        buf = (C.c_uint8 * n.value)()
        _check(load_library().rfim_save(self._h, buf, C.byref(n)))
        return bytes(buf)

    @classmethod
    def load(cls, blob: bytes, stream=None):
        buf = (C.c_uint8 * len(blob)).from_buffer_copy(blob)
        sptr = C.c_void_p(int(stream.cuda_stream)) if stream is not None else None
        h = load_library().rfim_load(buf, len(blob), sptr)
        if not h:
            raise ValueError(last_error())
        L = load_library().rfim_lattice_size(h)
        obj = cls._wrap(h, L)
        obj._torch_stream = stream
        return obj


class _Borrowed(Rfim):
    """A batch item's handle: usable for observables and state, owned by the
    batch (closing it does nothing)."""

    def close(self):
        self._h = None


class Batch:
    """Many independent realizations advanced together (rfim_batch_*)."""

    def __init__(self, realizations, stream=None):
        """realizations: iterable of objects with L, R, J, h, fields, temps,
        seed, realization and optionally R_cap / field_kind attributes."""
        items = list(realizations)
        n = len(items)
        arr = (rfim_params_t * n)()
        self._keep = []
        self.L = []
        for q, w in enumerate(items):
            f = np.ascontiguousarray(w.fields, dtype=np.float32).reshape(-1)
            T = np.ascontiguousarray(w.temps, dtype=np.float64).reshape(-1)
            self._keep += [f, T]
            arr[q] = rfim_params_t(int(w.L), int(w.R), int(getattr(w, "R_cap", 0) or 0), float(w.J),
                                   float(w.h), f.ctypes.data, T.ctypes.data,
                                   int(getattr(w, "seed", 0)) & 0xFFFFFFFFFFFFFFFF,
                                   int(getattr(w, "realization", 0)),
                                   int(getattr(w, "field_kind", FIELDS_AUTO)))
            self.L.append(int(w.L))
        self._torch_stream = stream
        sptr = C.c_void_p(int(stream.cuda_stream)) if stream is not None else None
        self._b = load_library().rfim_batch_create(n, arr, sptr)
        self._keep = None
        if not self._b:
            raise ValueError(last_error())
        self._items = [None] * n

    def close(self):
        if getattr(self, "_b", None):
            self._items = []
            load_library().rfim_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return load_library().rfim_batch_size(self._b)

    def sweep(self, n, every=0):
        _check(load_library().rfim_batch_sweep(self._b, int(n), int(every)))

    def synchronize(self):
        _check(load_library().rfim_batch_synchronize(self._b))

    def set_shape(self, L, field_kind, mode, nw, wg):
        """Launch shape of the class (L, field_kind) (rfim_batch_set_shape):
        a streaming or LDS-resident shape in byte storage, or
        (MODE_BITS, 0, 0), one bit per spin (L = 64, 128, 256; the default
        there)."""
        _check(load_library().rfim_batch_set_shape(self._b, int(L), int(field_kind), int(mode),
                                                    int(nw), int(wg)))

    def set_group_bytes(self, nbytes):
        """Group budget of the temporal blocking of large streaming classes
        (rfim_batch_set_group_bytes); 0 turns it off."""
        _check(load_library().rfim_batch_set_group_bytes(self._b, int(nbytes)))

    def group_bytes(self) -> int:
        return _check(load_library().rfim_batch_get_group_bytes(self._b))

    def item(self, i) -> Rfim:
        if self._items[i] is None:
            h = load_library().rfim_batch_item(self._b, int(i))
            if not h:
                raise IndexError(last_error())
            self._items[i] = _Borrowed._wrap(h, self.L[i])
        return self._items[i]


def _params_of(w):
    """rfim_params_t for a realization spec, plus the arrays it points to."""
    f = np.ascontiguousarray(w.fields, dtype=np.float32).reshape(-1)
    T = np.ascontiguousarray(w.temps, dtype=np.float64).reshape(-1)
    prm = rfim_params_t(int(w.L), int(w.R), int(getattr(w, "R_cap", 0) or 0), float(w.J), float(w.h),
                        f.ctypes.data, T.ctypes.data, int(getattr(w, "seed", 0)) & 0xFFFFFFFFFFFFFFFF,
                        int(getattr(w, "realization", 0)), int(getattr(w, "field_kind", FIELDS_AUTO)))
    return prm, (f, T)


class Pool:
    """Continuous batching (rfim_pool_*): realizations admitted against a
    device-memory budget, advanced together, released when done."""

    def __init__(self, budget_bytes, stream=None):
        self._torch_stream = stream
        sptr = C.c_void_p(int(stream.cuda_stream)) if stream is not None else None
        self._p = load_library().rfim_pool_create(int(budget_bytes), sptr)
        if not self._p:
            raise ValueError(last_error())
        self._L = {}

    def close(self):
        if getattr(self, "_p", None):
            load_library().rfim_pool_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def bytes_needed(w) -> int:
        prm, keep = _params_of(w)
        return int(load_library().rfim_pool_bytes_needed(C.byref(prm)))

    def admit(self, w):
        """Slot id, or None when the budget cannot hold it now."""
        prm, keep = _params_of(w)
        rc = load_library().rfim_pool_admit(self._p, C.byref(prm))
        if rc == RFIM_EBUSY:
            return None
        _check(rc)
        self._L[rc] = int(w.L)
        return rc

    def admit_job(self, w):
        """Admit a realization with its schedule (w.adapt: trials,
        sweeps_per_trial, rate_threshold, max_insert_per_trial; w.sweeps:
        production sweeps); the pool runs it to completion.  Slot id, or None
        when the budget cannot hold it now."""
        prm, keep = _params_of(w)
        a = getattr(w, "adapt", None) or {}
        job = rfim_job_t(prm, int(a.get("trials", 0)), int(a.get("sweeps_per_trial", 0)),
                         float(a.get("rate_threshold", 0.0)), int(a.get("max_insert_per_trial", 0)),
                         int(w.sweeps))
        rc = load_library().rfim_pool_admit_job(self._p, C.byref(job))
        if rc == RFIM_EBUSY:
            return None
        _check(rc)
        self._L[rc] = int(w.L)
        return rc

    def step(self, quantum, every):
        _check(load_library().rfim_pool_step(self._p, int(quantum), int(every)))

    def poll(self):
        """Slot ids of finished jobs not yet released (ascending)."""
        n = _check(load_library().rfim_pool_poll(self._p, None, 0))
        if n == 0:
            return []
        buf = (C.c_int * n)()
        m = _check(load_library().rfim_pool_poll(self._p, buf, n))
        return list(buf[:m])

    def result(self, slot) -> dict:
        """State of a slot through rfim_pool_result: R, temperatures,
        energies, magnetisations and permutation by slot, counters, the
        attempts issued and whether its schedule is complete."""
        res = rfim_result_t()
        res.capacity = 0
        _check(load_library().rfim_pool_result(self._p, int(slot), C.byref(res)))
        R = res.R
        T = np.zeros(R, dtype=np.float64)
        E = np.zeros(R, dtype=np.float64)
        M = np.zeros(R, dtype=np.int64)
        P = np.zeros(R, dtype=np.int32)
        res = rfim_result_t(0, R, T.ctypes.data, E.ctypes.data, M.ctypes.data, P.ctypes.data, 0, 0, 0, 0)
        _check(load_library().rfim_pool_result(self._p, int(slot), C.byref(res)))
        return dict(R=res.R, temps=T, energies=E, magnetizations=M, perm=P, sweeps=res.sweeps,
                    exchanges=res.exchanges, attempts=res.attempts, finished=bool(res.finished))

    def adapt(self, slot, rate_threshold, max_insert, R_cap) -> int:
        return _check(load_library().rfim_pool_adapt(self._p, int(slot), float(rate_threshold),
                                                     int(max_insert), int(R_cap)))

    def release(self, slot):
        _check(load_library().rfim_pool_release(self._p, int(slot)))
        self._L.pop(slot, None)

    def item(self, slot) -> Rfim:
        h = load_library().rfim_pool_item(self._p, int(slot))
        if not h:
            raise IndexError(last_error())
        return _Borrowed._wrap(h, self._L[slot])

    @property
    def active(self) -> int:
        return load_library().rfim_pool_active(self._p)

    @property
    def reserved(self) -> int:
        return int(load_library().rfim_pool_reserved(self._p))

    def set_shape(self, L, field_kind, mode, nw, wg):
        """Shape of the class (L, field_kind) for its items (rfim_pool_set_shape;
        see Batch.set_shape)."""
        _check(load_library().rfim_pool_set_shape(self._p, int(L), int(field_kind), int(mode), int(nw),
                                                   int(wg)))

    def synchronize(self):
        _check(load_library().rfim_pool_synchronize(self._p))
