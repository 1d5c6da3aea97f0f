"""ctypes wrapper of the C oracle (test infrastructure; see oracle/__init__.py).

Lattices are NumPy int8 arrays of shape (L, L), +1 / -1, row-major: the
canonical layout. Functions mirror ising_oracle.c; each cites the passage of
the paper it follows there.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def load(path=None):
    """Load (building first if absent) the oracle library."""
    global _lib
    if path is None:
        if _lib is not None:
            return _lib
        path = _build.LIB
        if not os.path.exists(path):
            _build.compile_oracle()
    lib = C.CDLL(path)
    u32, u64, i32, dbl = C.c_uint32, C.c_uint64, C.c_int, C.c_double
    p = C.c_void_p
    lib.oracle_philox4x32_10.argtypes = [p, p, p]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_draw.argtypes = [u64, u32, u32, u32, u32, u32, u32]
    lib.oracle_draw.restype = u32
    lib.oracle_threshold_table.argtypes = [dbl, dbl, dbl, p]
    lib.oracle_threshold_table.restype = i32
    lib.oracle_init.argtypes = [u32, u64, dbl, p]
    lib.oracle_init.restype = i32
    lib.oracle_half_sweep.argtypes = [u32, p, u64, u32, u32, p]
    lib.oracle_half_sweep.restype = i32
    lib.oracle_observables.argtypes = [u32, p, p, p]
    lib.oracle_observables.restype = None
    lib.oracle_run.argtypes = [u32, dbl, dbl, dbl, u64, u64, u64, p, p, p]
    lib.oracle_run.restype = i32
    lib.oracle_fnv1a64.argtypes = [p, C.c_size_t]
    lib.oracle_fnv1a64.restype = u64
    lib.oracle_window_run.argtypes = [u32, dbl, dbl, dbl, u64, u64, u64, u32, u32, u32, p, p]
    lib.oracle_window_run.restype = i32
    lib.oracle_init_window.argtypes = [u32, u64, dbl, u32, u32, u32, p]
    lib.oracle_init_window.restype = i32
    lib.oracle_creutz_half_sweep.argtypes = [u32, u32, p, p]
    lib.oracle_creutz_half_sweep.restype = i32
    lib.oracle_demon_sum.argtypes = [u32, p]
    lib.oracle_demon_sum.restype = C.c_int64
    lib.oracle_creutz_run.argtypes = [u32, u64, i32, p, p, p, p, p]
    lib.oracle_creutz_run.restype = i32
    lib.oracle_perc_medium.argtypes = [u32, dbl, u64, p]
    lib.oracle_perc_medium.restype = i32
    lib.oracle_perc_invade.argtypes = [u32, p, u32, u32, u32, p, p]
    lib.oracle_perc_invade.restype = i32
    lib.oracle_perc_summary.argtypes = [u32, p, p, p, p]
    lib.oracle_perc_summary.restype = None
    lib.oracle_set_threads.argtypes = [i32]
    lib.oracle_set_threads.restype = i32
    lib.oracle_get_threads.argtypes = []
    lib.oracle_get_threads.restype = i32
    if path == _build.LIB:
        _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Oracle:
    """Thin object over one loaded oracle library (the default one, or a
    variant built from a modified source for negative-control tests)."""

    def __init__(self, path=None):
        self.lib = load(path)

    def set_threads(self, n):
        if self.lib.oracle_set_threads(int(n)) != 0:
            raise ValueError("thread count must be >= 1")

    def threads(self):
        return self.lib.oracle_get_threads()

    def philox(self, ctr, key):
        c = np.asarray(ctr, dtype=np.uint32)
        k = np.asarray(key, dtype=np.uint32)
        out = np.zeros(4, dtype=np.uint32)
        self.lib.oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
        return out

    def draw(self, seed, L, t, c, d, i, j):
        return int(self.lib.oracle_draw(seed, L, t, c, d, i, j))

    def table(self, J, h, T):
        thr = np.zeros(10, dtype=np.uint64)
        rc = self.lib.oracle_threshold_table(J, h, T, _ptr(thr))
        if rc != 0:
            raise ValueError("invalid J/h/T")
        return thr

    def init(self, L, seed, p_up):
        s = np.zeros((L, L), dtype=np.int8)
        rc = self.lib.oracle_init(L, seed, p_up, _ptr(s))
        if rc != 0:
            raise ValueError("invalid init arguments")
        return s

    def half_sweep(self, s, thr, seed, t, c):
        L = s.shape[0]
        thr = np.ascontiguousarray(thr, dtype=np.uint64)
        rc = self.lib.oracle_half_sweep(L, _ptr(thr), seed, t, c, _ptr(s))
        if rc != 0:
            raise ValueError("invalid half-sweep arguments")
        return s

    def observables(self, s):
        b = C.c_int64()
        m = C.c_int64()
        self.lib.oracle_observables(s.shape[0], _ptr(s), C.byref(b), C.byref(m))
        return b.value, m.value

    def run(self, s, J, h, T, seed, t0, n, series=True):
        """Sweep `s` in place n times from sweep index t0; returns (B, M)
        arrays of length n (or (None, None) when series=False)."""
        L = s.shape[0]
        assert s.dtype == np.int8 and s.flags.c_contiguous and s.shape == (L, L)
        if series:
            B = np.zeros(n, dtype=np.int64)
            M = np.zeros(n, dtype=np.int64)
            pb, pm = _ptr(B), _ptr(M)
        else:
            B = M = None
            pb = pm = None
        rc = self.lib.oracle_run(L, J, h, T, seed, t0, n, _ptr(s), pb, pm)
        if rc != 0:
            raise ValueError(f"oracle_run failed ({rc})")
        return B, M

    def creutz_run(self, s, d, n, reverse=False, series=True):
        """Creutz demon sweeps in place (spins s, demons d: uint8 (L, L));
        returns (B, M, D) series of length n (or Nones)."""
        L = s.shape[0]
        assert d.dtype == np.uint8 and d.shape == s.shape and d.flags.c_contiguous
        if series:
            B, M, D = (np.zeros(n, dtype=np.int64) for _ in range(3))
            args = (_ptr(B), _ptr(M), _ptr(D))
        else:
            B = M = D = None
            args = (None, None, None)
        rc = self.lib.oracle_creutz_run(L, n, 1 if reverse else 0, _ptr(s), _ptr(d), *args)
        if rc != 0:
            raise ValueError("invalid Creutz arguments")
        return B, M, D

    def demon_sum(self, d):
        return int(self.lib.oracle_demon_sum(d.shape[0], _ptr(d)))

    # -- percolation (Section 2.3) -------------------------------------------
    PERC_TOP_ROW = 0
    PERC_POINT = 1

    def perc_medium(self, L, P, seed):
        """(L, L) uint8 pore map: 1 = pore."""
        pore = np.zeros((L, L), dtype=np.uint8)
        if self.lib.oracle_perc_medium(L, P, seed, _ptr(pore)) != 0:
            raise ValueError("invalid medium arguments")
        return pore

    def perc_invade(self, pore, source=0, i0=0, j0=0):
        """(L, L) int32 arrival passes (-1 = never invaded)."""
        pore = np.ascontiguousarray(pore, dtype=np.uint8)
        L = pore.shape[0]
        arr = np.zeros((L, L), dtype=np.int32)
        queue = np.zeros(L * L, dtype=np.uint32)
        if self.lib.oracle_perc_invade(L, _ptr(pore), source, i0, j0, _ptr(arr), _ptr(queue)) != 0:
            raise ValueError("invalid invasion arguments")
        return arr

    def perc_summary(self, arrival):
        """(invaded sites, max arrival pass, spanning bits)."""
        arrival = np.ascontiguousarray(arrival, dtype=np.int32)
        n, mx, sp = C.c_uint64(), C.c_int32(), C.c_uint32()
        self.lib.oracle_perc_summary(arrival.shape[0], _ptr(arrival), C.byref(n), C.byref(mx), C.byref(sp))
        return n.value, mx.value, sp.value

    def fnv1a64(self, s):
        b = np.ascontiguousarray(s).view(np.uint8)
        return int(self.lib.oracle_fnv1a64(_ptr(b), b.size))

    def init_window(self, L, seed, p_up, i0, j0, W):
        win = np.zeros((W, W), dtype=np.int8)
        rc = self.lib.oracle_init_window(L, seed, p_up, i0, j0, W, _ptr(win))
        if rc != 0:
            raise ValueError("invalid window")
        return win

    def window_run(self, L, J, h, T, seed, t0, n, i0, j0, win):
        W = win.shape[0]
        valid = np.zeros((W, W), dtype=np.uint8)
        rc = self.lib.oracle_window_run(L, J, h, T, seed, t0, n, i0, j0, W, _ptr(win),
                                        _ptr(valid))
        if rc != 0:
            raise ValueError(f"oracle_window_run failed ({rc})")
        return win, valid.astype(bool)


_default = None


def default():
    global _default
    if _default is None:
        _default = Oracle()
    return _default
