"""ctypes binding of the C ABI in include/ising.h (argument marshalling only).

Every function keeps the C name and returns what the C call returns in its
out-parameters; a negative status raises IsingError. Device memory and
streams may come from PyTorch: pass ``tensor.data_ptr()`` and
``torch.cuda.Stream().cuda_stream`` as integers.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libising_mi355x.so")

ISING_OK = 0
ISING_EINVAL = -1
ISING_ENOMEM = -2
ISING_EDEVICE = -3
ISING_ERANGE = -4
ISING_EUNSUPPORTED = -5
ISING_ESTATE = -6
ISING_EIO = -7

ISING_MAX_L = 65536
ISING_STATIC_SCRATCH_PAIRS = 65536

ISING_PLAN_AUTO = 0
ISING_PLAN_TWO_PASS = 1
ISING_PLAN_FUSED = 2
ISING_PLAN_RESIDENT = 3
ISING_PLAN_GENERIC = 4
ISING_PLAN_FUSED_ROWS = 5
ISING_PLAN_BANDS = 6
ISING_BAND_SWEEPS_PER_LAUNCH = 512

ISING_BATCH_AUTO = 0
ISING_BATCH_RESIDENT = 1
ISING_BATCH_STEPPED = 2

ISING_TUNE_RETIME = 1

ISING_OBS_HASH = 1
ISING_OBS_SERIES = 2


class ising_params(C.Structure):
    _fields_ = [("L", C.c_uint32), ("flags", C.c_uint32), ("J", C.c_double), ("h", C.c_double),
                ("T", C.c_double), ("seed", C.c_uint64), ("p_up", C.c_double)]


class ising_obs(C.Structure):
    _fields_ = [("sweeps_done", C.c_uint64), ("bond_sum", C.c_int64), ("mag_sum", C.c_int64),
                ("energy", C.c_double), ("e_per_site", C.c_double), ("m_per_site", C.c_double),
                ("lattice_hash", C.c_uint64), ("series_len", C.c_uint64)]


class ising_averages(C.Structure):
    _fields_ = [("n", C.c_uint64), ("e", C.c_double), ("e2", C.c_double), ("m", C.c_double),
                ("abs_m", C.c_double), ("m2", C.c_double)]


class ising_batch_rate(C.Structure):
    _fields_ = [("max_side", C.c_uint32), ("field", C.c_uint32), ("resident_per_workgroup", C.c_double),
                ("resident_fixed_ns", C.c_double), ("stepped", C.c_double * 3)]


class perc_params(C.Structure):
    _fields_ = [("L", C.c_uint32), ("porosity", C.c_double), ("seed", C.c_uint64), ("source", C.c_uint32),
                ("i0", C.c_uint32), ("j0", C.c_uint32)]


class perc_result(C.Structure):
    _fields_ = [("pores", C.c_uint64), ("invaded", C.c_uint64), ("passes", C.c_int32), ("spans", C.c_uint32),
                ("launches", C.c_uint32), ("pad", C.c_uint32), ("tile_visits", C.c_uint64),
                ("tile_iterations", C.c_uint64), ("arrival_hash", C.c_uint64)]


PERC_SOURCE_TOP_ROW = 0
PERC_SOURCE_POINT = 1


class IsingError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = lib().ising_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


# Every entry point declared in include/ising.h, with its ctypes signature.
SIGNATURES = {
    "ising_state_bytes": (C.c_size_t, [C.c_uint32, C.c_uint32]),
    "ising_create": (C.c_int, [C.POINTER(ising_params), C.c_void_p, C.POINTER(C.c_void_p)]),
    "ising_reset": (C.c_int, [C.c_void_p, C.POINTER(ising_params)]),
    "ising_reserve": (C.c_int, [C.c_void_p, C.c_uint64]),
    "ising_create_in": (C.c_int, [C.POINTER(ising_params), C.c_void_p, C.c_size_t, C.c_void_p,
                                  C.POINTER(C.c_void_p)]),
    "ising_sweep": (C.c_int, [C.c_void_p, C.c_uint64]),
    "ising_sweep_static": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p]),
    "ising_observables": (C.c_int, [C.c_void_p, C.POINTER(ising_obs), C.c_void_p, C.c_void_p, C.c_uint64,
                                    C.c_uint32]),
    "ising_prefetch_observables": (C.c_int, [C.c_void_p, C.c_uint32]),
    "ising_copy_spins": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "ising_load_spins": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_uint64]),
    "ising_sweep_batch": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.c_uint64), C.c_size_t, C.c_void_p]),
    "ising_sweep_batch_plan": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.c_uint64), C.c_size_t, C.c_void_p,
                                         C.c_uint32]),
    "ising_batch_tune": (C.c_int, [C.c_int, C.c_char_p, C.c_uint32, C.POINTER(C.c_int)]),
    "ising_batch_rates": (C.c_int, [C.c_int, C.POINTER(ising_batch_rate), C.c_size_t, C.POINTER(C.c_int),
                                    C.POINTER(C.c_double)]),
    "ising_batch_choice": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.c_uint64), C.c_size_t,
                                     C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_double)]),
    "ising_series_averages": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32, C.c_double,
                                        C.c_double, C.POINTER(ising_averages)]),
    "ising_plan_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                  C.POINTER(C.c_uint32)]),
    "ising_plan_set": (C.c_int, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32]),
    "ising_tune": (C.c_int, [C.c_void_p, C.c_uint32]),
    "ising_creutz_init": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_uint8]),
    "ising_creutz_sweep": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int]),
    "ising_demon_sum": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "ising_copy_demons": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "ising_destroy": (C.c_int, [C.c_void_p]),
    "perc_create": (C.c_int, [C.POINTER(perc_params), C.c_void_p, C.POINTER(C.c_void_p)]),
    "perc_run": (C.c_int, [C.c_void_p]),
    "perc_result_get": (C.c_int, [C.c_void_p, C.POINTER(perc_result), C.c_uint32]),
    "perc_copy_medium": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "perc_copy_arrival": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "perc_destroy": (C.c_int, [C.c_void_p]),
    "perc_run_batch": (C.c_int, [C.POINTER(C.c_void_p), C.c_size_t]),
    "perc_set_params": (C.c_int, [C.c_void_p, C.POINTER(perc_params)]),
    "mb_vector_op": (C.c_int, [C.c_uint32, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "mb_copy_lattice": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int,
                                  C.c_void_p]),
    "mb_philox": (C.c_int, [C.c_void_p, C.c_size_t, C.c_uint32, C.c_uint64, C.c_void_p]),
    "ising_strerror": (C.c_char_p, [C.c_int]),
    "ising_device_error": (C.c_char_p, [C.c_void_p]),
}

_lib = None


def _share_torch_hip_runtime():
    """PyTorch ships its own HIP runtime (same soname as ROCm's). Loading it
    first makes the library bind to that one, so torch tensors, streams and
    this library share one runtime in the process."""
    try:
        import torch  # noqa: F401
    except Exception:
        pass


def lib(path=None):
    """Load the HIP library (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise OSError(f"{p} is missing: build it with paper_cs_0312006_amd/build.py")
    _share_torch_hip_runtime()
    handle = C.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(handle, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = handle
    return handle


def _check(rc, what, ctx=None):
    if rc != ISING_OK:
        if rc == ISING_EDEVICE and ctx:
            detail = lib().ising_device_error(ctx)
            if detail:
                what = f"{what} [{detail.decode()}]"
        raise IsingError(rc, what)


def _params(L, J=1.0, h=0.0, T=2.269185, seed=0, p_up=0.5, flags=ISING_PLAN_AUTO):
    return ising_params(int(L), int(flags), float(J), float(h), float(T), int(seed) & (2 ** 64 - 1),
                        float(p_up))


def ising_state_bytes(L, flags=ISING_PLAN_AUTO):
    return int(lib().ising_state_bytes(int(L), int(flags)))


def ising_create(L, J=1.0, h=0.0, T=2.269185, seed=0, p_up=0.5, flags=ISING_PLAN_AUTO, stream=None):
    """Returns an opaque context handle (int)."""
    p = _params(L, J, h, T, seed, p_up, flags)
    out = C.c_void_p()
    _check(lib().ising_create(C.byref(p), stream, C.byref(out)), "ising_create")
    return out.value


def ising_reset(ctx, L, J=1.0, h=0.0, T=2.269185, seed=0, p_up=0.5, flags=ISING_PLAN_AUTO):
    """Re-initialise ctx for new parameters of the same side, keeping its buffers."""
    p = _params(L, J, h, T, seed, p_up, flags)
    _check(lib().ising_reset(ctx, C.byref(p)), "ising_reset", ctx)


def ising_reserve(ctx, sweeps):
    """Make room for the series of `sweeps` further sweeps."""
    _check(lib().ising_reserve(ctx, int(sweeps)), "ising_reserve", ctx)


def ising_create_in(dev_ptr, nbytes, L, J=1.0, h=0.0, T=2.269185, seed=0, p_up=0.5, flags=ISING_PLAN_AUTO,
                    stream=None):
    p = _params(L, J, h, T, seed, p_up, flags)
    out = C.c_void_p()
    _check(lib().ising_create_in(C.byref(p), C.c_void_p(dev_ptr), int(nbytes), stream, C.byref(out)),
           "ising_create_in")
    return out.value


def ising_sweep(ctx, n):
    _check(lib().ising_sweep(ctx, int(n)), "ising_sweep", ctx)


def ising_sweep_static(ctx, n, series_dev):
    """series_dev: device address (int) of 2 n int64."""
    _check(lib().ising_sweep_static(ctx, int(n), C.c_void_p(int(series_dev))), "ising_sweep_static", ctx)


def ising_observables(ctx, want=0, capacity=None):
    """Returns (ising_obs, bond_series or None, mag_series or None)."""
    obs = ising_obs()
    bs = ms = None
    pb = pm = None
    cap = 0
    if want & ISING_OBS_SERIES:
        if capacity is None:
            rc = lib().ising_observables(ctx, C.byref(obs), None, None, 0, 0)
            _check(rc, "ising_observables")
            capacity = obs.series_len
        cap = int(capacity)
        bs = np.zeros(cap, dtype=np.int64)
        ms = np.zeros(cap, dtype=np.int64)
        pb, pm = bs.ctypes.data, ms.ctypes.data
    _check(lib().ising_observables(ctx, C.byref(obs), pb, pm, cap, int(want)), "ising_observables", ctx)
    if bs is not None:
        n = obs.series_len
        bs, ms = bs[:n], ms[:n]
    return obs, bs, ms


def ising_prefetch_observables(ctx, want):
    """Start the read-back of a later ising_observables(ctx, want) without
    waiting. Returns False when the library declines (too much to stage), in
    which case ising_observables reads back on its own."""
    rc = lib().ising_prefetch_observables(ctx, int(want))
    if rc == ISING_EUNSUPPORTED:
        return False
    _check(rc, "ising_prefetch_observables", ctx)
    return True


def ising_copy_spins(ctx, L):
    out = np.empty((L, L), dtype=np.int8)
    _check(lib().ising_copy_spins(ctx, out.ctypes.data, out.size), "ising_copy_spins", ctx)
    return out


def ising_load_spins(ctx, spins, t):
    a = np.ascontiguousarray(spins, dtype=np.int8)
    _check(lib().ising_load_spins(ctx, a.ctypes.data, a.size, int(t)), "ising_load_spins", ctx)


def ising_sweep_batch(ctxs, n_sweeps, stream=None):
    k = len(ctxs)
    arr = (C.c_void_p * k)(*ctxs)
    ns = (C.c_uint64 * k)(*[int(n) for n in n_sweeps])
    _check(lib().ising_sweep_batch(arr, ns, k, stream), "ising_sweep_batch", ctxs[0] if ctxs else None)


def ising_sweep_batch_plan(ctxs, n_sweeps, plan, stream=None):
    k = len(ctxs)
    arr = (C.c_void_p * k)(*ctxs)
    ns = (C.c_uint64 * k)(*[int(n) for n in n_sweeps])
    _check(lib().ising_sweep_batch_plan(arr, ns, k, stream, int(plan)), "ising_sweep_batch_plan",
           ctxs[0] if ctxs else None)


def ising_batch_tune(device=0, cache_path=None, flags=0):
    """Returns True when the rates were loaded from cache_path."""
    hit = C.c_int(0)
    path = os.fsencode(cache_path) if cache_path is not None else None
    _check(lib().ising_batch_tune(int(device), path, int(flags), C.byref(hit)), "ising_batch_tune")
    return bool(hit.value)


def ising_batch_rates(device=0):
    """(list of dicts per class, tuned, floor_ns)."""
    out = (ising_batch_rate * 10)()
    tuned, floor = C.c_int(0), C.c_double(0.0)
    _check(lib().ising_batch_rates(int(device), out, 10, C.byref(tuned), C.byref(floor)), "ising_batch_rates")
    rows = [{"max_side": r.max_side, "field": r.field, "resident_per_workgroup": r.resident_per_workgroup,
             "resident_fixed_ns": r.resident_fixed_ns, "stepped": list(r.stepped)} for r in out]
    return rows, bool(tuned.value), floor.value


def ising_batch_choice(ctxs, n_sweeps):
    """(plan, stepped tile rows, (predicted resident ns, predicted stepped ns))."""
    k = len(ctxs)
    arr = (C.c_void_p * k)(*ctxs)
    ns = (C.c_uint64 * k)(*[int(n) for n in n_sweeps])
    plan, rows, pred = C.c_uint32(), C.c_uint32(), (C.c_double * 2)()
    _check(lib().ising_batch_choice(arr, ns, k, C.byref(plan), C.byref(rows), pred), "ising_batch_choice")
    return plan.value, rows.value, (pred[0], pred[1])


def ising_series_averages(bond, mag, L, J=1.0, h=0.0):
    b = np.ascontiguousarray(bond, dtype=np.int64)
    m = np.ascontiguousarray(mag, dtype=np.int64)
    out = ising_averages()
    _check(lib().ising_series_averages(b.ctypes.data, m.ctypes.data, len(b), int(L), float(J), float(h),
                                       C.byref(out)), "ising_series_averages")
    return out


def ising_plan_info(ctx):
    p, cw, r = C.c_uint32(), C.c_uint32(), C.c_uint32()
    _check(lib().ising_plan_info(ctx, C.byref(p), C.byref(cw), C.byref(r)), "ising_plan_info", ctx)
    return p.value, cw.value, r.value


def ising_plan_set(ctx, plan, cw=0, rows=0):
    _check(lib().ising_plan_set(ctx, int(plan), int(cw), int(rows)), "ising_plan_set", ctx)


def ising_tune(ctx, trial_sweeps=4):
    _check(lib().ising_tune(ctx, int(trial_sweeps)), "ising_tune", ctx)


def ising_creutz_init(ctx, demons=None, fill=0):
    """Demons from an (L, L) uint8 array (canonical layout) or, when None,
    every demon = fill."""
    if demons is None:
        rc = lib().ising_creutz_init(ctx, None, 0, int(fill))
    else:
        a = np.ascontiguousarray(demons, dtype=np.uint8)
        rc = lib().ising_creutz_init(ctx, a.ctypes.data, a.size, 0)
    _check(rc, "ising_creutz_init")


def ising_creutz_sweep(ctx, n, reverse=False):
    _check(lib().ising_creutz_sweep(ctx, int(n), 1 if reverse else 0), "ising_creutz_sweep", ctx)


def ising_demon_sum(ctx):
    v = C.c_int64()
    _check(lib().ising_demon_sum(ctx, C.byref(v)), "ising_demon_sum", ctx)
    return v.value


def ising_copy_demons(ctx, L):
    out = np.empty((L, L), dtype=np.uint8)
    _check(lib().ising_copy_demons(ctx, out.ctypes.data, out.size), "ising_copy_demons", ctx)
    return out


def ising_destroy(ctx):
    _check(lib().ising_destroy(ctx), "ising_destroy")


def perc_create(L, porosity, seed=0, source=PERC_SOURCE_TOP_ROW, i0=0, j0=0, stream=None):
    p = perc_params(int(L), float(porosity), int(seed), int(source), int(i0), int(j0))
    out = C.c_void_p()
    _check(lib().perc_create(C.byref(p), stream, C.byref(out)), "perc_create")
    return out.value


def perc_run(ctx):
    _check(lib().perc_run(ctx), "perc_run")


def perc_run_batch(ctxs):
    k = len(ctxs)
    arr = (C.c_void_p * k)(*ctxs)
    _check(lib().perc_run_batch(arr, k), "perc_run_batch")


def perc_set_params(ctx, L, porosity, seed=0, source=PERC_SOURCE_TOP_ROW, i0=0, j0=0):
    p = perc_params(int(L), float(porosity), int(seed), int(source), int(i0), int(j0))
    _check(lib().perc_set_params(ctx, C.byref(p)), "perc_set_params")


def perc_result_get(ctx, want_hash=False):
    r = perc_result()
    _check(lib().perc_result_get(ctx, C.byref(r), 1 if want_hash else 0), "perc_result_get")
    return r


def perc_copy_medium(ctx, L):
    out = np.empty((L, L), dtype=np.uint8)
    _check(lib().perc_copy_medium(ctx, out.ctypes.data, out.size), "perc_copy_medium")
    return out


def perc_copy_arrival(ctx, L):
    out = np.empty((L, L), dtype=np.int32)
    _check(lib().perc_copy_arrival(ctx, out.ctypes.data, out.size), "perc_copy_arrival")
    return out


def perc_destroy(ctx):
    _check(lib().perc_destroy(ctx), "perc_destroy")


MB_OPS = {"=": 0, "+": 1, "-": 2, "*": 3, "/": 4, "sin": 5, "cos": 6, "log": 7, "exp": 8}
MB_HOST_TO_DEVICE = 0
MB_DEVICE_TO_HOST = 1


def mb_vector_op(op, a_ptr, c_ptr, n, stream=None):
    """op: a key of MB_OPS or its code; a_ptr / c_ptr: device addresses."""
    code = MB_OPS[op] if isinstance(op, str) else int(op)
    _check(lib().mb_vector_op(code, a_ptr, c_ptr, int(n), stream), "mb_vector_op")


def mb_copy_lattice(dst_ptr, src_ptr, L, elem, direction, border=False, stream=None):
    _check(lib().mb_copy_lattice(dst_ptr, src_ptr, int(L), int(elem), int(direction), 1 if border else 0, stream),
           "mb_copy_lattice")


def mb_philox(out_ptr, n_threads, calls_per_thread, seed=0, stream=None):
    _check(lib().mb_philox(out_ptr, int(n_threads), int(calls_per_thread), int(seed), stream), "mb_philox")


def ising_strerror(code):
    return lib().ising_strerror(int(code)).decode()


class Lattice:
    """Convenience owner of one context (destroyed on close / garbage)."""

    def __init__(self, L, J=1.0, h=0.0, T=2.269185, seed=0, p_up=0.5, flags=ISING_PLAN_AUTO, stream=None):
        self.L, self.J, self.h = int(L), float(J), float(h)
        self.ctx = ising_create(L, J, h, T, seed, p_up, flags, stream)

    def sweep(self, n):
        ising_sweep(self.ctx, n)

    def observables(self, want=ISING_OBS_SERIES):
        return ising_observables(self.ctx, want)

    def spins(self):
        return ising_copy_spins(self.ctx, self.L)

    def load(self, spins, t):
        ising_load_spins(self.ctx, spins, t)

    def plan(self):
        return ising_plan_info(self.ctx)

    def close(self):
        if self.ctx:
            ising_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
