"""CPU-only checks of the C ABI library: it loads, exports every entry point
include/ising.h declares, and its host-side logic (argument validation,
sizes, error strings, series averages) behaves as documented. No call here
reaches a GPU."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def declared_functions():
    """Every function declared in include/*.h."""
    names = set()
    for h in sorted(os.listdir(INCLUDE)):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(INCLUDE, h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"^\s*(?:const\s+)?[\w ]+\**\s*\**\b((?:ising|perc|mb)_\w+)\s*\(", text, re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def b():
    from paper_cs_0312006_amd import binding
    binding.lib()
    return binding


def test_header_declares_the_four_core_calls():
    names = declared_functions()
    for core in ("ising_create", "ising_sweep", "ising_observables", "ising_destroy", "perc_create", "perc_run"):
        assert core in names


def test_binding_constants_equal_the_headers(b):
    """Every integer #define of include/*.h that the binding mirrors under
    the same name has the same value there."""
    checked = 0
    for h in sorted(os.listdir(INCLUDE)):
        if not h.endswith(".h"):
            continue
        for name, val in re.findall(r"^#define\s+(\w+)\s+\(?(-?(?:0x[0-9a-fA-F]+|\d+))u?\)?",
                                    open(os.path.join(INCLUDE, h)).read(), re.M):
            if hasattr(b, name):
                assert getattr(b, name) == int(val, 0), name
                checked += 1
    assert checked >= 20


def test_library_exports_every_declared_symbol(b):
    names = declared_functions()
    assert len(names) >= 10
    lib = b.lib()
    for name in names:
        assert hasattr(lib, name), name
        assert name in b.SIGNATURES, name


def test_state_bytes(b):
    assert b.ising_state_bytes(64) == 64 * 64
    assert b.ising_state_bytes(6) == 36
    assert b.ising_state_bytes(3) == 0
    assert b.ising_state_bytes(0) == 0
    assert b.ising_state_bytes(65538) == 0
    assert b.ising_state_bytes(10, b.ISING_PLAN_TWO_PASS) == 0  # 10 % 8 != 0
    assert b.ising_state_bytes(16, b.ISING_PLAN_TWO_PASS) == 256


@pytest.mark.parametrize("kw", [
    dict(L=3), dict(L=0), dict(L=1), dict(L=65538), dict(L=64, T=0.0), dict(L=64, T=-1.0),
    dict(L=64, T=float("nan")), dict(L=64, T=float("inf")), dict(L=64, J=float("nan")),
    dict(L=64, h=float("inf")), dict(L=64, p_up=-0.1), dict(L=64, p_up=1.5),
    dict(L=64, p_up=float("nan")), dict(L=64, flags=99),
])
def test_create_rejects_invalid_parameters(b, kw):
    with pytest.raises(b.IsingError) as e:
        b.ising_create(**kw)
    assert e.value.code == b.ISING_EINVAL


def test_forced_plan_that_cannot_serve_is_unsupported(b):
    with pytest.raises(b.IsingError) as e:
        b.ising_create(L=10, flags=b.ISING_PLAN_TWO_PASS)
    assert e.value.code == b.ISING_EUNSUPPORTED


def test_null_handles(b):
    lib = b.lib()
    assert lib.ising_sweep(None, 1) == b.ISING_EINVAL
    assert lib.ising_observables(None, None, None, None, 0, 0) == b.ISING_EINVAL
    assert lib.ising_copy_spins(None, None, 0) == b.ISING_EINVAL
    assert lib.ising_destroy(None) == b.ISING_OK
    assert lib.ising_create(None, None, None) == b.ISING_EINVAL
    assert lib.ising_create_in(None, None, 0, None, None) == b.ISING_EINVAL


def test_strerror(b):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert b.ising_strerror(code)
    assert b.ising_strerror(-100) == "unknown error"


def test_series_averages_match_plain_sums(b):
    """Host FP64 averages of the integer series (Eq. (1) as a time average),
    compared with NumPy to 1e-12 relative."""
    rng = np.random.default_rng(0)
    L, J, h = 64, 1.0, 0.1
    N = L * L
    B = 4 * rng.integers(-N // 2, N // 2, size=5000)
    M = 2 * rng.integers(-N // 2, N // 2, size=5000)
    avg = b.ising_series_averages(B, M, L, J, h)
    E = (-J * B.astype(np.float64) - h * M.astype(np.float64)) / N
    m = M.astype(np.float64) / N
    for got, want in ((avg.e, E.mean()), (avg.e2, (E * E).mean()), (avg.m, m.mean()),
                      (avg.abs_m, np.abs(m).mean()), (avg.m2, (m * m).mean())):
        assert got == pytest.approx(want, rel=1e-12, abs=1e-15)
    assert avg.n == 5000


def test_series_averages_rejects_empty(b):
    with pytest.raises(b.IsingError):
        b.ising_series_averages(np.zeros(0, np.int64), np.zeros(0, np.int64), 8)


def test_microbench_rejects_bad_arguments(b):
    """Argument checks that return before any device work."""
    lib = b.lib()
    assert lib.mb_vector_op(9, 16, 16, 4, None) == b.ISING_EINVAL     # unknown op
    assert lib.mb_vector_op(1, None, 16, 4, None) == b.ISING_EINVAL   # no a
    assert lib.mb_vector_op(1, 16, None, 4, None) == b.ISING_EINVAL   # c read but NULL
    assert lib.mb_vector_op(1, 20, 16, 4, None) == b.ISING_EINVAL     # misaligned
    assert lib.mb_vector_op(5, 16, None, 0, None) == b.ISING_OK       # empty
    assert lib.mb_copy_lattice(None, 16, 4, 1, 0, 0, None) == b.ISING_EINVAL
    assert lib.mb_copy_lattice(16, 16, 0, 1, 0, 0, None) == b.ISING_EINVAL
    assert lib.mb_copy_lattice(16, 16, 4, 1, 2, 0, None) == b.ISING_EINVAL


def test_percolation_rejects_bad_parameters(b):
    for kw in (dict(L=0, porosity=0.5), dict(L=65537, porosity=0.5), dict(L=8, porosity=-0.1),
               dict(L=8, porosity=float("nan")), dict(L=8, porosity=0.5, source=2),
               dict(L=8, porosity=0.5, source=1, j0=8)):
        with pytest.raises(b.IsingError) as e:
            b.perc_create(**kw)
        assert e.value.code == b.ISING_EINVAL


def test_device_error_of_null_context_is_empty(b):
    assert b.lib().ising_device_error(None) == b""


def test_batch_rates_before_tuning(b):
    """Until a device is tuned the batch model uses the built-in rates: ten
    classes (five side bands, without and with a field), every rate
    positive, the bands in increasing side order, the last open-ended."""
    rows, tuned, floor_ns = b.ising_batch_rates(0)
    assert not tuned and floor_ns > 0
    assert [r["field"] for r in rows] == [0, 1] * 5
    sides = [r["max_side"] for r in rows[::2]]
    assert sides == [128, 256, 512, 1072, b.ISING_MAX_L]
    for r in rows:
        assert r["resident_per_workgroup"] > 0 and all(x > 0 for x in r["stepped"])
    lib = b.lib()
    out = (b.ising_batch_rate * 10)()
    assert lib.ising_batch_rates(0, out, 9, None, None) == b.ISING_EINVAL
    assert lib.ising_batch_rates(-1, out, 10, None, None) == b.ISING_EINVAL
    assert lib.ising_batch_tune(0, None, 2, None) == b.ISING_EINVAL  # unknown flag
    assert b.lib().ising_strerror(b.ISING_EIO)
