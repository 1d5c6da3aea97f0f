"""GPU parity of the percolation engine (Section 2.3) through the C ABI:
medium, arrival map and summary bit-exact against the oracle on seeded
media; at the full 32768^2 size, sampled draws against the NumPy Philox and
the local conditions that fix breadth-first arrival passes uniquely."""
import numpy as np
import pytest

from oracle import mini
from paper_cs_0312006_amd import workloads as W
from tests import gpu_util as G
from tests.perc_checks import check_arrival_local

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def b():
    from paper_cs_0312006_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def o():
    from oracle import ref
    orc = ref.Oracle()
    orc.set_threads(G.host_threads())
    return orc


def _gpu(b, m, want_hash=True):
    ctx = b.perc_create(m.L, m.porosity, m.seed, m.source, m.i0, m.j0)
    try:
        b.perc_run(ctx)
        r = b.perc_result_get(ctx, want_hash)
        return r, b.perc_copy_medium(ctx, m.L), b.perc_copy_arrival(ctx, m.L)
    finally:
        b.perc_destroy(ctx)


CASES = [
    W.Medium(1, 0.5, 1), W.Medium(1, 1.0, 1, 1, 0, 0), W.Medium(7, 0.6, 2), W.Medium(63, 0.6, 3),
    W.Medium(64, 0.5927, 4), W.Medium(65, 0.65, 5, 1, 32, 40), W.Medium(100, 0.7, 6, 1, 99, 0),
    W.Medium(128, 0.55, 7), W.Medium(130, 1.0, 8), W.Medium(64, 0.0, 9), W.Medium(257, 0.6, 10),
    W.PERC_FIG3, W.Medium(512, 0.5927, 12, 1, 256, 256), W.Medium(1000, 0.6, 13), W.Medium(2048, 0.62, 14),
]


@pytest.mark.parametrize("m", CASES, ids=lambda m: f"L{m.L}-P{m.porosity}-s{m.seed}-src{m.source}")
def test_percolation_parity(b, o, m):
    G.log(f"percolation {m}")
    r, pore, arr = _gpu(b, m)
    pore_o = o.perc_medium(m.L, m.porosity, m.seed)
    assert np.array_equal(pore, pore_o), "medium differs"
    arr_o = o.perc_invade(pore_o, m.source, m.i0, m.j0)
    if not np.array_equal(arr, arr_o):
        bad = np.argwhere(arr != arr_o)
        raise AssertionError(f"{len(bad)} arrival passes differ, first {bad[:5].tolist()}")
    inv, mx, sp = o.perc_summary(arr_o)
    assert (r.pores, r.invaded, r.passes, r.spans) == (int(pore_o.sum()), inv, mx, sp)
    assert r.arrival_hash == o.fnv1a64(arr_o)


def test_rerun_and_errors(b):
    m = W.Medium(96, 0.6, 5)
    ctx = b.perc_create(m.L, m.porosity, m.seed)
    try:
        with pytest.raises(b.IsingError) as e:
            b.perc_result_get(ctx)
        assert e.value.code == b.ISING_ESTATE
        b.perc_run(ctx)
        r1 = b.perc_result_get(ctx, True)
        b.perc_run(ctx)
        r2 = b.perc_result_get(ctx, True)
        assert (r1.arrival_hash, r1.invaded, r1.passes) == (r2.arrival_hash, r2.invaded, r2.passes)
    finally:
        b.perc_destroy(ctx)
    for kw in (dict(L=0, porosity=0.5), dict(L=65537, porosity=0.5), dict(L=8, porosity=1.5),
               dict(L=8, porosity=float("nan")), dict(L=8, porosity=0.5, source=2),
               dict(L=8, porosity=0.5, source=1, i0=8)):
        with pytest.raises(b.IsingError) as e:
            b.perc_create(**kw)
        assert e.value.code == b.ISING_EINVAL


def test_full_size_medium_and_arrival(b):
    """32768 x 32768 at porosity 0.6 (the configuration bench.py times): 4096
    sampled sites of the medium equal the NumPy Philox draw; the arrival map
    satisfies the local conditions of breadth-first distances; the summary
    equals the one recomputed from the copied maps."""
    m = W.PERC_HEADLINE
    G.log(f"percolation full size {m}")
    r, pore, arr = _gpu(b, m, want_hash=False)
    rng = np.random.default_rng(0)
    ords = rng.integers(0, m.L * m.L, size=4096, dtype=np.uint64)
    words = mini.philox4x32_10(ords >> np.uint64(2), 0, 0, 2, m.seed & 0xFFFFFFFF, m.seed >> 32)
    u = np.choose((ords & np.uint64(3)).astype(np.int64), words)
    expect = (u < np.uint64(int(np.floor(m.porosity * 2.0 ** 32)))).astype(np.uint8)
    assert np.array_equal(pore.ravel()[ords.astype(np.int64)], expect)
    G.log("percolation full size: local conditions")
    check_arrival_local(pore, arr, m.source)
    inv = arr >= 0
    spans = (1 if inv[0].any() and inv[-1].any() else 0) | (2 if inv[:, 0].any() and inv[:, -1].any() else 0)
    assert (r.pores, r.invaded, r.passes, r.spans) == (int(pore.sum(dtype=np.int64)), int(inv.sum()),
                                                      int(arr.max()), spans)


def _span_threshold_gpu(b, L, seed, lo=0.3, hi=0.9, iters=14):
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        ctx = b.perc_create(L, mid, seed)
        try:
            b.perc_run(ctx)
            sp = b.perc_result_get(ctx).spans & 1
        finally:
            b.perc_destroy(ctx)
        lo, hi = (lo, mid) if sp else (mid, hi)
    return hi


def test_spanning_thresholds_equal_oracle(b, o):
    """Section 2.3's question, the porosity from which a spanning cluster
    exists: per-seed spanning thresholds of 128 x 128 media found by
    bisection on the GPU equal the oracle's exactly, and their median lies
    near p_c = 0.592746."""
    from tests.test_oracle_percolation import _span_threshold
    G.log("spanning thresholds, 40 media of 128^2")
    gpu = [_span_threshold_gpu(b, 128, s) for s in range(40)]
    cpu = [_span_threshold(o, 128, s) for s in range(40)]
    assert gpu == cpu
    assert abs(float(np.median(gpu)) - 0.592746) < 0.012


BATCH = [W.Medium(1, 0.5, 21), W.Medium(7, 0.6, 22), W.Medium(64, 0.5927, 23), W.Medium(65, 0.65, 24, 1, 32, 40),
         W.Medium(130, 1.0, 25), W.Medium(257, 0.6, 26), W.Medium(512, 0.55, 27, 1, 500, 3),
         W.Medium(200, 0.0, 28), W.Medium(512, 0.6, 29)]


def test_batch_equals_oracle_and_single_runs(b, o):
    """Nine media of mixed sides, porosities and sources in one batched run:
    each arrival map equals the oracle's and each summary the one of the
    same medium run alone."""
    G.log("percolation batch of 9 media")
    ctxs = [b.perc_create(m.L, m.porosity, m.seed, m.source, m.i0, m.j0) for m in BATCH]
    try:
        b.perc_run_batch(ctxs)
        got = [(b.perc_result_get(c, True), b.perc_copy_arrival(c, m.L)) for c, m in zip(ctxs, BATCH)]
    finally:
        for c in ctxs:
            b.perc_destroy(c)
    for (r, arr), m in zip(got, BATCH):
        arr_o = o.perc_invade(o.perc_medium(m.L, m.porosity, m.seed), m.source, m.i0, m.j0)
        assert np.array_equal(arr, arr_o), f"{m}: arrival differs"
        solo, _, _ = _gpu(b, m)
        assert (r.arrival_hash, r.invaded, r.passes, r.spans, r.pores) == (
            solo.arrival_hash, solo.invaded, solo.passes, solo.spans, solo.pores)


def test_set_params_and_batch_errors(b, o):
    ctx = b.perc_create(96, 0.5, 1)
    other = b.perc_create(64, 0.5, 1)
    try:
        b.perc_set_params(ctx, 96, 0.62, 7, b.PERC_SOURCE_POINT, 40, 41)
        b.perc_run(ctx)
        arr = b.perc_copy_arrival(ctx, 96)
        pore = o.perc_medium(96, 0.62, 7)
        assert np.array_equal(arr, o.perc_invade(pore, 1, 40, 41))
        for bad in (dict(L=95, porosity=0.5), dict(L=96, porosity=1.5), dict(L=96, porosity=0.5, source=1, i0=96)):
            with pytest.raises(b.IsingError) as e:
                b.perc_set_params(ctx, **bad)
            assert e.value.code == b.ISING_EINVAL
        with pytest.raises(b.IsingError) as e:
            b.perc_run_batch([ctx, other, ctx])
        assert e.value.code == b.ISING_EINVAL
        b.perc_run_batch([])
    finally:
        b.perc_destroy(ctx)
        b.perc_destroy(other)


def test_batched_spanning_thresholds_equal_oracle(b, o):
    """The spanning-threshold bisection run for 40 media of 128^2 at once
    (one batched run per bisection step, porosities changed in place)
    gives the oracle's per-seed thresholds exactly."""
    from tests.test_oracle_percolation import _span_threshold
    n, L = 40, 128
    G.log("batched spanning thresholds, 40 media of 128^2")
    lo, hi = np.full(n, 0.3), np.full(n, 0.9)
    ctxs = [b.perc_create(L, 0.5, s) for s in range(n)]
    try:
        for _ in range(14):
            mid = 0.5 * (lo + hi)
            for s, c in enumerate(ctxs):
                b.perc_set_params(c, L, float(mid[s]), s)
            b.perc_run_batch(ctxs)
            sp = np.array([b.perc_result_get(c).spans & 1 for c in ctxs], dtype=bool)
            hi = np.where(sp, mid, hi)
            lo = np.where(sp, lo, mid)
    finally:
        for c in ctxs:
            b.perc_destroy(c)
    assert list(hi) == [_span_threshold(o, L, s) for s in range(n)]
