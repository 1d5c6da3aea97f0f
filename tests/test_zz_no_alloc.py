"""The allocation-free sweep entry point, ising_sweep_static, against
ising_sweep on identical contexts: the same per-sweep (B, M) and the same
lattice, for calls of decreasing size in a row (each call reuses the
library's device array the previous one left its partial sums in), in
every plan, replayed from a captured graph, plus the size limit of that
array."""
import numpy as np
import pytest

from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def b():
    from paper_cs_0312006_amd import binding
    binding.lib()
    return binding


def _pair(b, L, plan, cw, rows, J, h, T, seed):
    ctxs = []
    for _ in range(2):
        c = b.ising_create(L, J, h, T, seed, 0.5)
        if plan:
            b.ising_plan_set(c, plan, cw, rows)
        ctxs.append(c)
    return ctxs


def _check(b, torch, ref, ctx, L, n, what):
    """n sweeps on ref through ising_sweep and on ctx through
    ising_sweep_static; both must agree bit for bit."""
    b.ising_sweep(ref, n)
    series = torch.full((2 * n,), -7, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    b.ising_sweep_static(ctx, n, series.data_ptr())
    spins = b.ising_copy_spins(ctx, L)  # synchronises the context's stream
    obs_r, B, M = b.ising_observables(ref, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
    obs_s, B_s, _ = b.ising_observables(ctx, b.ISING_OBS_SERIES)
    got = series.cpu().numpy()
    assert np.array_equal(got[0::2], B), f"{what}: bond series differ"
    assert np.array_equal(got[1::2], M), f"{what}: magnetisation series differ"
    assert np.array_equal(spins, b.ising_copy_spins(ref, L)), f"{what}: lattices differ"
    assert obs_s.sweeps_done == obs_r.sweeps_done
    assert B_s is None or len(B_s) == 0, f"{what}: the context's own series must stay empty"


def test_static_sweeps_equal_ising_sweep(b):
    import torch
    cases = [
        # (L, plan, cw, rows, J, h, T, seed, sweeps)
        (8192, b.ISING_PLAN_FUSED_ROWS, 4, 128, 1.0, 0.0, 2.269185, 6, 8),
        (4096, b.ISING_PLAN_FUSED, 4, 32, 1.0, 0.0, 2.269185, 7, 12),
        (2048, b.ISING_PLAN_TWO_PASS, 0, 0, 1.0, 0.1, 2.0, 8, 9),
        (1024, b.ISING_PLAN_FUSED, 1, 8, -1.0, 0.05, 3.0, 9, 7),
        (64, b.ISING_PLAN_RESIDENT, 0, 0, 1.0, 0.0, 2.269185, 10, 6),
        (34, b.ISING_PLAN_GENERIC, 0, 0, 1.0, 0.2, 1.5, 11, 5),
        (4096, b.ISING_PLAN_BANDS, 0, 16, 1.0, 0.0, 2.269185, 12, 10),
        # 256 one-row bands: 256 pairs a sweep, launches of 256 sweeps
        (256, b.ISING_PLAN_BANDS, 0, 1, 1.0, 0.1, 2.0, 13, 600),
        (8192, b.ISING_PLAN_BANDS, 0, 32, -1.0, 0.05, 2.5, 14, 6),  # rows of two 64-word chunks
        (2048, b.ISING_PLAN_BANDS, 0, 8, 1.0, 0.05, 2.269185, 15, 40),  # bands kept as bytes
    ]
    for L, plan, cw, rows, J, h, T, seed, n in cases:
        G.log(f"static scratch L={L} plan={plan}")
        ref, ctx = _pair(b, L, plan, cw, rows, J, h, T, seed)
        try:
            _check(b, torch, ref, ctx, L, n, f"L={L} plan={plan}")
            # a second, shorter call on the same contexts continues exactly
            _check(b, torch, ref, ctx, L, max(1, n // 2), f"L={L} plan={plan}, second call")
        finally:
            b.ising_destroy(ref)
            b.ising_destroy(ctx)


def test_static_sweeps_replayed_from_a_graph(b):
    """ising_sweep_static captured into a graph (the callers it is for) and
    replayed three times from the same start, with the host's own work and
    synchronisations between replays: every replay's series and lattice
    equal the same sweeps run eagerly through ising_sweep. A band-plan
    context is captured as two-pass launches, a fused-plan context as its
    own launches; ising_sweep itself refuses to be captured on the band
    plan."""
    import torch
    n = 8
    for L, plan, cw, rows in [(1024, b.ISING_PLAN_BANDS, 1, 4), (2048, b.ISING_PLAN_FUSED, 1, 8)]:
        G.log(f"static sweeps in a graph L={L} plan={plan}")
        s = torch.cuda.Stream()
        ctx = b.ising_create(L, 1.0, 0.05, 2.3, 41, 0.5, stream=s.cuda_stream)
        ref = b.ising_create(L, 1.0, 0.05, 2.3, 41, 0.5)
        try:
            b.ising_plan_set(ctx, plan, cw, rows)
            b.ising_plan_set(ref, plan, cw, rows)
            start = b.ising_copy_spins(ctx, L)
            b.ising_sweep(ref, n)
            _, B, M = b.ising_observables(ref, b.ISING_OBS_SERIES)
            want = b.ising_copy_spins(ref, L)
            series = torch.full((2 * n,), -7, dtype=torch.int64, device="cuda")
            # one eager call first: the library looks its array up on first use
            b.ising_sweep_static(ctx, n, series.data_ptr())
            b.ising_load_spins(ctx, start, 0)
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=s):
                if plan == b.ISING_PLAN_BANDS:
                    with pytest.raises(b.IsingError) as e:
                        b.ising_sweep(ctx, 1)
                    assert e.value.code == b.ISING_EUNSUPPORTED
                b.ising_sweep_static(ctx, n, series.data_ptr())
            for rep in range(3):
                b.ising_load_spins(ctx, start, 0)
                series.fill_(-7)
                torch.cuda.synchronize()
                graph.replay()
                torch.cuda.synchronize()
                got = series.cpu().numpy()
                assert np.array_equal(got[0::2], B), f"L={L} plan={plan} replay {rep}: bond series differ"
                assert np.array_equal(got[1::2], M), f"L={L} plan={plan} replay {rep}: magnetisation series differ"
                assert np.array_equal(b.ising_copy_spins(ctx, L), want), f"L={L} plan={plan} replay {rep}: lattices"
            del graph
        finally:
            b.ising_destroy(ctx)
            b.ising_destroy(ref)


def test_static_sweeps_reject_plans_beyond_the_array(b):
    """A tiling with more partial slots than the array holds is refused
    before anything is launched, and the context stays usable."""
    import torch
    L = 16384
    ctx = b.ising_create(L, 1.0, 0.0, 2.269185, 3, 0.5)
    try:
        b.ising_plan_set(ctx, b.ISING_PLAN_FUSED, 1, 4)  # 131072 tiles: 262144 pairs
        series = torch.zeros(2, dtype=torch.int64, device="cuda")
        with pytest.raises(b.IsingError) as e:
            b.ising_sweep_static(ctx, 1, series.data_ptr())
        assert e.value.code == b.ISING_ERANGE
        b.ising_plan_set(ctx, b.ISING_PLAN_FUSED, 4, 32)  # 8192 tiles
        b.ising_sweep_static(ctx, 1, series.data_ptr())
        obs, _, _ = b.ising_observables(ctx, 0)
        assert obs.sweeps_done == 1
    finally:
        b.ising_destroy(ctx)
