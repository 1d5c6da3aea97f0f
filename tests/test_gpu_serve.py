"""GPU tests of the request server: results are the same alone and in the
mix (bit-exact lattice hashes, identical FP64 averages of identical integer
series), under continuous batching and under a tight HBM budget; small
requests also match the oracle."""
import numpy as np
import pytest

from paper_cs_0312006_amd import serve
from paper_cs_0312006_amd import workloads as W
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def b():
    from paper_cs_0312006_amd import binding
    binding.lib()
    return binding


def _solo(b, run):
    ctx = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up)
    try:
        b.ising_sweep(ctx, run.sweeps)
        obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
    finally:
        b.ising_destroy(ctx)
    half = len(B) // 2
    avg = b.ising_series_averages(B[half:], M[half:], run.L, run.J, run.h)
    return obs.lattice_hash, obs.bond_sum, obs.mag_sum, avg.e, avg.abs_m


@pytest.mark.parametrize("budget,epoch", [(8 << 30, 16), (3 * 512 * 512, 7)])
def test_served_results_equal_solo_results(b, budget, epoch):
    reqs = W.request_stream(2000.0, count=24, rng_seed=11, sweeps_range=(40, 300), side_units=(1, 8))
    G.log(f"serve 24 requests budget={budget} epoch={epoch}")
    ex = serve.GpuExecutor()
    try:
        res, stats = serve.serve(reqs, ex, hbm_budget=budget, epoch_sweeps=epoch)
    finally:
        ex.close()
    assert len(res) == 24 and all(not r.error for r in res)
    assert stats["epochs"] > 1
    for r in res:
        run = reqs[r.rid].run
        h, bs, ms, e, am = _solo(b, run)
        assert (r.lattice_hash, r.bond_sum, r.mag_sum) == (h, bs, ms), f"request {r.rid} L={run.L}"
        assert r.e_mean == e and r.abs_m_mean == am
    s = serve.summarize(res, stats["makespan_s"])
    assert s["completed"] == 24 and s["p99_s"] >= s["p50_s"]


def test_served_small_requests_match_oracle(b):
    from oracle import ref
    o = ref.Oracle()
    o.set_threads(G.host_threads())
    reqs = W.request_stream(5000.0, count=8, rng_seed=4, sweeps_range=(20, 60), side_units=(1, 2))
    G.log("serve 8 small requests vs oracle")
    ex = serve.GpuExecutor()
    try:
        res, _ = serve.serve(reqs, ex, epoch_sweeps=9)
    finally:
        ex.close()
    for r in res:
        run = reqs[r.rid].run
        s = o.init(run.L, run.seed, run.p_up)
        B, M = o.run(s, run.J, run.h, run.T, run.seed, 0, run.sweeps)
        assert r.lattice_hash == o.fnv1a64(s)
        assert (r.bond_sum, r.mag_sum) == (int(B[-1]), int(M[-1]))
