"""The batch autotuner on the GPU: it times every lattice class, keeps the
rates in a cache file keyed by the device and loads them from there, the
plan ISING_BATCH_AUTO then runs is the one its model predicts faster, and
the results of the tuned plan equal the oracle's."""
import numpy as np
import pytest

from paper_cs_0312006_amd import workloads as W
from tests import gpu_util as G

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


@pytest.fixture(scope="module")
def tuned(b, tmp_path_factory):
    path = tmp_path_factory.mktemp("tune") / "rates.txt"
    G.log("batch tune: timing every class")
    hit = b.ising_batch_tune(0, str(path))
    return path, hit


def test_tune_times_then_loads_from_its_cache(b, tuned):
    path, hit = tuned
    assert not hit
    text = path.read_text().splitlines()
    assert text[0].startswith("ising-batch-rates 2 gfx950")
    assert len([ln for ln in text if ln.startswith("class ")]) == 10
    rows, is_tuned, floor_ns = b.ising_batch_rates(0)
    assert is_tuned and floor_ns > 0
    for r in rows:
        assert r["resident_per_workgroup"] > 0 and all(x > 0 for x in r["stepped"])
    G.log("batch tune: rates " + " | ".join(
        f"{r['max_side']}{'h' if r['field'] else ''}: {r['resident_per_workgroup']:.2f}/wg "
        f"+{r['resident_fixed_ns'] / 1e3:.1f}us {'/'.join(f'{x:.0f}' for x in r['stepped'])}" for r in rows)
        + f" floor {floor_ns:.0f} ns")
    # a second call loads the same rates from the file
    assert b.ising_batch_tune(0, str(path))
    rows2, _, floor2 = b.ising_batch_rates(0)
    for r, r2 in zip(rows, rows2):
        assert r2["resident_per_workgroup"] == pytest.approx(r["resident_per_workgroup"], rel=1e-5)
        assert r2["resident_fixed_ns"] == pytest.approx(r["resident_fixed_ns"], rel=1e-5, abs=1e-3)
        assert r2["stepped"] == pytest.approx(r["stepped"], rel=1e-5)
    assert floor2 == pytest.approx(floor_ns, rel=1e-5)


def test_cache_of_another_device_is_not_used(b, tuned, tmp_path):
    path, _ = tuned
    lines = path.read_text().splitlines()
    other = tmp_path / "other.txt"
    other.write_text("\n".join([lines[0].replace("gfx950", "gfx000")] + lines[1:]) + "\n")
    G.log("batch tune: cache keyed by another device is re-timed")
    assert not b.ising_batch_tune(0, str(other))
    assert open(other).readline().startswith("ising-batch-rates 2 gfx950")


def _ctxs(b, runs):
    return [b.ising_create(r.L, r.J, r.h, r.T, r.seed, r.p_up) for r in runs]


def test_auto_plan_follows_the_model(b, tuned):
    """For batches of different make-up the plan the model names is the one
    with the smaller predicted time, and tile heights are 8, 16 or 32."""
    rng = np.random.default_rng(3)
    cases = [[W.Run(L=64, seed=k) for k in range(32)],
             [W.Run(L=512, h=0.05, T=2.0, seed=k) for k in range(300)],
             [W.Run(L=1024, h=0.05, T=2.0, seed=k) for k in range(300)],
             [W.Run(L=2048, seed=k) for k in range(4)],
             [W.Run(L=int(16 * rng.integers(2, 65)), h=float(rng.choice([0.0, 0.05])), seed=k)
              for k in range(200)]]
    for runs in cases:
        ctxs = _ctxs(b, runs)
        try:
            plan, rows, (t_res, t_st) = b.ising_batch_choice(ctxs, [100] * len(ctxs))
        finally:
            for c in ctxs:
                b.ising_destroy(c)
        G.log(f"batch choice: {len(runs)} lattices, sides {runs[0].L}..{max(r.L for r in runs)}: "
              f"plan {plan} rows {rows} resident {t_res / 1e6:.2f} ms stepped {t_st / 1e6:.2f} ms")
        assert plan == (b.ISING_BATCH_STEPPED if t_st < t_res else b.ISING_BATCH_RESIDENT)
        assert rows in (8, 16, 32)
        assert t_res > 0 and t_st > 0


def test_tuned_auto_plan_equals_oracle(b, o, tuned):
    """A mixed batch (sides 16 to 1088, h = 0 and h != 0, J of both signs)
    run with the tuned AUTO plan, twice in a row: every lattice equals the
    oracle's run of it alone."""
    rng = np.random.default_rng(11)
    runs = []
    for k in range(48):
        L = int(16 * rng.integers(1, 69))
        runs.append(W.Run(L=L, J=float(rng.choice([1.0, -1.0, 0.5])), h=float(rng.choice([0.0, 0.05, -0.2])),
                          T=float(rng.uniform(1.0, 4.0)), seed=int(rng.integers(0, 2 ** 63)),
                          p_up=float(rng.choice([0.5, 1.0])), sweeps=int(rng.integers(1, 30))))
    ctxs = _ctxs(b, runs)
    try:
        choice = b.ising_batch_choice(ctxs, [r.sweeps for r in runs])
        G.log(f"tuned AUTO batch of 48: plan {choice[0]} rows {choice[1]}")
        b.ising_sweep_batch(ctxs, [r.sweeps for r in runs])
        extra = [int(rng.integers(0, 20)) for _ in runs]
        b.ising_sweep_batch(ctxs, extra)
        for r, ctx, e in zip(runs, ctxs, extra):
            obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
            spins = b.ising_copy_spins(ctx, r.L)
            G.assert_same({"spins": spins, "B": B, "M": M, "hash": obs.lattice_hash},
                          G.oracle_run(o, r, sweeps=r.sweeps + e), f"tuned AUTO L={r.L} h={r.h} J={r.J}")
    finally:
        for c in ctxs:
            b.ising_destroy(c)
