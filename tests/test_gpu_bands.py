"""GPU parity of the band-resident plan against the oracle: lattice sides
with full and partial last bit words, band heights from one row (a wave
that holds both edges of its band) to 32 rows and ragged bands (heights
differing by one), h = 0 and h != 0, J < 0, zero thresholds, cold and
hot starts, calls that cross the per-launch sweep limit, switches into
and out of the plan (which reuse or regrow its edge slots and flags), and
calls after a batched sweep moved the lattice."""
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


def _bands(b, run, rows, chunks, per_wave=1):
    ctx = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up)
    try:
        b.ising_plan_set(ctx, b.ISING_PLAN_BANDS, per_wave, rows)
        assert b.ising_plan_info(ctx) == (b.ISING_PLAN_BANDS, per_wave, rows)
        for k in chunks:
            b.ising_sweep(ctx, k)
        obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
        spins = b.ising_copy_spins(ctx, run.L)
    finally:
        b.ising_destroy(ctx)
    return {"spins": spins, "B": B, "M": M, "hash": obs.lattice_hash}


CASES = [
    # L, J, h, T, p_up, seed, band rows, rows a wave, calls
    (16, 1.0, 0.0, 2.269185, 0.5, 3, 1, 1, [4, 5]),       # 16 one-row bands
    (16, 1.0, 0.1, 2.0, 0.5, 4, 8, 1, [9]),               # two bands
    (16, 1.0, 0.1, 2.0, 0.5, 4, 8, 4, [9]),               # two bands of two waves
    (64, 1.0, 0.0, 2.269185, 0.5, 5, 3, 1, [6, 1, 5]),    # 22 bands of 2 or 3 rows
    (64, 1.0, 0.0, 2.269185, 0.5, 5, 3, 2, [6, 1, 5]),    # one wave holding both edges of a 2-row band
    (136, 1.0, 0.1, 1.8, 0.5, 7, 4, 1, [7, 5]),           # 17 quads a row: 4 valid bits in the last word
    (256, -1.0, 0.0, 2.0, 1.0, 9, 16, 1, [12]),           # J < 0, cold start
    (512, 0.5, -0.2, 2.5, 0.3, 11, 8, 1, [5, 7]),
    (520, 1.0, 0.0, 2.269185, 0.5, 19, 7, 2, [4, 4]),     # 75 bands of 6 or 7 rows, waves of 2 rows
    (1000, 1.0, 0.0, 2.269185, 0.5, 12, 5, 1, [6, 6]),    # 125 quads a row: 20 valid bits in the last word
    (1024, 1.0, 0.0, 0.2, 0.5, 13, 16, 1, [10]),          # zero thresholds
    (2048, 1.0, 0.05, 2.269185, 0.5, 15, 32, 1, [4, 8]),  # 16 waves of 2 rows
    (2048, 1.0, 0.05, 2.269185, 0.5, 15, 32, 4, [4, 8]),
    (4096, 1.0, 0.0, 2.269185, 0.5, 7, 16, 1, [5, 7]),
    (4096, 1.0, 0.0, 2.269185, 0.5, 7, 16, 2, [5, 7]),
    (4096, 1.0, 0.1, 1.5, 0.5, 17, 8, 1, [6, 6]),
    (4096, 1.0, 0.0, 1e300, 0.5, 18, 4, 1, [3]),          # every proposal accepted
    (4104, 1.0, 0.1, 2.0, 0.5, 20, 17, 1, [3, 2]),        # 65-word rows (a second chunk of one word), 17-row bands
    (8192, 1.0, 0.0, 2.269185, 0.5, 21, 32, 1, [2, 3]),   # two chunks a row, two rows a wave
    (16384, -1.0, 0.05, 2.5, 0.5, 22, 64, 1, [2, 1]),     # four chunks a row, 128 KiB of LDS a band
]


@pytest.mark.parametrize("L,J,h,T,p_up,seed,rows,per_wave,chunks", CASES)
def test_bands_equal_oracle(b, o, L, J, h, T, p_up, seed, rows, per_wave, chunks):
    run = W.Run(L=L, J=J, h=h, T=T, seed=seed, p_up=p_up, sweeps=sum(chunks))
    G.log(f"bands L={L} rows={rows} per_wave={per_wave} J={J} h={h} T={T} calls={chunks}")
    G.assert_same(_bands(b, run, rows, chunks, per_wave), G.oracle_run(o, run), f"bands L={L} rows={rows}")


def test_bands_across_launch_limit(b, o):
    """1100 sweeps in two calls: launches of at most 512 sweeps, each
    resuming from the flags the previous one left."""
    run = W.Run(L=64, h=0.05, T=2.4, seed=21, sweeps=1100)
    G.log("bands L=64 1100 sweeps in calls of 600 and 500")
    G.assert_same(_bands(b, run, 2, [600, 500]), G.oracle_run(o, run), "bands 1100 sweeps")


def test_switches_into_and_out_of_bands(b, o):
    run = W.Run(L=512, h=0.02, T=2.3, seed=23, sweeps=24)
    ref = G.oracle_run(o, run)
    ctx = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up)
    try:
        steps = [(b.ISING_PLAN_FUSED_ROWS, 0, 0, 5), (b.ISING_PLAN_BANDS, 2, 16, 6), (b.ISING_PLAN_TWO_PASS, 0, 0, 4),
                 (b.ISING_PLAN_BANDS, 0, 4, 3), (b.ISING_PLAN_BANDS, 0, 32, 2), (b.ISING_PLAN_FUSED, 0, 0, 4)]
        for plan, cw, rows, n in steps:
            G.log(f"switch to plan {plan} rows {rows} for {n} sweeps")
            b.ising_plan_set(ctx, plan, cw, rows)
            b.ising_sweep(ctx, n)
        obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
        got = {"spins": b.ising_copy_spins(ctx, run.L), "B": B, "M": M, "hash": obs.lattice_hash}
    finally:
        b.ising_destroy(ctx)
    G.assert_same(got, ref, "plan switches through bands")


def test_bands_after_batched_sweeps(b, o):
    """A stepped batch leaves the lattice in the other buffer; the band plan
    then continues from there."""
    runs = [W.Run(L=1024, seed=31 + k, T=2.0 + 0.3 * k, sweeps=9) for k in range(3)]
    ctxs = [b.ising_create(r.L, r.J, r.h, r.T, r.seed, r.p_up) for r in runs]
    try:
        for c in ctxs:
            b.ising_plan_set(c, b.ISING_PLAN_BANDS, 0, 16)
            b.ising_sweep(c, 2)
        G.log("bands then stepped batch then bands")
        b.ising_sweep_batch_plan(ctxs, [4] * 3, plan=b.ISING_BATCH_STEPPED)
        for c in ctxs:
            b.ising_sweep(c, 3)
        for r, c in zip(runs, ctxs):
            obs, B, M = b.ising_observables(c, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
            got = {"spins": b.ising_copy_spins(c, r.L), "B": B, "M": M, "hash": obs.lattice_hash}
            G.assert_same(got, G.oracle_run(o, r), f"bands around a batch T={r.T}")
    finally:
        for c in ctxs:
            b.ising_destroy(c)


def test_band_plan_limits(b):
    """Sides whose rows are wider than 256 words (32768: 512), band heights
    that need more bands than can be resident at once (8192 with 16-row
    bands: 512), and heights that leave fewer than two bands are refused;
    the context keeps its plan."""
    for L, rows in ((32768, 128), (8192, 16), (64, 64)):
        ctx = b.ising_create(L, 1.0, 0.0, 2.269185, 1, 0.5)
        try:
            before = b.ising_plan_info(ctx)
            with pytest.raises(b.IsingError) as e:
                b.ising_plan_set(ctx, b.ISING_PLAN_BANDS, 0, rows)
            assert e.value.code == b.ISING_EUNSUPPORTED, (L, rows)
            assert b.ising_plan_info(ctx) == before
        finally:
            b.ising_destroy(ctx)


def test_single_lattice_batches_run_on_bands(b, o):
    """ISING_BATCH_AUTO with one lattice to sweep (sides the band plan
    serves; other contexts of the batch with no sweeps): the band plan runs
    it, on an explicit stream or the library's, in order with the batches
    before and after that include the same context, and every context
    equals the oracle."""
    import torch
    runs = [W.Run(L=512, h=0.05, T=2.3, seed=51, sweeps=14), W.Run(L=1088, T=2.5, seed=52, sweeps=14),
            W.Run(L=64, seed=53, sweeps=14)]
    ctxs = [b.ising_create(r.L, r.J, r.h, r.T, r.seed, r.p_up, b.ISING_PLAN_TWO_PASS) for r in runs]
    s = torch.cuda.Stream()
    try:
        G.log("batch of three, then single-lattice batches, then a batch of three")
        b.ising_sweep_batch_plan(ctxs, [3, 3, 3], b.ISING_BATCH_AUTO)
        b.ising_sweep_batch_plan(ctxs, [5, 0, 0], b.ISING_BATCH_AUTO, stream=s.cuda_stream)
        b.ising_sweep_batch_plan(ctxs, [0, 5, 0], b.ISING_BATCH_AUTO)
        b.ising_sweep_batch_plan(ctxs, [0, 0, 5], b.ISING_BATCH_AUTO)  # 64: a batch plan
        b.ising_sweep_batch_plan(ctxs, [6, 6, 6], b.ISING_BATCH_AUTO, stream=s.cuda_stream)
        torch.cuda.synchronize()
        for r, c in zip(runs, ctxs):
            assert b.ising_plan_info(c)[0] == b.ISING_PLAN_TWO_PASS  # the context's own plan is kept
            obs, B, M = b.ising_observables(c, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
            got = {"spins": b.ising_copy_spins(c, r.L), "B": B, "M": M, "hash": obs.lattice_hash}
            G.assert_same(got, G.oracle_run(o, r), f"single-lattice batches L={r.L}")
    finally:
        for c in ctxs:
            b.ising_destroy(c)
