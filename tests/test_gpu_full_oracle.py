"""Whole-configuration parity: the HIP path against independent oracle runs
of the same full configurations, element by element.

- the three 4096 x 4096 runs over all 2000 sweeps (final lattice, hash and
  every (B_t, M_t)), in the default plan and in the autotuned plan the
  benchmark times;
- the four 32768 x 32768 runs after their first 8 sweeps (the whole 1 GiB
  lattice, hash and series), in every fused tile shape the autotuner can
  pick at that side;
- the batched configuration: the largest lattices (side 1024) and lattices
  of every size band, over all 10000 sweeps, in both batch plans (these
  results are computed once by the oracle and shared by both plans).
"""
import numpy as np
import pytest

from paper_cs_0312006_amd import workloads as W
from tests import gpu_util as G
from tests import physics

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


def _ctx_result(b, ctx, L):
    obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
    return {"spins": b.ising_copy_spins(ctx, L), "B": B, "M": M, "hash": obs.lattice_hash}


@pytest.mark.parametrize("k", [0, 1, 2])
def test_c1_4096_all_2000_sweeps(b, o, k):
    """4096 x 4096 at T in {1.5, 2.269185, 3.5}, seed 7, 2000 sweeps: the
    final lattice, its hash and all 2000 (B_t, M_t) equal a full oracle run,
    in the default plan (band-resident), in the plan the autotuner picks
    (50-sweep trials, as the benchmark does) and in the fused wave-tile
    plan."""
    run = W.C1[k]
    G.log(f"C1 4096 T={run.T} 2000 sweeps: oracle")
    ref = G.oracle_run(o, run)
    for how in ("default", "tuned", "fused"):
        G.log(f"C1 4096 T={run.T} 2000 sweeps: GPU ({how} plan)")
        ctx = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up)
        try:
            if how == "tuned":
                b.ising_tune(ctx, 50)
            elif how == "fused":
                b.ising_plan_set(ctx, b.ISING_PLAN_FUSED, 1, 8)
            b.ising_sweep(ctx, run.sweeps)
            g = _ctx_result(b, ctx, run.L)
            plan = tuple(b.ising_plan_info(ctx))
        finally:
            b.ising_destroy(ctx)
        G.assert_same(g, ref, f"C1 T={run.T} plan={plan}")
    # physics on the oracle's own series: the disordered phase equilibrates
    # quickly; at T_c the energy per site approaches the exact finite-lattice
    # (Kaufman) value
    e = -ref["B"][1000:] / run.L ** 2
    if run.T > 3.0:
        assert abs(e.mean() - physics.onsager_energy(run.T)) < 2e-3
    elif run.T == W.T_C_CONFIG:
        assert abs(e.mean() - physics.kaufman_energy(run.L, run.T)) < 0.03


C2_SWEEPS = 8
C2_SHAPES = [("FUSED", 4, 16), ("FUSED", 4, 32), ("FUSED", 4, 64), ("FUSED", 4, 128), ("FUSED", 2, 32),
             ("FUSED_ROWS", 4, 32), ("FUSED_ROWS", 4, 64), ("FUSED_ROWS", 4, 128)]


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_c2_32768_whole_lattice_first_sweeps(b, o, k):
    """32768 x 32768 (1 GiB), h in {0, 0.1} x {cold, hot}, seed 11: after the
    first 8 sweeps the whole lattice, its hash and the 8 (B_t, M_t) equal a
    full oracle run, for the default plan and each fused shape (wave tiles
    and full-row workgroups) the autotuner picks at this side (the later
    sweeps are checked through light-cone windows in test_gpu_parity)."""
    run = W.C2[k]
    G.log(f"C2 32768 h={run.h} p_up={run.p_up}: oracle {C2_SWEEPS} sweeps")
    ref = G.oracle_run(o, run, sweeps=C2_SWEEPS)
    for shape in [None] + C2_SHAPES:
        G.log(f"C2 32768 h={run.h} p_up={run.p_up}: GPU plan {shape or 'default'}")
        ctx = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up)
        try:
            if shape:
                b.ising_plan_set(ctx, getattr(b, "ISING_PLAN_" + shape[0]), shape[1], shape[2])
            b.ising_sweep(ctx, C2_SWEEPS)
            g = _ctx_result(b, ctx, run.L)
            plan = tuple(b.ising_plan_info(ctx))
        finally:
            b.ising_destroy(ctx)
        G.assert_same(g, ref, f"C2 h={run.h} p_up={run.p_up} plan={plan}")
        del g


# Oracle results of the batched lattices checked below, computed once for
# both batch plans.
_BATCH_REF = {}


def _batched_checked(runs):
    """Indices of the batched lattices compared with the oracle: the four
    largest (side 1024) and one lattice from each of four size bands."""
    order = sorted(range(len(runs)), key=lambda k: (-runs[k].L, k))
    pick = order[:4]
    for lo, hi in ((32, 128), (128, 384), (384, 640), (640, 896)):
        band = [k for k in range(len(runs)) if lo <= runs[k].L < hi]
        if band:
            pick.append(band[0])
    return pick


@pytest.mark.parametrize("plan", ["RESIDENT", "STEPPED"])
def test_batched_largest_lattices_against_oracle(b, o, plan):
    """The batched configuration (1024 lattices, 10000 sweeps, one batch
    call): the four lattices of side 1024 and one of each size band equal
    the oracle over all 10000 sweeps (lattice, hash and every (B_t, M_t))."""
    runs = W.batched(count=1024, sweeps=10000)
    pick = _batched_checked(runs)
    ctxs = [b.ising_create(r.L, r.J, r.h, r.T, r.seed, r.p_up) for r in runs]
    try:
        G.log(f"batched 1024 x 10000 sweeps ({plan})")
        b.ising_sweep_batch_plan(ctxs, [r.sweeps for r in runs], getattr(b, "ISING_BATCH_" + plan))
        for k in pick:
            r = runs[k]
            g = _ctx_result(b, ctxs[k], r.L)
            if k not in _BATCH_REF:
                G.log(f"batched lattice {k} L={r.L} T={r.T:.4f}: oracle 10000 sweeps")
                _BATCH_REF[k] = G.oracle_run(o, r)
            G.assert_same(g, _BATCH_REF[k], f"batched {plan} lattice {k} L={r.L}")
    finally:
        for c in ctxs:
            b.ising_destroy(c)
