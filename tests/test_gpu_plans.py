"""GPU parity of every execution plan and tile shape, plan switches,
the batched persistent path and the autotuner, all against the oracle."""
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


def _run_plan(b, run, plan, cw=0, rows=0, chunks=None):
    ctx = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up)
    try:
        b.ising_plan_set(ctx, plan, cw, rows)
        for k in (chunks or [run.sweeps]):
            b.ising_sweep(ctx, k)
        obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
        spins = b.ising_copy_spins(ctx, run.L)
        info = b.ising_plan_info(ctx)
    finally:
        b.ising_destroy(ctx)
    return {"spins": spins, "B": B, "M": M, "hash": obs.lattice_hash, "plan": info}


@pytest.mark.parametrize("L,h,T", [(2048, 0.0, 2.269185), (2048, 0.1, 1.8), (1024, 0.0, 0.2), (512, -0.05, 3.0)])
def test_fused_every_tile_shape(b, o, L, h, T):
    run = W.Run(L=L, h=h, T=T, seed=L + 3, sweeps=12)
    ref = G.oracle_run(o, run)
    tried = 0
    for cw in (1, 2, 4):
        for rows in (4, 8, 16, 32, 64):
            if (L // 8) % (64 * cw) != 0:
                continue
            G.log(f"fused L={L} cw={cw} rows={rows} h={h} T={T}")
            g = _run_plan(b, run, b.ISING_PLAN_FUSED, cw, rows, chunks=[5, 7])
            assert g["plan"] == (b.ISING_PLAN_FUSED, cw, rows)
            G.assert_same(g, ref, f"fused L={L} cw={cw} rows={rows}")
            tried += 1
    assert tried >= 4


@pytest.mark.parametrize("L,h,T", [(2048, 0.0, 2.269185), (2048, 0.1, 1.8), (1024, 0.0, 0.2), (512, -0.05, 3.0),
                                   (4096, 0.0, 1e300), (1536, 0.02, 2.5)])
def test_fused_rows_every_shape(b, o, L, h, T):
    """The fused sweep by full-row workgroups (neighbouring waves trade their
    edge words through local memory) in every chunk width and band height
    that fits the side, against the oracle; also the zero thresholds of
    T = 0.2 and the certain flips of T = 1e300."""
    run = W.Run(L=L, h=h, T=T, seed=L + 5, sweeps=12)
    ref = G.oracle_run(o, run)
    tried = 0
    for cw in (1, 2, 4):
        for rows in (8, 16, 32, 64, 128):
            nw = (L // 8) // (64 * cw)
            if (L // 8) % (64 * cw) or nw > 16 or L % rows:
                continue
            G.log(f"fused rows L={L} cw={cw} rows={rows} h={h} T={T}")
            g = _run_plan(b, run, b.ISING_PLAN_FUSED_ROWS, cw, rows, chunks=[5, 7])
            assert g["plan"] == (b.ISING_PLAN_FUSED_ROWS, cw, rows)
            G.assert_same(g, ref, f"fused rows L={L} cw={cw} rows={rows}")
            tried += 1
    assert tried >= 3


@pytest.mark.parametrize("L", [8, 16, 24, 40, 64, 128, 200, 520])
def test_resident_plan(b, o, L):
    run = W.Run(L=L, h=0.03, T=2.1, seed=L, sweeps=30)
    G.log(f"resident L={L}")
    g = _run_plan(b, run, b.ISING_PLAN_RESIDENT, chunks=[1, 29])
    G.assert_same(g, G.oracle_run(o, run), f"resident L={L}")


@pytest.mark.parametrize("L", [64, 1024])
def test_two_pass_chunk_widths(b, o, L):
    run = W.Run(L=L, h=0.0, seed=L + 1, sweeps=10)
    ref = G.oracle_run(o, run)
    for cw in (1, 2, 4):
        G.log(f"two-pass L={L} cw={cw}")
        G.assert_same(_run_plan(b, run, b.ISING_PLAN_TWO_PASS, cw), ref, f"two-pass L={L} cw={cw}")


def test_plan_switches_mid_run(b, o):
    """The lattice and the sweep index carry over between plans (the fused
    plan's ping-pong buffer included)."""
    run = W.Run(L=1024, h=0.02, T=2.3, seed=99, sweeps=29)
    ref = G.oracle_run(o, run)
    ctx = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up)
    G.log("plan switches 1024")
    for plan, cw, rows, n in [(b.ISING_PLAN_FUSED, 1, 8, 3), (b.ISING_PLAN_TWO_PASS, 2, 0, 4),
                              (b.ISING_PLAN_FUSED, 2, 16, 5), (b.ISING_PLAN_RESIDENT, 0, 0, 2),
                              (b.ISING_PLAN_GENERIC, 0, 0, 2), (b.ISING_PLAN_FUSED, 1, 64, 7),
                              (b.ISING_PLAN_FUSED_ROWS, 2, 8, 3), (b.ISING_PLAN_FUSED_ROWS, 1, 128, 3)]:
        b.ising_plan_set(ctx, plan, cw, rows)
        b.ising_sweep(ctx, n)
    obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
    spins = b.ising_copy_spins(ctx, run.L)
    b.ising_destroy(ctx)
    G.assert_same({"spins": spins, "B": B, "M": M, "hash": obs.lattice_hash}, ref, "plan switches")


def test_two_pass_graph_replays_follow_the_lattice(b, o):
    """Two-pass calls of 16 or more sweeps run as graph replays (16 sweeps
    each, the rest launched directly). Between them the lattice moves to the
    other buffer (a fused sweep, a batch call with an odd sweep count): each
    later replay still updates the lattice in place, continues the sweep
    index and fills the next series slots."""
    run = W.Run(L=512, h=0.05, T=2.1, seed=2024, sweeps=37 + 3 + 16 + 3 + 33 + 15)
    ref = G.oracle_run(o, run)
    ctx = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up)
    try:
        G.log("two-pass graph replays 512")
        b.ising_plan_set(ctx, b.ISING_PLAN_TWO_PASS, 4, 0)
        b.ising_sweep(ctx, 37)
        b.ising_plan_set(ctx, b.ISING_PLAN_FUSED, 1, 8)
        b.ising_sweep(ctx, 3)
        b.ising_plan_set(ctx, b.ISING_PLAN_TWO_PASS, 2, 0)
        b.ising_sweep(ctx, 16)
        b.ising_sweep_batch_plan([ctx], [3], b.ISING_BATCH_STEPPED)
        b.ising_sweep(ctx, 33)
        b.ising_sweep(ctx, 15)
        obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
        spins = b.ising_copy_spins(ctx, run.L)
    finally:
        b.ising_destroy(ctx)
    assert obs.sweeps_done == run.sweeps
    G.assert_same({"spins": spins, "B": B, "M": M, "hash": obs.lattice_hash}, ref, "two-pass graph replays")


@pytest.mark.parametrize("plan", ["RESIDENT", "STEPPED"])
def test_batch_equals_solo_and_oracle(b, o, plan):
    """Uneven lattices (sizes, temperatures, fields, seeds, sweep counts,
    including zero) in one batch call, with either batch plan: each result is
    bit-identical to the oracle's run of that lattice alone; a second batch
    call continues from where the first stopped."""
    bplan = getattr(b, "ISING_BATCH_" + plan)
    rng = np.random.default_rng(5)
    runs = []
    for k in range(40):
        L = int(8 * rng.integers(1, 66))
        runs.append(W.Run(L=L, J=1.0, h=float(rng.choice([0.0, 0.05, -0.1])), T=float(rng.uniform(1.0, 4.0)),
                          seed=int(rng.integers(0, 2 ** 63)), p_up=float(rng.choice([0.5, 1.0])),
                          sweeps=int(rng.integers(0, 25))))
    runs.append(W.Run(L=64, T=0.2, seed=3, sweeps=10))  # thresholds of 0: exact compare
    ctxs = [b.ising_create(r.L, r.J, r.h, r.T, r.seed, r.p_up, b.ISING_PLAN_TWO_PASS) for r in runs]
    G.log(f"batch of 41 ({plan}), first call")
    b.ising_sweep_batch_plan(ctxs, [r.sweeps for r in runs], bplan)
    extra = [int(rng.integers(0, 40)) for _ in runs]
    G.log(f"batch of 41 ({plan}), second call")
    b.ising_sweep_batch_plan(ctxs, extra, bplan)
    for r, ctx, e in zip(runs, ctxs, extra):
        obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
        spins = b.ising_copy_spins(ctx, r.L)
        b.ising_destroy(ctx)
        ref = G.oracle_run(o, r, sweeps=r.sweeps + e)
        assert obs.sweeps_done == r.sweeps + e
        G.assert_same({"spins": spins, "B": B, "M": M, "hash": obs.lattice_hash}, ref, f"batch L={r.L}")


def test_batch_bit_packed_couplings_and_sides(b, o):
    """A resident batch with fewer lattices than workgroups: sides up to 256
    are held as bytes, the largest sides that fit local memory only as bits
    (1072, 1080) bit-packed, and one that fits neither (1088) is swept in
    global memory. J > 0, J < 0 and J = 0, thresholds of 0 (T = 0.05), near 1
    (T = 50) and at T_c, in one batch call: each result equals the oracle's
    run of that lattice alone."""
    runs = [W.Run(L=8, J=1.0, T=2.269185, seed=1, p_up=0.5, sweeps=40),
            W.Run(L=24, J=-1.0, T=2.0, seed=2, p_up=0.5, sweeps=30),
            W.Run(L=40, J=1.0, T=0.05, seed=3, p_up=0.5, sweeps=20),
            W.Run(L=136, J=-2.0, T=0.3, seed=4, p_up=0.5, sweeps=20),
            W.Run(L=64, J=0.0, T=1.0, seed=5, p_up=0.5, sweeps=10),
            W.Run(L=96, J=0.5, T=50.0, seed=6, p_up=1.0, sweeps=10),
            W.Run(L=1072, J=1.0, T=2.269185, seed=7, p_up=0.5, sweeps=6),
            W.Run(L=1080, J=-1.0, T=1.5, seed=8, p_up=1.0, sweeps=4),
            W.Run(L=1088, J=1.0, T=3.0, seed=9, p_up=0.5, sweeps=3)]
    ctxs = [b.ising_create(r.L, r.J, r.h, r.T, r.seed, r.p_up) for r in runs]
    G.log("bit-packed batch of 9 (RESIDENT)")
    b.ising_sweep_batch_plan(ctxs, [r.sweeps for r in runs], b.ISING_BATCH_RESIDENT)
    for r, ctx in zip(runs, ctxs):
        obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
        spins = b.ising_copy_spins(ctx, r.L)
        b.ising_destroy(ctx)
        G.log(f"bit-packed batch: L={r.L} J={r.J} T={r.T} vs oracle")
        G.assert_same({"spins": spins, "B": B, "M": M, "hash": obs.lattice_hash}, G.oracle_run(o, r),
                      f"bit-packed L={r.L} J={r.J} T={r.T}")


def test_batch_bit_packed_field_classes(b, o):
    """h != 0 lattices too large to hold as bytes (sides 264 to 1080) run
    bit-packed with one compare per (spin, m) class: weak and strong fields
    of both signs, J > 0 and J < 0, classes never accepted (T = 0.05, and a
    field so strong that some classes are), classes always accepted, and
    one lattice with every threshold 2^32 (T = 1e300). Each result equals
    the oracle's run of that lattice alone; the single-context resident plan
    takes the same path."""
    runs = [W.Run(L=264, J=1.0, h=0.05, T=2.269185, seed=11, p_up=0.5, sweeps=40),
            W.Run(L=320, J=1.0, h=-0.3, T=1.5, seed=12, p_up=1.0, sweeps=30),
            W.Run(L=512, J=1.0, h=3.0, T=2.0, seed=13, p_up=0.0, sweeps=20),
            W.Run(L=392, J=-1.0, h=0.2, T=1.8, seed=14, p_up=0.5, sweeps=25),
            W.Run(L=600, J=1.0, h=0.1, T=0.05, seed=15, p_up=0.5, sweeps=12),
            W.Run(L=272, J=-0.5, h=-5.0, T=0.3, seed=16, p_up=0.5, sweeps=15),
            W.Run(L=1024, J=1.0, h=0.05, T=3.0, seed=17, p_up=0.5, sweeps=8),
            W.Run(L=1072, J=1.0, h=0.5, T=1e300, seed=18, p_up=0.5, sweeps=5),
            W.Run(L=1080, J=2.0, h=-0.7, T=2.5, seed=19, p_up=1.0, sweeps=4)]
    ctxs = [b.ising_create(r.L, r.J, r.h, r.T, r.seed, r.p_up) for r in runs]
    try:
        G.log("field bit-packed batch of 9 (RESIDENT)")
        b.ising_sweep_batch_plan(ctxs, [r.sweeps for r in runs], b.ISING_BATCH_RESIDENT)
        for r, ctx in zip(runs, ctxs):
            obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
            spins = b.ising_copy_spins(ctx, r.L)
            G.log(f"field bit-packed: L={r.L} J={r.J} h={r.h} T={r.T} vs oracle")
            G.assert_same({"spins": spins, "B": B, "M": M, "hash": obs.lattice_hash}, G.oracle_run(o, r),
                          f"field bit-packed L={r.L} J={r.J} h={r.h} T={r.T}")
    finally:
        for ctx in ctxs:
            b.ising_destroy(ctx)
    r = runs[3]
    G.log("field bit-packed: single-context resident plan L=392")
    G.assert_same(_run_plan(b, r, b.ISING_PLAN_RESIDENT, chunks=[7, 18]), G.oracle_run(o, r),
                  "single-context resident, field classes")


def test_batch_bit_packed_saturated_batch(b, o):
    """A resident batch with more lattices (400) than the launch has
    workgroups, so every h = 0 lattice that fits local memory as bits is
    bit-packed, small ones included: sides with partial 32-site words (8 to
    136 in steps of 8), J > 0, J < 0 and J = 0, thresholds of 0 (T = 0.05),
    near 1 (T = 50) and at T_c, one to five sweeps, plus a few h != 0
    lattices (held as bytes). Each result equals the oracle's run of that
    lattice alone."""
    rng = np.random.default_rng(2024)
    Js = [1.0, -1.0, 0.0, 0.5, -2.0]
    Ts = [0.05, 1.0, 2.269185, 3.5, 50.0]
    runs = []
    for k in range(400):
        L = int(8 * rng.integers(1, 18))
        h = 0.1 if k % 50 == 7 else 0.0
        runs.append(W.Run(L=L, J=Js[k % 5], h=h, T=Ts[(k // 5) % 5], seed=1000 + k,
                          p_up=float(rng.choice([0.5, 1.0])), sweeps=int(rng.integers(1, 6))))
    ctxs = [b.ising_create(r.L, r.J, r.h, r.T, r.seed, r.p_up) for r in runs]
    try:
        G.log("saturated bit-packed batch of 400 (RESIDENT)")
        b.ising_sweep_batch_plan(ctxs, [r.sweeps for r in runs], b.ISING_BATCH_RESIDENT)
        for r, ctx in zip(runs, ctxs):
            obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
            spins = b.ising_copy_spins(ctx, r.L)
            G.assert_same({"spins": spins, "B": B, "M": M, "hash": obs.lattice_hash}, G.oracle_run(o, r),
                          f"saturated batch L={r.L} J={r.J} h={r.h} T={r.T} seed={r.seed}")
    finally:
        for ctx in ctxs:
            b.ising_destroy(ctx)


def test_batches_alternate_between_named_and_own_streams(b, o):
    """Consecutive batch calls on the same contexts, alternating between a
    caller's stream and the library's own (no stream named), with both
    plans: every call follows the previous one, and each result equals the
    oracle's run of that lattice alone."""
    import torch
    runs = [W.Run(L=L, J=1.0, h=h, T=T, seed=40 + k, p_up=0.5, sweeps=0)
            for k, (L, h, T) in enumerate([(64, 0.0, 2.269185), (96, 0.05, 1.8), (256, 0.0, 3.0), (528, -0.1, 2.2)])]
    ctxs = [b.ising_create(r.L, r.J, r.h, r.T, r.seed, r.p_up) for r in runs]
    side = torch.cuda.Stream()
    calls = [(b.ISING_BATCH_STEPPED, side.cuda_stream, 5), (b.ISING_BATCH_RESIDENT, None, 3),
             (b.ISING_BATCH_STEPPED, None, 4), (b.ISING_BATCH_RESIDENT, side.cuda_stream, 2),
             (b.ISING_BATCH_STEPPED, None, 1)]
    try:
        total = 0
        for plan, stream, n in calls:
            G.log(f"alternating streams: plan {plan} stream {'named' if stream else 'own'} {n} sweeps")
            b.ising_sweep_batch_plan(ctxs, [n] * len(runs), plan, stream=stream)
            total += n
        for r, ctx in zip(runs, ctxs):
            obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
            G.assert_same({"spins": b.ising_copy_spins(ctx, r.L), "B": B, "M": M, "hash": obs.lattice_hash},
                          G.oracle_run(o, r, sweeps=total), f"alternating streams L={r.L}")
    finally:
        for ctx in ctxs:
            b.ising_destroy(ctx)


def test_batch_stepped_fused_walk_ragged_tiles(b, o):
    """The stepped plan's one-pass walk (every side a multiple of 16): sides
    whose tiles end before the last lane (plane rows of 2 to 258 words) and
    after 16 of 32 rows, h = 0 and h != 0, J < 0, thresholds of 0 (T = 0.2),
    odd and even sweep counts (each lattice alternates between two buffers),
    and a second call that continues the first: every result equals the
    oracle's run of that lattice alone."""
    runs = [W.Run(L=16, J=1.0, h=0.0, T=2.269185, seed=1, p_up=0.5, sweeps=7),
            W.Run(L=48, J=1.0, h=0.1, T=1.8, seed=2, p_up=1.0, sweeps=12),
            W.Run(L=80, J=-1.0, h=0.05, T=2.5, seed=3, p_up=0.5, sweeps=9),
            W.Run(L=144, J=1.0, h=0.0, T=0.2, seed=4, p_up=0.5, sweeps=10),
            W.Run(L=272, J=0.7, h=-0.2, T=3.0, seed=5, p_up=0.5, sweeps=5),
            W.Run(L=1040, J=1.0, h=0.0, T=2.269185, seed=6, p_up=0.5, sweeps=3),
            W.Run(L=2064, J=1.0, h=0.05, T=2.0, seed=7, p_up=0.5, sweeps=2),
            W.Run(L=512, J=1.0, h=0.0, T=2.269185, seed=8, p_up=0.5, sweeps=0)]
    extra = [4, 1, 6, 3, 2, 1, 1, 3]
    ctxs = [b.ising_create(r.L, r.J, r.h, r.T, r.seed, r.p_up) for r in runs]
    G.log("stepped fused walk: first call")
    b.ising_sweep_batch_plan(ctxs, [r.sweeps for r in runs], b.ISING_BATCH_STEPPED)
    G.log("stepped fused walk: second call")
    b.ising_sweep_batch_plan(ctxs, extra, b.ISING_BATCH_STEPPED)
    for r, ctx, e in zip(runs, ctxs, extra):
        obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
        spins = b.ising_copy_spins(ctx, r.L)
        b.ising_destroy(ctx)
        G.log(f"stepped fused walk: L={r.L} vs oracle")
        assert obs.sweeps_done == r.sweeps + e
        G.assert_same({"spins": spins, "B": B, "M": M, "hash": obs.lattice_hash},
                      G.oracle_run(o, r, sweeps=r.sweeps + e), f"stepped fused L={r.L}")


def test_batch_stepped_fused_walk_packed_columns_tall_tiles(b, o):
    """A stepped batch with enough tiles (560 lattices, about 17000 tiles)
    for the walk to use 32-row tiles, mixing the tile kinds: full 128-word
    columns with ragged bottom tiles (1040, 2064), narrow last columns
    packed several row bands to a wave with 32-row bands (512, 1056, 1088)
    and with 16-row bands where 32 does not divide the side (48, 80, 144,
    272, 496, 1040, 1072, 1104, 2064), lattices too wide to pack (528) and
    too short to (16, 32); h = 0 and h != 0, J < 0. Two calls (2 then 1
    sweeps): every lattice equals the oracle's run of it alone."""
    sides = [1040, 1072, 1056, 528, 48, 80, 144, 272, 496, 512, 16, 32, 1088, 1104, 2064]
    runs = [W.Run(L=sides[k % len(sides)], J=-1.0 if k % 7 == 3 else 1.0, h=0.05 if k % 3 == 1 else 0.0,
                  T=1.5 + 0.01 * (k % 200), seed=5000 + k, p_up=0.5, sweeps=3) for k in range(560)]
    ctxs = [b.ising_create(r.L, r.J, r.h, r.T, r.seed, r.p_up) for r in runs]
    try:
        G.log("stepped fused walk: 560 lattices, 32-row tiles, packed columns")
        b.ising_sweep_batch_plan(ctxs, [2] * len(runs), b.ISING_BATCH_STEPPED)
        b.ising_sweep_batch_plan(ctxs, [1] * len(runs), b.ISING_BATCH_STEPPED)
        for k, (r, ctx) in enumerate(zip(runs, ctxs)):
            obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
            spins = b.ising_copy_spins(ctx, r.L)
            G.assert_same({"spins": spins, "B": B, "M": M, "hash": obs.lattice_hash}, G.oracle_run(o, r),
                          f"packed-column batch lattice {k} L={r.L} J={r.J} h={r.h}")
    finally:
        for ctx in ctxs:
            b.ising_destroy(ctx)


def test_batch_stepped_fused_walk_many_large_lattices(b, o):
    """A stepped batch of 48 lattices of 2048^2 (h = 0 and h = 0.05): tiles
    of fewer rows are used when the batch has too few tiles to fill the GPU
    (this batch sits between the 8-lattice test above and the 1024-lattice
    configuration, which use the shortest and the tallest tiles). Every
    sixth lattice's series and final lattice equal its own run alone
    (two-pass plan), over an odd and then an even number of sweeps, and the
    first two (h = 0 and h = 0.05) equal the oracle."""
    runs = [W.Run(L=2048, J=1.0, h=0.05 * (k % 2), T=2.0 + 0.02 * k, seed=100 + k, p_up=0.5, sweeps=3)
            for k in range(48)]
    ctxs = [b.ising_create(r.L, r.J, r.h, r.T, r.seed, r.p_up) for r in runs]
    G.log("stepped fused walk: 48 x 2048^2")
    b.ising_sweep_batch_plan(ctxs, [3] * 48, b.ISING_BATCH_STEPPED)
    b.ising_sweep_batch_plan(ctxs, [2] * 48, b.ISING_BATCH_STEPPED)
    for k, (r, ctx) in enumerate(zip(runs, ctxs)):
        obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
        spins = b.ising_copy_spins(ctx, r.L) if k < 2 else None
        b.ising_destroy(ctx)
        if k < 2:
            G.log(f"stepped fused walk: 2048^2 lattice {k} (h={r.h}) vs the oracle")
            G.assert_same({"spins": spins, "B": B, "M": M, "hash": obs.lattice_hash}, G.oracle_run(o, r, sweeps=5),
                          f"stepped 2048^2 lattice {k}")
        if k % 6:
            continue
        G.log(f"stepped fused walk: 2048^2 lattice {k} vs its solo run")
        ref = G.gpu_run(b, r, sweeps=5, plan=b.ISING_PLAN_TWO_PASS)
        assert obs.lattice_hash == ref["hash"]
        assert np.array_equal(B, ref["B"]) and np.array_equal(M, ref["M"])


def test_batch_rejects_before_launching(b):
    good = b.ising_create(16)
    bad = b.ising_create(10)  # L % 8 != 0
    with pytest.raises(b.IsingError) as e:
        b.ising_sweep_batch([good, bad], [3, 3])
    assert e.value.code == b.ISING_EUNSUPPORTED
    obs, _, _ = b.ising_observables(good)
    assert obs.sweeps_done == 0
    with pytest.raises(b.IsingError):
        b.ising_sweep_batch([good, good], [1, 1])
    b.ising_destroy(good)
    b.ising_destroy(bad)


def test_autotune_keeps_lattice_and_picks_a_plan(b, o):
    run = W.Run(L=4096, seed=7, sweeps=6)
    ctx = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up)
    b.ising_sweep(ctx, 2)
    before = b.ising_copy_spins(ctx, run.L)
    G.log("autotune 4096")
    b.ising_tune(ctx, 3)
    after = b.ising_copy_spins(ctx, run.L)
    assert np.array_equal(before, after)
    plan = b.ising_plan_info(ctx)
    assert plan[0] in (b.ISING_PLAN_FUSED, b.ISING_PLAN_FUSED_ROWS, b.ISING_PLAN_TWO_PASS, b.ISING_PLAN_RESIDENT,
                       b.ISING_PLAN_BANDS)
    b.ising_sweep(ctx, 4)
    obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
    spins = b.ising_copy_spins(ctx, run.L)
    b.ising_destroy(ctx)
    ref = G.oracle_run(o, run)
    assert np.array_equal(spins, ref["spins"]) and obs.lattice_hash == ref["hash"]
    assert np.array_equal(B, ref["B"]) and np.array_equal(M, ref["M"])
    # the tuned plan is remembered for AUTO contexts of the same side
    ctx2 = b.ising_create(run.L)
    assert b.ising_plan_info(ctx2) == plan
    b.ising_destroy(ctx2)


def test_c2_plans_agree_at_full_size(b):
    """32768 x 32768, 40 sweeps: the fused plans (wave tiles and full-row
    workgroups) and the two-pass plan give the same lattice hash and series
    (plan independence at the full size)."""
    run = W.Run(L=32768, seed=11, p_up=0.5, sweeps=40)
    G.log("C2 fused vs two-pass 40 sweeps")
    f = _run_plan(b, run, b.ISING_PLAN_FUSED)
    t = _run_plan(b, run, b.ISING_PLAN_TWO_PASS)
    r = _run_plan(b, run, b.ISING_PLAN_FUSED_ROWS)
    assert f["hash"] == t["hash"] == r["hash"]
    assert np.array_equal(f["B"], t["B"]) and np.array_equal(f["M"], t["M"])
    assert np.array_equal(r["B"], t["B"]) and np.array_equal(r["M"], t["M"])
