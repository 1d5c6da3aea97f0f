"""GPU parity of the Creutz demon dynamics (Section 2.2's deterministic
alternative) through the C ABI: spins, demons and every per-sweep (B, M)
bit-exact against the oracle on seeded inputs; at the full 32768^2 size,
exact energy conservation and exact reversal."""
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


def _gpu(b, L, seed, p_up, demons, steps, plan=0):
    """steps: list of (n, reverse). Returns spins, demons, B, M, demon sum."""
    ctx = b.ising_create(L, 1.0, 0.0, 2.0, seed, p_up, plan)
    try:
        b.ising_creutz_init(ctx, demons)
        for n, rev in steps:
            b.ising_creutz_sweep(ctx, n, rev)
        _, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES)
        return (b.ising_copy_spins(ctx, L), b.ising_copy_demons(ctx, L), B, M, b.ising_demon_sum(ctx))
    finally:
        b.ising_destroy(ctx)


def _oracle(o, L, seed, p_up, demons, steps):
    s = o.init(L, seed, p_up)
    d = demons.copy()
    Bs, Ms = [], []
    for n, rev in steps:
        B, M, _ = o.creutz_run(s, d, n, reverse=rev)
        Bs.append(B)
        Ms.append(M)
    return s, d, np.concatenate(Bs), np.concatenate(Ms), o.demon_sum(d)


CASES = [
    # L, seed, p_up, demon max, plan; L % 8 != 0 takes the per-site kernel
    (8, 1, 0.5, 3, 0), (16, 2, 0.3, 255, 0), (64, 3, 0.5, 0, 0), (136, 4, 0.5, 2, 0),
    (520, 5, 0.8, 1, 0), (10, 6, 0.5, 3, 0), (30, 7, 0.5, 255, 0), (6, 8, 0.5, 4, 0),
    (512, 9, 0.5, 3, 2), (1024, 10, 0.5, 1, 0),
]


@pytest.mark.parametrize("L,seed,p_up,hi,plan", CASES)
def test_creutz_parity(b, o, L, seed, p_up, hi, plan):
    demons = W.random_demons(L, seed, hi)
    steps = [(7, False), (1, False), (5, True), (12, False)]
    G.log(f"creutz L={L} seed={seed} demons<= {hi} plan={plan}")
    g = _gpu(b, L, seed, p_up, demons, steps, plan)
    r = _oracle(o, L, seed, p_up, demons, steps)
    for name, x, y in zip(("spins", "demons", "B", "M", "demon sum"), g, r):
        assert np.array_equal(x, y), f"L={L}: {name} differ"


def test_creutz_fill_and_errors(b, o):
    L = 32
    ctx = b.ising_create(L, 1.0, 0.0, 2.0, 3, 0.5)
    try:
        with pytest.raises(b.IsingError) as e:
            b.ising_creutz_sweep(ctx, 1)
        assert e.value.code == b.ISING_ESTATE
        b.ising_creutz_init(ctx, None, fill=2)
        assert b.ising_demon_sum(ctx) == 2 * L * L
        b.ising_creutz_sweep(ctx, 0)
        b.ising_creutz_sweep(ctx, 9)
        obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES)
        assert obs.sweeps_done == 0 and len(B) == 9  # no Metropolis sweep index used
    finally:
        b.ising_destroy(ctx)
    s = o.init(L, 3, 0.5)
    d = np.full((L, L), 2, dtype=np.uint8)
    Bo, Mo, _ = o.creutz_run(s, d, 9)
    assert np.array_equal(B, Bo) and np.array_equal(M, Mo)
    for h, J in ((0.1, 1.0), (0.0, -1.0)):
        ctx = b.ising_create(L, J, h, 2.0, 3, 0.5)
        try:
            with pytest.raises(b.IsingError) as e:
                b.ising_creutz_init(ctx, None, fill=0)
            assert e.value.code == b.ISING_EUNSUPPORTED
        finally:
            b.ising_destroy(ctx)


def test_creutz_then_metropolis_continues(b, o):
    """Creutz sweeps leave the Metropolis sweep index alone: Metropolis
    sweeps after them use indices 0, 1, ... of the seed."""
    L, seed, T = 48, 4, 2.4
    ctx = b.ising_create(L, 1.0, 0.0, T, seed, 0.5)
    try:
        b.ising_creutz_init(ctx, None, fill=1)
        b.ising_creutz_sweep(ctx, 6)
        b.ising_sweep(ctx, 5)
        obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
        spins = b.ising_copy_spins(ctx, L)
    finally:
        b.ising_destroy(ctx)
    s = o.init(L, seed, 0.5)
    d = np.full((L, L), 1, dtype=np.uint8)
    Bc, Mc, _ = o.creutz_run(s, d, 6)
    Bm, Mm = o.run(s, 1.0, 0.0, T, seed, 0, 5)
    assert np.array_equal(B, np.concatenate([Bc, Bm])) and np.array_equal(M, np.concatenate([Mc, Mm]))
    assert np.array_equal(spins, s) and obs.lattice_hash == o.fnv1a64(s) and obs.sweeps_done == 5


def test_creutz_full_size_conserves_and_reverses(b):
    """32768 x 32768 hot start, empty demons, in the configuration bench.py
    times: -B + 4 D is the same after each of 40 sweeps (D from the
    conservation law at the end matches the demon total read back), and
    40 reversed sweeps return the starting lattice and demons exactly."""
    run = W.CREUTZ
    G.log("creutz 32768^2 forward 40 + reverse 40")
    ctx = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up)
    try:
        b.ising_creutz_init(ctx, None, fill=0)
        obs0, _, _ = b.ising_observables(ctx, b.ISING_OBS_HASH)
        e0 = -obs0.bond_sum
        b.ising_creutz_sweep(ctx, 40)
        obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES)
        D = b.ising_demon_sum(ctx)
        assert -int(B[-1]) + 4 * D == e0
        # every sweep conserves: demon totals implied by B are integers in range
        implied = (np.asarray(B, dtype=np.int64) + e0)
        assert np.all(implied % 4 == 0) and np.all(implied >= 0)
        assert (int(B[-1]), int(M[-1])) == (obs.bond_sum, obs.mag_sum)
        moved = B[-1] != obs0.bond_sum
        b.ising_creutz_sweep(ctx, 40, reverse=True)
        obs1, _, _ = b.ising_observables(ctx, b.ISING_OBS_HASH | b.ISING_OBS_SERIES)
        assert moved and obs1.lattice_hash == obs0.lattice_hash
        assert b.ising_demon_sum(ctx) == 0
    finally:
        b.ising_destroy(ctx)
