"""Pins of the oracle's Creutz demon dynamics (the deterministic,
random-number-free checkerboard dynamics Section 2.2 cites): exact energy
conservation, exact reversibility, the frozen ground state, the demon
thermometer against the exact finite-lattice energy, and agreement with the
NumPy oracle."""
import numpy as np
import pytest

from oracle import mini
from tests import pins


@pytest.mark.parametrize("L,seed,p_up,demons", [
    (2, 1, 0.5, 1), (6, 2, 0.5, ("uniform", 3)), (10, 3, 0.3, 0), (16, 4, 0.5, ("uniform", 255)),
    (32, 5, 0.9, 254), (64, 6, 0.5, 255), (24, 7, 1.0, 2)])
def test_energy_conserved_exactly(oracle, L, seed, p_up, demons):
    pins.check_creutz_conservation(oracle, L, seed, p_up, demons)


@pytest.mark.parametrize("L,seed,p_up,demons", [
    (6, 2, 0.5, ("uniform", 3)), (16, 4, 0.5, 0), (32, 5, 0.9, ("uniform", 255)), (40, 8, 0.5, 255)])
def test_reversed_sweeps_undo(oracle, L, seed, p_up, demons):
    pins.check_creutz_reversible(oracle, L, seed, p_up, demons)


@pytest.mark.parametrize("fill", [0, 1])
def test_ground_state_with_poor_demons_is_frozen(oracle, fill):
    """From all spins up every move costs 8J (e = 2): demons holding less
    can pay for none, so nothing ever changes."""
    s = np.ones((16, 16), dtype=np.int8)
    d = np.full((16, 16), fill, dtype=np.uint8)
    B, M, D = oracle.creutz_run(s, d, 5)
    assert np.all(B == 2 * 256) and np.all(M == 256) and np.all(D == fill * 256)
    assert np.all(s == 1) and np.all(d == fill)


def test_single_demon_blinks(oracle):
    """One demon holding exactly 2 (8J) in an all-up lattice: in its colour
    pass that spin flips and empties the demon; its neighbours' demons are
    empty, so no neighbour can follow, and in the next sweep the flip is
    undone (it gives the 8J back). The state blinks with period two:
    B = 2N - 8, 2N, 2N - 8, ...; M = N - 2, N, ...; D = 0, 2, ..."""
    L = 8
    N = L * L
    s = np.ones((L, L), dtype=np.int8)
    d = np.zeros((L, L), dtype=np.uint8)
    d[3, 4] = 2  # colour (3 + 4) & 1 = 1
    B, M, D = oracle.creutz_run(s, d, 5)
    odd = np.arange(5) % 2 == 0  # after sweeps 1, 3, 5 the spin is down
    assert np.array_equal(B, np.where(odd, 2 * N - 8, 2 * N))
    assert np.array_equal(M, np.where(odd, N - 2, N))
    assert np.array_equal(D, np.where(odd, 0, 2))
    assert s[3, 4] == -1 and d[3, 4] == 0 and (s == -1).sum() == 1


def test_demon_thermometer_matches_exact_energy(oracle):
    """Microcanonical run from a random start with empty demons (total
    energy about 0): its demon temperature lies above T_c and the mean
    energy there equals the exact (Kaufman) energy of the 64 x 64 torus."""
    T = pins.check_creutz_thermometer(oracle, 64, 7, 0.5)
    assert 2.3 < T < 2.8


def test_demon_energies_are_boltzmann(oracle):
    """In equilibrium each demon's energy 4J k is Boltzmann-distributed at
    the demon temperature: the occupation of levels 0, 1, 2 falls by the
    same factor exp(-4 / T) per level (snapshots 200 sweeps apart)."""
    s, d = pins.creutz_start(oracle, 64, 7, 0.5, 0)
    oracle.creutz_run(s, d, 2000, series=False)
    hist = np.zeros(3)
    means = []
    for _ in range(30):
        oracle.creutz_run(s, d, 200, series=False)
        hist += np.bincount(d.ravel(), minlength=3)[:3]
        means.append(d.mean())
    x = np.exp(-4.0 / pins.demon_temperature(np.mean(means)))
    for k in (0, 1):
        r = hist[k + 1] / hist[k]
        se = r * np.sqrt(1 / hist[k + 1] + 1 / hist[k]) * 3  # snapshots are correlated: inflate
        assert abs(r - x) < 4 * se + 0.01, (k, r, x)


@pytest.mark.parametrize("L,reverse", [(6, False), (16, False), (16, True), (30, True)])
def test_cross_numpy(oracle, L, reverse):
    """The C oracle and the NumPy one agree sweep by sweep."""
    s, d = pins.creutz_start(oracle, L, 9, 0.5, ("uniform", 4))
    s2, d2 = s.copy(), d.copy()
    B, M, D = oracle.creutz_run(s, d, 20, reverse=reverse)
    for k in range(20):
        assert mini.creutz_sweep(s2, d2, reverse=reverse) == (B[k], M[k], D[k])
    assert np.array_equal(s, s2) and np.array_equal(d, d2)
