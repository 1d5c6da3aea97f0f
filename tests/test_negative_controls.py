"""Negative controls: copies of the oracle with one planted mistake each,
built on the CPU, must fail at least one of the pins that the real oracle
passes. This shows the pins can detect the kind of slip they guard against.
"""
import os

import numpy as np
import pytest

from oracle import build as obuild
from oracle import mini
from oracle.ref import Oracle
from tests import pins

SRC = open(obuild.SRC).read()

MUTANTS = {
    # every site updated in each pass (no checkerboard): not the Ising chain
    # (the same test guards the Creutz pass further down: mutate the first)
    "no_checkerboard": ("if (((i + j) & 1u) != c) continue;", "(void)0;", 0),
    # wrong sign of the energy change
    "energy_sign": ("double dE = 2.0 * s * (J * n + h);", "double dE = -2.0 * s * (J * n + h);"),
    # field term dropped
    "field_dropped": ("double dE = 2.0 * s * (J * n + h);", "double dE = 2.0 * s * (J * n);"),
    # left neighbour counted twice, right one never
    "wrong_neighbour": ("s[(size_t)i * L + rt];\n            int8_t me",
                        "s[(size_t)i * L + lf];\n            int8_t me"),
    # bond sum counts the right neighbour twice and misses the lower one
    "bond_sum": ("b += (int64_t)(me * (right + down));", "b += (int64_t)(me * (right + right));"),
    # Philox key words swapped in the round
    "philox_key": ("^ x1 ^ k0;", "^ x1 ^ k1;"),
    # colour order reversed (a valid chain, but not the frozen one)
    "colour_order": ("oracle_half_sweep(L, thr, seed, t, 0, s);\n        oracle_half_sweep(L, thr, seed, t, 1, s);",
                     "oracle_half_sweep(L, thr, seed, t, 1, s);\n        oracle_half_sweep(L, thr, seed, t, 0, s);"),
    # Creutz: demon credited with the wrong sign of the energy change
    "creutz_sign": ("int e = s[at] * n / 2;", "int e = -s[at] * n / 2;"),
    # Creutz: demon capacity not enforced (the byte wraps)
    "creutz_cap": ("if (e <= dem && dem - e <= 255) {", "if (e <= dem) {"),
    # Creutz: a demon must hold strictly more than the move costs
    "creutz_strict": ("if (e <= dem && dem - e <= 255) {", "if (e < dem && dem - e <= 255) {"),
    # Creutz: left neighbour counted twice
    "creutz_neighbour": ("s[(size_t)i * L + rt];\n            size_t at",
                         "s[(size_t)i * L + lf];\n            size_t at"),
    # percolation: invasion wraps around top and bottom (periodic, not open)
    "perc_wrap": ("if (i > 0) nb[cnt++] = at - L;", "nb[cnt++] = i > 0 ? at - L : at + (size_t)(L - 1) * L;"),
    # percolation: arrival counts two passes per step
    "perc_arrival": ("arrival[nb[k]] = arrival[at] + 1;", "arrival[nb[k]] = arrival[at] + 2;"),
    # percolation: a diagonal neighbour also invades
    "perc_diagonal": ("if (j + 1 < L) nb[cnt++] = at + 1;",
                      "if (j + 1 < L) nb[cnt++] = at + 1;\n        size_t nb5 = (i + 1 < L && j + 1 < L) ? at + L + 1 : at;\n"
                      "        if (pore[nb5] && arrival[nb5] < 0) { arrival[nb5] = arrival[at] + 1; queue[tail++] = (uint32_t)nb5; }"),
    # percolation: porosity threshold taken as 1 - P
    "perc_porosity": ("uint64_t pthr = (uint64_t)floor(P * 4294967296.0);\n    uint32_t key[2]",
                      "uint64_t pthr = (uint64_t)floor((1.0 - P) * 4294967296.0);\n    uint32_t key[2]"),
    # initial state uses the wrong comparison
    "init_compare": ("s[(size_t)i * L + j] = ((uint64_t)u < pthr)", "s[(size_t)i * L + j] = ((uint64_t)u >= pthr)"),
}


@pytest.fixture(scope="module")
def mutants(tmp_path_factory):
    out = {}
    d = tmp_path_factory.mktemp("mutants")
    for name, spec in MUTANTS.items():
        old, new = spec[:2]
        if len(spec) == 3:  # mutate the k-th of several occurrences
            k = spec[2]
            assert SRC.count(old) > k, name
            at = -1
            for _ in range(k + 1):
                at = SRC.index(old, at + 1)
            text = SRC[:at] + new + SRC[at + len(old):]
        else:
            assert SRC.count(old) == 1, name
            text = SRC.replace(old, new)
        src = d / f"{name}.c"
        src.write_text(text)
        lib = str(d / f"lib{name}.so")
        obuild.compile_oracle(str(src), lib)
        out[name] = Oracle(lib)
    return out


def _fails(fn, *a, **k):
    try:
        fn(*a, **k)
    except AssertionError:
        return True
    return False


@pytest.mark.parametrize("name", ["no_checkerboard", "energy_sign", "wrong_neighbour"])
def test_physics_pins_catch(mutants, name):
    o = mutants[name]
    assert _fails(pins.check_bruteforce, o, 4, 1.0, 0.0, 2.269185, sweeps=50_000)


def test_observable_pins_catch_bond_sum(mutants):
    o = mutants["bond_sum"]
    assert _fails(pins.check_observables_definition, o)
    assert _fails(pins.check_bm_histogram, o, 4, 1.0, 0.0, 2.269185, sweeps=100_000)


def test_field_pin_catches_dropped_field(mutants):
    o = mutants["field_dropped"]
    assert _fails(pins.check_bruteforce, o, 4, 1.0, 0.1, 2.269185, sweeps=50_000)


def test_kat_catches_philox_slip(mutants):
    o = mutants["philox_key"]
    got = [int(v) for v in o.philox([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344],
                                    [0xa4093822, 0x299f31d0])]
    assert got != [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]


def test_cross_oracle_catches_colour_order(mutants):
    o = mutants["colour_order"]
    a = o.init(16, 5, 0.5)
    b = mini.initial_state(16, 5, 0.5)
    Ba, _ = o.run(a, 1.0, 0.0, 2.269185, 5, 0, 10)
    Bb, _ = mini.run(b, 1.0, 0.0, 2.269185, 5, 0, 10)
    assert not np.array_equal(a, b)


def test_init_pin_catches_compare(mutants):
    o = mutants["init_compare"]
    assert not np.all(o.init(16, 1, 1.0) == 1)


def test_real_oracle_passes_the_same_checks(oracle1):
    pins.check_observables_definition(oracle1)
    pins.check_bm_histogram(oracle1, 4, 1.0, 0.0, 2.269185, sweeps=100_000)
    pins.check_bruteforce(oracle1, 4, 1.0, 0.0, 2.269185, sweeps=50_000)
    pins.check_bruteforce(oracle1, 4, 1.0, 0.1, 2.269185, sweeps=50_000)


@pytest.mark.parametrize("name", ["creutz_sign", "creutz_neighbour", "creutz_cap"])
def test_creutz_conservation_catches(mutants, name):
    o = mutants[name]
    caught = any(_fails(pins.check_creutz_conservation, o, L, 5, 0.5, dem)
                 for L, dem in [(16, ("uniform", 3)), (32, 255)])
    assert caught


def test_creutz_reversibility_catches_strict_demon(mutants):
    o = mutants["creutz_strict"]
    assert _fails(pins.check_creutz_reversible, o, 16, 4, 0.5, 0)


def test_real_oracle_passes_the_creutz_checks(oracle1):
    for L, dem in [(16, ("uniform", 3)), (32, 255)]:
        pins.check_creutz_conservation(oracle1, L, 5, 0.5, dem)
    pins.check_creutz_reversible(oracle1, 16, 4, 0.5, 0)


@pytest.mark.parametrize("name", ["perc_wrap", "perc_arrival", "perc_diagonal"])
def test_percolation_library_pins_catch(mutants, name):
    from tests import test_oracle_percolation as tp
    o = mutants[name]
    caught = any(_fails(tp.test_cluster_and_arrival_match_library, o, L, P, seed)
                 for L, P, seed in [(31, 0.59, 2), (64, 0.62, 3)])
    assert caught


def test_percolation_fraction_catches_porosity(mutants):
    from tests import test_oracle_percolation as tp
    assert _fails(tp.test_medium_fraction, mutants["perc_porosity"], 64, 0.3, 1)


def test_real_oracle_passes_the_percolation_checks(oracle1):
    from tests import test_oracle_percolation as tp
    for L, P, seed in [(31, 0.59, 2), (64, 0.62, 3)]:
        tp.test_cluster_and_arrival_match_library(oracle1, L, P, seed)
    tp.test_medium_fraction(oracle1, 64, 0.3, 1)
