"""Pins for the acceptance thresholds (Section 2.2, Metropolis steps 2-4).

The threshold for a spin s whose neighbours sum to n is
floor(exp(-dE/T) * 2^32) with dE = 2 s (J n + h), or 2^32 when dE <= 0.
Here each entry is recomputed at 60 significant digits with mpmath from the
same double-precision inputs; the oracle's libm value may differ from the
exact floor by at most one unit (exp's rounding) and must match it
whenever the exact product is not within 2^-20 of an integer.
"""
import math

import mpmath
import numpy as np
import pytest

CASES = [
    (1.0, 0.0, 2.269185), (1.0, 0.1, 2.269185), (1.0, 0.0, 1.5), (1.0, 0.0, 3.5),
    (1.0, 0.05, 1.0), (1.0, 0.0, 4.0), (0.5, -0.3, 0.7), (-1.0, 0.0, 2.0),
    (1.0, 2.5, 1.3), (1.0, 0.0, 1e-3), (1.0, 0.0, 1e300),
]


def _exact(J, h, T, s, n):
    dE = 2.0 * s * (J * n + h)          # same double evaluation as the oracle
    if dE <= 0.0:
        return 1 << 32, None
    mpmath.mp.dps = 60
    x = mpmath.exp(-mpmath.mpf(dE) / mpmath.mpf(T)) * (2 ** 32)
    fl = int(mpmath.floor(x))
    return fl, float(x - fl)


@pytest.mark.parametrize("J,h,T", CASES)
def test_thresholds_against_high_precision(oracle, J, h, T):
    thr = oracle.table(J, h, T)
    for si, s in enumerate((-1, 1)):
        for ni, n in enumerate((-4, -2, 0, 2, 4)):
            want, frac = _exact(J, h, T, s, n)
            got = int(thr[si * 5 + ni])
            assert 0 <= got <= 1 << 32
            if frac is None:
                assert got == want
            elif 2 ** -20 < frac < 1 - 2 ** -20:
                assert got == want, (s, n, got, want)
            else:
                assert abs(got - want) <= 1


def test_special_temperatures(oracle):
    # very high T: every move accepted; very low T: no uphill move accepted
    assert all(int(v) == 1 << 32 for v in oracle.table(1.0, 0.0, 1e300))
    low = oracle.table(1.0, 0.0, 1e-3)
    for si, s in enumerate((-1, 1)):
        for ni, n in enumerate((-4, -2, 0, 2, 4)):
            dE = 2 * s * n
            assert int(low[si * 5 + ni]) == (1 << 32 if dE <= 0 else 0)


def test_symmetry_at_zero_field(oracle):
    # at h = 0, dE(s, n) = dE(-s, -n)
    thr = oracle.table(1.0, 0.0, 2.269185).reshape(2, 5)
    assert np.array_equal(thr[0], thr[1][::-1])


def test_single_flip_detailed_balance(oracle):
    """For each neighbour sum n, the stationary weights of the two values of
    one spin, pi(s) ~ exp(s (J n + h) / T), balance the integer acceptance
    probabilities: pi(+) p(+ -> -) = pi(-) p(- -> +), up to the table's
    2^-32 resolution (Section 2.2, Boltzmann ratio)."""
    for J, h, T in [(1.0, 0.1, 2.269185), (1.0, 0.0, 1.5), (0.5, -0.3, 0.7)]:
        thr = oracle.table(J, h, T).reshape(2, 5)
        for ni, n in enumerate((-4, -2, 0, 2, 4)):
            w_up = math.exp((J * n + h) / T)
            w_dn = math.exp(-(J * n + h) / T)
            z = w_up + w_dn
            lhs = w_up / z * (int(thr[1][ni]) / 2.0 ** 32)
            rhs = w_dn / z * (int(thr[0][ni]) / 2.0 ** 32)
            assert abs(lhs - rhs) <= 2.0 ** -31


def test_mini_table_agrees(oracle):
    from oracle import mini
    for J, h, T in CASES:
        thr = oracle.table(J, h, T)
        m = mini.acceptance_thresholds(J, h, T)
        for si, s in enumerate((-1, 1)):
            for ni, n in enumerate((-4, -2, 0, 2, 4)):
                assert int(thr[si * 5 + ni]) == m[(s, n)]


def test_invalid_parameters_rejected(oracle):
    for J, h, T in [(1.0, 0.0, 0.0), (1.0, 0.0, -1.0), (1.0, 0.0, float("nan")),
                    (float("inf"), 0.0, 1.0), (1.0, float("nan"), 1.0), (1.0, 0.0, float("inf"))]:
        with pytest.raises(ValueError):
            oracle.table(J, h, T)
