"""Exact results for the 2D periodic Ising model, used to pin the oracle.

None of this code touches the oracle: brute-force enumeration, Onsager's
energy, Yang's spontaneous magnetisation and Kaufman's finite-lattice
partition function are written from their textbook definitions.
Energy convention (Section 2.2 of the paper, with coupling J and field h):
E = -J B - h M, B = sum over edges of s_j s_k, M = sum of spins.
"""
import math

import mpmath as mp
import numpy as np

T_C = 2.0 / math.log(1.0 + math.sqrt(2.0))


def enumerate_states(L):
    """All 2^(L*L) states of an L x L lattice (L*L <= 16) as int64 arrays,
    with their bond sums B and magnetisations M."""
    n = L * L
    idx = np.arange(2 ** n, dtype=np.int64)
    s = ((((idx[:, None] >> np.arange(n)) & 1) * 2) - 1).reshape(-1, L, L)
    B = (s * (np.roll(s, -1, 2) + np.roll(s, -1, 1))).sum(axis=(1, 2))
    M = s.sum(axis=(1, 2))
    return s, B, M


def boltzmann_weights(B, M, J, h, T):
    """Normalised Boltzmann probabilities of states with given (B, M)."""
    logw = (J * B.astype(np.float64) + h * M.astype(np.float64)) / T
    logw -= logw.max()
    w = np.exp(logw)
    return w / w.sum()


def exact_averages(L, J, h, T):
    _, B, M = enumerate_states(L)
    p = boltzmann_weights(B, M, J, h, T)
    N = L * L
    E = -J * B - h * M
    return {
        "e": float((p * E).sum() / N),
        "abs_m": float((p * np.abs(M)).sum() / N),
        "m": float((p * M).sum() / N),
        "m2": float((p * M.astype(np.float64) ** 2).sum() / N ** 2),
    }


def onsager_energy(T, J=1.0):
    """Energy per site of the infinite lattice at zero field (Onsager 1944):
    u = -J coth(2K) [1 + (2/pi) (2 tanh^2(2K) - 1) K1(k)], K = J/T,
    k = 2 sinh(2K) / cosh^2(2K), K1 the complete elliptic integral of the
    first kind (mpmath's ellipk takes the parameter k^2)."""
    mp.mp.dps = 30
    K = mp.mpf(J) / mp.mpf(T)
    k = 2 * mp.sinh(2 * K) / mp.cosh(2 * K) ** 2
    u = -J / mp.tanh(2 * K) * (1 + (2 / mp.pi) * (2 * mp.tanh(2 * K) ** 2 - 1) * mp.ellipk(k ** 2))
    return float(u)


def yang_magnetisation(T, J=1.0):
    """Spontaneous magnetisation per site (Yang 1952): (1 - sinh^-4(2J/T))^(1/8)
    below T_c, 0 above."""
    if T >= T_C:
        return 0.0
    return (1.0 - math.sinh(2.0 * J / T) ** -4) ** 0.125


def kaufman_log_z(L, K):
    """ln Z of the periodic L x L lattice at zero field, K = J/T (Kaufman 1949,
    in the form of Ferdinand and Fisher 1969): Z = 1/2 (2 sinh 2K)^(N/2)
    (Z1 + Z2 + Z3 + Z4), with products over r = 0..L-1 of 2cosh/2sinh of
    L gamma_(2r+1)/2 and L gamma_(2r)/2, where
    cosh gamma_l = cosh 2K coth 2K - cos(pi l / L) and gamma_0 = 2K + ln tanh K."""
    K = mp.mpf(K)
    c = mp.cosh(2 * K) / mp.tanh(2 * K)

    def gamma(l):
        if l == 0:
            return 2 * K + mp.log(mp.tanh(K))
        return mp.acosh(c - mp.cos(mp.pi * l / L))

    z1 = z2 = z3 = z4 = mp.mpf(1)
    for r in range(L):
        a, b = gamma(2 * r + 1), gamma(2 * r)
        z1 *= 2 * mp.cosh(L * a / 2)
        z2 *= 2 * mp.sinh(L * a / 2)
        z3 *= 2 * mp.cosh(L * b / 2)
        z4 *= 2 * mp.sinh(L * b / 2)
    return mp.log(mp.mpf(1) / 2) + (L * L / mp.mpf(2)) * mp.log(2 * mp.sinh(2 * K)) + mp.log(z1 + z2 + z3 + z4)


def kaufman_energy(L, T, J=1.0):
    """Exact <E>/N of the finite periodic L x L lattice at zero field:
    -(J/N) d ln Z / dK."""
    mp.mp.dps = 40
    K = mp.mpf(J) / mp.mpf(T)
    return float(-J * mp.diff(lambda k: kaufman_log_z(L, k), K) / (L * L))


def binned_mean_se(x, n_blocks=100):
    """Mean and standard error of a correlated series from the spread of
    n_blocks block means (block length >> autocorrelation time)."""
    x = np.asarray(x, dtype=np.float64)
    m = len(x) // n_blocks
    blocks = x[: m * n_blocks].reshape(n_blocks, m).mean(axis=1)
    return float(blocks.mean()), float(blocks.std(ddof=1) / math.sqrt(n_blocks))
