"""Second, independently written oracle in NumPy, for small lattices only.

TEST INFRASTRUCTURE (see oracle/__init__.py). It is written from the same
reading of Section 2.2 of the paper as the C oracle but with different code
(whole-array operations, np.roll neighbours, a vectorised Philox), so that a
slip in one of them shows up as a mismatch between the two.
"""
import math

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 on arrays of counters (uint64 arrays holding 32-bit
    values) and a scalar key; returns the four output words as uint64 arrays."""
    x0, x1, x2, x3 = (np.asarray(v, dtype=np.uint64) & _MASK for v in (c0, c1, c2, c3))
    ka, kb = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for r in range(10):
        if r:
            ka = (ka + _W0) & 0xFFFFFFFF
            kb = (kb + _W1) & 0xFFFFFFFF
        prod0 = _M0 * x0
        prod1 = _M1 * x2
        x0, x1, x2, x3 = (
            (prod1 >> np.uint64(32)) ^ x1 ^ np.uint64(ka),
            prod1 & _MASK,
            (prod0 >> np.uint64(32)) ^ x3 ^ np.uint64(kb),
            prod0 & _MASK,
        )
    return x0, x1, x2, x3


def uniforms(L, seed, t, colour, domain):
    """Per-site 32-bit draws for every site of the given colour of an L x L
    lattice (array of shape (L, L); entries of the other colour are 0)."""
    i, j = np.meshgrid(np.arange(L, dtype=np.uint64), np.arange(L, dtype=np.uint64),
                       indexing="ij")
    ordinal = (i * np.uint64(L) + j) >> np.uint64(1)
    group = ordinal >> np.uint64(2)
    words = philox4x32_10(group, np.full_like(group, t), np.full_like(group, colour),
                          np.full_like(group, domain), seed & 0xFFFFFFFF, seed >> 32)
    lane = (ordinal & np.uint64(3)).astype(np.int64)
    stacked = np.stack(words, axis=0)
    u = np.take_along_axis(stacked, lane[None, :, :], axis=0)[0]
    mine = ((i + j) & np.uint64(1)) == np.uint64(colour)
    return np.where(mine, u, np.uint64(0))


def acceptance_thresholds(J, h, T):
    """dict (s, n) -> integer threshold in [0, 2^32]: flip when draw < value."""
    out = {}
    for s in (-1, 1):
        for n in (-4, -2, 0, 2, 4):
            dE = 2.0 * s * (J * n + h)
            out[(s, n)] = 1 << 32 if dE <= 0.0 else int(math.floor(math.exp(-dE / T) * 4294967296.0))
    return out


def initial_state(L, seed, p_up):
    cut = int(math.floor(p_up * 4294967296.0))
    up = np.zeros((L, L), dtype=bool)
    for colour in (0, 1):
        u = uniforms(L, seed, 0, colour, 1)
        idx = np.indices((L, L)).sum(axis=0) % 2 == colour
        up |= idx & (u < np.uint64(cut))
    return np.where(up, 1, -1).astype(np.int8)


def sweep(s, J, h, T, seed, t):
    """One sweep (colour 0 then colour 1) in place; returns (B, M)."""
    L = s.shape[0]
    thr = acceptance_thresholds(J, h, T)
    parity = np.indices((L, L)).sum(axis=0) % 2
    for colour in (0, 1):
        nb = (np.roll(s, 1, 0).astype(np.int64) + np.roll(s, -1, 0) + np.roll(s, 1, 1)
              + np.roll(s, -1, 1))
        limit = np.zeros((L, L), dtype=np.uint64)
        for (sv, nv), val in thr.items():
            sel = (s == sv) & (nb == nv)
            limit[sel] = np.uint64(val)
        u = uniforms(L, seed, t, colour, 0)
        flip = (parity == colour) & (u < limit)
        s[flip] = -s[flip]
    return bond_sum(s), int(s.astype(np.int64).sum())


def bond_sum(s):
    s64 = s.astype(np.int64)
    return int((s64 * (np.roll(s64, -1, 1) + np.roll(s64, -1, 0))).sum())


def run(s, J, h, T, seed, t0, n):
    B = np.zeros(n, dtype=np.int64)
    M = np.zeros(n, dtype=np.int64)
    for k in range(n):
        B[k], M[k] = sweep(s, J, h, T, seed, t0 + k)
    return B, M


def creutz_sweep(s, d, reverse=False):
    """One Creutz demon sweep in place (Section 2.2's deterministic
    alternative): per colour, a site moves iff its demon (units of 4J) can
    take the energy change and stay within 0..255. Returns (B, M, D)."""
    L = s.shape[0]
    parity = np.indices((L, L)).sum(axis=0) % 2
    for colour in ((1, 0) if reverse else (0, 1)):
        nb = (np.roll(s, 1, 0).astype(np.int64) + np.roll(s, -1, 0) + np.roll(s, 1, 1)
              + np.roll(s, -1, 1))
        e = s.astype(np.int64) * nb // 2
        dem = d.astype(np.int64)
        move = (parity == colour) & (e <= dem) & (dem - e <= 255)
        s[move] = -s[move]
        d[move] = (dem - e)[move].astype(np.uint8)
    return bond_sum(s), int(s.astype(np.int64).sum()), int(d.astype(np.int64).sum())
