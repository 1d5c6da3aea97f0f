"""Seeded synthetic inputs for the benchmark and the tests.

This module holds no arithmetic of the method: it only names the workload
configurations (lattice sides, temperatures, fields, seeds, sweep counts,
request streams) and draws the random choices they call for, so that the
HIP path and the oracle are fed identical inputs. The paper measures no
public dataset; its workloads are synthetic L x L lattices (Table 4, Figs.
2-3), which these stand in for.
"""
from dataclasses import dataclass, field

import numpy as np

T_C_CONFIG = 2.269185


@dataclass(frozen=True)
class Run:
    L: int
    J: float = 1.0
    h: float = 0.0
    T: float = T_C_CONFIG
    seed: int = 0
    p_up: float = 0.5
    sweeps: int = 1

    def attempts(self):
        return self.L * self.L * self.sweeps


# 64 x 64 at the critical temperature, seed 1, 1000 sweeps
C0 = Run(L=64, seed=1, sweeps=1000)

# 4096 x 4096 (16 MiB int8, cache-resident), three temperatures, seed 7
C1 = [Run(L=4096, T=T, seed=7, sweeps=2000) for T in (1.5, T_C_CONFIG, 3.5)]

# 32768 x 32768 (1 GiB int8), h in {0, 0.1}, cold (all up) and hot starts; seed 11
C2 = [Run(L=32768, h=h, T=T_C_CONFIG, seed=11, p_up=p, sweeps=500)
      for h in (0.0, 0.1) for p in (1.0, 0.5)]
C2_HEADLINE = C2[1]  # h = 0, hot start


def batched(count=1024, sweeps=10000, rng_seed=0):
    """Independent lattices of uneven sizes: L = 32 + 16 * U{0..62},
    T ~ U[1.5, 3.5], h = 0, seed = index."""
    rng = np.random.default_rng(rng_seed)
    Ls = 32 + 16 * rng.integers(0, 63, size=count)
    Ts = rng.uniform(1.5, 3.5, size=count)
    return [Run(L=int(L), T=float(T), seed=i, sweeps=sweeps) for i, (L, T) in enumerate(zip(Ls, Ts))]


@dataclass
class Request:
    arrival: float      # seconds after the stream starts
    run: Run


def request_stream(rate, count=256, rng_seed=1, sweeps_range=(1000, 20000), side_units=(1, 32)):
    """Poisson arrivals at `rate` requests/s of solves with L = 64 * U{1..32},
    T ~ U[1, 4], h in {0, 0.05}, sweeps ~ U{1000..20000}, random 64-bit seed."""
    rng = np.random.default_rng(rng_seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    Ls = 64 * rng.integers(side_units[0], side_units[1] + 1, size=count)
    Ts = rng.uniform(1.0, 4.0, size=count)
    hs = rng.choice([0.0, 0.05], size=count)
    sw = rng.integers(sweeps_range[0], sweeps_range[1] + 1, size=count)
    seeds = rng.integers(0, 2 ** 63, size=count, dtype=np.int64).astype(np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=count).astype(np.uint64)
    return [Request(float(a), Run(L=int(L), T=float(T), h=float(h), seed=int(s), sweeps=int(n)))
            for a, L, T, h, s, n in zip(t, Ls, Ts, hs, seeds, sw)]


def random_lattice(L, seed, p_up=0.5):
    """A canonical +1/-1 int8 lattice with i.i.d. spins (NumPy generator)."""
    rng = np.random.default_rng(seed)
    return np.where(rng.random((L, L)) < p_up, 1, -1).astype(np.int8)


def random_demons(L, seed, hi):
    """Canonical (L, L) uint8 demon energies, i.i.d. uniform on 0..hi
    (NumPy generator); units of 4J."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, hi + 1, size=(L, L), dtype=np.uint8)


# Creutz demon dynamics at the headline lattice size: hot start (p = 0.5)
# with empty demons, so the total energy is near 0 and the demons settle at
# a temperature of about 2.56 J.
CREUTZ = Run(L=32768, seed=11, p_up=0.5, sweeps=500)


@dataclass(frozen=True)
class Medium:
    """A porous medium and its invasion source (Section 2.3)."""
    L: int
    porosity: float
    seed: int = 0
    source: int = 0  # 0: every pore of row 0; 1: the point (i0, j0)
    i0: int = 0
    j0: int = 0

    def sites(self):
        return self.L * self.L


# The medium of the paper's Figure 3 (512 x 512, porosity 0.6), and the
# same porosity at the headline lattice size.
PERC_FIG3 = Medium(L=512, porosity=0.6, seed=3)
PERC_HEADLINE = Medium(L=32768, porosity=0.6, seed=11)
