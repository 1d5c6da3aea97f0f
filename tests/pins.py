"""Checks that tie an oracle (default or deliberately broken) to results
fixed outside it. Each raises AssertionError when the oracle disagrees.

Used by test_oracle_physics.py on the real oracle and by
test_negative_controls.py on copies with planted mistakes, which must fail
at least one of them.
"""
import numpy as np

from paper_cs_0312006_amd import workloads
from tests import physics


def mc_series(o, L, J, h, T, seed, sweeps, p_up=0.5, burn_frac=0.1):
    s = o.init(L, seed, p_up)
    B, M = o.run(s, J, h, T, seed, 0, sweeps)
    k = int(sweeps * burn_frac)
    return B[k:], M[k:], s


def check_bruteforce(o, L, J, h, T, seed=3, sweeps=200_000, nsig=3.0):
    """<E>/N, <|M|>/N and <M>/N of the Markov chain agree with exact
    enumeration of all 2^(L*L) states within nsig binned standard errors."""
    exact = physics.exact_averages(L, J, h, T)
    B, M, _ = mc_series(o, L, J, h, T, seed, sweeps)
    N = L * L
    E = (-J * B - h * M) / N
    for name, series in (("e", E), ("abs_m", np.abs(M) / N), ("m", M / N)):
        mean, se = physics.binned_mean_se(series)
        tol = nsig * se + 1e-6
        assert abs(mean - exact[name]) <= tol, (name, L, T, h, mean, exact[name], se)


def check_bm_histogram(o, L, J, h, T, seed=5, sweeps=400_000, thin=10):
    """The joint histogram of (B, M) over thinned sweeps matches the exact
    Boltzmann distribution of (B, M) (chi-square, 0.1% level)."""
    _, Bx, Mx = physics.enumerate_states(L)
    p = physics.boltzmann_weights(Bx, Mx, J, h, T)
    keys = Bx * 100003 + Mx
    uniq, inv = np.unique(keys, return_inverse=True)
    pk = np.bincount(inv, weights=p)
    B, M, _ = mc_series(o, L, J, h, T, seed, sweeps)
    B, M = B[::thin], M[::thin]
    obs_keys = B * 100003 + M
    pos = np.searchsorted(uniq, obs_keys)
    assert np.all(uniq[np.minimum(pos, len(uniq) - 1)] == obs_keys), "impossible (B, M) pair"
    counts = np.bincount(pos, minlength=len(uniq)).astype(np.float64)
    n = counts.sum()
    exp = pk * n
    big = exp >= 5
    chi2 = (((counts - exp) ** 2 / np.where(big, exp, 1.0))[big]).sum()
    rest_obs, rest_exp = counts[~big].sum(), exp[~big].sum()
    dof = int(big.sum()) - 1
    if rest_exp >= 5:
        chi2 += (rest_obs - rest_exp) ** 2 / rest_exp
        dof += 1
    from scipy.stats import chi2 as chi2dist
    assert chi2 < chi2dist.ppf(0.999, dof), (chi2, dof, L, T, h)


def half_sweep_transition_matrix(thr, L, c):
    """Exact one-colour transition matrix P_c(s -> s') of an L x L lattice
    (L*L <= 16): colour-c sites flip independently with probability
    thr(s, n) / 2^32, the other colour is unchanged."""
    states, _, _ = physics.enumerate_states(L)
    nstate = len(states)
    colour = np.indices((L, L)).sum(axis=0) % 2
    P = np.zeros((nstate, nstate))
    flat = ((states.reshape(nstate, -1) + 1) // 2)
    weights = 1 << np.arange(L * L)
    for a in range(nstate):
        s = states[a]
        nb = np.roll(s, 1, 0) + np.roll(s, -1, 0) + np.roll(s, 1, 1) + np.roll(s, -1, 1)
        sites = np.argwhere(colour == c)
        probs = []
        for (i, j) in sites:
            si = 1 if s[i, j] > 0 else 0
            ni = (nb[i, j] + 4) // 2
            probs.append(int(thr[si * 5 + ni]) / 2.0 ** 32)
        for mask in range(1 << len(sites)):
            t = s.copy()
            pr = 1.0
            for k, (i, j) in enumerate(sites):
                if mask >> k & 1:
                    t[i, j] = -t[i, j]
                    pr *= probs[k]
                else:
                    pr *= 1.0 - probs[k]
            b = int((((t.reshape(-1) + 1) // 2) * weights).sum())
            P[a, b] += pr
    return P, flat


def check_half_sweep_transitions(o, L=2, J=1.0, h=0.1, T=2.269185, reps=8000, nsig=4.5):
    """Starting the oracle's one-colour pass from every state of a 2 x 2
    lattice, with reps different sweep indices each, the empirical
    distribution of the resulting state matches the exact transition matrix
    of the Metropolis rule (binomial errors), for both colours."""
    thr = o.table(J, h, T)
    states, _, _ = physics.enumerate_states(L)
    weights = 1 << np.arange(L * L)
    for c in (0, 1):
        P, _ = half_sweep_transition_matrix(thr, L, c)
        for a in range(len(states)):
            counts = np.zeros(len(states))
            for t in range(reps):
                s = states[a].astype(np.int8).copy()
                o.half_sweep(s, thr, 17, t, c)
                b = int((((s.reshape(-1).astype(np.int64) + 1) // 2) * weights).sum())
                counts[b] += 1
            freq = counts / reps
            se = np.sqrt(np.maximum(P[a] * (1 - P[a]), 1e-12) / reps)
            assert np.all(np.abs(freq - P[a]) <= nsig * se + 1e-9), (c, a, freq, P[a])


def check_kaufman(o, L, T, seed=9, sweeps=200_000, nsig=3.0):
    """<E>/N at zero field matches Kaufman's exact finite-lattice value."""
    exact = physics.kaufman_energy(L, T)
    B, _, _ = mc_series(o, L, 1.0, 0.0, T, seed, sweeps)
    mean, se = physics.binned_mean_se(-B / (L * L))
    assert abs(mean - exact) <= nsig * se, (L, T, mean, exact, se)


def check_onsager(o, L, T, p_up, seed=21, sweeps=20_000, nsig=3.0):
    """At T far from T_c on a lattice much larger than the correlation
    length, <E>/N matches Onsager's infinite-lattice energy and <|M|>/N
    matches Yang's spontaneous magnetisation (0 above T_c)."""
    B, M, _ = mc_series(o, L, 1.0, 0.0, T, seed, sweeps, p_up=p_up)
    N = L * L
    mean, se = physics.binned_mean_se(-B / N)
    assert abs(mean - physics.onsager_energy(T)) <= nsig * se, (T, mean, se)
    mabs, mse = physics.binned_mean_se(np.abs(M) / N)
    yang = physics.yang_magnetisation(T)
    if yang > 0:
        assert abs(mabs - yang) <= nsig * mse, (T, mabs, yang, mse)
    else:
        assert mabs < 0.05


def check_observables_definition(o, sizes=(2, 4, 8, 12), seed=4):
    """B counts each periodic edge once and M = #up - #down (Section 2.2),
    compared with an edge-by-edge loop on random lattices."""
    rng = np.random.default_rng(seed)
    for L in sizes:
        s = np.where(rng.random((L, L)) < 0.4, 1, -1).astype(np.int8)
        b_edges = 0
        for i in range(L):
            for j in range(L):
                b_edges += int(s[i, j]) * int(s[i, (j + 1) % L]) + int(s[i, j]) * int(s[(i + 1) % L, j])
        up = int((s > 0).sum())
        assert o.observables(s) == (b_edges, up - (L * L - up)), L


# ---------------------------------------------------------------------------
# Creutz demon dynamics (the deterministic alternative of Section 2.2)
# ---------------------------------------------------------------------------
def creutz_start(o, L, seed, p_up, demons):
    """Seeded start: spins from the oracle's initial draw, demons either a
    constant or uniform on 0..demons[1] (demons = ("uniform", hi))."""
    s = o.init(L, seed, p_up)
    if isinstance(demons, tuple):
        d = workloads.random_demons(L, seed, demons[1])
    else:
        d = np.full((L, L), demons, dtype=np.uint8)
    return s, d


def check_creutz_conservation(o, L, seed, p_up, demons, sweeps=200):
    """Spin energy plus demon energy, -B + 4 D in units of J, is the same
    after every sweep, and the series agree with recomputed observables."""
    s, d = creutz_start(o, L, seed, p_up, demons)
    b0, _ = o.observables(s)
    e0 = -b0 + 4 * o.demon_sum(d)
    B, M, D = o.creutz_run(s, d, sweeps)
    assert np.all(-B + 4 * D == e0), "energy not conserved"
    assert (int(B[-1]), int(M[-1])) == o.observables(s)
    assert int(D[-1]) == int(d.astype(np.int64).sum())


def check_creutz_reversible(o, L, seed, p_up, demons, sweeps=100):
    """n sweeps followed by n reversed sweeps restore spins and demons."""
    s, d = creutz_start(o, L, seed, p_up, demons)
    s0, d0 = s.copy(), d.copy()
    o.creutz_run(s, d, sweeps, series=False)
    moved = not np.array_equal(s, s0)
    o.creutz_run(s, d, sweeps, reverse=True, series=False)
    assert moved, "dynamics froze: the reversibility check would be vacuous"
    assert np.array_equal(s, s0) and np.array_equal(d, d0), "reversed sweeps do not undo the forward ones"


def demon_temperature(d_mean):
    """Temperature (units of J) at which a demon with energies 4J k,
    k = 0, 1, 2, ..., has mean k = d_mean: <k> = 1 / (exp(4 / T) - 1)."""
    return 4.0 / np.log1p(1.0 / d_mean)


def check_creutz_thermometer(o, L, seed, p_up, sweeps=12_000, burn=2_000, n_bins=40, nsig=4.0):
    """Creutz's microcanonical chain, read through its demons, reproduces
    the canonical energy: the mean energy per site equals the exact finite-
    lattice energy (Kaufman) at the temperature the mean demon energy
    indicates. Residuals are taken per time bin, so the correlated errors
    of the energy and of the demon temperature are both accounted for."""
    s, d = creutz_start(o, L, seed, p_up, 0)
    B, M, D = o.creutz_run(s, d, sweeps)
    N = L * L
    u = -B[burn:] / N
    dm = D[burn:] / N
    k = len(u) // n_bins
    r = []
    for b in range(n_bins):
        ub = u[b * k:(b + 1) * k].mean()
        T = demon_temperature(dm[b * k:(b + 1) * k].mean())
        r.append(ub - physics.kaufman_energy(L, T))
    r = np.array(r)
    se = r.std(ddof=1) / np.sqrt(n_bins)
    assert abs(r.mean()) < nsig * se + 2e-4, (r.mean(), se)
    return demon_temperature(dm.mean())
