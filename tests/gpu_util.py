"""Helpers shared by the GPU parity tests: run one configuration through the
HIP library (via the C ABI binding) and through the oracle on the same
seeded inputs."""
import os
import sys

import numpy as np


def log(msg):
    """Name the case on stdout before each GPU step (flushed), so a run that
    ends abruptly still says what it was doing."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def host_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def gpu_run(b, run, sweeps=None, plan=0, chunks=None):
    """Run `run` (a workloads.Run) on the GPU; returns dict with spins,
    B, M series, hash and obs. `chunks` splits the sweeps over calls."""
    n = run.sweeps if sweeps is None else sweeps
    ctx = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up, plan)
    try:
        parts = chunks or [n]
        assert sum(parts) == n
        for k in parts:
            b.ising_sweep(ctx, k)
        obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES | b.ISING_OBS_HASH)
        spins = b.ising_copy_spins(ctx, run.L)
        info = b.ising_plan_info(ctx)
    finally:
        b.ising_destroy(ctx)
    return {"spins": spins, "B": B, "M": M, "hash": obs.lattice_hash, "obs": obs, "plan": info}


def oracle_run(o, run, sweeps=None):
    n = run.sweeps if sweeps is None else sweeps
    s = o.init(run.L, run.seed, run.p_up)
    B, M = o.run(s, run.J, run.h, run.T, run.seed, 0, n)
    return {"spins": s, "B": B, "M": M, "hash": o.fnv1a64(s)}


def assert_same(g, r, what=""):
    assert np.array_equal(g["B"], r["B"]), f"{what}: bond series differ"
    assert np.array_equal(g["M"], r["M"]), f"{what}: magnetisation series differ"
    if not np.array_equal(g["spins"], r["spins"]):
        bad = np.argwhere(g["spins"] != r["spins"])
        raise AssertionError(f"{what}: {len(bad)} sites differ, first {bad[:5].tolist()}")
    assert g["hash"] == r["hash"], f"{what}: hash differs"
