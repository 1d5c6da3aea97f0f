"""Benchmark of the checkerboard Metropolis engine on one MI355X.

One step is one full sweep (colour 0, colour 1, per-sweep bond sum and
magnetisation) of a 32768 x 32768 lattice at T = 2.269185, J = 1, h = 0, hot
start with seed 11; the lattice (1 GiB of int8 spins in colour planes) is
resident in HBM before the timed region. Prints one JSON line.

Also reported: the other three 32768^2 runs (h = 0.1, cold starts), the
batched configuration (1024 lattices of uneven size, against one launch per
lattice on a sample), the served request stream, Creutz demon sweeps,
percolation media, the vector-op and transfer micro-benchmarks, the oracle
timed on the host cores (cpu_baseline), and roofline figures for the
dominant kernel.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9  # 256 CUs x 64 lanes x 2.4 GHz (32-bit ops)

# Figures measured with rocprofv3 for the kernels as built from these
# sources (profiles/*.md). Each is keyed by a hash of the kernel's sources
# and reported only while the tree still hashes to it (otherwise null): a
# changed kernel is profiled again, never carried forward. HBM bytes are
# FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB per dispatch): a 1 GiB device
# copy in the same runs reads 524300 KiB of FETCH_SIZE and writes 1048576
# KiB of WRITE_SIZE. VALU lane-ops are SQ_INSTS_VALU x 64; VALU busy is
# SQ_ACTIVE_INST_VALU / 256 compute units / (GRBM_GUI_ACTIVE / 8 XCDs).
PROFILED_SOURCES = "aaf5cc389756ada4"
PROFILED = {
    # profiles/k_fused_rows_ising2d_32768.md: FETCH/WRITE means of 140
    # dispatches, VALU counters of the 35 in the counter pass
    "k_fused_rows<4,128>": {"hbm_bytes_per_launch": (532789.7 * 2.0 + 1048621.0) * 1024,
                            "valu_lane_ops_per_attempt": 231620842.4 * 64 / 2 ** 30,
                            "valu_busy_rocprof": 0.845},
    # the wave-tile shape the autotuner takes when it beats the full rows by
    # more than its margin (same passes: 27 dispatches for bytes, 132 for VALU)
    "k_fused<4,32>": {"hbm_bytes_per_launch": (647856.8 * 2.0 + 1048835.0) * 1024,
                      "valu_lane_ops_per_attempt": 227870305.6 * 64 / 2 ** 30,
                      "valu_busy_rocprof": 0.842},
}


# Creutz: the fused sweep at 32768^2 (profiles/k_creutz_fused_creutz_32768.md,
# mean of 22 dispatches)
PROFILED_CREUTZ_SOURCES = "6787c46f73def973"
PROFILED_CREUTZ = {"kernel": "k_creutz_fused<4,32>",
                   "hbm_bytes_per_sweep": (1246597.4 * 2.0 + 2097426.2) * 1024}

# Batched configuration (1024 lattices): the resident kernel the tuned AUTO
# plan runs (profiles/k_batch_bits_batched_1024.md, one dispatch of 2000
# sweeps) and the stepped plan's fused walk (profiles/k_multi_fused_batched_1024.md,
# mean of 160 dispatches, 16-row tiles)
BATCH_FILES = ("ising_batch.hip", "ising_bits.hpp", "ising_device.hpp", "ising_launch.hpp")
PROFILED_BATCH_SOURCES = "e86f8f0d0ff597dc"
PROFILED_BATCH = {"kernel": "k_batch (bit-packed lattices in workgroup memory)",
                  "valu_lane_ops_per_attempt": 192905902547.0 * 64 / (388630784 * 2000),
                  "valu_busy_rocprof": 0.932}
MULTI_FUSED_FILES = ("ising_multi_fused.hip", "ising_fused_core.hpp", "ising_device.hpp", "ising_launch.hpp")
PROFILED_MULTI_FUSED_SOURCES = "562f1a3a50200cd3"
PROFILED_MULTI_FUSED = {"kernel": "k_multi_fused (one launch per sweep)",
                        "valu_lane_ops_per_attempt": 131454301.0 * 64 / 388630784,
                        "valu_busy_rocprof": 0.887,
                        "hbm_bytes_per_sweep": (244661.1 * 2.0 + 412989.1) * 1024}


def batched_roofline(res, stepped):
    """ALU roof of the batched leg's kernel from its profiled ops per site
    update, or None when its sources have changed since the profile."""
    files, src, prof = ((MULTI_FUSED_FILES, PROFILED_MULTI_FUSED_SOURCES, PROFILED_MULTI_FUSED) if stepped
                        else (BATCH_FILES, PROFILED_BATCH_SOURCES, PROFILED_BATCH))
    if kernel_sources_hash(files) != src:
        return None
    ops = prof["valu_lane_ops_per_attempt"] * res["value"] * 1e9
    roof = {"bound": "alu", "achieved": ops / 1e12, "peak": VALU_PEAK_LANE_OPS / 1e12,
            "unit": "T lane-ops/s (32-bit VALU)", "frac": ops / VALU_PEAK_LANE_OPS, "kernel": prof["kernel"],
            "ops_per_attempt": prof["valu_lane_ops_per_attempt"], "valu_busy_rocprof": prof["valu_busy_rocprof"],
            "traffic": None}
    if stepped:
        sweep_s = res["ms"] * 1e-3 / res["sweeps"]
        roof["traffic"] = prof["hbm_bytes_per_sweep"] / sweep_s / 1e9
        roof["traffic_unit"] = "GB/s"
        roof["algorithmic_hbm_GBs"] = 2.0 * res["attempts"] / res["sweeps"] / sweep_s / 1e9
    return roof


HEADLINE_FILES = ("ising_fused.hip", "ising_fused_rows.hip", "ising_fused_core.hpp", "ising_device.hpp",
                  "ising_launch.hpp")


def headline_profile(kname):
    """The recorded counters of the timed headline kernel, or None when the
    sources changed since they were taken."""
    if kernel_sources_hash() != PROFILED_SOURCES:
        return None
    return PROFILED.get(kname)


def kernel_sources_hash(files=HEADLINE_FILES):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_cs_0312006_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


CREUTZ_FILES = ("ising_creutz_fused.hip", "ising_creutz.hpp", "ising_device.hpp", "ising_launch.hpp")


def progress(msg):
    """One line on stderr per finished leg (the JSON result goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cores():
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


def run_headline(b, torch, stream, run, steps, warmup, tune=True, force=None, first=2, force_plan=5):
    """Returns dict with timing, plan and the series of the first sweeps."""
    ctx = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up, stream=stream.cuda_stream)
    try:
        # first sweeps from the initial state, kept for the oracle cross-check
        b.ising_sweep(ctx, first)
        _, B0, M0 = b.ising_observables(ctx, b.ISING_OBS_SERIES)
        if force:
            b.ising_plan_set(ctx, force_plan, force[0], force[1])
        elif tune:
            b.ising_tune(ctx, 8)
        plan = b.ising_plan_info(ctx)
        if warmup:
            b.ising_sweep(ctx, warmup)
        b.ising_observables(ctx, b.ISING_OBS_SERIES)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t_host0 = time.perf_counter()
        e0.record(stream)
        b.ising_sweep(ctx, steps)
        e1.record(stream)
        e1.synchronize()
        torch.cuda.synchronize()
        host_s = time.perf_counter() - t_host0
        ms = e0.elapsed_time(e1)
        obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES)
    finally:
        b.ising_destroy(ctx)
    return {"ms": ms, "host_s": host_s, "plan": plan, "B0": B0, "M0": M0, "B": B, "M": M, "obs": obs}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(run, sweeps, B0, M0):
    """The oracle (plain C, OpenMP over rows) on the host cores: initial
    state plus `sweeps` sweeps of the same lattice; its series must equal
    the GPU's first sweeps."""
    from oracle import ref
    o = ref.Oracle()
    cores = min(16, host_cores())
    o.set_threads(cores)
    t0 = time.perf_counter()
    s = o.init(run.L, run.seed, run.p_up)
    t1 = time.perf_counter()
    B, M = o.run(s, run.J, run.h, run.T, run.seed, 0, sweeps)
    t2 = time.perf_counter()
    attempts = run.L * run.L * sweeps
    parity = bool((list(B) == list(B0[:sweeps])) and (list(M) == list(M0[:sweeps])))
    del s
    return {
        "value": attempts / (t2 - t1) / 1e9,
        "unit": "spin-update attempts/ns",
        "cores": cores,
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": f"{sweeps} sweeps of the {run.L}x{run.L} lattice from its initial state "
                  f"(init {t1 - t0:.1f} s not counted); series equal to the GPU's: {parity}",
    }, parity


def run_batched(b, torch, stream, count, sweeps, sample, plan=0):
    """1024 lattices (L = 32 + 16 U{0..62}, T ~ U[1.5, 3.5], h = 0, seed =
    index) in one batch call with the given plan (0: the tuned AUTO plan).
    Comparator (sample > 0): one lattice of every side (the first of that
    side in the generator's order), each on its own context with the
    single-lattice plan ising_tune picks for its side (graph replays for the
    two-pass plan), its whole run as one ising_sweep call, back to back on
    one stream; per-lattice device times give a rate per side, from which
    the whole configuration's time one lattice at a time is estimated."""
    from paper_cs_0312006_amd import workloads as W
    runs = W.batched(count=count, sweeps=sweeps)
    total = sum(r.attempts() for r in runs)
    firsts = {}
    for k, r in enumerate(runs):
        firsts.setdefault(r.L, k)
    picked = sorted(firsts.values()) if sample > 0 else []
    ctxs = [b.ising_create(r.L, r.J, r.h, r.T, r.seed, r.p_up, stream=stream.cuda_stream) for r in runs]
    try:
        choice = b.ising_batch_choice(ctxs, [r.sweeps for r in runs])
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.ising_sweep_batch_plan(ctxs, [r.sweeps for r in runs], plan, stream=stream.cuda_stream)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        hashes = {}
        for k in sorted(set(range(min(64, len(runs)))) | set(picked)):
            obs, _, _ = b.ising_observables(ctxs[k], b.ISING_OBS_HASH | b.ISING_OBS_SERIES)
            hashes[k] = obs.lattice_hash
    finally:
        for c in ctxs:
            b.ising_destroy(c)
    plan_run = plan or choice[0]
    res = {"lattices": count, "sweeps": sweeps, "attempts": total,
           "value": total / ms / 1e6, "unit": "spin-update attempts/ns", "ms": ms,
           "plan": {1: "resident", 2: "stepped"}[plan_run] + (" (auto)" if plan == 0 else ""),
           "model_prediction_ms": {"resident": choice[2][0] / 1e6, "stepped": choice[2][1] / 1e6,
                                   "stepped_tile_rows": choice[1]}}
    if not picked:
        return res, hashes
    sub = [runs[k] for k in picked]
    ctxs = [b.ising_create(r.L, r.J, r.h, r.T, r.seed, r.p_up, stream=stream.cuda_stream) for r in sub]
    same = True
    try:
        plans = {}
        for c, r in zip(ctxs, sub):
            # the side's plan (remembered for later contexts of that side),
            # from trials long enough that a plan's per-call costs weigh as
            # little as in the timed 10000-sweep call
            b.ising_tune(c, 128)
            plans[r.L] = b.ising_plan_info(c)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(sub) + 1)]
        ev[0].record(stream)
        for k, (c, r) in enumerate(zip(ctxs, sub)):
            b.ising_sweep(c, r.sweeps)
            ev[k + 1].record(stream)
        ev[-1].synchronize()
        per = [ev[k].elapsed_time(ev[k + 1]) for k in range(len(sub))]
        for k, c in zip(picked, ctxs):
            obs, _, _ = b.ising_observables(c, b.ISING_OBS_HASH | b.ISING_OBS_SERIES)
            same &= obs.lattice_hash == hashes[k]
    finally:
        for c in ctxs:
            b.ising_destroy(c)
    rate = {r.L: r.attempts() / t / 1e6 for r, t in zip(sub, per)}  # attempts/ns per side
    est_ms = sum(r.attempts() / rate[r.L] for r in runs) / 1e6
    sub_attempts = sum(r.attempts() for r in sub)
    res["one_launch_per_lattice"] = {
        "sample": f"one lattice per side ({len(sub)} sides, 32 to 1024), each on its own tuned single-lattice plan",
        "lattices": len(sub), "attempts": sub_attempts, "ms": sum(per), "value": sub_attempts / sum(per) / 1e6,
        "plans_by_side": {str(L): {"kind": p[0], "chunk_words": p[1], "tile_rows": p[2]} for L, p in plans.items()},
        "whole_config_estimate_ms": est_ms, "whole_config_estimate_value": total / est_ms / 1e6,
        "results_identical_to_batched": bool(same)}
    res["speedup_vs_one_launch_per_lattice"] = est_ms / ms
    return res, hashes


def plan_report(b, plan, sweeps):
    """A plan as the bench reports it: kind, chunk words and tile (band)
    height, and how many sweeps each pass of the lattice through HBM serves
    for a call of `sweeps` sweeps."""
    per_pass = {b.ISING_PLAN_BANDS: min(sweeps, b.ISING_BAND_SWEEPS_PER_LAUNCH), b.ISING_PLAN_RESIDENT: sweeps,
                b.ISING_PLAN_FUSED: 1, b.ISING_PLAN_FUSED_ROWS: 1, b.ISING_PLAN_TWO_PASS: 0.5,
                b.ISING_PLAN_GENERIC: 0.5}.get(plan[0])
    return {"kind": plan[0], "chunk_words": plan[1], "tile_rows": plan[2], "sweeps_per_hbm_pass": per_pass}


def warm_up(b, ctx, run, sweeps=20):
    """Series room for the timed calls, untimed sweeps and a read-back of
    their series (the context's first-call allocations, the clock ramp, and
    the runtime's one-time set-up of its first large device-to-host copy:
    the first read-back of a 2000-sweep series in a process took 7 ms of
    host time, later ones 0.1 ms), then the context back at the run's
    initial state, plan kept."""
    b.ising_reserve(ctx, run.sweeps + 2000 + sweeps)
    b.ising_sweep(ctx, sweeps)
    b.ising_observables(ctx, b.ISING_OBS_SERIES)
    b.ising_reset(ctx, run.L, run.J, run.h, run.T, run.seed, run.p_up)


def run_small_configs(b, torch, stream, repeats=3):
    """The 64^2 config (1000 sweeps) and the three 4096^2 configs (2000
    sweeps each): throughput over the whole run with the autotuned plan (the
    median of `repeats` runs from the initial state: a run lasts 1.5 to 17
    ms of host clock, where one stall of the host thread would decide a
    single reading), and p50/p99 latency of 10-sweep calls (enqueue to
    result on the host, one call at a time)."""
    import numpy as np
    from paper_cs_0312006_amd import workloads as W
    out = []
    for run in [W.C0] + list(W.C1):
        ctx = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up, stream=stream.cuda_stream)
        try:
            b.ising_tune(ctx, 50)
            plan = b.ising_plan_info(ctx)
            warm_up(b, ctx, run, run.sweeps)  # a whole run: its series read-back is as long as the timed ones
            runs_s = []
            for rep in range(repeats):
                if rep:
                    b.ising_reset(ctx, run.L, run.J, run.h, run.T, run.seed, run.p_up)
                b.ising_observables(ctx, b.ISING_OBS_SERIES)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                b.ising_sweep(ctx, run.sweeps)
                b.ising_observables(ctx, b.ISING_OBS_SERIES)
                runs_s.append(time.perf_counter() - t0)
            whole = float(np.median(runs_s))
            lat = []
            for _ in range(200):
                t1 = time.perf_counter()
                b.ising_sweep(ctx, 10)
                b.ising_observables(ctx, b.ISING_OBS_SERIES)
                lat.append(time.perf_counter() - t1)
        finally:
            b.ising_destroy(ctx)
        lat = np.array(lat)
        out.append({"workload": f"ising2d {run.L}x{run.L} T={run.T} seed {run.seed}, {run.sweeps} sweeps",
                    "plan": plan_report(b, plan, run.sweeps),
                    "value": run.attempts() / whole / 1e9, "unit": "attempts/ns (host clock, incl. series copy)",
                    "s": whole, "runs_s": runs_s, "chunk10_p50_us": float(np.percentile(lat, 50) * 1e6),
                    "chunk10_p99_us": float(np.percentile(lat, 99) * 1e6)})
    return out


def run_c1(b, torch, stream):
    """The three 4096^2 configs on the default plan (no tuning trials, no
    latency calls): 2000 sweeps each, for profiling the sweep kernel alone."""
    from paper_cs_0312006_amd import workloads as W
    out = []
    for run in W.C1:
        ctx = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up, stream=stream.cuda_stream)
        try:
            plan = b.ising_plan_info(ctx)
            warm_up(b, ctx, run)
            b.ising_observables(ctx, 0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.ising_sweep(ctx, run.sweeps)
            b.ising_observables(ctx, b.ISING_OBS_SERIES)
            whole = time.perf_counter() - t0
        finally:
            b.ising_destroy(ctx)
        out.append({"workload": f"ising2d {run.L}x{run.L} T={run.T} seed {run.seed}, {run.sweeps} sweeps",
                    "plan": plan_report(b, plan, run.sweeps),
                    "value": run.attempts() / whole / 1e9, "unit": "attempts/ns (host clock, incl. series copy)",
                    "s": whole})
    return out


def run_served(rates, count, epoch_sweeps):
    """Poisson request streams (L = 64 U{1..32}, T ~ U[1, 4], h in {0, 0.05},
    sweeps ~ U{1000..20000}, random seeds) through the continuous-batching
    server; p50/p99 latency from scheduled arrival to result on the host."""
    from paper_cs_0312006_amd import serve
    from paper_cs_0312006_amd import workloads as W
    out = []
    for rate in [float(x) for x in rates.split(",") if x]:
        ex = serve.GpuExecutor(hash_results=False)
        try:
            reqs = W.request_stream(rate, count=count)
            res, stats = serve.serve(reqs, ex, epoch_sweeps=epoch_sweeps)
        finally:
            ex.close()
        s = serve.summarize(res, stats["makespan_s"])
        progress(f"served {rate:g}/s: {s['attempts_per_ns']:.0f} attempts/ns")
        s.update({"rate_per_s": rate, "epochs": stats["epochs"], "epoch_sweeps": epoch_sweeps,
                  "offered_attempts_per_ns": rate * sum(r.run.attempts() for r in reqs) / len(reqs) / 1e9})
        out.append(s)
    return out


def run_fifo(b, rate, count):
    """Comparator for the served leg: the same request stream, one request
    at a time in arrival order, each on its own context with the
    single-lattice plan ising_tune picked for its side (every side tuned
    before the stream starts), its sweeps as one ising_sweep call, the
    series read back, the context destroyed; p50/p99 from scheduled arrival
    to result on the host."""
    from paper_cs_0312006_amd import serve
    from paper_cs_0312006_amd import workloads as W
    reqs = W.request_stream(rate, count=count)
    for L in sorted({q.run.L for q in reqs}):
        ctx = b.ising_create(L)
        try:
            b.ising_tune(ctx, 128)  # trials long enough for per-call costs to weigh as in a request
        finally:
            b.ising_destroy(ctx)
    results = []
    t0 = time.perf_counter()
    for k, q in enumerate(reqs):
        now = time.perf_counter() - t0
        if now < q.arrival:
            time.sleep(q.arrival - now)
        start = time.perf_counter() - t0
        r = q.run
        ctx = b.ising_create(r.L, r.J, r.h, r.T, r.seed, r.p_up)
        try:
            b.ising_sweep(ctx, r.sweeps)
            obs, _, _ = b.ising_observables(ctx, b.ISING_OBS_SERIES)
        finally:
            b.ising_destroy(ctx)
        results.append(serve.Result(k, r.L, r.sweeps, q.arrival, start, time.perf_counter() - t0,
                                    bond_sum=obs.bond_sum, mag_sum=obs.mag_sum))
    s = serve.summarize(results, max(x.done for x in results))
    progress(f"FIFO {rate:g}/s: {s['attempts_per_ns']:.0f} attempts/ns")
    s.update({"rate_per_s": rate, "comparator": "one request at a time (FIFO), tuned single-lattice plans"})
    return s


def run_creutz(b, torch, stream, sweeps, metropolis_value, cpu=True):
    """Creutz demon sweeps of the 32768^2 hot start with empty demons
    (Section 2.2's random-number-free alternative), timed like the headline;
    algorithmic traffic 4 B per site and sweep (spin and demon bytes, each
    read and written once)."""
    from paper_cs_0312006_amd import workloads as W
    run = W.CREUTZ
    ctx = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up, stream=stream.cuda_stream)
    try:
        b.ising_creutz_init(ctx, None, 0)
        obs0, _, _ = b.ising_observables(ctx, 0)
        b.ising_creutz_sweep(ctx, 2)
        b.ising_observables(ctx, b.ISING_OBS_SERIES)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.ising_creutz_sweep(ctx, sweeps)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        obs, B, M = b.ising_observables(ctx, b.ISING_OBS_SERIES)
        demons = b.ising_demon_sum(ctx)
    finally:
        b.ising_destroy(ctx)
    N = run.L * run.L
    value = N * sweeps / ms / 1e6
    achieved = 4.0 * N / (ms / sweeps * 1e-3) / 1e9
    same = kernel_sources_hash(CREUTZ_FILES) == PROFILED_CREUTZ_SOURCES
    traffic = PROFILED_CREUTZ["hbm_bytes_per_sweep"] / (ms / sweeps * 1e-3) / 1e9 if same else None
    t_demon = 4.0 / __import__("math").log1p(N / demons) if demons else None
    res_cpu = None
    if cpu:
        # the oracle's Creutz sweeps on a 16384^2 sample of the same start
        import numpy as np
        from oracle import ref
        o = ref.Oracle()
        cores = min(16, host_cores())
        o.set_threads(cores)
        Ls, n_cpu = 16384, 4
        s_ = o.init(Ls, run.seed, run.p_up)
        d_ = np.zeros((Ls, Ls), dtype=np.uint8)
        t0 = time.perf_counter()
        o.creutz_run(s_, d_, n_cpu, series=False)
        dt = time.perf_counter() - t0
        res_cpu = {"value": Ls * Ls * n_cpu / dt / 1e9, "unit": "site updates/ns", "cores": cores,
                   "kind": "oracle", "sample": f"{n_cpu} Creutz sweeps of a {Ls}x{Ls} hot start (seed {run.seed}), "
                                               f"empty demons, {dt:.2f} s"}
        del s_, d_
    return {"workload": f"creutz demons {run.L}x{run.L}, hot start seed {run.seed}, demons 0",
            "cpu_baseline": res_cpu,
            "sweeps": sweeps, "value": value, "unit": "site updates/ns", "ms_per_sweep": ms / sweeps,
            "vs_metropolis_headline": value / metropolis_value,
            "energy_conserved": bool(-obs.bond_sum + 4 * demons == -obs0.bond_sum),
            "demon_temperature": t_demon,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                         "kernel": PROFILED_CREUTZ["kernel"] + " (one launch per sweep)",
                         "algorithmic_bytes_per_sweep": 4.0 * N}}


def run_percolation(b, cpu=True, spanning=True):
    """Porous media of Section 2.3 (porosity 0.6): the paper's Figure 3
    size and the headline lattice size; the oracle (plain breadth-first
    search) timed on an 8192^2 medium of the same kind."""
    from paper_cs_0312006_amd import workloads as W
    out = []
    for m in (W.PERC_FIG3, W.PERC_HEADLINE):
        ctx = b.perc_create(m.L, m.porosity, m.seed, m.source, m.i0, m.j0)
        try:
            b.perc_run(ctx)  # warm
            t0 = time.perf_counter()
            b.perc_run(ctx)
            s = time.perf_counter() - t0
            r = b.perc_result_get(ctx)
        finally:
            b.perc_destroy(ctx)
        N = m.L * m.L
        out.append({"workload": f"percolation {m.L}x{m.L} porosity {m.porosity} seed {m.seed}, top-row invasion",
                    "ms": s * 1e3, "value": N / s / 1e9, "unit": "medium sites/ns (draw + invasion to steady state)",
                    "passes_to_steady_state": r.passes, "invaded": r.invaded, "spans": r.spans,
                    "relax_launches": r.launches, "tile_visits": r.tile_visits,
                    "levels_per_visit": r.tile_iterations / max(1, r.tile_visits),
                    "paper_method_equivalent": {
                        "value": N * max(1, r.passes) / s / 1e9,
                        "unit": "site-passes/ns (one full pass per invasion step, as in Section 2.3)"}})
    res = {"runs": out}
    if not spanning:
        return res
    # the spanning threshold (Section 2.3): per-seed porosity from which the
    # medium spans, by bisection (14 halvings of [0.3, 0.9]), for 64 media of
    # the paper's Figure 3 size: all media in one batched run per step, and
    # (comparator) one medium at a time
    import numpy as np
    n_media, side, steps = 64, 512, 14
    ctxs = [b.perc_create(side, 0.5, 1000 + k) for k in range(n_media)]
    try:
        b.perc_run_batch(ctxs)  # warm
        t0 = time.perf_counter()
        lo, hi = np.full(n_media, 0.3), np.full(n_media, 0.9)
        for _ in range(steps):
            mid = 0.5 * (lo + hi)
            for k, c in enumerate(ctxs):
                b.perc_set_params(c, side, float(mid[k]), 1000 + k)
            b.perc_run_batch(ctxs)
            sp = np.array([b.perc_result_get(c).spans & 1 for c in ctxs], dtype=bool)
            hi = np.where(sp, mid, hi)
            lo = np.where(sp, lo, mid)
        t_batch = time.perf_counter() - t0
        t0 = time.perf_counter()
        th_one = []
        for k, c in enumerate(ctxs):
            a, z = 0.3, 0.9
            for _ in range(steps):
                m = 0.5 * (a + z)
                b.perc_set_params(c, side, m, 1000 + k)
                b.perc_run(c)
                a, z = (a, m) if b.perc_result_get(c).spans & 1 else (m, z)
            th_one.append(z)
        t_one = time.perf_counter() - t0
    finally:
        for c in ctxs:
            b.perc_destroy(c)
    res["spanning_threshold_512"] = {"media": n_media, "median": float(np.median(hi)), "mean": float(hi.mean()),
                                     "sd": float(hi.std(ddof=1)), "reference_p_c": 0.592746,
                                     "s_batched": t_batch, "s_one_medium_at_a_time": t_one,
                                     "same_thresholds": bool(list(hi) == th_one)}
    if cpu:
        from oracle import ref
        o = ref.Oracle()
        cores = min(16, host_cores())
        o.set_threads(cores)
        L = 8192
        t0 = time.perf_counter()
        pore = o.perc_medium(L, 0.6, 11)
        t1 = time.perf_counter()
        arr = o.perc_invade(pore, 0)
        t2 = time.perf_counter()
        res["cpu_baseline"] = {"value": L * L / (t2 - t0) / 1e9, "unit": "medium sites/ns", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{L}x{L} medium, porosity 0.6: draw {t1 - t0:.2f} s on {cores} threads, "
                                         f"breadth-first invasion {t2 - t1:.2f} s on one thread; "
                                         f"{int((arr >= 0).sum())} sites invaded"}
    return res


def run_micro(b, torch, stream):
    """The paper's GPU calibration on the MI355X: Table 2's vector ops on
    float vectors of 4 values per site (the paper's 256^2 and 512^2, and a
    1 GiB vector), and Table 5's whole-lattice and border-only transfers
    between pinned host memory and HBM."""
    ops = ["=", "+", "-", "*", "/", "sin", "cos", "log", "exp"]
    vec = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for side in (256, 512, 8192):
        n = 4 * side * side
        a = torch.rand(n, device="cuda") + 0.5
        c = torch.rand(n, device="cuda") + 0.5
        reps = 200 if side < 8192 else 10
        for op in ops:
            torch.cuda.synchronize()
            b.mb_vector_op(op, a.data_ptr(), c.data_ptr(), n, stream.cuda_stream)
            if op in ("sin", "cos", "log", "exp"):
                a.uniform_(0.5, 1.5)  # keep log and exp in range
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(reps):
                b.mb_vector_op(op, a.data_ptr(), c.data_ptr(), n, stream.cuda_stream)
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            nbytes = 4 * n * (2 if op == "=" else (3 if op in "+-*/" else 2))
            vec.append({"op": op, "lattice": side, "floats": n, "s": ms * 1e-3, "GB_per_s": nbytes / ms / 1e6})
        del a, c
    tr = []
    for side in (64, 128, 256, 512, 8192):
        elem = 16  # a float4 texel per site, as the paper's textures
        host = torch.empty(side * side * elem, dtype=torch.uint8).pin_memory()
        dev = torch.empty(side * side * elem, dtype=torch.uint8, device="cuda")
        for name, direction, border in (("read bdr", 1, True), ("read all", 1, False),
                                        ("write bdr", 0, True), ("write all", 0, False)):
            dst, src = (host, dev) if direction == 1 else (dev, host)
            reps = 50 if side < 8192 else 5
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(reps):
                b.mb_copy_lattice(dst.data_ptr(), src.data_ptr(), side, elem, direction, border, stream.cuda_stream)
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            nbytes = (4 * side - 4 if border and side > 2 else side * side) * elem
            tr.append({"op": name, "lattice": side, "bytes": nbytes, "s": ms * 1e-3, "MB_per_s": nbytes / ms / 1e3})
        del host, dev
    # Philox4x32-10 rate (the draws alone): 2^20 threads x 2048 calls
    out = torch.empty(1 << 20, dtype=torch.int32, device="cuda")
    b.mb_philox(out.data_ptr(), 1 << 20, 2048, 11, stream.cuda_stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(5):
        b.mb_philox(out.data_ptr(), 1 << 20, 2048, 11, stream.cuda_stream)
    e1.record(stream)
    e1.synchronize()
    calls_per_ns = 5 * (1 << 20) * 2048 / e0.elapsed_time(e1) / 1e6
    philox = {"calls_per_ns": calls_per_ns, "site_updates_per_ns_if_only_draws": 4 * calls_per_ns,
              "note": "one Philox4x32-10 call per four site updates; the draws alone cap the Metropolis sweep here"}
    copy_gbs = max(v["GB_per_s"] for v in vec if v["op"] == "=" and v["lattice"] == 8192)
    return {"vector_ops": vec, "transfers": tr, "achievable_hbm_copy_GB_per_s": copy_gbs, "philox": philox,
            "roofline": {"bound": "hbm", "achieved": copy_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": copy_gbs / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k_vec<copy>, 1 GiB float vector (8 bytes moved per float)"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--cw", type=int, default=0, help="force a fused plan with this chunk width")
    ap.add_argument("--rows", type=int, default=0, help="force a fused plan with this tile / band height")
    ap.add_argument("--plan", type=int, default=5, help="fused plan forced by --cw/--rows (2: wave tiles, 5: full rows)")
    ap.add_argument("--no-extra", action="store_true", help="headline only")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=8,
                    help="oracle sweeps of the headline lattice for cpu_baseline (about 10 s on 16 cores)")
    ap.add_argument("--batched-sweeps", type=int, default=10000)
    ap.add_argument("--batched-sample", type=int, default=1,
                    help="0: no one-launch-per-lattice comparator (else one lattice per side)")
    ap.add_argument("--no-batch-tune", action="store_true",
                    help="use the built-in batch rates instead of timing them first")
    ap.add_argument("--no-fifo", action="store_true", help="skip the one-request-at-a-time served comparator")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-rates", type=str, default="100,200,500,1000,2000,5000")
    ap.add_argument("--served-subsat-rate", type=float, default=10.0,
                    help="one extra, sub-saturation arrival rate (0: skip)")
    ap.add_argument("--served-requests", type=int, default=256)
    ap.add_argument("--epoch-sweeps", type=int, default=128,
                    help="sweeps per request per server epoch (128 beat 64 by 1-3% in throughput and latency)")
    ap.add_argument("--creutz-sweeps", type=int, default=100)
    ap.add_argument("--only", default=None,
                    choices=["creutz", "percolation", "percolation-media", "micro", "batched", "batched-stepped",
                             "batched-resident", "served", "fifo", "small-configs", "c1"],
                    help="run one extra leg alone (for profiling it); prints that leg's JSON only")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB copy (for scaling rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_cs_0312006_amd import binding as b
    from paper_cs_0312006_amd import workloads as W
    b.lib()
    torch.cuda.init()
    stream = torch.cuda.Stream()

    if args.only:
        if args.only == "creutz":
            leg = run_creutz(b, torch, stream, args.creutz_sweeps, float("nan"), cpu=False)
        elif args.only == "percolation":
            leg = run_percolation(b, cpu=False)
        elif args.only == "percolation-media":
            leg = run_percolation(b, cpu=False, spanning=False)
        elif args.only == "served":
            leg = run_served(args.served_rates, args.served_requests, args.epoch_sweeps)
        elif args.only == "fifo":
            leg = run_fifo(b, float(args.served_rates.split(",")[0]), args.served_requests)
        elif args.only == "small-configs":
            leg = run_small_configs(b, torch, stream)
        elif args.only == "c1":
            leg = run_c1(b, torch, stream)
        elif args.only.startswith("batched"):
            leg, _ = run_batched(b, torch, stream, 1024, args.batched_sweeps, 0,
                                 plan={"batched": 0, "batched-resident": 1, "batched-stepped": 2}[args.only])
        else:
            leg = run_micro(b, torch, stream)
        print(json.dumps({"leg": args.only, "result": leg}), flush=True)
        return

    run = W.C2_HEADLINE
    force = (args.cw, args.rows) if (args.cw or args.rows) else None
    head = run_headline(b, torch, stream, run, args.steps, args.warmup, tune=not args.no_tune, force=force,
                        first=max(2, args.cpu_sweeps), force_plan=args.plan)
    ms, steps = head["ms"], args.steps
    progress(f"headline: {run.L * run.L * steps / ms / 1e6:.1f} attempts/ns")
    attempts = run.L * run.L * steps
    value = attempts / ms / 1e6  # attempts per ns
    launch_ms = ms / steps      # one fused launch per sweep (plus one tiny reduce per call)
    plan_names = {1: "two-pass", 2: "fused", 3: "resident", 4: "generic", 5: "fused-rows", 6: "bands"}
    plan = head["plan"]
    alg_bytes = 2.0 * run.L * run.L if plan[0] in (2, 5) else 3.0 * run.L * run.L
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9

    kname = {2: f"k_fused<{plan[1]},{plan[2]}>", 5: f"k_fused_rows<{plan[1]},{plan[2]}>"}.get(plan[0], "k_two_pass")
    prof = headline_profile(kname)
    same_kernel = prof is not None
    traffic = prof["hbm_bytes_per_launch"] / (launch_ms * 1e-3) / 1e9 if same_kernel else None
    roof_hbm = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "traffic_frac": traffic / HBM_PEAK_GBS if traffic else None, "kernel": kname,
                "algorithmic_bytes_per_launch": alg_bytes, "avg_launch_ms": launch_ms,
                "avg_launch_ms_from": "HIP events on the context's stream around the timed sweeps"}
    roof_alu = None
    if same_kernel:
        ops = prof["valu_lane_ops_per_attempt"] * run.L * run.L / (launch_ms * 1e-3)
        roof_alu = {"bound": "alu", "achieved": ops / 1e12, "peak": VALU_PEAK_LANE_OPS / 1e12,
                    "unit": "T lane-ops/s (32-bit VALU)", "frac": ops / VALU_PEAK_LANE_OPS, "traffic": traffic,
                    "traffic_unit": "GB/s", "kernel": kname,
                    "ops_per_attempt": prof["valu_lane_ops_per_attempt"],
                    "valu_busy_rocprof": prof["valu_busy_rocprof"], "avg_launch_ms": launch_ms}
    out = {
        "metric": "spin-update attempts/ns",
        "value": value,
        "unit": "attempts/ns",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "ising2d 32768x32768 periodic, J=1 h=0 T=2.269185, hot start seed 11",
                   "L": run.L, "T": run.T, "h": run.h, "p_up": run.p_up, "seed": run.seed,
                   "step": "one full sweep (both colours) with per-sweep B and M",
                   "plan": {"kind": plan_names.get(plan[0], str(plan[0])), "chunk_words": plan[1],
                            "tile_rows": plan[2]}},
        "roofline": roof_hbm,
        "roofline_alu": roof_alu,
        "host_wall_s": head["host_s"],
        # the paper's own figures, as context only (another machine, another
        # metric): its fragment-program Ising sweep on an NV30 (Section 5)
        "paper_context": {"nv30_gflops": 7.0, "nv30_fraction_of_peak": 0.44,
                          "site_visits_per_ns_table4": [0.004, 0.01],
                          "note": "context only, not a baseline for this metric"},
    }

    if not args.no_cpu:
        cpu, parity = cpu_baseline(run, args.cpu_sweeps, head["B0"], head["M0"])
        out["cpu_baseline"] = cpu
        out["parity_first_sweeps_vs_oracle"] = parity
        progress("cpu baseline")

    if not args.no_extra:
        extra = []
        for r in W.C2:
            if r == run:
                continue
            h = run_headline(b, torch, stream, r, steps, args.warmup, tune=False)
            extra.append({"h": r.h, "p_up": r.p_up, "sweeps": steps,
                          "value": r.L * r.L * steps / h["ms"] / 1e6, "unit": "attempts/ns"})
        out["c2_other_runs"] = extra
        progress("other 32768^2 runs")
        # the plan ISING_BATCH_AUTO picks: resident, every lattice of this
        # configuration (h = 0, L <= 1024) held bit-packed in workgroup memory
        if not args.no_batch_tune:
            b.ising_batch_tune(0, None, b.ISING_TUNE_RETIME)
        auto, h_au = run_batched(b, torch, stream, 1024, args.batched_sweeps, args.batched_sample, plan=0)
        auto["batch_rates_tuned_in_this_run"] = not args.no_batch_tune
        auto["roofline"] = batched_roofline(auto, stepped=auto["plan"].startswith("stepped"))
        other = 1 if auto["plan"].startswith("stepped") else 2
        alt, h_alt = run_batched(b, torch, stream, 1024, args.batched_sweeps, 0, plan=other)
        auto["other_plan_same_config"] = {"plan": alt["plan"], "value": alt["value"], "ms": alt["ms"],
                                          "results_identical": h_alt == {k: h_au[k] for k in h_alt},
                                          "roofline": batched_roofline(alt, stepped=other == 2)}
        auto["hbm_roof_fraction_at_2B_per_attempt"] = auto["value"] / (HBM_PEAK_GBS / 2.0)
        out["batched"] = auto
        progress("batched")

    if not args.no_extra and not args.no_served:
        out["served"] = run_served(args.served_rates, args.served_requests, args.epoch_sweeps)
        progress("served")
        if args.served_subsat_rate > 0:
            sub = run_served(str(args.served_subsat_rate), args.served_requests, args.epoch_sweeps)
            for x in sub:
                x["label"] = "sub-saturation point (extra, not a configured rate)"
            out["served_subsaturation"] = sub
        if not args.no_fifo:
            rates = [float(x) for x in args.served_rates.split(",") if x][:1]
            if args.served_subsat_rate > 0:
                rates.append(args.served_subsat_rate)
            out["served_fifo_comparator"] = [run_fifo(b, r, args.served_requests) for r in rates]
            progress("served FIFO comparator")

    if not args.no_extra:
        out["small_configs"] = run_small_configs(b, torch, stream)
        progress("small configs")

    if not args.no_extra:
        out["creutz"] = run_creutz(b, torch, stream, args.creutz_sweeps, value, cpu=not args.no_cpu)
        progress("creutz")
        out["percolation"] = run_percolation(b, cpu=not args.no_cpu)
        progress("percolation")
        out["micro"] = run_micro(b, torch, stream)
        progress("micro")
        # the headline against what this part measurably streams, and against
        # the rate its Philox draws alone would allow
        copy_gbs = out["micro"]["achievable_hbm_copy_GB_per_s"]
        out["roofline"]["frac_of_measured_copy"] = achieved / copy_gbs
        draws_only = out["micro"]["philox"]["site_updates_per_ns_if_only_draws"]
        out["frac_of_philox_only_rate"] = value / draws_only

    if args.calibrate_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 1 << 30

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
