"""Request server for Ising solves: continuous batching on one GPU.

A request asks for `sweeps` checkerboard Metropolis sweeps of an L x L
lattice (J, h, T, seed, p_up) and gets back the final lattice hash, the
final bond sum and magnetisation and FP64 averages of the per-sweep series.

The loop works in epochs. Every request admitted so far advances by up to
`epoch_sweeps` sweeps in one batched call (`ising_sweep_batch_plan` with
the AUTO plan: with lattices above 256 on a side in flight, the stepped
plan, which spreads every lattice over the whole GPU, one pass per sweep
over the tiles of all lattices, each alternating between two buffers;
with only small lattices, one workgroup per lattice). Between
epochs, requests that have arrived are admitted first come, first served,
as long as the HBM budget (the sum of the admitted lattices' device bytes)
and the slot limit allow; requests whose sweeps are done are retired.
Lattice and draw state stay on the device for a request's whole life.
Because the draws are keyed by (seed, sweep, colour, site), a request's
result does not depend on which epochs or which other requests it shared
the GPU with.

The HBM budget covers every context the executor holds on the device: the
admitted requests' and the idle ones it keeps for reuse. An admission that
would not fit first reuses an idle context of its side (no new bytes) and
otherwise frees idle contexts of other sides, oldest retired first, while
that makes room (freeing synchronises the device, so it happens only when
the budget requires it).

Up to `depth` epochs are enqueued before the oldest one is waited for:
which requests take part and how many sweeps each runs is known in
advance, and every request has its own stream. A request's results are
read back by copies enqueued right behind its last epoch (the executor's
prefetch), so retiring it waits for that epoch only, not for the epochs
enqueued after it.
"""
import collections
import math
import time
from dataclasses import dataclass, field


@dataclass
class Result:
    rid: int
    L: int
    sweeps: int
    arrival: float        # scheduled arrival, seconds after the stream start
    admitted: float       # when it was admitted
    done: float           # when its result was on the host
    lattice_hash: int = 0
    bond_sum: int = 0
    mag_sum: int = 0
    e_mean: float = 0.0   # <E/N> over the second half of the sweeps
    abs_m_mean: float = 0.0
    error: str = ""

    @property
    def latency(self):
        return self.done - self.arrival


class GpuExecutor:
    """Executor over the C ABI (one stream per request).

    Retired contexts are kept, while their device bytes total at most
    `pool_bytes`, and re-initialised for later requests of the same side
    (ising_reset) instead of being freed and allocated again: freeing device
    memory synchronises the device, which would drain the epochs queued
    behind it. The server counts the kept bytes against its HBM budget
    (pooled_bytes, reusable) and has them freed when an admission needs the
    room (evict). Every context's series is reserved at admission for at
    least `series_floor` sweeps (and the whole request), so neither an epoch
    nor a reuse grows it. close() releases the kept contexts."""

    def __init__(self, hash_results=True, pool_bytes=8 << 30, series_floor=32768):
        from . import binding as b
        self.b = b
        b.lib()
        self.hash_results = hash_results
        self.pool_bytes = pool_bytes      # device bytes of idle contexts kept for reuse, at most
        self.pooled = 0                   # device bytes of the idle contexts now kept
        self.series_floor = series_floor  # every context's series holds at least this many sweeps
        self.pool = collections.defaultdict(list)  # side -> idle contexts
        self.order = collections.deque()           # idle contexts, oldest retired first
        self.side = {}                             # context -> side

    def _bytes(self, L):
        # the stepped plan alternates a lattice between two buffers (the
        # second is allocated on the first stepped epoch)
        return self.b.ising_state_bytes(L, self.b.ISING_PLAN_FUSED) or 2 * L * L

    def bytes_for(self, run):
        return self._bytes(run.L)

    def pooled_bytes(self):
        return self.pooled

    def reusable(self, run):
        """Whether create(run) takes an idle context (no new device bytes)."""
        return bool(self.pool.get(run.L))

    def evict(self, nbytes, keep_side=None):
        """Free idle contexts (not of side keep_side), oldest retired first,
        until `nbytes` are freed or none is left; returns the bytes freed."""
        freed = 0
        for handle in list(self.order):
            if freed >= nbytes:
                break
            L = self.side[handle]
            if L == keep_side:
                continue
            self.order.remove(handle)
            self.pool[L].remove(handle)
            del self.side[handle]
            self.b.ising_destroy(handle)
            self.pooled -= self._bytes(L)
            freed += self._bytes(L)
        return freed

    def create(self, run):
        b = self.b
        idle = self.pool.get(run.L)
        if idle:
            handle = idle.pop()
            self.order.remove(handle)
            self.pooled -= self._bytes(run.L)
            b.ising_reset(handle, run.L, run.J, run.h, run.T, run.seed, run.p_up, b.ISING_PLAN_TWO_PASS)
        else:
            handle = b.ising_create(run.L, run.J, run.h, run.T, run.seed, run.p_up, b.ISING_PLAN_TWO_PASS)
            self.side[handle] = run.L
        b.ising_reserve(handle, max(run.sweeps, self.series_floor))
        return handle

    def step(self, handles, sweeps):
        self.b.ising_sweep_batch_plan(handles, sweeps, self.b.ISING_BATCH_AUTO)

    def prefetch(self, handle):
        """Start reading back a request's results as soon as its last epoch
        is enqueued, so that result() waits for that epoch only and not for
        the epochs enqueued after it."""
        b = self.b
        b.ising_prefetch_observables(handle, b.ISING_OBS_SERIES | (b.ISING_OBS_HASH if self.hash_results else 0))

    def result(self, handle, run):
        b = self.b
        want = b.ISING_OBS_SERIES | (b.ISING_OBS_HASH if self.hash_results else 0)
        obs, B, M = b.ising_observables(handle, want)
        half = len(B) // 2
        avg = b.ising_series_averages(B[half:], M[half:], run.L, run.J, run.h)
        return {"lattice_hash": obs.lattice_hash, "bond_sum": obs.bond_sum, "mag_sum": obs.mag_sum,
                "e_mean": avg.e, "abs_m_mean": avg.abs_m}

    def destroy(self, handle):
        L = self.side[handle]
        need = self._bytes(L)
        if self.pooled + need <= self.pool_bytes:
            self.pool[L].append(handle)
            self.order.append(handle)
            self.pooled += need
        else:
            del self.side[handle]
            self.b.ising_destroy(handle)

    def close(self):
        for handles in self.pool.values():
            for handle in handles:
                self.b.ising_destroy(handle)
                del self.side[handle]
        self.pool.clear()
        self.order.clear()
        self.pooled = 0


def serve(requests, executor, hbm_budget=16 << 30, max_slots=4096, epoch_sweeps=128,
          clock=time.perf_counter, sleep=time.sleep, depth=2):
    """Run a stream of workloads.Request through the executor. Returns
    (results sorted by request id, stats). Up to `depth` epochs are enqueued
    ahead of the one being retired, so that the host's admission and
    retirement work overlaps the GPU's sweeps."""
    order = sorted(range(len(requests)), key=lambda k: requests[k].arrival)
    future = collections.deque(order)          # not yet arrived
    waiting = collections.deque()              # arrived, not admitted
    active = {}                                # rid -> [handle, remaining, bytes, admitted]
    used = 0
    results = {}
    epochs = 0
    t0 = clock()
    in_flight = collections.deque()            # (ids, sweeps) of enqueued epochs not yet retired, oldest first
    prefetch = getattr(executor, "prefetch", None)
    # executors that keep idle contexts report their bytes: they count too
    pooled = getattr(executor, "pooled_bytes", lambda: 0)
    reusable = getattr(executor, "reusable", lambda run: False)
    evict = getattr(executor, "evict", None)

    def now():
        return clock() - t0

    def admit():
        nonlocal used
        t = now()
        while future and requests[future[0]].arrival <= t:
            waiting.append(future.popleft())
        while waiting and len(active) < max_slots:
            rid = waiting[0]
            run = requests[rid].run
            need = executor.bytes_for(run)
            if need > hbm_budget:   # can never fit: refuse rather than block the queue
                waiting.popleft()
                results[rid] = Result(rid, run.L, run.sweeps, requests[rid].arrival, t, t,
                                      error="larger than the HBM budget")
                continue
            extra = 0 if reusable(run) else need  # device bytes the admission adds
            over = used + pooled() + extra - hbm_budget
            if over > 0 and extra and evict is not None:
                evict(over, run.L)
                over = used + pooled() + extra - hbm_budget
            if over > 0:
                break
            waiting.popleft()
            active[rid] = [executor.create(run), run.sweeps, need, t]
            used += need

    def retire(ids, sweeps):
        nonlocal used
        for rid, n in zip(ids, sweeps):
            slot = active[rid]
            slot[1] -= n
        finished = [rid for rid in ids if active[rid][1] == 0]
        for rid in finished:
            handle, _, need, adm = active.pop(rid)
            run = requests[rid].run
            res = executor.result(handle, run)   # waits for this request's last epoch only
            executor.destroy(handle)
            used -= need
            results[rid] = Result(rid, run.L, run.sweeps, requests[rid].arrival, adm, now(), **res)

    while future or waiting or active or in_flight:
        admit()
        # the next epoch: every active request with sweeps left after the
        # epochs in flight advances by up to epoch_sweeps
        pending = collections.Counter()
        for e_ids, e_sweeps in in_flight:
            for rid, n in zip(e_ids, e_sweeps):
                pending[rid] += n
        ids, sweeps = [], []
        for rid, slot in active.items():
            left = slot[1] - pending[rid]
            if left > 0:
                ids.append(rid)
                sweeps.append(min(epoch_sweeps, left))
        if ids:
            executor.step([active[r][0] for r in ids], sweeps)
            epochs += 1
            in_flight.append((ids, sweeps))
            if prefetch:
                # requests whose last sweeps are in this epoch
                for rid, n in zip(ids, sweeps):
                    if active[rid][1] - pending[rid] == n:
                        prefetch(active[rid][0])
        # retire the oldest epoch once `depth` are queued behind it, or when
        # nothing new could be enqueued
        if in_flight and (len(in_flight) > depth or not ids):
            retire(*in_flight.popleft())
        if not in_flight and not active and future and not waiting:
            sleep(max(0.0, requests[future[0]].arrival - now()))
    makespan = now()
    res = [results[k] for k in sorted(results)]
    return res, {"epochs": epochs, "makespan_s": makespan}


def summarize(results, makespan_s):
    ok = [r for r in results if not r.error]
    lat = sorted(r.latency for r in ok)

    def pct(p):
        if not lat:
            return float("nan")
        k = min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))
        return lat[k]

    attempts = sum(r.L * r.L * r.sweeps for r in ok)
    return {"requests": len(results), "completed": len(ok), "p50_s": pct(50), "p99_s": pct(99),
            "mean_s": sum(lat) / len(lat) if lat else float("nan"),
            "attempts": attempts, "makespan_s": makespan_s,
            "attempts_per_ns": attempts / makespan_s / 1e9 if makespan_s > 0 else float("nan")}
