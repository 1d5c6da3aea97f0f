"""CPU tests of the request server's scheduling (admission by HBM budget and
slots, epochs, retirement, latencies) with a fake executor and a virtual
clock. The fake executor only counts sweeps; no Ising arithmetic here."""
import pytest

from paper_cs_0312006_amd import serve
from paper_cs_0312006_amd import workloads as W


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(0.0, dt)


class FakeExecutor:
    """Each epoch costs `per_site` seconds per site-sweep on the virtual clock."""

    def __init__(self, clock, per_site=1e-12, bytes_per_site=1):
        self.clock = clock
        self.per_site = per_site
        self.bpp = bytes_per_site
        self.live = {}
        self.next = 1
        self.log = []          # (handles, sweeps) per step
        self.done = {}         # handle -> sweeps run
        self.max_live_bytes = 0

    def bytes_for(self, run):
        return run.L * run.L * self.bpp

    def create(self, run):
        h = self.next
        self.next += 1
        self.live[h] = run
        self.done[h] = 0
        self.max_live_bytes = max(self.max_live_bytes, sum(self.bytes_for(r) for r in self.live.values()))
        return h

    def step(self, handles, sweeps):
        self.log.append((list(handles), list(sweeps)))
        cost = 0.0
        for h, n in zip(handles, sweeps):
            assert h in self.live and n > 0
            self.done[h] += n
            cost += self.live[h].L ** 2 * n * self.per_site
        self.clock.t += cost

    def result(self, handle, run):
        assert self.done[handle] == run.sweeps, "retired before all its sweeps ran"
        return {"lattice_hash": handle, "bond_sum": 0, "mag_sum": 0, "e_mean": 0.0, "abs_m_mean": 0.0}

    def destroy(self, handle):
        del self.live[handle]


def _stream(n=40, rate=200.0, seed=3):
    return W.request_stream(rate, count=n, rng_seed=seed, sweeps_range=(50, 400), side_units=(1, 8))


def test_every_request_completes_with_all_its_sweeps():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = _stream()
    res, stats = serve.serve(reqs, ex, epoch_sweeps=32, clock=clk, sleep=clk.sleep)
    assert len(res) == len(reqs) and all(not r.error for r in res)
    for r in res:
        assert r.sweeps == reqs[r.rid].run.sweeps
        assert r.done >= r.admitted >= r.arrival - 1e-12
    assert not ex.live
    # epochs never give a request more than epoch_sweeps
    assert all(max(s) <= 32 for _, s in ex.log)
    s = serve.summarize(res, stats["makespan_s"])
    assert s["completed"] == len(reqs) and s["p99_s"] >= s["p50_s"] > 0


def test_hbm_budget_is_never_exceeded_and_forces_queueing():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = _stream(n=30, rate=1e6)  # all arrive at once
    budget = 3 * 512 * 512
    res, _ = serve.serve(reqs, ex, hbm_budget=budget, epoch_sweeps=16, clock=clk, sleep=clk.sleep)
    assert ex.max_live_bytes <= budget
    assert all(not r.error for r in res)
    # queueing happened: some request was admitted well after it arrived
    assert max(r.admitted - r.arrival for r in res) > 0


def test_slot_limit():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = _stream(n=25, rate=1e6)
    res, _ = serve.serve(reqs, ex, max_slots=3, epoch_sweeps=64, clock=clk, sleep=clk.sleep)
    assert all(len(h) <= 3 for h, _ in ex.log)
    assert len(res) == 25


def test_first_come_first_served_admission():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = _stream(n=20, rate=1e6)
    res, _ = serve.serve(reqs, ex, max_slots=1, epoch_sweeps=1000, clock=clk, sleep=clk.sleep)
    by_arrival = sorted(res, key=lambda r: (reqs[r.rid].arrival, r.rid))
    adm = [r.admitted for r in by_arrival]
    assert adm == sorted(adm)


def test_request_larger_than_budget_is_refused_not_blocking():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    reqs = _stream(n=10, rate=1e6)
    big = max(range(10), key=lambda k: reqs[k].run.L)
    budget = reqs[big].run.L ** 2 - 1
    res, _ = serve.serve(reqs, ex, hbm_budget=budget, clock=clk, sleep=clk.sleep)
    bad = [r for r in res if r.error]
    assert any(r.rid == big for r in bad)
    assert all(not r.error for r in res if reqs[r.rid].run.L ** 2 <= budget)


def test_continuous_batching_admits_between_epochs():
    """Requests arriving while others run join at the next epoch, so some
    epoch contains requests admitted at different times."""
    clk = FakeClock()
    ex = FakeExecutor(clk, per_site=1e-9)
    reqs = _stream(n=30, rate=50.0)
    serve.serve(reqs, ex, epoch_sweeps=8, clock=clk, sleep=clk.sleep)
    sizes = [len(h) for h, _ in ex.log]
    assert max(sizes) > 1
    members = [set(h) for h, _ in ex.log]
    assert any(a != b and a & b for a, b in zip(members, members[1:]))


def test_idle_server_sleeps_until_next_arrival():
    clk = FakeClock()
    ex = FakeExecutor(clk, per_site=0.0)
    reqs = W.request_stream(1.0, count=3, rng_seed=2, sweeps_range=(10, 20), side_units=(1, 1))
    res, stats = serve.serve(reqs, ex, clock=clk, sleep=clk.sleep)
    assert stats["makespan_s"] >= max(r.arrival for r in reqs)
    for r in res:
        assert r.latency == pytest.approx(0.0, abs=1e-9)


class PrefetchingExecutor(FakeExecutor):
    """Records when each request's read-back is started."""

    def __init__(self, clock):
        super().__init__(clock)
        self.prefetched = {}   # handle -> sweeps enqueued when prefetched

    def prefetch(self, handle):
        assert handle in self.live and handle not in self.prefetched, "prefetched twice"
        self.prefetched[handle] = self.done[handle]

    def result(self, handle, run):
        assert self.prefetched.get(handle) == run.sweeps, "read-back not started right after its last epoch"
        return super().result(handle, run)


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_read_back_starts_right_after_the_last_epoch(depth):
    """With an executor that can prefetch, every request's read-back is
    started once, right after the epoch holding its last sweeps is enqueued
    (all its sweeps enqueued, none after), whatever the queue depth."""
    clk = FakeClock()
    ex = PrefetchingExecutor(clk)
    reqs = _stream(n=60)
    res, _ = serve.serve(reqs, ex, epoch_sweeps=32, clock=clk, sleep=clk.sleep, depth=depth)
    assert len(res) == len(reqs) and all(not r.error for r in res)
    assert len(ex.prefetched) == len(reqs)


class PoolingExecutor(FakeExecutor):
    """Keeps retired contexts for reuse by side, like the GPU executor."""

    def __init__(self, clock, **kw):
        super().__init__(clock, **kw)
        self.pool = {}       # side -> handles
        self.order = []
        self.evicted = 0
        self.max_total = 0

    def pooled_bytes(self):
        return sum(self.bytes_for(W.Run(L=L)) * len(hs) for L, hs in self.pool.items())

    def reusable(self, run):
        return bool(self.pool.get(run.L))

    def evict(self, nbytes, keep_side=None):
        freed = 0
        for h, L in list(self.order):
            if freed >= nbytes:
                break
            if L == keep_side:
                continue
            self.order.remove((h, L))
            self.pool[L].remove(h)
            freed += self.bytes_for(W.Run(L=L))
            self.evicted += 1
        return freed

    def create(self, run):
        if self.pool.get(run.L):
            h = self.pool[run.L].pop()
            self.order.remove((h, run.L))
            self.live[h] = run
            self.done[h] = 0
        else:
            h = super().create(run)
        self._track()
        return h

    def destroy(self, handle):
        run = self.live.pop(handle)
        self.pool.setdefault(run.L, []).append(handle)
        self.order.append((handle, run.L))
        self._track()

    def _track(self):
        live = sum(self.bytes_for(r) for r in self.live.values())
        self.max_total = max(self.max_total, live + self.pooled_bytes())


def test_pooled_contexts_count_against_the_budget():
    """Idle contexts kept for reuse count against the HBM budget: the device
    bytes held (admitted plus pooled) never pass it, and pooled contexts are
    freed when an admission needs the room."""
    clk = FakeClock()
    ex = PoolingExecutor(clk)
    reqs = _stream(n=60)
    budget = 3 * 512 * 512
    res, _ = serve.serve(reqs, ex, hbm_budget=budget, epoch_sweeps=32, clock=clk, sleep=clk.sleep)
    assert all(not r.error for r in res if r.L * r.L <= budget)
    assert ex.max_total <= budget
    assert ex.evicted > 0

