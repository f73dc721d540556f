"""CPU tests of the continuous-batching scheduler with a fake executor.

The fake executor models the device with a simulated clock: binning takes a
fixed time, a labelling launch a fixed overhead plus a time per voxel, and
the labels come from the CPU oracle, so that the scheduler's admission,
memory accounting, batching and retirement are checked without a GPU.
"""
import numpy as np
import pytest

import oracle
from paper_2201_13234_amd import inputs as I
from paper_2201_13234_amd import serve as S


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


def oracle_digest(w):
    p = oracle.problem(w.n, w.L, w.kind, w.periodic, w.growth)
    lab, _, _ = oracle.tessellate(p, w.coords, w.param, nthreads=1)
    return S.digest_host(lab)


class FakeExecutor(S.Executor):
    def __init__(self, clock, bin_time=2e-4, launch_overhead=1e-3, per_vox=2e-9, fail_ids=()):
        self.clock, self.bin_time, self.launch_overhead, self.per_vox = clock, bin_time, launch_overhead, per_vox
        self.fail_ids = set(fail_ids)
        self.launches = 0

    def prepare(self, req):
        if req.rid in self.fail_ids:
            raise MemoryError("simulated allocation failure")

    def start_binning(self, req):
        req.state["bin_ready"] = self.clock() + self.bin_time

    def binning_done(self, req):
        return self.clock() >= req.state["bin_ready"]

    def start_labelling(self, reqs):
        self.launches += 1
        for r in reqs:
            r.state["digest"] = oracle_digest(r.workload)
        return self.clock() + self.launch_overhead + self.per_vox * sum(r.nvox for r in reqs)

    def labelling_done(self, token):
        return self.clock() >= token

    def finish(self, req):
        req.status, req.digest = 0, req.state["digest"]

    def run_alone(self, req):
        self.clock.sleep(self.bin_time + self.launch_overhead + self.per_vox * req.nvox)
        req.status, req.digest = 0, oracle_digest(req.workload)


def small_stream(n, rate, seed=0):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    reqs = []
    for i in range(n):
        d = 2 + int(rng.integers(0, 2))
        side = tuple(int(v) for v in rng.integers(6, 40 if d == 2 else 14, d))
        w = I.make(side, int(rng.integers(0, 3)), bool(rng.integers(0, 2)), int(rng.integers(1, 30)),
                   seed=1000 + i)
        reqs.append(S.Request(rid=i, workload=w, arrival=float(t[i])))
    return reqs


def copy(reqs):
    return [S.Request(r.rid, r.workload, r.arrival) for r in reqs]


def test_every_request_completes_with_the_right_labels():
    clk = SimClock()
    ex = FakeExecutor(clk)
    reqs = small_stream(40, rate=2000.0)
    srv = S.Server(ex, mem_budget=1 << 30, clock=clk, sleep=clk.sleep)
    out = srv.run(copy(reqs))
    assert [r.rid for r in out] == list(range(40))
    for r in out:
        assert r.status == 0
        assert r.digest == oracle_digest(r.workload)
        assert r.done >= r.admitted >= r.arrival
    # requests that arrived while a launch was running were batched together
    assert max(srv.batches) > 1 and sum(srv.batches) == 40


def test_memory_budget_is_respected_and_requests_wait_for_it():
    clk = SimClock()
    ex = FakeExecutor(clk)
    reqs = small_stream(30, rate=1e5)
    budget = 3 * max(S.device_bytes(r.workload) for r in reqs)
    srv = S.Server(ex, mem_budget=budget, clock=clk, sleep=clk.sleep)
    out = srv.run(copy(reqs))
    assert all(r.status == 0 for r in out)
    assert srv.peak_mem <= budget
    assert srv.mem_in_use == 0


def test_slot_limit_and_batch_limit():
    clk = SimClock()
    ex = FakeExecutor(clk)
    srv = S.Server(ex, max_slots=4, max_batch=3, clock=clk, sleep=clk.sleep)
    out = srv.run(copy(small_stream(25, rate=1e6)))
    assert all(r.status == 0 for r in out)
    assert max(srv.batches) <= 3


def test_oversized_and_failing_requests_do_not_block_others():
    clk = SimClock()
    ex = FakeExecutor(clk, fail_ids={5})
    reqs = small_stream(12, rate=500.0)
    big = I.make((64, 64, 64), 0, True, 10, seed=3)
    reqs[3] = S.Request(3, big, reqs[3].arrival)
    srv = S.Server(ex, mem_budget=S.device_bytes(big) - 1, clock=clk, sleep=clk.sleep)
    out = srv.run(copy(reqs))
    assert out[3].status == -2
    assert out[5].status == -3
    assert all(r.status == 0 for r in out if r.rid not in (3, 5))


def test_batching_beats_one_by_one_when_launches_cost_overhead():
    clk1, clk2 = SimClock(), SimClock()
    reqs = small_stream(60, rate=1500.0)
    b = S.Server(FakeExecutor(clk1), clock=clk1, sleep=clk1.sleep).run(copy(reqs))
    a = S.Server(FakeExecutor(clk2), clock=clk2, sleep=clk2.sleep).run_one_by_one(copy(reqs))
    sb, sa = S.summarize(b), S.summarize(a)
    assert [r.digest for r in a] == [r.digest for r in b]
    assert sb["p99_ms"] < sa["p99_ms"]


def test_digest_host_matches_definition():
    lab = np.array([[0, 1], [2, -1]], dtype=np.int32)
    P = 2147483647
    want = sum((int(v) + 3) * ((i * 48271 + 97) % P) for i, v in enumerate(lab.reshape(-1))) % P
    assert S.digest_host(lab) == want


def test_batches_capped_by_voxels():
    """A burst is cut into launches of at most batch_voxels (in arrival
    order); a request larger than the cap goes alone."""
    clock = SimClock()
    reqs = small_stream(30, rate=1e9, seed=7)       # everything arrives at once
    big = S.Request(rid=99, workload=I.make((60, 60, 60), 0, True, 20, seed=5), arrival=0.0)
    cap = 4000
    srv = S.Server(FakeExecutor(clock), max_batch=64, batch_voxels=cap, clock=clock, sleep=clock.sleep)
    launched = []
    orig = srv.ex.start_labelling

    def spy(batch):
        launched.append([r.rid for r in batch])
        return orig(batch)
    srv.ex.start_labelling = spy
    done = srv.run(copy(reqs) + [big])
    assert all(r.status == 0 for r in done)
    sizes = {r.rid: r.nvox for r in reqs + [big]}
    for b in launched:
        assert len(b) == 1 or sum(sizes[i] for i in b) <= cap
    assert [99] in launched
    order = [i for b in launched for i in b]
    assert sorted(order) == sorted(sizes)
