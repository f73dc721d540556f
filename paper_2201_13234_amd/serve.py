"""Continuous-batching request loop for tessellation jobs.

Requests (one diagram each) arrive over time.  The scheduler
  - admits a request as soon as a slot is free and its device memory
    (labels, sites, bins) fits in the memory budget, in arrival order;
  - bins every admitted request's sites on a binning stream right away (the
    bins stay resident on the device);
  - whenever the labelling stream is idle, labels every admitted request whose
    bins are ready in one persistent launch (vt_label_batch), so requests that
    arrived while others were on the GPU join the next batch, and their binning
    overlaps the running batch;
  - retires finished requests, releasing their memory and slot.
Latency is completion time minus arrival time.  The one-by-one baseline runs
each request alone (vt_tessellate), in arrival order.

The device work sits behind a small executor interface so that the
scheduling logic can be tested on the CPU with a fake executor.
"""
import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    workload: object          # inputs.Workload (host arrays)
    arrival: float            # seconds since the start of the replay
    admitted: float = math.nan
    done: float = math.nan
    status: int = -1          # 0 ok, 5 bad input, or an error code
    digest: int = 0           # hash of the label image
    error: str = ""
    state: dict = field(default_factory=dict)

    @property
    def nvox(self):
        return self.workload.nvox

    @property
    def latency(self):
        return self.done - self.arrival


def device_bytes(w):
    """Device memory one request holds while in flight: labels (4 B/voxel),
    site coordinates and parameters (input), and the library's bins (about
    48 B per site plus 8 B per bin)."""
    ns = w.nsites
    return 4 * w.nvox + 8 * ns * (w.ndim + 1) + 48 * ns + 8 * (4 * ns + 64) + 4096


class Executor:
    """Device operations the scheduler needs (all asynchronous except
    run_alone)."""

    def prepare(self, req):           # allocate and upload; raises MemoryError
        raise NotImplementedError

    def start_binning(self, req):
        raise NotImplementedError

    def binning_done(self, req):
        raise NotImplementedError

    def start_labelling(self, reqs):  # returns a token
        raise NotImplementedError

    def labelling_done(self, token):
        raise NotImplementedError

    def finish(self, req):            # status + digest, release device memory
        raise NotImplementedError

    def run_alone(self, req):         # prepare + tessellate + finish, synchronous
        raise NotImplementedError


class GpuExecutor(Executor):
    """Executor over the device library, two HIP streams (binning, labelling)."""

    def __init__(self, ctx, device="cuda:0"):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.dev = torch.device(device)
        self.s_bin = torch.cuda.Stream(device=self.dev)
        self.s_lab = torch.cuda.Stream(device=self.dev)

    def _job(self, req):
        from . import vtess
        torch = self.torch
        w = req.workload
        st = req.state
        with torch.cuda.stream(self.s_bin):
            st["coords"] = torch.from_numpy(np.ascontiguousarray(w.coords)).pin_memory().to(
                self.dev, non_blocking=True)
            st["param"] = None if w.param is None else torch.from_numpy(
                np.ascontiguousarray(w.param)).pin_memory().to(self.dev, non_blocking=True)
            st["labels"] = torch.empty(w.shape, dtype=torch.int32, device=self.dev)
            st["status"] = torch.zeros(1, dtype=torch.int32, device=self.dev)
        return vtess.Job(n=w.n, L=w.L, kind=w.kind, periodic=w.periodic, growth=w.growth,
                         coords=st["coords"], param=st["param"], labels=st["labels"])

    def prepare(self, req):
        req.state["job"] = self._job(req)

    def start_binning(self, req):
        st = req.state
        st["bins"] = self.ctx.bins_build(st["job"], status=st["status"], stream=self.s_bin)
        ev = self.torch.cuda.Event()
        ev.record(self.s_bin)
        st["ev_bin"] = ev

    def binning_done(self, req):
        return req.state["ev_bin"].query()

    def start_labelling(self, reqs):
        torch = self.torch
        for r in reqs:
            self.s_lab.wait_event(r.state["ev_bin"])
        self.ctx.label_batch([r.state["bins"] for r in reqs], stream=self.s_lab)
        with torch.cuda.stream(self.s_lab):
            for r in reqs:
                r.state["hash"] = digest_device(r.state["labels"])
        ev = torch.cuda.Event()
        ev.record(self.s_lab)
        return ev

    def labelling_done(self, token):
        return token.query()

    def finish(self, req):
        st = req.state
        req.status = int(st["status"].item())
        req.digest = int(st["hash"].item())
        st["bins"].free(stream=self.s_lab)
        req.state = {}

    def run_alone(self, req):
        torch = self.torch
        job = self._job(req)
        st = req.state
        self.s_lab.wait_stream(self.s_bin)
        self.ctx.tessellate(job, status=st["status"], stream=self.s_lab)
        with torch.cuda.stream(self.s_lab):
            h = digest_device(st["labels"])
        self.s_lab.synchronize()
        req.status = int(st["status"].item())
        req.digest = int(h.item())
        req.state = {}

    def labels_of(self, req):
        return req.state.get("labels")


# Order-sensitive hash of a label image: sum over voxels i of
# (label_i + 3) * ((i * 48271 + 97) mod P), mod P, P = 2^31 - 1.  Every term
# stays below 2^62, so int64 arithmetic is exact on both sides.
_P = 2147483647


def digest_device(labels):
    """Hash of a device label image (torch ops on the current stream)."""
    import torch
    flat = labels.reshape(-1).to(torch.int64)
    w = (torch.arange(flat.numel(), device=labels.device, dtype=torch.int64) * 48271 + 97) % _P
    return ((flat + 3) * w % _P).sum() % _P


def digest_host(labels):
    """The same hash of a host label image (numpy)."""
    flat = np.asarray(labels).reshape(-1).astype(np.int64)
    w = (np.arange(flat.size, dtype=np.int64) * 48271 + 97) % _P
    return int(((flat + 3) * w % _P).sum() % _P)


class Server:
    """Continuous-batching scheduler.

    mem_budget: bytes of device memory the in-flight requests may hold;
    max_slots: requests in flight at once; max_batch: requests per labelling
    launch.  A request larger than the whole budget is rejected (status -2)
    without blocking the others.
    """

    def __init__(self, executor, mem_budget=8 << 30, max_slots=64, max_batch=64,
                 clock=time.perf_counter, sleep=time.sleep):
        self.ex = executor
        self.mem_budget = int(mem_budget)
        self.max_slots = int(max_slots)
        self.max_batch = int(max_batch)
        self.clock = clock
        self.sleep = sleep
        self.mem_in_use = 0
        self.peak_mem = 0
        self.batches = []     # sizes of the labelling launches

    def run(self, requests):
        """Replays the requests (sorted by arrival) and returns them completed."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        now = lambda: self.clock() - t0
        queue = list(reqs)            # not yet admitted, arrival order
        binning = []                  # admitted, bins being built
        ready = []                    # bins ready, waiting for a labelling launch
        running = None                # (token, [requests]) of the launch in flight
        active = 0
        done = []
        while queue or binning or ready or running:
            progressed = False
            t = now()
            # admission, in arrival order
            while queue and queue[0].arrival <= t and active < self.max_slots:
                r = queue[0]
                need = device_bytes(r.workload)
                if need > self.mem_budget:
                    queue.pop(0)
                    r.status, r.error = -2, "request larger than the memory budget"
                    r.admitted = r.done = t
                    done.append(r)
                    progressed = True
                    continue
                if self.mem_in_use + need > self.mem_budget:
                    break
                queue.pop(0)
                try:
                    self.ex.prepare(r)
                    self.ex.start_binning(r)
                except MemoryError as e:
                    r.status, r.error = -3, str(e)
                    r.admitted = r.done = now()
                    done.append(r)
                    progressed = True
                    continue
                r.admitted = t
                r.state["bytes"] = need
                self.mem_in_use += need
                self.peak_mem = max(self.peak_mem, self.mem_in_use)
                active += 1
                binning.append(r)
                progressed = True
            # bins that finished
            still = []
            for r in binning:
                if self.ex.binning_done(r):
                    ready.append(r)
                    progressed = True
                else:
                    still.append(r)
            binning = still
            # retire the running launch
            if running is not None and self.ex.labelling_done(running[0]):
                t_done = now()
                for r in running[1]:
                    r.done = t_done
                    nbytes = r.state.get("bytes", 0)
                    self.ex.finish(r)
                    self.mem_in_use -= nbytes
                    active -= 1
                    done.append(r)
                running = None
                progressed = True
            # launch everything that is ready while the labelling stream is idle
            if running is None and ready:
                batch, ready = ready[: self.max_batch], ready[self.max_batch:]
                running = (self.ex.start_labelling(batch), batch)
                self.batches.append(len(batch))
                progressed = True
            if not progressed:
                if queue and not (binning or ready or running) and queue[0].arrival > now():
                    self.sleep(min(queue[0].arrival - now(), 0.001))
                else:
                    self.sleep(0)
        return sorted(done, key=lambda r: r.rid)

    def run_one_by_one(self, requests):
        """Baseline: each request alone (vt_tessellate), in arrival order."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        for r in reqs:
            while self.clock() - t0 < r.arrival:
                self.sleep(min(r.arrival - (self.clock() - t0), 0.001))
            r.admitted = self.clock() - t0
            if device_bytes(r.workload) > self.mem_budget:
                r.status, r.error = -2, "request larger than the memory budget"
                r.done = r.admitted
                continue
            self.ex.run_alone(r)
            r.done = self.clock() - t0
        return sorted(reqs, key=lambda r: r.rid)


def summarize(reqs):
    ok = [r for r in reqs if r.status == 0]
    lat = np.array([r.latency for r in ok]) if ok else np.array([math.nan])
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    vox = sum(r.nvox for r in ok)
    return {"jobs": len(reqs), "ok": len(ok),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "mean_ms": round(float(np.mean(lat)) * 1e3, 3),
            "gvox_per_s": round(vox / span / 1e9, 3) if span > 0 else None}


def make_stream(n_jobs, rate, side_scale=0.25, first_job=0):
    """The request stream: seeded jobs (inputs.stream_job) with Poisson
    arrivals at `rate` per second."""
    from . import inputs
    t = inputs.arrivals(n_jobs, rate)
    return [Request(rid=i, workload=inputs.stream_job(first_job + i, side_scale), arrival=float(t[i]))
            for i in range(n_jobs)]


def benchmark(ctx, n_jobs=96, side_scale=0.25, load=0.8, mem_budget=8 << 30):
    """Replays a request stream twice on the GPU -- continuous batching and one
    by one -- with the same arrival times.  The arrival rate is `load` times
    the one-by-one service rate measured on a warm-up of the first jobs.
    Returns p50/p99 latency and throughput of both, and whether every job's
    labels are identical in both modes."""
    ex = GpuExecutor(ctx)
    warm = make_stream(min(16, n_jobs), 1.0, side_scale)
    for r in warm:                       # warm-up and service-rate calibration
        r.arrival = 0.0
    Server(ex).run_one_by_one(warm)
    t0 = time.perf_counter()
    Server(ex).run_one_by_one([Request(r.rid, r.workload, 0.0) for r in warm])
    service = (time.perf_counter() - t0) / len(warm)
    rate = load / service
    stream = make_stream(n_jobs, rate, side_scale)
    srv = Server(ex, mem_budget=mem_budget)
    batched = srv.run([Request(r.rid, r.workload, r.arrival) for r in stream])
    alone = Server(ex, mem_budget=mem_budget).run_one_by_one(
        [Request(r.rid, r.workload, r.arrival) for r in stream])
    same = all(a.digest == b.digest and a.status == b.status for a, b in zip(batched, alone))
    return {"jobs": n_jobs, "side_scale": side_scale, "rate_per_s": round(rate, 2),
            "service_ms_alone": round(service * 1e3, 3),
            "batched": summarize(batched), "one_by_one": summarize(alone),
            "mean_batch": round(float(np.mean(srv.batches)), 2) if srv.batches else 0,
            "labels_identical": bool(same)}
