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
    labels: object = None     # device label image kept after completion

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
    run_alone).  max_inflight: labelling launches that may run at once."""
    max_inflight = 1

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

    def finish(self, req):            # status, release device memory
        raise NotImplementedError

    def run_alone(self, req):         # prepare + tessellate + finish, synchronous
        raise NotImplementedError


class GpuExecutor(Executor):
    """Executor over the device library.

    Uploads run on their own stream.  Labelling launches alternate between
    `lanes` (context, stream) pairs so that one batch can be binned while the
    previous one is still labelling.  Two modes:
      resident_bins=False  each launch is one vt_tessellate_batch call:
                           segmented binning of the batch plus one persistent
                           labelling launch;
      resident_bins=True   every request is binned on arrival (vt_bins_build,
                           bins stay on the device) and a launch is one
                           vt_label_batch over the resident bins.
    With keep_labels the label images stay on the device after completion so
    that digest_all() can hash them outside the timed replay.
    """

    def __init__(self, ctx, device="cuda:0", lanes=2, resident_bins=False, keep_labels=True):
        import torch
        from . import vtess
        self.torch = torch
        self.dev = torch.device(device)
        self.ctxs = [ctx] + [vtess.Context(self.dev.index or 0) for _ in range(lanes - 1)]
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(lanes)]
        self.s_up = torch.cuda.Stream(device=self.dev)
        self.free_lanes = list(range(lanes))
        self.max_inflight = lanes
        self.resident_bins = resident_bins
        self.keep_labels = keep_labels

    def _job(self, req):
        from . import vtess
        torch = self.torch
        w = req.workload
        st = req.state
        with torch.cuda.stream(self.s_up):
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
        if self.resident_bins:
            st["bins"] = self.ctxs[0].bins_build(st["job"], status=st["status"], stream=self.s_up)
        ev = self.torch.cuda.Event()
        ev.record(self.s_up)
        st["ev_ready"] = ev

    def binning_done(self, req):
        return req.state["ev_ready"].query()

    def start_labelling(self, reqs):
        torch = self.torch
        lane = self.free_lanes.pop(0)
        s = self.streams[lane]
        for r in reqs:
            s.wait_event(r.state["ev_ready"])
        if self.resident_bins:
            st = torch.empty(len(reqs), dtype=torch.int32, device=self.dev)
            self.ctxs[lane].label_batch([r.state["bins"] for r in reqs], status=st, stream=s)
        else:
            with torch.cuda.stream(s):
                st = torch.empty(len(reqs), dtype=torch.int32, device=self.dev)
            self.ctxs[lane].tessellate_batch([r.state["job"] for r in reqs], status=st, stream=s)
        for k, r in enumerate(reqs):
            r.state["status"] = st[k:k + 1]
        ev = torch.cuda.Event()
        ev.record(s)
        return (lane, ev)

    def labelling_done(self, token):
        if token[1].query():
            if token[0] not in self.free_lanes:
                self.free_lanes.append(token[0])
            return True
        return False

    def finish(self, req):
        st = req.state
        req.status = int(st["status"].item())
        if self.resident_bins:
            st["bins"].free(stream=self.s_up)
        if self.keep_labels:
            req.labels = st["labels"]
        req.state = {}

    def run_alone(self, req):
        job = self._job(req)
        st = req.state
        s = self.streams[0]
        s.wait_stream(self.s_up)
        self.ctxs[0].tessellate(job, status=st["status"], stream=s)
        s.synchronize()
        req.status = int(st["status"].item())
        if self.keep_labels:
            req.labels = st["labels"]
        req.state = {}

    def digest_all(self, reqs):
        """Hashes the kept label images (after the replay) and drops them."""
        for r in reqs:
            if getattr(r, "labels", None) is not None:
                r.digest = int(digest_device(r.labels).item())
                r.labels = None


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
        running = []                  # (token, [requests]) of the launches in flight
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
            # requests whose inputs (or bins) are ready
            still = []
            for r in binning:
                if self.ex.binning_done(r):
                    ready.append(r)
                    progressed = True
                else:
                    still.append(r)
            binning = still
            # retire finished launches
            keep = []
            for token, batch in running:
                if self.ex.labelling_done(token):
                    t_done = now()
                    for r in batch:
                        r.done = t_done
                        nbytes = r.state.get("bytes", 0)
                        self.ex.finish(r)
                        self.mem_in_use -= nbytes
                        active -= 1
                        done.append(r)
                    progressed = True
                else:
                    keep.append((token, batch))
            running = keep
            # launch what is ready while a lane is free
            if ready and len(running) < self.ex.max_inflight:
                batch, ready = ready[: self.max_batch], ready[self.max_batch:]
                running.append((self.ex.start_labelling(batch), batch))
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


def benchmark(ctx, n_jobs=96, side_scale=0.25, load=0.8, mem_budget=8 << 30, lanes=2):
    """Replays a request stream twice on the GPU -- continuous batching and one
    by one -- with the same arrival times.  The arrival rate is `load` times
    the one-by-one service rate, measured on the same jobs run back to back.
    Returns p50/p99 latency and throughput of both, and whether every job's
    labels are identical in both modes."""
    ex = GpuExecutor(ctx, lanes=lanes)
    jobs = make_stream(n_jobs, 1.0, side_scale)
    # warm-up of both paths, then the one-by-one service time of exactly these
    # jobs, back to back
    Server(ex).run_one_by_one([Request(r.rid, r.workload, 0.0) for r in jobs[:16]])
    Server(ex).run([Request(r.rid, r.workload, 0.0) for r in jobs[:16]])
    cal = Server(ex).run_one_by_one([Request(r.rid, r.workload, 0.0) for r in jobs])
    service = max(r.done for r in cal) / len(cal)
    for r in cal:
        r.labels = None
    rate = load / service
    from . import inputs
    t = inputs.arrivals(n_jobs, rate)
    stream = [Request(r.rid, r.workload, float(t[k])) for k, r in enumerate(jobs)]
    srv = Server(ex, mem_budget=mem_budget)
    batched = srv.run([Request(r.rid, r.workload, r.arrival) for r in stream])
    ex.digest_all(batched)
    alone = Server(ex, mem_budget=mem_budget).run_one_by_one(
        [Request(r.rid, r.workload, r.arrival) for r in stream])
    ex.digest_all(alone)
    same = all(a.digest == b.digest and a.status == b.status for a, b in zip(batched, alone))
    return {"jobs": n_jobs, "side_scale": side_scale, "rate_per_s": round(rate, 2),
            "service_ms_alone": round(service * 1e3, 3), "lanes": lanes,
            "batched": summarize(batched), "one_by_one": summarize(alone),
            "mean_batch": round(float(np.mean(srv.batches)), 2) if srv.batches else 0,
            "labels_identical": bool(same)}
