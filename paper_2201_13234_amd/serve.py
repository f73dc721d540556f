"""Continuous-batching request loop for tessellation jobs.

Requests (one diagram each) arrive over time.  The scheduler
  - admits a request as soon as a slot is free and its device memory
    (labels, sites, bins) fits in the memory budget, in arrival order, and
    starts uploading its sites right away (and, with resident bins, binning
    them, so the bins stay on the device until the request completes);
  - whenever a launch lane is free, launches every admitted request whose
    inputs are ready as one batch (vt_tessellate_batch, or vt_label_batch over
    resident bins), so requests that arrived while others were on the GPU join
    the next batch and their uploads overlap the running batches;
  - retires finished batches, releasing memory and slots.
Latency is completion time minus arrival time.  The one-by-one baseline runs
each request alone (vt_tessellate) in arrival order.

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


class PinnedRing:
    """Host staging for uploads: one pinned buffer used as a ring.  A slice
    is reused only after the copy that read it has completed (its event)."""

    def __init__(self, torch, nbytes):
        self.torch = torch
        self.buf = torch.empty(int(nbytes), dtype=torch.uint8, pin_memory=True)
        self.np = self.buf.numpy()
        self.size = int(nbytes)
        self.head = 0
        self.inflight = []            # (start, end, event), oldest first

    def _wait_overlap(self, a, b):
        keep = []
        for s0, e0, ev in self.inflight:
            if e0 <= a or s0 >= b:
                if not ev.query():
                    keep.append((s0, e0, ev))
            else:
                ev.synchronize()
        self.inflight = keep

    def put(self, arr):
        """Copies a numpy array into the ring; returns a pinned tensor view."""
        raw = np.ascontiguousarray(arr).view(np.uint8).reshape(-1)
        n = (raw.size + 255) // 256 * 256
        if n > self.size:
            raise MemoryError("upload larger than the staging ring")
        if self.head + n > self.size:
            self.head = 0
        a, b = self.head, self.head + n
        self._wait_overlap(a, b)
        self.np[a:a + raw.size] = raw
        self.head = b
        return self.buf[a:a + raw.size], (a, b)

    def mark(self, span, event):
        self.inflight.append((span[0], span[1], event))


class GpuExecutor(Executor):
    """Executor over the device library.

    Uploads go through a pinned staging ring on their own stream.  Labelling
    launches alternate between `lanes` (context, stream) pairs so that one
    batch can be uploaded and binned while the previous one is still
    labelling.  Two modes:
      resident_bins=False  each launch is one vt_tessellate_batch call:
                           segmented binning of the batch plus one labelling
                           launch per kind/shape group (a launch of
                           a single request is a plain vt_tessellate call);
      resident_bins=True   every request is binned on arrival (vt_bins_build,
                           bins stay on the device) and a launch is one
                           vt_label_batch over the resident bins.
    Statuses come back through pinned host memory copied on the lane stream,
    so retiring a batch never synchronises.  With digest=True every label
    image is hashed on the device (vt_label_digest) on a separate stream once
    its batch has completed -- after the completion time is taken -- and the
    image is released; collect_digests() returns the hashes.
    """

    def __init__(self, ctx, device="cuda:0", lanes=2, resident_bins=False, digest=True,
                 staging_bytes=256 << 20, reserve_bytes=512 << 20, max_batch=256):
        import torch
        from . import vtess
        self.torch = torch
        self.dev = torch.device(device)
        self.ctxs = [ctx] + [vtess.Context(self.dev.index or 0) for _ in range(lanes - 1)]
        for c in self.ctxs:
            c.reserve(reserve_bytes)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(lanes)]
        self.s_up = torch.cuda.Stream(device=self.dev)
        self.s_dig = torch.cuda.Stream(device=self.dev)
        self.ring = PinnedRing(torch, staging_bytes)
        self.status_host = [torch.empty(max_batch, dtype=torch.int32, pin_memory=True) for _ in range(lanes)]
        self.status_dev = [torch.empty(max_batch, dtype=torch.int32, device=self.dev) for _ in range(lanes)]
        self.free_lanes = list(range(lanes))
        self.max_inflight = lanes
        self.max_batch = max_batch
        self.resident_bins = resident_bins
        self.digest = digest
        self.pending = []             # (request id, accumulator tensor)

    def _upload(self, arr):
        host, span = self.ring.put(arr)
        with self.torch.cuda.stream(self.s_up):
            dev = self.torch.empty(arr.shape, dtype=self.torch.float64, device=self.dev)
            dev.view(-1).view(self.torch.uint8).copy_(host, non_blocking=True)
        return dev, span

    def _job(self, req):
        from . import vtess
        torch = self.torch
        w = req.workload
        st = req.state
        st["coords"], span = self._upload(w.coords)
        spans = [span]
        st["param"] = None
        if w.param is not None:
            st["param"], span = self._upload(w.param)
            spans.append(span)
        with torch.cuda.stream(self.s_up):
            st["labels"] = torch.empty(w.shape, dtype=torch.int32, device=self.dev)
        ev = torch.cuda.Event()
        ev.record(self.s_up)
        for sp in spans:
            self.ring.mark(sp, ev)
        st["ev_up"] = ev
        return vtess.Job(n=w.n, L=w.L, kind=w.kind, periodic=w.periodic, growth=w.growth,
                         coords=st["coords"], param=st["param"], labels=st["labels"])

    def prepare(self, req):
        req.state["job"] = self._job(req)

    def start_binning(self, req):
        st = req.state
        if self.resident_bins:
            st["bstat"] = self.torch.empty(1, dtype=self.torch.int32, device=self.dev)
            st["bins"] = self.ctxs[0].bins_build(st["job"], status=st["bstat"], stream=self.s_up)
        ev = self.torch.cuda.Event()
        ev.record(self.s_up)
        st["ev_ready"] = ev

    def binning_done(self, req):
        return req.state["ev_ready"].query()

    def start_labelling(self, reqs):
        torch = self.torch
        if len(reqs) > self.max_batch:
            raise ValueError("batch larger than max_batch")
        lane = self.free_lanes.pop(0)
        s = self.streams[lane]
        for r in reqs:
            s.wait_event(r.state["ev_ready"])
        st = self.status_dev[lane][: len(reqs)]
        if self.resident_bins:
            self.ctxs[lane].label_batch([r.state["bins"] for r in reqs], status=st, stream=s)
        elif len(reqs) == 1:
            # a launch of one request takes the plain path (no job table)
            self.ctxs[lane].tessellate(reqs[0].state["job"], status=st, stream=s)
        else:
            self.ctxs[lane].tessellate_batch([r.state["job"] for r in reqs], status=st, stream=s)
        with torch.cuda.stream(s):
            self.status_host[lane][: len(reqs)].copy_(st, non_blocking=True)
        for k, r in enumerate(reqs):
            r.state["lane"], r.state["slot"] = lane, k
        ev = torch.cuda.Event()
        ev.record(s)
        return (lane, ev)

    def labelling_done(self, token):
        # The scheduler retires (finish) every request of a completed launch
        # before it starts another one, so the lane's status slots are read
        # before the lane is reused.
        if token[1].query():
            if self.digest:
                self.s_dig.wait_event(token[1])
            if token[0] not in self.free_lanes:
                self.free_lanes.append(token[0])
            return True
        return False

    def finish(self, req):
        st = req.state
        lane = st["lane"]
        req.status = int(self.status_host[lane][st["slot"]])
        if self.resident_bins:
            st["bins"].free(stream=self.streams[lane])
        self._digest(req, st["labels"])
        req.state = {}

    def _digest(self, req, labels):
        if not self.digest:
            return
        torch = self.torch
        with torch.cuda.stream(self.s_dig):
            acc = torch.zeros(1, dtype=torch.int64, device=self.dev)
        self.ctxs[0].label_digest_async(labels, acc, stream=self.s_dig)
        labels.record_stream(self.s_dig)
        self.pending.append((req.rid, acc))

    def run_alone(self, req):
        job = self._job(req)
        st = req.state
        s = self.streams[0]
        s.wait_event(st["ev_up"])
        status = self.status_dev[0][:1]
        self.ctxs[0].tessellate(job, status=status, stream=s)
        with self.torch.cuda.stream(s):
            self.status_host[0][:1].copy_(status, non_blocking=True)
        s.synchronize()
        req.status = int(self.status_host[0][0])
        if self.digest:
            self.s_dig.wait_stream(s)
        self._digest(req, st["labels"])
        req.state = {}

    def collect_digests(self):
        """Waits for the digest stream; returns {request id: checksum}."""
        self.s_dig.synchronize()
        out = {rid: int(acc.item()) % _P for rid, acc in self.pending}
        self.pending = []
        return out


# Order-sensitive hash of a label image: sum over voxels i of
# (label_i + 3) * ((i * 48271 + 97) mod P), mod P, P = 2^31 - 1 (the device
# library's vt_label_digest computes the same; every term stays below 2^62, so
# int64 arithmetic is exact).
_P = 2147483647


def digest_host(labels):
    """The same hash of a host label image (numpy)."""
    flat = np.asarray(labels).reshape(-1).astype(np.int64)
    w = (np.arange(flat.size, dtype=np.int64) * 48271 + 97) % _P
    return int(((flat + 3) * w % _P).sum() % _P)


class Server:
    """Continuous-batching scheduler.

    mem_budget: bytes of device memory the in-flight requests may hold;
    max_slots: requests in flight at once; max_batch: requests per labelling
    launch; batch_voxels: a launch takes ready requests in arrival order until
    their voxels would exceed this (a larger request goes alone), so that a
    burst of arrivals drains as a sequence of short launches rather than one
    long one that every request in it has to wait for.  A request larger than
    the whole budget is rejected (status -2) without blocking the others.
    """

    def __init__(self, executor, mem_budget=8 << 30, max_slots=64, max_batch=64, batch_voxels=24 << 20,
                 clock=time.perf_counter, sleep=time.sleep):
        self.ex = executor
        self.mem_budget = int(mem_budget)
        self.max_slots = int(max_slots)
        self.max_batch = int(max_batch)
        self.batch_voxels = int(batch_voxels)
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
                k, vox = 0, 0
                while k < len(ready) and k < self.max_batch and (k == 0 or vox + ready[k].nvox <= self.batch_voxels):
                    vox += ready[k].nvox
                    k += 1
                batch, ready = ready[:k], ready[k:]
                running.append((self.ex.start_labelling(batch), batch))
                self.batches.append(len(batch))
                progressed = True
            if not progressed:
                wait = queue[0].arrival - now() if queue else 0.0
                if wait > 0 and not (binning or ready or running):
                    self.sleep(min(wait, 0.001))
                else:
                    self.sleep(0)
        return sorted(done, key=lambda r: r.rid)

    def run_one_by_one(self, requests):
        """Baseline: each request alone (vt_tessellate), in arrival order."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        for r in reqs:
            while True:
                wait = r.arrival - (self.clock() - t0)
                if wait <= 0:
                    break
                self.sleep(min(wait, 0.001))
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


def benchmark(ctx, n_jobs=2000, side_scale=1.0, load=0.8, mem_budget=64 << 30, lanes=2, calib_jobs=0,
              max_batch=64, extra_loads=(0.95, 1.5), burst=True, log=None, keep=None):
    """Replays a request stream twice on the GPU -- continuous batching and one
    by one -- with the same arrival times.  The arrival rate is `load` times
    the one-by-one service rate, measured on all jobs (or the first
    `calib_jobs`) run back to back.  Returns p50/p99 latency and throughput of both modes, and
    whether every job's labels (device checksums) are the same in both.  Each
    of `extra_loads` repeats the comparison at that load (reported under
    "other_loads"); a load above 1 saturates the one-by-one server.  burst
    adds a replay with every job arriving at once (reported under "burst"):
    the throughput of each mode when the queue never empties.  keep (a dict,
    optional) receives the jobs and the
    batched replay's per-job label checksums at `load`, so that a caller
    can check a sample of them against another implementation."""
    say = log or (lambda msg: None)
    ex = GpuExecutor(ctx, lanes=lanes, max_batch=max(max_batch, 1))
    say(f"generating {n_jobs} jobs")
    jobs = make_stream(n_jobs, 1.0, side_scale)
    copy = lambda rs, t=None: [Request(r.rid, r.workload, r.arrival if t is None else t) for r in rs]
    # warm-up of both paths, then the one-by-one service time, back to back
    Server(ex, mem_budget=mem_budget).run_one_by_one(copy(jobs[:16], 0.0))
    Server(ex, mem_budget=mem_budget, max_batch=max_batch).run(copy(jobs[:16], 0.0))
    ex.collect_digests()
    # every job once, back to back: the one-by-one service rate, and warm
    # device allocations for every label size before either measured replay
    cal = Server(ex, mem_budget=mem_budget).run_one_by_one(copy(jobs[:calib_jobs] if calib_jobs else jobs, 0.0))
    ex.collect_digests()
    service = max(r.done for r in cal) / len(cal)
    from . import inputs
    last_digests = {}

    def replay(ld):
        if ld is None:  # burst: every job arrives at once
            rate = math.inf
            stream = [Request(r.rid, r.workload, 0.0) for r in jobs]
        else:
            rate = ld / service
            t = inputs.arrivals(n_jobs, rate)
            stream = [Request(r.rid, r.workload, float(t[k])) for k, r in enumerate(jobs)]
        say(f"load {ld if ld is not None else 'burst'}: batched replay at {rate:.1f} jobs/s")
        srv = Server(ex, mem_budget=mem_budget, max_batch=max_batch)
        batched = srv.run(copy(stream))
        db = ex.collect_digests()
        last_digests.clear()
        last_digests.update(db)
        say(f"load {ld if ld is not None else 'burst'}: one-by-one replay")
        alone = Server(ex, mem_budget=mem_budget).run_one_by_one(copy(stream))
        da = ex.collect_digests()
        same = all(a.status == b.status and db.get(a.rid) == da.get(b.rid) for a, b in zip(batched, alone))
        return {"load": ld if ld is not None else "burst",
                "rate_per_s": round(rate, 2) if math.isfinite(rate) else None, "batched": summarize(batched),
                "one_by_one": summarize(alone),
                "mean_batch": round(float(np.mean(srv.batches)), 2) if srv.batches else 0,
                "peak_mem_gb": round(srv.peak_mem / 2 ** 30, 2),
                "labels_identical": bool(same), "checked_jobs": len(db)}

    out = replay(load)
    if keep is not None:
        keep["jobs"] = jobs
        keep["digests"] = dict(last_digests)
    nvox = [r.nvox for r in jobs]
    out.update({"jobs": n_jobs, "side_scale": side_scale, "service_ms_alone": round(service * 1e3, 3),
                "lanes": lanes, "max_batch": max_batch, "voxels_total": int(sum(nvox)),
                "voxels_p50": int(np.percentile(nvox, 50))})
    out["other_loads"] = [replay(ld) for ld in extra_loads]
    if burst:
        out["burst"] = replay(None)
    return out
