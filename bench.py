#!/usr/bin/env python3
"""Throughput of the device library on 3D Voronoi 512^3 with 100,000 sites.

One step = one whole plain-path call (vt_tessellate): counting-sort binning of
the sites plus labelling of all 134,217,728 voxels, inputs already resident
in HBM.  The line printed at the end also carries
  - roofline: the labelling kernel is bound by binary64 arithmetic
    ("alu"): its algorithmic work, the paper's ln N + 1 key evaluations per
    voxel (eq. dl) times the operations of one key, over its average
    duration (HIP events recorded by the library on the stream the kernel
    runs on), against the FP64 vector peak of 78.6 TFLOP/s; beside it the
    HBM write roofline (4 B per voxel against 8 TB/s), and the HBM traffic
    and FP64 / VALU issue rates measured by hardware counters (committed
    counter summary, used only while it matches the kernel source and plan);
  - configs: the same measurement on the other benchmark configurations
    (M1 64^3 Voronoi, M3 512^3 Laguerre, M4 384^3 Johnson-Mehl);
  - autotune: the autotuner on a non-uniform class (clustered sites),
    built-in against tuned plan on a held-out job of the class;
  - cpu_baseline: the CPU oracle (paper's two-step ball algorithm) timed on
    the host's cores on the same workload, its times on the other
    configurations, the device labels of every timed configuration checked
    against the oracle at sampled voxels, and every 125th served job's labels
    (checksums) against the oracle's;
  - general_path (unless --no-nd): the general-dimension kernel on a 4D Voronoi
    diagram, 64^4 voxels and 16,384 sites, and on a 3D Voronoi diagram of
    20,000 sites in a triclinic periodic cell (128^3 voxels);
  - serving: the request stream replayed through the continuous-batching
    loop and one job at a time (p50/p99 latency, throughput) at 0.8, 0.95 and
    1.5 times the one-by-one service rate and as a burst, unless --no-serving.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations per
# second (a wavefront-64 instruction occupies a SIMD for four cycles).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# the sources of the labelling kernel (device code, launch code, shared types)
LABEL_KERNEL_SRC = [os.path.join(ROOT, "paper_2201_13234_amd", "csrc", f)
                    for f in ("label_core.h", "label_kernel.hip", "vt_internal.h")]


def counters_path(workload):
    return os.path.join(ROOT, "profiles", f"label_counters_{workload.split('_')[0].lower()}.json")


def source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in LABEL_KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def plan_key(plan):
    """A launch plan (bins per axis, tile configuration, bin factor) in the
    form the counter summary stores."""
    return {"bins": [int(b) for b in plan["bins"]], "tile_cfg": int(plan["tile_cfg"]),
            "bin_factor": float(plan["bin_factor"])}


def load_counters(workload, plan):
    """Committed counter summary for this workload, if it was taken on the
    current labelling kernel source with the same launch plan (else None)."""
    try:
        rec = json.load(open(counters_path(workload)))
    except (OSError, ValueError):
        return None
    if rec.get("label_kernel_sha256") != source_digest() or rec.get("workload") != workload:
        return None
    if rec.get("plan") != plan_key(plan):
        return None
    return rec


def _pmc_rows(path):
    """Per-kernel sums of each counter and the number of dispatches, from a
    rocprofv3 counter_collection.csv."""
    import csv
    import collections
    sums = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for r in csv.DictReader(open(path)):
        k = r["Kernel_Name"]
        sums[k][r["Counter_Name"]] += float(r["Counter_Value"])
        disp[k].add(r["Dispatch_Id"])
    return sums, {k: len(v) for k, v in disp.items()}


def _per_dispatch(path, counter, match):
    sums, nd = _pmc_rows(path)
    hits = [k for k in sums if match(k) and counter in sums[k]]
    if not hits:
        raise SystemExit(f"{path}: no kernel matching the probe has {counter}")
    tot = sum(sums[k][counter] for k in hits)
    n = sum(nd[k] for k in hits)
    return tot / n, n, hits


def plan_from_log(path):
    """The launch plan printed in the bench line of a counter run's log."""
    lines = [l for l in open(path) if l.startswith("{") and '"metric"' in l]
    if not lines:
        raise SystemExit(f"{path}: no bench line")
    return plan_key(json.loads(lines[-1])["config"]["plan"])


def summarize_counters(args):
    """Turns three rocprofv3 --pmc runs of `bench.py --copy-probe-mib M`
    (the probe is torch's int32 -> float32 direct copy kernel)
    (FETCH_SIZE, WRITE_SIZE, SQ instruction counters) into the committed
    counter summary.  FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled
    by what they read for the plain copy of known size in the same run."""
    fetch_csv, write_csv, sq_csv = args.summarize
    copy_bytes = args.copy_probe_mib * 2 ** 20
    is_label = lambda k: "k_label_single" in k
    is_copy = lambda k: "direct_copy_kernel" in k
    lf, n_lf, names = _per_dispatch(fetch_csv, "FETCH_SIZE", is_label)
    cf, n_cf, cnames = _per_dispatch(fetch_csv, "FETCH_SIZE", is_copy)
    lw, _, _ = _per_dispatch(write_csv, "WRITE_SIZE", is_label)
    cw, _, _ = _per_dispatch(write_csv, "WRITE_SIZE", is_copy)
    fetch_scale = copy_bytes / (cf * 1024.0)
    write_scale = copy_bytes / (cw * 1024.0)
    rec = {
        "workload": args.workload_name,
        "label_kernel_sha256": source_digest(),
        "kernel": names[0],
        "copy_probe": {"kernel": cnames[0][:96] + "...", "bytes_read": copy_bytes, "bytes_written": copy_bytes,
                       "fetch_kib": round(cf, 1), "write_kib": round(cw, 1),
                       "fetch_scale": round(fetch_scale, 4), "write_scale": round(write_scale, 4)},
        "label_fetch_kib": round(lf, 1),
        "label_write_kib": round(lw, 1),
        "hbm_read_bytes_per_launch": round(lf * 1024.0 * fetch_scale),
        "hbm_write_bytes_per_launch": round(lw * 1024.0 * write_scale),
        "dispatches": n_lf,
        "plan": plan_from_log(args.plan_from),
        "commands": args.commands,
    }
    rec["hbm_bytes_per_launch"] = rec["hbm_read_bytes_per_launch"] + rec["hbm_write_bytes_per_launch"]
    if sq_csv != "-":
        sums, nd = _pmc_rows(sq_csv)
        ks = [k for k in sums if is_label(k)]
        per = {c: sum(sums[k][c] for k in ks) / sum(nd[k] for k in ks)
               for c in sums[ks[0]]}
        rec["sq_per_launch"] = {c: round(v) for c, v in sorted(per.items())}
    out = counters_path(args.workload_name)
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec, indent=1))


def cpu_baseline(w, labels):
    """The oracle on the host cores (one full diagram), and the device labels
    `labels` of the same workload checked at 2,000 sampled voxels."""
    import numpy as np
    import oracle
    p = oracle.problem(w.n, w.L, w.kind, w.periodic, w.growth)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.tessellate(p, w.coords, w.param, nthreads=threads)
    dt = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    vox = np.stack([rng.integers(0, n, 2000) for n in w.n], axis=1)
    ref, _ = oracle.label_points(p, w.coords, w.param, vox)
    got = labels[tuple(vox[:, a] for a in reversed(range(len(w.n))))]
    return {"value": round(w.nvox / dt / 1e9, 6), "unit": "Gvoxels/s", "cores": threads,
            "kind": "oracle", "seconds": round(dt, 3),
            "sample": f"one full diagram of the benchmark workload ({w.name}), two-step ball algorithm",
            "sampled_parity": {"voxels": int(len(vox)), "mismatches": int((got != ref).sum())}}


def serving_sampled_parity(keep, every=125):
    """Part of the CPU leg: labels of a stratified sample of the served jobs
    (every `every`-th job of the stream), as checksums of the batched replay,
    against the oracle's labels of the same jobs."""
    import oracle
    from paper_2201_13234_amd import serve
    jobs, dig = keep["jobs"], keep["digests"]
    checked = bad = 0
    vox = 0
    for r in jobs[::every]:
        w = r.workload
        p = oracle.problem(w.n, w.L, w.kind, w.periodic, w.growth)
        lab, _, _ = oracle.tessellate(p, w.coords, w.param)
        checked += 1
        vox += int(lab.size)
        bad += int(dig.get(r.rid) != serve.digest_host(lab))
    return {"jobs": checked, "voxels": vox, "mismatches": bad}


def oracle_survey(skip=()):
    """Oracle wall times on the benchmark configurations (all host cores):
    M1 as the median of 3, with one thread and by brute force too; M2-M4 one
    run each.  Names in `skip` are left out (already timed)."""
    import statistics
    import oracle
    from paper_2201_13234_amd import inputs
    out = {"cores": oracle.max_threads()}
    for name in ("M1", "M2", "M3", "M4"):
        w = inputs.CONFIGS[name]()
        if w.name in skip:
            continue
        p = oracle.problem(w.n, w.L, w.kind, w.periodic, w.growth)
        reps = 3 if name == "M1" else 1
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.tessellate(p, w.coords, w.param)
            ts.append(time.perf_counter() - t0)
        out[name] = {"seconds": round(statistics.median(ts), 3), "gvox_per_s": round(w.nvox / statistics.median(ts) / 1e9, 5)}
        if name == "M1":
            t0 = time.perf_counter()
            oracle.tessellate(p, w.coords, w.param, nthreads=1)
            out["M1_one_thread_seconds"] = round(time.perf_counter() - t0, 3)
            t0 = time.perf_counter()
            oracle.brute(p, w.coords, w.param)
            out["M1_brute_force_seconds"] = round(time.perf_counter() - t0, 3)
    return out


def nd_workload():
    """4D Voronoi, 64^4 voxels, 16,384 uniform periodic sites (about M2's
    voxels per site), seed 6."""
    import numpy as np
    from paper_2201_13234_amd import inputs
    n = (64, 64, 64, 64)
    L = tuple(float(v) for v in n)
    rng = np.random.default_rng(6)
    return n, L, inputs.uniform_sites(rng, 16384, L)


# Triclinic cell of the general-period workload (rows = period vectors).
LATTICE_CELL = [[128.0, 0.0, 0.0], [40.0, 120.0, 0.0], [25.0, -18.0, 110.0]]


def lattice_workload():
    """3D Voronoi in a triclinic periodic cell, 128^3 voxels, 20,000 sites
    uniform in the cell, seed 7."""
    import numpy as np
    n = (128, 128, 128)
    rng = np.random.default_rng(7)
    return n, np.array(LATTICE_CELL), rng.random((20000, 3)) @ np.array(LATTICE_CELL)


def nd_sampled_parity(labels, lat_labels=None):
    """Part of the CPU leg: the general kernel's labels at sampled voxels
    against the oracle (4D workload, and the triclinic one if given)."""
    import numpy as np
    import oracle
    n, L, coords = nd_workload()
    rng = np.random.default_rng(1)
    vox = np.stack([rng.integers(0, v, 2000) for v in n], axis=1)
    ref, _ = oracle.label_points(oracle.problem(n, L, oracle.VORONOI, True), coords, None, vox)
    got = labels[tuple(vox[:, a] for a in reversed(range(len(n))))]
    out = {"voxels": int(len(vox)), "mismatches": int((got != ref).sum())}
    if lat_labels is not None:
        n, P, coords = lattice_workload()
        vox = np.stack([rng.integers(0, v, 2000) for v in n], axis=1)
        ref, _ = oracle.label_points(oracle.problem(n, [1.0] * 3, oracle.VORONOI, True, periods=P),
                                     coords, None, vox)
        got = lat_labels[tuple(vox[:, a] for a in reversed(range(3)))]
        out["lattice_voxels"] = int(len(vox))
        out["lattice_mismatches"] = int((got != ref).sum())
    return out


def general_path(ctx, steps, warmup):
    """The general-dimension kernel (vt_tessellate_nd) on nd_workload(),
    timed with events on the stream the kernels run on."""
    import numpy as np
    import torch
    from paper_2201_13234_amd import inputs, vtess
    n, L, coords = nd_workload()
    dev = torch.device("cuda:0")
    job = vtess.Job(n=n, L=L, kind=inputs.VORONOI, periodic=True,
                    coords=torch.from_numpy(coords).to(dev))
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        ctx.tessellate_nd(job, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        ctx.tessellate_nd(job, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nvox = int(np.prod(n))
    out = {"workload": "4D Voronoi 64^4, 16,384 sites, periodic, seed 6", "ms_per_call": round(ms, 4),
           "value": round(nvox / (ms * 1e-3) / 1e9, 3), "unit": "Gvoxels/s",
           "hbm_write_frac": round(4.0 * nvox / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "labels": job.labels.cpu().numpy()}
    # general period vectors
    n, P, coords = lattice_workload()
    lj = vtess.Job(n=n, L=(1.0, 1.0, 1.0), kind=inputs.VORONOI, periodic=True,
                   coords=torch.from_numpy(coords).to(dev), periods=P.tolist())
    for _ in range(warmup):
        ctx.tessellate_nd(lj, stream=stream)
    e0.record(stream)
    for _ in range(steps):
        ctx.tessellate_nd(lj, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nvox = int(np.prod(n))
    out["lattice"] = {"workload": "3D Voronoi 128^3, triclinic periodic cell, 20,000 sites, seed 7",
                      "ms_per_call": round(ms, 4), "value": round(nvox / (ms * 1e-3) / 1e9, 3),
                      "unit": "Gvoxels/s"}
    out["lattice_labels"] = lj.labels.cpu().numpy()
    return out


def time_config(ctx, w, steps, warmup, stream):
    """Timed plain-path steps on workload w: wall time per step and the
    library's event-timed phases (binning, labelling kernel, overflow)."""
    import torch
    from paper_2201_13234_amd import vtess
    dev = torch.device("cuda:0")
    job = vtess.Job(n=w.n, L=w.L, kind=w.kind, periodic=w.periodic, growth=w.growth,
                    coords=torch.from_numpy(w.coords).to(dev),
                    param=None if w.param is None else torch.from_numpy(w.param).to(dev))
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    for _ in range(warmup):
        ctx.tessellate(job, status=status, stream=stream)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.tessellate(job, status=status, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.profile_enable(False)
    bin_ms, label_ms, ovf_ms, calls = ctx.profile_read()
    return {"job": job, "elapsed": elapsed, "ms_per_step": elapsed * 1e3 / steps,
            "gvox": w.nvox * steps / elapsed / 1e9, "bin_ms": bin_ms / max(calls, 1),
            "label_ms": label_ms / max(calls, 1), "ovf_ms": ovf_ms / max(calls, 1), "plan": ctx.plan(job)}


def roofline_of(w, label_ms, cnt=None):
    """Roofline of the labelling kernel on workload w (see the module doc)."""
    write_bytes = 4.0 * w.nvox
    hbm = write_bytes / (label_ms * 1e-3) / 1e9
    # The kernel is bound by binary64 arithmetic.  Algorithmic work: the
    # paper's key evaluations per voxel, ln N + 1 (eq. dl), times the
    # operations of one key (3D: 3 subtractions, 3 multiplications, 2
    # additions; Laguerre one subtraction more; Johnson-Mehl a square root
    # and a multiplication more; 2D one subtraction, one multiplication and
    # one addition fewer).
    per_key = {0: 8, 1: 9, 2: 10}[w.kind] - (3 if w.ndim == 2 else 0)
    evals = math.log(w.nsites) + 1.0
    alg_flops = w.nvox * evals * per_key
    tflops = alg_flops / (label_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(tflops, 2), "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(tflops / FP64_PEAK_TFLOPS, 4),
            "traffic": cnt["hbm_bytes_per_launch"] if cnt else None,
            "kernel": "k_label_single (main labelling kernel)",
            "kernel_avg_ms": round(label_ms, 4),
            "algorithmic_flops": alg_flops,
            "algorithmic_basis": f"{evals:.2f} key evaluations per voxel (ln N + 1) x {per_key} binary64 "
                                 f"operations per key, {w.nvox} voxels",
            "hbm_write": {"achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(hbm / HBM_PEAK_GBS, 4), "algorithmic_bytes": write_bytes}}
    if cnt and "sq_per_launch" in cnt:
        sq = cnt["sq_per_launch"]
        sec = label_ms * 1e-3
        if "SQ_INSTS_VALU_FLOPS_FP64" in sq:
            # the counter sums FP64 operations per wavefront instruction (FMA = 2);
            # times 64 lanes (an upper bound: it assumes full execution masks)
            f64 = sq["SQ_INSTS_VALU_FLOPS_FP64"] * 64 / sec / 1e12
            roof["fp64_counted"] = {"achieved": round(f64, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                    "frac": round(f64 / FP64_PEAK_TFLOPS, 4)}
        if "SQ_INSTS_VALU" in sq:
            v = sq["SQ_INSTS_VALU"] * 64 / sec / 1e12
            roof["valu_issue"] = {"achieved": round(v, 2), "peak": round(VALU_PEAK_TOPS, 2),
                                  "unit": "Tlane-op/s", "frac": round(v / VALU_PEAK_TOPS, 4)}
            if "SQ_WAVES" in sq and sq["SQ_WAVES"]:
                roof["valu_per_wave"] = round(sq["SQ_INSTS_VALU"] / sq["SQ_WAVES"], 1)
    return roof


def sampled_parity(w, labels, nvox=2000, seed=0):
    """Device labels of workload w against the oracle at sampled voxels."""
    import numpy as np
    import oracle
    p = oracle.problem(w.n, w.L, w.kind, w.periodic, w.growth)
    rng = np.random.default_rng(seed)
    vox = np.stack([rng.integers(0, n, nvox) for n in w.n], axis=1)
    ref, _ = oracle.label_points(p, w.coords, w.param, vox)
    got = labels[tuple(vox[:, a] for a in reversed(range(len(w.n))))]
    return {"voxels": int(len(vox)), "mismatches": int((got != ref).sum())}


def autotune_clustered(log):
    """The autotuner on a non-uniform class (3D Voronoi 256^3, 40,000 sites in
    200 Gaussian clusters of sigma 6 voxels, periodic): tuned on two samples
    (seeds 41, 42), then the built-in and the tuned plan timed on a held-out
    job of the class (seed 43), in contexts of their own."""
    import json
    import tempfile
    import torch
    from paper_2201_13234_amd import inputs, vtess
    samples = [inputs.clustered(s) for s in (41, 42)]
    held = inputs.clustered(43)
    dev = torch.device("cuda:0")
    to_job = lambda w: vtess.Job(n=w.n, L=w.L, kind=w.kind, periodic=w.periodic,
                                 coords=torch.from_numpy(w.coords).to(dev))
    tuned, plain = vtess.Context(0), vtess.Context(0)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        t0 = time.perf_counter()
        tuned.autotune([to_job(w) for w in samples], cache_path=path)
        tune_s = time.perf_counter() - t0
        entry = json.load(open(path))[0]
    log(f"autotune: {tune_s:.1f} s, entry {entry}")
    stream = torch.cuda.current_stream()
    rt = time_config(tuned, held, 20, 3, stream)
    rd = time_config(plain, held, 20, 3, stream)
    same = bool(torch.equal(rt["job"].labels, rd["job"].labels))
    tuned.close()
    plain.close()
    return {"class": "3D Voronoi 256^3, 40,000 sites in 200 Gaussian clusters (sigma 6 voxels), periodic",
            "samples": [w.name for w in samples], "held_out": held.name, "tuning_s": round(tune_s, 2),
            "cache_entry": entry,
            "default": {"plan": rd["plan"], "ms_per_step": round(rd["ms_per_step"], 4),
                        "label_ms": round(rd["label_ms"], 4)},
            "tuned": {"plan": rt["plan"], "ms_per_step": round(rt["ms_per_step"], 4),
                      "label_ms": round(rt["label_ms"], 4)},
            "labels_identical": same, "_held": held, "_labels": rt["job"].labels.cpu().numpy()}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="M2", help="M1..M4 (default M2, the headline workload)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-stream replay")
    ap.add_argument("--no-others", action="store_true", help="time only --config (not M1-M4)")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner run on the clustered class")
    ap.add_argument("--nd", action="store_true", help="(default) time the general-dimension kernel")
    ap.add_argument("--no-nd", action="store_true", help="skip the general-dimension kernel (4D, triclinic)")
    ap.add_argument("--serving-jobs", type=int, default=2000,
                    help="request-stream length (the stream of 2,000 seeded jobs by default)")
    ap.add_argument("--serving-scale", type=float, default=1.0,
                    help="scale of the request-stream grid sides (1.0 = full size)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed steps, copy a buffer of this size three times (a plain "
                         "copy kernel of known traffic, for scaling HBM counters)")
    ap.add_argument("--summarize", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "SQ_CSV"),
                    help="no GPU run: write the counter summary of --config from three rocprofv3 "
                         "counter_collection.csv files (SQ_CSV may be '-')")
    ap.add_argument("--commands", default="", help="with --summarize: the commands that made the CSVs")
    ap.add_argument("--plan-from", default="", help="with --summarize: a log of one of those runs (its "
                                                     "bench line gives the launch plan)")
    args = ap.parse_args()
    if args.summarize:
        from paper_2201_13234_amd import inputs
        args.workload_name = inputs.CONFIGS[args.config]().name
        if args.copy_probe_mib <= 0:
            raise SystemExit("--summarize needs --copy-probe-mib (the size the runs copied)")
        if not args.plan_from:
            raise SystemExit("--summarize needs --plan-from (a log with the runs' bench line)")
        summarize_counters(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the labelling path "
              "has no multi-GPU part (one process labels whole diagrams on one device).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2201_13234_amd import inputs, vtess

    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)
    w = inputs.CONFIGS[args.config]()
    ctx = vtess.Context(0)
    stream = torch.cuda.current_stream()
    log(f"{w.name}: warmup {args.warmup}, {args.steps} steps")
    r = time_config(ctx, w, args.steps, args.warmup, stream)
    log(f"{args.steps} steps in {r['elapsed']:.4f} s")
    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib * 2 ** 20
        # int32 -> float32 conversion: one elementwise kernel per call that
        # reads and writes nb bytes (a same-type copy_ would go to the
        # runtime's blit kernels, mixed with other transfers).
        src = torch.ones(nb // 4, dtype=torch.int32, device="cuda:0")
        dst = torch.empty(nb // 4, dtype=torch.float32, device="cuda:0")
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cnt = load_counters(w.name, r["plan"])
    out = {
        "metric": "Gvoxels/s at 3D 512^3/100k sites; batched p50/p99 latency vs one-by-one",
        "value": round(r["gvox"], 3),
        "unit": "Gvoxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(w.n), "sites": w.nsites,
                   "kind": inputs.KIND_NAMES[w.kind], "periodic": w.periodic,
                   "seed": w.meta.get("seed"), "path": "plain (vt_tessellate)", "plan": r["plan"]},
        "phases_ms": {"binning": round(r["bin_ms"], 4), "labelling": round(r["label_ms"], 4),
                      "overflow": round(r["ovf_ms"], 4)},
        "roofline": roofline_of(w, r["label_ms"], cnt),
    }
    labels = {w.name: (w, r["job"].labels.cpu().numpy())}
    del r
    if not args.no_others:
        # the other benchmark configurations, same measurement (not the value)
        out["configs"] = {}
        for name in ("M1", "M2", "M3", "M4"):
            wc = inputs.CONFIGS[name]()
            if wc.name == w.name:
                rc = {"ms_per_step": out["ms_per_step"], "gvox": out["value"], "bin_ms": out["phases_ms"]["binning"],
                      "label_ms": out["phases_ms"]["labelling"], "plan": out["config"]["plan"]}
                roof = out["roofline"]
            else:
                log(f"{wc.name}: warmup {args.warmup}, {args.steps} steps")
                rc = time_config(ctx, wc, args.steps, args.warmup, stream)
                labels[wc.name] = (wc, rc["job"].labels.cpu().numpy())
                roof = roofline_of(wc, rc["label_ms"], load_counters(wc.name, rc["plan"]))
            out["configs"][name] = {
                "workload": wc.name, "ms_per_step": round(rc["ms_per_step"], 4), "gvox_per_s": round(rc["gvox"], 3),
                "binning_ms": round(rc["bin_ms"], 4), "labelling_ms": round(rc["label_ms"], 4), "plan": rc["plan"],
                "alu_frac": roof["frac"], "alu_tflops": roof["achieved"],
                "hbm_write_frac": roof["hbm_write"]["frac"], "hbm_write_gbs": roof["hbm_write"]["achieved"],
                **({"valu_issue_frac": roof["valu_issue"]["frac"]} if "valu_issue" in roof else {}),
                **({"traffic": roof["traffic"]} if roof.get("traffic") else {})}
    tuned = None
    if not args.no_tune:
        log("autotuner on the clustered class")
        tuned = autotune_clustered(log)
        out["autotune"] = {k: v for k, v in tuned.items() if not k.startswith("_")}
    if not args.no_nd:
        log("general-dimension kernel (4D, triclinic)")
        g = general_path(ctx, max(args.steps // 4, 2), 1)
        nd_labels = g.pop("labels")
        lat_labels = g.pop("lattice_labels")
        out["general_path"] = g
    keep = {}
    if not args.no_serving:
        from paper_2201_13234_amd import serve
        log(f"serving replay ({args.serving_jobs} jobs)")
        out["serving"] = serve.benchmark(ctx, n_jobs=args.serving_jobs, side_scale=args.serving_scale,
                                         log=lambda m: log(f"serving: {m}"), keep=keep)
    if not args.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(w, labels[w.name][1])
        log("oracle survey of the other configurations")
        survey = oracle_survey(skip=(w.name,))
        survey[w.name.split("_")[0]] = {"seconds": out["cpu_baseline"]["seconds"],
                                        "gvox_per_s": out["cpu_baseline"]["value"]}
        out["cpu_baseline"]["oracle_survey"] = survey
        out["cpu_baseline"]["configs_sampled_parity"] = {name: sampled_parity(wc, lab)
                                                         for name, (wc, lab) in labels.items()}
        if tuned is not None:
            out["cpu_baseline"]["autotune_sampled_parity"] = sampled_parity(tuned["_held"], tuned["_labels"],
                                                                          nvox=20000)
        if keep:
            log("CPU oracle on a sample of the served jobs")
            out["cpu_baseline"]["serving_sampled_parity"] = serving_sampled_parity(keep)
        if not args.no_nd:
            out["cpu_baseline"]["general_path_sampled_parity"] = nd_sampled_parity(nd_labels, lat_labels)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
