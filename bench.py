#!/usr/bin/env python3
"""Throughput of the device library on 3D Voronoi 512^3 with 100,000 sites.

One step = one whole plain-path call (vt_tessellate): counting-sort binning of
the sites plus labelling of all 134,217,728 voxels, inputs already resident
in HBM.  The line printed at the end also carries
  - roofline: the labelling kernel's algorithmic HBM write bytes (4 B per
    voxel) over its average duration, timed with HIP events recorded by the
    library on the stream the kernel runs on, against 8 TB/s;
  - cpu_baseline: the CPU oracle (paper's two-step ball algorithm) timed on
    the host's cores on the same workload;
  - serving: a short request stream replayed through the continuous-batching
    loop and one job at a time (p50/p99 latency), unless --no-serving.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def traffic_from_profiles(nvox):
    """HBM bytes per labelling launch from the committed counter summary, if
    it was taken on the current kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "label_traffic_m2.json")
    src = os.path.join(ROOT, "paper_2201_13234_amd", "csrc", "label_kernel.hip")
    try:
        rec = json.load(open(path))
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if rec.get("label_kernel_sha256") != digest:
            return None
        return rec.get("hbm_bytes_per_launch")
    except (OSError, ValueError):
        return None


def cpu_baseline(w):
    import oracle
    p = oracle.problem(w.n, w.L, w.kind, w.periodic, w.growth)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.tessellate(p, w.coords, w.param, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(w.nvox / dt / 1e9, 6), "unit": "Gvoxels/s", "cores": threads,
            "kind": "oracle", "seconds": round(dt, 3),
            "sample": f"one full diagram of the benchmark workload ({w.name}), two-step ball algorithm"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="M2", help="M1..M4 (default M2, the headline workload)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-stream replay")
    ap.add_argument("--serving-jobs", type=int, default=96)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the labelling path "
              "has no multi-GPU part; see DESIGN.md for how it would shard.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2201_13234_amd import inputs, vtess

    w = inputs.CONFIGS[args.config]()
    dev = torch.device("cuda:0")
    ctx = vtess.Context(0)
    job = vtess.Job(n=w.n, L=w.L, kind=w.kind, periodic=w.periodic, growth=w.growth,
                    coords=torch.from_numpy(w.coords).to(dev),
                    param=None if w.param is None else torch.from_numpy(w.param).to(dev))
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    print(f"[bench] {w.name}: warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        ctx.tessellate(job, status=status, stream=stream)
    torch.cuda.synchronize()
    assert int(status.item()) == 0

    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.tessellate(job, status=status, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.profile_enable(False)
    bin_ms, label_ms, calls = ctx.profile_read()
    print(f"[bench] {args.steps} steps in {elapsed:.4f} s", file=sys.stderr, flush=True)

    ms_per_step = elapsed * 1e3 / args.steps
    gvox = w.nvox * args.steps / elapsed / 1e9
    label_avg_ms = label_ms / max(calls, 1)
    bin_avg_ms = bin_ms / max(calls, 1)
    write_bytes = 4.0 * w.nvox
    achieved = write_bytes / (label_avg_ms * 1e-3) / 1e9
    out = {
        "metric": "Gvoxels/s at 3D 512^3/100k sites; batched p50/p99 latency vs one-by-one",
        "value": round(gvox, 3),
        "unit": "Gvoxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(w.n), "sites": w.nsites,
                   "kind": inputs.KIND_NAMES[w.kind], "periodic": w.periodic,
                   "seed": w.meta.get("seed"), "path": "plain (vt_tessellate)"},
        "phases_ms": {"binning": round(bin_avg_ms, 4), "labelling": round(label_avg_ms, 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profiles(w.nvox),
                     "kernel": "k_label_single (labelling)",
                     "algorithmic_bytes": write_bytes},
    }
    # correctness of the timed configuration: sampled voxels against the oracle
    import oracle
    rng = np.random.default_rng(0)
    vox = np.stack([rng.integers(0, n, 2000) for n in w.n], axis=1)
    lab = job.labels.cpu().numpy()
    ref, _ = oracle.label_points(oracle.problem(w.n, w.L, w.kind, w.periodic, w.growth),
                                 w.coords, w.param, vox)
    got = lab[tuple(vox[:, a] for a in reversed(range(len(w.n))))]
    out["sampled_parity"] = {"voxels": int(len(vox)), "mismatches": int((got != ref).sum())}

    if not args.no_serving:
        from paper_2201_13234_amd import serve
        print(f"[bench] serving replay ({args.serving_jobs} jobs)", file=sys.stderr, flush=True)
        out["serving"] = serve.benchmark(ctx, n_jobs=args.serving_jobs)
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
