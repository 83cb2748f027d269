#!/usr/bin/env python3
"""Benchmark: exact single-source geodesic fields with PCH on one MI355X.

A step is one exact FP64 distance field on the bumpy icosphere with 7
subdivisions (327,680 faces, the face count of the paper's Sphere row in
Table 3), from one seeded random source vertex; every step uses a new source,
like the paper's mean over random sources (Section 5.3). The mesh is resident
in device memory before the timed region; each step runs every phase of the
method (selection, propagation, organization, events) until the window pool
is empty.

Prints one JSON line. Besides the headline (ms per field) it carries:
  roofline     - the propagation kernel's algorithmic bytes per launch over
                 its average launch time, measured with HIP events on the
                 library's stream during the timed steps, against 8 TB/s;
  cpu_baseline - the CPU oracle (sequential ICH, one core) on a bounded
                 sample of the same workload, whose fields also check the
                 first GPU fields.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of one propagation (Algorithm 2) per processed window:
# the window record (6 doubles, 2 ints), its 64-byte half-edge record,
# geod_dist of the face's three vertices and the corner's angle_split pair.
PROP_READ_BYTES = 56 + 64 + 24 + 16
WINDOW_BYTES = 56        # one child window written
DIST_EVENT_BYTES = 20    # vertex id, distance, incoming angle
ANGLE_EVENT_BYTES = 20   # oriented edge id, distance, crossing


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_1305_1293_amd", "csrc", "pch_gpu.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def traffic_from_profile(workload_tag: str):
    """HBM bytes per propagation launch from the committed counter summary, or
    None when the summary is missing or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", f"k_propagate_{workload_tag}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not b or m.group(1) != kernel_source_hash():
        return None
    return float(b.group(1))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--k", type=int, default=8192, help="windows selected per round")
    ap.add_argument("--select", type=int, default=1, help="0: k-th smallest key, 1: adaptive step")
    ap.add_argument("--delta0", type=float, default=0.0, help="first adaptive step (0 = 2x mean edge)")
    ap.add_argument("--hops", type=int, default=1, help="propagation hops per round")
    ap.add_argument("--time-every", type=int, default=8,
                    help="time the propagation kernel of every n-th round with HIP events")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes 5 times (the reference "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters to bytes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the method's fields are "
              "independent per GPU, see the multi-GPU design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1305_1293_amd import meshgen as G
    from paper_1305_1293_amd import pch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_bytes > 0:
        n = args.copy_bytes // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 8 * n, "copies": 5}), flush=True)
        return
    m = G.config_mesh(2)
    rng = np.random.default_rng(2024)
    srcs = rng.choice(m.nv, size=args.warmup + args.steps, replace=False).astype(np.int32)
    mesh = pch.Mesh.from_generated(m)
    out = torch.empty(m.nv, dtype=torch.float64, device="cuda")
    opts = dict(k=args.k, collect_timing=args.time_every, select_mode=args.select, delta0=args.delta0, hops=args.hops)

    for i in range(args.warmup):
        pch.geodesic(mesh, [int(srcs[i])], out=out, **opts)
    torch.cuda.synchronize()

    keep = []
    tot = dict(processed=0, created=0, fan_windows=0, dist_events=0, angle_events=0, rounds=0,
               ms_propagate=0.0, propagate_launches=0)
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, st = pch.geodesic(mesh, [int(srcs[args.warmup + i])], out=out, return_stats=True, **opts)
        for kk in tot:
            tot[kk] += st[kk]
        if len(keep) < 8:
            keep.append(out.clone())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ms_per_field = 1000.0 * wall / args.steps

    kids = tot["created"] - tot["fan_windows"]
    prop_bytes = (PROP_READ_BYTES * tot["processed"] + WINDOW_BYTES * kids
                  + DIST_EVENT_BYTES * tot["dist_events"] + ANGLE_EVENT_BYTES * tot["angle_events"])
    # every round launches the propagation kernel once per hop; the HIP events
    # bracket the launches of every n-th round
    timed = max(tot["propagate_launches"], 1)
    avg_launch_s = tot["ms_propagate"] / 1000.0 / timed
    all_launches = max(tot["rounds"] * args.hops, 1)
    bytes_per_launch = prop_bytes / all_launches
    achieved = bytes_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    traffic = traffic_from_profile("icosphere7")
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": "k_propagate", "avg_launch_us": round(avg_launch_s * 1e6, 3),
                "alg_bytes_per_launch": round(bytes_per_launch, 1), "launches": all_launches,
                "timed_launches": tot["propagate_launches"],
                "propagate_share_of_wall": round(avg_launch_s * all_launches / wall, 4)}

    cpu = None
    max_err = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        hbar = float(O.lengths(m).mean())
        n, t_cpu, errs = 0, 0.0, []
        while n < len(keep) and (t_cpu < args.cpu_seconds or n < 2):
            s = int(srcs[args.warmup + n])
            tc = time.perf_counter()
            ref, _ = O.ich(m, [s])
            t_cpu += time.perf_counter() - tc
            got = keep[n].cpu().numpy()
            errs.append(float(np.max(np.abs(got - ref) / np.maximum(ref, hbar))))
            n += 1
        cpu = {"value": round(1000.0 * t_cpu / n, 3), "unit": "ms", "cores": 1, "kind": "oracle",
               "sample": f"{n} fields (the first timed sources) on the same mesh, sequential ICH on one core"}
        max_err = max(errs)

    line = {
        "metric": "ms per exact single-source field",
        "value": round(ms_per_field, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_field, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "bumpy icosphere, 7 midpoint subdivisions, 327,680 faces, one seeded random "
                               "source per field", "faces": m.nf, "vertices": m.nv, "k": args.k,
                   "select": ["kth", "adaptive-step"][args.select], "hops": args.hops},
        "windows_per_s": round(tot["processed"] / wall, 1),
        "fields_per_s": round(args.steps / wall, 3),
        "windows_per_field": round(tot["processed"] / args.steps, 1),
        "rounds_per_field": round(tot["rounds"] / args.steps, 1),
        "max_rel_err_vs_oracle": max_err,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    mesh.close()


if __name__ == "__main__":
    main()
