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
                 first GPU fields;
  batched      - 512 fields (16 meshes of 20k-330k faces, 32 sources each)
                 in one persistent launch against plain PCH (k-th-key
                 selection, one face per round, k tuned per mesh) run field
                 after field on a sample of the same fields.

--workload learned prints a separate line for the learned selection cutoff:
the network is trained on 200 fields of bumpy icospheres and sets the
cutoffs on 1024 x 1024 bump grids, against plain PCH on the same fields.
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


def traffic_from_profile(kernel: str, workload_tag: str, config_tag: str):
    """HBM bytes per propagation launch from the committed counter summary, or
    None when the summary is missing or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload_tag}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    cfg = re.search(r"bench_config:\s*(.+)", text)
    if not m or not b or not cfg or m.group(1) != kernel_source_hash() or cfg.group(1).strip() != config_tag:
        return None
    return float(b.group(1))



def _timed(torch, fn):
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t, r


def batch_roofline(windows_per_s: float) -> dict:
    """Lower bound of a batched launch's algorithmic HBM rate: per processed
    window the propagation's reads and one window written (events, fans and
    the pool scans are not counted)."""
    per_window = PROP_READ_BYTES + WINDOW_BYTES
    achieved = windows_per_s * per_window / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_window": per_window, "lower_bound": True}


def measure_batched(pch, G, torch):
    """512 fields in one persistent launch against plain PCH field by field."""
    gens = G.batch_meshes(3)
    meshes = [pch.Mesh.from_generated(m) for m in gens]
    fm = np.repeat(np.arange(len(gens)), 32).astype(np.int32)
    fs = np.concatenate([m.meta["sources"] for m in gens]).astype(np.int32)
    opts = dict(k=32768, team_threads=512, teams_per_cu=1, hops=4, gang=8)
    b = pch.Batch(meshes, fm, fs, **opts)
    out, _ = b.run()  # first run captures the graph and measures each field's time
    dt, (out, st) = _timed(torch, lambda: b.run(out))
    batch_ms = 1000.0 * dt
    windows = int(b.field_stats()[:, 2].sum())
    got = out.cpu().numpy()
    ks = (4096, 8192, 16384, 32768)
    plain_ms, worst = 0.0, 0.0
    for i, (g, dm) in enumerate(zip(gens, meshes)):
        srcs = [int(x) for x in g.meta["sources"]]
        times = {k: _timed(torch, lambda: pch.geodesic(dm, [srcs[0]], k=k, select_mode=0))[0] for k in ks}
        kbest = min(times, key=times.get)
        tt = 0.0
        for j in (1, 2):
            t, d = _timed(torch, lambda: pch.geodesic(dm, [srcs[j]], k=kbest, select_mode=0))
            tt += t
            f = i * 32 + j
            ref = got[b.offsets[f]:b.offsets[f + 1]]
            worst = max(worst, float(np.max(np.abs(d.cpu().numpy() - ref) / np.maximum(ref, 1e-3))))
        plain_ms += 1000.0 * 32 * tt / 2
    b.close()
    for dm in meshes:
        dm.close()
    return {"fields": int(fm.size), "meshes": len(gens), "faces": [int(m.nf) for m in gens], "ms": round(batch_ms, 2),
            "ms_per_field": round(batch_ms / fm.size, 4), "windows_per_s": round(windows / dt, 1), "options": opts,
            "plain_ms_est": round(plain_ms, 1),
            "plain": "k-th-key selection, one face per round, k per mesh the fastest of 4096..32768 on its first "
                     "source; 2 more sources per mesh timed and scaled to 32",
            "speedup_vs_plain": round(plain_ms / batch_ms, 3), "max_rel_diff_vs_plain": worst,
            "roofline": batch_roofline(windows / dt)}


def measure_concurrent(args, pch, m, mesh, srcs, keep, torch):
    """Fields of the same mesh computed together: 64 sources (the timed ones
    first) in one batched launch whose idle workgroups share running fields;
    same selection rule, k and hops as the single-field steps, so each field
    equals its single-field result bit for bit."""
    extra = np.setdiff1d(np.random.default_rng(7).choice(m.nv, size=128, replace=False), srcs)
    fs = np.concatenate([srcs[args.warmup:], extra])[:64].astype(np.int32)
    opts = dict(k=args.k, team_threads=512, teams_per_cu=1, hops=args.hops, gang=16)
    b = pch.Batch([mesh], np.zeros(fs.size, np.int32), fs, **opts)
    out, _ = b.run()  # first run captures the graph and measures each field's time
    dt, (out, st) = _timed(torch, lambda: b.run(out))
    same = all(torch.equal(b.field(out, f), keep[f]) for f in range(min(len(keep), fs.size)))
    windows = int(b.field_stats()[:, 2].sum())
    b.close()
    return {"fields": int(fs.size), "ms": round(1000.0 * dt, 2), "ms_per_field": round(1000.0 * dt / fs.size, 4),
            "windows_per_s": round(windows / dt, 1), "options": opts, "reruns": int(st["reruns"]),
            "equal_to_single_field_runs": bool(same), "roofline": batch_roofline(windows / dt)}


def measure_learned(args, pch, G, torch):
    """Learned selection cutoff against plain PCH on the 1024 x 1024 bump grids."""
    from paper_1305_1293_amd import learned as Lr
    train, test = G.learned_cutoff_sets(4)
    t0 = time.perf_counter()
    data, _ = Lr.build_training_set(train, k=8192)
    mlp = pch.MLP(7)
    losses = Lr.train(mlp, data, epochs=6, batch=16384, lr=2e-3, log_every=50)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    k = args.k_learned
    rows = []
    for g in test:
        dm = pch.Mesh.from_generated(g)
        xyz = torch.from_numpy(g.xyz).cuda()
        for s in [int(x) for x in g.meta["sources"][:args.learned_sources]]:
            tp, (dp, sp) = _timed(torch, lambda: pch.geodesic(dm, [s], k=k, select_mode=0, return_stats=True))
            tl, (dl, sl) = _timed(torch, lambda: Lr.learned_geodesic(mlp, g, dm, xyz, s, k=k))
            td, (dd, sd) = _timed(torch, lambda: pch.geodesic(dm, [s], k=k, select_mode=1, return_stats=True))
            ref = dp.cpu().numpy()
            err = float(np.max(np.abs(dl.cpu().numpy() - ref) / np.maximum(ref, 1e-3)))
            rows.append((tp, tl, td, sp["rounds"], sl["rounds"], sd["rounds"], sp["processed"], sl["processed"], err))
        dm.close()
    a = np.array(rows)
    plain_ms, learned_ms, step_ms = 1000 * a[:, 0].mean(), 1000 * a[:, 1].mean(), 1000 * a[:, 2].mean()
    return {"metric": "learned-cutoff vs plain speedup (ms per exact single-source field)",
            "value": round(plain_ms / learned_ms, 4), "unit": "x", "higher_is_better": True,
            "n_gpus": 1, "dtype": "f64 fields, bf16/f32 network", "data": "synthetic",
            "config": {"workload": "train: 200 fields of bumpy icospheres (levels 5 and 6, 20 meshes x 10 sources); "
                                   "test: 1024 x 1024 bump grids (seeds 2, 20, 21), 2,093,058 faces",
                       "fields": len(rows), "k": k, "hops": 1},
            "ms_per_field": {"plain_kth": round(plain_ms, 2), "learned": round(learned_ms, 2),
                             "adaptive_step": round(step_ms, 2)},
            "rounds_per_field": {"plain_kth": float(a[:, 3].mean()), "learned": float(a[:, 4].mean()),
                                 "adaptive_step": float(a[:, 5].mean())},
            "windows_per_field": {"plain_kth": float(a[:, 6].mean()), "learned": float(a[:, 7].mean())},
            "max_rel_diff_learned_vs_plain": float(a[:, 8].max()),
            "training": {"samples": int(data.feats.shape[0]), "seconds": round(train_s, 2),
                         "loss_first": losses[0], "loss_last": losses[-1]}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["field", "learned"], default="field")
    ap.add_argument("--k", type=int, default=12288, help="windows selected per round")
    ap.add_argument("--select", type=int, default=1, help="0: k-th smallest key, 1: adaptive step")
    ap.add_argument("--delta0", type=float, default=0.0, help="first adaptive step (0 = 2x mean edge)")
    ap.add_argument("--hops", type=int, default=5, help="propagation hops per round")
    ap.add_argument("--fuse-hops", type=int, default=1,
                    help="1: all hops of a round in one propagation launch (hops <= 6); 0: one launch per hop")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-versus-plain measurement")
    ap.add_argument("--k-learned", type=int, default=131072, help="k of the learned-cutoff comparison")
    ap.add_argument("--learned-sources", type=int, default=4, help="sources per test mesh (learned workload)")
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
    if args.workload == "learned":
        print(json.dumps(measure_learned(args, pch, G, torch)), flush=True)
        return
    m = G.config_mesh(2)
    rng = np.random.default_rng(2024)
    srcs = rng.choice(m.nv, size=args.warmup + args.steps, replace=False).astype(np.int32)
    mesh = pch.Mesh.from_generated(m)
    out = torch.empty(m.nv, dtype=torch.float64, device="cuda")
    opts = dict(k=args.k, collect_timing=args.time_every, select_mode=args.select, delta0=args.delta0, hops=args.hops,
                fuse_hops=args.fuse_hops)

    for i in range(args.warmup):
        pch.geodesic(mesh, [int(srcs[i])], out=out, **opts)
    torch.cuda.synchronize()

    keep = []
    tot = dict(processed=0, rounds=0, ms_propagate=0.0, propagate_launches=0)
    hop_launches = None
    t0 = time.perf_counter()
    for i in range(args.steps):
        # the statistics counters (windows created, events) stay off in the
        # timed fields, as in a plain call; they are taken below
        _, st = pch.geodesic(mesh, [int(srcs[args.warmup + i])], out=out, return_stats=True, counts=0, **opts)
        for kk in tot:
            tot[kk] += st[kk]
        hop_launches = st["hop_launches"]
        if len(keep) < 8:
            keep.append(out.clone())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ms_per_field = 1000.0 * wall / args.steps
    # the same fields again, untimed, with the counters on (the method is
    # deterministic: same rounds, windows and events)
    cnt = dict(processed=0, rounds=0, created=0, fan_windows=0, dist_events=0, angle_events=0)
    copts = dict(opts, collect_timing=0)
    for i in range(args.steps):
        _, st = pch.geodesic(mesh, [int(srcs[args.warmup + i])], out=out, return_stats=True, counts=1, **copts)
        for kk in cnt:
            cnt[kk] += st[kk]
    assert cnt["processed"] == tot["processed"] and cnt["rounds"] == tot["rounds"]
    tot.update({kk: cnt[kk] for kk in ("created", "fan_windows", "dist_events", "angle_events")})

    kids = tot["created"] - tot["fan_windows"]
    prop_bytes = (PROP_READ_BYTES * tot["processed"] + WINDOW_BYTES * kids
                  + DIST_EVENT_BYTES * tot["dist_events"] + ANGLE_EVENT_BYTES * tot["angle_events"])
    # every round launches the propagation kernel once (all hops fused) or
    # once per hop; the HIP events bracket the launches of every n-th round
    timed = max(tot["propagate_launches"], 1)
    avg_launch_s = tot["ms_propagate"] / 1000.0 / timed
    all_launches = max(tot["rounds"] * hop_launches, 1)
    bytes_per_launch = prop_bytes / all_launches
    achieved = bytes_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    kernel = "k_propagate_fused" if hop_launches == 1 else "k_propagate"
    traffic = traffic_from_profile(kernel, "icosphere7", f"select={args.select} k={args.k} hops={args.hops} "
                                                        f"fuse_hops={args.fuse_hops}")
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": kernel, "avg_launch_us": round(avg_launch_s * 1e6, 3),
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

    batched = None if args.no_batched else measure_batched(pch, G, torch)
    concurrent = None if args.no_batched or args.select != 1 else measure_concurrent(args, pch, m, mesh, srcs, keep,
                                                                                       torch)

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
                   "select": ["kth", "adaptive-step"][args.select], "hops": args.hops,
                   "propagation_launches_per_round": hop_launches},
        "windows_per_s": round(tot["processed"] / wall, 1),
        "fields_per_s": round(args.steps / wall, 3),
        "windows_per_field": round(tot["processed"] / args.steps, 1),
        "rounds_per_field": round(tot["rounds"] / args.steps, 1),
        "max_rel_err_vs_oracle": max_err,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched": batched,
        "same_mesh_concurrent": concurrent,
    }
    print(json.dumps(line), flush=True)
    mesh.close()


if __name__ == "__main__":
    main()
