#!/usr/bin/env python3
"""Benchmark: exact single-source geodesic fields with PCH on one MI355X.

A step is one exact FP64 distance field on the 1024 x 1024 jittered bump grid
(2,093,058 faces, 16 seeded Gaussian bumps, anisotropic and obtuse
triangles): the first timed step starts at vertex 0, the others at seeded
random vertices. The mesh is resident in device memory before the timed
region; each step runs every phase of the method (selection, propagation,
organization, events) until the window pool is empty.

Prints one JSON line. Besides the headline (ms per field) it carries:
  roofline     - the propagation kernel's algorithmic bytes (and FP64
                 operations) per launch over its average launch time,
                 measured with HIP events on the library's stream during
                 the timed steps, against 8 TB/s (78.6 TFLOP/s FP64);
  phases       - the GPU time of each phase of the timed rounds;
  cpu_baseline - the CPU oracle (sequential ICH, one core) on a bounded
                 sample of the vertex-0 field, run in a child process that
                 starts before any GPU work;
  icosphere    - the same measurement on the bumpy icosphere with 7
                 subdivisions (327,680 faces, the face count of the paper's
                 Sphere row), the mean over 100 seeded random sources as in
                 the paper's Sphere timing;
  batched      - 512 fields (16 meshes of 14k-330k faces, 32 sources each)
                 in one persistent launch against the single-field path run
                 field after field, both with the best single-field setting
                 and with plain k-th-key selection; its roofline carries the
                 launch's counter-measured HBM bytes and FP64 operations, and
                 its cpu_baseline the oracle on all host cores (one whole
                 ICH field per mesh in a pool of processes, in the same
                 child, after the one-core sample and the GPU legs);
  learned_batched - the same 512 fields in one launch with the learned
                 cutoff (the network trained first, on the GPU, on 200 PCH
                 fields of bumpy icospheres), against the chord-length
                 ablation, the adaptive step and plain PCH field by field.

--workload icosphere and --workload batched run only that leg (for
profiling its kernels alone).

--workload learned prints a separate line for the learned selection cutoff:
the network is trained on 200 fields of bumpy icospheres and sets the
cutoffs on 1024 x 1024 bump grids, against the same rule without the
network (chord-length predictions) and the adaptive step.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# Algorithmic bytes of one propagation (Algorithm 2) per processed window:
# the window record (6 doubles, 2 ints), its 64-byte half-edge record,
# geod_dist of the face's three vertices and the corner's angle_split pair.
PROP_READ_BYTES = 56 + 64 + 24 + 16
WINDOW_BYTES = 56        # one child window written
DIST_EVENT_BYTES = 20    # vertex id, distance, incoming angle
ANGLE_EVENT_BYTES = 20   # oriented edge id, distance, crossing
# the selection's pool scan, per live window it does not select: key and
# sigma (16), half-edge and pseudo-source (8), geod_dist of the pseudo-source
# (8); a selected window's record is counted once, in PROP_READ_BYTES
SCAN_BYTES = 32
# Algorithmic FP64 operations (add, mul, div, sqrt) of Algorithm 2: the apex
# crossing, occupancy test and apex distance of a window, and the interval,
# unfolded pseudo-source, filter distances and key of each child it examines.
FLOP_PER_WINDOW = 18
FLOP_PER_CHILD = 50
# cpu_baseline sample: windows the ICH oracle propagates (about 15-25 s on one
# host core)
CPU_SAMPLE_WINDOWS = 20_000_000
GOLDEN_C3 = os.path.join(ROOT, "tests", "golden", "bump_grid1024_s2_ich.npz")
GOLDEN_C2 = os.path.join(ROOT, "tests", "golden", "icosphere7_ich.npz")


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_1305_1293_amd", "csrc", "pch_gpu.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def profile_value(name: str, key: str, config_tag: str, config_key: str = "bench_config"):
    """A per-launch figure from a committed counter summary, or None when the
    summary is missing or the kernel source or configuration changed since."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    b = re.search(r"^" + key + r":\s*([0-9.eE+]+)", text, re.M)
    cfg = re.search(r"^" + config_key + r":\s*(.+)", text, re.M)
    if not m or not b or not cfg or m.group(1) != kernel_source_hash() or cfg.group(1).strip() != config_tag:
        return None
    return float(b.group(1))


def host_cpu():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count(), "cpu_model": model}


def _ich_field_seconds(job):
    """One whole ICH field of a batch mesh (a worker of the all-core leg)."""
    from oracle import oracle as O
    i, m, s = job
    t = time.perf_counter()
    _, st = O.ich(m, [s])
    return i, time.perf_counter() - t, st["processed"]


def cpu_child(windows: int, batched: bool):
    """The CPU-baseline legs (child process, no GPU). First sequential ICH on
    one core over the first `windows` propagated windows of the bump-grid
    field from vertex 0; then, with `batched`, whole ICH fields of the batch's
    16 meshes (the first source of each) in a pool of processes over the host
    cores, leaving two cores to the GPU process; that leg waits for a line on
    stdin, which the parent writes once its GPU legs are over, so that the
    pool does not compete with them for host cores. Prints one JSON line per
    leg."""
    from oracle import oracle as O
    from paper_1305_1293_amd import meshgen as G
    m = G.config_mesh(3)
    O.lib()
    t = time.perf_counter()
    _, st = O.ich(m, [0], max_processed=windows)
    el = time.perf_counter() - t
    print(json.dumps({"seconds": el, "processed": st["processed"], **host_cpu()}), flush=True)
    if not batched:
        return
    sys.stdin.readline()  # the GPU legs are over (or the parent is gone)
    import multiprocessing as mp
    del m
    gens = G.batch_meshes(3)
    jobs = [(i, g, int(g.meta["sources"][0])) for i, g in enumerate(gens)]
    jobs.sort(key=lambda j: -j[1].nf)  # largest meshes first
    workers = max(1, min(len(jobs), len(os.sched_getaffinity(0)) - 2))
    t = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = sorted(pool.map(_ich_field_seconds, jobs, chunksize=1))
    wall = time.perf_counter() - t
    print(json.dumps({"workers": workers, "wall_s": wall, "field_s": [r[1] for r in res],
                      "processed": [r[2] for r in res], "fields_per_mesh": int(gens[0].meta["sources"].size),
                      **host_cpu()}), flush=True)


def start_cpu_child(windows: int, batched: bool):
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-child", str(windows)]
    if batched:
        cmd.append("--cpu-child-batched")
    return subprocess.Popen(cmd, stdin=subprocess.PIPE, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)


def finish_cpu_child(proc):
    out, err = proc.communicate(input="go\n", timeout=900)
    if proc.returncode != 0:
        raise RuntimeError(f"CPU-baseline child failed ({proc.returncode}): {err[-2000:]}")
    return [json.loads(x) for x in out.strip().splitlines() if x.startswith("{")]


def batched_cpu_baseline(c, batch_ms: float) -> dict:
    """The all-core oracle leg of the batch: ICH times of one field per mesh,
    scaled to the 32 fields of each mesh and spread evenly over the pool's
    processes."""
    per_mesh = np.asarray(c["field_s"]) * c["fields_per_mesh"]
    est_ms = 1000.0 * float(per_mesh.sum()) / c["workers"]
    return {"value": round(est_ms, 1), "unit": "ms", "cores": c["workers"], "kind": "oracle",
            "nproc": c["nproc"], "cpu_model": c["cpu_model"],
            "sample": f"sequential ICH, one whole field per mesh (its first source, 16 fields) in a pool of "
                      f"{c['workers']} processes: {sum(c['field_s']):.1f} s of fields in {c['wall_s']:.1f} s "
                      f"wall; value = the 512 fields (each mesh's field time x {c['fields_per_mesh']}) spread "
                      f"evenly over the {c['workers']} processes",
            "field_s_sum": round(float(sum(c["field_s"])), 2), "wall_s": round(c["wall_s"], 2),
            "gpu_speedup": round(est_ms / batch_ms, 1) if batch_ms > 0 else None}


def _timed(torch, fn):
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t, r


def batch_config_tag(opts: dict) -> str:
    return " ".join(f"{k}={int(opts[k])}" for k in ("k", "team_threads", "teams_per_cu", "hops", "gang"))


def batch_roofline(fs, seconds: float, leg: str, opts: dict) -> dict:
    """A batched launch (one dispatch of k_batch) against the HBM and FP64
    peaks. `achieved` is a lower bound of its algorithmic HBM rate: per
    processed window the propagation's reads and one window written (events,
    fans and the pool scans are not counted). `traffic` is the launch's HBM
    bytes and `fp64.counter_flop_per_launch` its issued FP64 lane operations,
    both from the committed counter summary of this kernel source and batch
    configuration (null when either changed since)."""
    processed, created = float(fs[:, 2].sum()), float(fs[:, 3].sum())
    per_window = PROP_READ_BYTES + WINDOW_BYTES
    achieved = processed * per_window / seconds / 1e9
    flops = FLOP_PER_WINDOW * processed + FLOP_PER_CHILD * created
    tag = batch_config_tag(opts)
    traffic = profile_value("k_batch_c4_traffic.md", leg + "_hbm_bytes_per_launch", tag, "bench_config_" + leg)
    cflops = profile_value("k_batch_c4_traffic.md", leg + "_fp64_flop_per_launch", tag, "bench_config_" + leg)
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_window": per_window, "lower_bound": True,
           "launch_ms": round(1000.0 * seconds, 3), "traffic": traffic,
           "traffic_gbs": round(traffic / seconds / 1e9, 1) if traffic else None,
           "traffic_frac": round(traffic / seconds / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
           "traffic_basis": "HBM bytes of the launch: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (scaled by a 512 MiB "
                            "copy), from the committed counter summary of this kernel source and options"}
    tflops = flops / seconds / 1e12
    out["fp64"] = {"bound": "fp64", "achieved": round(tflops, 4), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": round(tflops / FP64_PEAK_TFLOPS, 6), "alg_flop_per_launch": round(flops, 1),
                   "counter_flop_per_launch": cflops,
                   "counter_tflops": round(cflops / seconds / 1e12, 4) if cflops else None,
                   "counter_frac": round(cflops / seconds / 1e12 / FP64_PEAK_TFLOPS, 6) if cflops else None,
                   "counter_basis": "64 lanes x SQ_INSTS_VALU_FLOPS_FP64 of the launch (FP64 lane operations "
                                    "issued, FMA as 2), from the committed counter summary"}
    return out


def single_field_steps(pch, torch, mesh, srcs, warmup, opts, keep_first=0):
    """Warm-up fields, then the timed fields (statistics counters off), then
    the same fields again untimed with the counters on."""
    out = torch.empty(mesh.info()["nv"], dtype=torch.float64, device="cuda")
    for s in srcs[:warmup]:
        pch.geodesic(mesh, [int(s)], out=out, **opts)
    torch.cuda.synchronize()
    timed = srcs[warmup:]
    keep = []
    tot = dict(processed=0, rounds=0, ms_propagate=0.0, propagate_launches=0, timed_rounds=0)
    phase = dict(select=0.0, propagate=0.0, organize=0.0, events=0.0)
    hop_launches = 1
    t0 = time.perf_counter()
    for i, s in enumerate(timed):
        _, st = pch.geodesic(mesh, [int(s)], out=out, return_stats=True, counts=0, **opts)
        for kk in ("processed", "rounds", "ms_propagate", "propagate_launches", "timed_rounds"):
            tot[kk] += st[kk]
        for kk in phase:
            phase[kk] += st["ms_phase"][kk]
        hop_launches = st["hop_launches"]
        tot["scan_fused"] = st["scan_fused"]  # the launch plan (the same every field)
        tot["fused_workgroups"] = st["fused_workgroups"]
        if i < keep_first:
            keep.append(out.clone())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cnt = dict(processed=0, rounds=0, created=0, fan_windows=0, dist_events=0, angle_events=0, tiny=0,
               ich_dropped=0, pool_windows=0, selected=0)
    copts = dict(opts, collect_timing=0)
    for s in timed:
        _, st = pch.geodesic(mesh, [int(s)], out=out, return_stats=True, counts=1, **copts)
        for kk in cnt:
            cnt[kk] += st[kk]
    assert cnt["processed"] == tot["processed"] and cnt["rounds"] == tot["rounds"]
    tot.update({kk: cnt[kk] for kk in cnt if kk not in ("processed", "rounds")})
    return wall, tot, phase, hop_launches, keep


def roofline_of(tot, phase, hop_launches, wall, steps, traffic, counter_flops):
    kids = tot["created"] - tot["fan_windows"]
    prop_bytes = (PROP_READ_BYTES * tot["processed"] + WINDOW_BYTES * kids
                  + DIST_EVENT_BYTES * tot["dist_events"] + ANGLE_EVENT_BYTES * tot["angle_events"])
    fused_scan = tot["scan_fused"] > 0
    plan_kernel = {2: "k_select_propagate_r", 1: "k_select_propagate"}
    if fused_scan:  # the same launch scans the pool
        prop_bytes += SCAN_BYTES * (tot["pool_windows"] - tot["selected"])
    flops = FLOP_PER_WINDOW * tot["processed"] + FLOP_PER_CHILD * (kids + tot["tiny"] + tot["ich_dropped"])
    # every round launches the propagation kernel once (all hops fused) or
    # once per hop; the HIP events bracket the phases of every n-th round
    timed = max(tot["propagate_launches"], 1)
    avg_launch_s = tot["ms_propagate"] / 1000.0 / timed
    all_launches = max(tot["rounds"] * hop_launches, 1)
    bytes_per_launch = prop_bytes / all_launches
    flops_per_launch = flops / all_launches
    achieved = bytes_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    tflops = flops_per_launch / avg_launch_s / 1e12 if avg_launch_s > 0 else 0.0
    kernel = plan_kernel.get(tot["scan_fused"], "k_propagate_fused" if hop_launches == 1 else "k_propagate")
    fp64 = {"bound": "fp64", "achieved": round(tflops, 4), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tflops / FP64_PEAK_TFLOPS, 6), "alg_flop_per_launch": round(flops_per_launch, 1),
            "counter_flop_per_launch": counter_flops,
            "counter_basis": "64 lanes x SQ_INSTS_VALU_FLOPS_FP64 per launch (FP64 lane operations issued, "
                             "FMA as 2), from the committed counter summary of this kernel source"}
    # share of the timed rounds' GPU time per phase
    ptot = sum(phase.values())
    phases = {"ms_per_field": {k: round(v / max(tot["timed_rounds"], 1) * tot["rounds"] / steps, 3)
                               for k, v in phase.items()},
              "share": {k: round(v / ptot, 4) if ptot > 0 else 0.0 for k, v in phase.items()},
              "timed_rounds": tot["timed_rounds"]}
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
            "traffic_basis": "HBM bytes per launch: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (scaled by a 512 MiB "
                             "copy), from the committed counter summary of this kernel source; null when the "
                             "kernel or the configuration changed since",
            "kernel": kernel, "avg_launch_us": round(avg_launch_s * 1e6, 3),
            "alg_bytes_per_launch": round(bytes_per_launch, 1), "launches": all_launches,
            "timed_launches": tot["propagate_launches"],
            "propagate_share_of_wall": round(avg_launch_s * all_launches / wall, 4), "fp64": fp64}, phases


def measure_icosphere(args, pch, G, torch):
    """The bumpy icosphere (327,680 faces) at its own best setting, the mean
    over 100 seeded random sources (the paper's protocol for its Sphere);
    after the timed fields, the fields from the two sources of the stored
    exact ICH fields are computed with the same options and checked against
    them."""
    m = G.config_mesh(2)
    rng = np.random.default_rng(2024)
    steps = args.ico_steps
    srcs = rng.choice(m.nv, size=args.warmup + steps, replace=False).astype(np.int32)
    mesh = pch.Mesh.from_generated(m)
    opts = dict(k=16384, collect_timing=args.time_every, select_mode=1, hops=5)
    wall, tot, phase, hl, _ = single_field_steps(pch, torch, mesh, srcs, args.warmup, opts, keep_first=0)
    errs = []
    if os.path.exists(GOLDEN_C2):
        gold = np.load(GOLDEN_C2)
        hbar = float(gold["mean_edge"])
        for s, ref in zip(gold["sources"], gold["dist"]):
            d = pch.geodesic(mesh, [int(s)], **{k: v for k, v in opts.items() if k != "collect_timing"})
            errs.append(float(np.max(np.abs(d.cpu().numpy() - ref) / np.maximum(ref, hbar))))
    mesh.close()
    kernel = {2: "k_select_propagate_r", 1: "k_select_propagate"}.get(tot["scan_fused"], "k_propagate_fused")
    tag = "select=1 k=16384 hops=5 fuse_hops=1"
    traffic = profile_value(f"{kernel}_icosphere7_traffic.md", "hbm_bytes_per_launch", tag)
    cflops = profile_value(f"{kernel}_icosphere7_traffic.md", "fp64_flop_per_launch", tag)
    roof, phases = roofline_of(tot, phase, hl, wall, steps, traffic, cflops)
    return {"workload": "bumpy icosphere, 7 midpoint subdivisions, 327,680 faces, seeded random sources",
            "ms_per_field": round(1000.0 * wall / steps, 4), "steps": steps,
            "windows_per_s": round(tot["processed"] / wall, 1), "rounds_per_field": tot["rounds"] / steps,
            "options": {k: v for k, v in opts.items() if k != "collect_timing"},
            "max_rel_err_vs_oracle": max(errs) if errs else None, "roofline": roof, "phases": phases}


def measure_batched(args, pch, G, torch):
    """512 fields in one persistent launch, with the options the autotuner
    recorded for the batch's size bucket (a tuning run when it has none),
    against the single-field path run field after field: with the batch's
    own rule, k and hops, with the best single-field setting, and with plain
    k-th-key selection."""
    gens = G.batch_meshes(3)
    meshes = [pch.Mesh.from_generated(m) for m in gens]
    fm = np.repeat(np.arange(len(gens)), 32).astype(np.int32)
    fs = np.concatenate([m.meta["sources"] for m in gens]).astype(np.int32)
    if args.tune_cache and os.path.exists(args.tune_cache):
        pch.tune_cache_load(args.tune_cache)
    b = pch.Batch(meshes, fm, fs, k=32768, team_threads=512, teams_per_cu=1, hops=4, gang=8)
    out = b.empty_output()
    t0 = time.perf_counter()
    chosen, hit = b.tune_cached(out)
    tune_s = time.perf_counter() - t0
    if not hit and args.tune_cache_save:
        pch.tune_cache_save(args.tune_cache_save)
    opts = {k: chosen[k] for k in ("k", "team_threads", "teams_per_cu", "hops", "gang")}
    k_b, hops_b = int(opts["k"]), int(opts["hops"])
    out, _ = b.run(out)  # first run captures the graph and measures each field's time
    dt, (out, st) = _timed(torch, lambda: b.run(out))
    batch_ms = 1000.0 * dt
    fstats = b.field_stats()
    windows = int(fstats[:, 2].sum())
    got = out.cpu().numpy()
    ks = (4096, 8192, 16384, 32768)
    plain_ms, same_ms, best_ms, worst = 0.0, 0.0, 0.0, 0.0
    for i, (g, dm) in enumerate(zip(gens, meshes)):
        srcs = [int(x) for x in g.meta["sources"]]
        times = {k: _timed(torch, lambda: pch.geodesic(dm, [srcs[0]], k=k, select_mode=0))[0] for k in ks}
        kbest = min(times, key=times.get)
        tp = ts = tb = 0.0
        for j in (1, 2):
            t, d = _timed(torch, lambda: pch.geodesic(dm, [srcs[j]], k=kbest, select_mode=0))
            tp += t
            t, _ = _timed(torch, lambda: pch.geodesic(dm, [srcs[j]], k=k_b, select_mode=1, hops=hops_b))
            ts += t
            t, _ = _timed(torch, lambda: pch.geodesic(dm, [srcs[j]], k=16384, select_mode=1, hops=5))
            tb += t
            f = i * 32 + j
            ref = got[b.offsets[f]:b.offsets[f + 1]]
            worst = max(worst, float(np.max(np.abs(d.cpu().numpy() - ref) / np.maximum(ref, 1e-3))))
        plain_ms += 1000.0 * 32 * tp / 2
        same_ms += 1000.0 * 32 * ts / 2
        best_ms += 1000.0 * 32 * tb / 2
    b.close()
    for dm in meshes:
        dm.close()
    return {"fields": int(fm.size), "meshes": len(gens), "faces": [int(m.nf) for m in gens], "ms": round(batch_ms, 2),
            "ms_per_field": round(batch_ms / fm.size, 4), "windows_per_s": round(windows / dt, 1), "options": opts,
            "tuner": {"cache_hit": hit, "seconds": round(tune_s, 2),
                      "bucket": "largest mesh, total half-edges and field count by power of two"},
            "single_field_ms_est": {"same_rule": round(same_ms, 1), "best_setting": round(best_ms, 1),
                                    "plain_kth": round(plain_ms, 1)},
            "single_field_settings": {
                "same_rule": "adaptive step with the batch's k and hops (equal results bit for bit)",
                "best_setting": "adaptive step, k 16384, 5 hops, scan and hops in one launch per round",
                "plain_kth": "k-th-key selection, one face per round, k per mesh the fastest of 4096..32768 on "
                             "its first source"},
            "sample": "2 sources per mesh timed field by field and scaled to 32",
            "speedup": {"vs_same_rule": round(same_ms / batch_ms, 3), "vs_best_setting": round(best_ms / batch_ms, 3),
                        "vs_plain_kth": round(plain_ms / batch_ms, 3)},
            "max_rel_diff_vs_plain": worst, "roofline": batch_roofline(fstats, dt, "c4", opts)}


def measure_concurrent(pch, m, mesh, torch):
    """Fields of the same mesh computed together: 64 seeded sources in one
    batched launch whose idle workgroups share running fields; same selection
    rule, k and hops as the icosphere's single-field steps, so each field
    equals its single-field result bit for bit."""
    fs = np.random.default_rng(7).choice(m.nv, size=64, replace=False).astype(np.int32)
    opts = dict(k=12288, team_threads=512, teams_per_cu=1, hops=5, gang=16)
    b = pch.Batch([mesh], np.zeros(fs.size, np.int32), fs, **opts)
    out, _ = b.run()  # first run captures the graph and measures each field's time
    dt, (out, st) = _timed(torch, lambda: b.run(out))
    same = all(torch.equal(b.field(out, f), pch.geodesic(mesh, [int(fs[f])], k=12288, select_mode=1, hops=5))
               for f in range(8))
    fstats = b.field_stats()
    windows = int(fstats[:, 2].sum())
    b.close()
    return {"fields": int(fs.size), "ms": round(1000.0 * dt, 2), "ms_per_field": round(1000.0 * dt / fs.size, 4),
            "windows_per_s": round(windows / dt, 1), "options": opts, "reruns": int(st["reruns"]),
            "equal_to_single_field_runs": bool(same), "roofline": batch_roofline(fstats, dt, "same_mesh", opts)}


def measure_learned_batched(pch, G, Lr, mlp, torch):
    """The learned cutoff in the batched launch: the 512 fields of the batch
    workload with the network's predictions, against the same batch with the
    chord lengths (no network) and with the adaptive step, and against plain
    PCH field by field (k-th-key selection, one face per round)."""
    gens = G.batch_meshes(3)
    meshes = [pch.Mesh.from_generated(m) for m in gens]
    fm = np.repeat(np.arange(len(gens)), 32).astype(np.int32)
    fs = np.concatenate([m.meta["sources"] for m in gens]).astype(np.int32)
    opts = dict(k=32768, team_threads=512, teams_per_cu=1, hops=4, gang=8)
    res, outs = {}, {}
    for name in ("learned", "chord", "adaptive_step"):
        if name == "adaptive_step":
            b = pch.Batch(meshes, fm, fs, **opts)
        else:
            off = np.zeros(fm.size + 1, np.int64)
            off[1:] = np.cumsum([gens[i].nv for i in fm])
            # the second of two calls is timed (the first loads the kernels),
            # as the batched launch's second run is
            pred = Lr.batch_predictions(mlp, gens, fm, fs, off, chord=name == "chord")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pred = Lr.batch_predictions(mlp, gens, fm, fs, off, chord=name == "chord")
            torch.cuda.synchronize()
            tpred = time.perf_counter() - t0
            b = pch.Batch(meshes, fm, fs, predicted=pred, **opts)
        out, _ = b.run()
        dt, (out, st) = _timed(torch, lambda: b.run(out))
        res[name] = {"ms": round(1000.0 * dt, 2), "reruns": int(st["reruns"]),
                     "windows": int(b.field_stats()[:, 2].sum()), "max_rounds": int(st["max_rounds"])}
        if name != "adaptive_step":
            res[name]["predict_ms"] = round(1000.0 * tpred, 2)
        outs[name] = out.cpu().numpy()
        b.close()
    ref = outs["adaptive_step"]
    diff = max(float(np.max(np.abs(outs[n] - ref) / np.maximum(ref, 1e-3))) for n in ("learned", "chord"))
    ks = (4096, 8192, 16384, 32768)
    plain_ms = 0.0
    for g, dm in zip(gens, meshes):
        srcs = [int(x) for x in g.meta["sources"]]
        times = {k: _timed(torch, lambda: pch.geodesic(dm, [srcs[0]], k=k, select_mode=0))[0] for k in ks}
        kbest = min(times, key=times.get)
        tt = sum(_timed(torch, lambda: pch.geodesic(dm, [srcs[j]], k=kbest, select_mode=0))[0] for j in (1, 2))
        plain_ms += 1000.0 * 32 * tt / 2
    for dm in meshes:
        dm.close()
    lb = res["learned"]["ms"] + res["learned"]["predict_ms"]
    return {"fields": int(fm.size), "options": opts, "runs": res, "plain_kth_ms_est": round(plain_ms, 1),
            "learned_batched_vs_plain": round(plain_ms / lb, 3),
            "learned_batched_vs_adaptive_batched": round(res["adaptive_step"]["ms"] / lb, 3),
            "learned_vs_chord_batched": round((res["chord"]["ms"] + res["chord"]["predict_ms"]) / lb, 3),
            "max_rel_diff_vs_adaptive": diff,
            "note": "runs[...].ms is the batched launch alone; the ratios add the predictions of all 512 "
                    "fields (predict_ms) to the learned and chord launches"}


def train_network(pch, G, torch):
    """The cutoff network trained on the GPU with the library's kernels on 200
    exact fields of bumpy icospheres that PCH itself computes."""
    from paper_1305_1293_amd import learned as Lr
    train, test = G.learned_cutoff_sets(4)
    t0 = time.perf_counter()
    data, _ = Lr.build_training_set(train, k=8192)
    mlp = pch.MLP(7)
    losses = Lr.train(mlp, data, epochs=6, batch=16384, lr=2e-3, log_every=50)
    torch.cuda.synchronize()
    info = {"samples": int(data.feats.shape[0]), "seconds": round(time.perf_counter() - t0, 2),
            "loss_first": losses[0], "loss_last": losses[-1]}
    return mlp, test, info


def measure_learned(args, pch, G, torch):
    """Learned selection cutoff on the 1024 x 1024 bump grids against the same
    rule without the network and the other selection rules."""
    from paper_1305_1293_amd import learned as Lr
    mlp, test, training = train_network(pch, G, torch)
    k, hops = args.k_learned, args.hops_learned
    names = ("learned", "chord", "adaptive_step", "kth")
    rows = {n: [] for n in names}
    err = 0.0
    for g in test:
        dm = pch.Mesh.from_generated(g)
        xyz = torch.from_numpy(g.xyz).cuda()
        for s in [int(x) for x in g.meta["sources"][:args.learned_sources]]:
            runs = {
                "learned": lambda: Lr.learned_geodesic(mlp, g, dm, xyz, s, k=k, hops=hops),
                "chord": lambda: Lr.chord_geodesic(g, dm, xyz, s, k=k, hops=hops),
                "adaptive_step": lambda: pch.geodesic(dm, [s], k=k, select_mode=1, hops=hops, return_stats=True),
                "kth": lambda: pch.geodesic(dm, [s], k=k, select_mode=0, hops=hops, return_stats=True),
            }
            ref = None
            for n in names:
                t, (d, st) = _timed(torch, runs[n])
                rows[n].append((t, st["rounds"], st["processed"]))
                if ref is None:
                    ref = d.cpu().numpy()
                else:
                    err = max(err, float(np.max(np.abs(d.cpu().numpy() - ref) / np.maximum(ref, 1e-3))))
        dm.close()
    mean = {n: np.array(rows[n]).mean(axis=0) for n in names}
    ms = {n: round(1000 * float(mean[n][0]), 2) for n in names}
    batched = measure_learned_batched(pch, G, Lr, mlp, torch)
    return {"metric": "learned-cutoff vs plain speedup (ms per exact single-source field)",
            "value": round(ms["kth"] / ms["learned"], 4), "unit": "x", "higher_is_better": True,
            "n_gpus": 1, "dtype": "f64 fields, bf16/f32 network", "data": "synthetic",
            "config": {"workload": "train: 200 fields of bumpy icospheres (levels 5 and 6, 20 meshes x 10 sources); "
                                   "test: 1024 x 1024 bump grids (seeds 2, 20, 21), 2,093,058 faces",
                       "fields": len(rows["learned"]), "k": k, "hops": hops},
            "ms_per_field": ms,
            "speedup_of_learned": {n: round(ms[n] / ms["learned"], 4) for n in names if n != "learned"},
            "rounds_per_field": {n: float(mean[n][1]) for n in names},
            "windows_per_field": {n: float(mean[n][2]) for n in names},
            "max_rel_diff_vs_learned": err,
            "batched": batched,
            "training": training}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["field", "learned", "icosphere", "batched"], default="field",
                    help="field: the bench line; learned: the learned-cutoff comparison; icosphere, batched: "
                         "only that leg (for profiling its kernels alone)")
    ap.add_argument("--k", type=int, default=524288, help="windows selected per round (bump grid)")
    ap.add_argument("--select", type=int, default=1, help="0: k-th smallest key, 1: adaptive step")
    ap.add_argument("--delta0", type=float, default=0.0, help="first adaptive step (0 = 2x mean edge)")
    ap.add_argument("--hops", type=int, default=5, help="propagation hops per round")
    ap.add_argument("--fuse-hops", type=int, default=1,
                    help="1: all hops of a round in one propagation launch (hops <= 6); 0: one launch per hop")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched measurements")
    ap.add_argument("--no-icosphere", action="store_true", help="skip the icosphere measurement")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-cutoff batched leg of the bench line (training included)")
    ap.add_argument("--ico-steps", type=int, default=100, help="timed fields of the icosphere leg")
    ap.add_argument("--k-learned", type=int, default=131072, help="k of the learned-cutoff comparison")
    ap.add_argument("--hops-learned", type=int, default=5, help="hops of the learned-cutoff comparison")
    ap.add_argument("--learned-sources", type=int, default=4, help="sources per test mesh (learned workload)")
    ap.add_argument("--time-every", type=int, default=32,
                    help="time the phases of every n-th round with HIP events")
    ap.add_argument("--cpu-windows", type=int, default=CPU_SAMPLE_WINDOWS,
                    help="windows of the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1305_1293_amd", "tune_cache.txt"),
                    help="autotuner cache read before the batched measurement")
    ap.add_argument("--tune-cache-save", default="", help="write the autotuner cache here after a tuning run")
    ap.add_argument("--cpu-child", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-child-batched", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes 5 times (the reference "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters to bytes)")
    args = ap.parse_args()
    if args.cpu_child:
        cpu_child(args.cpu_child, args.cpu_child_batched)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the method's fields are "
              "independent per GPU, see the multi-GPU design notes)", file=sys.stderr)
        sys.exit(2)
    # the CPU-oracle leg runs beside the GPU legs, started before any GPU call
    child = None
    if args.workload == "field" and not args.no_cpu_baseline and args.copy_bytes == 0:
        child = start_cpu_child(args.cpu_windows, not args.no_batched)

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
    if args.workload == "icosphere":
        print(json.dumps(measure_icosphere(args, pch, G, torch)), flush=True)
        return
    if args.workload == "batched":
        mi = G.config_mesh(2)
        dmi = pch.Mesh.from_generated(mi)
        print(json.dumps({"batched": measure_batched(args, pch, G, torch),
                          "same_mesh_concurrent": measure_concurrent(pch, mi, dmi, torch)}), flush=True)
        dmi.close()
        return
    m = G.config_mesh(3)
    rng = np.random.default_rng(2024)
    pool = [int(x) for x in rng.choice(m.nv, size=args.warmup + args.steps, replace=False) if x != 0]
    srcs = pool[:args.warmup] + [0] + pool[args.warmup:args.warmup + args.steps - 1]
    mesh = pch.Mesh.from_generated(m)
    opts = dict(k=args.k, collect_timing=args.time_every, select_mode=args.select, delta0=args.delta0,
                hops=args.hops, fuse_hops=args.fuse_hops)
    print(f"bench: bump grid 1024^2, {args.steps} fields, k {args.k}, hops {args.hops}", file=sys.stderr, flush=True)
    wall, tot, phase, hop_launches, keep = single_field_steps(pch, torch, mesh, srcs, args.warmup, opts, keep_first=1)
    ms_per_field = 1000.0 * wall / args.steps
    tag = f"select={args.select} k={args.k} hops={args.hops} fuse_hops={args.fuse_hops}"
    kernel = {2: "k_select_propagate_r", 1: "k_select_propagate"}.get(
        tot["scan_fused"], "k_propagate_fused" if hop_launches == 1 else "k_propagate")
    traffic = profile_value(f"{kernel}_bump_grid1024_traffic.md", "hbm_bytes_per_launch", tag)
    cflops = profile_value(f"{kernel}_bump_grid1024_traffic.md", "fp64_flop_per_launch", tag)
    roofline, phases = roofline_of(tot, phase, hop_launches, wall, args.steps, traffic, cflops)

    # the vertex-0 field against the stored exact field (every vertex)
    max_err = None
    if os.path.exists(GOLDEN_C3):
        gold = np.load(GOLDEN_C3)
        ref = gold["dist"]
        hbar = float(gold["mean_edge"])
        got = keep[0].cpu().numpy()
        fin = np.isfinite(ref)
        assert np.array_equal(fin, np.isfinite(got)), "reachability differs from the stored field"
        max_err = float(np.max(np.abs(got[fin] - ref[fin]) / np.maximum(ref[fin], hbar)))

    print("bench: icosphere and batched legs", file=sys.stderr, flush=True)
    ico = None if args.no_icosphere else measure_icosphere(args, pch, G, torch)
    batched = None if args.no_batched else measure_batched(args, pch, G, torch)
    concurrent = None
    if not args.no_batched:
        mi = G.config_mesh(2)
        dmi = pch.Mesh.from_generated(mi)
        concurrent = measure_concurrent(pch, mi, dmi, torch)
        dmi.close()
    learned_batched = None
    if not args.no_batched and not args.no_learned:
        from paper_1305_1293_amd import learned as Lr
        print("bench: learned cutoff, batched", file=sys.stderr, flush=True)
        mlp, _, training = train_network(pch, G, torch)
        learned_batched = dict(measure_learned_batched(pch, G, Lr, mlp, torch), training=training)

    cpu = None
    if child is not None:
        legs = finish_cpu_child(child)
        c = legs[0]
        if batched is not None and len(legs) > 1:
            batched["cpu_baseline"] = batched_cpu_baseline(legs[1], batched["ms"])
        full = None
        if os.path.exists(GOLDEN_C3):
            full = int(np.load(GOLDEN_C3)["processed"])
        rate = c["processed"] / c["seconds"]
        cpu = {"value": round(1000.0 * full / rate, 1) if full else None, "unit": "ms", "cores": 1,
               "kind": "oracle", "windows_per_s": round(rate, 1), "nproc": c["nproc"], "cpu_model": c["cpu_model"],
               "sample": f"sequential ICH on one core, the vertex-0 field of the same mesh stopped after its first "
                         f"{c['processed']:,} propagated windows ({c['seconds']:.1f} s); value = the full field's "
                         f"{full:,} ICH windows at the sample's rate" if full else "no stored full-field count"}

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
        "config": {"workload": "1024 x 1024 jittered bump grid (16 Gaussian bumps, seed 2), 2,093,058 faces; the "
                               "first timed field from vertex 0, the others from seeded random vertices",
                   "faces": m.nf, "vertices": m.nv, "k": args.k,
                   "select": ["kth", "adaptive-step"][args.select], "hops": args.hops,
                   "propagation_launches_per_round": hop_launches,
                   "propagation_workgroups": tot["fused_workgroups"]},
        "windows_per_s": round(tot["processed"] / wall, 1),
        "fields_per_s": round(args.steps / wall, 3),
        "windows_per_field": round(tot["processed"] / args.steps, 1),
        "rounds_per_field": round(tot["rounds"] / args.steps, 1),
        "max_rel_err_vs_oracle": max_err,
        "roofline": roofline,
        "phases": phases,
        "cpu_baseline": cpu,
        "icosphere": ico,
        "batched": batched,
        "same_mesh_concurrent": concurrent,
        "learned_batched": learned_batched,
    }
    print(json.dumps(line), flush=True)
    mesh.close()


if __name__ == "__main__":
    main()
