"""GPU parity: the HIP path through the C ABI against the CPU oracle.

* distances: within 1e-9 relative (|gpu - oracle| <= 1e-9 * max(oracle, mean
  edge length)) of ICH on every vertex, and the closed forms;
* bookkeeping: per-round integer records (pool size, cutoff, selected,
  stale, children, drops, events, fans) identical to the round-based replica
  with the same k, and the distance bit patterns identical to it;
* full size: the bumpy icosphere against live ICH on every vertex and the
  1024^2 bump grid against its stored exact ICH field on every vertex, at the
  benchmark's setting, with the adaptive step below the pool size and with
  plain k-th-key selection.
"""
import os
import sys

import numpy as np
import pytest

from paper_1305_1293_amd import meshgen as G

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1305_1293_amd import pch as P
    P.lib()
    return P


def gpu_field(pch, m, sources, **opts):
    dm = pch.Mesh.from_generated(m)
    d, st = pch.geodesic(dm, sources, return_stats=True, **opts)
    import torch
    torch.cuda.synchronize()
    log = dm.round_log() if opts.get("collect_stats") else None
    out = d.cpu().numpy()
    dm.close()
    return out, st, log


def mean_edge(oracle, m):
    return float(oracle.lengths(m).mean())


def assert_close(gpu, ref, hbar, tol=1e-9, what=""):
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(gpu)), f"{what}: reachability differs"
    err = np.abs(gpu[fin] - ref[fin]) / np.maximum(ref[fin], hbar)
    assert err.max() <= tol, f"{what}: max rel err {err.max():.3e} at vertex {np.nonzero(fin)[0][np.argmax(err)]}"


# ---------------------------------------------------------------------------
# closed forms and the small configuration
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 64, 1 << 30])
def test_closed_forms(pch, oracle, k):
    from test_oracle_closed_form import cone_expect, cube_corner_expect, lshape_expect
    cases = []
    m = G.jittered_plane(12, 0)
    cases.append((m, 5, np.linalg.norm(m.xyz - m.xyz[5], axis=1)))
    m = G.lshape(6)
    s = int(np.argmin(np.linalg.norm(m.xyz[:, :2] - [2.0, 0.0], axis=1)))
    cases.append((m, s, lshape_expect(m)))
    m = G.cube(4)
    cases.append((m, int(np.argmin(np.linalg.norm(m.xyz, axis=1))), cube_corner_expect(m.xyz)))
    for ns in (7, 5):
        m = G.cone_fan(ns, 4)
        cases.append((m, 5, cone_expect(m.meta["polar"], m.meta["total_angle"], 5)))
    for m, s, exp in cases:
        say(f"closed form {m.name} source {s} k {k}")
        d, st, _ = gpu_field(pch, m, [s], k=k)
        assert np.max(np.abs(d - exp)) <= 1e-12 * max(1.0, exp.max()), m.name


@pytest.mark.parametrize("k", [64, 1024, 65536])
def test_small_config_vs_ich(pch, oracle, k):
    m = G.config_mesh(1)
    say(f"sinusoid grid 64 vs ICH, k {k}")
    ref, _ = oracle.ich(m, [0])
    d, st, _ = gpu_field(pch, m, [0], k=k)
    assert_close(d, ref, mean_edge(oracle, m), what=f"k={k}")
    assert st["rounds"] > 0 and st["processed"] > 0


@pytest.mark.parametrize("case", [("sinusoid64", 0, 64), ("sinusoid64", 0, 1024), ("sphere4", 17, 512),
                                  ("lshape", -1, 16), ("cone7", 5, 8), ("grid48", 100, 4096),
                                  ("sinusoid64", 0, 1024, 0.02), ("sphere4", 17, 512, 0.05),
                                  ("grid48", 100, 2048, 0.01),
                                  ("sinusoid64", 0, 256, None, 3), ("sphere4", 17, 1 << 20, None, 4),
                                  ("lshape", -1, 16, None, 16), ("cone7", 5, 64, None, 2),
                                  ("grid48", 100, 2048, 0.01, 4), ("sinusoid64", 0, 1024, 0.02, 8),
                                  ("cube6", -2, 64), ("plane15", 112, 32), ("plane15", 112, 256, None, 4),
                                  ("cube6", -2, 512, 0.05, 3)])
def test_round_log_matches_replica(pch, oracle, case):
    name, s, k = case[:3]
    delta0 = case[3] if len(case) > 3 else None
    hops = case[4] if len(case) > 4 else 1
    sel = dict(mode=1, delta0=delta0) if delta0 else {}
    gsel = dict(select_mode=1, delta0=delta0) if delta0 else {}
    sel["hops"] = gsel["hops"] = hops
    m = {"sinusoid64": lambda: G.config_mesh(1), "sphere4": lambda: G.bumpy_icosphere(4, seed=9),
         "lshape": lambda: G.lshape(6), "cone7": lambda: G.cone_fan(7, 6),
         "grid48": lambda: G.bump_grid(48, seed=4), "cube6": lambda: G.cube(6),
         "plane15": lambda: G.jittered_plane(15, 0, jitter=0.0)}[name]()
    if s == -2:  # a cube corner: symmetric paths tie exactly
        s = int(np.argmin(np.linalg.norm(m.xyz, axis=1)))
    elif s < 0:
        s = int(np.argmin(np.linalg.norm(m.xyz[:, :2] - [2.0, 0.0], axis=1)))
    say(f"round log parity {name} source {s} k {k} delta0 {delta0} hops {hops}")
    dr, st_r, log_r = oracle.replica(m, [s], k, **sel)
    d, st, log = gpu_field(pch, m, [s], k=k, collect_stats=1, **gsel)
    assert log.shape == log_r.shape, f"rounds: gpu {log.shape[0]} replica {log_r.shape[0]}"
    bad = np.nonzero(np.any(log != log_r, axis=1))[0]
    assert bad.size == 0, f"first differing round {bad[0]}: gpu {log[bad[0]].tolist()} replica {log_r[bad[0]].tolist()}"
    assert np.array_equal(d.view(np.uint64), dr.view(np.uint64)), "distance bits differ from the replica"
    ref, _ = oracle.ich(m, [s])
    assert_close(d, ref, mean_edge(oracle, m), what=name)


@pytest.mark.parametrize("hops", [1, 4])
def test_organize_by_edge_changes_nothing(pch, oracle, hops):
    """Grouping the selected windows by edge only reorders them: the per-round
    records and the distance bits equal the unorganized run and the replica."""
    for m, s, kw in [(G.config_mesh(1), 0, dict(k=1024)), (G.bumpy_icosphere(4, seed=9), 17, dict(k=512)),
                     (G.bump_grid(48, seed=4), 100, dict(k=2048, select_mode=1, delta0=0.01))]:
        say(f"organize by edge {m.name} source {s} {kw} hops {hops}")
        d0, _, log0 = gpu_field(pch, m, [s], collect_stats=1, hops=hops, **kw)
        d1, _, log1 = gpu_field(pch, m, [s], collect_stats=1, hops=hops, organize=1, **kw)
        assert np.array_equal(log0, log1)
        assert np.array_equal(d0.view(np.uint64), d1.view(np.uint64))
        rkw = dict(k=kw["k"], hops=hops)
        if "select_mode" in kw:
            rkw.update(mode=1, delta0=kw["delta0"])
        dr, _, log_r = oracle.replica(m, [s], **rkw)
        assert np.array_equal(log1, log_r)


@pytest.mark.parametrize("k,hops", [(64, 1), (1024, 1), (1024, 4)])
def test_strided_selection_exact(pch, oracle, k, hops):
    """The paper's approximate (strided) selection changes which windows a
    round takes, not the distances: every vertex within 1e-9 of ICH; the
    round log marks its rounds (shift -5), and such a round takes at most
    one window per thread of its scan and no further hop."""
    for m, s in [(G.config_mesh(1), 0), (G.bumpy_icosphere(4, seed=9), 17), (G.bump_grid(48, seed=4), 100),
                 (G.cone_fan(7, 5), 5)]:
        say(f"strided selection {m.name} source {s} k {k} hops {hops}")
        d, st, log = gpu_field(pch, m, [s], k=k, hops=hops, select_mode=pch.PCH_SELECT_STRIDED, collect_stats=1)
        ref, _ = oracle.ich(m, [s])
        assert_close(d, ref, mean_edge(oracle, m), what=f"{m.name} strided k={k}")
        strided = log[:, 2] == -5
        if (log[:, 0] > k).any():
            assert strided.any()
        threads = ((k + 255) // 256) * 256
        assert np.all(log[strided, 3] <= threads)


def test_counts_off_changes_no_result(pch):
    """Without the statistics counters the rounds, the processed windows and
    the distance bits are those of a run with them; the skipped counts read 0."""
    import torch
    for m, s, kw in [(G.bumpy_icosphere(4, seed=9), 17, dict(k=512, hops=4)),
                     (G.bump_grid(48, seed=4), 100, dict(k=2048, select_mode=1, hops=1))]:
        say(f"counts off {m.name} source {s} {kw}")
        dm = pch.Mesh.from_generated(m)
        d1, s1 = pch.geodesic(dm, [s], return_stats=True, counts=1, **kw)
        d0, s0 = pch.geodesic(dm, [s], return_stats=True, counts=0, **kw)
        torch.cuda.synchronize()
        assert torch.equal(d0, d1)
        assert (s0["rounds"], s0["processed"]) == (s1["rounds"], s1["processed"])
        assert s1["created"] > 0 and s0["created"] == 0 and s0["dist_events"] == 0
        dm.close()


@pytest.mark.parametrize("hops", [2, 4, 6])
def test_fused_hops_equal_per_hop_launches(pch, hops):
    """All hops of a round in one launch (hop lists in LDS, depth first) and
    one launch per hop propagate the same windows at the same hops: per-round
    records, statistics and distance bits are equal. k = 2^20 selects whole
    pools, so the lists see their largest fills."""
    import torch
    for m, s, kw in [(G.config_mesh(1), 0, dict(k=1024)), (G.bumpy_icosphere(4, seed=9), 17, dict(k=1 << 20)),
                     (G.bump_grid(48, seed=4), 100, dict(k=2048, select_mode=1, delta0=0.01)),
                     (G.bumpy_icosphere(5, seed=3), 5, dict(k=16384, select_mode=1)),
                     (G.bump_grid(64, seed=12), 0, dict(k=256, select_mode=4))]:
        say(f"fused hops {hops} {m.name} source {s} {kw}")
        d0, s0, log0 = gpu_field(pch, m, [s], collect_stats=1, hops=hops, fuse_hops=0, **kw)
        d1, s1, log1 = gpu_field(pch, m, [s], collect_stats=1, hops=hops, fuse_hops=1, **kw)
        torch.cuda.synchronize()
        assert s0["hop_launches"] == hops and s1["hop_launches"] == 1
        assert s0["restarts"] == 0 and s1["restarts"] == 0
        if kw.get("select_mode") != 4:  # the strided selection depends on the pool's layout
            assert np.array_equal(log0, log1)
            assert np.array_equal(d0.view(np.uint64), d1.view(np.uint64))
            for key in ("rounds", "processed", "created", "dist_events", "angle_events", "fans", "fan_windows"):
                assert s0[key] == s1[key], key
        else:
            hbar = float(np.mean(np.linalg.norm(m.xyz[m.faces[:, 0]] - m.xyz[m.faces[:, 1]], axis=1)))
            assert np.max(np.abs(d0 - d1) / np.maximum(d0, hbar)) <= 1e-9


@pytest.mark.parametrize("case", [("sinusoid64", 0, 1024, 1), ("sphere5", 5, 4096, 4), ("grid64", 0, 1024, 5),
                                  ("sphere5", 5, 4096, 8)])
def test_propagation_retest_matches_replica(pch, oracle, case):
    """Stronger filtering (filters bit 3) on the GPU: the per-round records and
    distance bits equal the replica with the same option, the distances ICH's."""
    name, s, k, hops = case
    m = {"sinusoid64": lambda: G.config_mesh(1), "sphere5": lambda: G.bumpy_icosphere(5, seed=3),
         "grid64": lambda: G.bump_grid(64, seed=12)}[name]()
    hbar = mean_edge(oracle, m)
    kw = dict(mode=1, delta0=2 * hbar) if name != "sinusoid64" else {}
    gkw = dict(select_mode=1, delta0=2 * hbar) if name != "sinusoid64" else {}
    say(f"retest {name} source {s} k {k} hops {hops}")
    dr, _, log_r = oracle.replica(m, [s], k, filters=11, hops=hops, **kw)
    d, st, log = gpu_field(pch, m, [s], k=k, collect_stats=1, filters=11, hops=hops, **gkw)
    assert log.shape == log_r.shape
    bad = np.nonzero(np.any(log != log_r, axis=1))[0]
    assert bad.size == 0, f"first differing round {bad[0]}: gpu {log[bad[0]].tolist()} replica {log_r[bad[0]].tolist()}"
    assert np.array_equal(d.view(np.uint64), dr.view(np.uint64))
    ref, _ = oracle.ich(m, [s])
    assert_close(d, ref, hbar, what=name)


def test_grazing_boundary_regression(pch, oracle):
    m = G.bump_grid(96, seed=23)
    say("bump grid 96 seed 23 (grazing convex boundary)")
    ref, _ = oracle.ich(m, [0])
    assert np.isfinite(ref).all()
    for mode in (0, 1):
        d, _, _ = gpu_field(pch, m, [0], k=4096, select_mode=mode)
        assert_close(d, ref, mean_edge(oracle, m), what=f"mode {mode}")


def test_multi_source_min(pch, oracle):
    m = G.config_mesh(1)
    srcs = [0, 1000, 4095, 1000]
    say("multi-source min field")
    ref, _ = oracle.ich(m, srcs)
    d, _, _ = gpu_field(pch, m, srcs, k=2048)
    assert_close(d, ref, mean_edge(oracle, m), what="multi-source")


def test_pool_overflow_restarts_with_same_result(pch, oracle):
    m = G.config_mesh(1)
    say("pool overflow restart")
    d0, st0, log0 = gpu_field(pch, m, [0], k=512, collect_stats=1)
    d1, st1, log1 = gpu_field(pch, m, [0], k=512, collect_stats=1, pool_capacity=600)
    assert st1["restarts"] >= 1
    assert np.array_equal(d0.view(np.uint64), d1.view(np.uint64))
    assert np.array_equal(log0, log1)


def test_pool_limit_reports_overflow(pch):
    m = G.config_mesh(1)
    dm = pch.Mesh.from_generated(m)
    with pytest.raises(pch.PchError) as e:
        pch.geodesic(dm, [0], k=512, pool_capacity=256, pool_limit=512)
    assert e.value.code == -5
    dm.close()


def test_argument_errors(pch):
    m = G.config_mesh(1)
    dm = pch.Mesh.from_generated(m)
    for bad in ([-1], [m.nv]):
        with pytest.raises(pch.PchError) as e:
            pch.geodesic(dm, bad)
        assert e.value.code == -1
    with pytest.raises(pch.PchError) as e:
        pch.geodesic(dm, [0], k=0)
    assert e.value.code == -1
    for hops in (-1, 17):
        with pytest.raises(pch.PchError) as e:
            pch.geodesic(dm, [0], hops=hops)
        assert e.value.code == -1
    info = dm.info()
    assert info["nv"] == m.nv and info["nf"] == m.nf and info["n_boundary_he"] == 4 * 63
    dm.close()


def test_vertex_tables_match_oracle(pch, oracle):
    for m in (G.config_mesh(1), G.cone_fan(7, 3), G.cube(3)):
        dm = pch.Mesh.from_generated(m)
        th, fl = dm.vertex_tables()
        inf = oracle.mesh_info(m)
        assert np.array_equal(th.view(np.uint64), inf["theta"].view(np.uint64)), m.name
        assert np.array_equal(fl, inf["flags"]), m.name
        dm.close()


def test_random_cutoff_table(pch, oracle):
    m = G.config_mesh(1)
    rng = np.random.default_rng(11)
    cut = np.cumsum(rng.uniform(0.0, 0.05, 200))
    say("cutoff table")
    dr, _, log_r = oracle.replica(m, [0], 64, cutoffs=cut)
    d, st, log = gpu_field(pch, m, [0], k=64, cutoff_table=cut, collect_stats=1)
    assert np.array_equal(log, log_r)
    assert np.array_equal(d.view(np.uint64), dr.view(np.uint64))


def test_filters_off_and_full_fan_same_distances(pch, oracle):
    m = G.sinusoid_grid(24, 1)
    ref, _ = oracle.ich(m, [7])
    for f in (0, 1, 2, 7):
        say(f"filters {f}")
        d, _, _ = gpu_field(pch, m, [7], k=256, filters=f)
        assert_close(d, ref, mean_edge(oracle, m), tol=1e-12, what=f"filters {f}")


# ---------------------------------------------------------------------------
# full-size configurations
# ---------------------------------------------------------------------------

def test_full_size_bumpy_icosphere_all_vertices(pch, oracle):
    m = G.config_mesh(2)
    s = m.meta["source"]
    say(f"bumpy icosphere level 7 (327,680 faces) source {s}")
    ref, _ = oracle.ich(m, [s])
    d, st, _ = gpu_field(pch, m, [s], k=16384)
    assert_close(d, ref, mean_edge(oracle, m), what="icosphere L7")
    say(f"  rounds {st['rounds']} processed {st['processed']}")
    # the launch configuration of the bench line's icosphere object: adaptive
    # step, k = 16384, 5 hops, scan and hops in one launch per round
    d, st, _ = gpu_field(pch, m, [s], k=16384, select_mode=1, hops=5)
    assert st["hop_launches"] == 1 and st["scan_fused"] == 2
    # the 5-hop launch holds three workgroups per compute unit (LDS and
    # registers both allow three)
    import torch
    assert st["fused_workgroups"] == 3 * torch.cuda.get_device_properties(0).multi_processor_count
    assert_close(d, ref, mean_edge(oracle, m), what="icosphere L7, adaptive step, 5 hops")
    say(f"  adaptive step, 5 hops: rounds {st['rounds']} processed {st['processed']}")


@pytest.fixture(scope="module")
def bump_grid_gold():
    path = os.path.join(HERE, "golden", "bump_grid1024_s2_ich.npz")
    gold = np.load(path)
    m = G.config_mesh(3)
    assert m.nv == int(gold["nv"]) and m.nf == int(gold["nf"])
    return m, gold


@pytest.mark.parametrize("setting", [
    # the timed benchmark's launch configuration: adaptive step, k = 524288,
    # 5 hops, the pool scan and all hops in one launch per round
    dict(k=524288, select_mode=1, hops=5),
    # the adaptive step below the pool size (the cutoff decides)
    dict(k=131072, select_mode=1, hops=4, fuse_scan=0),
    # plain k-th-key selection, one face per round
    dict(k=1 << 17, select_mode=0, hops=1),
])
def test_full_size_bump_grid_every_vertex(pch, oracle, bump_grid_gold, setting):
    m, gold = bump_grid_gold
    s = int(gold["source"])
    say(f"bump grid 1024^2 (2,093,058 faces) source {s} {setting}")
    d, st, _ = gpu_field(pch, m, [s], **setting)
    # every vertex against the stored exact field
    assert_close(d, gold["dist"], float(gold["mean_edge"]), what=f"bump grid {setting}")
    # properties at every vertex
    he = oracle.lengths(m)
    a = m.faces.reshape(-1)
    b = np.roll(m.faces, -1, axis=1).reshape(-1)
    assert np.all(np.abs(d[a] - d[b]) <= he * (1 + 1e-12) + 1e-15)
    chord = np.linalg.norm(m.xyz - m.xyz[s], axis=1)
    assert np.all(d >= chord * (1 - 1e-12))
    say(f"  rounds {st['rounds']} processed {st['processed']}")


def test_round_graph_replays_equal_launch_by_launch(pch, oracle):
    """round_graph: rounds enqueued as one captured HIP graph, replayed across
    fields with other eager work in between, give the same bits as launch by
    launch."""
    import torch
    m = G.config_mesh(1)
    dm = pch.Mesh.from_generated(m)
    ref = {s: pch.geodesic(dm, [s], k=1024, select_mode=1, hops=4).cpu().numpy() for s in (0, 77, 1234)}
    for rep in range(3):
        for s in (0, 77, 1234):
            say(f"round graph replay {rep} source {s}")
            d = pch.geodesic(dm, [s], k=1024, select_mode=1, hops=4, round_graph=1)
            torch.cuda.synchronize()
            assert np.array_equal(d.cpu().numpy().view(np.uint64), ref[s].view(np.uint64)), (rep, s)
            pch.geodesic(dm, [5], k=64, select_mode=0)  # eager work between the replays
    d_ich, _ = oracle.ich(m, [77])
    assert np.max(np.abs(ref[77] - d_ich) / np.maximum(d_ich, mean_edge(oracle, m))) <= 1e-9
    dm.close()


@pytest.mark.parametrize("hops", [1, 5])
def test_degenerate_inputs_gpu(pch, oracle, hops):
    """Two components (the one without a source stays +inf, with both sources
    each component takes its own field), a single triangle from each corner,
    and a repeated source: every field equals ICH at every vertex."""
    from test_oracle_invariants import _two_components
    m, na = _two_components()
    hbar = mean_edge(oracle, m)
    for srcs in ([3], [3, na + 7], [na + 7, na + 7]):
        say(f"two components, sources {srcs}, hops {hops}")
        d, st, _ = gpu_field(pch, m, srcs, k=256, select_mode=1, hops=hops)
        assert_close(d, oracle.ich(m, srcs)[0], hbar, what=f"two components {srcs}")
    tri = G.Mesh("triangle", np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.3, 0.8, 0.0]]), np.array([[0, 1, 2]]))
    for s in range(3):
        d, st, _ = gpu_field(pch, tri, [s], k=16, hops=hops)
        assert np.max(np.abs(d - np.linalg.norm(tri.xyz - tri.xyz[s], axis=1))) <= 1e-15, s


def test_metric_only_mesh_matches_coordinates(pch, oracle):
    """The same bump grid given by coordinates and by its edge lengths only
    (pch_mesh_create_from_lengths, Section 4.1: the method needs the metric
    alone): both fields equal ICH at every vertex."""
    m = G.bump_grid(48, seed=4)
    he = oracle.lengths(m)
    mm = G.Mesh("bump48_metric", None, m.faces, he_len=he, nv=m.nv)
    hbar = mean_edge(oracle, m)
    ref = oracle.ich(m, [5])[0]
    for mesh, what in ((m, "coordinates"), (mm, "lengths")):
        d, st, _ = gpu_field(pch, mesh, [5], k=1024, select_mode=1, hops=5)
        say(f"{what}: rounds {st['rounds']} processed {st['processed']}")
        assert_close(d, ref, hbar, what=what)
