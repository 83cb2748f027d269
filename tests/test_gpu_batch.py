"""GPU tests of the batched persistent launch (many fields, uneven meshes).

Every batched field must equal the single-field run with the same selection
rule (adaptive step, same k and first step) bit for bit, and ICH to 1e-9;
graph replays with eager work in between give the same bits again.
"""
import sys

import numpy as np
import pytest

from paper_1305_1293_amd import meshgen as G

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pch():
    import torch
    assert torch.cuda.is_available()
    from paper_1305_1293_amd import pch as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def setup(pch):
    gens = [G.sinusoid_grid(24, 0), G.bumpy_icosphere(3, seed=5), G.bump_grid(32, seed=7), G.cone_fan(7, 5),
            G.bump_grid(96, seed=23)]
    meshes = [pch.Mesh.from_generated(m) for m in gens]
    rng = np.random.default_rng(1)
    fm, fs = [], []
    for i, m in enumerate(gens):
        for s in rng.choice(m.nv, 4, replace=False):
            fm.append(i)
            fs.append(int(s))
    return gens, meshes, np.array(fm), np.array(fs)


def single(pch, mesh, s, k, hops=1):
    import torch
    d = pch.geodesic(mesh, [s], k=k, select_mode=1, hops=hops)
    torch.cuda.synchronize()
    return d.cpu().numpy()


@pytest.mark.parametrize("use_graph,hops", [(1, 1), (0, 1), (1, 4)])
def test_batch_equals_single_fields(pch, oracle, setup, use_graph, hops):
    import torch
    gens, meshes, fm, fs = setup
    k = 256
    b = pch.Batch(meshes, fm, fs, k=k, teams_per_cu=1, use_graph=use_graph, hops=hops)
    say(f"batch of {b.n_fields} fields, graph {use_graph}, hops {hops}")
    out, st = b.run()
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert st["fields"] == b.n_fields
    fstat = b.field_stats()
    assert np.all(fstat[:, 0] == 0), fstat[:, 0]
    assert np.all(fstat[:, 7] > 0)  # each field's time in its workgroup
    for f in range(b.n_fields):
        ref = single(pch, meshes[fm[f]], int(fs[f]), k, hops)
        gf = got[b.offsets[f]:b.offsets[f + 1]]
        assert np.array_equal(gf.view(np.uint64), ref.view(np.uint64)), f"field {f} differs from the single run"
        d_ich, _ = oracle.ich(gens[fm[f]], [int(fs[f])])
        hbar = float(oracle.lengths(gens[fm[f]]).mean())
        assert np.max(np.abs(gf - d_ich) / np.maximum(d_ich, hbar)) <= 1e-9, f
    # replays with eager work in between
    for rep in range(3):
        single(pch, meshes[0], 3, 64)
        out2, _ = b.run(out)
        torch.cuda.synchronize()
        assert np.array_equal(out2.cpu().numpy().view(np.uint64), got.view(np.uint64)), f"replay {rep}"
    b.close()


@pytest.mark.parametrize("gang,tpc,threads", [(2, 1, 256), (8, 2, 256), (32, 1, 256), (4, 1, 1024), (8, 1, 512)])
def test_batch_gangs_equal_single_fields(pch, setup, gang, tpc, threads):
    """Workgroups that find the queue empty join running fields of their XCD;
    the shared rounds give the single-field bits, on every replay."""
    import torch
    gens, meshes, fm, fs = setup
    k = 256
    b = pch.Batch(meshes, fm, fs, k=k, teams_per_cu=tpc, team_threads=threads, hops=4, gang=gang)
    say(f"batch of {b.n_fields} fields, gang {gang}, teams per CU {tpc}, {threads} threads")
    refs = [single(pch, meshes[fm[f]], int(fs[f]), k, 4) for f in range(b.n_fields)]
    out = None
    for rep in range(3):
        out, st = b.run(out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        fstat = b.field_stats()
        assert st["reruns"] == 0 and np.all(fstat[:, 0] == 0), fstat[:, 0]
        for f in range(b.n_fields):
            gf = got[b.offsets[f]:b.offsets[f + 1]]
            assert np.array_equal(gf.view(np.uint64), refs[f].view(np.uint64)), f"run {rep} field {f}"
    b.close()


@pytest.mark.parametrize("gang", [1, 8])
def test_batch_stronger_filtering_equals_single_fields(pch, setup, gang):
    """filters bit 3 (windows re-take the ICH endpoint tests when they
    propagate) in the batched launch: every field equals its single-field run
    with the same option bit for bit."""
    import torch
    gens, meshes, fm, fs = setup
    k = 256
    b = pch.Batch(meshes, fm, fs, k=k, teams_per_cu=1, hops=4, gang=gang, filters=11)
    say(f"batch of {b.n_fields} fields, filters 11, gang {gang}")
    out, st = b.run()
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert st["reruns"] == 0
    for f in range(b.n_fields):
        d = pch.geodesic(meshes[fm[f]], [int(fs[f])], k=k, select_mode=1, hops=4, filters=11)
        torch.cuda.synchronize()
        ref = d.cpu().numpy()
        gf = got[b.offsets[f]:b.offsets[f + 1]]
        assert np.array_equal(gf.view(np.uint64), ref.view(np.uint64)), f"field {f}"
    b.close()


def test_batch_gangs_many_fields(pch):
    """More fields than workgroups (every XCD runs 32 or more teams): the last
    fields are shared by the teams that ran out of work."""
    import torch
    gens = [G.bumpy_icosphere(2, seed=40 + i) for i in range(3)] + [G.bump_grid(40, seed=43)]
    meshes = [pch.Mesh.from_generated(m) for m in gens]
    rng = np.random.default_rng(5)
    fm = np.repeat(np.arange(len(gens)), 160)
    fs = np.concatenate([rng.choice(m.nv, 160) for m in gens])
    k = 512
    say(f"{fm.size} fields, gang 8")
    b1 = pch.Batch(meshes, fm, fs, k=k, teams_per_cu=1, hops=4, gang=1)
    b8 = pch.Batch(meshes, fm, fs, k=k, teams_per_cu=1, hops=4, gang=8)
    o1, st1 = b1.run()
    f1 = b1.field_stats()
    say(f"gang 1: status counts {np.bincount(f1[:, 0], minlength=5).tolist()}")
    for rep in range(3):
        o8, st = b8.run()
        torch.cuda.synchronize()
        f8 = b8.field_stats()
        say(f"gang 8 run {rep}: status counts {np.bincount(f8[:, 0], minlength=5).tolist()}, "
            f"rerun fields {np.nonzero(f8[:, 0])[0].tolist()}, helpers {int(f8[:, 8].sum())}")
        # the shared rounds never give up (status 3) or leave a field unrun (4);
        # pool overflows rerun the same fields as without helpers
        assert np.array_equal(f8[:, 0] != 0, f1[:, 0] != 0), rep
        assert np.array_equal(o8.cpu().numpy().view(np.uint64), o1.cpu().numpy().view(np.uint64)), rep
    for f in rng.choice(fm.size, 6, replace=False):
        ref = single(pch, meshes[fm[f]], int(fs[f]), k, 4)
        assert np.array_equal(b1.field(o1, f).cpu().numpy().view(np.uint64), ref.view(np.uint64)), f
    b1.close()
    b8.close()


def test_batch_gang_waits_run_out(pch, setup):
    """A wait limit of one tick makes every shared field give up (forced from
    the host: every wait in the kernel is bounded by it); such fields are
    rerun with pch_geodesic, so every field still equals its single run."""
    import torch
    gens, meshes, fm, fs = setup
    k = 256
    b = pch.Batch(meshes, fm, fs, k=k, teams_per_cu=1, hops=4, gang=8, wait_ticks=1)
    out, st = b.run()
    torch.cuda.synchronize()
    fstat = b.field_stats()
    say(f"status counts {np.bincount(fstat[:, 0], minlength=5).tolist()}, reruns {st['reruns']}")
    assert st["reruns"] == int(np.count_nonzero(fstat[:, 0]))
    got = out.cpu().numpy()
    for f in range(b.n_fields):
        ref = single(pch, meshes[fm[f]], int(fs[f]), k, 4)
        assert np.array_equal(got[b.offsets[f]:b.offsets[f + 1]].view(np.uint64), ref.view(np.uint64)), f
    b.close()


@pytest.mark.parametrize("hops", [1, 3])
def test_batch_overflow_reruns(pch, setup, hops):
    import torch
    gens, meshes, fm, fs = setup
    b0 = pch.Batch(meshes, fm, fs, k=256, teams_per_cu=1, hops=hops)
    out0, _ = b0.run()
    b1 = pch.Batch(meshes, fm, fs, k=256, teams_per_cu=1, pool_capacity=128, hops=hops)
    out1, st = b1.run()
    torch.cuda.synchronize()
    assert st["reruns"] > 0
    assert np.array_equal(out0.cpu().numpy().view(np.uint64), out1.cpu().numpy().view(np.uint64))
    b0.close()
    b1.close()


def test_voronoi_labels(pch, oracle):
    """Voronoi labels: each vertex's label is the first nearest source of the
    single-source fields (argmin, ties to the lowest index) and its distance
    their minimum, bit for bit; the minimum is the multi-source field of ICH
    within 1e-9."""
    import torch
    for m, k in [(G.bumpy_icosphere(4, seed=9), 512), (G.bump_grid(48, seed=4), 1024)]:
        srcs = np.random.default_rng(11).choice(m.nv, 7, replace=False).astype(np.int32)
        say(f"voronoi {m.name}, {srcs.size} sources")
        dm = pch.Mesh.from_generated(m)
        dist, label = pch.voronoi(dm, srcs, k=k)
        torch.cuda.synchronize()
        fields = np.stack([single(pch, dm, int(s), k, 4) for s in srcs])
        assert np.array_equal(label.cpu().numpy(), np.argmin(fields, axis=0).astype(np.int32))
        assert np.array_equal(dist.cpu().numpy().view(np.uint64), fields.min(axis=0).view(np.uint64))
        assert np.array_equal(label.cpu().numpy()[srcs], np.arange(srcs.size, dtype=np.int32))
        ref, _ = oracle.ich(m, [int(s) for s in srcs])
        hbar = float(oracle.lengths(m).mean())
        assert np.max(np.abs(dist.cpu().numpy() - ref) / np.maximum(ref, hbar)) <= 1e-9
        dm.close()


def test_batch_argument_errors(pch, setup):
    gens, meshes, fm, fs = setup
    with pytest.raises(pch.PchError):
        pch.Batch(meshes, [0], [gens[0].nv])
    with pytest.raises(pch.PchError):
        pch.Batch(meshes, [len(meshes)], [0])
    for gang in (-1, 33):
        with pytest.raises(pch.PchError):
            pch.Batch(meshes, [0], [0], gang=gang)
    with pytest.raises(pch.PchError):
        pch.Batch(meshes, [0], [0], wait_ticks=-1)
    with pytest.raises(pch.PchError):
        pch.voronoi(meshes[0], [gens[0].nv])


def test_tune_keeps_fields_exact(pch, setup):
    """The autotuner times its grid of (k, workgroup shape, hops, gang size)
    settings on the batch and keeps the fastest; the batch then still equals
    the single-field runs with the chosen k and hops, bit for bit."""
    import torch
    gens, meshes, fm, fs = setup
    b = pch.Batch(meshes[:3], fm[fm < 3], fs[fm < 3], k=256, teams_per_cu=1)
    out, _ = b.run()
    chosen = b.tune(out)
    say(f"tuned: {chosen}")
    assert chosen["k"] in (8192, 16384, 32768, 65536) and chosen["hops"] in (1, 4)
    assert (chosen["team_threads"], chosen["teams_per_cu"]) in ((256, 1), (512, 1), (1024, 1))
    assert chosen["gang"] in (1, 2, 4, 8, 16)
    out, st = b.run(out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for f in range(b.n_fields):
        ref = single(pch, meshes[int(b.field_mesh[f])], int(b.field_source[f]), chosen["k"], chosen["hops"])
        assert np.array_equal(got[b.offsets[f]:b.offsets[f + 1]].view(np.uint64), ref.view(np.uint64)), f
    b.close()


def test_full_size_batch_every_field(pch, oracle):
    """The 512-field batch at full size (16 meshes of 14k-330k faces, 32
    sources each) with the benchmark's options (the choice the committed
    tuner cache records for this batch): every field equals its single-field
    run with the same rule, k and hops bit for bit, and the first field of
    every mesh is within 1e-9 of ICH."""
    import os
    import torch
    gens = G.batch_meshes(3)
    meshes = [pch.Mesh.from_generated(m) for m in gens]
    fm = np.repeat(np.arange(len(gens)), 32).astype(np.int32)
    fs = np.concatenate([m.meta["sources"] for m in gens]).astype(np.int32)
    cache = os.path.join(os.path.dirname(os.path.abspath(pch.__file__)), "tune_cache.txt")
    assert os.path.exists(cache)
    pch.tune_cache_load(cache)
    b = pch.Batch(meshes, fm, fs, k=32768, team_threads=512, teams_per_cu=1, hops=4, gang=8)
    chosen, hit = b.tune_cached()
    k, hops = int(chosen["k"]), int(chosen["hops"])
    say(f"batch of {b.n_fields} fields on {len(gens)} meshes, cache hit {hit}: k {k} hops {hops} "
        f"team {chosen['team_threads']} gang {chosen['gang']}")
    out, _ = b.run()
    out, st = b.run(out)  # a graph replay, as timed by the benchmark
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    say(f"  reruns {st['reruns']} processed {st['processed']}")
    for f in range(b.n_fields):
        ref = single(pch, meshes[fm[f]], int(fs[f]), k, hops)
        gf = got[b.offsets[f]:b.offsets[f + 1]]
        assert np.array_equal(gf.view(np.uint64), ref.view(np.uint64)), f"field {f} differs from the single run"
    for i, g in enumerate(gens):
        f = 32 * i
        d_ich, _ = oracle.ich(g, [int(fs[f])])
        hbar = float(oracle.lengths(g).mean())
        gf = got[b.offsets[f]:b.offsets[f + 1]]
        assert np.array_equal(np.isfinite(gf), np.isfinite(d_ich))
        assert np.max(np.abs(gf - d_ich) / np.maximum(d_ich, hbar)) <= 1e-9, (g.name, f)
    b.close()
    for dm in meshes:
        dm.close()
