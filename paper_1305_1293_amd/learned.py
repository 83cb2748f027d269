"""Learned selection cutoff: train the distance predictor on PCH's own fields
and use its predictions to set each round's cutoff (PCH_SELECT_LEARNED).

The network only steers how far a round's selection reaches; every field it
is used on is still computed exactly by the PCH rounds.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

from . import pch


def mesh_frame(xyz: np.ndarray):
    """Centre (bounding-box centre) and radius used to normalise features."""
    lo, hi = xyz.min(axis=0), xyz.max(axis=0)
    c = 0.5 * (lo + hi)
    r = float(np.linalg.norm(xyz - c, axis=1).max())
    return c, r


def frame_of(gen_mesh):
    """mesh_frame of a generated mesh, computed once per mesh (a per-mesh
    constant, not part of a field's cost)."""
    if "frame" not in gen_mesh.meta:
        gen_mesh.meta["frame"] = mesh_frame(gen_mesh.xyz)
    return gen_mesh.meta["frame"]


@dataclass
class FieldSamples:
    feats: "object"   # device float [n, 7]
    base: "object"    # device float [n]
    target: "object"  # device float [n]
    scale: "object"   # device float [n]


def field_samples(gen_mesh, dev_mesh: pch.Mesh, xyz_dev, source: int, k: int = 8192):
    """Features and exact PCH distances of one field (all vertices)."""
    import torch
    c, r = frame_of(gen_mesh)
    feats, base = pch.MLP.features(xyz_dev, source, c, r)
    d = pch.geodesic(dev_mesh, [source], k=k, select_mode=pch.PCH_SELECT_DELTA)
    hbar = float(np.mean(np.linalg.norm(gen_mesh.xyz[gen_mesh.faces[:, 1]] - gen_mesh.xyz[gen_mesh.faces[:, 0]],
                                        axis=1)))
    target = d.to(torch.float32)
    scale = torch.clamp(target, min=hbar)
    return FieldSamples(feats, base, target, scale), d


def build_training_set(gens: Sequence, k: int = 8192):
    """Samples of every vertex of every (mesh, source) in gens[i].meta['sources']."""
    import torch
    parts: List[FieldSamples] = []
    fields = []
    for g in gens:
        dm = pch.Mesh.from_generated(g)
        xyz = torch.from_numpy(g.xyz).to("cuda")
        for s in g.meta["sources"]:
            fs, d = field_samples(g, dm, xyz, int(s), k)
            parts.append(fs)
            fields.append((g, int(s), d))
        dm.close()
    cat = lambda name: torch.cat([getattr(p, name) for p in parts])
    return FieldSamples(cat("feats"), cat("base"), cat("target"), cat("scale")), fields


def train(mlp: pch.MLP, data: FieldSamples, epochs: int = 3, batch: int = 16384, lr: float = 1e-3,
          weight_decay: float = 1e-4, seed: int = 0, log_every: int = 0):
    """Mini-batch AdamW on the GPU; returns the loss of every logged step."""
    import torch
    n = int(data.feats.shape[0])
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    losses = []
    step = 0
    for _ in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=g)
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch]
            want = log_every > 0 and step % log_every == 0
            l = mlp.train_step(data.feats[idx].contiguous(), data.base[idx].contiguous(),
                               data.target[idx].contiguous(), data.scale[idx].contiguous(), lr, weight_decay,
                               want_loss=want)
            if want:
                losses.append(l)
            step += 1
    return losses


def predict_field(mlp: pch.MLP, gen_mesh, xyz_dev, source: int):
    c, r = frame_of(gen_mesh)
    feats, base = pch.MLP.features(xyz_dev, source, c, r)
    return mlp.forward(feats, base)


def learned_geodesic(mlp: pch.MLP, gen_mesh, dev_mesh: pch.Mesh, xyz_dev, source: int, k: int = 8192,
                     w0: float = 4.0, **opts):
    """Exact field with the learned cutoff; returns (distances, stats)."""
    pred = predict_field(mlp, gen_mesh, xyz_dev, source)
    return pch.geodesic(dev_mesh, [source], k=k, predicted=pred, w0=w0, return_stats=True, **opts)


def chord_geodesic(gen_mesh, dev_mesh: pch.Mesh, xyz_dev, source: int, k: int = 8192, w0: float = 4.0, **opts):
    """The same cutoff rule without the network: the predicted distance of a
    vertex is its chord length to the source (the network's base term, a
    lower bound of the geodesic distance). Returns (distances, stats)."""
    c, r = frame_of(gen_mesh)
    _, base = pch.MLP.features(xyz_dev, source, c, r)
    return pch.geodesic(dev_mesh, [source], k=k, predicted=base, w0=w0, return_stats=True, **opts)


def batch_predictions(mlp, gens: Sequence, field_mesh, field_source, offsets, chord: bool = False):
    """Predicted distances of every field of a batch in the output's layout
    (field f at offsets[f]): the network's, or with chord=True the chord
    lengths (the same rule without the network). Returns a device float
    tensor for Batch(..., predicted=...)."""
    import torch
    n = int(offsets[-1])
    feats = torch.empty((n, 7), dtype=torch.float32, device="cuda")
    base = torch.empty(n, dtype=torch.float32, device="cuda")
    xyz = [torch.from_numpy(g.xyz).to("cuda") for g in gens]
    frames = [frame_of(g) for g in gens]
    # every field's features straight into its slice of one buffer, then one
    # network pass over all of them (each sample's prediction depends on its
    # own features only)
    for f, (mi, s) in enumerate(zip(field_mesh, field_source)):
        c, r = frames[int(mi)]
        o0, o1 = int(offsets[f]), int(offsets[f + 1])
        pch.MLP.features(xyz[int(mi)], int(s), c, r, feats=feats[o0:o1], base=base[o0:o1])
    return base if chord else mlp.forward(feats, base)
