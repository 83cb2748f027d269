"""The stored exact fields (tests/golden/) against the oracle that wrote
them and against what the metric fixes.

* icosphere (327,680 faces): the field from the first stored source is
  recomputed by sequential ICH and must equal the stored one bit for bit;
* 1024^2 bump grid from vertex 0 (too long to recompute here): zero at the
  source, finite everywhere, 1-Lipschitz along every edge, at least the
  straight-line distance and at most the edge-graph (Dijkstra) distance.
"""
import os

import numpy as np

from paper_1305_1293_amd import meshgen as G

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_icosphere_golden_is_the_oracle_field(oracle):
    gold = np.load(os.path.join(HERE, "icosphere7_ich.npz"))
    m = G.config_mesh(2)
    assert int(gold["nv"]) == m.nv and int(gold["nf"]) == m.nf
    assert gold["dist"].shape == (2, m.nv)
    assert float(gold["mean_edge"]) == float(oracle.lengths(m).mean())
    s = int(gold["sources"][0])
    d, _ = oracle.ich(m, [s])
    assert np.array_equal(d.view(np.uint64), gold["dist"][0].view(np.uint64))


def test_bump_grid_golden_metric_bounds(oracle):
    gold = np.load(os.path.join(HERE, "bump_grid1024_s2_ich.npz"))
    m = G.config_mesh(3)
    d = gold["dist"]
    s = int(gold["source"])
    assert int(gold["nv"]) == m.nv and int(gold["nf"]) == m.nf and d.shape == (m.nv,)
    assert s == int(m.meta["source"]) and d[s] == 0.0 and np.all(np.isfinite(d))
    he = oracle.lengths(m)
    assert abs(float(gold["mean_edge"]) - float(he.mean())) <= 1e-15 * float(he.mean())
    # 1-Lipschitz along every edge of every face
    f = m.faces
    for a, b, k in ((0, 1, 0), (1, 2, 1), (2, 0, 2)):
        u, v = f[:, a], f[:, b]
        L = he[k::3]
        assert np.all(np.abs(d[u] - d[v]) <= L * (1.0 + 1e-12) + 1e-12)
    # straight-line distance <= geodesic <= edge-graph distance
    chord = np.linalg.norm(m.xyz - m.xyz[s], axis=1)
    assert np.all(d >= chord * (1.0 - 1e-12))
    dj = oracle.dijkstra(m, [s])
    assert np.all(d <= dj * (1.0 + 1e-12))
