"""ICH against exhaustive enumeration of unfolded straight segments (tiny meshes).

The enumerator (oracle/brute.py) knows nothing of windows: it builds the
vertex visibility graph from every no-repeat face sequence and runs Dijkstra,
which is exact by the theorem of Mitchell, Mount and Papadimitriou.
"""
import numpy as np
import pytest

from oracle import brute as B
from paper_1305_1293_amd import meshgen as G

MESHES = G.random_tiny_meshes(0, 6) + [G.cube(2), G.tetrahedron(3), G.cone_fan(7, 2), G.cone_fan(5, 2)]


@pytest.mark.parametrize("m", MESHES, ids=[m.name for m in MESHES])
def test_ich_equals_brute(oracle, m):
    he = oracle.lengths(m)
    for s in sorted({0, m.nv // 2, m.nv - 1}):
        bd = B.brute_distances(m.faces, he, m.nv, [s])
        d, _ = oracle.ich(m, [s])
        assert np.max(np.abs(d - bd)) < 1e-12 * max(1.0, bd.max())
        dr, _, _ = oracle.replica(m, [s], 4)
        assert np.max(np.abs(dr - bd)) < 1e-12 * max(1.0, bd.max())
