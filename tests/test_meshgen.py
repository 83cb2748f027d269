"""Seeded generators produce the stated workload shapes (no method arithmetic)."""
import numpy as np

from paper_1305_1293_amd import meshgen as G


def _signed_volume(m):
    a, b, c = m.xyz[m.faces[:, 0]], m.xyz[m.faces[:, 1]], m.xyz[m.faces[:, 2]]
    return np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0


def _euler(m):
    e = np.concatenate([m.faces[:, [0, 1]], m.faces[:, [1, 2]], m.faces[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return m.nv - e.shape[0] + m.nf


def test_grid_counts():
    m = G.sinusoid_grid(64, 0)
    assert m.nv == 4096 and m.nf == 7938
    assert G.grid_faces(1024, 1024).shape[0] == 2_093_058


def test_icosphere_counts_and_orientation():
    for lvl, nv, nf in [(0, 12, 20), (2, 162, 320), (5, 10242, 20480)]:
        v, f = G.icosphere(lvl)
        assert v.shape[0] == nv and f.shape[0] == nf
        m = G.Mesh("ico", v, f)
        assert _signed_volume(m) > 0.0  # outward CCW faces
        assert _euler(m) == 2


def test_bumpy_icosphere_level7_size():
    m = G.bumpy_icosphere(7, seed=1)
    assert m.nv == 163_842 and m.nf == 327_680
    r = np.linalg.norm(m.xyz, axis=1)
    assert 0.9 < r.min() and r.max() < 1.1
    assert 0 <= m.meta["source"] < m.nv


def test_closed_solids():
    for m in [G.cube(3), G.tetrahedron(3)]:
        assert _euler(m) == 2
        assert _signed_volume(m) > 0.0


def test_cone_metric():
    m = G.cone_fan(7, 3)
    assert m.xyz is None and np.allclose(m.he_len, 1.0 / 3.0)
    assert m.meta["polar"].shape == (m.nv, 2)


def test_seeded_determinism():
    a = G.bump_grid(40, seed=5)
    b = G.bump_grid(40, seed=5)
    assert np.array_equal(a.xyz, b.xyz)
    c = G.bump_grid(40, seed=6)
    assert not np.array_equal(a.xyz, c.xyz)
