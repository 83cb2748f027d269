"""Pins of the oracle's mesh layer and elementary functions (CPU only)."""
import math

import numpy as np
import pytest

from paper_1305_1293_amd import meshgen as G


def test_twin_involution_and_euler(oracle):
    for m in [G.cube(3), G.tetrahedron(3), G.bumpy_icosphere(2, seed=3), G.sinusoid_grid(9, 0)]:
        info = oracle.mesh_info(m)
        tw = info["twin"]
        inner = tw >= 0
        assert np.all(tw[tw[inner]] == np.nonzero(inner)[0])
        if m.name.startswith(("cube", "tetra", "bumpy")):
            assert inner.all()  # closed surfaces
            ne = tw.size // 2
            assert m.nv - ne + m.nf == 2


def test_total_angles_closed_forms(oracle):
    tet = G.tetrahedron(3)
    th = oracle.mesh_info(tet)["theta"]
    corners = [int(np.argmin(np.linalg.norm(tet.xyz - c, axis=1))) for c in tet.meta["corners"]]
    assert np.allclose(th[corners], math.pi, atol=1e-12)
    others = np.setdiff1d(np.arange(tet.nv), corners)
    assert np.allclose(th[others], 2 * math.pi, atol=1e-12)

    cube = G.cube(4)
    info = oracle.mesh_info(cube)
    is_corner = np.all((cube.xyz == 0) | (cube.xyz == 1), axis=1)
    assert np.allclose(info["theta"][is_corner], 1.5 * math.pi, atol=1e-12)
    assert np.allclose(info["theta"][~is_corner], 2 * math.pi, atol=1e-12)
    assert not info["pseudo"].any()  # spherical corners, flat elsewhere

    for ns, tot in [(7, 7 * math.pi / 3), (5, 5 * math.pi / 3)]:
        cone = G.cone_fan(ns, 3)
        info = oracle.mesh_info(cone)
        apex = int(np.argmin(cone.meta["polar"][:, 0]))
        assert abs(info["theta"][apex] - tot) < 1e-12
        assert info["pseudo"][apex] == (ns == 7)
        assert info["boundary"].sum() == ns * 3  # rim vertices


def test_apex_coordinates_match_3d_triangles(oracle):
    m = G.bumpy_icosphere(2, seed=0)
    info = oracle.mesh_info(m)
    f = m.faces
    start = f.reshape(-1)
    end = np.roll(f, -1, axis=1).reshape(-1)
    opp = np.roll(f, -2, axis=1).reshape(-1)
    a, b, c = m.xyz[start], m.xyz[end], m.xyz[opp]
    u = b - a
    L = np.linalg.norm(u, axis=1)
    x = np.einsum("ij,ij->i", c - a, u) / L
    y = np.linalg.norm(np.cross(u, c - a), axis=1) / L
    assert np.allclose(info["ax"], x, rtol=0, atol=1e-13)
    assert np.allclose(info["ay"], y, rtol=0, atol=1e-13)
    assert np.all(info["ay"] > 0)


def test_boundary_flags_grid(oracle):
    n = 7
    m = G.sinusoid_grid(n, 0)
    info = oracle.mesh_info(m)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    on_b = ((i == 0) | (j == 0) | (i == n - 1) | (j == n - 1)).ravel()
    assert np.array_equal(info["boundary"], on_b)
    assert np.all(info["pseudo"][on_b])


def _err(oracle, m):
    with pytest.raises(oracle.OracleError) as e:
        oracle.mesh_info(m)
    return e.value.code


def test_invalid_meshes(oracle):
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], float)
    # three faces on one edge
    assert _err(oracle, G.Mesh("nm", xyz, np.array([[0, 1, 2], [1, 0, 3], [0, 1, 4]]))) == -2
    # inconsistent orientation across an edge
    assert _err(oracle, G.Mesh("flip", xyz, np.array([[0, 1, 2], [0, 1, 3]]))) == -2
    # zero-area face
    xyz2 = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0]], float)
    assert _err(oracle, G.Mesh("flat", xyz2, np.array([[0, 1, 2]]))) == -2
    # index out of range
    assert _err(oracle, G.Mesh("oob", xyz, np.array([[0, 1, 7]]), nv=5)) == -1
    # bow-tie: two fans meet at vertex 0
    xyz3 = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [-1, 0, 0], [-1, -1, 0]], float)
    assert _err(oracle, G.Mesh("bowtie", xyz3, np.array([[0, 1, 2], [0, 3, 4]]))) == -2


def test_own_atan2_and_sincos(oracle):
    rng = np.random.default_rng(0)
    for _ in range(2000):
        y, x = rng.normal(size=2) * 10.0 ** rng.uniform(-8, 3)
        assert abs(oracle.fn_atan2(y, x) - math.atan2(y, x)) <= 1e-15 * max(1.0, abs(math.atan2(y, x)))
    for t in np.concatenate([rng.uniform(0, math.pi, 2000), [0.0, math.pi / 4, math.pi / 2, math.pi]]):
        s, c = oracle.fn_sincos(float(t))
        assert abs(s - math.sin(t)) < 5e-16 and abs(c - math.cos(t)) < 5e-16
