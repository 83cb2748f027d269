"""The oracle against surfaces whose geodesic distances have closed forms.

Each case fixes the exact distance field independently of any window logic:
planar meshes (Euclidean distance), a planar L-shape whose reflex corner is a
boundary pseudo-source, a plane folded isometrically, the unit cube and the
regular tetrahedron through their unfoldings, and flat cones of total angle
7 pi / 3 (saddle apex) and 5 pi / 3 (spherical apex).
Both oracle paths run: ICH (priority queue) and the round-based replica.
"""
import math

import numpy as np
import pytest

from paper_1305_1293_amd import meshgen as G

RTOL = 1e-12


def runs(oracle, m, s, eps=0.0):
    d_ich, _ = oracle.ich(m, [s], eps_tiny=eps)
    yield "ich", d_ich
    for k in (1, 7, 64, 1 << 30):
        d, _, _ = oracle.replica(m, [s], k, eps_tiny=eps)
        yield f"replica k={k}", d


def check(oracle, m, s, expect, eps=0.0, tol=RTOL):
    scale = max(1.0, float(np.max(expect[np.isfinite(expect)])))
    for name, d in runs(oracle, m, s, eps):
        err = np.abs(d - expect).max() / scale
        assert err < tol, f"{m.name} source {s} {name}: max rel err {err:.3e}"


@pytest.mark.parametrize("seed", [0, 1])
def test_t1_plane(oracle, seed):
    m = G.jittered_plane(12, seed)
    for s in (0, 5, 66, m.nv - 1):
        check(oracle, m, s, np.linalg.norm(m.xyz - m.xyz[s], axis=1))


def lshape_expect(m):
    s = np.array([2.0, 0.0])
    c = np.array([1.0, 1.0])
    p = m.xyz[:, :2]
    direct = np.linalg.norm(p - s, axis=1)
    around = math.sqrt(2.0) + np.linalg.norm(p - c, axis=1)
    visible = (p[:, 1] <= 1.0) | (p[:, 0] + p[:, 1] <= 2.0 + 1e-12)
    return np.where(visible, direct, around)


def test_t2_lshape_reflex_corner(oracle):
    m = G.lshape(6)
    s = int(np.argmin(np.linalg.norm(m.xyz[:, :2] - [2.0, 0.0], axis=1)))
    exp = lshape_expect(m)
    assert (exp > np.linalg.norm(m.xyz[:, :2] - [2.0, 0.0], axis=1) + 1e-9).sum() > 10  # bends present
    check(oracle, m, s, exp)


def test_t3_folded_plane(oracle):
    m = G.folded_plane(12, 0)
    flat = m.meta["flat_xyz"]
    for s in (0, 77, 143):
        check(oracle, m, s, np.linalg.norm(flat - flat[s], axis=1))


def cube_corner_expect(P):
    x, y, z = P[:, 0], P[:, 1], P[:, 2]
    out = np.full(P.shape[0], np.inf)
    near = (x == 0) | (y == 0) | (z == 0)
    out[near] = np.linalg.norm(P[near], axis=1)
    for a, b, c in [(x, y, z), (y, x, z), (z, x, y)]:  # far face a == 1, coordinates (b, c)
        far = a == 1
        cand = np.minimum(np.hypot(1 + b, c), np.hypot(1 + c, b))
        out[far] = np.minimum(out[far], cand[far])
    return out


@pytest.mark.parametrize("n", [2, 4])
def test_t4_cube_corner(oracle, n):
    m = G.cube(n)
    s = int(np.argmin(np.linalg.norm(m.xyz, axis=1)))
    exp = cube_corner_expect(m.xyz)
    opp = int(np.argmin(np.linalg.norm(m.xyz - 1.0, axis=1)))
    assert abs(exp[opp] - math.sqrt(5.0)) < 1e-15
    check(oracle, m, s, exp)


def test_t4_cube_face_centre(oracle):
    m = G.cube(4)
    vid = lambda p: int(np.argmin(np.linalg.norm(m.xyz - p, axis=1)))
    s = vid([0.5, 0.5, 0.0])
    for name, d in runs(oracle, m, s):
        assert abs(d[vid([0.5, 0.5, 1.0])] - 2.0) < 1e-13, name
        assert abs(d[vid([1.0, 0.5, 0.5])] - 1.0) < 1e-13, name
        assert abs(d[vid([0.5, 0.0, 0.5])] - 1.0) < 1e-13, name
        bottom = m.xyz[:, 2] == 0
        assert np.allclose(d[bottom], np.linalg.norm(m.xyz[bottom] - m.xyz[s], axis=1), atol=1e-13), name


def test_t5_tetrahedron(oracle):
    a = 1.0
    m = G.tetrahedron(3, a)
    C = m.meta["corners"]
    vid = lambda p: int(np.argmin(np.linalg.norm(m.xyz - p, axis=1)))
    A, B, Cc, D = (vid(c) for c in C)
    for name, d in runs(oracle, m, A):
        assert abs(d[B] - a) < 1e-13, name
        third = vid(C[1] + (C[2] - C[1]) / 3.0)  # on BC, one third from B
        assert abs(d[third] - math.sqrt(7.0 / 9.0) * a) < 1e-13, name
        cen = vid((C[1] + C[2] + C[3]) / 3.0)
        assert abs(d[cen] - 2.0 * a / math.sqrt(3.0)) < 1e-13, name
        # points on the three faces at A: straight chords
        for f in ([0, 1, 2], [0, 3, 1], [0, 2, 3]):
            nrm = np.cross(C[f[1]] - C[f[0]], C[f[2]] - C[f[0]])
            on = np.abs((m.xyz - C[f[0]]) @ nrm) < 1e-12
            assert np.allclose(d[on], np.linalg.norm(m.xyz[on] - C[0], axis=1), atol=1e-13), name


def cone_expect(polar, total, s):
    r1, t1 = polar[s]
    r2, t2 = polar[:, 0], polar[:, 1]
    phi1 = np.abs(t2 - t1) % total
    phi2 = total - phi1
    best = np.full(r2.shape, np.inf)
    for phi in (phi1, phi2):
        loc = np.sqrt(np.maximum(r1 * r1 + r2 * r2 - 2 * r1 * r2 * np.cos(phi), 0.0))
        best = np.minimum(best, np.where(phi < math.pi, loc, r1 + r2))
    return best


@pytest.mark.parametrize("nsect", [7, 5])
def test_t6_t7_cones(oracle, nsect):
    m = G.cone_fan(nsect, 4)
    pol = m.meta["polar"]
    apex = int(np.argmin(pol[:, 0]))
    srcs = [int(np.argmin(np.abs(pol[:, 0] - 0.5) + np.abs(pol[:, 1] - 0.3))), int(np.argmax(pol[:, 0]))]
    if nsect == 7:
        exp = cone_expect(pol, m.meta["total_angle"], srcs[0])
        assert np.any(np.isclose(exp, pol[srcs[0], 0] + pol[:, 0]) & (pol[:, 0] > 0.2))  # paths via the apex
    for s in srcs + [apex]:
        check(oracle, m, s, cone_expect(pol, m.meta["total_angle"], s))


def test_paper_tolerance_keeps_closed_forms(oracle):
    """With the tiny-window tolerance 1e-6 of Section 5 the fields stay exact
    on the closed-form surfaces (to 1e-9)."""
    m = G.cube(4)
    s = int(np.argmin(np.linalg.norm(m.xyz, axis=1)))
    check(oracle, m, s, cube_corner_expect(m.xyz), eps=1e-6, tol=1e-9)
    m = G.cone_fan(7, 4)
    pol = m.meta["polar"]
    check(oracle, m, 5, cone_expect(pol, m.meta["total_angle"], 5), eps=1e-6, tol=1e-9)
