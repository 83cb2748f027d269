"""Seeded synthetic triangle meshes for the exact-geodesic workloads.

This module only builds inputs: vertex coordinates, CCW faces and, for
metric-only surfaces, per-half-edge lengths. It holds none of the geodesic
method's arithmetic, so the CPU oracle and the GPU path can both consume its
output without sharing any computation.

Conventions
-----------
* ``faces`` is int32 ``[nf, 3]``; half-edge ``j = 3 f + i`` runs from
  ``faces[f, i]`` to ``faces[f, (i + 1) % 3]`` (the paper's half-edge layout,
  Section 4.1).
* Grid cells are split along the (i, j)-(i+1, j+1) diagonal; faces are CCW
  when seen from +z. Closed meshes have outward CCW faces.
* Every generator takes an explicit seed and uses ``numpy.random.default_rng``.

The paper's own test models (Section 5, Table 3) are scanned meshes that are
not available here; the workloads below are seeded stand-ins of the same face
counts and character (a smooth bumpy sphere with the Sphere row's 327,680
faces, large anisotropic heightfield grids, and batches of uneven meshes).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Mesh:
    """A triangle mesh plus optional metric-only edge lengths."""

    name: str
    xyz: Optional[np.ndarray]            # float64 [nv, 3] or None (metric-only)
    faces: np.ndarray                    # int32 [nf, 3]
    he_len: Optional[np.ndarray] = None  # float64 [3 nf] for metric-only meshes
    nv: int = 0
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        self.faces = np.ascontiguousarray(self.faces, dtype=np.int32)
        if self.xyz is not None:
            self.xyz = np.ascontiguousarray(self.xyz, dtype=np.float64)
            self.nv = int(self.xyz.shape[0])
        elif self.nv <= 0:
            self.nv = int(self.faces.max()) + 1
        if self.he_len is not None:
            self.he_len = np.ascontiguousarray(self.he_len, dtype=np.float64)

    @property
    def nf(self) -> int:
        return int(self.faces.shape[0])


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------

def grid_faces(nx: int, ny: int) -> np.ndarray:
    """Faces of an nx-by-ny vertex grid (vertex id = j*nx + i), CCW from +z."""
    i, j = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="xy")
    a = (j * nx + i).ravel()
    b = a + 1
    c = a + nx + 1
    d = a + nx
    f1 = np.stack([a, b, c], axis=1)
    f2 = np.stack([a, c, d], axis=1)
    out = np.empty((2 * a.size, 3), dtype=np.int32)
    out[0::2] = f1
    out[1::2] = f2
    return out


def grid_xy(nx: int, ny: int, x0=0.0, x1=1.0, y0=0.0, y1=1.0) -> np.ndarray:
    xs = np.linspace(x0, x1, nx)
    ys = np.linspace(y0, y1, ny)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int32)
    return v, f


def midpoint_subdivide(v: np.ndarray, f: np.ndarray, project_sphere: bool = False):
    """1-to-4 midpoint subdivision (each triangle into four, orientation kept)."""
    nv = v.shape[0]
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
    key = np.minimum(e[:, 0], e[:, 1]).astype(np.int64) * nv + np.maximum(e[:, 0], e[:, 1])
    uniq, inv = np.unique(key, return_inverse=True)
    ea = (uniq // nv).astype(np.int64)
    eb = (uniq % nv).astype(np.int64)
    mid = 0.5 * (v[ea] + v[eb])
    if project_sphere:
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
    nf = f.shape[0]
    m = (inv + nv).reshape(3, nf).T  # m[:,0] on edge (0,1), m[:,1] on (1,2), m[:,2] on (2,0)
    a, b, c = f[:, 0], f[:, 1], f[:, 2]
    m01, m12, m20 = m[:, 0], m[:, 1], m[:, 2]
    nfaces = np.concatenate([
        np.stack([a, m01, m20], 1), np.stack([m01, b, m12], 1),
        np.stack([m20, m12, c], 1), np.stack([m01, m12, m20], 1)], axis=0).astype(np.int32)
    return np.concatenate([v, mid], axis=0), nfaces


def icosphere(level: int):
    v, f = icosahedron()
    for _ in range(level):
        v, f = midpoint_subdivide(v, f, project_sphere=True)
    return v, f


def vertex_neighbor_mean(values: np.ndarray, faces: np.ndarray, nv: int) -> np.ndarray:
    """Mean of ``values`` over each vertex's one-ring (unique edge neighbours)."""
    import scipy.sparse as sp
    e = np.concatenate([faces[:, [0, 1]], faces[:, [1, 2]], faces[:, [2, 0]]], axis=0)
    e = np.concatenate([e, e[:, ::-1]], axis=0)
    A = sp.coo_matrix((np.ones(e.shape[0]), (e[:, 0], e[:, 1])), shape=(nv, nv)).tocsr()
    A.data[:] = 1.0  # duplicates from the two faces of an edge collapse to 1
    deg = np.asarray(A.sum(axis=1)).ravel()
    return (A @ values) / deg


# ---------------------------------------------------------------------------
# benchmark workloads
# ---------------------------------------------------------------------------

def sinusoid_grid(n: int = 64, seed: int = 0) -> Mesh:
    """n x n grid on [0,1]^2, z = 0.05 * sum of 4 seeded sinusoids.

    Frequencies U[1,4] per axis, phases U[0, 2 pi). 64 x 64 gives 7,938 faces.
    """
    rng = np.random.default_rng(seed)
    xy = grid_xy(n, n)
    fx = rng.uniform(1.0, 4.0, 4)
    fy = rng.uniform(1.0, 4.0, 4)
    ph = rng.uniform(0.0, 2.0 * np.pi, 4)
    z = np.zeros(xy.shape[0])
    for i in range(4):
        z += np.sin(2.0 * np.pi * (fx[i] * xy[:, 0] + fy[i] * xy[:, 1]) + ph[i])
    z *= 0.05
    xyz = np.concatenate([xy, z[:, None]], axis=1)
    return Mesh(f"sinusoid_grid{n}_s{seed}", xyz, grid_faces(n, n), meta={"source": 0})


def bumpy_icosphere(level: int = 7, seed: int = 1, amp: float = 0.02) -> Mesh:
    """Icosphere with radial noise r = 1 + amp * n, n ~ N(0,1) smoothed 3 times.

    Each smoothing pass sets n_v <- (n_v + mean over the one-ring) / 2.
    Level 7 gives V = 163,842 and F = 327,680.
    """
    rng = np.random.default_rng(seed)
    v, f = icosphere(level)
    nv = v.shape[0]
    noise = rng.standard_normal(nv)
    for _ in range(3):
        noise = 0.5 * (noise + vertex_neighbor_mean(noise, f, nv))
    v = v * (1.0 + amp * noise)[:, None]
    src = int(rng.integers(0, nv))
    return Mesh(f"bumpy_icosphere_l{level}_s{seed}", v, f, meta={"source": src})


def bump_grid(n: int = 1024, seed: int = 2, jitter: float = 0.4, nbumps: int = 16) -> Mesh:
    """n x n jittered grid on [0,1]^2 with a height field of Gaussian bumps.

    Interior vertices move by U[-jitter, jitter] cells per axis; boundary
    vertices move only along their boundary line (corners stay). Heights:
    z = sum_i a_i exp(-|p - c_i|^2 / (2 s_i^2)), s ~ U[0.02, 0.2],
    c ~ U[0,1]^2, a ~ +-U[0.05, 0.25]. A vertex whose incident 3-D
    triangles get an area below 1e-3 * h^2 / 2 is drawn again.
    """
    rng = np.random.default_rng(seed)
    h = 1.0 / (n - 1)
    xy = grid_xy(n, n)
    faces = grid_faces(n, n)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ii = ii.ravel()
    jj = jj.ravel()
    bx = (ii == 0) | (ii == n - 1)
    by = (jj == 0) | (jj == n - 1)
    sig = rng.uniform(0.02, 0.2, nbumps)
    cen = rng.uniform(0.0, 1.0, (nbumps, 2))
    amp = rng.uniform(0.05, 0.25, nbumps) * rng.choice([-1.0, 1.0], nbumps)

    def height(p):
        z = np.zeros(p.shape[0])
        for k in range(nbumps):
            d2 = (p[:, 0] - cen[k, 0]) ** 2 + (p[:, 1] - cen[k, 1]) ** 2
            z += amp[k] * np.exp(-d2 / (2.0 * sig[k] ** 2))
        return z

    def draw(idx):
        dx = rng.uniform(-jitter, jitter, idx.size) * h
        dy = rng.uniform(-jitter, jitter, idx.size) * h
        dx[bx[idx]] = 0.0   # left/right boundary: move only along y
        dy[by[idx]] = 0.0   # bottom/top boundary: move only along x
        p = xy[idx].copy()
        p[:, 0] += dx
        p[:, 1] += dy
        return p

    pos = xy.copy()
    allidx = np.arange(n * n)
    pos[allidx] = draw(allidx)
    xyz = np.concatenate([pos, height(pos)[:, None]], axis=1)
    thresh = 1e-3 * h * h / 2.0
    for _ in range(50):
        a = xyz[faces[:, 0]]
        b = xyz[faces[:, 1]]
        c = xyz[faces[:, 2]]
        area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
        bad = area < thresh
        if not bad.any():
            break
        vbad = np.unique(faces[bad].ravel())
        vbad = vbad[~(bx[vbad] & by[vbad])]
        if vbad.size == 0:
            break
        p = draw(vbad)
        xyz[vbad, :2] = p
        xyz[vbad, 2] = height(p)
    return Mesh(f"bump_grid{n}_s{seed}", xyz, faces, meta={"source": 0})


def batch_meshes(seed: int = 3):
    """16 meshes of uneven size: 8 bumpy icospheres and 8 bump grids.

    Icosphere levels 5,5,5,6,6,6,7,7 (20,480 / 81,920 / 327,680 faces);
    grids with n log-uniform in [72, 501] (about 10k to 500k faces).
    Each mesh gets 32 distinct random source vertices (512 fields in all).
    """
    rng = np.random.default_rng(seed)
    out = []
    for i, lvl in enumerate([5, 5, 5, 6, 6, 6, 7, 7]):
        m = bumpy_icosphere(lvl, seed=seed + i)
        out.append(m)
    for i in range(8):
        n = int(round(math.exp(rng.uniform(math.log(72), math.log(501)))))
        m = bump_grid(n, seed=seed + 8 + i)
        out.append(m)
    for i, m in enumerate(out):
        r = np.random.default_rng(seed * 1000 + i)
        m.meta["sources"] = r.choice(m.nv, size=32, replace=False).astype(np.int32)
    return out


def learned_cutoff_sets(seed: int = 4):
    """Training and test meshes for the learned selection cutoff.

    Train: 20 bumpy icospheres (levels 5 and 6, noise seeds 100..119),
    10 random sources each. Test: the 1024^2 bump grid and two more bump
    grid seeds, 8 sources each; the first source of the seed-2 grid is
    vertex 0.
    """
    rng = np.random.default_rng(seed)
    train = []
    for i in range(20):
        lvl = 5 if i % 2 == 0 else 6
        m = bumpy_icosphere(lvl, seed=100 + i)
        m.meta["sources"] = rng.choice(m.nv, size=10, replace=False).astype(np.int32)
        train.append(m)
    test = []
    for s in (2, 20, 21):
        m = bump_grid(1024, seed=s)
        m.meta["sources"] = rng.choice(m.nv, size=8, replace=False).astype(np.int32)
        if s == 2 and 0 not in m.meta["sources"]:
            m.meta["sources"][0] = 0  # the single-field benchmark's first source
        test.append(m)
    return train, test


# ---------------------------------------------------------------------------
# closed-form test surfaces
# ---------------------------------------------------------------------------

def jittered_plane(n: int = 12, seed: int = 0, jitter: float = 0.2) -> Mesh:
    """Planar grid on [0,1]^2 with interior jitter <= 0.2 cell (no flips)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / (n - 1)
    xy = grid_xy(n, n)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    interior = ((ii > 0) & (ii < n - 1) & (jj > 0) & (jj < n - 1)).ravel()
    d = rng.uniform(-jitter, jitter, (n * n, 2)) * h
    xy[interior] += d[interior]
    xyz = np.concatenate([xy, np.zeros((n * n, 1))], axis=1)
    return Mesh(f"plane{n}_s{seed}", xyz, grid_faces(n, n))


def lshape(n: int = 8) -> Mesh:
    """Planar L = [0,2]x[0,1] U [0,1]x[1,2]; reflex corner (1,1) is a vertex.

    Built from the (2n+1)^2 grid on [0,2]^2 with the cells of (1,2]^2 removed.
    """
    m = 2 * n + 1
    xy = grid_xy(m, m, 0.0, 2.0, 0.0, 2.0)
    faces = grid_faces(m, m)
    cen = (xy[faces[:, 0]] + xy[faces[:, 1]] + xy[faces[:, 2]]) / 3.0
    keep = ~((cen[:, 0] > 1.0) & (cen[:, 1] > 1.0))
    faces = faces[keep]
    used = np.unique(faces.ravel())
    remap = -np.ones(m * m, dtype=np.int64)
    remap[used] = np.arange(used.size)
    xyz = np.concatenate([xy[used], np.zeros((used.size, 1))], axis=1)
    return Mesh(f"lshape{n}", xyz, remap[faces].astype(np.int32))


def folded_plane(n: int = 12, seed: int = 0, fold_col: Optional[int] = None) -> Mesh:
    """The jittered plane folded by 90 degrees along a vertical grid line.

    Vertices with x > x_f are rotated about the line x = x_f into the plane
    x = x_f (z grows with x - x_f): the surface is isometric to the plane.
    Jitter is kept off the fold column so the fold line is straight.
    """
    base = jittered_plane(n, seed)
    h = 1.0 / (n - 1)
    if fold_col is None:
        fold_col = n // 2
    xf = fold_col * h
    ii = np.tile(np.arange(n), n)
    xy = base.xyz[:, :2].copy()
    col = ii == fold_col
    xy[col, 0] = xf
    flat = np.concatenate([xy, np.zeros((n * n, 1))], axis=1)
    xyz = flat.copy()
    right = ii > fold_col
    xyz[right, 0] = xf
    xyz[right, 2] = flat[right, 0] - xf
    m = Mesh(f"folded{n}_s{seed}", xyz, base.faces)
    m.meta["flat_xyz"] = flat
    return m


def cube(n: int = 4) -> Mesh:
    """Unit cube [0,1]^3, each face split into an n x n grid of cells."""
    verts = {}
    pts = []
    faces = []

    def vid(p):
        key = tuple(int(round(c * n)) for c in p)
        if key not in verts:
            verts[key] = len(pts)
            pts.append([k / n for k in key])
        return verts[key]

    # (origin, u axis, v axis) with u x v pointing outward
    sides = [
        ((0, 0, 0), (0, 1, 0), (1, 0, 0)),  # z = 0, normal -z
        ((0, 0, 1), (1, 0, 0), (0, 1, 0)),  # z = 1, normal +z
        ((0, 0, 0), (1, 0, 0), (0, 0, 1)),  # y = 0, normal -y
        ((0, 1, 0), (0, 0, 1), (1, 0, 0)),  # y = 1, normal +y
        ((0, 0, 0), (0, 0, 1), (0, 1, 0)),  # x = 0, normal -x
        ((1, 0, 0), (0, 1, 0), (0, 0, 1)),  # x = 1, normal +x
    ]
    for o, u, v in sides:
        o = np.array(o, float)
        u = np.array(u, float)
        v = np.array(v, float)
        for a in range(n):
            for b in range(n):
                p00 = vid(o + (a / n) * u + (b / n) * v)
                p10 = vid(o + ((a + 1) / n) * u + (b / n) * v)
                p11 = vid(o + ((a + 1) / n) * u + ((b + 1) / n) * v)
                p01 = vid(o + (a / n) * u + ((b + 1) / n) * v)
                faces.append([p00, p10, p11])
                faces.append([p00, p11, p01])
    return Mesh(f"cube{n}", np.array(pts, float), np.array(faces, np.int32))


def subdivided_triangle_mesh(base_v: np.ndarray, base_f: np.ndarray, n: int, name: str) -> Mesh:
    """Split each triangle of a base mesh into n^2 congruent triangles."""
    verts = {}
    pts = []

    def key_of(p):
        return tuple(np.round(p * 1e9).astype(np.int64).tolist())

    def vid(p):
        k = key_of(p)
        if k not in verts:
            verts[k] = len(pts)
            pts.append(p)
        return verts[k]

    faces = []
    for f in base_f:
        A, B, C = base_v[f[0]], base_v[f[1]], base_v[f[2]]

        def P(i, j):  # i steps toward B, j toward C
            return A + (B - A) * (i / n) + (C - A) * (j / n)

        for i in range(n):
            for j in range(n - i):
                a = vid(P(i, j))
                b = vid(P(i + 1, j))
                c = vid(P(i, j + 1))
                faces.append([a, b, c])
                if i + j < n - 1:
                    d = vid(P(i + 1, j + 1))
                    faces.append([b, d, c])
    return Mesh(name, np.array(pts, float), np.array(faces, np.int32))


def tetrahedron(n: int = 3, a: float = 1.0) -> Mesh:
    """Regular tetrahedron with edge a, each face split n x n (outward CCW)."""
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    v *= a / (2.0 * math.sqrt(2.0))
    f = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], np.int32)
    m = subdivided_triangle_mesh(v, f, n, f"tetra{n}")
    m.meta["corners"] = v
    return m


def cone_fan(nsect: int, n: int) -> Mesh:
    """Metric-only cone: nsect equilateral triangles (edge 1) around an apex.

    Each triangle is split into n^2 equilateral triangles of edge 1/n, so
    every half-edge length is 1/n. The apex has total angle nsect*pi/3
    (7 -> saddle, 5 -> spherical). ``meta['polar']`` holds each vertex's
    (r, theta) in the unfolded cone.
    """
    # build in an unrolled plane: sector k spans angles [k*pi/3, (k+1)*pi/3]
    verts = {}
    polar = []
    faces = []

    def vid(k, i, j):
        # point = i/n * e_k + j/n * e_{k+1}; i, j >= 0, i + j <= n
        if i == 0 and j == 0:
            key = ("apex",)
        elif j == 0:
            key = ("ray", k % nsect, i)
        elif i == 0:
            key = ("ray", (k + 1) % nsect, j)
        else:
            key = ("in", k, i, j)
        if key not in verts:
            verts[key] = len(polar)
            a0 = k * math.pi / 3.0
            e0 = np.array([math.cos(a0), math.sin(a0)])
            e1 = np.array([math.cos(a0 + math.pi / 3), math.sin(a0 + math.pi / 3)])
            p = (i / n) * e0 + (j / n) * e1
            r = float(np.hypot(p[0], p[1]))
            th = 0.0 if r == 0 else a0 + math.atan2(p[1] * e0[0] - p[0] * e0[1], p @ e0)
            if key[0] == "ray":
                th = key[1] * math.pi / 3.0
            polar.append((r, th))
        return verts[key]

    for k in range(nsect):
        for i in range(n):
            for j in range(n - i):
                a = vid(k, i, j)
                b = vid(k, i + 1, j)
                c = vid(k, i, j + 1)
                faces.append([a, b, c])
                if i + j < n - 1:
                    d = vid(k, i + 1, j + 1)
                    faces.append([b, d, c])
    faces = np.array(faces, np.int32)
    he_len = np.full(3 * faces.shape[0], 1.0 / n)
    m = Mesh(f"cone{nsect}_{n}", None, faces, he_len=he_len, nv=len(polar))
    m.meta["polar"] = np.array(polar)
    m.meta["total_angle"] = nsect * math.pi / 3.0
    return m


def random_tiny_meshes(seed: int = 0, count: int = 6) -> List[Mesh]:
    """Small random meshes (<= 48 faces) for the exhaustive-enumeration check."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        kind = t % 3
        if kind == 0:  # open bumpy grid
            n = int(rng.integers(3, 5))
            xy = grid_xy(n, n)
            xy += rng.uniform(-0.15, 0.15, xy.shape) / (n - 1)
            z = rng.uniform(-0.3, 0.3, n * n) / (n - 1)
            xyz = np.concatenate([xy, z[:, None]], axis=1)
            out.append(Mesh(f"tinygrid{n}_{t}", xyz, grid_faces(n, n)))
        elif kind == 1:  # noisy icosahedron (20 faces, closed)
            v, f = icosahedron()
            v = v * (1.0 + rng.uniform(-0.25, 0.25, 12))[:, None]
            out.append(Mesh(f"tinyico_{t}", v, f))
        else:  # noisy subdivided octahedron-like: icosahedron with 1 level, first 40 faces disk
            v, f = icosahedron()
            v, f = midpoint_subdivide(v, f, project_sphere=True)
            v = v * (1.0 + rng.uniform(-0.15, 0.15, v.shape[0]))[:, None]
            # keep the faces whose centroid has z > -0.2: an open cap (boundary)
            cz = v[f].mean(axis=1)[:, 2]
            f = f[cz > 0.1]
            used = np.unique(f.ravel())
            remap = -np.ones(v.shape[0], np.int64)
            remap[used] = np.arange(used.size)
            out.append(Mesh(f"tinycap_{t}", v[used], remap[f].astype(np.int32)))
    return out


def config_mesh(cfg: int) -> Mesh:
    """The single-field benchmark meshes by configuration number (1..3)."""
    if cfg == 1:
        return sinusoid_grid(64, seed=0)
    if cfg == 2:
        return bumpy_icosphere(7, seed=1)
    if cfg == 3:
        return bump_grid(1024, seed=2)
    raise ValueError(f"no single-mesh configuration {cfg}")
