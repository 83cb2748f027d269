"""Test infrastructure only: iso-contours of a distance field, written from
their definition (only the tests may import this module).

The contour of level c is that of the linear interpolant of the per-vertex
distances over each triangle. A face whose three values are not all on the
same side of c (side: d >= c, decided in FP64) holds one segment; its
endpoints lie on the face's crossing edges, the edges whose two ends are on
different sides, at the fraction t = (c - d_a) / (d_b - d_a) from the edge's
start a to its end b. Edges of face f are the half-edges j = 3 f + k from
faces[f][k] to faces[f][(k + 1) % 3], and the endpoints are listed in that
order of k. Faces with a non-finite vertex value have no interpolant and no
segment.

Pins (tests/test_oracle_isolines.py): a hand-worked triangle, linear fields
(whose contours are straight lines of known length and position) and the
circumference of a cone-shaped field.
"""
from __future__ import annotations

import numpy as np


def isolines(faces: np.ndarray, dist: np.ndarray, levels) -> np.ndarray:
    """All segments as a structured array with fields face, level, j0, t0, j1,
    t1, sorted by (face, level)."""
    faces = np.asarray(faces, dtype=np.int64)
    dist = np.asarray(dist, dtype=np.float64)
    rows = []
    for li, c in enumerate(np.asarray(levels, dtype=np.float64)):
        for f in range(faces.shape[0]):
            d = dist[faces[f]]
            if not np.all(np.isfinite(d)):
                continue
            side = [bool(x >= c) for x in d]
            if side[0] == side[1] == side[2]:
                continue
            ends = []
            for k in range(3):
                a, b = k, (k + 1) % 3
                if side[a] != side[b]:
                    ends.append((3 * f + k, (c - d[a]) / (d[b] - d[a])))
            assert len(ends) == 2
            rows.append((f, li, ends[0][0], ends[0][1], ends[1][0], ends[1][1]))
    out = np.array(rows, dtype=[("face", np.int64), ("level", np.int64), ("j0", np.int64), ("t0", np.float64),
                                ("j1", np.int64), ("t1", np.float64)])
    return np.sort(out, order=["face", "level"])


def endpoints(faces: np.ndarray, xyz: np.ndarray, seg: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """3-D endpoints of the segments: start + t (end - start) of each half-edge."""
    faces = np.asarray(faces, dtype=np.int64)
    xyz = np.asarray(xyz, dtype=np.float64)

    def point(j, t):
        f, k = j // 3, j % 3
        a = xyz[faces[f, k]]
        b = xyz[faces[f, (k + 1) % 3]]
        return a + t[:, None] * (b - a)

    return point(seg["j0"], seg["t0"]), point(seg["j1"], seg["t1"])
