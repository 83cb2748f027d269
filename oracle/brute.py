"""Test infrastructure only: exact geodesic distances on tiny meshes by brute force.

Independent of the window machinery. By the theorem of Mitchell, Mount and
Papadimitriou quoted in Section 3, a shortest path is a polyline whose corners
are mesh vertices and whose pieces are straight in the unfolding of the faces
they cross. So:

1. For every vertex u, enumerate every face sequence that starts at a face of u
   and never repeats a face (a shortest path crosses a convex face once),
   unfolding it into the plane and keeping the cone of directions from u that
   pass through all crossed edges. A vertex c of the next face that lies
   strictly inside the cone is visible from u at the unfolded distance |uc|.
   Mesh edges give the remaining straight pieces.
2. Dijkstra over this visibility graph gives the exact distance at every
   vertex.

Pure Python; meant for meshes of a few dozen faces.
"""
from __future__ import annotations

import heapq
import math
from typing import Dict, List, Tuple

import numpy as np


def _half_edge_tables(faces: np.ndarray, he_len: np.ndarray):
    nf = faces.shape[0]
    start = faces.reshape(-1)
    end = np.roll(faces, -1, axis=1).reshape(-1)
    pair: Dict[Tuple[int, int], int] = {}
    for j in range(3 * nf):
        pair[(int(start[j]), int(end[j]))] = j
    twin = np.full(3 * nf, -1, np.int64)
    for j in range(3 * nf):
        twin[j] = pair.get((int(end[j]), int(start[j])), -1)
    return start, end, twin


def visibility_graph(faces: np.ndarray, he_len: np.ndarray, nv: int, eps: float = 1e-13):
    faces = np.asarray(faces, np.int64)
    start, end, twin = _half_edge_tables(faces, he_len)
    L = {}
    for j in range(3 * faces.shape[0]):
        L[(int(start[j]), int(end[j]))] = float(he_len[j])
        L[(int(end[j]), int(start[j]))] = float(he_len[j])
    vfaces: List[List[int]] = [[] for _ in range(nv)]
    for f in range(faces.shape[0]):
        for v in faces[f]:
            vfaces[int(v)].append(f)

    def cross(a, b):
        return a[0] * b[1] - a[1] * b[0]

    def place(pl, pr, a, b):
        """Third vertex of a triangle on (pl, pr) at distances a from pl, b from
        pr, on the side of line pl-pr away from the origin."""
        ex, ey = pr[0] - pl[0], pr[1] - pl[1]
        Lb = math.hypot(ex, ey)
        x = (Lb * Lb + a * a - b * b) / (2.0 * Lb)
        h = math.sqrt(max(a * a - x * x, 0.0))
        s = -1.0 if cross((ex, ey), (-pl[0], -pl[1])) > 0 else 1.0
        return (pl[0] + x * ex / Lb + s * h * (-ey) / Lb, pl[1] + x * ey / Lb + s * h * ex / Lb)

    def unit(p):
        n = math.hypot(p[0], p[1])
        return (p[0] / n, p[1] / n)

    adj: List[Dict[int, float]] = [dict() for _ in range(nv)]

    def add(u, v, d):
        if v != u and (v not in adj[u] or d < adj[u][v]):
            adj[u][v] = d

    for u in range(nv):
        for f in vfaces[u]:
            tri = [int(x) for x in faces[f]]
            i = tri.index(u)
            a_id, b_id = tri[(i + 1) % 3], tri[(i + 2) % 3]
            lua, lub, lab = L[(u, a_id)], L[(u, b_id)], L[(a_id, b_id)]
            add(u, a_id, lua)
            add(u, b_id, lub)
            pa = (lua, 0.0)
            bx = (lua * lua + lub * lub - lab * lab) / (2.0 * lua)
            pb = (bx, math.sqrt(max(lub * lub - bx * bx, 0.0)))
            # cone from direction of a (right, CW) to direction of b (left, CCW)
            stack = [(f, a_id, b_id, pa, pb, unit(pa), unit(pb), (f,))]
            while stack:
                face, r_id, l_id, pr, pl, dr, dl, seen = stack.pop()
                # cross edge r-l into the neighbour face
                j = None
                for k in range(3):
                    hh = 3 * face + k
                    if int(start[hh]) == r_id and int(end[hh]) == l_id:
                        j = hh
                    elif int(start[hh]) == l_id and int(end[hh]) == r_id:
                        j = hh
                t = int(twin[j])
                if t < 0:
                    continue
                g = t // 3
                if g in seen:
                    continue
                tri2 = [int(x) for x in faces[g]]
                c_id = [x for x in tri2 if x != r_id and x != l_id][0]
                pc = place(pr, pl, L[(r_id, c_id)], L[(l_id, c_id)])
                dc = unit(pc)
                inside_r = cross(dr, dc) > eps
                inside_l = cross(dc, dl) > eps
                if inside_r and inside_l:
                    add(u, c_id, math.hypot(pc[0], pc[1]))
                # sub-cone through edge (r, c): directions from dr to min(dl, dc)
                if inside_r:
                    nl = dc if inside_l else dl
                    stack.append((g, r_id, c_id, pr, pc, dr, nl, seen + (g,)))
                if inside_l:
                    nr = dc if inside_r else dr
                    stack.append((g, c_id, l_id, pc, pl, nr, dl, seen + (g,)))
    return adj


def brute_distances(faces, he_len, nv: int, sources) -> np.ndarray:
    adj = visibility_graph(faces, he_len, nv)
    dist = np.full(nv, np.inf)
    pq = []
    for s in np.atleast_1d(sources):
        dist[int(s)] = 0.0
        pq.append((0.0, int(s)))
    heapq.heapify(pq)
    while pq:
        d, u = heapq.heappop(pq)
        if d > dist[u]:
            continue
        for v, w in adj[u].items():
            nd = d + w
            if nd < dist[v]:
                dist[v] = nd
                heapq.heappush(pq, (nd, v))
    return dist
