"""Test infrastructure only: ctypes wrapper of the CPU oracle library.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this module. ``build()`` compiles ``mesh.cpp``, ``ich.cpp`` and
``pch_oracle.cpp`` with g++ (FP contraction off, no fast-math) into
``liboracle.so`` next to this file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, f) for f in ("mesh.cpp", "ich.cpp", "pch_oracle.cpp")]
LIB = os.path.join(HERE, "liboracle.so")

# per-round log columns written by orc_replica
RL_FIELDS = ["N", "cutbits", "shift", "sel", "stale", "kids", "tiny", "ich", "dev", "aev",
             "fans", "fanwin", "defer", "nend"]
STAT_FIELDS = ["created", "processed", "stale", "tiny", "ich", "updates", "angle_updates", "fans",
               "fan_windows", "rounds", "peak", "notwin", "deferred"]

_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
               "-o", LIB + ".tmp", *SRCS]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        i32 = ctypes.c_int32
        d = ctypes.c_double
        L.orc_last_error.restype = ctypes.c_char_p
        L.orc_lengths.argtypes = [P, i64, P, i64, P]
        L.orc_mesh_info.argtypes = [P, i64, i64, P, P, P, P, P, P, P, P]
        L.orc_ich.argtypes = [P, i64, i64, P, P, i32, d, i32, P, P]
        L.orc_ich_bounded.argtypes = [P, i64, i64, P, P, i32, d, i32, i64, P, P]
        L.orc_replica.argtypes = [P, i64, i64, P, P, i32, i64, i32, d, i32, i32, d, P, i64, P, P, P, i64, P, P]
        L.orc_dijkstra.argtypes = [P, i64, i64, P, P, i32, P]
        L.orc_fn_atan2.argtypes = [d, d]
        L.orc_fn_atan2.restype = d
        L.orc_fn_sincos.argtypes = [d, P, P]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != 0:
        raise OracleError(rc, lib().orc_last_error().decode())


def lengths(mesh) -> np.ndarray:
    """Per-half-edge lengths of a mesh (given, or from its coordinates)."""
    if mesh.he_len is not None:
        return np.ascontiguousarray(mesh.he_len, np.float64)
    out = np.empty(3 * mesh.nf, np.float64)
    _check(lib().orc_lengths(_ptr(mesh.xyz), mesh.nv, _ptr(mesh.faces), mesh.nf, _ptr(out)))
    return out


def mesh_info(mesh) -> dict:
    nh = 3 * mesh.nf
    he = lengths(mesh)
    out = dict(twin=np.empty(nh, np.int32), ax=np.empty(nh), ay=np.empty(nh), alpha=np.empty(nh),
               phi=np.empty(nh), theta=np.empty(mesh.nv), flags=np.empty(mesh.nv, np.uint8))
    _check(lib().orc_mesh_info(_ptr(mesh.faces), mesh.nf, mesh.nv, _ptr(he), _ptr(out["twin"]), _ptr(out["ax"]),
                               _ptr(out["ay"]), _ptr(out["alpha"]), _ptr(out["phi"]), _ptr(out["theta"]),
                               _ptr(out["flags"])))
    out["boundary"] = (out["flags"] & 1).astype(bool)
    out["pseudo"] = (out["flags"] & 2).astype(bool)
    out["he_len"] = he
    return out


def _sources(sources) -> np.ndarray:
    return np.ascontiguousarray(np.atleast_1d(np.asarray(sources)), dtype=np.int32)


def ich(mesh, sources, eps_tiny: float = 0.0, filters: int = 3, max_processed: int = 0):
    """Exact distance field by sequential ICH.

    filters: bit 0 the CH one-angle-one-split rule, bit 1 the ICH window
    filter, bit 2 full fans (every direction at a pseudo-source).
    max_processed > 0 stops after that many propagated windows: a bounded
    sample of the run for timing, whose distances are incomplete.
    """
    s = _sources(sources)
    he = lengths(mesh)
    dist = np.empty(mesh.nv, np.float64)
    stats = np.zeros(16, np.int64)
    _check(lib().orc_ich_bounded(_ptr(mesh.faces), mesh.nf, mesh.nv, _ptr(he), _ptr(s), s.size, eps_tiny, filters,
                                 int(max_processed), _ptr(dist), _ptr(stats)))
    return dist, dict(zip(STAT_FIELDS, stats.tolist()))


def replica(mesh, sources, k: int, eps_tiny: float = 0.0, filters: int = 3, cutoffs=None,
            max_log: int = 1 << 16, vertex_updates: Optional[np.ndarray] = None, mode: int = 0,
            delta0: float = 0.0, hops: int = 1):
    """Round-based PCH with delayed updates; returns (dist, stats, round_log).

    mode 0 selects the k smallest keys each round; mode 1 selects keys up to
    the pool's smallest key plus an adaptive step that starts at ``delta0``.
    ``cutoffs`` (optional float64 array) replaces the rule of round r by
    ``cutoffs[r]`` (select key <= cutoff) for as many rounds as it holds.
    ``hops`` > 1 lets children that pass the round's selection test propagate
    again within the round (up to ``hops`` propagations), against the same
    round-start snapshot; the log's selected count covers every hop.
    """
    s = _sources(sources)
    he = lengths(mesh)
    dist = np.empty(mesh.nv, np.float64)
    stats = np.zeros(16, np.int64)
    rlog = np.zeros((max_log, len(RL_FIELDS)), np.int64)
    nr = np.zeros(1, np.int64)
    ct = None if cutoffs is None else np.ascontiguousarray(cutoffs, np.float64)
    _check(lib().orc_replica(_ptr(mesh.faces), mesh.nf, mesh.nv, _ptr(he), _ptr(s), s.size, int(k), int(hops), eps_tiny,
                             filters, int(mode), float(delta0), _ptr(ct), 0 if ct is None else ct.size, _ptr(dist),
                             _ptr(stats), _ptr(rlog),
                             max_log, _ptr(nr), _ptr(vertex_updates)))
    n = int(nr[0])
    return dist, dict(zip(STAT_FIELDS, stats.tolist())), rlog[:min(n, max_log)]


def dijkstra(mesh, sources) -> np.ndarray:
    s = _sources(sources)
    he = lengths(mesh)
    dist = np.empty(mesh.nv, np.float64)
    _check(lib().orc_dijkstra(_ptr(mesh.faces), mesh.nf, mesh.nv, _ptr(he), _ptr(s), s.size, _ptr(dist)))
    return dist


def fn_atan2(y: float, x: float) -> float:
    return lib().orc_fn_atan2(y, x)


def fn_sincos(t: float):
    s = ctypes.c_double()
    c = ctypes.c_double()
    lib().orc_fn_sincos(t, ctypes.byref(s), ctypes.byref(c))
    return s.value, c.value
