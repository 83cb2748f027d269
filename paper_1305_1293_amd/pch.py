"""Python binding of the PCH C ABI (include/pch.h).

Argument marshalling only: meshes and sources are passed as host arrays,
distances come back in a device tensor written by the library's kernels.
torch supplies device memory and the stream. There is no fallback: if
``libpch.so`` is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpch.so")

PCH_SELECT_KTH = 0
PCH_SELECT_DELTA = 1
PCH_SELECT_TABLE = 2
PCH_SELECT_LEARNED = 3
PCH_SELECT_STRIDED = 4

ROUND_LOG_FIELDS = ["N", "cutbits", "shift", "sel", "stale", "kids", "tiny", "ich", "dev", "aev",
                    "fans", "fanwin", "defer", "nend"]

# every entry point declared in include/pch.h
EXPORTS = ["pch_mesh_create", "pch_mesh_create_from_lengths", "pch_mesh_destroy", "pch_mesh_info",
           "pch_mesh_vertex_tables", "pch_options_default", "pch_geodesic", "pch_geodesic_noalloc", "pch_round_log",
           "pch_status_string", "pch_last_error"]


class PchError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pch error {code}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("select_mode", ctypes.c_int32), ("filters", ctypes.c_int32), ("k", ctypes.c_int64),
                ("eps_tiny", ctypes.c_double), ("pool_capacity", ctypes.c_int64),
                ("pool_limit", ctypes.c_int64), ("collect_stats", ctypes.c_int32),
                ("rounds_per_sync", ctypes.c_int32), ("cutoff_table", ctypes.c_void_p),
                ("n_cutoff", ctypes.c_int64), ("collect_timing", ctypes.c_int32), ("hops", ctypes.c_int32),
                ("delta0", ctypes.c_double), ("predicted", ctypes.c_void_p), ("w0", ctypes.c_double),
                ("organize", ctypes.c_int32), ("counts", ctypes.c_int32), ("fuse_hops", ctypes.c_int32),
                ("fuse_scan", ctypes.c_int32), ("round_graph", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ["rounds", "created", "processed", "stale", "tiny", "ich_dropped", "dist_events",
                 "angle_events", "fans", "fan_windows", "deferred", "peak_pool", "restarts"]] + \
               [("ms_total", ctypes.c_double), ("ms_propagate", ctypes.c_double),
                ("propagate_launches", ctypes.c_int64), ("delta0", ctypes.c_double),
                ("hop_launches", ctypes.c_int64), ("ms_phase", ctypes.c_double * 4),
                ("timed_rounds", ctypes.c_int64), ("pool_windows", ctypes.c_int64), ("selected", ctypes.c_int64),
                ("scan_fused", ctypes.c_int32), ("fused_workgroups", ctypes.c_int32)]

    def as_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_}
        d["ms_phase"] = dict(zip(("select", "propagate", "organize", "events"), list(self.ms_phase)))
        return d


_lib = None


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.pch_last_error.restype = ctypes.c_char_p
        L.pch_status_string.restype = ctypes.c_char_p
        L.pch_status_string.argtypes = [ctypes.c_int]
        L.pch_mesh_create.argtypes = [P, i64, P, i64, P, ctypes.POINTER(P)]
        L.pch_mesh_create_from_lengths.argtypes = [P, i64, i64, P, P, ctypes.POINTER(P)]
        L.pch_mesh_destroy.argtypes = [P]
        L.pch_mesh_destroy.restype = None
        L.pch_mesh_info.argtypes = [P, P, P, P, P]
        L.pch_mesh_vertex_tables.argtypes = [P, P, P]
        L.pch_options_default.argtypes = [ctypes.POINTER(Options)]
        L.pch_options_default.restype = None
        L.pch_geodesic.argtypes = [P, P, i32, P, P, ctypes.POINTER(Options), ctypes.POINTER(Stats)]
        L.pch_geodesic_noalloc.argtypes = [P, P, i32, P, P, ctypes.POINTER(Options), ctypes.POINTER(Stats)]
        L.pch_round_log.argtypes = [P, P, i64, P]
        _lib = L
        for n in EXPORTS:
            getattr(L, n)
    return _lib


def _check(rc: int):
    if rc != 0:
        raise PchError(rc, lib().pch_last_error().decode())


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


class Mesh:
    """A mesh uploaded to the current device (owns the library handle)."""

    def __init__(self, faces, xyz=None, he_len=None, nv: Optional[int] = None, stream=None):
        L = lib()
        self.faces = np.ascontiguousarray(faces, dtype=np.int32)
        nf = self.faces.shape[0]
        h = ctypes.c_void_p()
        if xyz is not None:
            xyz = np.ascontiguousarray(xyz, dtype=np.float64)
            self.nv = xyz.shape[0]
            rc = L.pch_mesh_create(xyz.ctypes.data, self.nv, self.faces.ctypes.data, nf,
                                   _stream_handle(stream), ctypes.byref(h))
        else:
            he_len = np.ascontiguousarray(he_len, dtype=np.float64)
            self.nv = int(nv if nv is not None else self.faces.max() + 1)
            rc = L.pch_mesh_create_from_lengths(self.faces.ctypes.data, nf, self.nv, he_len.ctypes.data,
                                                _stream_handle(stream), ctypes.byref(h))
        _check(rc)
        self.handle = h
        self.nf = nf

    @classmethod
    def from_generated(cls, m, stream=None) -> "Mesh":
        if m.xyz is not None:
            return cls(m.faces, xyz=m.xyz, stream=stream)
        return cls(m.faces, he_len=m.he_len, nv=m.nv, stream=stream)

    def info(self) -> dict:
        v = [ctypes.c_int64() for _ in range(4)]
        _check(lib().pch_mesh_info(self.handle, *[ctypes.byref(x) for x in v]))
        return dict(zip(["nv", "nf", "n_boundary_he", "n_pseudo"], [x.value for x in v]))

    def vertex_tables(self):
        th = np.empty(self.nv, np.float64)
        fl = np.empty(self.nv, np.uint8)
        _check(lib().pch_mesh_vertex_tables(self.handle, th.ctypes.data, fl.ctypes.data))
        return th, fl

    def round_log(self) -> np.ndarray:
        n = ctypes.c_int64()
        _check(lib().pch_round_log(self.handle, None, 0, ctypes.byref(n)))
        out = np.zeros((max(n.value, 0), len(ROUND_LOG_FIELDS)), np.int64)
        if n.value:
            _check(lib().pch_round_log(self.handle, out.ctypes.data, n.value, ctypes.byref(n)))
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().pch_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def options(**kw) -> Options:
    o = Options()
    lib().pch_options_default(ctypes.byref(o))
    table = kw.pop("cutoff_table", None)
    predicted = kw.pop("predicted", None)
    if predicted is not None:
        o.select_mode = PCH_SELECT_LEARNED
        o.predicted = predicted.data_ptr() if hasattr(predicted, "data_ptr") else int(predicted)
        o._pred = predicted  # keep alive
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    if table is not None:
        arr = np.ascontiguousarray(table, dtype=np.float64)
        o._table = arr  # keep alive
        o.cutoff_table = arr.ctypes.data
        o.n_cutoff = arr.size
        o.select_mode = PCH_SELECT_TABLE
    return o


def geodesic(mesh: Mesh, sources: Sequence[int], out=None, stream=None, return_stats: bool = False,
             noalloc: bool = False, **opts):
    """Exact geodesic distance from ``sources`` at every vertex (device float64
    tensor). noalloc=True calls pch_geodesic_noalloc (no device allocation in
    the call; pass ``out``)."""
    import torch
    src = np.ascontiguousarray(np.atleast_1d(np.asarray(sources)), dtype=np.int32)
    if out is None:
        out = torch.empty(mesh.nv, dtype=torch.float64, device="cuda")
    if out.dtype != torch.float64 or not out.is_cuda or out.numel() < mesh.nv or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 CUDA tensor with nv elements")
    o = options(**opts)
    st = Stats()
    fn = lib().pch_geodesic_noalloc if noalloc else lib().pch_geodesic
    _check(fn(mesh.handle, src.ctypes.data, src.size, out.data_ptr(), _stream_handle(stream), ctypes.byref(o),
              ctypes.byref(st)))
    return (out, st.as_dict()) if return_stats else out


# ---------------------------------------------------------------------------
# batched fields
# ---------------------------------------------------------------------------

class BatchOptions(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("teams_per_cu", ctypes.c_int32), ("filters", ctypes.c_int32),
                ("eps_tiny", ctypes.c_double), ("pool_capacity", ctypes.c_int64), ("use_graph", ctypes.c_int32),
                ("team_threads", ctypes.c_int32), ("hops", ctypes.c_int32), ("gang", ctypes.c_int32),
                ("wait_ticks", ctypes.c_int64), ("select_mode", ctypes.c_int32), ("predicted", ctypes.c_void_p),
                ("w0", ctypes.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class BatchStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ["fields", "reruns", "max_rounds", "processed", "created", "teams", "k"]] \
        + [("ms_total", ctypes.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


BATCH_FIELD_STATS = ["status", "rounds", "processed", "created", "fans", "peak_pool", "stale", "team_ticks",
                     "helpers", "helper_ticks"]
EXPORTS += ["pch_batch_options_default", "pch_batch_create", "pch_batch_destroy", "pch_batch_offsets",
            "pch_batch_run", "pch_batch_field_stats", "pch_batch_tune", "pch_voronoi", "pch_field_status_string",
            "pch_batch_tune_cached", "pch_tune_cache_save", "pch_tune_cache_load"]
# field status codes (first column of Batch.field_stats)
FIELD_STATUS = {0: "PCH_FIELD_OK", 1: "PCH_FIELD_OVERFLOW", 2: "PCH_FIELD_MAX_ROUNDS", 3: "PCH_FIELD_ABANDONED",
                4: "PCH_FIELD_NOT_RUN", 5: "PCH_FIELD_NONFINITE", 6: "PCH_FIELD_BAD_INDEX"}


def field_status_string(status: int) -> str:
    L = lib()
    L.pch_field_status_string.restype = ctypes.c_char_p
    L.pch_field_status_string.argtypes = [ctypes.c_int64]
    return L.pch_field_status_string(int(status)).decode()


def _batch_lib():
    L = lib()
    if not getattr(L, "_batch_ready", False):
        P, i32 = ctypes.c_void_p, ctypes.c_int32
        L.pch_batch_options_default.argtypes = [ctypes.POINTER(BatchOptions)]
        L.pch_batch_options_default.restype = None
        L.pch_batch_create.argtypes = [P, i32, P, P, i32, ctypes.POINTER(BatchOptions), ctypes.POINTER(P)]
        L.pch_batch_destroy.argtypes = [P]
        L.pch_batch_destroy.restype = None
        L.pch_batch_offsets.argtypes = [P, P]
        L.pch_batch_run.argtypes = [P, P, P, ctypes.POINTER(BatchStats)]
        L.pch_batch_field_stats.argtypes = [P, P]
        L.pch_batch_tune.argtypes = [P, P, P, ctypes.POINTER(BatchOptions)]
        L.pch_voronoi.argtypes = [P, P, i32, P, P, P, ctypes.POINTER(BatchOptions)]
        L.pch_batch_tune_cached.argtypes = [P, P, P, ctypes.POINTER(BatchOptions), ctypes.POINTER(i32)]
        L.pch_tune_cache_save.argtypes = [ctypes.c_char_p]
        L.pch_tune_cache_load.argtypes = [ctypes.c_char_p]
        L._batch_ready = True
    return L


class Batch:
    """Many single-source fields on several meshes in one persistent launch."""

    def __init__(self, meshes: Sequence[Mesh], field_mesh, field_source, **opts):
        L = _batch_lib()
        self.meshes = list(meshes)  # keep the handles alive
        self.field_mesh = np.ascontiguousarray(field_mesh, dtype=np.int32)
        self.field_source = np.ascontiguousarray(field_source, dtype=np.int32)
        if self.field_mesh.shape != self.field_source.shape:
            raise ValueError("field_mesh and field_source differ in length")
        o = BatchOptions()
        L.pch_batch_options_default(ctypes.byref(o))
        predicted = opts.pop("predicted", None)
        if predicted is not None:
            # device float tensor laid out like the output (field f at offsets[f])
            o.select_mode = PCH_SELECT_LEARNED
            o.predicted = predicted.data_ptr() if hasattr(predicted, "data_ptr") else int(predicted)
            self._pred = predicted  # keep alive
        for k, v in opts.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown batch option {k}")
            setattr(o, k, v)
        handles = (ctypes.c_void_p * len(self.meshes))(*[m.handle for m in self.meshes])
        h = ctypes.c_void_p()
        _check(L.pch_batch_create(handles, len(self.meshes), self.field_mesh.ctypes.data,
                                  self.field_source.ctypes.data, self.field_mesh.size, ctypes.byref(o),
                                  ctypes.byref(h)))
        self.handle = h
        self.n_fields = int(self.field_mesh.size)
        off = np.zeros(self.n_fields + 1, np.int64)
        _check(L.pch_batch_offsets(self.handle, off.ctypes.data))
        self.offsets = off

    def empty_output(self):
        import torch
        return torch.empty(int(self.offsets[-1]), dtype=torch.float64, device="cuda")

    def run(self, out=None, stream=None):
        """All fields into one device tensor (field f at offsets[f]:offsets[f+1])."""
        if out is None:
            out = self.empty_output()
        st = BatchStats()
        _check(_batch_lib().pch_batch_run(self.handle, out.data_ptr(), _stream_handle(stream), ctypes.byref(st)))
        return out, st.as_dict()

    def field(self, out, f):
        return out[int(self.offsets[f]):int(self.offsets[f + 1])]

    def field_stats(self) -> np.ndarray:
        fs = np.zeros((self.n_fields, len(BATCH_FIELD_STATS)), np.int64)
        _check(_batch_lib().pch_batch_field_stats(self.handle, fs.ctypes.data))
        return fs

    def tune_cached(self, out=None, stream=None):
        """The tuner's recorded choice for this batch's size bucket, or a
        tuning run when there is none; returns (options, hit)."""
        if out is None:
            out = self.empty_output()
        o = BatchOptions()
        hit = ctypes.c_int32()
        _check(_batch_lib().pch_batch_tune_cached(self.handle, out.data_ptr(), _stream_handle(stream), ctypes.byref(o),
                                                  ctypes.byref(hit)))
        return o.as_dict(), bool(hit.value)

    def tune(self, out=None, stream=None) -> dict:
        if out is None:
            out = self.empty_output()
        o = BatchOptions()
        _check(_batch_lib().pch_batch_tune(self.handle, out.data_ptr(), _stream_handle(stream), ctypes.byref(o)))
        return o.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            _batch_lib().pch_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def voronoi(mesh: Mesh, sources, stream=None, **opts):
    """Geodesic Voronoi labels: per vertex the index of the nearest of
    ``sources`` (-1 if none reaches it) and the distance to it, from the
    single-source fields of all sources in one batched launch. Batch options
    default to k 16384, 512-thread teams, 4 hops, up to 16 workgroups per
    field."""
    import torch
    L = _batch_lib()
    src = np.ascontiguousarray(np.atleast_1d(np.asarray(sources)), dtype=np.int32)
    o = BatchOptions()
    L.pch_batch_options_default(ctypes.byref(o))
    for k, v in dict(dict(k=16384, team_threads=512, teams_per_cu=1, hops=4, gang=16), **opts).items():
        if not hasattr(o, k):
            raise TypeError(f"unknown batch option {k}")
        setattr(o, k, v)
    nv = int(mesh.nv)
    dist = torch.empty(nv, dtype=torch.float64, device="cuda")
    label = torch.empty(nv, dtype=torch.int32, device="cuda")
    _check(L.pch_voronoi(mesh.handle, src.ctypes.data, src.size, dist.data_ptr(), label.data_ptr(),
                         _stream_handle(stream), ctypes.byref(o)))
    return dist, label


# ---------------------------------------------------------------------------
# iso-contours
# ---------------------------------------------------------------------------

ISO_MAX_LEVELS = 64
EXPORTS += ["pch_isolines"]


def isolines(faces, dist, levels, cap=None, stream=None):
    """Iso-contour segments of the distance field ``dist`` (device float64
    [nv]) over the mesh ``faces`` (device int32 [nf, 3]) at ``levels``, on the
    linear interpolant of each face. Returns device tensors (he [n, 2] int32,
    t [n, 2] float64, level [n] int32): segment i runs from the point at
    fraction t[i, 0] along half-edge he[i, 0] (half-edge j = 3 f + k of face f
    starts at faces[f, k] and ends at faces[f, (k + 1) % 3]) to the point at
    t[i, 1] along he[i, 1]; level[i] indexes ``levels``."""
    import torch
    L = lib()
    if not getattr(L, "_iso_ready", False):
        P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.pch_isolines.argtypes = [P, i64, i64, P, P, i32, P, P, P, i64, ctypes.POINTER(i64), P]
        L._iso_ready = True
    if faces.dtype != torch.int32 or not faces.is_cuda or not faces.is_contiguous() or faces.dim() != 2 \
            or faces.shape[1] != 3:
        raise ValueError("faces must be a contiguous int32 CUDA tensor [nf, 3]")
    if dist.dtype != torch.float64 or not dist.is_cuda or not dist.is_contiguous():
        raise ValueError("dist must be a contiguous float64 CUDA tensor")
    lv = np.ascontiguousarray(np.atleast_1d(np.asarray(levels, dtype=np.float64)))
    nf = int(faces.shape[0])
    if cap is None:
        cap = nf * lv.size
    he = torch.empty((max(cap, 1), 2), dtype=torch.int32, device="cuda")
    t = torch.empty((max(cap, 1), 2), dtype=torch.float64, device="cuda")
    lev = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    n = ctypes.c_int64()
    _check(L.pch_isolines(faces.data_ptr(), nf, int(dist.numel()), dist.data_ptr(), lv.ctypes.data, int(lv.size),
                          he.data_ptr(), t.data_ptr(), lev.data_ptr(), int(cap), ctypes.byref(n),
                          _stream_handle(stream)))
    k = int(n.value)
    return he[:k], t[:k], lev[:k]


# ---------------------------------------------------------------------------
# learned distance predictor
# ---------------------------------------------------------------------------

MLP_NPARAM = 4737
EXPORTS += ["pch_mlp_create", "pch_mlp_destroy", "pch_mlp_get_params", "pch_mlp_set_params", "pch_mlp_features",
            "pch_mlp_forward", "pch_mlp_gradients", "pch_mlp_train_step"]


def _mlp_lib():
    L = lib()
    if not getattr(L, "_mlp_ready", False):
        P, i64, i32, f, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_double
        L.pch_mlp_create.argtypes = [ctypes.c_uint64, ctypes.POINTER(P)]
        L.pch_mlp_destroy.argtypes = [P]
        L.pch_mlp_destroy.restype = None
        L.pch_mlp_get_params.argtypes = [P, P]
        L.pch_mlp_set_params.argtypes = [P, P]
        L.pch_mlp_features.argtypes = [P, i64, i32, P, d, P, P, P]
        L.pch_mlp_forward.argtypes = [P, P, P, i64, P, P]
        L.pch_mlp_gradients.argtypes = [P, P, P, P, P, i64, P, P, P]
        L.pch_mlp_train_step.argtypes = [P, P, P, P, P, i64, f, f, P, P]
        L._mlp_ready = True
    return L


class MLP:
    """Device-resident distance predictor (7 -> 64 -> 64 -> 1)."""

    def __init__(self, seed: int = 0):
        h = ctypes.c_void_p()
        _check(_mlp_lib().pch_mlp_create(seed, ctypes.byref(h)))
        self.handle = h

    def get_params(self) -> np.ndarray:
        p = np.empty(MLP_NPARAM, np.float32)
        _check(_mlp_lib().pch_mlp_get_params(self.handle, p.ctypes.data))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == MLP_NPARAM
        _check(_mlp_lib().pch_mlp_set_params(self.handle, p.ctypes.data))

    @staticmethod
    def features(xyz_dev, source: int, center, radius: float, stream=None, feats=None, base=None):
        """Features [nv, 7] and chord lengths [nv] of one field; feats and
        base may be given (contiguous float32 device views of those shapes,
        for instance slices of one buffer holding many fields)."""
        import torch
        nv = int(xyz_dev.shape[0])
        if feats is None:
            feats = torch.empty((nv, 7), dtype=torch.float32, device=xyz_dev.device)
        if base is None:
            base = torch.empty(nv, dtype=torch.float32, device=xyz_dev.device)
        if tuple(feats.shape) != (nv, 7) or tuple(base.shape) != (nv,) or not (feats.is_contiguous()
                                                                              and base.is_contiguous()):
            raise ValueError("feats must be a contiguous [nv, 7] and base a contiguous [nv] float32 tensor")
        if feats.dtype != torch.float32 or base.dtype != torch.float32:
            raise ValueError("feats and base must be float32")
        c = np.ascontiguousarray(center, dtype=np.float64)
        _check(_mlp_lib().pch_mlp_features(xyz_dev.data_ptr(), nv, int(source), c.ctypes.data, float(radius),
                                           feats.data_ptr(), base.data_ptr(), _stream_handle(stream)))
        return feats, base

    def forward(self, feats, base, stream=None, out=None):
        import torch
        n = int(feats.shape[0])
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=feats.device)
        if tuple(out.shape) != (n,) or out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor of the samples' count")
        _check(_mlp_lib().pch_mlp_forward(self.handle, feats.data_ptr(), base.data_ptr(), n, out.data_ptr(),
                                          _stream_handle(stream)))
        return out

    def gradients(self, feats, base, target, scale, stream=None):
        g = np.empty(MLP_NPARAM, np.float32)
        loss = ctypes.c_float()
        _check(_mlp_lib().pch_mlp_gradients(self.handle, feats.data_ptr(), base.data_ptr(), target.data_ptr(),
                                            scale.data_ptr(), int(feats.shape[0]), g.ctypes.data, ctypes.byref(loss),
                                            _stream_handle(stream)))
        return float(loss.value), g

    def train_step(self, feats, base, target, scale, lr=1e-3, weight_decay=1e-4, want_loss=False, stream=None):
        loss = ctypes.c_float()
        _check(_mlp_lib().pch_mlp_train_step(self.handle, feats.data_ptr(), base.data_ptr(), target.data_ptr(),
                                             scale.data_ptr(), int(feats.shape[0]), float(lr), float(weight_decay),
                                             ctypes.byref(loss) if want_loss else None, _stream_handle(stream)))
        return float(loss.value) if want_loss else None

    def close(self):
        if getattr(self, "handle", None):
            _mlp_lib().pch_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_cache_save(path: str):
    _check(_batch_lib().pch_tune_cache_save(path.encode()))


def tune_cache_load(path: str):
    _check(_batch_lib().pch_tune_cache_load(path.encode()))
