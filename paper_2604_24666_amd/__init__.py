"""Python binding of libnif (the deformation-aware neural intersection function on MI355X).

Argument marshalling only: every function below forwards to the C ABI of the same name in
libnif.so (declared in include/nif.h); all computation runs in the library's HIP kernels.
PyTorch supplies device memory (tensors) and the stream (torch.cuda.current_stream()).

The library must be built first (`python -m paper_2604_24666_amd.build`); importing this
package on a machine without it, or calling into it without a GPU, raises immediately -
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

import torch

__all__ = ["NifError", "lib", "ModelDesc", "Pose", "Rays", "Hits", "Segments", "Batch", "TrainCfg",
           "nif_model_create", "nif_model_destroy", "nif_model_sizes", "nif_model_set_params",
           "nif_model_get_params", "nif_model_get_grads", "nif_model_zero_grads", "nif_model_reserve",
           "nif_model_reserve_encoding",
           "nif_voxelize", "nif_label", "nif_label_noalloc", "nif_build_grid", "nif_grid_destroy", "nif_grid_info", "nif_grid_bounds", "nif_grid_update", "nif_trace", "nif_query", "nif_set_query_blocks_per_cu", "nif_wall_clock_khz", "nif_microbench",
           "nif_encode", "nif_forward", "nif_backward", "nif_train_step", "nif_loss",
           "Model", "Grid", "NifField", "NifMultiTaskLoss", "label"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnif.so")

PREC_FP32, PREC_BF16, PREC_FP16 = 0, 1, 2
DIST_LOG_RELU, DIST_SIGMOID = 0, 1
TABLE_F32, TABLE_F16 = 0, 1
Q_FIRST_HIT, Q_NO_NETWORK, Q_POSE_TIMES, Q_POSE_ORDER = 0, 8, 16, 32


class NifError(RuntimeError):
    pass


class ModelDesc(C.Structure):
    _fields_ = [("levels", C.c_int32), ("log2_table", C.c_int32), ("feat_dim", C.c_int32),
                ("table_dtype", C.c_int32), ("res", C.c_int32 * 32), ("pe_freqs", C.c_int32),
                ("hidden_width", C.c_int32), ("hidden_layers", C.c_int32), ("n_materials", C.c_int32),
                ("dist_head", C.c_int32), ("per_sample_tables", C.c_int32), ("concat_encoding", C.c_int32)]


class Pose(C.Structure):
    _fields_ = [("kind", C.c_int32), ("strength", C.c_float)]


class Rays(C.Structure):
    _fields_ = [("ox", C.c_void_p), ("oy", C.c_void_p), ("oz", C.c_void_p), ("dx", C.c_void_p),
                ("dy", C.c_void_p), ("dz", C.c_void_p), ("pose_offsets", C.c_void_p), ("tmax", C.c_void_p)]


class Segments(C.Structure):
    _fields_ = [("count", C.c_void_p), ("cell", C.c_void_p), ("t_in", C.c_void_p), ("t_out", C.c_void_p),
                ("x0", C.c_void_p), ("x1", C.c_void_p)]


class Hits(C.Structure):
    _fields_ = [("hit", C.c_void_p), ("t", C.c_void_p), ("nx", C.c_void_p), ("ny", C.c_void_p),
                ("nz", C.c_void_p), ("ar", C.c_void_p), ("ag", C.c_void_p), ("ab", C.c_void_p),
                ("material", C.c_void_p), ("cell", C.c_void_p), ("hit_logit", C.c_void_p),
                ("n_queried", C.c_void_p), ("xr", C.c_void_p), ("yr", C.c_void_p), ("zr", C.c_void_p),
                ("dnx", C.c_void_p), ("dny", C.c_void_p), ("dnz", C.c_void_p)]


class Batch(C.Structure):
    _fields_ = [("x0", C.c_void_p), ("x1", C.c_void_p), ("hit", C.c_void_p), ("t", C.c_void_p),
                ("n", C.c_void_p), ("a", C.c_void_p), ("m", C.c_void_p)]


class TrainCfg(C.Structure):
    _fields_ = [("lr_table", C.c_float), ("lr_mlp", C.c_float), ("lr_s", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("precision", C.c_int32),
                ("loss_scale_init", C.c_float), ("fixed_task_weights", C.c_int32), ("store_encoding", C.c_int32),
                ("loss_scale_growth_interval", C.c_int32)]


_lib = None


def lib():
    """The loaded libnif.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NifError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_24666_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, U32, F = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_float
        sigs = {
            "nif_status_string": ([C.c_int], C.c_char_p), "nif_last_error": ([], C.c_char_p),
            "nif_version": ([], C.c_int),
            "nif_model_create": ([P, P], C.c_int), "nif_model_destroy": ([P], C.c_int),
            "nif_model_sizes": ([P, P, P], C.c_int),
            "nif_model_set_params": ([P, P, P, P, P], C.c_int),
            "nif_model_get_params": ([P, P, P, P, P], C.c_int),
            "nif_model_get_grads": ([P, P, P, P, P], C.c_int),
            "nif_model_zero_grads": ([P, P], C.c_int), "nif_model_reserve": ([P, I64], C.c_int),
            "nif_model_reserve_encoding": ([P], C.c_int),
            "nif_voxelize": ([I32, P, I32, I32, P, P], C.c_int),
            "nif_label": ([I32, P, I32, I32, P, P, C.c_int64, P, P, P, P, P, P], C.c_int),
            "nif_label_noalloc": ([I32, P, I32, I32, P, P, C.c_int64, P, P, P, P, P, P], C.c_int),
            "nif_build_grid": ([P, I32, P, I32, I32, P, P], C.c_int), "nif_grid_destroy": ([P], C.c_int),
            "nif_grid_info": ([P, I32, P, P, P], C.c_int), "nif_grid_bounds": ([P, I32, P, P], C.c_int), "nif_grid_update": ([P, P, I32, P], C.c_int),
            "nif_trace": ([P, P, I64, I32, P, P], C.c_int),
            "nif_query": ([P, P, P, I64, P, U32, I32, P, P], C.c_int),
            "nif_set_query_blocks_per_cu": ([I32], C.c_int), "nif_set_query_rays_per_wave": ([I32], C.c_int),
            "nif_autotune_query": ([P, P, P, I64, P, I32, I32, P, P, P], C.c_int),
            "nif_wall_clock_khz": ([C.POINTER(C.c_int32)], C.c_int),
            "nif_microbench": ([I32, I64, I64, I32, P, P], C.c_int),
            "nif_encode": ([P, P, I64, P, P], C.c_int),
            "nif_forward": ([P, P, P, I64, P, I32, P], C.c_int),
            "nif_backward": ([P, P, P, I64, P, P, P, I32, I32, P], C.c_int),
            "nif_train_step": ([P, P, I64, P, P, P], C.c_int),
            "nif_loss": ([P, P, I64, P, P, I32, P, P, P, P], C.c_int),
        }
        for name, (args, res) in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        L = lib()
        raise NifError(f"{L.nif_status_string(rc).decode()}: {L.nif_last_error().decode()}")


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ thin wrappers (same names)

def nif_model_sizes(desc: ModelDesc):
    nt, nm = C.c_int64(), C.c_int64()
    _check(lib().nif_model_sizes(C.byref(desc), C.byref(nt), C.byref(nm)))
    return nt.value, nm.value


def nif_model_create(desc: ModelDesc):
    h = C.c_void_p()
    _check(lib().nif_model_create(C.byref(desc), C.byref(h)))
    return h


def nif_model_destroy(h):
    _check(lib().nif_model_destroy(h))


def nif_model_set_params(h, tables, mlp, s=None, stream=None):
    _check(lib().nif_model_set_params(h, _ptr(tables), _ptr(mlp), _ptr(s), _stream(stream)))


def nif_model_get_params(h, tables=None, mlp=None, s=None, stream=None):
    _check(lib().nif_model_get_params(h, _ptr(tables), _ptr(mlp), _ptr(s), _stream(stream)))


def nif_model_get_grads(h, g_tables=None, g_mlp=None, g_s=None, stream=None):
    _check(lib().nif_model_get_grads(h, _ptr(g_tables), _ptr(g_mlp), _ptr(g_s), _stream(stream)))


def nif_model_zero_grads(h, stream=None):
    _check(lib().nif_model_zero_grads(h, _stream(stream)))


def nif_model_reserve(h, max_batch: int):
    _check(lib().nif_model_reserve(h, C.c_int64(max_batch)))


def nif_model_reserve_encoding(h):
    """Stored-encoding buffer for training steps with store_encoding = 1."""
    _check(lib().nif_model_reserve_encoding(h))


def nif_voxelize(scene_kind: int, params, N: int, occ, stream=None):
    import numpy as np
    p = np.ascontiguousarray(params, dtype=np.float64)
    _check(lib().nif_voxelize(scene_kind, p.ctypes.data_as(C.c_void_p), len(p), N, _ptr(occ), _stream(stream)))


def nif_label(scene_kind: int, params, x0, x1, n: int, hit=None, t=None, normal=None, albedo=None, material=None,
              force_march: bool = False, stream=None):
    import numpy as np
    p = np.ascontiguousarray(params, dtype=np.float64)
    _check(lib().nif_label(scene_kind, p.ctypes.data_as(C.c_void_p), len(p), int(force_march), _ptr(x0), _ptr(x1), n,
                           _ptr(hit), _ptr(t), _ptr(normal), _ptr(albedo), _ptr(material), _stream(stream)))


def nif_label_noalloc(scene_kind: int, params, x0, x1, n: int, hit=None, t=None, normal=None, albedo=None,
                      material=None, force_march: bool = False, stream=None):
    """nif_label without allocation or synchronisation (scene parameters staged in the
    library's fixed per-device array, at most NIF_LABEL_NOALLOC_MAX_PARAMS values)."""
    import numpy as np
    p = np.ascontiguousarray(params, dtype=np.float64)
    _check(lib().nif_label_noalloc(scene_kind, p.ctypes.data_as(C.c_void_p), len(p), int(force_march), _ptr(x0),
                                   _ptr(x1), n, _ptr(hit), _ptr(t), _ptr(normal), _ptr(albedo), _ptr(material),
                                   _stream(stream)))


LABEL_NOALLOC_MAX_PARAMS = 4104


def label(scene_kind: int, params, x0, x1, force_march: bool = False):
    """Labels of rest segments x0, x1 (float32 [3][n] device tensors): dict of device tensors."""
    n = x0.shape[1]
    dev = x0.device
    out = dict(hit=torch.empty(n, dtype=torch.uint8, device=dev), t=torch.empty(n, device=dev),
               normal=torch.empty((3, n), device=dev), albedo=torch.empty((3, n), device=dev),
               material=torch.empty(n, dtype=torch.int32, device=dev))
    nif_label(scene_kind, params, x0, x1, n, out["hit"], out["t"], out["normal"], out["albedo"], out["material"],
              force_march)
    return out


def nif_build_grid(occ, N: int, kinds, strengths, bins_per_axis: int = 0, stream=None):
    n = len(kinds)
    poses = (Pose * n)(*[Pose(int(k), float(s)) for k, s in zip(kinds, strengths)])
    h = C.c_void_p()
    _check(lib().nif_build_grid(_ptr(occ), N, poses, n, bins_per_axis, C.byref(h), _stream(stream)))
    return h


def nif_grid_destroy(h):
    _check(lib().nif_grid_destroy(h))


def nif_grid_info(h, pose: int = 0):
    """(occupied voxels, bin-list entries of the pose at build, overflow flag of the last update)."""
    a, b, c = C.c_int64(), C.c_int64(), C.c_int32()
    _check(lib().nif_grid_info(h, pose, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def nif_grid_bounds(h, pose: int = 0):
    """Deformed-space box (lo[3], hi[3]) of a pose's occupied voxels."""
    lo, hi = (C.c_float * 3)(), (C.c_float * 3)()
    _check(lib().nif_grid_bounds(h, pose, lo, hi))
    return np.array(lo[:]), np.array(hi[:])


def nif_grid_update(h, kinds, strengths, stream=None):
    n = len(kinds)
    poses = (Pose * n)(*[Pose(int(k), float(s)) for k, s in zip(kinds, strengths)])
    _check(lib().nif_grid_update(h, poses, n, _stream(stream)))


def make_rays(o, d, pose_offsets, tmax=None) -> Rays:
    """o, d: float32 [3][n] device tensors; pose_offsets: int64 [P+1] device tensor;
    tmax: optional float32 [n] device tensor (occlusion bound of each ray)."""
    r = Rays(o[0].data_ptr(), o[1].data_ptr(), o[2].data_ptr(), d[0].data_ptr(), d[1].data_ptr(),
             d[2].data_ptr(), pose_offsets.data_ptr(), _ptr(tmax))
    r._keep = (o, d, pose_offsets, tmax)        # the struct holds raw pointers: keep the tensors alive
    return r


def nif_trace(grid, rays: Rays, n: int, max_seg: int, seg: Segments, stream=None):
    _check(lib().nif_trace(grid, C.byref(rays), n, max_seg, C.byref(seg), _stream(stream)))


def nif_query(model, grid, rays: Rays, n: int, hits: Hits, flags: int = 0, precision: int = 0, stats=None,
              stream=None):
    _check(lib().nif_query(model, grid, C.byref(rays), n, C.byref(hits), flags, precision, _ptr(stats),
                           _stream(stream)))


MB_HBM_READ, MB_GATHER4, MB_GATHER8, MB_MFMA_F32, MB_MFMA_BF16 = 0, 1, 2, 3, 4


def nif_microbench(kind: int, n_bytes: int, n_ops: int, reps: int = 5, stream=None):
    """(rate, ms per launch) of one device-ceiling microbenchmark (bytes/s or FLOP/s)."""
    r = (C.c_double * 2)()
    _check(lib().nif_microbench(int(kind), int(n_bytes), int(n_ops), int(reps), r, _stream(stream)))
    return r[0], r[1]


def nif_wall_clock_khz() -> int:
    v = C.c_int32(0)
    _check(lib().nif_wall_clock_khz(C.byref(v)))
    return int(v.value)


def nif_set_query_blocks_per_cu(v: int):
    _check(lib().nif_set_query_blocks_per_cu(int(v)))


def nif_autotune_query(model, grid, rays: Rays, n: int, hits: Hits, precision: int = 0, reps: int = 2,
                       stream=None):
    """Times the launch shapes of the fused query on these rays and keeps the fastest;
    returns (workgroups per CU, rays per wave, ms per launch)."""
    best = (C.c_int32 * 2)()
    ms = C.c_float()
    _check(lib().nif_autotune_query(model, grid, C.byref(rays), n, C.byref(hits), precision, reps, best,
                                    C.byref(ms), _stream(stream)))
    return int(best[0]), int(best[1]), float(ms.value)


def nif_set_query_rays_per_wave(v: int):
    """0 = by launch size, else 16 or 64 rays per wave of the fused query."""
    _check(lib().nif_set_query_rays_per_wave(int(v)))


def nif_encode(model, x, n: int, out, stream=None):
    _check(lib().nif_encode(model, _ptr(x), n, _ptr(out), _stream(stream)))


def nif_forward(model, x0, x1, B: int, heads, precision: int = 0, stream=None):
    _check(lib().nif_forward(model, _ptr(x0), _ptr(x1), B, _ptr(heads), precision, _stream(stream)))


def nif_backward(model, x0, x1, B: int, d_heads, d_x0=None, d_x1=None, accumulate: bool = False,
                 precision: int = 0, stream=None):
    _check(lib().nif_backward(model, _ptr(x0), _ptr(x1), B, _ptr(d_heads), _ptr(d_x0), _ptr(d_x1),
                              int(accumulate), precision, _stream(stream)))


def nif_train_step(model, batch: Batch, B: int, cfg: TrainCfg, losses, stream=None):
    _check(lib().nif_train_step(model, C.byref(batch), B, C.byref(cfg), _ptr(losses), _stream(stream)))


def nif_loss(model, heads, B: int, labels: Batch, s, fixed: bool, losses, d_heads=None, d_s=None, stream=None):
    _check(lib().nif_loss(model, _ptr(heads), B, C.byref(labels), _ptr(s), int(fixed), _ptr(losses), _ptr(d_heads),
                          _ptr(d_s), _stream(stream)))


# ------------------------------------------------------------------ convenience objects

def model_desc(levels, log2_table, feat_dim, table_dtype, res, pe_freqs, hidden_width, hidden_layers,
               n_materials, dist_head=0, per_sample_tables=0, concat_encoding=0) -> ModelDesc:
    d = ModelDesc()
    d.levels, d.log2_table, d.feat_dim, d.table_dtype = levels, log2_table, feat_dim, table_dtype
    for i, r in enumerate(res):
        d.res[i] = int(r)
    d.pe_freqs, d.hidden_width, d.hidden_layers, d.n_materials = pe_freqs, hidden_width, hidden_layers, n_materials
    d.dist_head = dist_head
    d.per_sample_tables = per_sample_tables
    d.concat_encoding = concat_encoding
    return d


class Model:
    """Owns a nif_model handle.  `m` is any object with the ModelDesc attributes."""

    def __init__(self, m, device="cuda", max_batch: int = 0):
        self.spec = m
        self.desc = model_desc(m.levels, m.log2_table, m.feat_dim, m.table_dtype, m.res, m.pe_freqs,
                               m.hidden_width, m.hidden_layers, m.n_materials, getattr(m, "dist_head", 0),
                               getattr(m, "per_sample_tables", 0), getattr(m, "concat_encoding", 0))
        self.n_table, self.n_mlp = nif_model_sizes(self.desc)
        self.H = 8 + m.n_materials
        concat = getattr(m, "concat_encoding", 0)
        self.S_grid = 1 if concat else 1 + 2 * m.pe_freqs
        self.E = 2 * (self.S_grid * m.levels * m.feat_dim + (3 * (1 + 2 * m.pe_freqs) if concat else 0))
        self.device = device
        self.h = nif_model_create(self.desc)
        self.max_batch = 0
        if max_batch > 0:
            self.reserve(max_batch)

    def reserve(self, max_batch: int):
        """Training / backward scratch for batches of up to max_batch samples (allocates)."""
        nif_model_reserve(self.h, max_batch)
        self.max_batch = max(self.max_batch, int(max_batch))

    def set_params(self, tables, mlp, s=None):
        t = torch.as_tensor(tables, dtype=torch.float32).reshape(-1).contiguous().to(self.device)
        p = torch.as_tensor(mlp, dtype=torch.float32).reshape(-1).contiguous().to(self.device)
        assert t.numel() == self.n_table and p.numel() == self.n_mlp
        sv = None if s is None else torch.as_tensor(s, dtype=torch.float32).contiguous().to(self.device)
        nif_model_set_params(self.h, t, p, sv)
        torch.cuda.synchronize()

    def get_params(self):
        t = torch.empty(self.n_table, device=self.device)
        p = torch.empty(self.n_mlp, device=self.device)
        s = torch.empty(5, device=self.device)
        nif_model_get_params(self.h, t, p, s)
        return t, p, s

    def get_grads(self):
        t = torch.empty(self.n_table, device=self.device)
        p = torch.empty(self.n_mlp, device=self.device)
        s = torch.empty(5, device=self.device)
        nif_model_get_grads(self.h, t, p, s)
        return t, p, s

    def forward(self, x0, x1, precision=PREC_FP32):
        B = x0.shape[1]
        heads = torch.empty((B, self.H), device=self.device)
        nif_forward(self.h, x0, x1, B, heads, precision)
        return heads

    def encode(self, x):
        n = x.shape[1]
        out = torch.empty((n, self.S_grid * self.spec.levels * self.spec.feat_dim), device=self.device)
        nif_encode(self.h, x, n, out)
        return out

    def __del__(self):
        try:
            if getattr(self, "h", None):
                nif_model_destroy(self.h)
                self.h = None
        except Exception:
            pass


class Grid:
    """Owns a nif_grid handle (per-pose deformed lattice + bin grid)."""

    def __init__(self, occ, N, kinds, strengths, bins_per_axis=0):
        self.N = N
        self.n_poses = len(kinds)
        self.h = nif_build_grid(occ, N, kinds, strengths, bins_per_axis)

    def info(self, pose=0):
        return nif_grid_info(self.h, pose)

    def bounds(self, pose=0):
        return nif_grid_bounds(self.h, pose)

    def update(self, kinds, strengths):
        nif_grid_update(self.h, kinds, strengths)

    def trace(self, o, d, pose_offsets, max_seg=64, with_points=True):
        n = o.shape[1]
        dev = o.device
        out = dict(count=torch.empty(n, dtype=torch.int32, device=dev),
                   cell=torch.full((n, max_seg), -1, dtype=torch.int32, device=dev),
                   t_in=torch.zeros((n, max_seg), device=dev), t_out=torch.zeros((n, max_seg), device=dev))
        if with_points:
            out["x0"] = torch.zeros((3, n, max_seg), device=dev)
            out["x1"] = torch.zeros((3, n, max_seg), device=dev)
        seg = Segments(out["count"].data_ptr(), out["cell"].data_ptr(), out["t_in"].data_ptr(),
                       out["t_out"].data_ptr(), out["x0"].data_ptr() if with_points else None,
                       out["x1"].data_ptr() if with_points else None)
        nif_trace(self.h, make_rays(o, d, pose_offsets), n, max_seg, seg)
        return out

    def query(self, model, o, d, pose_offsets, precision=PREC_FP32, no_network=False, stats=None, out=None,
              tmax=None):
        n = o.shape[1]
        dev = o.device
        if out is None:
            out = alloc_hits(n, dev)
        hits = hits_struct(out)
        nif_query(model.h if model is not None else None, self.h, make_rays(o, d, pose_offsets, tmax), n, hits,
                  Q_NO_NETWORK if no_network else Q_FIRST_HIT, precision, stats)
        return out

    def __del__(self):
        try:
            if getattr(self, "h", None):
                nif_grid_destroy(self.h)
                self.h = None
        except Exception:
            pass


def alloc_hits(n, dev):
    f = lambda: torch.empty(n, device=dev)
    return dict(hit=torch.empty(n, dtype=torch.uint8, device=dev), t=f(), nx=f(), ny=f(), nz=f(), ar=f(),
                ag=f(), ab=f(), material=torch.empty(n, dtype=torch.int32, device=dev),
                cell=torch.empty(n, dtype=torch.int32, device=dev), hit_logit=f(),
                n_queried=torch.empty(n, dtype=torch.int32, device=dev), xr=f(), yr=f(), zr=f(),
                dnx=f(), dny=f(), dnz=f())


def hits_struct(out) -> Hits:
    names = [f[0] for f in Hits._fields_]
    h = Hits(*[out[k].data_ptr() if out.get(k) is not None else None for k in names])
    h._keep = out                                # the struct holds raw pointers: keep the tensors alive
    return h


class NifMultiTaskLoss(torch.autograd.Function):
    """Uncertainty-weighted multi-task loss with a hand-written backward (libnif kernels).

    forward(heads [B][H], s [5], model, labels, fixed=False) -> total loss (0-d tensor);
    labels = (x0, x1, hit, t, n, a, m) as in a training batch (x0 / x1 SoA [3][B], used by the
    sigmoid distance head only; n, a SoA [3][B]).  Only the total is returned (nif_loss also
    gives the five task losses).  backward returns d total / d heads and d total / d s."""

    @staticmethod
    def forward(ctx, heads, s, model, labels, fixed=False):
        heads = heads.contiguous()
        s = s.contiguous()
        B = heads.shape[0]
        keep = [t.contiguous() for t in labels]
        b = Batch(*[t.data_ptr() for t in keep])
        losses = torch.empty(6, device=heads.device)
        d_heads = torch.empty_like(heads)
        d_s = torch.empty(5, device=heads.device)
        nif_loss(model.h, heads, B, b, s, fixed, losses, d_heads, d_s)
        ctx.save_for_backward(d_heads, d_s)
        return losses[5].clone()

    @staticmethod
    def backward(ctx, g):
        d_heads, d_s = ctx.saved_tensors
        return d_heads * g, d_s * g, None, None, None


class NifField(torch.autograd.Function):
    """Heads of point pairs with a hand-written backward (libnif kernels both ways).

    forward(x0, x1, model, precision) -> heads [B][H]; backward accumulates the parameter
    gradients into the model's accumulators (read them with Model.get_grads; zero them with
    nif_model_zero_grads) and returns d x0, d x1 through the hash grid and the positional
    encoding.  The model must be reserved for B samples beforehand (Model(..., max_batch=B)):
    the backward itself allocates nothing."""

    @staticmethod
    def forward(ctx, x0, x1, model, precision=PREC_FP32):
        ctx.save_for_backward(x0, x1)
        ctx.model, ctx.precision = model, precision
        return model.forward(x0.contiguous(), x1.contiguous(), precision)

    @staticmethod
    def backward(ctx, d_heads):
        x0, x1 = ctx.saved_tensors
        m = ctx.model
        B = x0.shape[1]
        if B > m.max_batch:
            raise NifError(f"NifField backward of {B} samples: reserve the model for them first "
                           f"(Model(..., max_batch=B) or Model.reserve(B); reserved {m.max_batch})")
        dx0 = torch.empty_like(x0)
        dx1 = torch.empty_like(x1)
        nif_backward(m.h, x0.contiguous(), x1.contiguous(), B, d_heads.contiguous(), dx0, dx1, True,
                     ctx.precision)
        return dx0, dx1, None, None
