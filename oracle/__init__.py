"""FP64 CPU oracle of the deformation-aware neural intersection function.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU-baseline leg
may import this package; the product path (the GPU library and its binding) never does.
It shares no code with the GPU library: the C sources here are compiled with gcc into
`liboracle.so` and called through ctypes.

Each function follows a passage of the paper (cited in the C sources):
  deform / deform_inv          parameterized deformation and its analytic inverse
  scene_f, scene_grad, scene_attr  the synthetic scenes' implicit function, gradient, attributes
  voxelize, label              rest-space voxelization, ground-truth labels of rest segments
  lattice_vertices, trace      deformed lattice; ordered occupied-voxel hit lists (brute/walk)
  encode, forward              psi = phi(gamma(x)) encoding; MLP heads on point pairs
  encode_backward              adjoint of the encoding with respect to the tables
  encode_corners               its sparse Jacobian: table entry and weight of every corner
  query                        front-to-back first hit with segmented distance
  loss_grad, adam              uncertainty-weighted multi-task loss, analytic gradient, Adam

"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["deform.c", "scene.c", "lattice.c", "network.c"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain FP64, no FMA contraction, OpenMP over rays)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               "-o", _LIB_PATH] + [os.path.join(_HERE, s) for s in _SOURCES] + ["-lm"]
        subprocess.run(cmd, check=True)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = C.CDLL(_LIB_PATH)
    return _lib


def set_threads(n: int) -> int:
    """Threads of the oracle's OpenMP loops (n <= 0 keeps the default); returns the count used."""
    return int(lib().orc_set_threads(C.c_int32(n)))


class Model(C.Structure):
    _fields_ = [("levels", C.c_int32), ("log2_table", C.c_int32), ("feat_dim", C.c_int32),
                ("pe_freqs", C.c_int32), ("res", C.c_int32 * 32), ("n_layers", C.c_int32),
                ("dims", C.c_int32 * 16), ("n_materials", C.c_int32), ("dist_head", C.c_int32),
                ("per_sample_tables", C.c_int32), ("concat_encoding", C.c_int32)]


def model_struct(desc) -> Model:
    """From any object with the ModelDesc attributes (levels, log2_table, ...)."""
    m = Model()
    m.levels, m.log2_table, m.feat_dim, m.pe_freqs = desc.levels, desc.log2_table, desc.feat_dim, desc.pe_freqs
    for i, r in enumerate(desc.res):
        m.res[i] = r
    dims = desc.layer_dims
    m.n_layers = len(dims) - 1
    for i, d in enumerate(dims):
        m.dims[i] = d
    m.n_materials = desc.n_materials
    m.dist_head = getattr(desc, "dist_head", 0)
    m.per_sample_tables = getattr(desc, "per_sample_tables", 0)
    m.concat_encoding = getattr(desc, "concat_encoding", 0)
    return m


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _aos(x):
    """SoA [3][n] or AoS [n][3] -> contiguous float64 [n][3]."""
    x = np.asarray(x)
    if x.ndim == 2 and x.shape[0] == 3 and x.shape[1] != 3:
        x = x.T
    return _f64(x)


# ------------------------------------------------------------------ deformation / scene

def deform(kind: int, s: float, p, inverse: bool = False) -> np.ndarray:
    p = _aos(p).reshape(-1, 3)
    q = np.empty_like(p)
    lib().orc_deform_batch(C.c_int32(kind), C.c_double(s), C.c_int64(len(p)), _p(p, C.c_double),
                           _p(q, C.c_double), C.c_int32(1 if inverse else 0))
    return q


def deform_inv(kind: int, s: float, q) -> np.ndarray:
    return deform(kind, s, q, inverse=True)


def jacdet(kind: int, s: float, p) -> np.ndarray:
    p = _aos(p).reshape(-1, 3)
    out = np.empty(len(p))
    lib().orc_jacdet_batch(C.c_int32(kind), C.c_double(s), C.c_int64(len(p)), _p(p, C.c_double),
                           _p(out, C.c_double))
    return out


def deform_normal(kind: int, s: float, p, n) -> np.ndarray:
    """Unit deformed-space normals (J^-1)^T n at rest points p (rows)."""
    p = _aos(p).reshape(-1, 3); n = _aos(n).reshape(-1, 3)
    out = np.empty_like(p)
    for i in range(len(p)):
        lib().orc_deform_normal(C.c_int(kind), C.c_double(s), _p(p[i], C.c_double), _p(n[i], C.c_double),
                                _p(out[i], C.c_double))
    return out


def scene_f(kind: int, sp, p) -> np.ndarray:
    sp = _f64(sp); p = _aos(p).reshape(-1, 3)
    out = np.empty(len(p))
    lib().orc_scene_f_batch(C.c_int32(kind), _p(sp, C.c_double), C.c_int64(len(p)),
                            _p(p, C.c_double), _p(out, C.c_double))
    return out


def scene_grad(kind: int, sp, p) -> np.ndarray:
    """grad f of the scene's implicit function at points p (rows)."""
    sp = _f64(sp); p = _aos(p).reshape(-1, 3)
    g = np.empty_like(p)
    lib().orc_scene_grad_batch(C.c_int32(kind), _p(sp, C.c_double), C.c_int64(len(p)), _p(p, C.c_double),
                               _p(g, C.c_double))
    return g


def scene_attr(kind: int, sp, p):
    """(albedo [n][3], material [n]) of the scene at points p (rows)."""
    sp = _f64(sp); p = _aos(p).reshape(-1, 3)
    al = np.empty_like(p)
    mt = np.empty(len(p), np.int32)
    lib().orc_scene_attr_batch(C.c_int32(kind), _p(sp, C.c_double), C.c_int64(len(p)), _p(p, C.c_double),
                               _p(al, C.c_double), _p(mt, C.c_int32))
    return al, mt


def voxelize(kind: int, sp, N: int) -> np.ndarray:
    sp = _f64(sp)
    occ = np.zeros(N * N * N, dtype=np.uint8)
    lib().orc_voxelize(C.c_int(kind), _p(sp, C.c_double), C.c_int32(N), _p(occ, C.c_uint8))
    return occ


def label(kind: int, sp, x0, x1, force_march: bool = False):
    """Ground truth of rest segments: (hit u8, t, normal[n][3], albedo[n][3], material)."""
    sp = _f64(sp); x0 = _aos(x0); x1 = _aos(x1)
    n = len(x0)
    hit = np.zeros(n, np.uint8); t = np.zeros(n); nr = np.zeros((n, 3)); al = np.zeros((n, 3))
    mt = np.zeros(n, np.int32)
    lib().orc_label_batch(C.c_int32(kind), _p(sp, C.c_double), C.c_int32(int(force_march)),
                          C.c_int64(n), _p(x0, C.c_double), _p(x1, C.c_double), _p(hit, C.c_uint8),
                          _p(t, C.c_double), _p(nr, C.c_double), _p(al, C.c_double), _p(mt, C.c_int32))
    return hit, t, nr, al, mt


# ------------------------------------------------------------------ lattice / traversal

def lattice_vertices(kind: int, s: float, N: int) -> np.ndarray:
    V = np.empty(((N + 1) ** 3, 3))
    lib().orc_lattice_vertices(C.c_int(kind), C.c_double(s), C.c_int32(N), _p(V, C.c_double))
    return V


def trace(N: int, occ, V, o, d, brute: bool = False, max_out: int | None = None,
          with_flags: bool = True, with_cos: bool = False):
    """Ordered occupied hit lists.  Returns (cells[n][max_out], tin, tout, count[n], flags[n]),
    plus (cos_in, cos_out) of each interval's bounding crossings when with_cos."""
    occ = np.ascontiguousarray(occ, dtype=np.uint8); V = _f64(V)
    o = _aos(o); d = _aos(d)
    n = len(o)
    mo = max_out or (4 * N + 16)
    cells = np.full((n, mo), -1, np.int32); tin = np.zeros((n, mo)); tout = np.zeros((n, mo))
    cnt = np.zeros(n, np.int32); fl = np.zeros(n, np.int32)
    ci = np.ones((n, mo)); co = np.ones((n, mo))
    lib().orc_trace_batch(C.c_int32(N), _p(occ, C.c_uint8), _p(V, C.c_double), C.c_int64(n),
                          _p(o, C.c_double), _p(d, C.c_double), C.c_int32(int(brute)), C.c_int32(mo),
                          _p(cells, C.c_int32), _p(tin, C.c_double), _p(tout, C.c_double),
                          _p(cnt, C.c_int32), _p(fl, C.c_int32) if with_flags else None,
                          _p(ci, C.c_double) if with_cos else None, _p(co, C.c_double) if with_cos else None)
    if with_cos:
        return cells, tin, tout, cnt, fl, ci, co
    return cells, tin, tout, cnt, fl


# ------------------------------------------------------------------ network

def encode(desc, tables, x) -> np.ndarray:
    m = model_struct(desc)
    tab = _f64(tables).reshape(-1)
    x = _aos(x)
    W = (1 if getattr(desc, "concat_encoding", 0) else 1 + 2 * desc.pe_freqs) * desc.levels * desc.feat_dim
    out = np.empty((len(x), W))
    lib().orc_encode_batch(C.byref(m), _p(tab, C.c_double), C.c_int64(len(x)), _p(x, C.c_double),
                           _p(out, C.c_double))
    return out


def encode_corners(desc, x):
    """(idx, w) [n][S][L][8]: the flat table entry ((set L + level) T + entry) and trilinear
    weight of every corner the encoding of each point reads (its sparse Jacobian)."""
    m = model_struct(desc)
    x = _aos(x)
    S = 1 if getattr(desc, "concat_encoding", 0) else 1 + 2 * desc.pe_freqs
    idx = np.zeros((len(x), S, desc.levels, 8), np.int64)
    w = np.zeros((len(x), S, desc.levels, 8))
    lib().orc_encode_corners_batch(C.byref(m), C.c_int64(len(x)), _p(x, C.c_double), _p(idx, C.c_int64),
                                   _p(w, C.c_double))
    return idx, w


def encode_backward(desc, tables, x, d_enc) -> np.ndarray:
    """J^T d_enc: the table gradient of sum(d_enc * psi(x)) over the points x (rows), shaped
    like the tables.  psi is linear in the tables with nonnegative (trilinear) coefficients."""
    m = model_struct(desc)
    tab = _f64(tables).reshape(-1)
    x = _aos(x)
    W = (1 if getattr(desc, "concat_encoding", 0) else 1 + 2 * desc.pe_freqs) * desc.levels * desc.feat_dim
    dv = _f64(d_enc).reshape(len(x), W)
    g = np.zeros_like(tab)
    lib().orc_encode_backward_batch(C.byref(m), _p(tab, C.c_double), C.c_int64(len(x)), _p(x, C.c_double),
                                    _p(dv, C.c_double), _p(g, C.c_double))
    return g.reshape(np.shape(tables))


def forward(desc, tables, params, x0, x1, with_scale: bool = False):
    """Heads z[n][H] of the MLP on psi(x0) ++ psi(x1)."""
    m = model_struct(desc)
    tab = _f64(tables).reshape(-1); prm = _f64(params)
    x0 = _aos(x0); x1 = _aos(x1)
    n = len(x0)
    z = np.empty((n, desc.n_heads)); sc = np.empty(n)
    lib().orc_forward_batch(C.byref(m), _p(tab, C.c_double), _p(prm, C.c_double), C.c_int64(n),
                            _p(x0, C.c_double), _p(x1, C.c_double), _p(z, C.c_double), _p(sc, C.c_double))
    return (z, sc) if with_scale else z


def query(desc, tables, params, N: int, occ, kind: int, s: float, o, d, tmax=None) -> dict:
    """Per-ray first-hit outputs; for hits also zhit (raw heads of the hit segment) and
    seginfo = (t_in, t_out, rest length, |cos| at entry, |cos| at exit) of that segment, and
    dnormal, the normal carried to deformed space.
    tmax (per ray, optional): occlusion form, hits at D >= tmax and voxels entered at or
    beyond tmax do not count."""
    m = model_struct(desc)
    tab = _f64(tables).reshape(-1); prm = _f64(params)
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    o = _aos(o); d = _aos(d)
    n = len(o)
    r = dict(hit=np.zeros(n, np.uint8), t=np.zeros(n), xrest=np.zeros((n, 3)), normal=np.zeros((n, 3)),
             albedo=np.zeros((n, 3)), material=np.zeros(n, np.int32), cell=np.zeros(n, np.int32),
             logit=np.zeros(n), n_queried=np.zeros(n, np.int32), margin=np.zeros(n),
             zhit=np.zeros((n, desc.n_heads)), seginfo=np.zeros((n, 5)), dnormal=np.zeros((n, 3)))
    tm = None if tmax is None else np.ascontiguousarray(np.broadcast_to(np.asarray(tmax, np.float64), (n,)))
    lib().orc_query_batch(C.byref(m), _p(tab, C.c_double), _p(prm, C.c_double), C.c_int32(N),
                          _p(occ, C.c_uint8), C.c_int32(kind), C.c_double(s), C.c_int64(n),
                          _p(o, C.c_double), _p(d, C.c_double), _p(r["hit"], C.c_uint8),
                          _p(r["t"], C.c_double), _p(r["xrest"], C.c_double), _p(r["normal"], C.c_double),
                          _p(r["albedo"], C.c_double), _p(r["material"], C.c_int32),
                          _p(r["cell"], C.c_int32), _p(r["logit"], C.c_double),
                          _p(r["n_queried"], C.c_int32), _p(r["margin"], C.c_double),
                          _p(r["zhit"], C.c_double), _p(r["seginfo"], C.c_double),
                          _p(tm, C.c_double) if tm is not None else None, _p(r["dnormal"], C.c_double))
    return r


def loss_grad(desc, tables, params, s, x0, x1, hit, t, nrm, alb, mat, want_x: bool = False,
              want_dz: bool = False, fixed_weights: bool = False):
    """Returns (losses[6], g_tables, g_params, g_s, g_x0, g_x1), plus dL/dz[B][H] if want_dz.
    fixed_weights: every task weighs 1 and s is unused (the ablation without uncertainty
    weighting)."""
    m = model_struct(desc)
    tab = _f64(tables).reshape(-1); prm = _f64(params); s = _f64(s)
    x0 = _aos(x0); x1 = _aos(x1)
    B = len(x0)
    hit = np.ascontiguousarray(hit, dtype=np.uint8); t = _f64(t); nrm = _aos(nrm); alb = _aos(alb)
    mat = np.ascontiguousarray(mat, dtype=np.int32)
    losses = np.zeros(6); gt = np.zeros_like(tab); gp = np.zeros_like(prm); gs = np.zeros(5)
    gx0 = np.zeros_like(x0) if want_x else None
    gx1 = np.zeros_like(x1) if want_x else None
    dz = np.zeros((B, desc.n_heads)) if want_dz else None
    lib().orc_loss_grad(C.byref(m), _p(tab, C.c_double), _p(prm, C.c_double), _p(s, C.c_double),
                        C.c_int64(B), _p(x0, C.c_double), _p(x1, C.c_double), _p(hit, C.c_uint8),
                        _p(t, C.c_double), _p(nrm, C.c_double), _p(alb, C.c_double), _p(mat, C.c_int32),
                        _p(losses, C.c_double), _p(gt, C.c_double), _p(gp, C.c_double), _p(gs, C.c_double),
                        _p(gx0, C.c_double) if want_x else None, _p(gx1, C.c_double) if want_x else None,
                        _p(dz, C.c_double) if want_dz else None, C.c_int32(int(fixed_weights)))
    if want_dz:
        return losses, gt.reshape(np.shape(tables)), gp, gs, gx0, gx1, dz
    return losses, gt.reshape(np.shape(tables)), gp, gs, gx0, gx1


def adam(theta, g, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """In-place Adam step on float64 arrays."""
    for a in (theta, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam(C.c_int64(theta.size), _p(theta, C.c_double), _p(g, C.c_double), _p(m, C.c_double),
                   _p(v, C.c_double), C.c_int32(step), C.c_double(lr), C.c_double(b1), C.c_double(b2),
                   C.c_double(eps))


# ------------------------------------------------------------------ precision helpers

def round_f16(a) -> np.ndarray:
    """IEEE binary16 round-to-nearest-even, widened back to float64."""
    return np.asarray(a, dtype=np.float32).astype(np.float16).astype(np.float64)


def round_bf16(a) -> np.ndarray:
    """bfloat16 round-to-nearest-even of float32 values, widened back to float64."""
    x = np.ascontiguousarray(a, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
