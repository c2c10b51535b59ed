"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and lays them out: scene parameters, poses,
rays, initial weights and the frozen per-workload hyper-parameters.  It holds none
of the method's arithmetic (no deformation, traversal, encoding, network or loss),
so both the CPU oracle and the GPU library can consume its output without sharing
any computation.

The paper's own test objects (bunny, cat, dragon) are not available; the synthetic
scenes below stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List

import numpy as np

# Deformation kinds; the numeric values are the ones the C interfaces use.
IDENTITY, TWIST, BEND, TAPER, TWIST_BEND = 0, 1, 2, 3, 4
# Scene kinds (implicit-surface families).
SCENE_TORUS, SCENE_SPHERES, SCENE_BLOBS = 0, 1, 2
# Table storage types.
TABLE_F32, TABLE_F16 = 0, 1
# MLP arithmetic.
PREC_FP32, PREC_BF16, PREC_FP16 = 0, 1, 2
# Distance head: ReLU rest-space distance (log-space loss), or sigmoid fraction of the segment.
DIST_LOG_RELU, DIST_SIGMOID = 0, 1


@dataclass
class ModelDesc:
    """Hyper-parameters of the hybrid encoding and the intersection MLP."""
    levels: int
    log2_table: int
    feat_dim: int
    table_dtype: int
    res: List[int]
    pe_freqs: int
    hidden_width: int
    hidden_layers: int
    n_materials: int
    dist_head: int = DIST_LOG_RELU
    per_sample_tables: int = 0           # 1: one table set per PE sample
    concat_encoding: int = 0             # 1: [phi(x), gamma(x)] instead of phi(gamma(x))

    @property
    def n_samples(self) -> int:          # PE samples per point that go through the grid
        return 1 if self.concat_encoding else 1 + 2 * self.pe_freqs

    @property
    def gamma_width(self) -> int:        # raw PE values per point appended by the concatenated form
        return 3 * (1 + 2 * self.pe_freqs) if self.concat_encoding else 0

    @property
    def enc_width(self) -> int:          # two points (entry, exit) x (samples x levels x features + gamma)
        return 2 * (self.n_samples * self.levels * self.feat_dim + self.gamma_width)

    @property
    def n_heads(self) -> int:            # hit, dist, normal(3), albedo(3), material logits
        return 8 + self.n_materials

    @property
    def layer_dims(self) -> List[int]:
        return [self.enc_width] + [self.hidden_width] * self.hidden_layers + [self.n_heads]

    @property
    def n_mlp_params(self) -> int:
        d = self.layer_dims
        return sum(d[i + 1] * d[i] + d[i + 1] for i in range(len(d) - 1))

    @property
    def table_size(self) -> int:
        return 1 << self.log2_table

    @property
    def table_levels(self) -> int:       # table sets x levels: the first axis of the tables
        return self.levels * (self.n_samples if self.per_sample_tables else 1)


def level_resolutions(levels: int, n_min: int, n_max: int) -> List[int]:
    """Exponentially spaced grid resolutions, frozen as integers (computed once in FP64)."""
    if levels == 1:
        return [n_min]
    b = (n_max / n_min) ** (1.0 / (levels - 1))
    return [int(math.floor(n_min * b ** l + 0.5)) for l in range(levels)]


@dataclass
class Workload:
    name: str
    scene_kind: int
    N: int
    model: ModelDesc
    seed: int
    pose_kinds: List[int] = field(default_factory=list)
    pose_strengths: List[float] = field(default_factory=list)
    rays: str = "random"                 # "random" | "camera" | "mixed"
    n_rays: int = 0                      # per pose for "camera" (res*res) or total for "random"
    cam_res: int = 0
    cam_az_deg: List[float] = field(default_factory=list)
    cam_tile: int = 0                    # camera rays issued in cam_tile^2 screen tiles (0: rows)
    precision: int = PREC_FP32
    scene_seed: int = -1                 # seed of the scene when it differs from `seed` (-1: seed)


# Torus workload (4,096 random rays, twist, 16^3 grid, 8-level 2^14 FP32 tables).
_C0_MODEL = ModelDesc(levels=8, log2_table=14, feat_dim=2, table_dtype=TABLE_F32,
                      res=level_resolutions(8, 16, 256), pe_freqs=6,
                      hidden_width=64, hidden_layers=2, n_materials=1)
# Sphere-union workloads (64^3 grid, 16-level 2^19 FP16 tables).
_C1_MODEL = ModelDesc(levels=16, log2_table=19, feat_dim=2, table_dtype=TABLE_F16,
                      res=level_resolutions(16, 16, 2048), pe_freqs=6,
                      hidden_width=64, hidden_layers=3, n_materials=4)
_C2_MODEL = replace(_C1_MODEL, hidden_width=128, hidden_layers=4)
# The configuration of the paper's comparison of deformation results: a two-level grid with
# base resolution 64 and three features per entry, three PE bands (the second level's
# resolution, the table size and the MLP are not stated: 128, 2^19 FP16, 3 x 64).
_PAPER_MODEL = ModelDesc(levels=2, log2_table=19, feat_dim=3, table_dtype=TABLE_F16, res=[64, 128], pe_freqs=3,
                         hidden_width=64, hidden_layers=3, n_materials=4)


def workload(name: str) -> Workload:
    """Frozen workload definitions.

    torus16      -- 16^3 torus, one twist (0.6 rad per unit z), 4,096 random rays, FP32.
    spheres64    -- 8 random spheres at 64^3; twist/bend/taper x 8 strengths = 24 poses,
                    1024x1024 pinhole rays each in 8x8 screen tiles, FP32 inference, MLP 3x64.
    spheres64_p  -- the same scene, 2 poses (twist, bend at full strength) x 1024^2 rays
                    in 8x8 tiles, MLP 4x128 for the FP32 / BF16 / FP16 comparison.
    blobs128     -- 32-Gaussian blob field at 128^3 for the training step, MLP 4x128.
    blobs128_b   -- the blobs128 scene with 16 poses of uneven ray counts (batched query).
    spheres32_paper -- the paper's deformation-comparison configuration: the sphere scene at
                    32^3 voxels, a 2-level grid (64, 128) with 3 features per entry, F = 3;
                    twist, bend and taper at full strength, 512x512 pinhole rays per pose.
    """
    strengths8 = [(i + 1) / 8.0 for i in range(8)]
    if name == "torus16":
        return Workload(name, SCENE_TORUS, 16, _C0_MODEL, seed=1000,
                        pose_kinds=[TWIST], pose_strengths=[1.0], rays="random", n_rays=4096)
    if name == "spheres64":
        kinds = [k for k in (TWIST, BEND, TAPER) for _ in strengths8]
        strengths = strengths8 * 3
        return Workload(name, SCENE_SPHERES, 64, _C1_MODEL, seed=1001,
                        pose_kinds=kinds, pose_strengths=strengths, rays="camera",
                        cam_res=1024, n_rays=1024 * 1024,
                        cam_az_deg=[15.0 * p for p in range(24)], cam_tile=8)
    if name == "spheres64_p":
        return Workload(name, SCENE_SPHERES, 64, _C2_MODEL, seed=1001,
                        pose_kinds=[TWIST, BEND], pose_strengths=[1.0, 1.0], rays="camera",
                        cam_res=1024, n_rays=1024 * 1024, cam_az_deg=[0.0, 90.0], cam_tile=8,
                        precision=PREC_BF16)
    if name == "blobs128":
        return Workload(name, SCENE_BLOBS, 128, replace(_C2_MODEL), seed=1003,
                        rays="random", precision=PREC_BF16)
    if name == "blobs128_b":
        return Workload(name, SCENE_BLOBS, 128, replace(_C2_MODEL), seed=1004,
                        rays="mixed", precision=PREC_BF16, scene_seed=1003)
    if name == "spheres32_paper":
        return Workload(name, SCENE_SPHERES, 32, _PAPER_MODEL, seed=1005, scene_seed=1001,
                        pose_kinds=[TWIST, BEND, TAPER], pose_strengths=[1.0, 1.0, 1.0], rays="camera",
                        cam_res=512, n_rays=512 * 512, cam_az_deg=[0.0, 120.0, 240.0])
    raise KeyError(name)


# ----------------------------------------------------------------------------- scenes

def scene_of(w: Workload) -> np.ndarray:
    """The scene parameters of a workload."""
    return scene_params(w.scene_kind, w.seed if w.scene_seed < 0 else w.scene_seed)


def scene_params(kind: int, seed: int) -> np.ndarray:
    """Flat float64 parameter vector of a scene (layout documented per kind).

    torus  : [cx, cy, cz, R, r]
    spheres: [n, then per sphere cx, cy, cz, radius, albedo r, g, b, material]
    blobs  : [n, then per blob mux, muy, muz, sigma, colour r, g, b, material]
    """
    rng = np.random.default_rng(seed)
    if kind == SCENE_TORUS:
        return np.array([0.5, 0.5, 0.5, 0.35, 0.12], dtype=np.float64)
    if kind == SCENE_SPHERES:
        n = 8
        c = rng.uniform(0.25, 0.75, size=(n, 3))
        r = rng.uniform(0.05, 0.2, size=n)
        alb = rng.uniform(0.1, 0.9, size=(n, 3))
        rows = [np.concatenate([c[i], [r[i]], alb[i], [i % 4]]) for i in range(n)]
        return np.concatenate([[n], np.concatenate(rows)]).astype(np.float64)
    if kind == SCENE_BLOBS:
        n = 32
        mu = rng.uniform(0.2, 0.8, size=(n, 3))
        sg = rng.uniform(0.03, 0.08, size=n)
        col = rng.uniform(0.1, 0.9, size=(n, 3))
        rows = [np.concatenate([mu[i], [sg[i]], col[i], [i % 4]]) for i in range(n)]
        return np.concatenate([[n], np.concatenate(rows)]).astype(np.float64)
    raise KeyError(kind)


# ----------------------------------------------------------------------------- poses

def poses(w: Workload):
    """(kinds int32[P], strengths float32[P]) of a workload's fixed pose list."""
    return (np.asarray(w.pose_kinds, dtype=np.int32),
            np.asarray(w.pose_strengths, dtype=np.float32))


def random_poses(n: int, seed: int, kinds=(TWIST, BEND), s_lo: float = 0.0, s_hi: float = 1.0):
    """n poses with kind uniform over `kinds` and strength uniform in (s_lo, s_hi]."""
    rng = np.random.default_rng(seed)
    k = np.asarray(kinds, dtype=np.int32)[rng.integers(0, len(kinds), size=n)]
    s = s_hi - rng.uniform(0.0, 1.0, size=n) * (s_hi - s_lo)      # in (s_lo, s_hi]
    return k.astype(np.int32), s.astype(np.float32)


# ----------------------------------------------------------------------------- rays

def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def rays_random(n: int, seed: int, radius: float = 2.0):
    """Origins uniform on a sphere of `radius` about the cube centre, aimed at points
    uniform in the unit cube.  Returns SoA float32 (o[3][n], d[3][n]), d of unit length
    in FP64 before rounding to FP32."""
    rng = np.random.default_rng(seed)
    u = _unit(rng.normal(size=(n, 3)))
    o = 0.5 + radius * u
    tgt = rng.uniform(0.0, 1.0, size=(n, 3))
    d = _unit(tgt - o)
    return (np.ascontiguousarray(o.T.astype(np.float32)),
            np.ascontiguousarray(d.T.astype(np.float32)))


def rays_inside(n: int, seed: int, lo: float = 0.0, hi: float = 1.0):
    """Secondary-style rays: origin uniform in [lo, hi]^3, direction uniform on S^2."""
    rng = np.random.default_rng(seed)
    o = rng.uniform(lo, hi, size=(n, 3))
    d = _unit(rng.normal(size=(n, 3)))
    return (np.ascontiguousarray(o.T.astype(np.float32)),
            np.ascontiguousarray(d.T.astype(np.float32)))


def rays_camera(res: int, az_deg: float, elev_deg: float = 20.0, dist: float = 2.0,
                vfov_deg: float = 45.0, sub: int = 1, sub_index: int = 0, tile: int = 0):
    """Pinhole primary rays through pixel centres, eye at distance `dist` from the cube
    centre at the given azimuth/elevation, looking at the centre with +z up.

    Rays come in row-major pixel order, or with `tile` > 0 (dividing `res`) in tile x tile
    screen tiles, the tiles row-major and the pixels of a tile row-major, as a tiled renderer
    issues them (with tile = 8 one 64-ray wave of the query covers one tile).
    `sub` > 1 keeps every sub-th ray of that order (a strided subset, used to bound CPU work)."""
    az, el = math.radians(az_deg), math.radians(elev_deg)
    eye = np.array([0.5 + dist * math.cos(el) * math.cos(az),
                    0.5 + dist * math.cos(el) * math.sin(az),
                    0.5 + dist * math.sin(el)])
    fwd = _unit(np.array([0.5, 0.5, 0.5]) - eye)
    right = _unit(np.cross(fwd, np.array([0.0, 0.0, 1.0])))
    up = np.cross(right, fwd)
    h = math.tan(math.radians(vfov_deg) / 2.0)
    pix = np.arange(res * res, dtype=np.int64)
    if tile > 0:
        assert res % tile == 0, "tile must divide res"
        i = pix
        t, r = i // (tile * tile), i % (tile * tile)
        pix = ((t // (res // tile)) * tile + r // tile) * res + (t % (res // tile)) * tile + r % tile
    pix = pix[sub_index::sub]
    px, py = (pix % res).astype(np.float64), (pix // res).astype(np.float64)
    sx = ((px + 0.5) / res * 2.0 - 1.0) * h
    sy = (1.0 - (py + 0.5) / res * 2.0) * h
    d = _unit(fwd[None, :] + sx[:, None] * right[None, :] + sy[:, None] * up[None, :])
    o = np.broadcast_to(eye, d.shape)
    return (np.ascontiguousarray(o.T.astype(np.float32)),
            np.ascontiguousarray(d.T.astype(np.float32)))


def uneven_counts(n_poses: int, seed: int, lo: int = 65536, hi: int = 1048576):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=n_poses).astype(np.int64)


def batched_rays(counts, seed: int, boxes):
    """The batched query's rays: per pose p, counts[p] rays, the first half pinhole primary rays
    (a square camera of at least that many pixels at a random azimuth, its first pixels), the
    rest secondary rays with origins uniform in boxes[p] = (lo[3], hi[3]) (the pose's occupied
    deformed box) and directions uniform on S^2.  SoA float32 (o[3][n], d[3][n])."""
    rng = np.random.default_rng(seed)
    os_, ds_ = [], []
    for p, c in enumerate(counts):
        c = int(c)
        half = c // 2
        res_ = int(np.ceil(np.sqrt(half)))
        o, d = rays_camera(res_, float(rng.uniform(0, 360)))
        lo, hi = boxes[p]
        o2, d2 = rays_inside(c - half, seed + p, lo, hi)
        os_ += [o[:, :half], o2]
        ds_ += [d[:, :half], d2]
    return (np.ascontiguousarray(np.concatenate(os_, axis=1)), np.ascontiguousarray(np.concatenate(ds_, axis=1)))


# ----------------------------------------------------------------------------- weights

def init_tables(m: ModelDesc, seed: int) -> np.ndarray:
    """FP32 master tables [sets x L][T][Fd], uniform in (-1e-4, 1e-4)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1e-4, 1e-4, size=(m.table_levels, m.table_size, m.feat_dim)).astype(np.float32)


def init_mlp(m: ModelDesc, seed: int) -> np.ndarray:
    """Canonical flat FP32 MLP parameters: per layer W[out][in] row-major then b[out].
    Xavier-uniform weights, zero biases."""
    rng = np.random.default_rng(seed + 1)
    d = m.layer_dims
    parts = []
    for i in range(len(d) - 1):
        a = math.sqrt(6.0 / (d[i] + d[i + 1]))
        parts.append(rng.uniform(-a, a, size=(d[i + 1], d[i])).reshape(-1))
        parts.append(np.zeros(d[i + 1]))
    return np.concatenate(parts).astype(np.float32)


def mlp_layers(m: ModelDesc, flat: np.ndarray):
    """Split a canonical flat parameter vector into [(W, b), ...] views."""
    d = m.layer_dims
    out, off = [], 0
    for i in range(len(d) - 1):
        W = flat[off:off + d[i + 1] * d[i]].reshape(d[i + 1], d[i]); off += d[i + 1] * d[i]
        b = flat[off:off + d[i + 1]]; off += d[i + 1]
        out.append((W, b))
    assert off == flat.size
    return out


def random_points(n: int, seed: int, lo: float = -0.05, hi: float = 1.05):
    """Rest-space point pairs (x0, x1) as SoA float32 [3][n], for network-only checks."""
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(lo, hi, size=(3, n))
    x1 = x0 + rng.normal(scale=0.02, size=(3, n))
    return x0.astype(np.float32), x1.astype(np.float32)
