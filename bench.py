"""Benchmark of the deformation-aware neural intersection query on one MI355X.

One step = one pass of the query path over the whole workload: every ray of every pose is
traversed through the occupied deformed voxels, its segments are mapped to rest space,
encoded and run through the MLP front to back until the first hit (one persistent kernel
launch).  The per-pose deformed grids are rebuilt each step as well (nif_grid_update), as an
animation would.  Default workload: 8 random spheres voxelized at 64^3, 24 poses
(twist/bend/taper x 8 strengths), 1024x1024 pinhole rays per pose, 16-level 2^19 FP16 hash
grid, 6 PE frequencies, MLP 832->64x3->12, FP32.

Prints one JSON line (see the keys below).  --gpus N > 1 is refused: the library runs on one
GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GATHER_BYTES_PER_EVAL = 13312   # 2 points x 13 PE samples x 16 levels x 8 corners x 4 B (FP16 pair)
GATHER_BYTES_PER_EVAL_C0 = 13312  # torus workload: 2 x 13 x 8 levels x 8 corners x 8 B (FP32 pair)
# training step per sample: forward gathers 13,312 B + the backward's recomputed gathers 13,312 B
# + the FP32 table-gradient payload (2 points x 13 samples x 16 levels x 8 corners x 8 B) 26,624 B
# + dense Adam over all parameters (~570 MB per step at B = 2^18) 2,176 B
TRAIN_BYTES_PER_SAMPLE = 13312 + 13312 + 26624 + 2176
HBM_PEAK_GBS = 8000.0

# HBM bytes that k_query moves per launch on the default workload, from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE; KiB summed over the launch) scaled by what the same counters read for a
# plain 1 GiB device copy (bench.py --calibrate-copy).  They hold only for the kernel sources they
# were taken on and the ray generator of the workload (SHA-256 of KQUERY_SOURCES); otherwise the
# traffic is reported as null.
KQUERY_SOURCES = ["paper_2604_24666_amd/csrc/nif_query.hip", "paper_2604_24666_amd/csrc/nif_net.hpp",
                  "paper_2604_24666_amd/csrc/nif_trace.hpp", "paper_2604_24666_amd/csrc/nif_device.hpp",
                  "paper_2604_24666_amd/csrc/nif_internal.hpp", "paper_2604_24666_amd/build.py",
                  "nif_synth/__init__.py"]
KQUERY_TRAFFIC = {
    "sources_sha256": "7bb9c2a0530250ba2433426a0daaf766a3013fcd580931cd0dedcc63e86ea54a",
    "fetch_kib": 1.04862e8, "write_kib": 1.93924e6,         # per k_query<64, FP32, 64> launch, default workload
    "fetch_scale": 1048576 / 524303, "write_scale": 1048576 / 1048577,   # 1 GiB copy reads 524,303 / writes 1,048,577 KiB
}


def kquery_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KQUERY_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kquery_traffic_bytes():
    t = KQUERY_TRAFFIC
    if t is None or t["sources_sha256"] != kquery_sources_sha():
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def setup(workload: str, precision: int):
    import torch

    import nif_synth as S
    import paper_2604_24666_amd as P

    w = S.workload(workload)
    m = w.model
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = torch.zeros(w.N ** 3, dtype=torch.uint8, device="cuda")
    P.nif_voxelize(w.scene_kind, sp, w.N, occ)
    model = P.Model(m)
    model.set_params(S.init_tables(m, w.seed + 100), S.init_mlp(m, w.seed + 100))
    kinds, strengths = S.poses(w)
    n_pose = w.cam_res ** 2
    n = n_pose * len(kinds)
    o_all = torch.empty((3, n), device="cuda")
    d_all = torch.empty((3, n), device="cuda")
    for p in range(len(kinds)):
        o, d = S.rays_camera(w.cam_res, w.cam_az_deg[p], tile=w.cam_tile)
        o_all[:, p * n_pose:(p + 1) * n_pose] = torch.as_tensor(o).cuda()
        d_all[:, p * n_pose:(p + 1) * n_pose] = torch.as_tensor(d).cuda()
    off = torch.as_tensor(np.arange(len(kinds) + 1, dtype=np.int64) * n_pose).cuda()
    grid = P.Grid(occ, w.N, kinds, strengths)
    out = P.alloc_hits(n, "cuda")
    return dict(w=w, m=m, sp=sp, occ=occ, model=model, grid=grid, o=o_all, d=d_all, off=off, out=out, n=n,
                kinds=kinds, strengths=strengths, precision=precision)


def cpu_baseline(ctx, sample_stride: int = 12, one_core_stride: int = 160):
    """The FP64 oracle's query on strided subsets of the camera rays of three poses (a twist, a
    bend and a taper), timed on the host with all cores, and on one core on a smaller subset."""
    import nif_synth as S
    import oracle

    w, m = ctx["w"], ctx["m"]
    occ = ctx["occ"].cpu().numpy()
    tab = S.init_tables(m, w.seed + 100)
    tab64 = oracle.round_f16(tab) if m.table_dtype == S.TABLE_F16 else tab.astype(np.float64)
    prm = S.init_mlp(m, w.seed + 100).astype(np.float64)
    kinds, strengths = ctx["kinds"], ctx["strengths"]
    picks = [int(np.flatnonzero((kinds == k) & (strengths == 0.5))[0]) for k in (S.TWIST, S.BEND, S.TAPER)]
    names = ["identity", "twist", "bend", "taper", "twist-bend"]

    def run(stride):
        n, dt = 0, 0.0
        for p in picks:
            o, d = S.rays_camera(w.cam_res, w.cam_az_deg[p], sub=stride, sub_index=p % stride)
            t0 = time.perf_counter()
            oracle.query(m, tab64, prm, w.N, occ, int(kinds[p]), float(strengths[p]), o, d)
            dt += time.perf_counter() - t0
            n += o.shape[1]
        return n, dt

    all_cores = oracle.set_threads(0)
    o, d = S.rays_camera(w.cam_res, w.cam_az_deg[0], sub=4096)
    oracle.query(m, tab64, prm, w.N, occ, int(kinds[0]), float(strengths[0]), o, d)        # warm-up
    n, dt = run(sample_stride)
    oracle.set_threads(1)
    n1, dt1 = run(one_core_stride)
    oracle.set_threads(all_cores)
    poses = ", ".join(f"{names[int(kinds[p])]} s={float(strengths[p])}" for p in picks)
    return {"value": n / dt, "unit": "rays/s", "cores": all_cores, "kind": "oracle",
            "sample": f"{n} rays (every {sample_stride}th pixel of 3 poses: {poses}), FP64 oracle, {dt:.1f} s",
            "one_core": {"value": n1 / dt1, "unit": "rays/s", "cores": 1,
                         "sample": f"{n1} rays (every {one_core_stride}th pixel of the same poses), {dt1:.1f} s"}}


def tuned_query_shape(key: str, model, grid, rays, n: int, hits, precision: int = 0, cache_path=None):
    """Launch shape for a workload `key` on this GPU architecture: read from the JSON cache
    (NIF_TUNE_CACHE, default ~/.cache/nif_tune.json) or found by nif_autotune_query and
    stored; applied process-wide.  Returns (workgroups per CU, rays per wave)."""
    import torch

    import paper_2604_24666_amd as P
    path = cache_path or os.environ.get("NIF_TUNE_CACHE", os.path.expanduser("~/.cache/nif_tune.json"))
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    full = f"{arch}/{key}/prec{precision}"
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    if full in cache:
        bpc, rpw = cache[full]["blocks_per_cu"], cache[full]["rays_per_wave"]
        P.nif_set_query_blocks_per_cu(bpc)
        P.nif_set_query_rays_per_wave(rpw)
        return bpc, rpw
    bpc, rpw, ms = P.nif_autotune_query(model, grid, rays, n, hits, precision)
    cache[full] = {"blocks_per_cu": bpc, "rays_per_wave": rpw, "ms": ms, "n_rays": int(n)}
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return bpc, rpw


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def torus_leg(replays=200, warmup=20):
    """The plain method at the smallest size: 4,096 random rays into the 16^3 torus under one
    twist, MLP 416-64x2-9 FP32 (Xavier, tables U(+-1e-4)), forward only; one launch replayed
    from a captured graph (a launch this small is bound by its latency)."""
    import torch

    import nif_synth as S
    import paper_2604_24666_amd as P

    w = S.workload("torus16")
    m = w.model
    sp = S.scene_of(w)
    occ = torch.zeros(w.N ** 3, dtype=torch.uint8, device="cuda")
    P.nif_voxelize(w.scene_kind, sp, w.N, occ)
    model = P.Model(m)
    model.set_params(S.init_tables(m, w.seed + 100), S.init_mlp(m, w.seed + 100))
    grid = P.Grid(occ, w.N, w.pose_kinds, w.pose_strengths)
    o, d = [torch.as_tensor(a).cuda() for a in S.rays_random(w.n_rays, w.seed)]
    off = torch.tensor([0, w.n_rays], dtype=torch.int64, device="cuda")
    rays = P.make_rays(o, d, off)
    out = P.alloc_hits(w.n_rays, "cuda")
    hits = P.hits_struct(out)
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    s_cap = torch.cuda.Stream()
    call = lambda: P.nif_query(model.h, grid.h, rays, w.n_rays, hits, 0, P.PREC_FP32, stats, stream=s_cap)
    with torch.cuda.stream(s_cap):
        call()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s_cap):
        call()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    e0 = int(stats.cpu()[1])
    ms = []
    for _ in range(replays):
        with torch.cuda.stream(s_cap):
            a.record(s_cap)
            g.replay()
            b.record(s_cap)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    evals = (int(stats.cpu()[1]) - e0) / replays
    med = float(np.median(ms))
    achieved = evals * GATHER_BYTES_PER_EVAL_C0 / (float(np.mean(ms)) * 1e-3) / 1e9
    log(f"torus leg: {med:.4f} ms per launch, {evals:.0f} network evaluations")
    del g
    return {"workload": "torus16: 16^3 torus (R 0.35, r 0.12), twist 0.6 z, 4,096 random rays, 8-level 2^14 FP32 grid, "
                        "F = 6, MLP 416-64x2-9 FP32; one launch replayed from a captured graph, median of "
                        f"{replays} after {warmup} warm-up",
            "rays_per_s": w.n_rays / (med * 1e-3), "ms_per_launch_median": med, "network_evals_per_launch": evals,
            "hit_rate": float(out["hit"].float().mean().item()),
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_query",
                         "algorithmic_bytes": f"{GATHER_BYTES_PER_EVAL_C0} B of hash-corner gathers per network evaluation"}}


def trained_model(P, S, w, steps, B=1 << 16, n_rays=1 << 20, seed_offset=300):
    """A model of workload w's architecture trained by this library's own FP32 training step:
    `steps` Adam steps on batches of B labelled segments of random rays through the rest pose
    and 31 random twist/bend/taper poses of w's scene (distance head's bias at half a voxel).
    Returns (model, seconds, final losses)."""
    import torch
    sp = S.scene_of(w)
    occ = torch.zeros(w.N ** 3, dtype=torch.uint8, device="cuda")
    P.nif_voxelize(w.scene_kind, sp, w.N, occ)
    o, d = [torch.as_tensor(a).cuda() for a in S.rays_random(n_rays, w.seed + seed_offset)]
    kd, sd = S.random_poses(31, w.seed + seed_offset + 1, kinds=(S.TWIST, S.BEND, S.TAPER))
    kd = np.concatenate([[S.IDENTITY], kd]).astype(np.int32)
    sd = np.concatenate([[0.0], sd]).astype(np.float32)
    g = P.Grid(occ, w.N, kd, sd)
    ds = _segment_dataset(P, g, o, d, torch.as_tensor(np.linspace(0, n_rays, 33).astype(np.int64)).cuda(),
                          w.scene_kind, sp, 16)
    del g, o, d
    model, secs, losses = _train_model(P, w.model, ds, steps, B, False, w.seed + seed_offset + 2,
                                       f"{w.name} model", dist_bias=0.5 / w.N)
    return model, secs, losses


def oracle_errors(P, model, m, w, kinds, strengths, occ_np, o, d, got):
    """Per-head errors of query outputs `got` (numpy, rays o, d of one pose) against the FP64
    oracle run on the model's FP32 master weights and the tables as the GPU reads them."""
    import torch

    import nif_synth as S
    import oracle
    t, prm, _ = [v.cpu().numpy() for v in model.get_params()]
    torch.cuda.synchronize()
    tab = t.reshape(m.table_levels, m.table_size, m.feat_dim)
    tab64 = oracle.round_f16(tab) if m.table_dtype == S.TABLE_F16 else tab.astype(np.float64)
    ref = oracle.query(m, tab64, prm.astype(np.float64), w.N, occ_np, kinds, strengths, o, d)
    both = (got["hit"] == 1) & (ref["hit"] == 1)
    q = lambda e: [float(np.quantile(e, 0.5)), float(np.quantile(e, 0.99))] if len(e) else [0.0, 0.0]
    rel_t = np.abs(got["t"][both] - ref["t"][both]) / np.maximum(np.abs(ref["t"][both]), 1e-6)
    ng = np.stack([got["nx"], got["ny"], got["nz"]], 1)[both]
    ang = np.degrees(np.arccos(np.clip(np.sum(ng * ref["normal"][both], 1), -1.0, 1.0)))
    alb = np.abs(np.stack([got["ar"], got["ag"], got["ab"]], 1)[both] - ref["albedo"][both]).sum(1)
    return {"hit_accuracy": float(np.mean(got["hit"] == ref["hit"])),
            "material_accuracy": float(np.mean(got["material"][both] == ref["material"][both])) if both.any() else 1.0,
            "distance_rel_p50_p99": q(rel_t), "normal_deg_p50_p99": q(ang), "albedo_l1_p50_p99": q(alb),
            "rays": int(len(o[0])), "hits_compared": int(both.sum())}


def precision_leg(steps=5, train_steps=1500, sample=512):
    """4x128 MLP on 2 poses x 1024^2 rays: query rays/s with the MLP in FP32, BF16 and FP16, on a
    model trained by this library (FP32); per-head errors of each precision against the FP64
    oracle on every `sample`-th ray of both poses."""
    import torch

    import nif_synth as S
    import paper_2604_24666_amd as P

    w = S.workload("spheres64_p")
    m = w.model
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = torch.zeros(w.N ** 3, dtype=torch.uint8, device="cuda")
    P.nif_voxelize(w.scene_kind, sp, w.N, occ)
    model, train_s, train_losses = trained_model(P, S, w, train_steps)
    kinds, strengths = S.poses(w)
    n_pose = w.cam_res ** 2
    o_all = torch.empty((3, 2 * n_pose), device="cuda")
    d_all = torch.empty((3, 2 * n_pose), device="cuda")
    cams = []
    for p in range(2):
        o, d = S.rays_camera(w.cam_res, w.cam_az_deg[p], tile=w.cam_tile)
        cams.append((o, d))
        o_all[:, p * n_pose:(p + 1) * n_pose] = torch.as_tensor(o).cuda()
        d_all[:, p * n_pose:(p + 1) * n_pose] = torch.as_tensor(d).cuda()
    off = torch.tensor([0, n_pose, 2 * n_pose], dtype=torch.int64, device="cuda")
    grid = P.Grid(occ, w.N, kinds, strengths)
    rays = P.make_rays(o_all, d_all, off)
    out = P.alloc_hits(2 * n_pose, "cuda")
    hits = P.hits_struct(out)
    occ_np = occ.cpu().numpy()
    res = {}
    ref = None
    for prec, name in ((0, "fp32"), (1, "bf16"), (2, "fp16")):
        ms = timed(lambda: P.nif_query(model.h, grid.h, rays, 2 * n_pose, hits, 0, prec, None), steps, 2)
        res[name] = {"rays_per_s": 2 * n_pose / (ms * 1e-3), "ms": ms}
        got = {k: v.cpu().numpy() for k, v in out.items()}
        if ref is None:
            ref = got
        else:
            res[name]["vs_fp32"] = head_errors(got, ref)
        per_pose = []
        for p in range(2):
            sl = np.arange(p * n_pose, (p + 1) * n_pose)[::sample]
            o, d = cams[p][0][:, ::sample], cams[p][1][:, ::sample]
            g = {k: v[sl].astype(np.float64) if v.dtype.kind == "f" else v[sl] for k, v in got.items()}
            per_pose.append(oracle_errors(P, model, m, w, int(kinds[p]), float(strengths[p]), occ_np, o, d, g))
        res[name]["vs_oracle"] = {"pose_twist": per_pose[0], "pose_bend": per_pose[1]}
        log(f"precision leg {name}: {ms:.2f} ms; vs oracle {res[name]['vs_oracle']}")
    return {"workload": "spheres64_p: 2 poses (twist, bend s=1) x 1024^2 pinhole rays in 8x8 tiles, 16-level 2^19 FP16 grid, "
                        f"MLP 832-128x4-12 trained by this library ({train_steps} FP32 Adam steps of 2^16 labelled "
                        f"segments, {train_s:.1f} s, final losses {[round(x, 4) for x in train_losses]})", **res,
            "note": f"vs_oracle: every {sample}th ray of each pose against the FP64 oracle on the FP32 master weights "
                    "(the BF16/FP16 error includes the rounding of the weights); vs_fp32: the FP32 path on all rays"}


def head_errors(got, ref):
    """Per-head disagreement of a low-precision query with the FP32 one."""
    both = (got["hit"] == 1) & (ref["hit"] == 1)
    q = lambda e: [float(np.quantile(e, 0.5)), float(np.quantile(e, 0.99))] if len(e) else [0.0, 0.0]
    rel_t = np.abs(got["t"][both] - ref["t"][both]) / np.maximum(np.abs(ref["t"][both]), 1e-6)
    ng = np.stack([got["nx"], got["ny"], got["nz"]], 1)[both]
    nr = np.stack([ref["nx"], ref["ny"], ref["nz"]], 1)[both]
    ang = np.degrees(np.arccos(np.clip(np.sum(ng * nr, 1), -1.0, 1.0)))
    alb = np.abs(np.stack([got["ar"], got["ag"], got["ab"]], 1)[both] -
                 np.stack([ref["ar"], ref["ag"], ref["ab"]], 1)[both]).sum(1)
    return {"hit_agreement": float(np.mean(got["hit"] == ref["hit"])),
            "material_agreement": float(np.mean(got["material"][both] == ref["material"][both])) if both.any() else 1.0,
            "distance_rel_p50_p99": q(rel_t), "normal_deg_p50_p99": q(ang), "albedo_l1_p50_p99": q(alb)}


TRAIN_VARIANTS = {"bf16": (1, 0), "fp32": (0, 0), "bf16_stored": (1, 1), "fp32_stored": (0, 1)}


def train_leg(steps=5, B=1 << 18, variants=tuple(TRAIN_VARIANTS)):
    """Training step on 2^18 ray-voxel segments of the 128^3 blob scene (fwd + loss + bwd + Adam);
    the segments are traced and labelled on the GPU (nif_trace, nif_label)."""
    import torch

    import nif_synth as S
    import paper_2604_24666_amd as P

    w = S.workload("blobs128")
    m = w.model
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = torch.zeros(w.N ** 3, dtype=torch.uint8, device="cuda")
    P.nif_voxelize(w.scene_kind, sp, w.N, occ)
    kinds, strengths = S.random_poses(8, w.seed, kinds=(S.TWIST, S.BEND))
    grid = P.Grid(occ, w.N, kinds, strengths)
    nr = 1 << 17
    o, d = S.rays_random(nr, w.seed)
    off = torch.as_tensor(np.linspace(0, nr, 9).astype(np.int64)).cuda()
    tr = grid.trace(torch.as_tensor(o).cuda(), torch.as_tensor(d).cuda(), off, max_seg=16)
    cnt = tr["count"].clamp(max=16)
    valid = (torch.arange(16, device="cuda")[None, :] < cnt[:, None]).reshape(-1)
    x0 = tr["x0"].reshape(3, -1)[:, valid][:, :B].contiguous()
    x1 = tr["x1"].reshape(3, -1)[:, valid][:, :B].contiguous()
    assert x0.shape[1] == B, f"only {x0.shape[1]} segments traced"
    # labels from the analytic scene along each rest-space chord, on the GPU (natural hit ratio)
    P.label(w.scene_kind, sp, x0[:, :4096].contiguous(), x1[:, :4096].contiguous())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lab = P.label(w.scene_kind, sp, x0, x1)
    torch.cuda.synchronize()
    label_ms = (time.perf_counter() - t0) * 1e3
    log(f"train leg: {B} segments labelled in {label_ms:.2f} ms")
    hit, t, nrm, alb, mat = lab["hit"], lab["t"], lab["normal"], lab["albedo"], lab["material"]
    hit_ratio = float(hit.float().mean().item())
    batch = P.Batch(x0.data_ptr(), x1.data_ptr(), hit.data_ptr(), t.data_ptr(), nrm.data_ptr(), alb.data_ptr(),
                    mat.data_ptr())
    res = {}
    for vname in variants:
        prec, store = TRAIN_VARIANTS[vname]
        name = vname.split("_")[0]
        if True:
            model = P.Model(m)
            model.set_params(S.init_tables(m, w.seed + 100), S.init_mlp(m, w.seed + 100))
            P.nif_model_reserve(model.h, B)
            if store:
                P.nif_model_reserve_encoding(model.h)
            cfg = P.TrainCfg(1e-2, 1e-3, 1e-3, 0.9, 0.999, 1e-8, prec, 0.0, 0, store)
            losses = torch.zeros(16, device="cuda")
            ms = timed(lambda: P.nif_train_step(model.h, batch, B, cfg, losses), steps, 2)
            achieved = TRAIN_BYTES_PER_SAMPLE * B / (ms * 1e-3) / 1e9
            r = {"samples_per_s": B / (ms * 1e-3), "ms_per_step": ms, "loss": float(losses[5]),
                 "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                              "kernel": "training step (all kernels of one step)",
                              "algorithmic_bytes": f"{TRAIN_BYTES_PER_SAMPLE} B per sample (gathers, recomputed "
                                                   "gathers, FP32 table-gradient payload, dense Adam)"}}
            if store:
                res.setdefault("stored_encoding", {})[name] = r
            else:
                res[name] = r
            log(f"train leg {name}{' stored encoding' if store else ''}: {ms:.2f} ms per step of {B}")
            del model
    return {"workload": "blobs128: 32-Gaussian blob field at 128^3, B = 2^18 segments traced on the GPU from random "
                        "rays through 8 random twist/bend poses, labelled on the GPU from the analytic scene, "
                        "MLP 832-128x4-12, 16-level 2^19 FP16 grid, Adam", "hit_ratio": hit_ratio,
            "label_ms": label_ms,
            "encoding_policy": "bf16 / fp32: the backward recomputes the encoding (chunks of 2^17 samples); "
                               "stored_encoding: the forward keeps the [B][832] FP32 encoding for the backward",
            **res}


def _segment_dataset(P, grid, o, d, off, scene_kind, sp, max_seg):
    """Every occupied-voxel segment of the rays (rest-space chords) with its labels."""
    import torch
    tr = grid.trace(o, d, off, max_seg=max_seg)
    cnt = tr["count"].clamp(max=max_seg)
    valid = (torch.arange(max_seg, device="cuda")[None, :] < cnt[:, None]).reshape(-1)
    x0 = tr["x0"].reshape(3, -1)[:, valid].contiguous()
    x1 = tr["x1"].reshape(3, -1)[:, valid].contiguous()
    lab = P.label(scene_kind, sp, x0, x1)
    return {"x0": x0, "x1": x1, "hit": lab["hit"], "t": lab["t"], "n": lab["normal"], "a": lab["albedo"],
            "m": lab["material"]}


def _ground_truth(P, grid, o, d, off, scene_kind, sp, max_seg=64):
    """Per ray, the first labelled hit along its occupied-voxel segments: distance along the
    ray (entry + hit fraction of the segment, the local linear approximation) and the
    rest-space normal there.  Rays with more than max_seg segments are flagged invalid."""
    import torch
    tr = grid.trace(o, d, off, max_seg=max_seg)
    n = o.shape[1]
    cnt = tr["count"]
    ok = cnt <= max_seg
    c = cnt.clamp(max=max_seg)
    valid = torch.arange(max_seg, device="cuda")[None, :] < c[:, None]
    x0 = tr["x0"].reshape(3, -1)[:, valid.reshape(-1)].contiguous()
    x1 = tr["x1"].reshape(3, -1)[:, valid.reshape(-1)].contiguous()
    lab = P.label(scene_kind, sp, x0, x1)
    hit = torch.zeros((n, max_seg), dtype=torch.bool, device="cuda")
    hit[valid] = lab["hit"].bool()
    lr = (x1 - x0).norm(dim=0)
    frac = torch.zeros((n, max_seg), device="cuda")
    frac[valid] = torch.where(lr > 0, (lab["t"] / lr).clamp(0, 1), torch.zeros_like(lr))
    nrm = torch.zeros((3, n, max_seg), device="cuda")
    nrm[:, valid] = lab["normal"]
    any_hit = hit.any(dim=1)
    first = torch.where(any_hit, hit.int().argmax(dim=1), torch.zeros_like(cnt, dtype=torch.int64))
    r = torch.arange(n, device="cuda")
    tin, tout = tr["t_in"][r, first], tr["t_out"][r, first]
    t = tin + frac[r, first] * (tout - tin)
    return {"valid": ok, "hit": any_hit & ok, "t": t, "n": nrm[:, r, first]}


def _errors(P, model, grid, o, d, off, gt):
    import torch
    q = grid.query(model, o, d, off)
    ph = q["hit"].bool()
    both = ph & gt["hit"]
    pn = torch.stack([q["nx"], q["ny"], q["nz"]])
    cos = (pn * gt["n"]).sum(0).clamp(-1, 1)
    ang = torch.rad2deg(torch.acos(cos))
    return {"distance_mae": float((q["t"] - gt["t"]).abs()[both].mean()),
            "normal_deg": float(ang[both].mean()),
            "hit_agreement": float((ph == gt["hit"])[gt["valid"]].float().mean()),
            "rays_compared": int(both.sum())}


def _train_model(P, m, ds, steps, B, fixed, seed, tag, dist_bias=0.0):
    """Adam on minibatches of B segments drawn uniformly from the labelled set ds; the distance
    head's bias starts at dist_bias (so that a ReLU distance head is live from the first step)."""
    import torch

    import nif_synth as S
    n_seg = ds["x0"].shape[1]
    model = P.Model(m)
    prm = S.init_mlp(m, seed)
    prm[m.n_mlp_params - m.n_heads + 1] = dist_bias
    model.set_params(S.init_tables(m, seed), prm)
    P.nif_model_reserve(model.h, B)
    cfg = P.TrainCfg(1e-2, 1e-3, 1e-3, 0.9, 0.999, 1e-8, P.PREC_FP32, 0.0, int(fixed))
    losses = torch.zeros(16, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed + 100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        idx = torch.randint(0, n_seg, (B,), device="cuda", generator=gen)
        b = {k: (v[:, idx] if v.dim() == 2 else v[idx]).contiguous() for k, v in ds.items()}
        batch = P.Batch(b["x0"].data_ptr(), b["x1"].data_ptr(), b["hit"].data_ptr(), b["t"].data_ptr(),
                        b["n"].data_ptr(), b["a"].data_ptr(), b["m"].data_ptr())
        P.nif_train_step(model.h, batch, B, cfg, losses)
        if (it + 1) % 500 == 0:
            torch.cuda.synchronize()
            log(f"{tag}: step {it + 1}/{steps}, loss {float(losses[5]):.4f}")
    torch.cuda.synchronize()
    return model, time.perf_counter() - t0, [float(x) for x in losses[:6].cpu()]


def _variant_study(w, variants, steps, B, eval_poses):
    """Train each (name, model, fixed task weights, training set, distance bias) variant on
    labelled segments of the workload's scene (2^20 random rays through the rest pose only, or
    through the rest pose and 31 random twist/bend/taper poses) and measure the first-hit
    query against labelled ground truth on 4 x 256^2 pinhole rays at the rest pose and at
    eval_poses (unseen)."""
    import torch

    import nif_synth as S
    import paper_2604_24666_amd as P

    sp = S.scene_of(w)
    occ = torch.zeros(w.N ** 3, dtype=torch.uint8, device="cuda")
    P.nif_voxelize(w.scene_kind, sp, w.N, occ)
    nr = 1 << 20
    o, d = [torch.as_tensor(a).cuda() for a in S.rays_random(nr, w.seed + 7)]
    k_dist, s_dist = S.random_poses(31, w.seed + 8, kinds=(S.TWIST, S.BEND, S.TAPER))
    k_dist = np.concatenate([[S.IDENTITY], k_dist]).astype(np.int32)
    s_dist = np.concatenate([[0.0], s_dist]).astype(np.float32)
    data = {}
    for name, kinds, strengths in (("rest", [S.IDENTITY], [0.0]), ("poses", k_dist, s_dist)):
        if not any(v[3] == name for v in variants):
            continue
        g = P.Grid(occ, w.N, kinds, strengths)
        off = torch.as_tensor(np.linspace(0, nr, len(kinds) + 1).astype(np.int64)).cuda()
        data[name] = _segment_dataset(P, g, o, d, off, w.scene_kind, sp, 16)
        log(f"{w.name}: {data[name]['x0'].shape[1]} training segments ({name}), "
            f"hit ratio {float(data[name]['hit'].float().mean()):.3f}")
        del g
    views = [S.rays_camera(256, az) for az in (0.0, 90.0, 180.0, 270.0)]
    eo = torch.as_tensor(np.concatenate([v[0] for v in views], 1)).cuda()
    ed = torch.as_tensor(np.concatenate([v[1] for v in views], 1)).cuda()
    ne = eo.shape[1]
    evals = {}
    for name, (kinds, strengths) in (("rest", ([S.IDENTITY], [0.0])), ("deformed", eval_poses)):
        g = P.Grid(occ, w.N, kinds, strengths)
        reps = len(kinds)
        o_e, d_e = eo.repeat(1, reps).contiguous(), ed.repeat(1, reps).contiguous()
        off = torch.as_tensor(np.arange(reps + 1, dtype=np.int64) * ne).cuda()
        evals[name] = (g, o_e, d_e, off, _ground_truth(P, g, o_e, d_e, off, w.scene_kind, sp))
    res = {}
    for vname, m, fixed, dname, db in variants:
        model, train_s, losses = _train_model(P, m, data[dname], steps, B, fixed, w.seed + 200, vname, dist_bias=db)
        r = {"train_s": train_s, "final_losses": losses}
        for ename, (g, o_e, d_e, off, gt) in evals.items():
            r[ename] = _errors(P, model, g, o_e, d_e, off, gt)
        log(f"{w.name} {vname}: {r}")
        res[vname] = r
        del model
    return res


def ablation_leg(steps=2000, B=1 << 16):
    """Table 1 analogue on a synthetic scene: the original LSNIF (trained on the rest pose only),
    the deformation-aware baseline without the proposed training and encoding changes (F = 0,
    sigmoid-fraction distance, fixed task weights; trained on a pose distribution) and the
    proposed model (F = 6, ReLU log distance, uncertainty weighting; same poses).  Errors of
    the first-hit query against the labelled ground truth on the static rest pose and on
    unseen deformed poses."""
    import dataclasses

    import nif_synth as S

    w = S.workload("spheres64")
    base = w.model
    baseline = dataclasses.replace(base, pe_freqs=0, dist_head=S.DIST_SIGMOID)
    bias = 0.5 / w.N           # half a voxel: the ReLU distance head is live from the first step
    variants = (("LSNIF", baseline, True, "rest", 0.0), ("Deformed", baseline, True, "poses", 0.0),
                ("Proposed", base, False, "poses", bias), ("Proposed (distance bias 0)", base, False, "poses", 0.0))
    res = _variant_study(w, variants, steps, B, ([S.TWIST, S.BEND, S.TAPER, S.TWIST], [0.85, 0.65, 0.9, 0.35]))
    return {"workload": f"spheres64 scene (8 spheres, 64^3), 16-level 2^19 FP16 grid, MLP 64x3; {steps} Adam steps of "
                        f"B = {B} segments (the proposed head's distance bias at half a voxel, and at 0) "
                        f"drawn from 2^20 random rays through the rest pose (LSNIF) or through the "
                        f"rest pose and 31 random twist/bend/taper poses (Deformed, Proposed); evaluated on 4 x 256^2 "
                        f"pinhole rays at the rest pose and at 4 unseen poses against labelled ground truth",
            **res}


def paper_leg(steps=2000, B=1 << 16):
    """The paper's comparison of deformation results in its own configuration (32^3 voxels, a
    two-level grid with base resolution 64 and three features per entry, F = 3): the
    deformation-aware LSNIF baseline without the proposed changes (F = 0, sigmoid-fraction
    distance, fixed task weights) against the full model, both trained on the same deformed
    poses and evaluated on the same rays."""
    import dataclasses

    import nif_synth as S

    w = S.workload("spheres32_paper")
    base = w.model
    baseline = dataclasses.replace(base, pe_freqs=0, dist_head=S.DIST_SIGMOID)
    variants = (("Deformed LSNIF baseline", baseline, True, "poses", 0.0),
                ("Full model", base, False, "poses", 0.5 / w.N))
    res = _variant_study(w, variants, steps, B, (list(S.poses(w)[0]), list(S.poses(w)[1])))
    return {"workload": f"sphere scene at 32^3, 2-level grid (64, 128) with 3 features per entry, 2^19 FP16 entries, "
                        f"F = 3, MLP 84-64x3-12; {steps} Adam steps of B = {B} segments from 2^20 random rays through "
                        f"the rest pose and 31 random twist/bend/taper poses; evaluated on 4 x 256^2 pinhole rays at "
                        f"the rest pose and under twist, bend and taper at full strength against labelled ground truth",
            **res}


def render_leg(steps=1500, B=1 << 16, res=1024, reps=5):
    """Renderer-style use of a trained field under a deformation: one frame of pinhole primary
    rays (first hit), shadow rays from every primary hit to a point light (occlusion query
    with tmax, visibility bit only) and one diffuse bounce per hit (incoherent first-hit
    rays).  Throughput of each ray population, and agreement of the predicted hits and
    shadows with the labelled ground truth of the same rays."""
    import torch

    import nif_synth as S
    import paper_2604_24666_amd as P

    w = S.workload("spheres64")
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = torch.zeros(w.N ** 3, dtype=torch.uint8, device="cuda")
    P.nif_voxelize(w.scene_kind, sp, w.N, occ)
    m = w.model
    # train on rays through the rest pose and 31 random poses (as the proposed model above)
    nr = 1 << 20
    o, d = [torch.as_tensor(a).cuda() for a in S.rays_random(nr, w.seed + 7)]
    kd, sd = S.random_poses(31, w.seed + 8, kinds=(S.TWIST, S.BEND, S.TAPER))
    kd = np.concatenate([[S.IDENTITY], kd]).astype(np.int32)
    sd = np.concatenate([[0.0], sd]).astype(np.float32)
    g = P.Grid(occ, w.N, kd, sd)
    ds = _segment_dataset(P, g, o, d, torch.as_tensor(np.linspace(0, nr, 33).astype(np.int64)).cuda(),
                          w.scene_kind, sp, 16)
    del g, o, d
    model, train_s, _ = _train_model(P, m, ds, steps, B, False, w.seed + 400, "render model", dist_bias=0.5 / w.N)
    del ds
    # one frame under an unseen twist
    grid = P.Grid(occ, w.N, [S.TWIST], [0.8])
    po, pd = [torch.as_tensor(a).cuda() for a in S.rays_camera(res, 35.0)]
    n_p = po.shape[1]
    off_p = torch.as_tensor(np.array([0, n_p], np.int64)).cuda()
    prim = grid.query(model, po, pd, off_p)
    torch.cuda.synchronize()
    hit = prim["hit"].bool()
    idx = torch.nonzero(hit).squeeze(1)
    n_h = int(idx.numel())
    off_h = torch.as_tensor(np.array([0, n_h], np.int64)).cuda()
    x = po[:, idx] + prim["t"][idx][None, :] * pd[:, idx]
    light = torch.tensor([[2.0], [1.5], [3.0]], device="cuda")
    to_l = light - x
    dist = to_l.norm(dim=0)
    sdir = (to_l / dist).contiguous()
    eps = 2.0 / w.N                                   # leave the hit voxel before looking for occluders
    so = (x + eps * sdir).contiguous()
    stmax = (dist - eps).contiguous()
    sbit = torch.empty(n_h, dtype=torch.uint8, device="cuda")
    shits = P.Hits(sbit.data_ptr(), *([None] * (len(P.Hits._fields_) - 1)))
    srays = P.make_rays(so, sdir, off_h, stmax)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(w.seed + 500)
    bdir = torch.randn((3, n_h), device="cuda", generator=gen)
    bdir = (bdir / bdir.norm(dim=0)).contiguous()
    bo = (x + eps * bdir).contiguous()
    bout = P.alloc_hits(n_h, "cuda")
    bh = P.hits_struct(bout)
    brays = P.make_rays(bo, bdir, off_h)
    pout = P.alloc_hits(n_p, "cuda")
    ph = P.hits_struct(pout)
    prays = P.make_rays(po, pd, off_p)
    timings = {}
    st = torch.zeros(4, dtype=torch.int64, device="cuda")
    for name, fn, n in (("primary", lambda: P.nif_query(model.h, grid.h, prays, n_p, ph, 0, 0, st), n_p),
                        ("shadow", lambda: P.nif_query(model.h, grid.h, srays, n_h, shits, 0, 0, st), n_h),
                        ("bounce", lambda: P.nif_query(model.h, grid.h, brays, n_h, bh, 0, 0, st), n_h)):
        st.zero_()
        ms = timed(fn, reps, 2)
        evals = float(st[1]) / (reps + 2)
        timings[name] = {"rays": n, "ms": ms, "rays_per_s": n / (ms * 1e-3), "network_evals": evals}
        log(f"render {name}: {n} rays in {ms:.3f} ms, {evals:.0f} network evaluations")
    full = grid.query(model, so, sdir, off_h, tmax=stmax)
    nq = full["n_queried"].float()
    timings["shadow"]["n_queried_mean_max"] = [float(nq.mean()), float(nq.max())]
    nq = bout["n_queried"].float()
    timings["bounce"]["n_queried_mean_max"] = [float(nq.mean()), float(nq.max())]
    nq = pout["n_queried"].float()
    timings["primary"]["n_queried_mean_max"] = [float(nq.mean()), float(nq.max())]
    # agreement with the labelled ground truth of the same rays
    gtp = _ground_truth(P, grid, po, pd, off_p, w.scene_kind, sp)
    gts = _ground_truth(P, grid, so, sdir, off_h, w.scene_kind, sp)
    occl_gt = gts["hit"] & (gts["t"] < stmax)
    lit = sbit == 0
    shade = torch.zeros(n_p, device="cuda")
    nrm = torch.stack([prim["dnx"], prim["dny"], prim["dnz"]])[:, idx]      # deformed-space normals
    alb = torch.stack([prim["ar"], prim["ag"], prim["ab"]])[:, idx].mean(0)
    shade[idx] = alb * (0.15 + 0.85 * lit.float() * (nrm * sdir).sum(0).abs())
    valid = gts["valid"]
    return {"workload": f"spheres64 scene, model trained {steps} steps (B = {B}) on the rest pose and 31 random poses; "
                        f"frame of {res}^2 pinhole rays under an unseen twist (0.8), shadow rays from every primary "
                        f"hit to a point light (tmax = distance to the light), one uniform-direction bounce per hit",
            "train_s": train_s, **timings,
            "frame_ms": sum(v["ms"] for v in timings.values()),
            "primary_hit_agreement": float((hit == gtp["hit"])[gtp["valid"]].float().mean()),
            "shadow_agreement": float(((sbit == 1) == occl_gt)[valid].float().mean()),
            "shadowed_fraction": float((sbit == 1).float().mean()), "bounce_hit_fraction": float(bout["hit"].float().mean()),
            "mean_shade": float(shade.mean())}


def batched_leg(replays=50, warmup=5, train_steps=1000):
    """16 poses of uneven ray counts (half pinhole, half secondary) in one persistent launch,
    replayed from a captured graph: aggregate rays/s (median launch) and per-pose completion
    latency p50/p99 over all replays (device wall-clock stamps)."""
    import torch

    import nif_synth as S
    import paper_2604_24666_amd as P

    w = S.workload("blobs128_b")
    m = w.model
    sp = S.scene_of(w)
    occ = torch.zeros(w.N ** 3, dtype=torch.uint8, device="cuda")
    P.nif_voxelize(w.scene_kind, sp, w.N, occ)
    n_p = 16
    kinds, strengths = S.random_poses(n_p, w.seed, kinds=(S.TWIST, S.BEND, S.TAPER))
    grid = P.Grid(occ, w.N, kinds, strengths)
    counts = S.uneven_counts(n_p, w.seed)
    n = int(counts.sum())
    o, d = S.batched_rays(counts, w.seed, [grid.bounds(p) for p in range(n_p)])
    o_all, d_all = torch.as_tensor(o).cuda(), torch.as_tensor(d).cuda()
    off = torch.as_tensor(np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)).cuda()
    model, train_s, train_losses = trained_model(P, S, S.workload("blobs128"), train_steps)
    rays = P.make_rays(o_all, d_all, off)
    out = P.alloc_hits(n, "cuda")
    hits = P.hits_struct(out)
    stats = torch.zeros(5 + 2 * n_p, dtype=torch.int64, device="cuda")
    khz = P.nif_wall_clock_khz()
    res = {}
    def measure(prec, dealing):
        """Median launch time and per-pose completion latencies of the graph-replayed launch."""
        torch.cuda.synchronize()
        s_cap = torch.cuda.Stream()
        call = lambda: P.nif_query(model.h, grid.h, rays, n, hits, P.Q_POSE_TIMES | dealing, prec, stats,
                                   stream=s_cap)
        with torch.cuda.stream(s_cap):
            call()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s_cap):
            call()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        launch_ms, lat = [], []
        evals = 0
        for i in range(warmup + replays):
            with torch.cuda.stream(s_cap):
                a.record(s_cap)
                g.replay()
                b.record(s_cap)
            torch.cuda.synchronize()
            st = stats.cpu().numpy()
            if i < warmup:
                evals = int(st[1])
                continue
            launch_ms.append(a.elapsed_time(b))
            assert np.array_equal(st[5 + n_p:5 + 2 * n_p], counts), "rays finished per pose"
            lat.append((st[5:5 + n_p] - st[4]).astype(np.float64) / khz)     # ticks -> ms
        del g
        lat = np.concatenate(lat)
        evals_per_launch = (int(stats.cpu().numpy()[1]) - evals) / replays
        return float(np.median(launch_ms)), float(np.mean(launch_ms)), lat, evals_per_launch

    for prec, name in ((1, "bf16"), (0, "fp32")):
        shape = tuned_query_shape("blobs128_b", model.h, grid.h, rays, n, hits, prec)
        ms, ms_mean, lat, evals_per_launch = measure(prec, 0)
        achieved = evals_per_launch * GATHER_BYTES_PER_EVAL / (ms_mean * 1e-3) / 1e9
        res[name] = {"rays_per_s": n / (ms * 1e-3), "ms_per_launch_median": ms,
                     "pose_latency_ms_p50": float(np.quantile(lat, 0.5)),
                     "pose_latency_ms_p99": float(np.quantile(lat, 0.99)),
                     "hit_rate": float(out["hit"].float().mean().item()),
                     "network_evals_per_launch": evals_per_launch,
                     "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                                  "kernel": "k_query (one persistent launch over the 16 poses)",
                                  "algorithmic_bytes": f"{GATHER_BYTES_PER_EVAL} B of hash-corner gathers per "
                                                       "network evaluation"},
                     "launch_shape": {"blocks_per_cu": shape[0], "rays_per_wave": shape[1]}}
        log(f"batched leg {name}: {ms:.2f} ms per launch, pose latency p50 {res[name]['pose_latency_ms_p50']:.2f} "
            f"p99 {res[name]['pose_latency_ms_p99']:.2f} ms")
        ms, _, lat, _ = measure(prec, P.Q_POSE_ORDER)
        res[name]["pose_ordered"] = {"rays_per_s": n / (ms * 1e-3), "ms_per_launch_median": ms,
                                     "pose_latency_ms_p50": float(np.quantile(lat, 0.5)),
                                     "pose_latency_ms_p99": float(np.quantile(lat, 0.99)),
                                     "note": "NIF_Q_POSE_ORDER: each XCD's ray range walks the poses in order"}
        log(f"batched leg {name} pose-ordered: {ms:.2f} ms per launch, pose latency p50 "
            f"{res[name]['pose_ordered']['pose_latency_ms_p50']:.2f} p99 "
            f"{res[name]['pose_ordered']['pose_latency_ms_p99']:.2f} ms")
    # traversal alone: the voxel proxy walks every ray to its first occupied voxel, against the
    # BF16 launch (a lower bound of the query's traversal, which walks on past empty segments)
    P.nif_query(model.h, grid.h, rays, n, hits, P.Q_NO_NETWORK, 1, None)
    pa, pb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    pa.record()
    for _ in range(3):
        P.nif_query(model.h, grid.h, rays, n, hits, P.Q_NO_NETWORK, 1, None)
    pb.record()
    torch.cuda.synchronize()
    proxy_ms = pa.elapsed_time(pb) / 3
    res["time_shares"] = {"traversal_to_first_occupied_voxel": proxy_ms / res["bf16"]["ms_per_launch_median"],
                          "proxy_ms": proxy_ms}
    log(f"batched leg voxel proxy: {proxy_ms:.2f} ms")
    return {"workload": f"blobs128_b: 16 poses (twist/bend/taper, s ~ U(0,1]), {n} rays in uneven counts "
                        f"[{int(counts.min())}, {int(counts.max())}], half pinhole (random azimuth), half secondary "
                        f"(origin uniform in the pose's occupied deformed box, direction uniform on S^2); one "
                        f"persistent launch replayed from a captured graph, median of {replays} after {warmup} "
                        f"warm-up; MLP 832-128x4-12 trained by this library on the scene ({train_steps} FP32 Adam "
                        f"steps, {train_s:.1f} s, final losses {[round(x, 4) for x in train_losses]})",
            "rays": n, **res}


def ceilings_leg():
    """Device ceilings measured on this GPU (nif_microbench), read beside the published peaks:
    streaming HBM reads; random 4- and 8-byte gathers from a 32 MiB table (the FP16 hash tables'
    size: resident in the Infinity Cache, not in one XCD's 4 MB L2) and from a 1 MiB one (L2
    resident); the FP32 16x16x4 and BF16 16x16x16 MFMA forms the kernels use."""
    import paper_2604_24666_amd as P
    out = {}
    for name, kind, nbytes, nops, unit in (
            ("hbm_read", P.MB_HBM_READ, 4 << 30, 1, "GB/s"),
            ("gather4_32MiB", P.MB_GATHER4, 32 << 20, 1 << 30, "GB/s"),
            ("gather8_32MiB", P.MB_GATHER8, 32 << 20, 1 << 30, "GB/s"),
            ("gather4_1MiB", P.MB_GATHER4, 1 << 20, 1 << 30, "GB/s"),
            ("mfma_f32_16x16x4", P.MB_MFMA_F32, 0, 1 << 26, "TFLOP/s"),
            ("mfma_bf16_16x16x16", P.MB_MFMA_BF16, 0, 1 << 26, "TFLOP/s")):
        rate, ms = P.nif_microbench(kind, nbytes, nops, 5)
        out[name] = {"value": rate / (1e9 if unit == "GB/s" else 1e12), "unit": unit, "ms": ms}
        if kind in (P.MB_GATHER4, P.MB_GATHER8):
            out[name]["gathers_per_s"] = rate / (4 if kind == P.MB_GATHER4 else 8)
        log(f"ceiling {name}: {out[name]['value']:.1f} {unit} ({ms:.3f} ms per launch)")
    return out


def run_legs(legs, train_variants=tuple(TRAIN_VARIANTS)):
    res = {}
    if "ceilings" in legs:
        res["ceilings"] = ceilings_leg()
    if "torus" in legs:
        res["torus16"] = torus_leg()
    if "precision" in legs:
        res["precision_compare"] = precision_leg()
    if "train" in legs:
        res["train"] = train_leg(variants=train_variants)
    if "batched" in legs:
        res["batched"] = batched_leg()
    if "ablation" in legs:
        res["ablation"] = ablation_leg()
    if "paper" in legs:
        res["paper"] = paper_leg()
    if "render" in legs:
        res["render"] = render_leg()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="spheres64")
    ap.add_argument("--precision", type=int, default=0, help="0 FP32, 1 BF16, 2 FP16 MLP")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rebuild", action="store_true", help="time the query only (grids built once)")
    ap.add_argument("--legs-only", action="store_true",
                    help="profiling runs: skip the headline query and the CPU baseline, print the legs' JSON")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 3 times (scale for HBM byte counters)")
    ap.add_argument("--train-variants", default=",".join(TRAIN_VARIANTS),
                    help="training-leg variants: " + ",".join(TRAIN_VARIANTS))
    ap.add_argument("--legs", default="ceilings,torus,precision,train,batched",
                    help="extra measurements: ceilings,torus,precision,train,batched,ablation,paper,render (empty for none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print("copied 3 x 1 GiB", flush=True)
        return

    import paper_2604_24666_amd as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.legs_only:
        res = run_legs([x for x in args.legs.split(",") if x], tuple(x for x in args.train_variants.split(",") if x))
        print(json.dumps(res), flush=True)
        return
    log("setup ...")
    ctx = setup(args.workload, args.precision)
    grid, model, out, n = ctx["grid"], ctx["model"], ctx["out"], ctx["n"]
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    rays = P.make_rays(ctx["o"], ctx["d"], ctx["off"])
    hits = P.hits_struct(out)
    stream = torch.cuda.current_stream()

    def rebuild():
        P.nif_grid_update(grid.h, ctx["kinds"], ctx["strengths"])

    def query():
        P.nif_query(model.h, grid.h, rays, n, hits, 0, args.precision, stats)

    rebuild()
    shape = tuned_query_shape(args.workload, model.h, grid.h, rays, n, hits, args.precision)
    log(f"launch shape: {shape[0]} workgroups per CU, {shape[1]} rays per wave")
    for i in range(args.warmup):
        if not args.no_rebuild:
            rebuild()
        query()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup}")
    # timed region: whole steps
    stats.zero_()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    evb = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        evb[i][0].record(stream)
        if not args.no_rebuild:
            rebuild()
        evb[i][1].record(stream)
        ev[i][0].record(stream)
        query()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    q_ms = np.array([a.elapsed_time(b) for a, b in ev])
    b_ms = np.array([a.elapsed_time(b) for a, b in evb])
    st = stats.cpu().numpy()
    evals_per_launch = st[1] / args.steps
    achieved = evals_per_launch * GATHER_BYTES_PER_EVAL / (q_ms.mean() * 1e-3) / 1e9
    ms_step = dt * 1e3 / args.steps
    log(f"query kernel {q_ms.mean():.3f} ms (min {q_ms.min():.3f}), grid rebuild {b_ms.mean():.3f} ms, "
        f"step {ms_step:.3f} ms, network evaluations/launch {evals_per_launch:.0f}")
    hit_rate = float(out["hit"].float().mean().item())
    # traversal alone: the voxel proxy (NIF_Q_NO_NETWORK) walks every ray to its first occupied
    # voxel, a lower bound of the traversal inside the query (which walks on past empty-hit segments)
    pe0, pe1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    P.nif_query(model.h, grid.h, rays, n, hits, P.Q_NO_NETWORK, args.precision, None)
    pe0.record(stream)
    for _ in range(3):
        P.nif_query(model.h, grid.h, rays, n, hits, P.Q_NO_NETWORK, args.precision, None)
    pe1.record(stream)
    torch.cuda.synchronize()
    proxy_ms = pe0.elapsed_time(pe1) / 3
    query()                                    # restore the outputs of the full query
    torch.cuda.synchronize()
    res = {
        "metric": "ray queries/sec (first-hit neural intersection, FP32 MLP; train samples/s reported separately)",
        "value": n / (ms_step * 1e-3),
        "unit": "rays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": ["f32", "bf16", "f16"][args.precision], "data": "synthetic",
        "config": {"workload": f"{args.workload}: 8 spheres at 64^3, 24 poses (twist/bend/taper x 8 strengths), "
                               f"24 x 1024^2 pinhole rays in 8x8 screen tiles, 16-level 2^19 FP16 hash grid, F=6, MLP 832-64x3-12",
                   "rays_per_step": n, "poses": len(ctx["kinds"]), "grid_rebuilt_each_step": not args.no_rebuild},
        "launch_shape": {"blocks_per_cu": shape[0], "rays_per_wave": shape[1], "chosen_by": "nif_autotune_query"},
        "query_kernel_ms": float(q_ms.mean()), "grid_rebuild_ms": float(b_ms.mean()),
        "network_evals_per_step": float(evals_per_launch), "hit_rate": hit_rate,
        "time_shares": {"grid_rebuild": float(b_ms.mean()) / ms_step,
                        "traversal_to_first_occupied_voxel": proxy_ms / float(q_ms.mean()),
                        "note": "grid re-pose per step and the voxel-proxy launch (traversal only, to each ray's "
                                "first occupied voxel) against the fused query; the paper reports 2-3 % for its BVH"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": kquery_traffic_bytes(),
                     "kernel": "k_query (fused traversal + encoding + MLP)",
                     "algorithmic_bytes": f"{GATHER_BYTES_PER_EVAL} B of hash-corner gathers per network evaluation"},
    }
    legs = [x for x in args.legs.split(",") if x]
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(ctx)
    del ctx, grid, model, out, hits, rays
    torch.cuda.empty_cache()
    P.nif_set_query_blocks_per_cu(12)           # the legs below use the default launch shape
    P.nif_set_query_rays_per_wave(0)            # unless they tune their own
    res.update(run_legs(legs, tuple(x for x in args.train_variants.split(",") if x)))
    if cpu is not None:
        res["cpu_baseline"] = cpu
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
