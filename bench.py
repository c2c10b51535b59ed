"""Benchmark of the deformation-aware neural intersection query on one MI355X.

One step = one pass of the query path over the whole workload: every ray of every pose is
traversed through the occupied deformed voxels, its segments are mapped to rest space,
encoded and run through the MLP front to back until the first hit (one persistent kernel
launch).  The per-pose deformed grids are rebuilt each step as well (nif_grid_update), as an
animation would.  Default workload: 8 random spheres voxelized at 64^3, 24 poses
(twist/bend/taper x 8 strengths), 1024x1024 pinhole rays per pose, 16-level 2^19 FP16 hash
grid, 6 PE frequencies, MLP 832->64x3->12, FP32.

Prints one JSON line (see the keys below).  --gpus N > 1 is refused: this build runs on one
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
HBM_PEAK_GBS = 8000.0

# HBM bytes that k_query moves per launch on the default workload, from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE; KiB summed over the launch) scaled by what the same counters read for a
# plain 1 GiB device copy (bench.py --calibrate-copy).  They hold only for the kernel sources they
# were taken on (SHA-256 of KQUERY_SOURCES); otherwise the traffic is reported as null.
KQUERY_SOURCES = ["csrc/nif_query.hip", "csrc/nif_net.hpp", "csrc/nif_trace.hpp", "csrc/nif_device.hpp",
                  "csrc/nif_internal.hpp", "build.py"]
KQUERY_TRAFFIC = {
    "sources_sha256": "ef32949a6190a51f12b9f6dc5fa50fb8a8c47a1779e7394a495445a50c7005b4",
    "fetch_kib": 1.1497e8, "write_kib": 1.70192e6,          # per k_query<64, FP32> launch, default workload
    "fetch_scale": 1048576 / 524302, "write_scale": 1048576 / 1048576,   # 1 GiB copy reads 524,302 / writes 1,048,576 KiB
}


def kquery_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KQUERY_SOURCES:
        with open(os.path.join(ROOT, "paper_2604_24666_amd", f), "rb") as fh:
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
        o, d = S.rays_camera(w.cam_res, w.cam_az_deg[p])
        o_all[:, p * n_pose:(p + 1) * n_pose] = torch.as_tensor(o).cuda()
        d_all[:, p * n_pose:(p + 1) * n_pose] = torch.as_tensor(d).cuda()
    off = torch.as_tensor(np.arange(len(kinds) + 1, dtype=np.int64) * n_pose).cuda()
    grid = P.Grid(occ, w.N, kinds, strengths)
    out = P.alloc_hits(n, "cuda")
    return dict(w=w, m=m, sp=sp, occ=occ, model=model, grid=grid, o=o_all, d=d_all, off=off, out=out, n=n,
                kinds=kinds, strengths=strengths, precision=precision)


def cpu_baseline(ctx, sample_stride: int = 16):
    """The FP64 oracle's query on a strided subset of pose 0's camera rays, timed on the host."""
    import nif_synth as S
    import oracle

    w, m = ctx["w"], ctx["m"]
    occ = ctx["occ"].cpu().numpy()
    tab = S.init_tables(m, w.seed + 100)
    tab64 = oracle.round_f16(tab) if m.table_dtype == S.TABLE_F16 else tab.astype(np.float64)
    prm = S.init_mlp(m, w.seed + 100).astype(np.float64)
    o, d = S.rays_camera(w.cam_res, w.cam_az_deg[0], sub=sample_stride)
    oracle.query(m, tab64, prm, w.N, occ, int(ctx["kinds"][0]), float(ctx["strengths"][0]), o[:, :256], d[:, :256])
    t0 = time.perf_counter()
    oracle.query(m, tab64, prm, w.N, occ, int(ctx["kinds"][0]), float(ctx["strengths"][0]), o, d)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": o.shape[1] / dt, "unit": "rays/s", "cores": cores, "kind": "oracle",
            "sample": f"{o.shape[1]} rays (every {sample_stride}th pixel of pose 0, "
                      f"{['identity', 'twist', 'bend', 'taper'][int(ctx['kinds'][0])]} s={float(ctx['strengths'][0])}), "
                      f"FP64 oracle, {dt:.1f} s"}


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


def precision_leg(steps=5):
    """4x128 MLP on 2 poses x 1024^2 rays: query rays/s with the MLP in FP32, BF16 and FP16."""
    import torch

    import nif_synth as S
    import paper_2604_24666_amd as P

    w = S.workload("spheres64_p")
    m = w.model
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = torch.zeros(w.N ** 3, dtype=torch.uint8, device="cuda")
    P.nif_voxelize(w.scene_kind, sp, w.N, occ)
    model = P.Model(m)
    model.set_params(S.init_tables(m, w.seed + 100), S.init_mlp(m, w.seed + 100))
    kinds, strengths = S.poses(w)
    n_pose = w.cam_res ** 2
    o_all = torch.empty((3, 2 * n_pose), device="cuda")
    d_all = torch.empty((3, 2 * n_pose), device="cuda")
    for p in range(2):
        o, d = S.rays_camera(w.cam_res, w.cam_az_deg[p])
        o_all[:, p * n_pose:(p + 1) * n_pose] = torch.as_tensor(o).cuda()
        d_all[:, p * n_pose:(p + 1) * n_pose] = torch.as_tensor(d).cuda()
    off = torch.tensor([0, n_pose, 2 * n_pose], dtype=torch.int64, device="cuda")
    grid = P.Grid(occ, w.N, kinds, strengths)
    rays = P.make_rays(o_all, d_all, off)
    out = P.alloc_hits(2 * n_pose, "cuda")
    hits = P.hits_struct(out)
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
        log(f"precision leg {name}: {ms:.2f} ms {res[name].get('vs_fp32', '')}")
    return {"workload": "spheres64_p: 2 poses (twist, bend s=1) x 1024^2 pinhole rays, 16-level 2^19 FP16 grid, "
                        "MLP 832-128x4-12 (Xavier init)", **res,
            "note": "vs_fp32 compares with the FP32 path on the same rays (which the parity tests hold to the "
                    "FP64 oracle); per-head errors against the oracle itself: tests/test_gpu_network.py"}


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


def train_leg(steps=5, B=1 << 18):
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
    for prec, name in ((1, "bf16"), (0, "fp32")):
        model = P.Model(m)
        model.set_params(S.init_tables(m, w.seed + 100), S.init_mlp(m, w.seed + 100))
        P.nif_model_reserve(model.h, B)
        cfg = P.TrainCfg(1e-2, 1e-3, 1e-3, 0.9, 0.999, 1e-8, prec, 0.0)
        losses = torch.zeros(16, device="cuda")
        ms = timed(lambda: P.nif_train_step(model.h, batch, B, cfg, losses), steps, 2)
        res[name] = {"samples_per_s": B / (ms * 1e-3), "ms_per_step": ms, "loss": float(losses[5])}
        log(f"train leg {name}: {ms:.2f} ms per step of {B}")
        del model
    return {"workload": "blobs128: 32-Gaussian blob field at 128^3, B = 2^18 segments traced on the GPU from random "
                        "rays through 8 random twist/bend poses, labelled on the GPU from the analytic scene, "
                        "MLP 832-128x4-12, 16-level 2^19 FP16 grid, Adam", "hit_ratio": hit_ratio,
            "label_ms": label_ms, **res}


def batched_leg(replays=50, warmup=5):
    """16 poses of uneven ray counts (half pinhole, half secondary) in one persistent launch,
    replayed from a captured graph: aggregate rays/s (median launch) and per-pose completion
    latency p50/p99 over all replays (device wall-clock stamps)."""
    import torch

    import nif_synth as S
    import paper_2604_24666_amd as P

    w = S.workload("blobs128_b")
    m = w.model
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = torch.zeros(w.N ** 3, dtype=torch.uint8, device="cuda")
    P.nif_voxelize(w.scene_kind, sp, w.N, occ)
    n_p = 16
    kinds, strengths = S.random_poses(n_p, w.seed, kinds=(S.TWIST, S.BEND, S.TAPER))
    grid = P.Grid(occ, w.N, kinds, strengths)
    counts = S.uneven_counts(n_p, w.seed)
    n = int(counts.sum())
    o_all = torch.empty((3, n), device="cuda")
    d_all = torch.empty((3, n), device="cuda")
    rng = np.random.default_rng(w.seed)
    start = 0
    for p in range(n_p):
        c = int(counts[p])
        half = c // 2
        res_ = int(np.ceil(np.sqrt(half)))
        o, d = S.rays_camera(res_, float(rng.uniform(0, 360)))
        o_all[:, start:start + half] = torch.as_tensor(o[:, :half]).cuda()
        d_all[:, start:start + half] = torch.as_tensor(d[:, :half]).cuda()
        lo, hi = grid.bounds(p)
        o2, d2 = S.rays_inside(c - half, w.seed + p, lo, hi)
        o_all[:, start + half:start + c] = torch.as_tensor(o2).cuda()
        d_all[:, start + half:start + c] = torch.as_tensor(d2).cuda()
        start += c
    off = torch.as_tensor(np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)).cuda()
    model = P.Model(m)
    model.set_params(S.init_tables(m, w.seed + 100), S.init_mlp(m, w.seed + 100))
    rays = P.make_rays(o_all, d_all, off)
    out = P.alloc_hits(n, "cuda")
    hits = P.hits_struct(out)
    stats = torch.zeros(5 + 2 * n_p, dtype=torch.int64, device="cuda")
    khz = P.nif_wall_clock_khz()
    res = {}
    for prec, name in ((1, "bf16"), (0, "fp32")):
        s_cap = torch.cuda.Stream()
        call = lambda: P.nif_query(model.h, grid.h, rays, n, hits, P.Q_POSE_TIMES, prec, stats, stream=s_cap)
        with torch.cuda.stream(s_cap):
            call()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s_cap):
            call()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        launch_ms, lat = [], []
        for i in range(warmup + replays):
            with torch.cuda.stream(s_cap):
                a.record(s_cap)
                g.replay()
                b.record(s_cap)
            torch.cuda.synchronize()
            if i < warmup:
                continue
            launch_ms.append(a.elapsed_time(b))
            st = stats.cpu().numpy()
            assert np.array_equal(st[5 + n_p:5 + 2 * n_p], counts), "rays finished per pose"
            lat.append((st[5:5 + n_p] - st[4]).astype(np.float64) / khz)     # ticks -> ms
        lat = np.concatenate(lat)
        ms = float(np.median(launch_ms))
        res[name] = {"rays_per_s": n / (ms * 1e-3), "ms_per_launch_median": ms,
                     "pose_latency_ms_p50": float(np.quantile(lat, 0.5)),
                     "pose_latency_ms_p99": float(np.quantile(lat, 0.99)),
                     "hit_rate": float(out["hit"].float().mean().item())}
        log(f"batched leg {name}: {ms:.2f} ms per launch, pose latency p50 {res[name]['pose_latency_ms_p50']:.2f} "
            f"p99 {res[name]['pose_latency_ms_p99']:.2f} ms")
        del g
    return {"workload": f"blobs128_b: 16 poses (twist/bend/taper, s ~ U(0,1]), {n} rays in uneven counts "
                        f"[{int(counts.min())}, {int(counts.max())}], half pinhole (random azimuth), half secondary "
                        f"(origin uniform in the pose's occupied deformed box, direction uniform on S^2); one "
                        f"persistent launch replayed from a captured graph, median of {replays} after {warmup} "
                        f"warm-up; untrained MLP 832-128x4-12",
            "rays": n, **res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="spheres64")
    ap.add_argument("--precision", type=int, default=0, help="0 FP32, 1 BF16, 2 FP16 MLP")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rebuild", action="store_true", help="time the query only (grids built once)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 3 times (scale for HBM byte counters)")
    ap.add_argument("--legs", default="precision,train,batched",
                    help="extra measurements: precision,train,batched (empty for none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is a design note in DESIGN.md",
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
    res = {
        "metric": "ray queries/sec (first-hit neural intersection, FP32 MLP; train samples/s reported separately)",
        "value": n / (ms_step * 1e-3),
        "unit": "rays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": ["f32", "bf16", "f16"][args.precision], "data": "synthetic",
        "config": {"workload": f"{args.workload}: 8 spheres at 64^3, 24 poses (twist/bend/taper x 8 strengths), "
                               f"24 x 1024^2 pinhole rays, 16-level 2^19 FP16 hash grid, F=6, MLP 832-64x3-12",
                   "rays_per_step": n, "poses": len(ctx["kinds"]), "grid_rebuilt_each_step": not args.no_rebuild},
        "query_kernel_ms": float(q_ms.mean()), "grid_rebuild_ms": float(b_ms.mean()),
        "network_evals_per_step": float(evals_per_launch), "hit_rate": hit_rate,
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
    if "precision" in legs:
        res["precision_compare"] = precision_leg()
    if "train" in legs:
        res["train"] = train_leg()
    if "batched" in legs:
        res["batched"] = batched_leg()
    if cpu is not None:
        res["cpu_baseline"] = cpu
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
