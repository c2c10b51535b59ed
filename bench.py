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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="spheres64")
    ap.add_argument("--precision", type=int, default=0, help="0 FP32, 1 BF16, 2 FP16 MLP")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rebuild", action="store_true", help="time the query only (grids built once)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is a design note in DESIGN.md",
              file=sys.stderr)
        sys.exit(2)

    import torch

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
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_query (fused traversal + encoding + MLP)",
                     "algorithmic_bytes": f"{GATHER_BYTES_PER_EVAL} B of hash-corner gathers per network evaluation"},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        res["cpu_baseline"] = cpu_baseline(ctx)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
