"""End-to-end parity of the fused first-hit query against the oracle's query on the same
rays, poses, tables and weights.

Rays that are grazing (geometry may legitimately differ) or ambiguous (some evaluated
segment has |hit logit| within 1e-4 of its scale |b| + sum|w||h|) are counted and excluded;
on the rest, hit decisions, voxels and segment counts must be exact.  The continuous
outputs are reported (p50 / p99 / max) and held to loose end-to-end bounds (t and rest point
2e-4, albedo 5e-4, normal 1e-2 times min(|z_n| / RMS, 1)): the encoding's
finest levels turn the ~1e-7-1e-6 FP32 error of the rest-space points into head errors well
above the 1e-5 that the network stage meets on identical inputs (test_gpu_network)."""
import numpy as np
import pytest

import nif_synth as S
from _helpers import dev_f32, model_params, offsets, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2604_24666_amd as P
    return P


def _grazing(orc, N, occ, kind, s, o, d):
    V = orc.lattice_vertices(kind, s, N)
    return orc.trace(N, occ, V, o, d, brute=N <= 16)[4] != 0


def _compare(orc, P, m, tab_seen, prm, N, occ, kind, s, o, d, got, sl=slice(None), tmax=None, exclude=None):
    s64 = float(np.float32(s))
    ref = orc.query(m, tab_seen, prm.astype(np.float64), N, occ, kind, s64, o, d, tmax=tmax)
    graz = _grazing(orc, N, occ, kind, s64, o, d)
    amb = ref["margin"] < 1e-4
    ok = ~graz & ~amb
    if exclude is not None:
        ok &= ~exclude
    g = {k: v[sl] for k, v in got.items()}
    say(f"  rays {len(ok)}  grazing {int(graz.sum())}  ambiguous {int((amb & ~graz).sum())}  "
        f"hits {int(ref['hit'][ok].sum())}")
    assert np.array_equal(g["hit"][ok], ref["hit"][ok])
    for name in ("n_queried", "cell"):
        bad = np.nonzero(ok & (g[name] != ref[name]))[0]
        for i in bad[:8]:
            say(f"    {name} mismatch ray {i}: got {g[name][i]} ref {ref[name][i]}  hit {ref['hit'][i]}  "
                f"t got {g['t'][i]:.6f} ref {ref['t'][i]:.6f}  nq got {g['n_queried'][i]} ref {ref['n_queried'][i]}  "
                f"margin {ref['margin'][i]:.3g}")
        assert len(bad) == 0, name
    h = ok & (ref["hit"] == 1)
    xr = np.stack([g["xr"], g["yr"], g["zr"]], 1)
    nrm = np.stack([g["nx"], g["ny"], g["nz"]], 1)
    alb = np.stack([g["ar"], g["ag"], g["ab"]], 1)
    # a normal is z_n / |z_n|: its error grows as 1 / |z_n| for small predicted vectors
    zn = np.linalg.norm(ref["zhit"][h][:, 2:5], axis=1)
    zn_rms = np.sqrt(np.mean(zn ** 2)) if len(zn) else 1.0
    dnrm = np.stack([g["dnx"], g["dny"], g["dnz"]], 1)
    errs = {"t": np.abs(g["t"][h] - ref["t"][h]), "xrest": np.abs(xr[h] - ref["xrest"][h]).max(1, initial=0),
            "normal": np.abs(nrm[h] - ref["normal"][h]).max(1, initial=0) * np.minimum(zn / zn_rms, 1.0),
            "dnormal": np.abs(dnrm[h] - ref["dnormal"][h]).max(1, initial=0) * np.minimum(zn / zn_rms, 1.0),
            "albedo": np.abs(alb[h] - ref["albedo"][h]).max(1, initial=0)}
    bounds = {"t": 2e-4, "xrest": 2e-4, "normal": 1e-2, "dnormal": 1e-2, "albedo": 5e-4}
    for k, e in errs.items():
        if len(e):
            say(f"    {k:7s} p50 {np.quantile(e, .5):.2e}  p99 {np.quantile(e, .99):.2e}  max {e.max():.2e}")
            assert e.max() <= bounds[k], k
    assert np.array_equal(g["material"][h], ref["material"][h])
    miss = ok & (ref["hit"] == 0)
    assert np.all(np.isinf(g["t"][miss])) and np.all(g["cell"][miss] == -1)
    return int(ok.sum()), int(h.sum())


def _np(out):
    return {k: v.cpu().numpy().astype(np.float64) if v.dtype.is_floating_point else v.cpu().numpy()
            for k, v in out.items()}


@pytest.mark.parametrize("kind,s", [(S.TWIST, 1.0), (S.BEND, 1.0), (S.TAPER, 0.5), (S.TWIST_BEND, 1.0)])
def test_query_torus16_fp32(orc, P, kind, s):
    import torch
    w = S.workload("torus16")
    m = w.model
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N)
    tab, prm, seen = model_params(m, w.seed + 100, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    grid = P.Grid(torch.as_tensor(occ).cuda(), w.N, [kind], [s])
    o, d = S.rays_random(4096, w.seed)
    say(f"query torus16 kind={kind} s={s}")
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    got = _np(grid.query(model, dev_f32(o), dev_f32(d), offsets([4096]), stats=stats))
    st = stats.cpu().numpy()
    assert st[0] == 4096 and st[1] == got["n_queried"].sum()
    n_ok, n_hit = _compare(orc, P, m, seen, prm, w.N, occ, kind, s, o, d, got)
    assert n_ok > 3500 and n_hit > 200


ABLATIONS = {"sigmoid_head": dict(dist_head=S.DIST_SIGMOID), "no_pe": dict(pe_freqs=0),
             "no_pe_sigmoid_head": dict(pe_freqs=0, dist_head=S.DIST_SIGMOID),
             "per_sample_tables": dict(per_sample_tables=1), "concat_encoding": dict(concat_encoding=1)}


@pytest.mark.parametrize("variant", list(ABLATIONS))
def test_query_torus16_ablation_switches(orc, P, variant):
    """The baselines' switches on the query path: the sigmoid-fraction distance head and F = 0
    (grid encoding alone), against the oracle under a twist."""
    import dataclasses
    import torch
    w = S.workload("torus16")
    m = dataclasses.replace(w.model, **ABLATIONS[variant])
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N)
    tab, prm, seen = model_params(m, w.seed + 101, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    grid = P.Grid(torch.as_tensor(occ).cuda(), w.N, [S.TWIST], [1.0])
    o, d = S.rays_random(4096, w.seed + 1)
    say(f"query torus16 ablation {variant}")
    got = _np(grid.query(model, dev_f32(o), dev_f32(d), offsets([4096])))
    n_ok, n_hit = _compare(orc, P, m, seen, prm, w.N, occ, S.TWIST, 1.0, o, d, got)
    assert n_ok > 3500 and n_hit > 50


def test_query_occlusion_tmax_matches_oracle(orc, P):
    """Shadow-ray form: per-ray tmax bounds the walk and the hit; the bit alone (every other
    output pointer null) equals the full query's.  Rays whose unbounded hit distance or any
    voxel entry lies within 1e-4 of tmax are decided by rounding and are excluded."""
    import torch
    w = S.workload("torus16")
    m = w.model
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N)
    tab, prm, seen = model_params(m, w.seed + 100, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    grid = P.Grid(torch.as_tensor(occ).cuda(), w.N, [S.BEND], [1.0])
    n = 4096
    o, d = S.rays_random(n, w.seed + 2)
    tmax = np.random.default_rng(w.seed + 3).uniform(1.0, 3.0, n).astype(np.float32)
    say("query torus16 occlusion tmax")
    got = _np(grid.query(model, dev_f32(o), dev_f32(d), offsets([n]), tmax=dev_f32(tmax)))
    full = orc.query(m, seen, prm.astype(np.float64), w.N, occ, S.BEND, 1.0, o, d)
    V = orc.lattice_vertices(S.BEND, 1.0, w.N)
    _, tin, _, cnt, _ = orc.trace(w.N, occ, V, o, d, with_flags=False)
    near = np.array([np.any(np.abs(tin[i, :cnt[i]] - tmax[i]) < 1e-4) for i in range(n)])
    near |= np.abs(full["t"] - tmax) < 1e-4
    n_ok, n_hit = _compare(orc, P, m, seen, prm, w.N, occ, S.BEND, 1.0, o, d, got, tmax=tmax.astype(np.float64),
                           exclude=near)
    cut = (full["hit"] == 1) & (full["t"] >= tmax)
    say(f"  hits beyond tmax (reported as misses) {int(cut.sum())}")
    assert n_ok > 3500 and n_hit > 100 and cut.sum() > 20
    bit = torch.empty(n, dtype=torch.uint8, device="cuda")
    hits = P.Hits(bit.data_ptr(), *([None] * (len(P.Hits._fields_) - 1)))
    keep = (dev_f32(o), dev_f32(d), offsets([n]), dev_f32(tmax))
    P.nif_query(model.h, grid.h, P.make_rays(*keep), n, hits, 0, 0, None)
    torch.cuda.synchronize()
    assert np.array_equal(bit.cpu().numpy(), got["hit"])


def test_query_rays_per_wave_does_not_change_results(P):
    """16-ray and 64-ray waves evaluate the same segments with the same arithmetic: every
    output is bit-identical, for a small and a large launch of the sphere workload."""
    import torch
    w = S.workload("spheres64")
    m = w.model
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = torch.zeros(w.N ** 3, dtype=torch.uint8, device="cuda")
    P.nif_voxelize(w.scene_kind, sp, w.N, occ)
    tab, prm, _ = model_params(m, w.seed + 100, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    grid = P.Grid(occ, w.N, [S.TWIST, S.BEND], [0.7, 0.9])
    for n in (3001, 300001):
        o, d = S.rays_inside(n, w.seed + n)
        off = offsets([n // 2, n - n // 2])
        outs = []
        for rpw in (16, 64, 0):
            P.nif_set_query_rays_per_wave(rpw)
            outs.append(_np(grid.query(model, dev_f32(o), dev_f32(d), off)))
        P.nif_set_query_rays_per_wave(0)
        say(f"rays per wave n={n}: hits {int(outs[0]['hit'].sum())}")
        for k in outs[0]:
            for other in outs[1:]:
                assert np.array_equal(outs[0][k], other[k], equal_nan=True), k


def test_autotuner_picks_a_shape_of_its_space_and_keeps_results(P):
    import torch
    w = S.workload("torus16")
    m = w.model
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = torch.zeros(w.N ** 3, dtype=torch.uint8, device="cuda")
    P.nif_voxelize(w.scene_kind, sp, w.N, occ)
    tab, prm, _ = model_params(m, w.seed + 100, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    grid = P.Grid(occ, w.N, [S.TWIST, S.TAPER], [1.0, 0.5])
    n = 20000
    o, d = S.rays_random(n, w.seed + 5)
    keep = (dev_f32(o), dev_f32(d), offsets([n // 3, n - n // 3]))
    rays = P.make_rays(*keep)
    ref = _np(grid.query(model, *keep))
    out = P.alloc_hits(n, "cuda")
    bpc, rpw, ms = P.nif_autotune_query(model.h, grid.h, rays, n, P.hits_struct(out), 0, 1)
    say(f"autotuned: {bpc} workgroups per CU, {rpw} rays per wave, {ms:.3f} ms")
    assert bpc in (4, 6, 8, 10, 12, 14, 16, 20, 24) and rpw in (16, 64) and 0 < ms < 1e3
    got = _np(out)
    for k in ref:
        assert np.array_equal(ref[k], got[k], equal_nan=True), k
    again = _np(grid.query(model, *keep))
    for k in ref:
        assert np.array_equal(ref[k], again[k], equal_nan=True), k
    with pytest.raises(P.NifError):
        P.nif_autotune_query(model.h, grid.h, rays, n, P.hits_struct(out), 0, 0)
    P.nif_set_query_blocks_per_cu(12)
    P.nif_set_query_rays_per_wave(0)


def test_query_voxel_proxy_is_the_first_segment(orc, P):
    import torch
    w = S.workload("torus16")
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N)
    grid = P.Grid(torch.as_tensor(occ).cuda(), w.N, [S.TWIST], [1.0])
    o, d = S.rays_random(2048, 3)
    say("query proxy torus16")
    got = _np(grid.query(None, dev_f32(o), dev_f32(d), offsets([2048]), no_network=True))
    tr = grid.trace(dev_f32(o), dev_f32(d), offsets([2048]), max_seg=4)
    cnt = tr["count"].cpu().numpy()
    assert np.array_equal(got["hit"], (cnt > 0).astype(np.uint8))
    h = cnt > 0
    assert np.array_equal(got["t"][h], tr["t_in"].cpu().numpy()[h, 0].astype(np.float64))
    assert np.array_equal(got["cell"][h], tr["cell"].cpu().numpy()[h, 0])
    nrm = np.stack([got["nx"], got["ny"], got["nz"]], 1)[h]
    assert np.allclose(np.abs(nrm).sum(1), 1.0)               # an axis-aligned rest-space face normal


def test_query_spheres64_full_workload_sampled(orc, P):
    """The 24-pose, 24 x 1024^2-ray workload in one launch; sampled rays of several poses are
    checked against the oracle one by one."""
    import torch
    w = S.workload("spheres64")
    m = w.model
    sp = S.scene_params(w.scene_kind, w.seed)
    occ_ref = orc.voxelize(w.scene_kind, sp, w.N)
    occ = torch.as_tensor(occ_ref).cuda()
    tab, prm, seen = model_params(m, w.seed + 100, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    kinds, strengths = S.poses(w)
    grid = P.Grid(occ, w.N, kinds, strengths)
    n_pose = w.cam_res ** 2
    say("query spheres64: 24 poses x 1024^2 rays")
    o_all = torch.empty((3, 24 * n_pose), device="cuda")
    d_all = torch.empty((3, 24 * n_pose), device="cuda")
    for p in range(24):
        o, d = S.rays_camera(w.cam_res, w.cam_az_deg[p], tile=w.cam_tile)
        o_all[:, p * n_pose:(p + 1) * n_pose] = dev_f32(o)
        d_all[:, p * n_pose:(p + 1) * n_pose] = dev_f32(d)
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    out = grid.query(model, o_all, d_all, offsets([n_pose] * 24), stats=stats)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    say(f"  rays done {st[0]}  network evaluations {st[1]}  degenerate voxel tests {st[2]}")
    assert st[0] == 24 * n_pose
    hit = out["hit"].cpu().numpy()
    assert 0.01 < hit.mean() < 0.5
    rng = np.random.default_rng(0)
    total_ok = 0
    for p in (0, 5, 11, 16, 23):
        # mostly rays that touch the geometry, plus a few that do not
        touch = np.nonzero(out["n_queried"][p * n_pose:(p + 1) * n_pose].cpu().numpy() > 0)[0]
        idx = np.sort(np.concatenate([rng.choice(touch, 300, replace=False), rng.integers(0, n_pose, 50)]))
        o, d = S.rays_camera(w.cam_res, w.cam_az_deg[p], tile=w.cam_tile)
        got = {k: v[p * n_pose:(p + 1) * n_pose][torch.as_tensor(idx).cuda()] for k, v in out.items()}
        say(f"  pose {p} kind {kinds[p]} s {strengths[p]}")
        n_ok, _ = _compare(orc, P, m, seen, prm, w.N, occ_ref, int(kinds[p]), float(strengths[p]),
                           o[:, idx], d[:, idx], _np(got))
        total_ok += n_ok
    assert total_ok > 1500


def test_query_pose_times_and_graph_replays(orc, P):
    """Several poses of uneven ray counts in one launch: per-pose finished counts and completion
    stamps; the same launch captured in a graph and replayed (with other GPU work between the
    replays) gives the eager launch's outputs bit for bit on every replay."""
    import torch
    w = S.workload("torus16")
    m = w.model
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N)
    tab, prm, _ = model_params(m, w.seed + 100, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    kinds, strengths = [S.TWIST, S.BEND, S.TAPER], [1.0, 0.5, 0.75]
    grid = P.Grid(torch.as_tensor(occ).cuda(), w.N, kinds, strengths)
    counts = [3000, 77, 5000]
    n = sum(counts)
    o, d = S.rays_random(n, 21)
    o, d = dev_f32(o), dev_f32(d)
    off = offsets(counts)
    rays = P.make_rays(o, d, off)
    say("query pose times + graph replays, torus16, 3 poses")
    ref = P.alloc_hits(n, "cuda")
    stats = torch.zeros(5 + 2 * 3, dtype=torch.int64, device="cuda")
    P.nif_query(model.h, grid.h, rays, n, P.hits_struct(ref), P.Q_POSE_TIMES, P.PREC_FP32, stats)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    assert st[0] == n and list(st[8:11]) == counts
    assert np.all(st[5:8] >= st[4]) and P.nif_wall_clock_khz() > 0
    out = P.alloc_hits(n, "cuda")
    s_cap = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s_cap):
        P.nif_query(model.h, grid.h, rays, n, P.hits_struct(out), P.Q_POSE_TIMES, P.PREC_FP32, stats,
                    stream=s_cap)
    other = P.alloc_hits(n, "cuda")
    for rep in range(3):
        for v in out.values():
            v.zero_()
        stats.zero_()
        g.replay()
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(out[k], ref[k]) or (out[k].dtype.is_floating_point and
                                                   torch.equal(torch.nan_to_num(out[k]), torch.nan_to_num(ref[k]))), k
        st = stats.cpu().numpy()
        assert st[0] == n and list(st[8:11]) == counts and np.all(st[5:8] >= st[4])
        # eager work between the replays
        grid.query(model, o, d, off, out=other)
        torch.cuda.synchronize()
    del g


def test_grid_bounds_hold_the_deformed_occupied_voxels(orc, P):
    import torch
    w = S.workload("torus16")
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N)
    kinds, strengths = [S.TWIST, S.BEND, S.TAPER], [1.0, 1.0, 1.0]
    grid = P.Grid(torch.as_tensor(occ).cuda(), w.N, kinds, strengths)
    N = w.N
    cells = np.nonzero(occ)[0]
    for p, (k, s) in enumerate(zip(kinds, strengths)):
        V = orc.lattice_vertices(k, s, N).reshape(N + 1, N + 1, N + 1, 3)
        i, j, kk = cells % N, (cells // N) % N, cells // (N * N)
        corners = np.concatenate([V[kk + c, j + b, i + a] for a in (0, 1) for b in (0, 1) for c in (0, 1)])
        lo, hi = grid.bounds(p)
        ext = corners.max(0) - corners.min(0)
        say(f"  pose {p}: box {np.round(lo, 4)} .. {np.round(hi, 4)}")
        assert np.all(lo <= corners.min(0) + 1e-6) and np.all(hi >= corners.max(0) - 1e-6)
        # padded by 1e-5 on each side; FP32 lattice vs the FP64 one differ by ~1e-7
        assert np.all(lo >= corners.min(0) - 2e-5) and np.all(hi <= corners.max(0) + 2e-5 + 1e-6 * ext)


def test_query_blobs128_multi_pose_fp32_sampled(orc, P):
    """The 128^3 blob scene with the 832-128x4-12 network (FP32) under three poses in one
    launch: camera and secondary rays of each pose against the oracle's query."""
    import torch
    w = S.workload("blobs128")
    m = w.model
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N)
    tab, prm, seen = model_params(m, w.seed + 100, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    kinds, strengths = [S.TWIST, S.BEND, S.TAPER], [0.9, 0.7, 1.0]
    grid = P.Grid(torch.as_tensor(occ).cuda(), w.N, kinds, strengths)
    os_, ds_ = [], []
    for p in range(3):
        o, d = S.rays_camera(64, 25.0 + 120.0 * p, sub=9)
        oi, di = S.rays_inside(250, 90 + p, lo=0.25, hi=0.75)
        os_.append(np.concatenate([o, oi], axis=1))
        ds_.append(np.concatenate([d, di], axis=1))
    counts = [x.shape[1] for x in os_]
    say(f"query blobs128 fp32, 3 poses in one launch, rays {counts}")
    got = _np(grid.query(model, dev_f32(np.concatenate(os_, axis=1)), dev_f32(np.concatenate(ds_, axis=1)),
                         offsets(counts)))
    start, total_ok, total_hit = 0, 0, 0
    for p in range(3):
        sl = slice(start, start + counts[p])
        say(f"  pose {p}: kind {kinds[p]} s {strengths[p]}")
        n_ok, n_hit = _compare(orc, P, m, seen, prm, w.N, occ, kinds[p], strengths[p], os_[p], ds_[p], got, sl=sl)
        total_ok += n_ok
        total_hit += n_hit
        start += counts[p]
    assert total_ok > 1200 and total_hit > 200


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16"])
def test_query_batched_workload_poses_sampled(orc, P, prec):
    """The batched workload's launch as the benchmark issues it (16 poses of the blob scene,
    8 M rays in uneven counts, half pinhole and half secondary), sampled rays of two poses (one
    twist or bend, one taper where present) against the oracle; at BF16 the decisions and heads
    are held to the rounding-error model (test_query_low_precision_end_to_end)."""
    import torch
    w = S.workload("blobs128_b")
    m = w.model
    sp = S.scene_of(w)
    occ_ref = orc.voxelize(w.scene_kind, sp, w.N)
    n_p = 16
    kinds, strengths = S.random_poses(n_p, w.seed, kinds=(S.TWIST, S.BEND, S.TAPER))
    grid = P.Grid(torch.as_tensor(occ_ref).cuda(), w.N, kinds, strengths)
    counts = S.uneven_counts(n_p, w.seed)
    o, d = S.batched_rays(counts, w.seed, [grid.bounds(p) for p in range(n_p)])
    tab, prm, seen = model_params(m, w.seed + 100, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    say(f"batched workload prec={prec}: {int(counts.sum())} rays, 16 poses")
    out = grid.query(model, dev_f32(o), dev_f32(d), offsets(counts), precision=prec)
    torch.cuda.synchronize()
    start = np.concatenate([[0], np.cumsum(counts)])
    picks = [int(np.flatnonzero(kinds != S.TAPER)[0]), int(np.flatnonzero(kinds == S.TAPER)[0])]
    rng = np.random.default_rng(7)
    total = 0
    for p in picks:
        c = int(counts[p])
        idx = np.sort(np.concatenate([rng.choice(c // 2, 200, replace=False), c // 2 + rng.choice(c - c // 2, 200, replace=False)]))
        sel = start[p] + idx
        got = _np({k: v[torch.as_tensor(sel).cuda()] for k, v in out.items()})
        say(f"  pose {p}: kind {kinds[p]} s {strengths[p]:.3f}, rays {c}")
        if prec == 0:
            n_ok, _ = _compare(orc, P, m, seen, prm, w.N, occ_ref, int(kinds[p]), float(strengths[p]),
                               o[:, sel], d[:, sel], got)
        else:
            n_ok = _compare_low(orc, m, seen, prm, w.N, occ_ref, int(kinds[p]), float(strengths[p]), o[:, sel],
                                d[:, sel], got, prec)
        total += n_ok
    assert total > 500


def _segment_points(kind, s, o, d, t0, t1, orc):
    o64, d64 = o.T.astype(np.float64), d.T.astype(np.float64)
    return (orc.deform_inv(kind, s, o64 + t0[:, None] * d64), orc.deform_inv(kind, s, o64 + t1[:, None] * d64))


def _compare_low(orc, m, seen, prm, N, occ, kind, s, o, d, g, prec):
    """End-to-end BF16 / FP16 query against the oracle on the same rounded weights.  Decisions
    (hit, voxel, segments evaluated) must agree on rays that are not grazing and whose smallest
    |hit logit| / (|b| + sum |w||h|) over the evaluated segments exceeds 7 times the largest
    sigma / scale the rounding-error model gives for the hit logit (twice that for safety);
    on hits, t, normal, albedo within 7 sigma of the model (plus the FP32 end-to-end bounds of
    the geometry) and the material wherever its two top logits are 7 sigma apart."""
    import _bounds as BD
    from _helpers import quantized_mlp
    q = quantized_mlp(prm, prec)
    s64 = float(np.float32(s))
    ref = orc.query(m, seen, q, N, occ, kind, s64, o, d)
    graz = _grazing(orc, N, occ, kind, s64, o, d)
    h = ref["hit"] == 1
    si = ref["seginfo"]
    x0, x1 = _segment_points(kind, s64, o[:, h], d[:, h], si[h, 0], si[h, 1], orc)
    fw = BD.forward(orc, m, seen, q, x0, x1, prec)
    W, b = BD.layers(m, q)[-1]
    scale0 = np.abs(fw["acts"][-1]) @ np.abs(W[0]) + abs(b[0])
    kappa = max(2.0 * BD.LAMBDA * float((fw["sz"][:, 0] / scale0).max()), 1e-4)
    amb = ref["margin"] <= kappa
    ok = ~graz & ~amb
    say(f"    rays {len(ok)}  grazing {int(graz.sum())}  ambiguous (margin <= {kappa:.2e}) {int((amb & ~graz).sum())}"
        f"  hits {int(ref['hit'][ok].sum())}")
    assert np.array_equal(g["hit"][ok], ref["hit"][ok])
    assert np.array_equal(g["cell"][ok], ref["cell"][ok]) and np.array_equal(g["n_queried"][ok], ref["n_queried"][ok])
    hh = ok[h]                                   # hit rays (in the order of fw's rows) that are compared
    z, sz = fw["z"][hh], fw["sz"][hh]
    lam = BD.LAMBDA
    t0, t1, lr = si[h][hh, 0], si[h][hh, 1], si[h][hh, 2]
    f = np.clip(np.maximum(z[:, 1], 0.0) / lr, 0.0, 1.0)
    inner = (f > 0) & (f < 1)
    tb = np.where(inner, (t1 - t0) * lam * sz[:, 1] / lr, (t1 - t0) * np.clip(lam * sz[:, 1] / lr, 0, 1)) + 2e-4
    idx = np.flatnonzero(ok & h)
    et = np.abs(g["t"][idx] - ref["t"][idx])
    nrm = np.stack([g["nx"], g["ny"], g["nz"]], 1)[idx]
    vl = np.linalg.norm(z[:, 2:5], axis=1)
    sv = lam * np.linalg.norm(sz[:, 2:5], axis=1)
    vrms = np.sqrt(np.mean(vl ** 2)) if len(vl) else 1.0
    # the model's share, and the FP32 end-to-end share of the geometry (1e-2 at the RMS |z_n|)
    nb = np.minimum(2.0, sv / np.maximum(vl - sv, 1e-30) + 1e-2 * np.maximum(1.0, vrms / np.maximum(vl, 1e-30)))
    en = np.abs(nrm - ref["normal"][idx]).max(1)
    alb = np.stack([g["ar"], g["ag"], g["ab"]], 1)[idx]
    ea = np.abs(alb - ref["albedo"][idx]).max(1)
    ab = 0.25 * lam * sz[:, 5:8].max(1) + 5e-4
    say(f"    t err p99 {np.quantile(et, .99) if len(et) else 0:.2e}  normal p99 {np.quantile(en, .99) if len(en) else 0:.2e}"
        f"  albedo p99 {np.quantile(ea, .99) if len(ea) else 0:.2e}")
    assert np.all(et <= tb) and np.all(en <= nb) and np.all(ea <= ab)
    zm = z[:, 8:]
    top2 = np.sort(zm, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > lam * (sz[:, 8:].max(1) * 2)
    assert np.array_equal(g["material"][idx][clear], ref["material"][idx][clear])
    return int(ok.sum())


@pytest.mark.parametrize("prec", [1, 2], ids=["bf16", "fp16"])
def test_query_low_precision_end_to_end(orc, P, prec):
    """The precision comparison's workload (the sphere scene, twist and bend at full strength,
    MLP 832-128x4-12) end to end at BF16 / FP16 on sampled camera rays of both poses."""
    import torch
    w = S.workload("spheres64_p")
    m = w.model
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N)
    tab, prm, seen = model_params(m, w.seed + 100, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    kinds, strengths = S.poses(w)
    grid = P.Grid(torch.as_tensor(occ).cuda(), w.N, kinds, strengths)
    os_, ds_ = [], []
    for p in range(2):
        o, d = S.rays_camera(w.cam_res, w.cam_az_deg[p], tile=w.cam_tile, sub=997)
        os_.append(o)
        ds_.append(d)
    counts = [x.shape[1] for x in os_]
    say(f"query spheres64_p prec={prec}, rays {counts}")
    got = _np(grid.query(model, dev_f32(np.concatenate(os_, axis=1)), dev_f32(np.concatenate(ds_, axis=1)),
                         offsets(counts), precision=prec))
    start, total = 0, 0
    for p in range(2):
        sl = slice(start, start + counts[p])
        say(f"  pose {p}: kind {kinds[p]} s {strengths[p]}")
        total += _compare_low(orc, m, seen, prm, w.N, occ, int(kinds[p]), float(strengths[p]), os_[p], ds_[p],
                              {k: v[sl] for k, v in got.items()}, prec)
        start += counts[p]
    assert total > 1500


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16"])
def test_query_paper_configuration(orc, P, prec):
    """The configuration of the paper's comparison of deformation results (the sphere scene at
    32^3, two grid levels of three features each, F = 3) under its three poses in one launch:
    sampled camera rays of every pose against the oracle (BF16 on the same rounded weights)."""
    import torch
    w = S.workload("spheres32_paper")
    m = w.model
    occ = orc.voxelize(w.scene_kind, S.scene_of(w), w.N)
    tab, prm, seen = model_params(m, w.seed + 100, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    kinds, strengths = S.poses(w)
    grid = P.Grid(torch.as_tensor(occ).cuda(), w.N, kinds, strengths)
    os_, ds_ = [], []
    for p in range(len(kinds)):
        o, d = S.rays_camera(w.cam_res, w.cam_az_deg[p], sub=97)
        os_.append(o)
        ds_.append(d)
    counts = [x.shape[1] for x in os_]
    say(f"query spheres32_paper prec={prec}, rays {counts}")
    got = _np(grid.query(model, dev_f32(np.concatenate(os_, axis=1)), dev_f32(np.concatenate(ds_, axis=1)),
                         offsets(counts), precision=prec))
    start, n_ok, n_hit = 0, 0, 0
    for p in range(len(kinds)):
        sl = slice(start, start + counts[p])
        say(f"  pose {p}: kind {kinds[p]} s {strengths[p]}")
        g = {k: v[sl] for k, v in got.items()}
        if prec == 0:
            a, b = _compare(orc, P, m, seen, prm, w.N, occ, int(kinds[p]), float(strengths[p]), os_[p], ds_[p], g)
        else:
            a, b = _compare_low(orc, m, seen, prm, w.N, occ, int(kinds[p]), float(strengths[p]), os_[p], ds_[p], g,
                                prec), 0
        n_ok += a
        n_hit += b
        start += counts[p]
    assert n_ok > 0.9 * sum(counts)
    if prec == 0:
        assert n_hit > 300


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16"])
def test_query_pose_ordered_dealing_gives_the_same_results(orc, P, prec):
    """NIF_Q_POSE_ORDER changes only which wave takes which ray: over poses of uneven counts
    (one empty, one with fewer rays than the 8 per-XCD ranges) every per-ray output equals the
    default dealing's bit for bit and every ray of every pose is done once.  (Completion order
    is a scheduling effect, not checked here: a launch this small has all its rays in flight at
    once; bench.py's batched leg measures the per-pose latencies.)"""
    import torch
    w = S.workload("torus16")
    m = w.model
    occ = orc.voxelize(w.scene_kind, S.scene_params(w.scene_kind, w.seed), w.N)
    tab, prm, _ = model_params(m, w.seed + 100, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    kinds, strengths = [S.TWIST, S.BEND, S.TAPER, S.TWIST, S.BEND], [1.0, 0.5, 0.75, 0.3, 0.9]
    grid = P.Grid(torch.as_tensor(occ).cuda(), w.N, kinds, strengths)
    counts = [20000, 0, 5, 9000, 30001]
    n = sum(counts)
    o, d = S.rays_random(n, 31)
    keep = (dev_f32(o), dev_f32(d), offsets(counts))
    rays = P.make_rays(*keep)
    say(f"query pose-ordered dealing, torus16, poses {counts}, prec {prec}")
    outs, sts = [], []
    for flags in (P.Q_POSE_TIMES, P.Q_POSE_TIMES | P.Q_POSE_ORDER):
        out = P.alloc_hits(n, "cuda")
        stats = torch.zeros(5 + 2 * len(counts), dtype=torch.int64, device="cuda")
        P.nif_query(model.h, grid.h, rays, n, P.hits_struct(out), flags, prec, stats)
        torch.cuda.synchronize()
        outs.append(out)
        sts.append(stats.cpu().numpy())
    for k in outs[0]:
        a, b = outs[0][k], outs[1][k]
        assert torch.equal(a, b) or (a.dtype.is_floating_point and torch.equal(torch.nan_to_num(a), torch.nan_to_num(b))), k
    P_ = len(counts)
    for st in sts:
        assert st[0] == n and list(st[5 + P_:5 + 2 * P_]) == counts
