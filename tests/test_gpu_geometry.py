"""GPU parity of the geometry stage (voxelization, deformed lattice, bin-grid traversal,
entry/exit points, inverse deformation) against the FP64 oracle on the same inputs.

Bar: voxel hit lists bit-exact on every non-grazing ray.  t_in / t_out and the rest-space
entry/exit points within the FP32 bound of the crossing (derivation in the design doc): an FP32
vertex error delta_V moves a crossing along the ray by delta_V / |cos| (cos between the ray
and the crossed face's normal), so
    tol_t = 4 ulp(t) + 3e-7 / max(|cos|, 1e-3),   tol_x = 2 (tol_t + 2 ulp(1)) + 3e-7,
(2 bounds the stretch of the inverse deformations on the domain)."""
import numpy as np
import pytest

import nif_synth as S
from _helpers import dev_f32, offsets, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2604_24666_amd as P
    return P


def _ulp(x):
    return np.spacing(np.abs(x).astype(np.float32)).astype(np.float64)


def _tol_t(t, c):
    return 4 * _ulp(t) + 3e-7 / np.maximum(np.abs(c), 1e-3)


def _compare_trace(orc, P, N, occ, kind, s, o, d, max_seg=96, brute=True):
    import torch
    grid = P.Grid(torch.as_tensor(occ).cuda(), N, [kind], [s])
    out = grid.trace(dev_f32(o), dev_f32(d), offsets([o.shape[1]]), max_seg=max_seg)
    torch.cuda.synchronize()
    return _check_segments(orc, N, occ, kind, s, o, d, {k: v.cpu().numpy() for k, v in out.items()}, max_seg, brute)


def _check_segments(orc, N, occ, kind, s, o, d, out, max_seg, brute):
    """Hit lists of rays o, d (SoA) traced on the GPU under one pose (out: numpy arrays of the
    rays, x0 / x1 as [3][rays][max_seg]) against the oracle's."""
    cnt = out["count"]
    cell = out["cell"]
    tin = out["t_in"].astype(np.float64)
    tout = out["t_out"].astype(np.float64)
    x0 = out["x0"].astype(np.float64)
    x1 = out["x1"].astype(np.float64)
    V = orc.lattice_vertices(kind, float(np.float32(s)), N)
    rc, rtin, rtout, rcnt, fl, cin, cout = orc.trace(N, occ, V, o, d, brute=brute, max_out=max_seg,
                                                     with_cos=True)
    ok = fl == 0
    say(f"  rays {len(cnt)}  grazing {int((~ok).sum())}  with segments {int((rcnt > 0).sum())}")
    assert np.array_equal(cnt[ok], rcnt[ok]), np.nonzero((cnt != rcnt) & ok)[0][:10]
    assert cnt.max() <= max_seg
    n_seg = 0
    worst = 0.0
    o64 = o.T.astype(np.float64)
    d64 = d.T.astype(np.float64)
    s64 = float(np.float32(s))
    for r in np.nonzero(ok & (rcnt > 0))[0]:
        k = rcnt[r]
        assert np.array_equal(cell[r, :k], rc[r, :k]), (r, cell[r, :k], rc[r, :k])
        ti, to = _tol_t(rtin[r, :k], cin[r, :k]), _tol_t(rtout[r, :k], cout[r, :k])
        assert np.all(np.abs(tin[r, :k] - rtin[r, :k]) <= ti), (r, tin[r, :k] - rtin[r, :k], cin[r, :k])
        assert np.all(np.abs(tout[r, :k] - rtout[r, :k]) <= to), (r, tout[r, :k] - rtout[r, :k], cout[r, :k])
        ref0 = orc.deform_inv(kind, s64, o64[r] + rtin[r, :k, None] * d64[r])
        ref1 = orc.deform_inv(kind, s64, o64[r] + rtout[r, :k, None] * d64[r])
        e0 = np.abs(x0[:, r, :k].T - ref0).max(1)
        e1 = np.abs(x1[:, r, :k].T - ref1).max(1)
        assert np.all(e0 <= 2 * (ti + 2 * _ulp(1.0)) + 3e-7), (r, e0, cin[r, :k])
        assert np.all(e1 <= 2 * (to + 2 * _ulp(1.0)) + 3e-7), (r, e1, cout[r, :k])
        worst = max(worst, e0.max(), e1.max())
        n_seg += k
    say(f"  segments {n_seg}  max rest-point error {worst:.2e}")
    return n_seg


@pytest.mark.parametrize("name,N", [("torus16", 16), ("spheres64", 64), ("blobs128", 40), ("blobs128", 128)])
def test_voxelization_matches_oracle(orc, P, name, N):
    import torch
    w = S.workload(name)
    sp = S.scene_params(w.scene_kind, w.seed)
    say(f"voxelize {name} N={N}")
    ref = orc.voxelize(w.scene_kind, sp, N)
    occ = torch.zeros(N ** 3, dtype=torch.uint8, device="cuda")
    P.nif_voxelize(w.scene_kind, sp, N, occ)
    got = occ.cpu().numpy()
    diff = np.nonzero(got != ref)[0]
    # a mismatch is only allowed where the sign test is decided by a value within FP32
    # rounding of zero on the 5^3 sub-lattice of the cell
    g = np.stack(np.meshgrid(*[np.arange(5) / 4.0] * 3, indexing="ij"), -1).reshape(-1, 3)
    for c in diff:
        ijk = np.array([c % N, (c // N) % N, c // (N * N)])
        f = orc.scene_f(w.scene_kind, sp, (ijk + g) / N)
        assert min(abs(f.min()), abs(f.max())) < 1e-5, (name, c, f.min(), f.max())
    assert ref.sum() > 0 and len(diff) <= max(2, 1e-4 * ref.sum())


@pytest.mark.parametrize("kind,s", [(S.TWIST, 1.0), (S.BEND, 1.0), (S.TAPER, 1.0), (S.IDENTITY, 0.0),
                                    (S.BEND, 0.05), (S.TWIST, 0.37), (S.TWIST_BEND, 1.0), (S.TWIST_BEND, 0.4)])
def test_hit_lists_torus16(orc, P, kind, s):
    w = S.workload("torus16")
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N)
    o, d = S.rays_random(4096, w.seed)
    oi, di = S.rays_inside(1024, w.seed + 1)
    o = np.concatenate([o, oi], axis=1)
    d = np.concatenate([d, di], axis=1)
    say(f"trace torus16 kind={kind} s={s}")
    n_seg = _compare_trace(orc, P, w.N, occ, kind, s, o, d, brute=True)
    assert n_seg > 2000


@pytest.mark.parametrize("kind,s", [(S.TWIST, 1.0), (S.BEND, 0.625), (S.TAPER, 1.0), (S.TWIST_BEND, 0.8)])
def test_hit_lists_spheres64_sampled(orc, P, kind, s):
    w = S.workload("spheres64")
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N)
    o, d = S.rays_camera(1024, 45.0, sub=509)
    oi, di = S.rays_inside(500, 77, lo=0.2, hi=0.8)
    o = np.concatenate([o, oi], axis=1)
    d = np.concatenate([d, di], axis=1)
    say(f"trace spheres64 kind={kind} s={s} rays={o.shape[1]}")
    n_seg = _compare_trace(orc, P, w.N, occ, kind, s, o, d, brute=False)
    assert n_seg > 1000


def test_hit_lists_blobs128_multi_pose_sampled(orc, P):
    """The training and batched-query scene (32 blobs at 128^3) under four poses of different
    kinds in one multi-pose launch: camera and secondary rays of every pose, bit-exact hit
    lists on non-grazing rays and the FP32 bounds on entry/exit and rest points."""
    import torch
    w = S.workload("blobs128")
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N)
    kinds, strengths = [S.TWIST, S.BEND, S.TAPER, S.TWIST_BEND], [1.0, 0.8, 0.6, 0.5]
    os_, ds_ = [], []
    for p in range(4):
        o, d = S.rays_camera(64, 40.0 + 90.0 * p, sub=7)
        oi, di = S.rays_inside(200, 80 + p, lo=0.25, hi=0.75)
        os_.append(np.concatenate([o, oi], axis=1))
        ds_.append(np.concatenate([d, di], axis=1))
    counts = [x.shape[1] for x in os_]
    o_all, d_all = np.concatenate(os_, axis=1), np.concatenate(ds_, axis=1)
    max_seg = 256
    say(f"trace blobs128 N=128, 4 poses in one launch, rays {counts}")
    grid = P.Grid(torch.as_tensor(occ).cuda(), w.N, kinds, strengths)
    out = grid.trace(dev_f32(o_all), dev_f32(d_all), offsets(counts), max_seg=max_seg)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in out.items()}
    start, n_seg = 0, 0
    for p in range(4):
        c = counts[p]
        part = {k: (v[:, start:start + c] if k in ("x0", "x1") else v[start:start + c]) for k, v in out.items()}
        say(f"  pose {p}: kind {kinds[p]} s {strengths[p]}")
        n_seg += _check_segments(orc, w.N, occ, kinds[p], strengths[p], os_[p], ds_[p], part, max_seg, brute=False)
        start += c
    assert n_seg > 5000


def test_multi_pose_grid_and_empty_and_degenerate_inputs(orc, P):
    import torch
    w = S.workload("torus16")
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N)
    kinds, strengths = [S.TWIST, S.BEND, S.TAPER], [1.0, 0.5, 0.75]
    o, d = S.rays_random(999, 5)          # ragged split over three poses
    counts = [400, 0, 599]
    say("trace multi-pose torus16 with an empty pose range")
    grid = P.Grid(torch.as_tensor(occ).cuda(), w.N, kinds, strengths)
    out = grid.trace(dev_f32(o), dev_f32(d), offsets(counts), max_seg=96)
    cnt = out["count"].cpu().numpy()
    cell = out["cell"].cpu().numpy()
    start = 0
    for p, c in enumerate(counts):
        if c == 0:
            continue
        V = orc.lattice_vertices(kinds[p], float(np.float32(strengths[p])), w.N)
        rc, _, _, rcnt, fl = orc.trace(w.N, occ, V, o[:, start:start + c], d[:, start:start + c])
        ok = fl == 0
        assert np.array_equal(cnt[start:start + c][ok], rcnt[ok])
        for r in np.nonzero(ok)[0]:
            assert np.array_equal(cell[start + r, :rcnt[r]], rc[r, :rcnt[r]])
        start += c
    # zero rays: a no-op
    grid.trace(dev_f32(o[:, :0]), dev_f32(d[:, :0]), offsets([0, 0, 0]))
    # an empty scene: every ray misses
    empty = torch.zeros(w.N ** 3, dtype=torch.uint8, device="cuda")
    g2 = P.Grid(empty, w.N, [S.TWIST], [1.0])
    out = g2.trace(dev_f32(o), dev_f32(d), offsets([o.shape[1]]))
    assert int(out["count"].sum()) == 0
    # max_seg smaller than the list: counts are still complete
    out = grid.trace(dev_f32(o), dev_f32(d), offsets(counts), max_seg=1)
    assert np.array_equal(out["count"].cpu().numpy(), cnt)


def test_grid_update_equals_a_fresh_build(orc, P):
    """Re-posing a grid on the device gives the same hit lists as building it for the new poses."""
    import torch
    w = S.workload("spheres64")
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = torch.as_tensor(orc.voxelize(w.scene_kind, sp, w.N)).cuda()
    o, d = S.rays_camera(256, 30.0)
    k0, s0 = [S.TWIST, S.BEND], [0.25, 0.5]
    k1, s1 = [S.TAPER, S.TWIST], [1.0, 0.9]
    say("grid update vs fresh build, spheres64")
    g = P.Grid(occ, w.N, k0, s0)
    g.update(k1, s1)
    fresh = P.Grid(occ, w.N, k1, s1)
    off = offsets([o.shape[1] // 2, o.shape[1] - o.shape[1] // 2])
    a = g.trace(dev_f32(o), dev_f32(d), off, max_seg=64, with_points=False)
    b = fresh.trace(dev_f32(o), dev_f32(d), off, max_seg=64, with_points=False)
    assert np.array_equal(a["count"].cpu().numpy(), b["count"].cpu().numpy())
    assert np.array_equal(a["cell"].cpu().numpy(), b["cell"].cpu().numpy())
    assert np.array_equal(a["t_in"].cpu().numpy(), b["t_in"].cpu().numpy())
    assert g.info(0)[2] == 0 and int(a["count"].sum()) > 1000
