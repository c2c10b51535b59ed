"""Pins of the oracle's deformations, voxelization, labels and hit lists against facts the
mathematics fixes (closed forms, invariants, textbook algorithms, brute force)."""
import math

import numpy as np
import pytest

import nif_synth as S

KINDS = [S.TWIST, S.BEND, S.TAPER, S.TWIST_BEND]


def _cube_points(n=4000, seed=0):
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(n, 3))


# ------------------------------------------------------------------ deformations

@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("s", [0.05, 0.5, 1.0])
def test_round_trip(orc, kind, s):
    p = _cube_points()
    q = orc.deform(kind, s, p)
    assert np.abs(orc.deform(kind, s, orc.deform_inv(kind, s, q)) - q).max() <= 1e-9
    assert np.abs(orc.deform_inv(kind, s, q) - p).max() <= 1e-9


@pytest.mark.parametrize("kind", KINDS)
def test_zero_strength_is_identity(orc, kind):
    p = _cube_points()
    assert np.array_equal(orc.deform(kind, 0.0, p), p)
    assert np.array_equal(orc.deform_inv(kind, 0.0, p), p)


def test_twist_bend_is_the_bend_on_the_twist_axis_and_keeps_the_twist_radius_at_zero_bend(orc):
    """Points on the twist axis are fixed by the twist, so the composed pose moves them as the
    bend alone; the composed pose also preserves every rest point's distance to the axis
    through the image of the vertical axis (twist: rotation, bend: isometric per fibre)."""
    z = np.linspace(0.0, 1.0, 41)
    p = np.stack([np.full_like(z, 0.5), np.full_like(z, 0.5), z], 1)
    for s in (0.3, 1.0):
        assert np.abs(orc.deform(S.TWIST_BEND, s, p) - orc.deform(S.BEND, s, p)).max() < 1e-15
    q = _cube_points(300, 5)
    tb = orc.deform(S.TWIST_BEND, 1.0, q)
    # undoing the bend leaves the twisted point: same height and radius about the axis
    t = orc.deform_inv(S.BEND, 1.0, tb)
    assert np.abs(t[:, 2] - q[:, 2]).max() < 1e-12
    r0 = np.hypot(q[:, 0] - 0.5, q[:, 1] - 0.5)
    assert np.abs(np.hypot(t[:, 0] - 0.5, t[:, 1] - 0.5) - r0).max() < 1e-12


def test_twist_preserves_height_and_radius_and_turns_by_0p6z(orc):
    p = _cube_points()
    q = orc.deform(S.TWIST, 1.0, p)
    assert np.array_equal(q[:, 2], p[:, 2])
    r0 = np.hypot(p[:, 0] - 0.5, p[:, 1] - 0.5)
    r1 = np.hypot(q[:, 0] - 0.5, q[:, 1] - 0.5)
    assert np.abs(r0 - r1).max() < 1e-12
    a0 = np.arctan2(p[:, 1] - 0.5, p[:, 0] - 0.5)
    a1 = np.arctan2(q[:, 1] - 0.5, q[:, 0] - 0.5)
    turn = np.angle(np.exp(1j * (a1 - a0)))
    assert np.abs(turn - 0.6 * p[:, 2]).max() < 1e-9


def test_taper_preserves_height_and_angle_and_halves_at_top(orc):
    p = _cube_points()
    q = orc.deform(S.TAPER, 1.0, p)
    assert np.array_equal(q[:, 2], p[:, 2])
    a0 = np.arctan2(p[:, 1] - 0.5, p[:, 0] - 0.5)
    a1 = np.arctan2(q[:, 1] - 0.5, q[:, 0] - 0.5)
    assert np.abs(np.angle(np.exp(1j * (a1 - a0)))).max() < 1e-12
    top = np.array([[1.0, 0.8, 1.0]])
    qt = orc.deform(S.TAPER, 1.0, top)[0]
    assert abs((qt[0] - 0.5) / (top[0, 0] - 0.5) - 0.5) < 1e-15


def test_bend_preserves_y_and_maps_centre_line_to_radius_1p5_arc(orc):
    p = _cube_points()
    q = orc.deform(S.BEND, 1.0, p)
    assert np.array_equal(q[:, 1], p[:, 1])
    z = np.linspace(0, 1, 101)
    line = np.stack([np.full_like(z, 0.5), np.full_like(z, 0.3), z], axis=1)
    arc = orc.deform(S.BEND, 1.0, line)
    dist = np.hypot(arc[:, 0] - (0.5 + 1.5), arc[:, 2] - 0.5)
    assert np.abs(dist - 1.5).max() < 1e-12
    # the centre line keeps its length (arc length = rest length)
    seg = np.linalg.norm(np.diff(arc, axis=0), axis=1).sum()
    assert abs(seg - 1.0) < 1e-4


@pytest.mark.parametrize("kind", KINDS)
def test_jacobian_determinant_matches_finite_differences(orc, kind):
    p = _cube_points(200, 3)
    h = 1e-5
    J = np.zeros((len(p), 3, 3))
    for a in range(3):
        e = np.zeros(3); e[a] = h
        J[:, :, a] = (orc.deform(kind, 1.0, p + e) - orc.deform(kind, 1.0, p - e)) / (2 * h)
    det = np.linalg.det(J)
    assert np.abs(det - orc.jacdet(kind, 1.0, p)).max() < 1e-8
    assert det.min() > 0.0                                  # orientation preserving on the cube


@pytest.mark.parametrize("kind", KINDS)
def test_deformed_normals_are_orthogonal_to_deformed_tangent_planes(orc, kind):
    """The deformed normal is unit, orthogonal to the images of two rest tangents (taken by
    deforming points of the rest tangent plane, not through the Jacobian) and on the side
    that the image of the rest normal direction points to."""
    rng = np.random.default_rng(11)
    p = _cube_points(100, 4)
    n = rng.normal(size=(100, 3)); n /= np.linalg.norm(n, axis=1, keepdims=True)
    t1 = np.cross(n, rng.normal(size=(100, 3))); t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(n, t1)
    nd = orc.deform_normal(kind, 1.0, p, n)
    assert np.abs(np.linalg.norm(nd, axis=1) - 1).max() < 1e-12
    e = 1e-4
    for t in (t1, t2):
        img = orc.deform(kind, 1.0, p + e * t) - orc.deform(kind, 1.0, p - e * t)
        cos = np.abs((img * nd).sum(1)) / np.linalg.norm(img, axis=1)
        assert cos.max() < 1e-7
    out = orc.deform(kind, 1.0, p + e * n) - orc.deform(kind, 1.0, p)
    assert ((out * nd).sum(1) > 0).all()


def test_deformed_normals_on_the_twist_axis_are_rotated(orc):
    """On the twist axis the Jacobian is the rotation by 0.6 z: normals turn by that angle."""
    rng = np.random.default_rng(12)
    z = rng.uniform(0, 1, 50)
    p = np.stack([np.full(50, 0.5), np.full(50, 0.5), z], 1)
    n = rng.normal(size=(50, 3)); n /= np.linalg.norm(n, axis=1, keepdims=True)
    th = 0.6 * z
    ref = np.stack([np.cos(th) * n[:, 0] - np.sin(th) * n[:, 1], np.sin(th) * n[:, 0] + np.cos(th) * n[:, 1],
                    n[:, 2]], 1)
    assert np.abs(orc.deform_normal(S.TWIST, 1.0, p, n) - ref).max() < 1e-9
    assert np.abs(orc.deform_normal(S.IDENTITY, 0.0, p, n) - n).max() < 1e-9


# ------------------------------------------------------------------ scenes, voxelization, labels

def test_sphere_voxelization_is_subset_of_exact_interval_test(orc):
    sp = np.array([1, 0.47, 0.52, 0.55, 0.31, 0.5, 0.5, 0.5, 0], dtype=np.float64)
    N = 24
    occ = orc.voxelize(S.SCENE_SPHERES, sp, N).reshape(N, N, N)   # [k][j][i]
    c, r = sp[1:4], sp[4]
    idx = np.arange(N)
    lo = idx / N; hi = (idx + 1) / N
    # exact: the distance from the centre ranges over [dmin, dmax] on the closed cell
    def axis_range(ci):
        near = np.clip(ci, lo, hi) - ci
        far = np.maximum(np.abs(lo - ci), np.abs(hi - ci))
        return near ** 2, far ** 2
    nx, fx = axis_range(c[0]); ny, fy = axis_range(c[1]); nz, fz = axis_range(c[2])
    dmin = np.sqrt(nz[:, None, None] + ny[None, :, None] + nx[None, None, :])
    dmax = np.sqrt(fz[:, None, None] + fy[None, :, None] + fx[None, None, :])
    exact = (dmin <= r) & (dmax >= r)
    assert np.all(exact[occ == 1])
    assert occ.sum() >= 0.9 * exact.sum()


def test_torus_voxelization_has_the_torus_symmetries(orc):
    w = S.workload("torus16")
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N).reshape(w.N, w.N, w.N)   # [k][j][i]
    assert occ.sum() > 0
    assert np.array_equal(occ, occ[:, :, ::-1])                 # x -> 1 - x
    assert np.array_equal(occ, occ[:, ::-1, :])                 # y -> 1 - y
    assert np.array_equal(occ, occ[::-1, :, :])                 # z -> 1 - z
    assert np.array_equal(occ, occ.transpose(0, 2, 1))           # x <-> y


def _segments(n, seed, lo=0.05, hi=0.95, scale=0.3):
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(lo, hi, size=(n, 3))
    x1 = x0 + rng.normal(scale=scale, size=(n, 3))
    return x0, x1


def test_sphere_labels_closed_form_equals_marching(orc):
    w = S.workload("spheres64")
    sp = S.scene_params(w.scene_kind, w.seed)
    x0, x1 = _segments(3000, 5)
    h1, t1, n1, a1, m1 = orc.label(w.scene_kind, sp, x0, x1)
    h2, t2, n2, a2, m2 = orc.label(w.scene_kind, sp, x0, x1, force_march=True)
    assert h1.sum() > 300
    # marching can only miss crossings thinner than one of its 256 steps
    both = (h1 == 1) & (h2 == 1)
    assert np.array_equal(h1[h2 == 1], h2[h2 == 1]) and both.sum() >= 0.99 * h1.sum()
    assert np.abs(t1[both] - t2[both]).max() < 1e-12
    assert np.abs(np.linalg.norm(n1[both], axis=1) - 1).max() < 1e-12
    assert np.array_equal(m1[both], m2[both])


def test_torus_labels_match_quartic_roots(orc):
    w = S.workload("torus16")
    sp = S.scene_params(w.scene_kind, w.seed)
    x0, x1 = _segments(400, 9, scale=0.4)
    hit, t, nrm, alb, mat = orc.label(w.scene_kind, sp, x0, x1)
    c, R, r = sp[:3], sp[3], sp[4]
    checked = 0
    for i in range(len(x0)):
        a = x0[i] - c
        e = x1[i] - x0[i]
        L = np.linalg.norm(e)
        u = e / L
        # (|p|^2 + R^2 - r^2)^2 = 4 R^2 (p_x^2 + p_y^2) along p = a + tau u
        A2 = np.polynomial.Polynomial([a @ a + R * R - r * r, 2 * (a @ u), 1.0])
        B2 = np.polynomial.Polynomial([a[0] ** 2 + a[1] ** 2, 2 * (a[0] * u[0] + a[1] * u[1]),
                                       u[0] ** 2 + u[1] ** 2]) * (4 * R * R)
        roots = (A2 * A2 - B2).roots()
        real = np.sort(roots[np.abs(roots.imag) < 1e-9].real)
        inside0 = (np.hypot(a[0], a[1]) - R) ** 2 + a[2] ** 2 - r * r <= 0
        cand = [0.0] if inside0 else [x for x in real if 0.0 <= x <= L]
        # marching cannot see a crossing pair closer than one step; skip those
        if len(real) >= 2 and np.min(np.diff(real)) < 2 * L / 256:
            continue
        if cand:
            assert hit[i] == 1
            assert abs(t[i] - cand[0]) < 1e-9
            checked += 1
        else:
            assert hit[i] == 0
    assert checked > 40


def test_blob_labels_lie_on_the_surface(orc):
    w = S.workload("blobs128")
    sp = S.scene_params(w.scene_kind, w.seed)
    x0, x1 = _segments(2000, 11, lo=0.2, hi=0.8)
    hit, t, nrm, alb, mat = orc.label(w.scene_kind, sp, x0, x1)
    sel = (hit == 1) & (t > 0)
    assert sel.sum() > 50
    u = (x1 - x0) / np.linalg.norm(x1 - x0, axis=1, keepdims=True)
    p = x0 + t[:, None] * u
    assert np.abs(orc.scene_f(w.scene_kind, sp, p[sel])).max() < 1e-9
    assert np.all(orc.scene_f(w.scene_kind, sp, (p - 1e-7 * u)[sel]) > 0)
    assert np.all((alb[sel] >= 0.1) & (alb[sel] <= 0.9))


# ------------------------------------------------------------------ lattice and hit lists

def _amanatides_woo(N, occ3, o, d):
    """Textbook 3D-DDA over the regular grid (Amanatides & Woo 1987) with slab entry/exit;
    returns [(cell, t_in, t_out)] of occupied cells, t clipped to >= 0."""
    t0, t1 = -np.inf, np.inf
    for a in range(3):
        if d[a] == 0:
            if not (0 <= o[a] <= 1):
                return []
            continue
        ta, tb = (0 - o[a]) / d[a], (1 - o[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    t0 = max(t0, 0.0)
    if t0 >= t1:
        return []
    p = o + t0 * d
    cell = [min(max(int(math.floor(p[a] * N)), 0), N - 1) for a in range(3)]
    step, tmax, tdel = [0] * 3, [np.inf] * 3, [np.inf] * 3
    for a in range(3):
        if d[a] > 0:
            step[a] = 1; tmax[a] = ((cell[a] + 1) / N - o[a]) / d[a]; tdel[a] = 1 / (N * d[a])
        elif d[a] < 0:
            step[a] = -1; tmax[a] = (cell[a] / N - o[a]) / d[a]; tdel[a] = -1 / (N * d[a])
    out, tc = [], t0
    while all(0 <= cell[a] < N for a in range(3)):
        a = int(np.argmin(tmax))
        te = min(tmax[a], t1)
        cid = cell[0] + N * (cell[1] + N * cell[2])
        if occ3[cid] and te > tc:
            out.append((cid, tc, te))
        tc = te
        cell[a] += step[a]
        tmax[a] += tdel[a]
    return out


def test_identity_pose_hit_lists_equal_textbook_dda(orc):
    w = S.workload("torus16")
    sp = S.scene_params(w.scene_kind, w.seed)
    N = w.N
    occ = orc.voxelize(w.scene_kind, sp, N)
    V = orc.lattice_vertices(S.IDENTITY, 0.0, N)
    o, d = S.rays_random(600, 21)
    oi, di = S.rays_inside(200, 22)
    o = np.concatenate([o, oi], axis=1); d = np.concatenate([d, di], axis=1)
    cells, tin, tout, cnt, fl = orc.trace(N, occ, V, o, d)
    compared = 0
    for r in range(o.shape[1]):
        if fl[r]:
            continue
        ref = _amanatides_woo(N, occ, o[:, r].astype(np.float64), d[:, r].astype(np.float64))
        assert cnt[r] == len(ref)
        for k, (c, a, b) in enumerate(ref):
            assert cells[r, k] == c
            assert abs(tin[r, k] - a) < 1e-12 and abs(tout[r, k] - b) < 1e-12
        compared += 1
    assert compared > 700


@pytest.mark.parametrize("kind,s", [(S.TWIST, 1.0), (S.BEND, 1.0), (S.TAPER, 1.0), (S.BEND, 0.3), (S.TWIST_BEND, 1.0)])
def test_walk_equals_brute_force_on_small_lattices(orc, kind, s):
    w = S.workload("torus16")
    sp = S.scene_params(w.scene_kind, w.seed)
    N = w.N
    occ = orc.voxelize(w.scene_kind, sp, N)
    V = orc.lattice_vertices(kind, s, N)
    o, d = S.rays_random(400, 31)
    oi, di = S.rays_inside(200, 32)
    o = np.concatenate([o, oi], axis=1); d = np.concatenate([d, di], axis=1)
    a = orc.trace(N, occ, V, o, d, brute=True)
    b = orc.trace(N, occ, V, o, d, brute=False)
    ok = (a[4] == 0) & (b[4] == 0)
    assert ok.sum() > 500
    assert np.array_equal(a[3][ok], b[3][ok])
    assert np.array_equal(a[0][ok], b[0][ok])
    assert np.abs(a[1][ok] - b[1][ok]).max() == 0.0
    assert np.abs(a[2][ok] - b[2][ok]).max() == 0.0
    assert (a[3][ok] > 0).sum() > 100


@pytest.mark.parametrize("kind", KINDS)
def test_hit_intervals_map_back_into_their_rest_voxel(orc, kind):
    """The midpoint of every kept interval, mapped through the analytic inverse, lies in the
    rest voxel the list names (up to the O(h^2) gap between the piecewise-linear lattice and
    the analytic deformation); consecutive voxels that share a face share the crossing."""
    w = S.workload("torus16")
    sp = S.scene_params(w.scene_kind, w.seed)
    N = w.N
    occ = orc.voxelize(w.scene_kind, sp, N)
    V = orc.lattice_vertices(kind, 1.0, N)
    o, d = S.rays_random(500, 41)
    cells, tin, tout, cnt, fl = orc.trace(N, occ, V, o, d)
    n_int = 0
    for r in range(o.shape[1]):
        for k in range(cnt[r]):
            mid = o[:, r] + 0.5 * (tin[r, k] + tout[r, k]) * d[:, r].astype(np.float64)
            x = orc.deform_inv(kind, 1.0, mid[None])[0]
            c = cells[r, k]
            ijk = np.array([c % N, (c // N) % N, c // (N * N)])
            assert np.all(x >= ijk / N - 2e-3) and np.all(x <= (ijk + 1) / N + 2e-3)
            n_int += 1
            if k > 0:
                assert tin[r, k] >= tout[r, k - 1]
    assert n_int > 500
