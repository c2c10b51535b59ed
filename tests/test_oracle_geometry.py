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


@pytest.mark.parametrize("workload", ["torus16", "spheres64", "blobs128"])
def test_scene_gradient_is_the_central_difference_of_f_and_points_outward(orc, workload):
    """grad f (which every label normal comes from) against FP64 central differences of f, and
    the label normals point outward: f grows along them across the surface."""
    w = S.workload(workload)
    sp = S.scene_params(w.scene_kind, w.seed)
    rng = np.random.default_rng(21)
    p = rng.uniform(0.15, 0.85, (3000, 3))
    f0 = orc.scene_f(w.scene_kind, sp, p)
    if w.scene_kind == S.SCENE_SPHERES:          # away from the switch between nearest spheres
        c = np.stack([sp[1 + 8 * i:4 + 8 * i] for i in range(int(sp[0]))])
        dist = np.linalg.norm(p[:, None, :] - c[None], axis=2) - sp[1 + 8 * np.arange(int(sp[0])) + 3][None]
        two = np.sort(dist, axis=1)[:, :2]
        p = p[two[:, 1] - two[:, 0] > 1e-3]
    g = orc.scene_grad(w.scene_kind, sp, p)
    h = 1e-6
    fd = np.stack([(orc.scene_f(w.scene_kind, sp, p + h * e) - orc.scene_f(w.scene_kind, sp, p - h * e)) / (2 * h)
                   for e in np.eye(3)], axis=1)
    scale = np.maximum(np.linalg.norm(g, axis=1), 1e-3)
    assert np.abs(g - fd).max(axis=1).max() / 1.0 <= 1e-6 * max(1.0, np.abs(fd).max())
    assert np.all(np.abs(g - fd).max(axis=1) <= 1e-6 * scale + 1e-9)
    x0, x1 = _segments(4000, 22, lo=0.1, hi=0.9)
    hit, t, nrm, _, _ = orc.label(w.scene_kind, sp, x0, x1)
    u = (x1 - x0) / np.linalg.norm(x1 - x0, axis=1, keepdims=True)
    sel = (hit == 1) & (t > 0)
    assert sel.sum() > 50
    q = x0[sel] + t[sel, None] * u[sel]
    n = nrm[sel]
    np.testing.assert_allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-12)
    gq = orc.scene_grad(w.scene_kind, sp, q)
    np.testing.assert_allclose(n, gq / np.linalg.norm(gq, axis=1, keepdims=True), atol=1e-12)
    assert np.all(orc.scene_f(w.scene_kind, sp, q + 1e-6 * n) > 0)
    assert np.all(orc.scene_f(w.scene_kind, sp, q - 1e-6 * n) < 0)


def test_torus_attributes_closed_form_spot_values(orc):
    """Torus albedo: channel c peaks at 0.9 where 2 p_c + c/3 = 1/4 (mod 1) and has period 1/2 in
    p_c; material flips at x = 1/2."""
    w = S.workload("torus16")
    sp = S.scene_params(w.scene_kind, w.seed)
    # channel 0 at p_x = 1/8, channel 1 at p_y = 11/24, channel 2 at p_z = 7/24: sine = 1
    p = np.array([[1 / 8, 11 / 24, 7 / 24], [1 / 8 + 0.5, 11 / 24 - 0.25, 7 / 24 + 0.5]])
    al, _ = orc.scene_attr(w.scene_kind, sp, p)
    np.testing.assert_allclose(al[0], [0.9, 0.9, 0.9], atol=1e-12)
    np.testing.assert_allclose(al[1], [0.9, 0.1, 0.9], atol=1e-12)       # p_y shifted a quarter: trough
    p = np.array([[3 / 8, 0.2, 0.3], [0.25, 0.2, 0.3]])                  # channel 0: 2 p = 3/4 -> -1; 1/2 -> 0
    al, _ = orc.scene_attr(w.scene_kind, sp, p)
    np.testing.assert_allclose(al[:, 0], [0.1, 0.5], atol=1e-12)
    _, mt = orc.scene_attr(w.scene_kind, sp, np.array([[0.5, 0.3, 0.3], [0.5 - 1e-12, 0.3, 0.3], [0.9, 0.1, 0.1]]))
    assert list(mt) == [1, 0, 1]


def test_sphere_attributes_are_those_of_the_nearest_sphere(orc):
    w = S.workload("spheres64")
    sp = S.scene_params(w.scene_kind, w.seed)
    n = int(sp[0])
    rec = sp[1:1 + 8 * n].reshape(n, 8)
    p = np.random.default_rng(23).uniform(0.0, 1.0, (2000, 3))
    al, mt = orc.scene_attr(w.scene_kind, sp, p)
    near = np.argmin(np.linalg.norm(p[:, None, :] - rec[None, :, :3], axis=2) - rec[None, :, 3], axis=1)
    np.testing.assert_array_equal(al, rec[near, 4:7])
    np.testing.assert_array_equal(mt, rec[near, 7].astype(np.int32))


def test_blob_attributes_single_blob_and_symmetric_pair(orc):
    """One blob: its own colour and material everywhere.  Two equal blobs: at the midpoint the
    colour is the mean of both (equal contributions, dyadic positions) and the material the
    first's (ties go to the lower index); next to one
    blob and far from the other, that blob's colour."""
    one = np.array([1, 0.5, 0.5, 0.5, 0.05, 0.2, 0.4, 0.6, 3.0])
    p = np.random.default_rng(24).uniform(0.3, 0.7, (50, 3))
    al, mt = orc.scene_attr(S.SCENE_BLOBS, one, p)
    np.testing.assert_allclose(al, np.tile([0.2, 0.4, 0.6], (50, 1)), atol=1e-15)
    assert np.all(mt == 3)
    two = np.array([2, 0.25, 0.5, 0.5, 0.05, 0.1, 0.2, 0.3, 1.0, 0.75, 0.5, 0.5, 0.05, 0.5, 0.6, 0.9, 2.0])
    al, mt = orc.scene_attr(S.SCENE_BLOBS, two, np.array([[0.5, 0.5, 0.5], [0.27, 0.5, 0.5], [0.73, 0.51, 0.5]]))
    np.testing.assert_allclose(al[0], [0.3, 0.4, 0.6], atol=1e-12)
    assert mt[0] == 1
    np.testing.assert_allclose(al[1], [0.1, 0.2, 0.3], atol=1e-12)
    np.testing.assert_allclose(al[2], [0.5, 0.6, 0.9], atol=1e-12)
    assert list(mt[1:]) == [1, 2]


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


def _line_segment_distance(o, d, a, e):
    """Distance from each line o + t d (rows, d unit; t over all reals) to each segment
    a + s e, s in [0, 1]: [rays][segments]."""
    w0 = o[:, None, :] - a[None, :, :]
    b = d @ e.T
    c = np.sum(e * e, axis=1)[None, :]
    dd = np.einsum("ri,rsi->rs", d, w0)
    ee = np.einsum("si,rsi->rs", e, w0)
    den = c - b * b
    s = np.clip(np.where(den > 1e-300, (ee - b * dd) / np.where(den > 1e-300, den, 1.0), 0.0), 0.0, 1.0)
    t = s * b - dd
    diff = w0 + t[..., None] * d[:, None, :] - s[..., None] * e[None, :, :]
    return np.linalg.norm(diff, axis=2)


def test_grazing_flags_equal_an_independent_identity_check(orc):
    """At the identity pose the lattice is the regular grid, so the grazing criteria have plain
    forms: the line within 1e-6 of an edge of an occupied voxel (which also covers crossings
    near an outer edge of a face of one), or an origin within 1e-6 of a face of the voxel the ray
    starts in (no ray here is near-parallel to a face).  Random rays, rays through
    edges and vertices of occupied voxels, origins on faces, and offsets of 3e-7 (grazing) and 3e-6
    (not); rays within a factor 2 of the threshold are left out."""
    N = 6
    rng = np.random.default_rng(31)
    occ = (rng.uniform(size=N ** 3) < 0.5).astype(np.uint8)
    V = orc.lattice_vertices(S.IDENTITY, 0.0, N)
    occ_ids = np.flatnonzero(occ)
    ijk = np.stack([occ_ids % N, (occ_ids // N) % N, occ_ids // (N * N)], axis=1)

    def unit(v):
        return v / np.linalg.norm(v, axis=1, keepdims=True)

    o_r, d_r = S.rays_random(300, 32)
    o_r, d_r = o_r.T.astype(np.float64), d_r.T.astype(np.float64)
    # lines through points of occupied voxels' edges, and offset from them by 3e-7 / 3e-6
    k = rng.integers(0, len(ijk), 300)
    ax = rng.integers(0, 3, 300)
    pe = (ijk[k] + (np.eye(3)[ax] * rng.uniform(0.1, 0.9, 300)[:, None])) / N
    de = unit(rng.normal(size=(300, 3)))
    off = unit(np.cross(de, rng.normal(size=(300, 3)))) * np.repeat([0.0, 3e-7, 3e-6], 100)[:, None]
    o_e = pe + off - 2.0 * de
    # origins on faces inside the lattice (a random axis coordinate snapped to the grid)
    o_f = rng.uniform(0.05, 0.95, (100, 3))
    a_f = rng.integers(0, 3, 100)
    o_f[np.arange(100), a_f] = np.round(o_f[np.arange(100), a_f] * N) / N
    d_f = unit(rng.normal(size=(100, 3)))
    o = np.concatenate([o_r, o_e, o_f])
    d = np.concatenate([d_r, de, d_f])
    flags = orc.trace(N, occ, V, o, d, brute=True)[4]
    # independent: edges of occupied voxels (12 per voxel, shared ones repeated)
    starts, dirs = [], []
    for m in range(8):
        for a in range(3):
            if m & (1 << a):
                continue
            corner = np.array([m & 1, (m >> 1) & 1, (m >> 2) & 1])
            starts.append((ijk + corner) / N)
            dirs.append(np.tile(np.eye(3)[a] / N, (len(ijk), 1)))
    dist_edge = _line_segment_distance(o, d, np.concatenate(starts), np.concatenate(dirs)).min(axis=1)
    # no ray here is within 1e-6 of parallel to a face, so the n . d criterion cannot fire
    assert np.abs(d).min() >= 1e-6
    # origin near a face of the voxel the ray is in just after t = 0 (if it starts in the lattice)
    ahead = o + 1e-9 * d
    inside = np.all((ahead > 0) & (ahead < 1), axis=1)
    cell = np.floor(ahead * N)
    frac = o * N - cell
    dist_face = np.where(inside, np.minimum(frac, 1 - frac).min(axis=1) / N, np.inf)
    crit = np.minimum(dist_edge, dist_face)
    clear = (crit < 0.5e-6) | (crit > 2e-6)
    want = crit < 1e-6
    got = flags != 0
    assert want[clear].sum() > 100 and (~want[clear]).sum() > 300
    bad = np.flatnonzero(clear & (want != got))
    assert len(bad) == 0, [(int(i), float(dist_edge[i]), float(dist_face[i]), int(flags[i])) for i in bad[:5]]


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
