"""Pins of the oracle's encoding, MLP, first-hit query, loss, gradient and Adam against
closed forms, invariants, library routines (numpy, torch) and finite differences."""
import dataclasses
import math

import numpy as np
import pytest

import nif_synth as S


def _small_model(**kw):
    base = dataclasses.replace(S.workload("torus16").model, hidden_width=16)
    return dataclasses.replace(base, **kw)


def _dense_linear_tables(m, coef, const):
    """Tables whose dense-level entries are coef[l][f] . v + const[l][f] at vertex v."""
    T = m.table_size
    tab = np.zeros((m.levels, T, m.feat_dim))
    for l in range(m.levels):
        n1 = m.res[l] + 1
        if n1 ** 3 > T:
            continue
        idx = np.arange(n1 ** 3)
        v = np.stack([idx % n1, (idx // n1) % n1, idx // (n1 * n1)], axis=1).astype(np.float64)
        for f in range(m.feat_dim):
            tab[l, :n1 ** 3, f] = v @ coef[l, f] + const[l, f]
    return tab


def _pe(x, F):
    """gamma(x) of Eq. (1) mapped to [0,1]: [x, (sin 2^k x + 1)/2, (cos 2^k x + 1)/2]."""
    out = [x]
    for k in range(F):
        out += [(np.sin(2.0 ** k * x) + 1) / 2, (np.cos(2.0 ** k * x) + 1) / 2]
    return np.stack(out, axis=1)                       # [n][S][3]


@pytest.mark.parametrize("fd", [2, 3], ids=["8_levels_2_features", "2_levels_3_features"])
def test_dense_levels_reproduce_linear_fields_through_every_pe_sample(orc, fd):
    """Trilinear interpolation has linear precision: with table entries linear in the vertex
    coordinates the encoding equals that linear function at pos = sample * N_l, for every
    sample of gamma, every dense level and every feature (pins Eq. (1)'s samples, the
    [0,1] mapping, the level resolutions and the output order (point, sample, level, feature),
    with two features per entry and with the paper's comparison configuration's three)."""
    if fd == 2:
        m = _small_model(res=[3, 5, 7, 9, 11, 13, 15, 17], log2_table=14)
    else:
        m = _small_model(levels=2, feat_dim=3, res=[5, 9], log2_table=14, pe_freqs=3)
    rng = np.random.default_rng(0)
    coef = rng.normal(size=(m.levels, m.feat_dim, 3))
    const = rng.normal(size=(m.levels, m.feat_dim))
    tab = _dense_linear_tables(m, coef, const)
    x = rng.uniform(0.0, 1.0, size=(64, 3))
    enc = orc.encode(m, tab, x).reshape(64, m.n_samples, m.levels, m.feat_dim)
    smp = _pe(x, m.pe_freqs)
    for l in range(m.levels):
        assert (m.res[l] + 1) ** 3 <= m.table_size
        ref = np.einsum("nsa,fa->nsf", smp * m.res[l], coef[l]) + const[l]
        assert np.abs(enc[:, :, l, :] - ref).max() < 1e-11


def test_no_frequencies_is_plain_grid_encoding(orc):
    m = _small_model(pe_freqs=0)
    rng = np.random.default_rng(1)
    tab = rng.normal(size=(m.levels, m.table_size, m.feat_dim))
    x = rng.uniform(0, 1, size=(32, 3))
    assert orc.encode(m, tab, x).shape == (32, m.levels * m.feat_dim)


def test_per_sample_tables_reduce_to_the_shared_table_and_stay_local(orc):
    """Per-sample tables holding S copies of one table encode exactly like the shared table;
    the table gradient summed over the copies is the shared gradient; changing set s moves
    only the features of PE sample s."""
    m = _small_model()
    mp = dataclasses.replace(m, per_sample_tables=1)
    S_ = m.n_samples
    tab = S.init_tables(m, 5).astype(np.float64) * 1e3
    tabp = np.concatenate([tab] * S_, axis=0)
    x = np.random.default_rng(6).uniform(-0.05, 1.05, (50, 3))
    a = orc.encode(m, tab, x)
    b = orc.encode(mp, tabp, x)
    assert np.array_equal(a, b)
    tabq = tabp.copy()
    k = 3
    tabq[k * m.levels:(k + 1) * m.levels] *= -2.0
    c = orc.encode(mp, tabq, x).reshape(50, S_, m.levels, m.feat_dim)
    a4 = a.reshape(50, S_, m.levels, m.feat_dim)
    same = np.ones(S_, bool); same[k] = False
    assert np.array_equal(c[:, same], a4[:, same]) and np.allclose(c[:, k], -2.0 * a4[:, k])
    _, _, x0, x1, hit, t, nr, al, mt = _batch(m, 24, 64)
    prm = S.init_mlp(m, 7).astype(np.float64)
    g = orc.loss_grad(m, tab, prm, np.zeros(5), x0, x1, hit, t, nr, al, mt)[1]
    gp = orc.loss_grad(mp, tabp, prm, np.zeros(5), x0, x1, hit, t, nr, al, mt)[1]
    gsum = gp.reshape(S_, m.levels, m.table_size, m.feat_dim).sum(0)
    assert np.abs(gsum - g).max() <= 1e-12 * np.abs(g).max()


def test_concatenated_encoding_is_the_plain_grid_and_the_raw_pe(orc):
    """[phi(x0), phi(x1), gamma(x0), gamma(x1)]: the grid parts equal the F = 0 encoding of the
    points themselves; the gamma parts are x, sin 2^k x, cos 2^k x of the clamped coordinates
    in (sample, axis) order; the heads see exactly that vector."""
    m = _small_model(concat_encoding=1, pe_freqs=3)
    m0 = _small_model(pe_freqs=0)
    tab = S.init_tables(m, 8).astype(np.float64) * 1e3
    rng = np.random.default_rng(9)
    x0 = rng.uniform(-0.05, 1.05, (40, 3)); x1 = rng.uniform(-0.05, 1.05, (40, 3))
    assert m.enc_width == 2 * (m.levels * m.feat_dim + 3 * 7)
    g0 = orc.encode(m0, tab, x0)
    assert np.array_equal(orc.encode(m, tab, x0), g0)
    # a one-layer probe: identity rows read the encoding back through forward()
    E = m.enc_width
    probe = dataclasses.replace(m, hidden_layers=1, hidden_width=16)
    prm = np.zeros(probe.n_mlp_params)
    W = prm[:16 * E].reshape(16, E)
    pw = m.levels * m.feat_dim
    cols = [2 * pw + 3 * s + a for s in (0, 1, 2, 6) for a in range(3)] + [2 * pw + 21 + 3 * 5 + 1]
    for r, c in enumerate(cols[:16]):
        W[r, c] = 1.0
    # output layer passes hidden unit r to head r (ReLU keeps the non-negative ones only)
    Wo = prm[16 * E + 16:16 * E + 16 + probe.n_heads * 16].reshape(probe.n_heads, 16)
    for r in range(probe.n_heads):
        Wo[r, r] = 1.0
    z = orc.forward(probe, tab, prm, x0, x1)
    xc0 = np.clip(x0, 0, 1); xc1 = np.clip(x1, 0, 1)
    ref = [xc0[:, 0], xc0[:, 1], xc0[:, 2], np.sin(xc0[:, 0]), np.sin(xc0[:, 1]), np.sin(xc0[:, 2]),
           np.cos(xc0[:, 0]), np.cos(xc0[:, 1]), np.cos(xc0[:, 2]), np.cos(4 * xc0[:, 0]), np.cos(4 * xc0[:, 1]),
           np.cos(4 * xc0[:, 2])]
    for r in range(min(probe.n_heads, len(ref))):
        assert np.abs(z[:, r] - np.maximum(ref[r], 0.0)).max() < 1e-14, r


def test_points_are_clamped_to_the_unit_cube(orc):
    m = _small_model()
    rng = np.random.default_rng(2)
    tab = rng.normal(size=(m.levels, m.table_size, m.feat_dim))
    x = rng.uniform(-0.5, 1.5, size=(64, 3))
    assert np.array_equal(orc.encode(m, tab, x), orc.encode(m, tab, np.clip(x, 0, 1)))


@pytest.mark.parametrize("name", ["spheres64", "spheres32_paper"])
def test_partition_of_unity_on_all_levels(orc, name):
    m = S.workload(name).model
    const = np.array([0.25, -3.0, 7.5])[:m.feat_dim]
    tab = np.empty((m.levels, m.table_size, m.feat_dim))
    tab[:, :, :] = const
    x = np.random.default_rng(3).uniform(0, 1, size=(16, 3))
    enc = orc.encode(m, tab, x).reshape(16, -1, m.feat_dim)
    assert np.abs(enc - const).max() < 1e-13


def test_hashed_level_reads_the_instant_ngp_hash_entry_at_a_vertex(orc):
    """At a sample that sits exactly on a vertex only that vertex's entry contributes; on a
    hashed level it is entry (x * 1 xor y * 2654435761 xor z * 805459861) mod T, the
    spatial hash of the grid encoding LSNIF uses."""
    m = S.workload("torus16").model                      # levels 2..7 are hashed
    T = m.table_size
    tab = np.zeros((m.levels, T, m.feat_dim))
    tab[:, :, 0] = np.arange(T)
    tab[:, :, 1] = -np.arange(T)
    rng = np.random.default_rng(4)
    for l in range(2, m.levels):
        N = m.res[l]
        assert (N + 1) ** 3 > T
        v = rng.integers(0, N, size=(20, 3))
        x = v / N                                        # exact in binary for N = 2^k only:
        enc = orc.encode(m, tab, x).reshape(20, m.n_samples, m.levels, 2)[:, 0, l, :]
        exact = np.all(np.abs(x * N - v) == 0, axis=1)
        for i in np.nonzero(exact)[0]:
            h = (int(v[i, 0]) ^ (int(v[i, 1]) * 2654435761) ^ (int(v[i, 2]) * 805459861)) & 0xFFFFFFFF
            assert enc[i, 0] == h % T and enc[i, 1] == -(h % T)
        assert exact.sum() >= 1


@pytest.mark.parametrize("per_sample,fd", [(0, 2), (1, 2), (0, 3), (1, 3)])
def test_encoding_adjoint_is_the_transpose_of_the_encoding(orc, per_sample, fd):
    """psi is linear in the tables, psi(x; t) = J(x) t, so <v, psi(x; t)> = <J^T v, t> for any
    tables t and any v: the adjoint scatter agrees with the encoding itself, on dense and
    hashed levels; and J^T |v| >= |J^T v| (trilinear weights are nonnegative)."""
    if fd == 2:
        m = _small_model(log2_table=12, per_sample_tables=per_sample)
    else:
        m = _small_model(levels=2, feat_dim=3, res=[12, 24], log2_table=12, pe_freqs=3, per_sample_tables=per_sample)
    rng = np.random.default_rng(3)
    x = rng.uniform(-0.05, 1.05, (200, 3))
    W = m.n_samples * m.levels * m.feat_dim
    v = rng.normal(size=(200, W))
    t = rng.normal(size=(m.table_levels, m.table_size, m.feat_dim))
    g = orc.encode_backward(m, t, x, v)
    assert g.shape == t.shape
    lhs = float(np.sum(v * orc.encode(m, t, x)))
    rhs = float(np.sum(g * t))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, np.abs(v).sum() * np.abs(t).max())
    ga = orc.encode_backward(m, t, x, np.abs(v))
    assert np.all(ga >= np.abs(g) - 1e-15) and np.count_nonzero(ga) > 0
    # the sparse Jacobian: scattering v with the listed corners and weights is the adjoint
    idx, w = orc.encode_corners(m, x)
    assert idx.shape == (200, m.n_samples, m.levels, 8)
    np.testing.assert_allclose(w.sum(axis=3), 1.0, rtol=0, atol=1e-12)          # partition of unity
    vv = v.reshape(200, m.n_samples, m.levels, m.feat_dim)
    gs = np.zeros(t.size)
    for f in range(m.feat_dim):
        np.add.at(gs, (idx * m.feat_dim + f).reshape(-1), (w * vv[:, :, :, None, f]).reshape(-1))
    np.testing.assert_allclose(gs, g.reshape(-1), rtol=0, atol=1e-12 * np.abs(g).max())


def test_mlp_matches_numpy_float64(orc):
    m = _small_model()
    tab = S.init_tables(m, 5).astype(np.float64) * 1e3
    prm = S.init_mlp(m, 5).astype(np.float64)
    prm += np.random.default_rng(6).normal(scale=0.01, size=prm.shape)   # non-zero biases
    x0, x1 = S.random_points(40, 7)
    z = orc.forward(m, tab, prm, x0, x1)
    h = np.concatenate([orc.encode(m, tab, x0.T.astype(np.float64)),
                        orc.encode(m, tab, x1.T.astype(np.float64))], axis=1)
    layers = S.mlp_layers(m, prm)
    for j, (W, b) in enumerate(layers):
        h = h @ W.T + b
        if j + 1 < len(layers):
            h = np.maximum(h, 0.0)
    assert np.abs(z - h).max() < 1e-13 * max(1.0, np.abs(h).max())


# ------------------------------------------------------------------ query

def _forced_params(m, hit_bias, dist_bias, nrm=(0.0, 0.0, 2.0), alb=(0.0, 1.0, -1.0), mat=0.5):
    """MLP whose output is a constant vector given by the last layer's bias."""
    prm = np.zeros(m.n_mlp_params)
    b = prm[-m.n_heads:]
    b[0] = hit_bias; b[1] = dist_bias; b[2:5] = nrm; b[5:8] = alb; b[8:] = mat
    return prm


@pytest.mark.parametrize("kind,dist_head", [(S.TWIST, S.DIST_LOG_RELU), (S.BEND, S.DIST_LOG_RELU),
                                             (S.TWIST, S.DIST_SIGMOID)])
def test_query_with_always_hit_network_returns_first_segment(orc, kind, dist_head):
    w = S.workload("torus16")
    m = dataclasses.replace(w.model, dist_head=dist_head)
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N)
    tab = np.zeros((m.levels, m.table_size, m.feat_dim))
    dist_bias = 0.01
    prm = _forced_params(m, 1.0, dist_bias)
    o, d = S.rays_random(300, 51)
    q = orc.query(m, tab, prm, w.N, occ, kind, 1.0, o, d)
    V = orc.lattice_vertices(kind, 1.0, w.N)
    cells, tin, tout, cnt, _ = orc.trace(w.N, occ, V, o, d, with_flags=False)
    hit = cnt > 0
    assert np.array_equal(q["hit"].astype(bool), hit) and hit.sum() > 50
    r = np.nonzero(hit)[0]
    assert np.array_equal(q["cell"][r], cells[r, 0])
    assert np.all(q["n_queried"][r] == 1)
    d64 = d.T.astype(np.float64); o64 = o.T.astype(np.float64)
    x0 = orc.deform_inv(kind, 1.0, o64[r] + tin[r, 0:1] * d64[r])
    x1 = orc.deform_inv(kind, 1.0, o64[r] + tout[r, 0:1] * d64[r])
    lr = np.linalg.norm(x1 - x0, axis=1)
    if dist_head == S.DIST_SIGMOID:        # the bounded head: the fraction is sigma(z1)
        f = np.full(len(r), 1 / (1 + math.exp(-dist_bias)))
    else:
        f = np.clip(dist_bias / lr, 0, 1)
    assert np.abs(q["t"][r] - (tin[r, 0] + f * (tout[r, 0] - tin[r, 0]))).max() < 1e-12
    assert np.abs(q["xrest"][r] - (x0 + f[:, None] * (x1 - x0))).max() < 1e-12
    assert np.allclose(q["normal"][r], [0, 0, 1]) and np.allclose(q["albedo"][r], [0.5, 1 / (1 + math.e ** -1), 1 / (1 + math.e)])
    assert np.all(q["material"][r] == 1)                 # one material logit: z8 > 0
    assert np.all(np.isinf(q["t"][~hit])) and np.all(q["cell"][~hit] == -1)


def test_query_tmax_is_the_occlusion_form_of_the_first_hit(orc):
    """Always-hit network: occluded iff the unbounded first hit lies before tmax; never-hit
    network: exactly the voxels entered before tmax are evaluated (brute-force hit lists)."""
    w = S.workload("torus16")
    m = w.model
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N)
    tab = np.zeros((m.levels, m.table_size, m.feat_dim))
    o, d = S.rays_random(300, 53)
    tmax = np.random.default_rng(54).uniform(1.0, 3.0, 300)
    always = _forced_params(m, 1.0, 0.01)
    full = orc.query(m, tab, always, w.N, occ, S.TWIST, 1.0, o, d)
    occl = orc.query(m, tab, always, w.N, occ, S.TWIST, 1.0, o, d, tmax=tmax)
    assert full["hit"].sum() > 50
    expect = (full["hit"] == 1) & (full["t"] < tmax)
    assert 0 < expect.sum() < full["hit"].sum()
    assert np.array_equal(occl["hit"].astype(bool), expect)
    assert np.array_equal(occl["t"][expect], full["t"][expect]) and np.all(np.isinf(occl["t"][~expect]))
    never = _forced_params(m, -1.0, 0.0)
    q = orc.query(m, tab, never, w.N, occ, S.TWIST, 1.0, o, d, tmax=tmax)
    V = orc.lattice_vertices(S.TWIST, 1.0, w.N)
    cells, tin, tout, cnt, _ = orc.trace(w.N, occ, V, o, d, brute=True, with_flags=False)
    before = np.array([(tin[i, :cnt[i]] < tmax[i]).sum() for i in range(300)])
    assert q["hit"].sum() == 0 and np.array_equal(q["n_queried"], before)
    assert np.any((before > 0) & (before < cnt))


def test_query_with_never_hit_network_visits_every_segment(orc):
    w = S.workload("torus16")
    m = w.model
    sp = S.scene_params(w.scene_kind, w.seed)
    occ = orc.voxelize(w.scene_kind, sp, w.N)
    tab = np.zeros((m.levels, m.table_size, m.feat_dim))
    prm = _forced_params(m, -1.0, 0.0)
    o, d = S.rays_random(300, 52)
    q = orc.query(m, tab, prm, w.N, occ, S.TWIST, 1.0, o, d)
    V = orc.lattice_vertices(S.TWIST, 1.0, w.N)
    cnt = orc.trace(w.N, occ, V, o, d, with_flags=False)[3]
    assert q["hit"].sum() == 0
    assert np.array_equal(q["n_queried"], cnt)


# ------------------------------------------------------------------ loss, gradient, Adam

def _batch(m, B, seed, scale_tables=100.0):
    rng = np.random.default_rng(seed)
    tab = S.init_tables(m, seed).astype(np.float64) * scale_tables
    prm = S.init_mlp(m, seed).astype(np.float64)
    x0 = rng.uniform(0.05, 0.95, (B, 3)); x1 = x0 + rng.normal(scale=0.05, size=(B, 3))
    hit = (rng.uniform(size=B) < 0.6).astype(np.uint8)
    t = rng.uniform(0.001, 0.05, B)
    nr = rng.normal(size=(B, 3)); nr /= np.linalg.norm(nr, axis=1, keepdims=True)
    al = rng.uniform(0.1, 0.9, (B, 3))
    mt = rng.integers(0, max(2, m.n_materials), B).astype(np.int32)
    if m.n_materials == 1:
        mt = np.minimum(mt, 1)
    return tab, prm, x0, x1, hit, t, nr, al, mt


def test_constant_network_losses_have_closed_forms(orc):
    m = _small_model(n_materials=4)
    B = 64
    _, _, x0, x1, hit, t, nr, al, mt = _batch(m, B, 60)
    tab = np.zeros((m.levels, m.table_size, m.feat_dim))
    prm = np.zeros(m.n_mlp_params)
    b = prm[-m.n_heads:]
    b[0] = 0.0                      # BCE(0, y) = log 2
    b[1] = 0.02                     # distance prediction 0.02
    b[2:5] = [0.0, 0.0, 3.0]        # normal (0,0,1)
    b[5:8] = 0.0                    # albedo 0.5
    b[8:] = 0.0                     # uniform material distribution: CE = log 4
    losses = orc.loss_grad(m, tab, prm, np.zeros(5), x0, x1, hit, t, nr, al, mt)[0]
    P = hit.astype(bool)
    assert abs(losses[0] - math.log(2)) < 1e-15
    assert abs(losses[1] - np.mean((math.log(0.02 + 1e-4) - np.log(t[P] + 1e-4)) ** 2)) < 1e-13
    assert abs(losses[2] - np.mean(1 - nr[P, 2])) < 1e-14
    assert abs(losses[3] - np.mean(np.abs(0.5 - al[P]))) < 1e-14
    assert abs(losses[4] - math.log(4)) < 1e-14
    # s = 0: regression terms weigh 1/2, classification terms 1
    ref = losses[0] + losses[4] + 0.5 * (losses[1] + losses[2] + losses[3])
    assert abs(losses[5] - ref) < 1e-13


def test_ablation_heads_and_fixed_weights_have_closed_forms(orc):
    """Sigmoid distance head: sigma(0) = 1/2 against t*/l clamped to [0,1]; fixed weights: the
    total is the plain sum of the five task losses and s gets no gradient."""
    m = _small_model(n_materials=4, dist_head=S.DIST_SIGMOID)
    B = 64
    _, _, x0, x1, hit, t, nr, al, mt = _batch(m, B, 63)
    t = t.copy(); t[:4] = 10.0                            # beyond the segment: target clamps to 1
    tab = np.zeros((m.levels, m.table_size, m.feat_dim))
    prm = np.zeros(m.n_mlp_params)
    b = prm[-m.n_heads:]
    b[2:5] = [0.0, 0.0, 3.0]
    s = np.array([0.3, -0.2, 0.1, 0.4, -0.5])
    L, _, _, gs, _, _ = orc.loss_grad(m, tab, prm, s, x0, x1, hit, t, nr, al, mt, fixed_weights=True)
    P = hit.astype(bool)
    tau = np.clip(t / np.linalg.norm(x1 - x0, axis=1), 0, 1)
    assert P[:4].any() and abs(L[1] - np.mean((0.5 - tau[P]) ** 2)) < 1e-14
    assert abs(L[0] - math.log(2)) < 1e-15 and abs(L[4] - math.log(4)) < 1e-14
    assert abs(L[5] - L[:5].sum()) < 1e-13
    assert np.all(gs == 0.0)
    # the log-distance head on the same batch is unchanged by the switch of weights only
    m0 = dataclasses.replace(m, dist_head=S.DIST_LOG_RELU)
    b[1] = 0.02
    L0 = orc.loss_grad(m0, tab, prm, np.zeros(5), x0, x1, hit, t, nr, al, mt, fixed_weights=True)[0]
    assert abs(L0[1] - np.mean((math.log(0.02 + 1e-4) - np.log(t[P] + 1e-4)) ** 2)) < 1e-13


def test_uncertainty_weights_are_stationary_at_log_loss(orc):
    """d/ds (0.5 e^-s L + 0.5 s) = 0 at s = log L; d/ds (e^-s L + 0.5 s) = 0 at s = log 2L."""
    m = _small_model()
    tab, prm, x0, x1, hit, t, nr, al, mt = _batch(m, 48, 61)
    L = orc.loss_grad(m, tab, prm, np.zeros(5), x0, x1, hit, t, nr, al, mt)[0]
    s_star = np.array([math.log(2 * L[0]), math.log(L[1]), math.log(L[2]), math.log(L[3]),
                       math.log(2 * L[4])])
    gs = orc.loss_grad(m, tab, prm, s_star, x0, x1, hit, t, nr, al, mt)[3]
    assert np.abs(gs).max() < 1e-12
    assert np.all(orc.loss_grad(m, tab, prm, s_star - 0.1, x0, x1, hit, t, nr, al, mt)[3] < 0)
    assert np.all(orc.loss_grad(m, tab, prm, s_star + 0.1, x0, x1, hit, t, nr, al, mt)[3] > 0)


@pytest.mark.parametrize("n_materials,dist_head,fixed,per_sample", [(1, S.DIST_LOG_RELU, False, 0),
                                                                   (4, S.DIST_LOG_RELU, False, 0),
                                                                   (4, S.DIST_SIGMOID, True, 0),
                                                                   (4, S.DIST_LOG_RELU, False, 1),
                                                                   (4, S.DIST_LOG_RELU, False, 2),
                                                                   (4, S.DIST_LOG_RELU, False, 3)])
def test_gradient_matches_central_finite_differences(orc, n_materials, dist_head, fixed, per_sample):
    """per_sample 2: the concatenated [gamma, phi] encoding (one table set); 3: two levels of
    three features with F = 3 (the paper's comparison configuration, small tables)."""
    m = _small_model(n_materials=n_materials, dist_head=dist_head, per_sample_tables=int(per_sample == 1),
                     concat_encoding=int(per_sample == 2))
    if per_sample == 3:
        m = dataclasses.replace(m, levels=2, feat_dim=3, res=[16, 40], pe_freqs=3)
    tab, prm, x0, x1, hit, t, nr, al, mt = _batch(m, 20, 62 + n_materials)
    s = np.array([0.1, -0.2, 0.3, 0.0, 0.5])
    L, gt, gp, gs, gx0, gx1 = orc.loss_grad(m, tab, prm, s, x0, x1, hit, t, nr, al, mt, want_x=True,
                                            fixed_weights=fixed)

    def total(tab_=tab, prm_=prm, s_=s, x0_=x0, x1_=x1):
        return orc.loss_grad(m, tab_, prm_, s_, x0_, x1_, hit, t, nr, al, mt, fixed_weights=fixed)[0][5]

    def check(fd, an, h=1e-6):
        # rounding floor of a central difference: a few ulps of the total over the step
        floor = 4 * np.finfo(float).eps * abs(L[5]) / h
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * scale) + 1e-10 + floor

    rng = np.random.default_rng(70)
    scale = np.abs(gp).max()
    for idx in rng.choice(prm.size, 12, replace=False):
        h = 1e-6 * max(1.0, abs(prm[idx]))
        p1 = prm.copy(); p1[idx] += h
        p2 = prm.copy(); p2[idx] -= h
        check((total(prm_=p1) - total(prm_=p2)) / (2 * h), gp[idx], h)
    flat = tab.reshape(-1)
    scale = np.abs(gt).max()
    for idx in rng.choice(np.nonzero(gt.reshape(-1))[0], 8, replace=False):
        h = 1e-6 * max(1.0, abs(flat[idx]))
        t1 = flat.copy(); t1[idx] += h
        t2 = flat.copy(); t2[idx] -= h
        check((total(tab_=t1.reshape(tab.shape)) - total(tab_=t2.reshape(tab.shape))) / (2 * h),
              gt.reshape(-1)[idx], h)
    scale = max(np.abs(gs).max(), 1.0)
    for k in range(5):
        s1 = s.copy(); s1[k] += 1e-6
        s2 = s.copy(); s2[k] -= 1e-6
        check((total(s_=s1) - total(s_=s2)) / 2e-6, gs[k])
    if dist_head == S.DIST_SIGMOID:
        return          # the target t*/l is a label computed from x: no gradient flows through it
    scale = max(np.abs(gx0).max(), np.abs(gx1).max())
    for i in range(4):
        for a in range(3):
            h = 1e-7
            a1 = x0.copy(); a1[i, a] += h
            a2 = x0.copy(); a2[i, a] -= h
            # a probe that moves a sample across a grid cell boundary is not differentiable
            if np.array_equal(np.floor(_pe(a1[i:i + 1], m.pe_freqs)[0][:, :, None] * np.array(m.res)[None, None, :]),
                              np.floor(_pe(a2[i:i + 1], m.pe_freqs)[0][:, :, None] * np.array(m.res)[None, None, :])):
                tol = 1e-5 * max(abs(gx0[i, a]), 1e-3 * scale)
                fd = (total(x0_=a1) - total(x0_=a2)) / (2 * h)
                assert abs(fd - gx0[i, a]) <= tol + 1e-8


def test_adam_first_step_closed_form_and_torch_agreement(orc):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(80)
    theta = rng.normal(size=100)
    m = np.zeros(100); v = np.zeros(100)
    g = rng.normal(size=100)
    th1 = theta.copy()
    orc.adam(th1, g, m, v, 1, 1e-2)
    assert np.abs(th1 - (theta - 1e-2 * g / (np.abs(g) + 1e-8))).max() < 1e-15
    # several steps against torch.optim.Adam in float64
    p = torch.nn.Parameter(torch.tensor(theta, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    th = theta.copy(); m[:] = 0; v[:] = 0
    for step in range(1, 6):
        gs = rng.normal(size=100)
        p.grad = torch.tensor(gs, dtype=torch.float64)
        opt.step()
        orc.adam(th, gs.copy(), m, v, step, 1e-3)
    assert np.abs(th - p.detach().numpy()).max() < 1e-14


def test_bf16_rounding_is_round_to_nearest_even(orc):
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(81).normal(size=10000).astype(np.float32)
    x[:4] = [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0]
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(orc.round_bf16(x), ref)
