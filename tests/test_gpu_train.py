"""GPU parity of the hand-written backward and of the training step against the FP64 oracle.

Bar: gradients within 1e-4 relative, norm-wise per tensor, and element-wise wherever
|g| > 1e-3 max|g|, both given the oracle's d loss / d heads and for a whole step (d loss /
d heads formed by the GPU from its own FP32 forward; the distance head's bias away from 0);
losses within 1e-5 relative; the first Adam update equals -lr g / (|g| + eps) element-wise."""
import ctypes as C
import dataclasses

import numpy as np
import pytest

import nif_synth as S
from _helpers import dev_f32, model_params, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2604_24666_amd as P
    return P


def _batch(m, B, seed):
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(0.02, 0.98, (3, B)).astype(np.float32)
    x1 = (x0 + rng.normal(scale=0.03, size=(3, B))).astype(np.float32)
    hit = (rng.uniform(size=B) < 0.55).astype(np.uint8)
    t = rng.uniform(0.001, 0.04, B).astype(np.float32)
    nr = rng.normal(size=(3, B))
    nr = (nr / np.linalg.norm(nr, axis=0)).astype(np.float32)
    al = rng.uniform(0.1, 0.9, (3, B)).astype(np.float32)
    mt = rng.integers(0, max(2, m.n_materials), B).astype(np.int32)
    if m.n_materials == 1:
        mt = np.minimum(mt, 1).astype(np.int32)
    return x0, x1, hit, t, nr, al, mt


def _grad_close(got, ref, name, big_frac=1e-3, el_tol=1e-4, sigma=None, lam=7.0):
    """Norm-wise 1e-4 and element-wise el_tol where |g| > big_frac max|g|; with sigma (the
    first-order rounding-error model of tests/_bounds.py), an element beyond el_tol passes if
    it lies within lam sigma (gradients that cancel over the batch: small against the sum of
    their terms, which sets their rounding error)."""
    got = np.asarray(got, dtype=np.float64).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1)
    nrm = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
    big = np.abs(ref) > big_frac * np.abs(ref).max()
    rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
    bad = big & (rel > el_tol)
    n_model = 0
    if sigma is not None:
        within = np.abs(got - ref) <= lam * np.asarray(sigma).reshape(-1)
        n_model = int((bad & within).sum())
        bad &= ~within
    el = rel[big].max(initial=0)
    say(f"  {name:8s} norm-wise {nrm:.2e}  element-wise (|g| > {big_frac:g} max) {el:.2e}  n={int(big.sum())}"
        + (f"  beyond {el_tol:g} but within the rounding model: {n_model}" if sigma is not None else ""))
    assert nrm <= 1e-4 and not bad.any(), name


MODELS = {
    "torus16": dataclasses.replace(S.workload("torus16").model, hidden_width=32),
    "torus16_per_sample": dataclasses.replace(S.workload("torus16").model, hidden_width=32, per_sample_tables=1),
    "torus16_concat": dataclasses.replace(S.workload("torus16").model, hidden_width=32, concat_encoding=1),
    "spheres64": S.workload("spheres64").model,
    "blobs128": S.workload("blobs128").model,
    "paper32": S.workload("spheres32_paper").model,
    "paper32_f32_per_sample": dataclasses.replace(S.workload("spheres32_paper").model, table_dtype=S.TABLE_F32,
                                                  log2_table=16, per_sample_tables=1, hidden_width=32),
    # 2^21-entry tables: 8192-entry buckets reduced in two LDS windows each, so the two entries
    # of a corner-pair record can fall into different windows
    "wide_table": dataclasses.replace(S.workload("torus16").model, levels=4, log2_table=21,
                                      res=[16, 64, 256, 1024], pe_freqs=2, hidden_width=32, hidden_layers=2),
    # 12 bands at width 128: the fill's first-layer rows (105 KiB) exceed its LDS budget, so it
    # reads them from memory
    "wide_pe": dataclasses.replace(S.workload("torus16").model, levels=4, res=[16, 32, 64, 128], pe_freqs=12,
                                   hidden_width=128, hidden_layers=1),
}


@pytest.mark.parametrize("name", list(MODELS))
def test_backward_matches_oracle_gradient(orc, P, name):
    import torch
    m = MODELS[name]
    say(f"backward {name}")
    tab, prm, seen = model_params(m, 5, scale_tables=300.0)
    B = 1500 + 37
    x0, x1, hit, t, nr, al, mt = _batch(m, B, 6)
    s = np.array([0.2, -0.1, 0.3, 0.1, -0.2])
    L, gt, gp, gs, gx0, gx1, dz = orc.loss_grad(m, seen, prm.astype(np.float64), s, x0.T, x1.T, hit, t, nr.T, al.T, mt,
                                                want_x=True, want_dz=True)
    model = P.Model(m)
    model.set_params(tab, prm, s.astype(np.float32))
    P.nif_model_reserve(model.h, B)
    dx0 = torch.empty((3, B), device="cuda")
    dx1 = torch.empty((3, B), device="cuda")
    P.nif_backward(model.h, dev_f32(x0), dev_f32(x1), B, dev_f32(dz), dx0, dx1, False, P.PREC_FP32)
    g_t, g_p, _ = model.get_grads()
    torch.cuda.synchronize()
    _grad_close(g_t.cpu().numpy(), gt, "tables")
    _grad_close(g_p.cpu().numpy(), gp, "mlp")
    _grad_close(dx0.cpu().numpy().T, gx0, "d x0")
    _grad_close(dx1.cpu().numpy().T, gx1, "d x1")


def _step_model(orc, m, seen, prm, batch, s, fixed=False):
    """sigma of the FP32 whole step's table and MLP gradients under the first-order
    rounding-error model (the step forms d heads from its own forward)."""
    import _bounds as BD
    x0, x1, hit, t, nr, al, mt = batch
    X0, X1, q = x0.T.astype(np.float64), x1.T.astype(np.float64), prm.astype(np.float64)
    dz = orc.loss_grad(m, seen, q, s, X0, X1, hit, t, nr.T, al.T, mt, want_dz=True, fixed_weights=fixed)[6]
    fw = BD.forward(orc, m, seen, q, X0, X1, 0)
    Cdz = BD.loss_dz_cov(m, fw, dz, hit, t.astype(np.float64), nr.T.astype(np.float64), al.T.astype(np.float64), s,
                         fixed=fixed, x0=X0, x1=X1)
    bw = BD.backward(orc, m, seen, q, fw, X0, X1, dz, Cdz, 0)
    return bw["tables"][1], bw["mlp"]


def _train_step(P, model, batch, B, prec=0, lr=(1e-2, 1e-3, 1e-3), fixed=False, store=False):
    import torch
    x0, x1, hit, t, nr, al, mt = batch
    keep = [dev_f32(x0), dev_f32(x1), torch.as_tensor(hit).cuda(), dev_f32(t), dev_f32(nr), dev_f32(al),
            torch.as_tensor(mt).cuda()]
    b = P.Batch(*[k.data_ptr() for k in keep])
    if store:
        P.nif_model_reserve_encoding(model.h)
    cfg = P.TrainCfg(lr[0], lr[1], lr[2], 0.9, 0.999, 1e-8, prec, 0.0, int(fixed), int(store))
    losses = torch.zeros(16, device="cuda")
    P.nif_train_step(model.h, b, B, cfg, losses)
    torch.cuda.synchronize()
    return losses.cpu().numpy()


@pytest.mark.parametrize("store", [False, True], ids=["recomputed_encoding", "stored_encoding"])
@pytest.mark.parametrize("name", ["torus16", "blobs128", "paper32"])
def test_train_step_matches_oracle(orc, P, name, store):
    m = MODELS[name]
    say(f"train step fp32 {name} store_encoding={int(store)}")
    tab, prm, seen = model_params(m, 7, scale_tables=300.0)
    # distance head live at half a voxel: with its bias at 0 the predicted distances sit near
    # 0, where the log-distance gradient 2 r / (d + eps) amplifies the forward's FP32 error by
    # up to 1 / eps
    prm[m.n_mlp_params - m.n_heads + 1] = 0.5 / 128
    B = 2048 + 11
    batch = _batch(m, B, 8)
    x0, x1, hit, t, nr, al, mt = batch
    s0 = np.zeros(5)
    L, gt, gp, gs, _, _ = orc.loss_grad(m, seen, prm.astype(np.float64), s0, x0.T, x1.T, hit, t, nr.T, al.T, mt)
    model = P.Model(m)
    model.set_params(tab, prm)
    P.nif_model_reserve(model.h, B)
    losses = _train_step(P, model, batch, B, store=store)
    say(f"  losses gpu {np.round(losses[:6], 6)}  oracle {np.round(L, 6)}")
    assert np.all(np.abs(losses[:6] - L) <= 1e-5 * np.maximum(np.abs(L), 1e-3))
    assert losses[12] == 0 and losses[13] == hit.sum()
    g_t, g_p, g_s = model.get_grads()
    st, sp = _step_model(orc, m, seen, prm, batch, s0)
    _grad_close(g_t.cpu().numpy(), gt, "tables", sigma=st)
    _grad_close(g_p.cpu().numpy(), gp, "mlp", sigma=sp)
    assert np.abs(g_s.cpu().numpy() - gs).max() <= 1e-5 * np.abs(gs).max()
    # first Adam step: theta - lr g / (|g| + eps), element-wise where the gradient is not tiny
    t1, p1, s1 = [v.cpu().numpy().astype(np.float64) for v in model.get_params()]
    for got, th0, g, lr in ((t1, tab.reshape(-1).astype(np.float64), gt.reshape(-1), 1e-2),
                            (p1, prm.astype(np.float64), gp, 1e-3)):
        ref = th0 - lr * g / (np.abs(g) + 1e-8)
        big = np.abs(g) > 1e-3 * np.abs(g).max()
        assert np.abs(got - ref)[big].max() <= 1e-6 * max(1.0, np.abs(th0).max()) + 1e-7
    assert np.abs(s1 - (s0 - 1e-3 * gs / (np.abs(gs) + 1e-8))).max() <= 1e-6


ABLATIONS = {
    "sigmoid_head_fixed_weights": (dict(dist_head=S.DIST_SIGMOID), True),
    "no_pe": (dict(pe_freqs=0), False),
    "no_pe_sigmoid_head_fixed_weights": (dict(pe_freqs=0, dist_head=S.DIST_SIGMOID), True),
    "per_sample_tables": (dict(per_sample_tables=1), False),
    "concat_encoding": (dict(concat_encoding=1), False),
}


@pytest.mark.parametrize("variant", list(ABLATIONS))
def test_train_step_ablation_switches_match_oracle(orc, P, variant):
    """The baselines' training: sigmoid-fraction distance (MSE against t*/l), unit task
    weights with s untouched, and F = 0; losses, gradients and the first Adam step."""
    kw, fixed = ABLATIONS[variant]
    m = dataclasses.replace(MODELS["torus16"], **kw)
    say(f"train step fp32 torus16 ablation {variant}")
    tab, prm, seen = model_params(m, 9, scale_tables=300.0)
    # distance bias 1: the log-distance gradient 2 r / (d + eps) would otherwise amplify the
    # FP32 rounding of the forward by up to 1 / eps wherever the predicted d is near 0 (the raw
    # gamma inputs of the concatenated encoding spread the first-layer outputs by O(1))
    prm[m.n_mlp_params - m.n_heads + 1] = 1.0
    B = 2048 + 13
    batch = _batch(m, B, 10)
    x0, x1, hit, t, nr, al, mt = batch
    t[:50] = 0.2                              # some targets beyond the segment: t*/l clamps to 1
    s0 = np.array([0.3, -0.2, 0.1, 0.4, -0.5]) if fixed else np.zeros(5)
    L, gt, gp, gs, _, _ = orc.loss_grad(m, seen, prm.astype(np.float64), s0, x0.T, x1.T, hit, t, nr.T, al.T, mt,
                                        fixed_weights=fixed)
    model = P.Model(m)
    model.set_params(tab, prm, s0.astype(np.float32))
    P.nif_model_reserve(model.h, B)
    losses = _train_step(P, model, batch, B, fixed=fixed)
    say(f"  losses gpu {np.round(losses[:6], 6)}  oracle {np.round(L, 6)}")
    assert np.all(np.abs(losses[:6] - L) <= 1e-5 * np.maximum(np.abs(L), 1e-3))
    g_t, g_p, g_s = model.get_grads()
    st, sp = _step_model(orc, m, seen, prm, batch, s0, fixed=fixed)
    _grad_close(g_t.cpu().numpy(), gt, "tables", sigma=st)
    _grad_close(g_p.cpu().numpy(), gp, "mlp", sigma=sp)
    t1, p1, s1 = [v.cpu().numpy().astype(np.float64) for v in model.get_params()]
    if fixed:
        assert np.all(g_s.cpu().numpy() == 0) and np.all(s1 == s0.astype(np.float32))
    else:
        assert np.abs(g_s.cpu().numpy() - gs).max() <= 1e-5 * np.abs(gs).max()
    for got, th0, g, lr in ((t1, tab.reshape(-1).astype(np.float64), gt.reshape(-1), 1e-2),
                            (p1, prm.astype(np.float64), gp, 1e-3)):
        ref = th0 - lr * g / (np.abs(g) + 1e-8)
        big = np.abs(g) > 1e-3 * np.abs(g).max()
        assert np.abs(got - ref)[big].max() <= 1e-6 * max(1.0, np.abs(th0).max()) + 1e-7


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_training_reduces_the_loss(orc, P, prec):
    m = MODELS["blobs128"]
    say(f"training loop prec={prec}")
    tab, prm, _ = model_params(m, 9)
    B = 8192
    batch = _batch(m, B, 10)
    model = P.Model(m)
    model.set_params(tab, prm)
    P.nif_model_reserve(model.h, B)
    first = last = None
    for it in range(30):
        losses = _train_step(P, model, batch, B, prec)
        assert np.all(np.isfinite(losses[:6]))
        if first is None:
            first = losses[5]
        last = losses[5]
    say(f"  total loss {first:.4f} -> {last:.4f}  loss scale {losses[11]}")
    assert last < first


@pytest.mark.parametrize("prec", [0, 1])
def test_stored_and_recomputed_encoding_give_the_same_step(P, prec):
    """The two encoding policies of the training step at a batch of several recomputation
    chunks (2^17 + 4321 samples, spatially ordered): same losses and task-weight gradients;
    table gradients equal up to FP32 rounding (that path never reads the encoding, but its
    register-merged runs and multi-part slices are summed in an order set by atomics); MLP
    gradients equal up to the summation order of the first layer's chunks."""
    import torch
    m = MODELS["blobs128"]
    tab, prm, _ = model_params(m, 21, scale_tables=300.0)
    B = (1 << 17) + 4321
    batch = _batch(m, B, 22)
    out = []
    for store in (False, True):
        say(f"train step policy store_encoding={int(store)} prec={prec} B={B}")
        model = P.Model(m)
        model.set_params(tab, prm)
        P.nif_model_reserve(model.h, B)
        losses = _train_step(P, model, batch, B, prec, store=store)
        g_t, g_p, g_s = [g.cpu().numpy().astype(np.float64) for g in model.get_grads()]
        out.append((losses, g_t, g_p, g_s))
        del model
    (l0, t0, p0, s0), (l1, t1, p1, s1) = out
    np.testing.assert_array_equal(l0[:6], l1[:6])
    np.testing.assert_array_equal(s0, s1)
    for name, a, b in (("tables", t0, t1), ("mlp", p0, p1)):
        rel = np.linalg.norm(a - b) / np.linalg.norm(a)
        say(f"  {name} gradient relative difference {rel:.2e}, max {np.abs(a - b).max():.2e}")
        assert np.linalg.norm(a) > 0 and rel <= 1e-6, name
        assert np.abs(a - b).max() <= 1e-5 * np.abs(a).max(), name


@pytest.mark.parametrize("store", [False, True], ids=["recomputed_encoding", "stored_encoding"])
def test_pipelined_step_at_full_batch_matches_the_separate_calls(P, store):
    """At the benchmark's training batch (2^18 samples: spatially ordered, two pipelined
    chunks of one table-gradient round on the side stream) the step's losses and gradients
    equal those of nif_forward -> nif_loss -> nif_backward on the same batch (calls held to the
    oracle by the tests above), within FP32 summation-order error."""
    import torch
    m = MODELS["blobs128"]
    tab, prm, _ = model_params(m, 41, scale_tables=300.0)
    B = 1 << 18
    x0, x1, hit, t, nr, al, mt = _batch(m, B, 42)
    labels = [dev_f32(x0), dev_f32(x1), torch.as_tensor(hit).cuda(), dev_f32(t), dev_f32(nr), dev_f32(al),
              torch.as_tensor(mt).cuda()]
    lb = P.Batch(*[k.data_ptr() for k in labels])
    say(f"pipelined step B={B} store_encoding={int(store)}")
    ref = P.Model(m)
    ref.set_params(tab, prm)
    P.nif_model_reserve(ref.h, B)
    heads = ref.forward(labels[0], labels[1])
    losses_ref = torch.zeros(6, device="cuda")
    d_heads = torch.empty_like(heads)
    d_s = torch.empty(5, device="cuda")
    P.nif_loss(ref.h, heads, B, lb, torch.zeros(5, device="cuda"), False, losses_ref, d_heads, d_s)
    P.nif_backward(ref.h, labels[0], labels[1], B, d_heads, None, None, False, P.PREC_FP32)
    r_t, r_p, _ = [g.cpu().numpy().astype(np.float64) for g in ref.get_grads()]
    del ref
    model = P.Model(m)
    model.set_params(tab, prm)
    P.nif_model_reserve(model.h, B)
    if store:
        P.nif_model_reserve_encoding(model.h)
    cfg = P.TrainCfg(1e-2, 1e-3, 1e-3, 0.9, 0.999, 1e-8, P.PREC_FP32, 0.0, 0, int(store))
    losses = torch.zeros(16, device="cuda")
    P.nif_train_step(model.h, lb, B, cfg, losses)
    g_t, g_p, g_s = [g.cpu().numpy().astype(np.float64) for g in model.get_grads()]
    torch.cuda.synchronize()
    got, want = losses.cpu().numpy()[:6].astype(np.float64), losses_ref.cpu().numpy().astype(np.float64)
    say(f"  losses step {np.round(got, 6)}  separate {np.round(want, 6)}")
    assert np.all(np.abs(got - want) <= 1e-5 * np.maximum(np.abs(want), 1e-3))
    assert np.abs(g_s - d_s.cpu().numpy()).max() <= 1e-5 * max(np.abs(d_s.cpu().numpy()).max(), 1e-3)
    for name, a, b in (("tables", g_t, r_t), ("mlp", g_p, r_p)):
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        say(f"  {name} gradient relative difference {rel:.2e}")
        assert np.linalg.norm(b) > 0 and rel <= 1e-5, name


def test_stored_encoding_step_needs_its_reservation(P):
    m = MODELS["torus16"]
    model = P.Model(m)
    tab, prm, _ = model_params(m, 3)
    model.set_params(tab, prm)
    P.nif_model_reserve(model.h, 64)
    import torch
    batch = _batch(m, 64, 1)
    x0, x1, hit, t, nr, al, mt = batch
    keep = [dev_f32(x0), dev_f32(x1), torch.as_tensor(hit).cuda(), dev_f32(t), dev_f32(nr), dev_f32(al),
            torch.as_tensor(mt).cuda()]
    b = P.Batch(*[k.data_ptr() for k in keep])
    cfg = P.TrainCfg(1e-2, 1e-3, 1e-3, 0.9, 0.999, 1e-8, 0, 0.0, 0, 1)
    with pytest.raises(P.NifError):
        P.nif_train_step(model.h, b, 64, cfg, torch.zeros(16, device="cuda"))


LOSS_CASES = {
    "torus16": ("torus16", {}, False, False),
    "blobs128": ("blobs128", {}, False, False),
    "blobs128_fixed_weights": ("blobs128", {}, True, False),
    "blobs128_sigmoid_head": ("blobs128", dict(dist_head=S.DIST_SIGMOID), False, False),
    "blobs128_no_hits": ("blobs128", {}, False, True),
}


@pytest.mark.parametrize("case", list(LOSS_CASES))
def test_multitask_loss_matches_oracle(orc, P, case):
    """nif_loss and its autograd wrapper on heads the oracle computed: the five task losses and
    the total to 1e-5, d total / d heads (through NifMultiTaskLoss.backward) and d total / d s
    to the gradient bar; with no positive label the masked terms are zero."""
    import torch
    name, kw, fixed, no_hits = LOSS_CASES[case]
    m = dataclasses.replace(MODELS[name], **kw)
    say(f"loss {case}")
    tab, prm, seen = model_params(m, 31, scale_tables=300.0)
    B = 1000 + 23
    x0, x1, hit, t, nr, al, mt = _batch(m, B, 32)
    if no_hits:
        hit = np.zeros_like(hit)
    s = np.array([0.2, -0.1, 0.3, 0.1, -0.2])
    z = orc.forward(m, seen, prm.astype(np.float64), x0.T, x1.T)
    L, _, _, gs, _, _, dz = orc.loss_grad(m, seen, prm.astype(np.float64), s, x0.T, x1.T, hit, t, nr.T, al.T, mt,
                                          want_dz=True, fixed_weights=fixed)
    model = P.Model(m)
    labels = [dev_f32(x0), dev_f32(x1), torch.as_tensor(hit).cuda(), dev_f32(t), dev_f32(nr), dev_f32(al),
              torch.as_tensor(mt).cuda()]
    heads = dev_f32(z).requires_grad_(True)
    s_dev = dev_f32(s).requires_grad_(True)
    total = P.NifMultiTaskLoss.apply(heads, s_dev, model, labels, fixed)
    (2.0 * total).backward()
    losses = torch.zeros(6, device="cuda")
    P.nif_loss(model.h, heads.detach(), B, P.Batch(*[k.data_ptr() for k in labels]), s_dev.detach(), fixed, losses)
    torch.cuda.synchronize()
    got = losses.cpu().numpy().astype(np.float64)
    say(f"  losses gpu {np.round(got, 6)}  oracle {np.round(L, 6)}")
    assert np.all(np.abs(got - L) <= 1e-5 * np.maximum(np.abs(L), 1e-3))
    assert abs(total.detach().item() - L[5]) <= 1e-5 * max(abs(L[5]), 1e-3)
    if no_hits:
        assert np.all(got[1:5] == 0.0)
        assert np.all(heads.grad.cpu().numpy()[:, 1:] == 0.0)
    _grad_close(heads.grad.cpu().numpy() / 2.0, dz, "d heads")
    g_s = s_dev.grad.cpu().numpy().astype(np.float64) / 2.0
    assert np.abs(g_s - gs).max() <= 1e-5 * max(np.abs(gs).max(), 1e-3)
    if fixed:
        assert np.all(g_s == 0.0)


def test_train_step_rejects_oversized_batches(P):
    m = MODELS["torus16"]
    model = P.Model(m)
    tab, prm, _ = model_params(m, 3)
    model.set_params(tab, prm)
    P.nif_model_reserve(model.h, 64)
    with pytest.raises(P.NifError):
        _train_step(P, model, _batch(m, 65, 1), 65)


@pytest.mark.parametrize("B", [(1 << 17) + 4321, (1 << 18) + 4321])
def test_backward_over_several_chunks_is_additive(P, B):
    """Batches of more than one chunk (2^17 samples) in one table-gradient round, and of more
    than one round (2^18 samples): the gradient of the whole batch equals the gradient of its
    two halves accumulated (the sum is linear in the samples), within FP32 summation-order
    error."""
    import torch
    m = MODELS["blobs128"]
    tab, prm, _ = model_params(m, 11, scale_tables=300.0)
    x0, x1, hit, t, nr, al, mt = _batch(m, B, 12)
    rng = np.random.default_rng(13)
    dz = rng.normal(size=(B, m.n_heads)).astype(np.float32)
    model = P.Model(m)
    model.set_params(tab, prm)
    P.nif_model_reserve(model.h, B)
    say(f"backward additivity B={B}")
    P.nif_backward(model.h, dev_f32(x0), dev_f32(x1), B, dev_f32(dz), None, None, False, P.PREC_FP32)
    g_t, g_p, _ = [g.clone() for g in model.get_grads()]
    h = B // 2 + 17
    parts = [(0, h), (h, B)]
    for i, (a, b) in enumerate(parts):
        P.nif_backward(model.h, dev_f32(np.ascontiguousarray(x0[:, a:b])), dev_f32(np.ascontiguousarray(x1[:, a:b])),
                       b - a, dev_f32(dz[a:b]), None, None, i > 0, P.PREC_FP32)
    h_t, h_p, _ = model.get_grads()
    torch.cuda.synchronize()
    for name, full, acc in (("tables", g_t, h_t), ("mlp", g_p, h_p)):
        full = full.cpu().numpy().astype(np.float64); acc = acc.cpu().numpy().astype(np.float64)
        nrm = np.linalg.norm(full - acc) / np.linalg.norm(full)
        say(f"  {name}: relative difference {nrm:.2e}")
        assert np.linalg.norm(full) > 0 and nrm <= 1e-5, name


def test_autograd_wrappers_compose_to_the_oracle_gradient(orc, P):
    """NifField (heads with the hand-written backward) composed with NifMultiTaskLoss under
    torch.autograd: the table and MLP gradients equal the oracle's gradient of the same loss to
    the whole step's bar (the composition is the step's forward, loss and backward), d s to
    1e-5; d x0 / d x1 equal the oracle's norm-wise and, element by element, the C-ABI backward
    fed the same d heads (the wrapper adds only plumbing; the two differ in the order of FP32
    atomic additions)."""
    import torch
    m = MODELS["blobs128"]
    tab, prm, seen = model_params(m, 51, scale_tables=300.0)
    B = 1500 + 13
    batch = _batch(m, B, 52)
    x0, x1, hit, t, nr, al, mt = batch
    s = np.array([0.1, -0.3, 0.2, 0.0, 0.4])
    say(f"autograd composition B={B}")
    L, gt, gp, gs, gx0, gx1 = orc.loss_grad(m, seen, prm.astype(np.float64), s, x0.T, x1.T, hit, t, nr.T, al.T, mt,
                                            want_x=True)
    sig_t, sig_p = _step_model(orc, m, seen, prm, batch, s)
    model = P.Model(m, max_batch=B)
    model.set_params(tab, prm)
    P.nif_model_zero_grads(model.h)
    X0 = dev_f32(x0).requires_grad_(True)
    X1 = dev_f32(x1).requires_grad_(True)
    sv = dev_f32(s).requires_grad_(True)
    labels = [X0.detach(), X1.detach(), torch.as_tensor(hit).cuda(), dev_f32(t), dev_f32(nr), dev_f32(al),
              torch.as_tensor(mt).cuda()]
    heads = P.NifField.apply(X0, X1, model, P.PREC_FP32)
    total = P.NifMultiTaskLoss.apply(heads, sv, model, labels)
    total.backward()
    g_t, g_p, _ = model.get_grads()
    # the C-ABI backward of the same d heads, on a second model
    d_heads = torch.empty_like(heads)
    d_s = torch.empty(5, device="cuda")
    P.nif_loss(model.h, heads.detach(), B, P.Batch(*[k.data_ptr() for k in labels]), sv.detach(), False,
               torch.empty(6, device="cuda"), d_heads, d_s)
    direct = P.Model(m, max_batch=B)
    direct.set_params(tab, prm)
    dx0 = torch.empty((3, B), device="cuda")
    dx1 = torch.empty((3, B), device="cuda")
    P.nif_backward(direct.h, X0.detach(), X1.detach(), B, d_heads, dx0, dx1, False, P.PREC_FP32)
    torch.cuda.synchronize()
    assert abs(total.item() - L[5]) <= 1e-5 * abs(L[5])
    _grad_close(g_t.cpu().numpy(), gt, "tables", sigma=sig_t)
    _grad_close(g_p.cpu().numpy(), gp, "mlp", sigma=sig_p)
    assert np.abs(sv.grad.cpu().numpy() - gs).max() <= 1e-5 * np.abs(gs).max()
    for name, got, ref, dref in (("d x0", X0.grad, gx0, dx0), ("d x1", X1.grad, gx1, dx1)):
        got = got.cpu().numpy().astype(np.float64)
        nrm = np.linalg.norm(got.T - ref) / np.linalg.norm(ref)
        say(f"  {name}  norm-wise vs oracle {nrm:.2e}")
        assert nrm <= 1e-4, name
        dref = dref.cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(got, dref, rtol=1e-5, atol=1e-6 * np.abs(dref).max(), err_msg=name)
    # a batch larger than the reservation is refused (the backward allocates nothing)
    small = P.Model(m, max_batch=64)
    small.set_params(tab, prm)
    h2 = P.NifField.apply(X0, X1, small, P.PREC_FP32)
    with pytest.raises(P.NifError):
        h2.sum().backward()


@pytest.mark.parametrize("B", [4096 + 7, (1 << 17) + 4099, (1 << 18) + (1 << 17) + 4099],
                         ids=["one_chunk", "two_chunks", "two_rounds"])
def test_train_step_captured_in_a_graph_replays_like_eager(P, B):
    """nif_train_step captured in a hipGraph (with its side-stream fork and join) and replayed
    three times, with eager work between the replays: every replay's losses and gradients
    equal an eager step's (learning rates 0, so each step sees the same parameters; losses and
    gradients to 1e-6, the order of their FP32 sums)."""
    import torch
    m = MODELS["blobs128"]
    tab, prm, _ = model_params(m, 61, scale_tables=300.0)
    batch = _batch(m, B, 62)
    x0, x1, hit, t, nr, al, mt = batch
    keep = [dev_f32(x0), dev_f32(x1), torch.as_tensor(hit).cuda(), dev_f32(t), dev_f32(nr), dev_f32(al),
            torch.as_tensor(mt).cuda()]
    b = P.Batch(*[k.data_ptr() for k in keep])
    cfg = P.TrainCfg(0.0, 0.0, 0.0, 0.9, 0.999, 1e-8, P.PREC_BF16, 0.0, 0, 0)
    model = P.Model(m, max_batch=B)
    model.set_params(tab, prm)
    say(f"train step graph capture B={B}")
    losses = torch.zeros(16, device="cuda")
    P.nif_train_step(model.h, b, B, cfg, losses)
    torch.cuda.synchronize()
    ref_l = losses.cpu().numpy().copy()
    ref_g = [g.cpu().numpy().astype(np.float64) for g in model.get_grads()]
    s_cap = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    cap_losses = torch.zeros(16, device="cuda")
    with torch.cuda.graph(g, stream=s_cap):
        P.nif_train_step(model.h, b, B, cfg, cap_losses, stream=s_cap)
    other = torch.zeros(16, device="cuda")
    for rep in range(3):
        cap_losses.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        got_l = cap_losses.cpu().numpy()
        np.testing.assert_allclose(got_l[:6], ref_l[:6], rtol=1e-6)
        assert got_l[12] == 0 and got_l[13] == ref_l[13]
        for name, a, r in zip(("tables", "mlp", "s"), model.get_grads(), ref_g):
            a = a.cpu().numpy().astype(np.float64)
            rel = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-300)
            assert rel <= 1e-6, f"replay {rep}: {name} gradient differs by {rel:.2e}"
        P.nif_train_step(model.h, b, B, cfg, other)          # eager work between replays
        torch.cuda.synchronize()
    del g


def test_backward_captured_in_a_graph_replays_like_eager(P):
    """nif_backward (accumulators zeroed by kernels, side-stream fork and join) captured in a
    hipGraph and replayed three times with eager work between: gradients and d x0 / d x1 of
    every replay equal an eager call's (FP32 atomic order: 1e-6 norm-wise)."""
    import torch
    m = MODELS["blobs128"]
    tab, prm, _ = model_params(m, 91, scale_tables=300.0)
    B = (1 << 16) + 333
    rng = np.random.default_rng(92)
    x0 = dev_f32(rng.uniform(0.02, 0.98, (3, B)))
    x1 = dev_f32(rng.uniform(0.02, 0.98, (3, B)))
    dh = dev_f32(rng.normal(size=(B, m.n_heads)) * 1e-3)
    model = P.Model(m, max_batch=B)
    model.set_params(tab, prm)
    say(f"backward graph capture B={B}")
    dx0 = torch.empty((3, B), device="cuda")
    dx1 = torch.empty((3, B), device="cuda")
    P.nif_backward(model.h, x0, x1, B, dh, dx0, dx1, False, P.PREC_FP32)
    torch.cuda.synchronize()
    ref = [g.cpu().numpy().astype(np.float64) for g in model.get_grads()] + [dx0.cpu().numpy(), dx1.cpu().numpy()]
    s_cap = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    cx0 = torch.empty((3, B), device="cuda")
    cx1 = torch.empty((3, B), device="cuda")
    with torch.cuda.graph(g, stream=s_cap):
        P.nif_backward(model.h, x0, x1, B, dh, cx0, cx1, False, P.PREC_FP32, stream=s_cap)
    ox0 = torch.empty((3, B), device="cuda")
    ox1 = torch.empty((3, B), device="cuda")
    for rep in range(3):
        cx0.fill_(7.0)
        g.replay()
        torch.cuda.synchronize()
        got = [a.cpu().numpy().astype(np.float64) for a in model.get_grads()] + [cx0.cpu().numpy(), cx1.cpu().numpy()]
        for name, a, r in zip(("tables", "mlp", "s", "d x0", "d x1"), got, ref):
            rel = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-300)
            assert rel <= 1e-6, f"replay {rep}: {name} differs by {rel:.2e}"
        P.nif_backward(model.h, x1, x0, B, dh, ox0, ox1, True, P.PREC_FP32)     # eager work between replays
        torch.cuda.synchronize()
    del g
