"""BF16 / FP16 (and FP32) network arithmetic against the FP64 oracle, at bounds derived from
the arithmetic rather than fitted to it.

The oracle runs on exactly the parameters the GPU uses (FP16 tables; BF16/FP16-rounded MLP
weights widened exactly), so what separates the two is the GPU's own rounding: the FP32
encoding, the rounding of every MFMA operand that is not a stored weight to the MLP precision,
and FP32 accumulation.  tests/_bounds.py carries a first-order running-error bound of that
arithmetic through the layers, element by element: the heads of nif_forward, the parameter
gradients of nif_backward given the oracle's d heads, and the training step (losses, d / d s
and the gradients, whose d heads the step forms from its own heads: the loss's second
derivative over the heads' error interval is added).  Every element must lie within its
bound; the norm-wise error and the worst |error| / bound are reported.

Models: the training workload's network (MLP 832-128x4-12, 16-level 2^19 FP16 grid) and the
paper's comparison configuration (two levels of three features, F = 3, MLP 84-64x3-12); tables
U(+-0.03), the distance head's bias at half a voxel so that its ReLU is live."""
import numpy as np
import pytest

import nif_synth as S
import _bounds as BD
from _helpers import dev_f32, model_params, quantized_mlp, say

pytestmark = pytest.mark.gpu

MODELS = {"blobs128": S.workload("blobs128").model, "paper32": S.workload("spheres32_paper").model}
PRECS = [(1, "bf16"), (2, "fp16"), (0, "fp32")]
HEADS = {"hit": [0], "dist": [1], "normal": [2, 3, 4], "albedo": [5, 6, 7], "material": [8, 9, 10, 11]}


@pytest.fixture(scope="module")
def P():
    import paper_2604_24666_amd as P
    return P


def _setup(seed, prec, name="blobs128"):
    m = MODELS[name]
    tab, prm, seen = model_params(m, seed, scale_tables=300.0)
    prm[m.n_mlp_params - m.n_heads + 1] = 0.004
    return m, tab, prm, seen, quantized_mlp(prm, prec)


def _w0(m, prm):
    """The FP32 master first-layer weights (the table gradient's d enc uses them)."""
    return BD.layers(m, prm.astype(np.float64))[0][0]


def _batch(m, B, seed):
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(0.02, 0.98, (3, B)).astype(np.float32)
    x1 = (x0 + rng.normal(scale=0.03, size=(3, B))).astype(np.float32)
    hit = (rng.uniform(size=B) < 0.55).astype(np.uint8)
    t = rng.uniform(0.001, 0.04, B).astype(np.float32)
    nr = rng.normal(size=(3, B))
    nr = (nr / np.linalg.norm(nr, axis=0)).astype(np.float32)
    al = rng.uniform(0.1, 0.9, (3, B)).astype(np.float32)
    mt = rng.integers(0, m.n_materials, B).astype(np.int32)
    return x0, x1, hit, t, nr, al, mt


@pytest.mark.parametrize("name", list(MODELS))
@pytest.mark.parametrize("prec,pname", PRECS)
def test_heads_within_the_derived_bound(orc, P, prec, pname, name):
    m, tab, prm, seen, q = _setup(61, prec, name)
    B = 3000 + 17
    x0, x1, *_ = _batch(m, B, 62)
    say(f"heads {pname}: B={B}")
    model = P.Model(m)
    model.set_params(tab, prm)
    got = model.forward(dev_f32(x0), dev_f32(x1), prec).cpu().numpy().astype(np.float64)
    fw = BD.forward(orc, m, seen, q, x0.T.astype(np.float64), x1.T.astype(np.float64), prec)
    ref = orc.forward(m, seen, q, x0.T.astype(np.float64), x1.T.astype(np.float64))
    assert np.abs(fw["z"] - ref).max() <= 1e-12 * np.abs(ref).max()      # the bound's activations are the oracle's
    for h, cols in HEADS.items():
        e = np.abs(got[:, cols] - ref[:, cols]) / np.maximum(np.abs(ref[:, cols]), 1e-3 * np.sqrt(np.mean(ref[:, cols] ** 2)))
        r = np.abs(got[:, cols] - ref[:, cols]) / fw["sz"][:, cols]
        say(f"  {h:8s} relative error p50 {np.quantile(e, .5):.2e} p99 {np.quantile(e, .99):.2e} max {e.max():.2e};"
            f" |err| / sigma p99 {np.quantile(r, .99):.2f} max {r.max():.2f}")
    BD.check(got, ref, fw["sz"], "heads", say)


@pytest.mark.parametrize("name", list(MODELS))
@pytest.mark.parametrize("prec,pname", PRECS)
def test_backward_within_the_derived_bound(orc, P, prec, pname, name):
    import torch
    m, tab, prm, seen, q = _setup(71, prec, name)
    B = 2048 + 37
    x0, x1, hit, t, nr, al, mt = _batch(m, B, 72)
    s = np.array([0.2, -0.1, 0.3, 0.1, -0.2])
    X0, X1 = x0.T.astype(np.float64), x1.T.astype(np.float64)
    _, gt, gp, _, _, _, dz = orc.loss_grad(m, seen, q, s, X0, X1, hit, t, nr.T, al.T, mt, want_dz=True)
    # FP16 needs the caller's scaling of d heads (deltas ~1e-6 would be FP16 subnormals): the
    # largest d head is brought to ~64, a power of two
    sc = 2.0 ** np.floor(np.log2(64.0 / np.abs(dz).max())) if prec == 2 else 1.0
    say(f"backward {pname}: B={B}, d heads scaled by {sc:g}")
    model = P.Model(m)
    model.set_params(tab, prm)
    P.nif_model_reserve(model.h, B)
    P.nif_backward(model.h, dev_f32(x0), dev_f32(x1), B, dev_f32(dz * sc), None, None, False, prec)
    g_t, g_p, _ = [g.cpu().numpy().astype(np.float64) / sc for g in model.get_grads()]
    torch.cuda.synchronize()
    fw = BD.forward(orc, m, seen, q, X0, X1, prec)
    dz32 = (dz * sc).astype(np.float32).astype(np.float64) / sc
    Cdz = np.zeros((B, m.n_heads, m.n_heads))
    ih = np.arange(m.n_heads)
    Cdz[:, ih, ih] = (dz32 - dz) ** 2
    bw = BD.backward(orc, m, seen, q, fw, X0, X1, dz, Cdz, prec, scale=sc, W0_gpu=_w0(m, prm))
    BD.check(g_p, gp, bw["mlp"], "mlp", say)
    BD.check(g_t, gt, bw["tables"][1], "tables", say, det=bw["tables"][0], lam=BD.LAMBDA_TABLE,
             max_frac=BD.TABLE_FLIP_FRAC)


@pytest.mark.parametrize("name", list(MODELS))
@pytest.mark.parametrize("prec,pname", PRECS)
def test_train_step_within_the_derived_bound(orc, P, prec, pname, name):
    import torch
    m, tab, prm, seen, q = _setup(81, prec, name)
    B = 2048 + 11
    x0, x1, hit, t, nr, al, mt = _batch(m, B, 82)
    s0 = np.zeros(5)
    X0, X1 = x0.T.astype(np.float64), x1.T.astype(np.float64)
    L, gt, gp, gs, _, _, dz = orc.loss_grad(m, seen, q, s0, X0, X1, hit, t, nr.T, al.T, mt, want_dz=True)
    model = P.Model(m)
    model.set_params(tab, prm)
    P.nif_model_reserve(model.h, B)
    keep = [dev_f32(x0), dev_f32(x1), torch.as_tensor(hit).cuda(), dev_f32(t), dev_f32(nr), dev_f32(al),
            torch.as_tensor(mt).cuda()]
    # the loss scale: 1 for BF16 / FP32; for FP16 a power of two that brings the largest d head
    # to ~64 (the default 2^15 would overflow the FP16 deltas of this batch and skip the step)
    sc0 = 2.0 ** np.floor(np.log2(64.0 / np.abs(dz).max())) if prec == 2 else 0.0
    cfg = P.TrainCfg(1e-2, 1e-3, 1e-3, 0.9, 0.999, 1e-8, prec, sc0, 0, 0)
    losses = torch.zeros(16, device="cuda")
    P.nif_train_step(model.h, P.Batch(*[k.data_ptr() for k in keep]), B, cfg, losses)
    lo = losses.cpu().numpy().astype(np.float64)
    sc = lo[11]
    g_t, g_p, g_s = [g.cpu().numpy().astype(np.float64) for g in model.get_grads()]
    torch.cuda.synchronize()
    g_t /= sc
    g_p /= sc
    say(f"train step {pname}: B={B}, loss scale {sc:g}, skipped {lo[12]:g}")
    assert lo[12] == 0
    fw = BD.forward(orc, m, seen, q, X0, X1, prec)
    # losses: first-order model plus the FP32 evaluation of the per-sample terms
    bl = BD.LAMBDA * BD.loss_sigma(m, fw, dz, s0) + 4e-6 * np.abs(L[:5])
    say(f"  losses gpu {np.round(lo[:6], 6)}  oracle {np.round(L, 6)}  bound {bl}")
    assert np.all(np.abs(lo[:5] - L[:5]) <= bl)
    w = np.array([1.0, 0.5, 0.5, 0.5, 1.0]) * np.exp(-s0)
    assert abs(lo[5] - L[5]) <= float(np.sum(w * bl)) + 4e-6 * abs(L[5])
    assert np.all(np.abs(g_s - gs) <= w * bl + 4e-6)
    Cdz = BD.loss_dz_cov(m, fw, dz, hit, t.astype(np.float64), nr.T.astype(np.float64), al.T.astype(np.float64), s0)
    bw = BD.backward(orc, m, seen, q, fw, X0, X1, dz, Cdz, prec, scale=sc, W0_gpu=_w0(m, prm))
    BD.check(g_p, gp, bw["mlp"], "mlp", say)
    BD.check(g_t, gt, bw["tables"][1], "tables", say, det=bw["tables"][0], lam=BD.LAMBDA_TABLE,
             max_frac=BD.TABLE_FLIP_FRAC)
