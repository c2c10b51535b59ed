"""Dynamic loss scaling and the non-finite skip of the training step (BF16/FP16 MLP with FP32
accumulation; the FP32 step keeps the scale at 1 but skips the same way).

 - A batch with one non-finite label (t = NaN on a hit sample) makes the loss and the
   gradients non-finite: the step reports skipped = 1 and the scale it used, halves the scale
   (BF16/FP16), and leaves parameters, the working copies (forward outputs), the Adam moments
   and the step counter untouched: the next clean step is Adam's second step, computed here
   from the first step's parameters and both steps' gradients.
 - FP16 with an initial scale of 2^40 overflows the FP16 deltas: every step is skipped and
   halves the scale until the scaled deltas fit, then the steps proceed.
 - With a growth interval of 2 clean steps the scale doubles every second step; the
   gradient is unscaled exactly (powers of two), so the parameters follow the run at a fixed
   scale."""
import dataclasses

import numpy as np
import pytest

import nif_synth as S
from _helpers import dev_f32, model_params, say

pytestmark = pytest.mark.gpu

MODEL = dataclasses.replace(S.workload("blobs128").model)
B = 2048 + 29


@pytest.fixture(scope="module")
def P():
    import paper_2604_24666_amd as P
    return P


def _batch(seed):
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(0.02, 0.98, (3, B)).astype(np.float32)
    x1 = (x0 + rng.normal(scale=0.03, size=(3, B))).astype(np.float32)
    hit = (rng.uniform(size=B) < 0.55).astype(np.uint8)
    t = rng.uniform(0.001, 0.04, B).astype(np.float32)
    nr = rng.normal(size=(3, B))
    nr = (nr / np.linalg.norm(nr, axis=0)).astype(np.float32)
    al = rng.uniform(0.1, 0.9, (3, B)).astype(np.float32)
    mt = rng.integers(0, MODEL.n_materials, B).astype(np.int32)
    return [x0, x1, hit, t, nr, al, mt]


def _model(P, seed=5):
    m = MODEL
    tab, prm, _ = model_params(m, seed, scale_tables=300.0)
    prm[m.n_mlp_params - m.n_heads + 1] = 0.004          # distance head live from the first step
    model = P.Model(m)
    model.set_params(tab, prm)
    P.nif_model_reserve(model.h, B)
    return model


class _Runner:
    def __init__(self, P, model, prec, scale_init=0.0, grow=0):
        self.P, self.model = P, model
        self.cfg = P.TrainCfg(1e-2, 1e-3, 1e-3, 0.9, 0.999, 1e-8, prec, scale_init, 0, 0, grow)

    def step(self, batch):
        import torch
        P = self.P
        x0, x1, hit, t, nr, al, mt = batch
        keep = [dev_f32(x0), dev_f32(x1), torch.as_tensor(hit).cuda(), dev_f32(t), dev_f32(nr), dev_f32(al),
                torch.as_tensor(mt).cuda()]
        losses = torch.zeros(16, device="cuda")
        P.nif_train_step(self.model.h, P.Batch(*[k.data_ptr() for k in keep]), B, self.cfg, losses)
        torch.cuda.synchronize()
        return losses.cpu().numpy()

    def params(self):
        import torch
        out = [v.cpu().numpy().copy() for v in self.model.get_params()]
        torch.cuda.synchronize()
        return out

    def heads(self, batch, prec):
        import torch
        h = self.model.forward(dev_f32(batch[0]), dev_f32(batch[1]), prec)
        torch.cuda.synchronize()
        return h.cpu().numpy()


def _adam2(theta1, g1, g2, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Parameters after a second Adam step (bias corrections of step 2) from those after the
    first, given both steps' gradients: the moments of step 1 are (1 - b1) g1, (1 - b2) g1^2."""
    m = b1 * (1 - b1) * g1 + (1 - b1) * g2
    v = b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2
    return theta1 - lr * (m / (1 - b1 ** 2)) / (np.sqrt(v / (1 - b2 ** 2)) + eps)


@pytest.mark.parametrize("prec", [1, 2, 0], ids=["bf16", "fp16", "fp32"])
def test_non_finite_step_is_skipped_and_halves_the_scale(P, prec):
    import torch
    say(f"non-finite skip prec={prec}")
    clean1, clean2 = _batch(1), _batch(2)
    bad = [a.copy() for a in _batch(3)]
    bad[3][int(np.flatnonzero(bad[2])[0])] = np.nan          # t of one hit sample
    # FP16 at the default initial scale (2^15) overflows the deltas of this untrained model and
    # would skip the first clean step too; start every precision at 1
    a = _Runner(P, _model(P), prec, scale_init=1.0)

    def grads(scale):
        g = [v.cpu().numpy().astype(np.float64) for v in a.model.get_grads()]
        torch.cuda.synchronize()
        return [g[0] / scale, g[1] / scale, g[2]]           # the s gradient is not loss-scaled

    l1 = a.step(clean1)
    scale = l1[11]
    assert l1[12] == 0 and np.all(np.isfinite(l1[:6]))
    p1, h1, g1 = a.params(), a.heads(clean2, prec), grads(l1[11])
    lb = a.step(bad)
    say(f"  bad step: skipped {lb[12]}, scale used {lb[11]}, total {lb[5]}")
    assert lb[12] == 1 and lb[11] == scale and not np.isfinite(lb[5])
    pb, hb = a.params(), a.heads(clean2, prec)
    for x, y in zip(p1, pb):
        np.testing.assert_array_equal(x, y)                 # masters untouched
    np.testing.assert_array_equal(h1, hb)                   # working copies untouched
    l2 = a.step(clean2)
    new_scale = scale / 2 if prec else scale
    assert l2[12] == 0 and l2[11] == new_scale
    g2, p2 = grads(l2[11]), a.params()
    # the clean step after the skipped one is Adam's second step from the first step's moments:
    # a step count taken by the skipped step (bias corrections of step 3) moves a table entry by
    # ~14 % of its learning rate, moments fed the bad batch make it NaN
    worst = 0.0
    for th1, th2, ga, gb, lr in zip(p1, p2, g1, g2, (1e-2, 1e-3, 1e-3)):
        want = _adam2(th1.astype(np.float64), ga, gb, lr)
        worst = max(worst, float(np.abs(th2 - want).max() / lr))
    say(f"  after the next clean step: largest |theta - Adam step 2| / lr = {worst:.2e}")
    assert worst <= 1e-4


def test_fp16_overflow_halves_until_the_deltas_fit(P):
    say("fp16 overflow: initial scale 2^40")
    a = _Runner(P, _model(P, 7), 2, scale_init=2.0 ** 40)
    batch = _batch(4)
    p0 = a.params()
    scales, skipped = [], []
    for _ in range(40):
        lo = a.step(batch)
        scales.append(float(lo[11]))
        skipped.append(int(lo[12]))
        if not lo[12]:
            break
    say(f"  scales used {[np.log2(s) for s in scales]}  skipped {skipped}")
    assert skipped[0] == 1 and skipped[-1] == 0 and all(skipped[:-1])
    assert scales == [2.0 ** (40 - i) for i in range(len(scales))]
    p1 = a.params()
    assert max(np.abs(x - y).max() for x, y in zip(p0, p1)) > 1e-3      # the first clean step updated


@pytest.mark.parametrize("prec", [1, 0], ids=["bf16", "fp32"])
def test_scale_grows_after_the_interval(P, prec):
    """Learning rates 0, so every step sees the same parameters: the scale used goes 1, 1, 2,
    2, 4 (FP32: stays 1), and each step's gradient accumulators, divided by the scale it used,
    equal those of a run at the default interval (BF16 has FP32's exponent range, so scaling
    by powers of two is exact; FP16 takes the same code path but rounds its small deltas
    differently at each scale)."""
    import torch
    say(f"growth interval 2, prec={prec}")
    batches = [_batch(10 + i) for i in range(5)]
    runs = [_Runner(P, _model(P, 9), prec, scale_init=1.0, grow=g) for g in (2, 0)]
    for r in runs:
        r.cfg.lr_table = r.cfg.lr_mlp = r.cfg.lr_s = 0.0
    used = []
    for b in batches:
        grads = []
        for r in runs:
            lo = r.step(b)
            g = [v.cpu().numpy().astype(np.float64) / lo[11] for v in r.model.get_grads()[:2]]
            torch.cuda.synchronize()
            grads.append((float(lo[11]), g))
        used.append(grads[0][0])
        assert grads[1][0] == 1.0
        for x, y in zip(grads[0][1], grads[1][1]):
            rel = np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300)
            assert rel <= 1e-6, f"unscaled gradients differ by {rel:.2e} at scale {grads[0][0]}"
    say(f"  scales used {used}")
    assert used == ([1.0, 1.0, 2.0, 2.0, 4.0] if prec else [1.0] * 5)
