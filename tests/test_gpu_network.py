"""GPU parity of the network stage on identical inputs: the psi encoding and the MLP heads of
libnif against the FP64 oracle fed the same FP32 rest-space points and the same table and
weight values (FP16 tables and BF16/FP16 weights widened exactly).

Bars (derivation in the design doc):
  encoding      |gpu - ref| <= 2e-6 * max|table|  (weights rounded to FP32, 8-term sums)
  FP32 heads    |gpu - ref| / max(|ref|, RMS of the head) <= 1e-5
  BF16 / FP16   per-head error reported; p99 of the same relative error <= 3e-2 / 4e-3."""
import dataclasses

import numpy as np
import pytest

import nif_synth as S
from _helpers import dev_f32, model_params, quantized_mlp, rel_err, say

pytestmark = pytest.mark.gpu

MODELS = {
    "torus16": S.workload("torus16").model,
    "spheres64": S.workload("spheres64").model,
    "spheres64_p": S.workload("spheres64_p").model,
    "small16": dataclasses.replace(S.workload("torus16").model, hidden_width=16, hidden_layers=1, n_materials=3),
    "w32": dataclasses.replace(S.workload("spheres64").model, hidden_width=32, hidden_layers=2, pe_freqs=2),
    "torus16_per_sample": dataclasses.replace(S.workload("torus16").model, per_sample_tables=1),
    "torus16_concat": dataclasses.replace(S.workload("torus16").model, concat_encoding=1),
    "w32_concat": dataclasses.replace(S.workload("spheres64").model, hidden_width=32, hidden_layers=2,
                                      concat_encoding=1),
    "w32_per_sample": dataclasses.replace(S.workload("spheres64").model, hidden_width=32, hidden_layers=2,
                                          pe_freqs=2, log2_table=16, per_sample_tables=1),
}


@pytest.fixture(scope="module")
def P():
    import paper_2604_24666_amd as P
    return P


def _points(n, seed):
    x0, x1 = S.random_points(n, seed, lo=-0.05, hi=1.05)
    return x0, x1


@pytest.mark.parametrize("name", ["torus16", "spheres64", "torus16_per_sample", "w32_per_sample", "torus16_concat"])
def test_encoding_matches_oracle(orc, P, name):
    m = MODELS[name]
    say(f"encode {name}")
    tab, prm, seen = model_params(m, 11, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    x, _ = _points(3001, 12)
    got = model.encode(dev_f32(x)).cpu().numpy().astype(np.float64)
    ref = orc.encode(m, seen, x.T.astype(np.float64))
    err = np.abs(got - ref).max()
    say(f"  max abs err {err:.3e}  max|table| {np.abs(seen).max():.3e}")
    assert err <= 2e-6 * np.abs(seen).max()


@pytest.mark.parametrize("name", list(MODELS))
def test_fp32_heads_match_oracle(orc, P, name):
    m = MODELS[name]
    say(f"forward fp32 {name}")
    tab, prm, seen = model_params(m, 21, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    rms = None
    for B in (2000 + 37, 63, 1):          # several tiles with a ragged tail, one partial tile, one
        x0, x1 = _points(B, 22 + B)
        got = model.forward(dev_f32(x0), dev_f32(x1), P.PREC_FP32).cpu().numpy().astype(np.float64)
        ref = orc.forward(m, seen, prm.astype(np.float64), x0.T.astype(np.float64), x1.T.astype(np.float64))
        if rms is None:
            rms = np.sqrt(np.mean(ref ** 2, axis=0, keepdims=True))
        e = np.abs(got - ref) / np.maximum(np.abs(ref), rms)
        say(f"  B={B}  max rel err {e.max():.3e}")
        assert e.max() <= 1e-5


def test_fp32_heads_at_the_training_batch_size_sampled(orc, P):
    """The training forward's size and model (B = 2^18 point pairs, MLP 832-128x4-12): every
    head of 1500 sampled rows against the oracle, to the FP32 bar."""
    m = S.workload("blobs128").model
    tab, prm, seen = model_params(m, 23, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    B = 1 << 18
    x0, x1 = _points(B, 24)
    got = model.forward(dev_f32(x0), dev_f32(x1), P.PREC_FP32).cpu().numpy().astype(np.float64)
    idx = np.sort(np.random.default_rng(25).choice(B, 1500, replace=False))
    idx[-1] = B - 1                                   # the last row of the last tile
    ref = orc.forward(m, seen, prm.astype(np.float64), x0[:, idx].T.astype(np.float64),
                      x1[:, idx].T.astype(np.float64))
    rms = np.sqrt(np.mean(ref ** 2, axis=0, keepdims=True))
    e = np.abs(got[idx] - ref) / np.maximum(np.abs(ref), rms)
    say(f"forward fp32 blobs128 B={B} sampled: max rel err {e.max():.3e}")
    assert e.max() <= 1e-5


@pytest.mark.parametrize("prec,p99", [(1, 3e-2), (2, 4e-3)])
@pytest.mark.parametrize("name", ["spheres64_p", "spheres64", "w32_concat"])
def test_low_precision_heads_error_per_head(orc, P, name, prec, p99):
    m = MODELS[name]
    say(f"forward prec={prec} {name}")
    tab, prm, seen = model_params(m, 31, scale_tables=1e3)
    model = P.Model(m)
    model.set_params(tab, prm)
    x0, x1 = _points(4096, 32)
    got = model.forward(dev_f32(x0), dev_f32(x1), prec).cpu().numpy().astype(np.float64)
    ref = orc.forward(m, seen, quantized_mlp(prm, prec), x0.T.astype(np.float64), x1.T.astype(np.float64))
    e = rel_err(got, ref)
    heads = {"hit": [0], "dist": [1], "normal": [2, 3, 4], "albedo": [5, 6, 7], "material": list(range(8, m.n_heads))}
    for h, cols in heads.items():
        say(f"  {h:8s} p50 {np.quantile(e[:, cols], 0.5):.2e}  p99 {np.quantile(e[:, cols], 0.99):.2e}")
    assert np.quantile(e, 0.99) <= p99


def test_fp32_heads_of_the_workload_models_are_not_trivial(orc, P):
    """The heads compared above span a useful range (not all ~0), so the relative bar bites."""
    m = MODELS["spheres64"]
    tab, prm, seen = model_params(m, 41)
    model = P.Model(m)
    model.set_params(tab, prm)
    x0, x1 = _points(512, 42)
    got = model.forward(dev_f32(x0), dev_f32(x1)).cpu().numpy()
    assert np.all(np.std(got, axis=0) > 0)
