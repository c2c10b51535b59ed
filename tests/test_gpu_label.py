"""GPU labels of rest-space segments (training-data generation) against the FP64 oracle's.

Chords x0 -> x0 + r u with x0 uniform in the unit cube, u uniform on S^2 and r in [0, 0.1]
(a few of length 0), through the torus, sphere (closed form and marched) and blob scenes of
the workloads.  Both sides decide in FP64 with the same algorithm, so hit and material must
match exactly; t, normal and albedo (FP32 outputs) within 1e-6."""
import numpy as np
import pytest

import nif_synth as S
from _helpers import dev_f32, say

pytestmark = pytest.mark.gpu


def _chords(n, seed):
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(0.0, 1.0, (n, 3))
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    r = rng.uniform(0.0, 0.1, n)
    r[:16] = 0.0
    x1 = x0 + r[:, None] * u
    return x0.astype(np.float32), x1.astype(np.float32)


@pytest.mark.parametrize("workload,force_march", [("torus16", False), ("spheres64", False), ("spheres64", True),
                                                  ("blobs128", False)])
def test_labels_match_oracle(orc, workload, force_march):
    import torch

    import paper_2604_24666_amd as P
    w = S.workload(workload)
    sp = S.scene_params(w.scene_kind, w.seed)
    x0, x1 = _chords(20000, 31)
    say(f"labels {workload} force_march={force_march}")
    got = P.label(w.scene_kind, sp, dev_f32(x0.T), dev_f32(x1.T), force_march=force_march)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in got.items()}
    hit, t, nr, al, mt = orc.label(w.scene_kind, sp, x0.astype(np.float64), x1.astype(np.float64), force_march=force_march)
    h = hit == 1
    say(f"  hits {int(h.sum())} of {len(hit)}  (starting inside: {int((h & (t == 0)).sum())})")
    assert 0.05 < h.mean() < 0.95
    assert np.array_equal(g["hit"], hit)
    assert np.array_equal(g["material"][h], mt[h])
    dt = np.abs(g["t"] - t)
    dn = np.abs(g["normal"].T - nr).max(1)
    da = np.abs(g["albedo"].T - al).max(1)
    say(f"  max |dt| {dt.max():.2e}  max |dn| {dn.max():.2e}  max |da| {da.max():.2e}")
    assert dt.max() <= 1e-6 and dn.max() <= 1e-6 and da.max() <= 1e-6
    assert np.all(g["t"][~h] == 0) and np.all(g["normal"][:, ~h] == 0) and np.all(g["material"][~h] == 0)


def test_labels_of_no_segments_and_bad_arguments():
    import torch

    import paper_2604_24666_amd as P
    w = S.workload("torus16")
    sp = S.scene_params(w.scene_kind, w.seed)
    e = torch.empty((3, 0), device="cuda")
    P.nif_label(w.scene_kind, sp, e, e, 0)
    with pytest.raises(P.NifError):
        P.nif_label(5, sp, e, e, 0)
    with pytest.raises(P.NifError):
        P.nif_label(w.scene_kind, sp[:3], e, e, 0)
