"""The allocation-free labelling entry point against nif_label, through the C ABI.

nif_label_noalloc stages the scene parameters in the library's fixed per-device array
instead of a buffer allocated per call; its outputs must equal nif_label's bit for bit.
Two calls in a row on the same stream, the second with a smaller input (fewer segments and a
shorter parameter vector), check that the array's leftover contents from the first call do
not leak into the second.  Parameter vectors beyond the array's capacity are rejected."""
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
    x1 = x0 + rng.uniform(0.0, 0.1, n)[:, None] * u
    return dev_f32(x0.T), dev_f32(x1.T)


def _label(P, fn, kind, sp, x0, x1):
    import torch
    n = x0.shape[1]
    out = dict(hit=torch.full((n,), 7, dtype=torch.uint8, device="cuda"), t=torch.full((n,), -1.0, device="cuda"),
               normal=torch.full((3, n), -1.0, device="cuda"), albedo=torch.full((3, n), -1.0, device="cuda"),
               material=torch.full((n,), -7, dtype=torch.int32, device="cuda"))
    fn(kind, sp, x0, x1, n, out["hit"], out["t"], out["normal"], out["albedo"], out["material"])
    return out


def test_label_noalloc_matches_label_on_two_calls():
    import torch

    import paper_2604_24666_amd as P
    cases = [("blobs128", 20000, 51), ("spheres64", 3001, 52)]     # second call: fewer segments and parameters
    sizes = []
    for workload, n, seed in cases:
        w = S.workload(workload)
        sp = S.scene_params(w.scene_kind, w.seed)
        sizes.append(len(sp))
        x0, x1 = _chords(n, seed)
        say(f"label_noalloc {workload}: {n} segments, {len(sp)} scene parameters")
        got = _label(P, P.nif_label_noalloc, w.scene_kind, sp, x0, x1)
        ref = _label(P, P.nif_label, w.scene_kind, sp, x0, x1)
        torch.cuda.synchronize()
        hits = int(ref["hit"].sum().item())
        assert 0 < hits < n
        for k in ref:
            assert torch.equal(got[k], ref[k]), f"{workload}: {k} differs from nif_label"
        say(f"  identical to nif_label ({hits} hits)")
    assert sizes[1] < sizes[0]


def test_label_noalloc_rejects_parameters_beyond_its_array():
    import torch

    import paper_2604_24666_amd as P
    n_max = P.LABEL_NOALLOC_MAX_PARAMS
    n_spheres = (n_max - 1) // 8 + 1                          # 1 + 8 n > n_max
    sp = np.zeros(1 + 8 * n_spheres)
    sp[0] = n_spheres
    x0, x1 = _chords(16, 3)
    out = torch.empty(16, device="cuda")
    with pytest.raises(P.NifError, match="NIF_LABEL_NOALLOC_MAX_PARAMS"):
        P.nif_label_noalloc(S.SCENE_SPHERES, sp, x0, x1, 16, None, out)
