"""The C-ABI library loads and exports every symbol include/nif.h declares, and its host-side
argument validation rejects bad input before touching the device (no compute calls here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "nif.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nif_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def P():
    import paper_2604_24666_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_2604_24666_amd import build
        build.build()
    return P


def test_every_declared_symbol_is_exported(P):
    L = C.CDLL(P.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings(P):
    L = P.lib()
    assert L.nif_status_string(0) == b"ok"
    assert L.nif_status_string(1) == b"invalid argument"
    assert L.nif_version() >= 1


def _desc(P, **kw):
    a = dict(levels=8, log2_table=14, feat_dim=2, table_dtype=0, res=[16, 24, 35, 53, 78, 116, 172, 256],
             pe_freqs=6, hidden_width=64, hidden_layers=2, n_materials=1)
    a.update(kw)
    return P.model_desc(**a)


def test_model_sizes_match_the_canonical_layout(P):
    nt, nm = P.nif_model_sizes(_desc(P))
    assert nt == 8 * 2 ** 14 * 2
    assert nm == (416 * 64 + 64) + (64 * 64 + 64) + (64 * 9 + 9)
    nt, nm = P.nif_model_sizes(_desc(P, levels=16, log2_table=19, res=[16] * 16, hidden_width=128,
                                     hidden_layers=4, n_materials=4))
    assert nm == (832 * 128 + 128) + 3 * (128 * 128 + 128) + (128 * 12 + 12)


def test_three_feature_entries_size_the_paper_configuration(P):
    """Two levels of three features (the paper's deformation comparison): 2 T 3 table floats,
    first layer 2 x 7 x 2 x 3 = 84 wide."""
    nt, nm = P.nif_model_sizes(_desc(P, levels=2, feat_dim=3, log2_table=19, res=[64, 128], pe_freqs=3,
                                     hidden_width=64, hidden_layers=3, n_materials=4))
    assert nt == 2 * 2 ** 19 * 3
    assert nm == (84 * 64 + 64) + 2 * (64 * 64 + 64) + (64 * 12 + 12)


@pytest.mark.parametrize("kw,code", [(dict(feat_dim=4), 1), (dict(feat_dim=3, levels=3, res=[16] * 3), 1),
                                     (dict(feat_dim=3, concat_encoding=1), 1), (dict(levels=6), 1),
                                     (dict(levels=2, res=[16, 32]), 1), (dict(log2_table=30), 1),
                                     (dict(hidden_width=48), 2), (dict(hidden_layers=0), 1),
                                     (dict(n_materials=0), 1), (dict(table_dtype=7), 1),
                                     (dict(res=[0] * 8), 1), (dict(pe_freqs=-1), 1), (dict(dist_head=2), 1),
                                     (dict(per_sample_tables=2), 1)])
def test_bad_model_descriptions_are_rejected(P, kw, code):
    L = P.lib()
    d = _desc(P, **kw)
    rc = L.nif_model_sizes(C.byref(d), None, None)
    assert rc == code
    assert L.nif_last_error()


def test_bad_grid_arguments_are_rejected_on_the_host(P):
    L = P.lib()
    poses = (P.Pose * 1)(P.Pose(1, 0.5))
    h = C.c_void_p()
    assert L.nif_build_grid(None, 16, poses, 1, 0, C.byref(h), None) == 1           # null occupancy
    dummy = C.c_void_p(1)
    assert L.nif_build_grid(dummy, 0, poses, 1, 0, C.byref(h), None) == 1           # N = 0
    bad = (P.Pose * 1)(P.Pose(9, 0.5))
    assert L.nif_build_grid(dummy, 16, bad, 1, 0, C.byref(h), None) == 1            # unknown kind
    bad = (P.Pose * 1)(P.Pose(3, 1.5))
    assert L.nif_build_grid(dummy, 16, bad, 1, 0, C.byref(h), None) == 1            # strength > 1
    assert L.nif_build_grid(dummy, 16, poses, 0, 0, C.byref(h), None) == 1          # no poses


def test_bad_query_arguments_are_rejected_on_the_host(P):
    L = P.lib()
    hits = P.Hits()
    rays = P.Rays()
    g = C.c_void_p(1)
    assert L.nif_query(None, None, C.byref(rays), 4, C.byref(hits), 0, 0, None, None) == 1   # null grid
    assert L.nif_query(None, g, C.byref(rays), 4, C.byref(hits), 0, 0, None, None) == 1      # null ray arrays
    assert L.nif_query(None, g, C.byref(rays), -1, C.byref(hits), 0, 0, None, None) == 1     # negative count
    assert L.nif_query(None, g, C.byref(rays), 0, C.byref(hits), 0, 7, None, None) == 1      # bad precision
    assert L.nif_query(None, g, C.byref(rays), 0, C.byref(hits), 0x40, 0, None, None) == 1   # unknown flag
    assert L.nif_query(None, g, C.byref(rays), 0, C.byref(hits), 0, 0, None, None) == 1      # null model


def test_launch_shape_setters_and_autotuner_validate_on_the_host(P):
    L = P.lib()
    assert L.nif_set_query_blocks_per_cu(0) == 1 and L.nif_set_query_blocks_per_cu(33) == 1
    assert L.nif_set_query_rays_per_wave(32) == 1 and L.nif_set_query_rays_per_wave(-1) == 1
    assert L.nif_set_query_rays_per_wave(0) == 0 and L.nif_set_query_blocks_per_cu(12) == 0
    best = (C.c_int32 * 2)()
    rays = P.Rays()
    hits = P.Hits()
    g = C.c_void_p(1)
    assert L.nif_autotune_query(None, g, C.byref(rays), 4, C.byref(hits), 0, 2, best, None, None) == 1   # null model
    assert L.nif_autotune_query(g, None, C.byref(rays), 4, C.byref(hits), 0, 2, best, None, None) == 1   # null grid
    assert L.nif_last_error()


def test_train_step_configuration_is_validated_on_the_host(P):
    L = P.lib()
    fake = C.c_void_p(1)
    batch = P.Batch(*([1] * 7))
    good = dict(lr_table=1e-2, lr_mlp=1e-3, lr_s=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, precision=0,
                loss_scale_init=0.0, fixed_task_weights=0, store_encoding=0, loss_scale_growth_interval=0)
    for k, v in [("store_encoding", 2), ("store_encoding", -1), ("fixed_task_weights", 3), ("precision", 3),
                 ("beta1", 1.0), ("eps", 0.0), ("loss_scale_growth_interval", -1), ("loss_scale_init", -1.0),
                 ("loss_scale_init", float("inf"))]:
        cfg = P.TrainCfg(**{**good, k: v})
        assert L.nif_train_step(fake, C.byref(batch), 4, C.byref(cfg), fake, None) == 1, k
    assert L.nif_train_step(fake, C.byref(batch), 0, C.byref(P.TrainCfg(**good)), fake, None) == 1   # empty batch
    assert L.nif_model_reserve_encoding(None) == 1


def test_binding_structures_match_the_header_layout(P, tmp_path):
    """Every struct the Python binding passes through the C ABI has the header's size and
    field offsets (a C program compiled from include/nif.h prints them)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    pairs = {"nif_model_desc": P.ModelDesc, "nif_pose": P.Pose, "nif_rays": P.Rays, "nif_segments": P.Segments,
             "nif_hits": P.Hits, "nif_batch": P.Batch, "nif_train_cfg": P.TrainCfg}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "nif.h"', 'int main(void) {']
    for cname, py in pairs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                         text=True).stdout.splitlines())
    for cname, py in pairs.items():
        assert int(got[f"{cname} size"]) == C.sizeof(py), cname
        for f in py._fields_:
            assert int(got[f"{cname} {f[0]}"]) == getattr(py, f[0]).offset, (cname, f[0])


def test_loss_arguments_are_validated_on_the_host(P):
    L = P.lib()
    fake = C.c_void_p(1)
    labels = P.Batch(*([1] * 7))
    assert L.nif_loss(None, fake, 4, C.byref(labels), fake, 0, fake, None, None, None) == 1   # null model
    assert L.nif_loss(fake, None, 4, C.byref(labels), fake, 0, fake, None, None, None) == 1   # null heads
    assert L.nif_loss(fake, fake, 0, C.byref(labels), fake, 0, fake, None, None, None) == 1   # empty batch
    assert L.nif_loss(fake, fake, 4, C.byref(labels), fake, 2, fake, None, None, None) == 1   # bad switch
    assert L.nif_loss(fake, fake, 4, C.byref(labels), None, 0, fake, None, None, None) == 1   # null s
    no_t = P.Batch(1, 1, 1, None, 1, 1, 1)
    assert L.nif_loss(fake, fake, 4, C.byref(no_t), fake, 0, fake, None, None, None) == 1     # missing labels


def test_label_noalloc_validates_on_the_host(P):
    """The allocation-free labelling call rejects, before touching the device, a parameter
    vector longer than its fixed array, and the same malformed inputs as nif_label."""
    L = P.lib()
    fake = C.c_void_p(1)
    n_max = 4104
    assert P.LABEL_NOALLOC_MAX_PARAMS == n_max
    ok = np.zeros(1 + 8 * 4)
    ok[0] = 4
    big = np.zeros(1 + 8 * 513)
    big[0] = 513
    args = lambda p, n: (1, p.ctypes.data_as(C.c_void_p), len(p), 0, fake, fake, n) + (None,) * 5 + (None,)
    assert L.nif_label_noalloc(*args(big, 4)) == 1 and b"NIF_LABEL_NOALLOC_MAX_PARAMS" in L.nif_last_error()
    assert L.nif_label_noalloc(*args(ok[:9], 4)) == 1           # parameter count does not match n
    assert L.nif_label_noalloc(*args(ok, -1)) == 1              # negative count
    assert L.nif_label_noalloc(3, ok.ctypes.data_as(C.c_void_p), len(ok), 0, fake, fake, 4, *([None] * 5), None) == 1
