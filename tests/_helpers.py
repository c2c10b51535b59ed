"""Shared set-up for the GPU parity tests: the same seeded inputs go to the oracle (FP64,
widened from the FP32/FP16 values the GPU uses) and to libnif through its C ABI."""
import sys

import numpy as np

import nif_synth as S


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_f32(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def offsets(counts):
    import torch
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return torch.as_tensor(off).cuda()


def model_params(m, seed, scale_tables=1.0):
    """(FP32 tables, FP32 MLP, FP64 tables as the kernels see them)."""
    import oracle
    tab = S.init_tables(m, seed) * np.float32(scale_tables)
    prm = S.init_mlp(m, seed)
    tab_seen = oracle.round_f16(tab) if m.table_dtype == S.TABLE_F16 else tab.astype(np.float64)
    return tab, prm, tab_seen


def quantized_mlp(prm, precision):
    import oracle
    if precision == S.PREC_BF16:
        return oracle.round_bf16(prm)
    if precision == S.PREC_FP16:
        return oracle.round_f16(prm)
    return prm.astype(np.float64)


def rel_err(gpu, ref):
    """|gpu - ref| / max(|ref|, 1e-3 RMS of that head over the batch), per element."""
    rms = np.sqrt(np.mean(ref ** 2, axis=0, keepdims=True)) + 1e-300
    return np.abs(gpu - ref) / np.maximum(np.abs(ref), 1e-3 * rms)
