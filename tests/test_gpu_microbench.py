"""The device-ceiling microbenchmarks behind the measurement (nif_microbench): each kind runs,
and its rate lies between a loose floor and the published peak of the unit it measures (a rate
above the peak would mean the work count or the timing is wrong)."""
import pytest

from _helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2604_24666_amd as P
    return P


@pytest.mark.parametrize("kind,n_bytes,n_ops,lo,hi", [
    (0, 1 << 30, 1, 1e12, 8.0e12 * 1.05),          # streaming HBM reads: bytes/s, published 8 TB/s
    (1, 32 << 20, 1 << 26, 1e10, 1e14),            # random 4-byte gathers, 32 MiB table
    (2, 32 << 20, 1 << 26, 1e10, 1e14),            # random 8-byte gathers
    (3, 0, 1 << 24, 1e12, 157.3e12 * 1.05),        # FP32 MFMA: FLOP/s, published 157.3 TFLOP/s
    (4, 0, 1 << 24, 1e13, 2.5e15 * 1.05),          # BF16 MFMA: FLOP/s, published 2.5 PFLOP/s dense
], ids=["hbm_read", "gather4", "gather8", "mfma_f32", "mfma_bf16"])
def test_microbenchmark_rates_are_physical(P, kind, n_bytes, n_ops, lo, hi):
    rate, ms = P.nif_microbench(kind, n_bytes, n_ops, 3)
    say(f"microbench kind {kind}: {rate:.3e} per s, {ms:.3f} ms per launch")
    assert ms > 0 and lo <= rate <= hi


def test_microbenchmark_rejects_bad_arguments(P):
    with pytest.raises(P.NifError):
        P.nif_microbench(9, 1 << 20, 1)
    with pytest.raises(P.NifError):
        P.nif_microbench(1, 1000, 1)                 # below 4096 bytes / not a multiple of 16
    with pytest.raises(P.NifError):
        P.nif_microbench(3, 0, 0)
