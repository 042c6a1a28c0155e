"""saq_encode_noalloc (the encode for callers that cannot allocate) against
saq_encode, through the C ABI: records and factors bit-identical on two calls
in a row, the second smaller, so stale scratch contents from the first call
cannot leak into the second; sizes past the fixed scratch are refused."""
import ctypes

import numpy as np
import pytest

import synth
import paper_2509_12086_amd as saq
from gpu_util import cuda, say, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _raw_noalloc(plan, X, rounds, stream):
    """One call through the C ABI; returns (status, codes, factors)."""
    n = X.shape[0]
    codes = torch.full((n, plan.code_bytes), 0xA5, dtype=torch.uint8, device=X.device)
    fac = torch.full((n, plan.n_factors), float("nan"), dtype=torch.float32, device=X.device)
    st = saq.lib().saq_encode_noalloc(plan._h, ctypes.c_void_p(X.data_ptr()), n, rounds,
                                      ctypes.c_void_p(codes.data_ptr()),
                                      ctypes.c_void_p(fac.data_ptr()),
                                      ctypes.c_void_p(stream.cuda_stream))
    return st, codes, fac


def _max_rows(plan):
    lo, hi = 0, 1 << 24
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if plan.encode_workspace_bytes(mid) <= saq.NOALLOC_SCRATCH_BYTES:
            lo = mid
        else:
            hi = mid - 1
    return lo


@pytest.mark.parametrize("which", ["cfg1 D=128", "cfg2 D=960"])
def test_noalloc_matches_encode_on_two_calls(which):
    if which.startswith("cfg1"):
        ds = synth.cfg1()
        X = ds.rows()
        plan = saq.Plan.fit(X, saq.PlanParams(bits_per_dim=4.0, fit_sample=0)).upload(0)
        sizes = [X.shape[0], 1000]
    else:
        ds = synth.cfg2(24_000)
        X = ds.rows()
        plan = saq.Plan.fit(X, saq.PlanParams(bits_per_dim=4.0, fit_sample=0)).upload(0)
        m = _max_rows(plan)
        assert 16_000 < m < X.shape[0]
        sizes = [m, 4097]
    stream = torch.cuda.Stream()
    Xd = to_dev(X)
    for i, n in enumerate(sizes):
        say(f"noalloc {which}: call {i + 1}, n={n}")
        xs = Xd[i * 37: i * 37 + n]          # the second call reads other rows
        with torch.cuda.stream(stream):
            st, codes, fac = _raw_noalloc(plan, xs, 4, stream)
        assert st == 0, saq.lib().saq_last_error()
        ref_c, ref_f = saq.encode(plan, xs, 4)
        torch.cuda.synchronize()
        assert torch.equal(codes, ref_c), (which, n)
        assert torch.equal(fac, ref_f), (which, n)


def test_noalloc_refuses_sizes_past_the_scratch():
    ds = synth.cfg2(4000)
    X = ds.rows()
    plan = saq.Plan.fit(X, saq.PlanParams(bits_per_dim=4.0, fit_sample=0)).upload(0)
    m = _max_rows(plan)
    big = torch.empty((m + 1, plan.D), dtype=torch.float32, device=cuda())
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL") as ei:
        saq.encode_noalloc(plan, big, 4)
    assert str(m) in str(ei.value)
    # n = 0 is a no-op, negative rounds an argument error
    st, _, _ = _raw_noalloc(plan, big[:0], 4, torch.cuda.current_stream())
    assert st == 0
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.encode_noalloc(plan, big[:10], -1)
