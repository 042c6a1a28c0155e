"""Sizes past 2^31 elements: every device offset (input rows, the tiled
projection, records, scan outputs) is 64-bit, so results at the far end of
such a batch equal those of the same rows handled alone, and the oracle's.
About 40 GB of device memory at the peak."""
import numpy as np
import pytest

import oracle
import paper_2509_12086_amd as saq
import synth
from gpu_util import compare, cuda, gpu_encode, gpu_project, oracle_encode, oracle_records, say, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 2e-5   # FP32 accumulation, relative to ||o||^2 + ||q - c||^2 (as in the scan tests)


def test_encode_past_2_31_elements():
    """2,600,037 x 960 rows (2.5e9 input floats; the tiled projection holds
    2.25e9): the last 3,000 records equal the same rows encoded alone, byte
    for byte, and 1,500 rows sampled past 2^31 input floats (plus the first
    100) meet the parity bar against the oracle."""
    n = 2_600_037
    ds = synth.cfg2(n)
    say(f"large encode: generating {n} x {ds.d} on the device")
    X = ds.rows_torch(n, cuda())
    assert n * ds.d > 2 ** 31
    plan = saq.Plan.fit(X[:65536].cpu().numpy(), saq.PlanParams(bits_per_dim=4.0, fit_sample=0)).upload(0)
    assert (n // 64) * 64 * plan.D_kept > 2 ** 31
    codes, fac = saq.encode(plan, X, 4)
    torch.cuda.synchronize()
    tail = X[n - 3000:].cpu().numpy()
    a = gpu_encode(plan, tail, 4)
    assert np.array_equal(codes[n - 3000:].cpu().numpy(), a[0])
    assert np.array_equal(fac[n - 3000:].cpu().numpy(), a[1])
    rng = np.random.default_rng(31)
    first = 2 ** 31 // ds.d + 1
    idx = np.concatenate([np.arange(100), np.sort(rng.choice(np.arange(first, n), 1500, replace=False))])
    it = torch.from_numpy(idx).to(cuda())
    Xs = X[it].cpu().numpy()
    packed, f = codes[it].cpu().numpy(), fac[it].cpu().numpy()
    del X, codes, fac
    torch.cuda.empty_cache()
    compare(plan, packed, f, oracle_encode(plan, Xs, 4), label="past 2^31",
            dev_O=gpu_project(plan, Xs))


def test_scans_past_2_31_outputs():
    """64 queries against 34,000,000 records at D = 128 (2.18e9 outputs):
    16,384 oracle-encoded records repeated, so each scanned row equals its
    base record's estimate.  On 3,000 rows sampled from the range whose
    outputs of the last queries lie past 2^31: the plain and 2-bit prefix
    scans equal the oracle's estimates, and the multi-stage scan's stages and
    values equal those of the same scan over the base records."""
    ds = synth.cfg5(0, 16_384)
    base_n, n, nq = 16_384, 34_000_000, 64
    assert nq * n > 2 ** 31
    Xb = ds.rows(0, base_n)
    mean, _, lam, V = oracle.pca(Xb)
    plan = saq.Plan.from_basis(mean, V, lam, saq.PlanParams(bits_per_dim=4.0)).upload(0)
    packed, fac, codes = oracle_records(plan, Xb, 4)
    say(f"large scans: {nq} queries x {n} records, D={ds.d}, record {plan.code_bytes} B")
    reps = torch.arange(n, device=cuda()) % base_n
    dev_packed = to_dev(packed)[reps].contiguous()
    dev_fac = to_dev(fac)[reps].contiguous()
    del reps
    Q = ds.queries(nq)
    M, c, _ = plan.arrays()
    f64 = fac.astype(np.float64)
    plain = oracle.estimate(Q, M, c, plan.kept_widths, plan.kept_bits, codes, f64[:, :-1], f64[:, -1])
    pre2 = oracle.estimate(Q, M, c, plan.kept_widths, plan.kept_bits, codes, f64[:, :-1], f64[:, -1],
                           prefix_bits=2)
    scale = f64[:, -1][None, :] + ((Q.astype(np.float64) - c) ** 2).sum(1)[:, None]
    rng = np.random.default_rng(32)
    lo = 2 ** 31 // nq - 1000
    sample = np.concatenate([rng.choice(np.arange(lo, n), 2900, replace=False),
                             np.arange(n - 100, n)])
    sb = sample % base_n
    idx = torch.from_numpy(sample).to(cuda())
    for label, kw, want in (("plain", {}, plain), ("prefix 2", {"prefix_bits": 2}, pre2)):
        d2 = saq.estimate_dist(plan, to_dev(Q), dev_packed, dev_fac, **kw)
        torch.cuda.synchronize()
        got = d2[:, idx].cpu().numpy()
        del d2
        err = np.max(np.abs(got - want[:, sb]) / scale[:, sb])
        say(f"  {label}: max err {err:.2e}")
        assert err < TOL, label
    torch.cuda.empty_cache()
    tau = to_dev(np.sort(plain, axis=1)[:, 9].astype(np.float32))
    bd, bs = saq.estimate_multistage(plan, to_dev(Q), to_dev(packed), to_dev(fac), tau, 4.0)
    md, ms = saq.estimate_multistage(plan, to_dev(Q), dev_packed, dev_fac, tau, 4.0)
    torch.cuda.synchronize()
    md, ms = md[:, idx].cpu().numpy(), ms[:, idx].cpu().numpy()
    bd, bs = bd.cpu().numpy()[:, sb], bs.cpu().numpy()[:, sb]
    del dev_packed, dev_fac
    torch.cuda.empty_cache()
    same = ms == bs
    say(f"  multi-stage: stages identical {same.mean():.6f}")
    assert same.mean() >= 0.999
    assert np.max(np.abs(md - bd)[same] / scale[:, sb][same]) < TOL
