"""Multi-stage scan (Section 4.3) on the device vs the oracle's multi-stage
estimator, through the C ABI.

Both sides read the same records (encoded and packed by the oracle).  The
device bounds each pair in FP32 from matrix-core partial sums, the oracle in
FP64, so a pair whose bound lies within the FP32 tolerance of its threshold
may close one stage apart.  What is unique is checked exactly: a device stage
must lie between the oracle's stages at tau - tol and tau + tol (stages only
grow with the threshold), at least 99.9 % of the stages must be identical,
and where the stages agree the values agree within the scan's 2e-5 of scale.
"""
import numpy as np
import pytest

import oracle
import synth
import paper_2509_12086_amd as saq
from gpu_util import cuda, oracle_records, say, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 2e-5        # the scan's FP32 tolerance, relative to ||o||^2 + ||q - c||^2


def _kept_axes(plan, V, lam):
    """The PCA axes (rows) and variances behind the plan's kept dims."""
    idx, pos = [], 0
    for w, b in zip(plan.widths, plan.bits):
        if b > 0:
            idx.extend(range(pos, pos + w))
        pos += w
    idx = np.asarray(idx)
    return V[:, idx].T, lam[idx]


@pytest.fixture(scope="module")
def gauss():
    """cfg1's Gaussian spectrum: a plan from the oracle's PCA basis (with the
    plan's own per-segment rotations), records from the oracle."""
    ds = synth.cfg1(50_000)
    X = ds.rows(0, 8000)
    mean, _, lam, V = oracle.pca(X)
    plan = saq.Plan.from_basis(mean, V, lam, saq.PlanParams(bits_per_dim=4.0)).upload(0)
    P, lk = _kept_axes(plan, V, lam)
    Xs = ds.rows(8000, 8000 + 5003)           # ragged: 39 full 128-record tiles + 11
    packed, fac, codes = oracle_records(plan, Xs, 4)
    return dict(ds=ds, plan=plan, P=P, lam=lk, packed=packed, fac=fac, codes=codes)


def _oracle_ms(S, Q, m, tau):
    plan = S["plan"]
    M, c, _ = plan.arrays()
    fac = S["fac"]
    return oracle.estimate_multistage(Q, M, c, plan.kept_widths, plan.kept_bits, S["codes"],
                                      fac[:, :-1].astype(np.float64), fac[:, -1].astype(np.float64),
                                      S["P"], S["lam"], m, tau)


def _device_ms(S, Q, m, tau):
    d2, st = saq.estimate_multistage(S["plan"], to_dev(Q), to_dev(S["packed"]), to_dev(S["fac"]),
                                     to_dev(np.asarray(tau, np.float32)), m)
    torch.cuda.synchronize()
    return d2.cpu().numpy(), st.cpu().numpy().astype(np.int32)


def _scale(S, Q):
    _, c, _ = S["plan"].arrays()
    return S["fac"][:, -1].astype(np.float64)[None, :] + ((Q.astype(np.float64) - c) ** 2).sum(1)[:, None]


def _check(S, Q, m, tau, label):
    say(f"multi-stage {label}: nq={len(Q)} n={len(S['packed'])} m={m}")
    d2, st = _device_ms(S, Q, m, tau)
    ref, rst, _ = _oracle_ms(S, Q, m, tau)
    scale = _scale(S, Q)
    tol = TOL * scale.max(axis=1)                     # per query
    _, lo, _ = _oracle_ms(S, Q, m, tau - tol)
    _, hi, _ = _oracle_ms(S, Q, m, tau + tol)
    assert np.all((st >= lo) & (st <= hi)), label
    same = st == rst
    say(f"  stages identical {same.mean():.6f}; histogram {np.bincount(st.ravel())}")
    assert same.mean() >= 0.999, label
    err = np.abs(d2 - ref)[same] / scale[same]
    assert err.max() < TOL, (label, err.max())
    return st, rst


def test_multistage_matches_oracle(gauss):
    S = gauss
    rng = np.random.default_rng(5)
    for nq, m in ((70, 4.0), (64, 2.0), (1, 4.0), (130, 1.0)):
        Q = S["ds"].queries(nq)
        plain = oracle.estimate(Q, *S["plan"].arrays()[:2], S["plan"].kept_widths,
                                S["plan"].kept_bits, S["codes"],
                                S["fac"][:, :-1].astype(np.float64),
                                S["fac"][:, -1].astype(np.float64))
        k = min(10, plain.shape[1])
        tau = np.sort(plain, axis=1)[:, k - 1] * rng.uniform(0.9, 1.1, nq)
        st, _ = _check(S, Q, m, tau, f"nq={nq}")
        if m >= 2.0:
            assert (st < len(S["plan"].kept_widths)).mean() > 0.5   # pruning happens


def test_multistage_no_threshold_is_the_plain_scan(gauss):
    """With tau = +inf nothing closes, and every estimate equals the plain
    scan's within the FP32 tolerance.  This plan's kept widths are multiples
    of 16, so the plain scan packs its k-steps across segment boundaries
    while the multi-stage scan steps segment by segment: the same products,
    summed in another order.  Tiles with few pairs (the last query tile
    here: 2 queries x 128 records) take the sparse finish from the first
    segment."""
    S = gauss
    Q = S["ds"].queries(66)
    d2, st = _device_ms(S, Q, 4.0, np.full(66, np.inf))
    assert np.all(st == len(S["plan"].kept_widths))
    plain = saq.estimate_dist(S["plan"], to_dev(Q), to_dev(S["packed"]), to_dev(S["fac"]))
    torch.cuda.synchronize()
    plain = plain.cpu().numpy()
    scale = _scale(S, Q)
    assert np.max(np.abs(d2 - plain) / scale) < TOL
    _check(S, Q, 4.0, np.full(66, np.inf), "tau=+inf")


def test_multistage_no_threshold_matches_the_plain_scan_on_ragged_segments():
    """Kept widths 13, 37, 70, 9, 51 (none a multiple of 16; the plain scan
    steps segment by segment with the records as the second operand and a
    9-bit segment whose codes take two bf16 terms): with tau = +inf the
    multi-stage scan reads every segment and agrees with the plain scan, and
    both with the oracle's estimator, within the FP32 accumulation
    tolerance."""
    rng = np.random.default_rng(41)
    widths, bits = [13, 37, 70, 9, 51], [9, 6, 4, 3, 2]
    D = sum(widths)
    sd = np.concatenate([np.full(w, v) for w, v in zip(widths, (3.0, 2.0, 1.2, 0.9, 0.6))])
    plan = saq.Plan.from_parts(widths, bits, np.eye(D, dtype=np.float32), np.zeros(D, np.float32),
                               variances=sd ** 2).upload(0)
    X = (rng.standard_normal((700, D)) * sd).astype(np.float32)
    packed, fac, codes = oracle_records(plan, X, 4)
    S = dict(plan=plan, P=np.eye(D), lam=sd ** 2, packed=packed, fac=fac, codes=codes)
    Q = (rng.standard_normal((64, D)) * sd).astype(np.float32)
    d2, st = _device_ms(S, Q, 4.0, np.full(64, np.inf))
    assert np.all(st == len(plan.kept_widths))
    plain = saq.estimate_dist(plan, to_dev(Q), to_dev(packed), to_dev(fac))
    torch.cuda.synchronize()
    plain = plain.cpu().numpy()
    f64 = fac.astype(np.float64)
    M, c, _ = plan.arrays()
    ref = oracle.estimate(Q, M, c, plan.kept_widths, plan.kept_bits, codes, f64[:, :-1], f64[:, -1])
    sc = _scale(S, Q)
    assert np.max(np.abs(d2 - plain) / sc) < TOL
    assert np.max(np.abs(plain - ref) / sc) < TOL
    assert np.max(np.abs(d2 - ref) / sc) < TOL


def test_multistage_everything_closes_at_stage_zero(gauss):
    S = gauss
    Q = S["ds"].queries(40)
    d2, st = _device_ms(S, Q, 4.0, np.full(40, -np.inf))
    assert np.all(st == 0)
    ref, rst, _ = _oracle_ms(S, Q, 4.0, np.full(40, -np.inf))
    assert np.max(np.abs(d2 - ref) / _scale(S, Q)) < TOL


def test_multistage_wide_bits_from_parts():
    """1- to 16-bit segments with widths that are not multiples of 32, on a
    plan given explicitly with per-dim variances (no rotation: M's rows are
    the axes)."""
    rng = np.random.default_rng(11)
    D = 160
    widths, bits = [16, 48, 32, 16, 16, 32], [16, 9, 5, 2, 1, 0]
    sd = np.repeat([4.0, 2.0, 1.0, 0.5, 0.3, 0.1], widths)
    Mw = np.eye(D, dtype=np.float32)[:128]
    plan = saq.Plan.from_parts(widths, bits, Mw, np.zeros(D, np.float32),
                               variances=sd ** 2).upload(0)
    X = (rng.standard_normal((1500, D)) * sd).astype(np.float32)
    packed, fac, codes = oracle_records(plan, X, 4)
    S = dict(plan=plan, P=np.eye(D)[:128], lam=(sd ** 2)[:128], packed=packed, fac=fac,
             codes=codes)
    Q = (rng.standard_normal((67, D)) * sd).astype(np.float32)
    M, c, _ = plan.arrays()
    plain = oracle.estimate(Q, M, c, plan.kept_widths, plan.kept_bits, codes,
                            fac[:, :-1].astype(np.float64), fac[:, -1].astype(np.float64))
    tau = np.sort(plain, axis=1)[:, 4]
    _check(S, Q, 3.0, tau, "wide bits")


def test_multistage_ragged_widths():
    """Segment widths that are not multiples of 8 or 32 (odd plane byte
    counts, so unaligned plane offsets and ragged last chunks on both the
    matrix-core and the one-group-per-pair paths), 1- to 12-bit codes, a
    ragged record count, and query counts that put a tile on either path
    from the first segment (1, 3 and 70 queries)."""
    rng = np.random.default_rng(23)
    widths, bits = [13, 37, 70, 9, 51, 3, 20], [12, 9, 5, 7, 3, 1, 0]
    D = sum(widths)
    kept = sum(w for w, b in zip(widths, bits) if b > 0)
    sd = np.concatenate([np.full(w, v) for w, v in zip(widths, (3.0, 2.0, 1.2, 0.9, 0.6, 0.4, 0.2))])
    Mw = np.eye(D, dtype=np.float32)[:kept]
    plan = saq.Plan.from_parts(widths, bits, Mw, np.zeros(D, np.float32), variances=sd ** 2).upload(0)
    assert plan.code_bytes % 4 != 0
    X = (rng.standard_normal((1337, D)) * sd).astype(np.float32)
    packed, fac, codes = oracle_records(plan, X, 4)
    S = dict(plan=plan, P=np.eye(D)[:kept], lam=(sd ** 2)[:kept], packed=packed, fac=fac,
             codes=codes)
    M, c, _ = plan.arrays()
    for nq, m in ((1, 4.0), (3, 2.0), (70, 4.0)):
        Q = (rng.standard_normal((nq, D)) * sd).astype(np.float32)
        plain = oracle.estimate(Q, M, c, plan.kept_widths, plan.kept_bits, codes,
                                fac[:, :-1].astype(np.float64), fac[:, -1].astype(np.float64))
        tau = np.sort(plain, axis=1)[:, 9]
        st, _ = _check(S, Q, m, tau, f"ragged widths nq={nq}")
        assert (st < len(plan.kept_widths)).mean() > 0.3


def test_multistage_narrow_segments():
    """A plan whose kept segments are all at most 32 dims (one 32-dim chunk
    each) runs the sparse finish with one lane per open pair: ragged widths
    below 32, 1- to 11-bit codes, 1, 3 and 70 queries."""
    rng = np.random.default_rng(31)
    widths, bits = [32, 7, 24, 13, 31, 16, 5], [11, 8, 6, 4, 3, 2, 0]
    D = sum(widths)
    kept = sum(w for w, b in zip(widths, bits) if b > 0)
    sd = np.concatenate([np.full(w, v) for w, v in zip(widths, (3.0, 2.2, 1.5, 1.0, 0.7, 0.5, 0.2))])
    Mw = np.eye(D, dtype=np.float32)[:kept]
    plan = saq.Plan.from_parts(widths, bits, Mw, np.zeros(D, np.float32), variances=sd ** 2).upload(0)
    assert max(plan.kept_widths) <= 32
    X = (rng.standard_normal((2003, D)) * sd).astype(np.float32)
    packed, fac, codes = oracle_records(plan, X, 4)
    S = dict(plan=plan, P=np.eye(D)[:kept], lam=(sd ** 2)[:kept], packed=packed, fac=fac,
             codes=codes)
    M, c, _ = plan.arrays()
    for nq, m in ((1, 4.0), (3, 2.0), (70, 4.0)):
        Q = (rng.standard_normal((nq, D)) * sd).astype(np.float32)
        plain = oracle.estimate(Q, M, c, plan.kept_widths, plan.kept_bits, codes,
                                fac[:, :-1].astype(np.float64), fac[:, -1].astype(np.float64))
        tau = np.sort(plain, axis=1)[:, 9]
        st, _ = _check(S, Q, m, tau, f"narrow segments nq={nq}")
        assert (st < len(plan.kept_widths)).mean() > 0.3


def test_multistage_argument_errors(gauss):
    S = gauss
    plan = S["plan"]
    Q = to_dev(S["ds"].queries(4))
    codes, fac = to_dev(S["packed"][:10]), to_dev(S["fac"][:10])
    tau = torch.zeros(4, dtype=torch.float32, device=cuda())
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.estimate_multistage(plan, Q, codes, fac, tau, -1.0)
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.estimate_multistage(plan, Q, codes, fac, tau, float("nan"))
    with pytest.raises(ValueError):
        saq.estimate_multistage(plan, Q, codes, fac, tau[:3], 4.0)
    D = 32
    novar = saq.Plan.from_parts([16, 16], [4, 2], np.eye(D, dtype=np.float32),
                                np.zeros(D, np.float32)).upload(0)
    q2 = to_dev(np.zeros((4, D), np.float32))
    c2 = torch.zeros((10, novar.code_bytes), dtype=torch.uint8, device=cuda())
    f2 = torch.zeros((10, novar.n_factors), dtype=torch.float32, device=cuda())
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.estimate_multistage(novar, q2, c2, f2, tau, 4.0)
    # empty inputs launch nothing
    empty_q = torch.empty((0, plan.D), dtype=torch.float32, device=cuda())
    d2, st = saq.estimate_multistage(plan, empty_q, codes, fac,
                                     torch.empty(0, dtype=torch.float32, device=cuda()), 4.0)
    assert d2.shape == (0, 10) and st.shape == (0, 10)


@pytest.mark.parametrize("which", [2, 0])
def test_full_size_scans_sampled(which):
    """Scans in the benchmark's launch shape: 64 queries against 1,000,000
    records at D = 768 and D = 128 (the scan leg's dataset shapes; at D = 128
    the plain scan packs its k-steps and the sparse finish takes one lane per
    pair).  The records are 16,384 oracle-encoded records repeated to 1M
    rows, so every input is the oracle's; every scanned row equals its base
    record's estimate.  Checked on a sample of 4,000 rows spread over the
    whole range: the plain scan, the 2-bit prefix scan and the multi-stage
    scan (m = 4)."""
    ds = synth.cfg5(which, 1_000_000)
    base_n, n, nq = 16_384, 1_000_000, 64
    Xb = ds.rows(0, base_n)
    mean, _, lam, V = oracle.pca(Xb)
    plan = saq.Plan.from_basis(mean, V, lam, saq.PlanParams(bits_per_dim=4.0)).upload(0)
    P, lk = _kept_axes(plan, V, lam)
    packed, fac, codes = oracle_records(plan, Xb, 4)
    reps = np.arange(n) % base_n
    dev_packed = to_dev(packed)[torch.from_numpy(reps).to(cuda())].contiguous()
    dev_fac = to_dev(fac)[torch.from_numpy(reps).to(cuda())].contiguous()
    Q = ds.queries(nq)
    M, c, _ = plan.arrays()
    f64 = fac.astype(np.float64)
    plain = oracle.estimate(Q, M, c, plan.kept_widths, plan.kept_bits, codes, f64[:, :-1], f64[:, -1])
    pre2 = oracle.estimate(Q, M, c, plan.kept_widths, plan.kept_bits, codes, f64[:, :-1], f64[:, -1],
                           prefix_bits=2)
    scale = f64[:, -1][None, :] + ((Q.astype(np.float64) - c) ** 2).sum(1)[:, None]
    sample = np.random.default_rng(12).choice(n, 4000, replace=False)
    sb = reps[sample]
    say(f"full-size scans: 64 queries x 1M records, D={ds.d}, kept widths {plan.kept_widths}")
    for label, kw, want in (("plain", {}, plain), ("prefix 2", {"prefix_bits": 2}, pre2)):
        d2 = saq.estimate_dist(plan, to_dev(Q), dev_packed, dev_fac, **kw)
        torch.cuda.synchronize()
        got = d2[:, torch.from_numpy(sample).to(cuda())].cpu().numpy()
        err = np.max(np.abs(got - want[:, sb]) / scale[:, sb])
        say(f"  {label}: max err {err:.2e}")
        assert err < TOL, label
    tau = np.sort(plain, axis=1)[:, 9]
    md, ms = saq.estimate_multistage(plan, to_dev(Q), dev_packed, dev_fac,
                                     to_dev(tau.astype(np.float32)), 4.0)
    torch.cuda.synchronize()
    idx = torch.from_numpy(sample).to(cuda())
    md = md[:, idx].cpu().numpy()
    ms = ms[:, idx].cpu().numpy().astype(np.int32)
    S = dict(plan=plan, P=P, lam=lk, packed=packed, fac=fac, codes=codes)
    ref, rst, _ = _oracle_ms(S, Q, 4.0, tau)
    tol = TOL * scale.max(axis=1)
    _, lo, _ = _oracle_ms(S, Q, 4.0, tau - tol)
    _, hi, _ = _oracle_ms(S, Q, 4.0, tau + tol)
    assert np.all((ms >= lo[:, sb]) & (ms <= hi[:, sb]))
    same = ms == rst[:, sb]
    say(f"  multi-stage: stages identical {same.mean():.6f}")
    assert same.mean() >= 0.999
    assert np.max(np.abs(md - ref[:, sb])[same] / scale[:, sb][same]) < TOL
