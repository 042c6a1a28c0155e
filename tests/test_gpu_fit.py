"""Device fit (Section 4.1) vs the oracle's PCA, through the C ABI.

The mean and covariance of the fit sample come from the device; the oracle
computes them in FP64 with numpy on the same sample rows.  Both are FP64
sums of the same products, so they agree to FP64 rounding: the mean within
1e-12 and the covariance within 1e-10 of its largest entry.  The plan fitted
from the device moments must then be the oracle's plan: the same segments
and bits (Algorithm 2 on the oracle's eigenvalues), variances within 1e-9,
and every kept segment spanning the oracle's eigenvectors (the projector
M_s^T M_s, which the per-segment rotation leaves unchanged, within the FP32
rounding of M)."""
import numpy as np
import pytest

import oracle
import synth
import paper_2509_12086_amd as saq
from gpu_util import cuda, say, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _sample(X, fit_sample):
    n = X.shape[0]
    m = fit_sample if 0 < fit_sample < n else n
    rows = np.arange(m, dtype=np.int64) if m == n else (np.arange(m, dtype=np.int64) * n) // m
    return X[rows]


CASES = [
    ("cfg1 10000 x 128", lambda: synth.cfg1(10_000).rows(), 0),
    ("D=99 exp spectrum, 1 row in 3", lambda: (
        (np.random.default_rng(9).standard_normal((30_000, 99)) * np.exp(-np.arange(99) / 30.0))
        @ synth.haar_rotation(99, 5).T + 3.0).astype(np.float32), 10_000),
    ("cfg2 shape 20000 x 960", lambda: synth.cfg2(20_000).rows(), 0),
]


@pytest.mark.parametrize("label,make,fit_sample", CASES, ids=[c[0] for c in CASES])
def test_covariance_matches_oracle(label, make, fit_sample):
    X = make()
    say(f"covariance {label} fit_sample={fit_sample}")
    mean, cov = saq.covariance(to_dev(X), fit_sample)
    mean2, cov2 = saq.covariance(to_dev(X), fit_sample)
    torch.cuda.synchronize()
    assert torch.equal(mean, mean2) and torch.equal(cov, cov2)          # run to run
    mean, cov = mean.cpu().numpy(), cov.cpu().numpy()
    c, C, _, _ = oracle.pca(_sample(X, fit_sample))
    assert np.array_equal(cov, cov.T)
    assert np.max(np.abs(mean - c)) <= 1e-12 * np.max(np.abs(X))
    err = np.max(np.abs(cov - C)) / np.max(np.abs(C))
    say(f"  max |cov - oracle| / max|cov| = {err:.2e}")
    assert err < 1e-10


@pytest.mark.parametrize("label,make,fit_sample", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_device_fit_is_the_oracle_plan(label, make, fit_sample):
    X = make()
    params = saq.PlanParams(bits_per_dim=3.0, fit_sample=fit_sample)
    say(f"device fit {label}")
    p = saq.Plan.fit_device(to_dev(X), params)
    _, _, lam, V = oracle.pca(_sample(X, fit_sample))
    ref = oracle.plan_search(lam, 3.0, params.granularity, params.max_bits, params.max_width)
    assert p.widths == ref.widths and p.bits == ref.bits
    M, c, var = p.arrays()
    np.testing.assert_allclose(var, lam, rtol=1e-9, atol=1e-12 * lam[0])
    pos = row = 0
    for w, b in zip(p.widths, p.bits):
        if b > 0:
            Ms = M[row:row + w].astype(np.float64)
            Vs = V[:, pos:pos + w]
            err = np.max(np.abs(Ms.T @ Ms - Vs @ Vs.T))
            assert err < 1e-5, (w, b, err)
            row += w
        pos += w
    # the host fit of the same rows gives the same plan
    h = saq.Plan.fit(X, params)
    assert h.widths == p.widths and h.bits == p.bits
    assert np.array_equal(h.arrays()[1], c)            # the same mean, to the bit


def test_fit_argument_errors():
    X = to_dev(np.zeros((100, 16), np.float32))
    with pytest.raises(ValueError):
        saq.covariance(X, -1)
    small = torch.empty(16, dtype=torch.uint8, device=X.device)
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.covariance(X, 0, workspace=small)
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.Plan.fit_device(X, saq.PlanParams(), workspace=small)


@pytest.mark.parametrize("D", [960, 3072])
def test_full_size_fit_sample(D):
    """The benchmark's fit shapes: 65,536 rows at D = 960 (the headline
    plan's fit rows) and D = 3072, generated on the device; the device moments
    against the oracle's on the same rows, and at D = 960 the fitted plan
    against the oracle's plan."""
    ds = synth.cfg2(65_536) if D == 960 else synth.cfg3(0, 65_536)
    say(f"full-size fit D={D}: 65,536 rows on the device")
    Xd = ds.rows_torch(65_536, torch.device("cuda", 0))
    mean, cov = saq.covariance(Xd, 0)
    torch.cuda.synchronize()
    X = Xd.cpu().numpy()
    c, C, lam, V = oracle.pca(X)
    err = np.max(np.abs(cov.cpu().numpy() - C)) / np.max(np.abs(C))
    say(f"  max |cov - oracle| / max|cov| = {err:.2e}")
    assert np.max(np.abs(mean.cpu().numpy() - c)) <= 1e-12 * np.max(np.abs(X))
    assert err < 1e-10
    if D == 960:
        params = saq.PlanParams(bits_per_dim=4.0, fit_sample=0)
        p = saq.Plan.fit_device(Xd, params)
        ref = oracle.plan_search(lam, 4.0, params.granularity, params.max_bits, params.max_width)
        assert p.widths == ref.widths and p.bits == ref.bits
        np.testing.assert_allclose(p.arrays()[2], lam, rtol=1e-9, atol=1e-12 * lam[0])


def _eig_checks(A, w, V, label, tol=1e-12):
    """Eigenvalues against numpy's (LAPACK) on the same matrix, the residual
    A V - V diag(w) and the orthogonality of V, all relative to max |A|."""
    n = A.shape[0]
    scale = max(np.max(np.abs(A)), 1e-300)
    ref = np.linalg.eigvalsh(A)
    ew = np.max(np.abs(np.sort(w) - ref)) / scale
    res = np.max(np.abs(A @ V - V * w[None, :])) / scale
    orth = np.max(np.abs(V.T @ V - np.eye(n)))
    say(f"  {label}: n={n} eigenvalues {ew:.1e} residual {res:.1e} orthogonality {orth:.1e}")
    assert ew < tol and res < tol and orth < tol, label


@pytest.mark.parametrize("n", [1, 2, 7, 64, 333])
def test_sym_eigen_random(n):
    rng = np.random.default_rng(n)
    B = rng.standard_normal((n, n))
    A = (B + B.T) / 2
    w, V = saq.sym_eigen(torch.from_numpy(A).to(cuda()))
    torch.cuda.synchronize()
    _eig_checks(A, w.cpu().numpy(), V.cpu().numpy(), "random symmetric")


def test_sym_eigen_special_matrices():
    """Degenerate cases: zero, diagonal (no rotation needed), repeated
    eigenvalues (identity plus a rank-one term), and a covariance whose
    spectrum spans ten orders of magnitude."""
    rng = np.random.default_rng(3)
    n = 50
    u = rng.standard_normal(n)
    cases = {"zero": np.zeros((n, n)), "diagonal": np.diag(rng.standard_normal(n)),
             "identity + rank one": np.eye(n) + np.outer(u, u)}
    X = rng.standard_normal((4000, n)) * np.logspace(0, -5, n)
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    cases["wide spectrum"] = Q @ ((X.T @ X) / 4000) @ Q.T
    cases["wide spectrum"] = (cases["wide spectrum"] + cases["wide spectrum"].T) / 2
    for label, A in cases.items():
        w, V = saq.sym_eigen(torch.from_numpy(np.ascontiguousarray(A)).to(cuda()))
        torch.cuda.synchronize()
        _eig_checks(A, w.cpu().numpy(), V.cpu().numpy(), label)


def test_sym_eigen_of_the_device_covariance():
    """The fit's own use: the device covariance of the cfg2 shape (20,000 x
    960) decomposed on the device, against LAPACK on the same matrix."""
    X = synth.cfg2(20_000).rows()
    _, cov = saq.covariance(to_dev(X), 0)
    w, V = saq.sym_eigen(cov)
    torch.cuda.synchronize()
    _eig_checks(cov.cpu().numpy(), w.cpu().numpy(), V.cpu().numpy(), "cfg2 covariance", tol=1e-11)
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.sym_eigen(cov, workspace=torch.empty(16, dtype=torch.uint8, device=cov.device))
