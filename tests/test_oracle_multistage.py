"""Pins for the oracle's multi-stage estimator (Section 4.3).

The estimator reads the kept segments in plan order and, before each one,
bounds the distance from below with the segments read so far plus m sigma_Seg
for every unread segment (Chebyshev).  The pins tie it to things fixed
outside the oracle:
  * with no threshold it is the plain Section 3.2 estimator;
  * sigma_Seg is the standard deviation over the data of the segment's inner
    product, measured on held-out rows in the rotated basis the codes use;
  * on Gaussian data the tail |<o_s, q_s>| >= m sigma_s has Chebyshev's
    bound 1/m^2 and the normal distribution's two-sided tail;
  * every stage's value is the plain estimator over the segments read
    (factors of the unread ones set to 0) minus 2 m times the unread sigmas;
  * stages grow with m and with the threshold;
  * at the paper's m = 4 the nearest neighbours survive and fewer bits are read.
"""
import math

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def setup(oracle_mod):
    ds = synth.cfg1(50_000)            # rows 6,000 on are held out
    X, Q = ds.rows(0, 6000), ds.queries(40)
    c, _, lam, V = oracle_mod.pca(X)
    plan = oracle_mod.plan_search(lam, 4.0, 16, 9)
    widths, bits = plan.widths, plan.bits
    kept = []
    pos = 0
    for w, b in zip(widths, bits):
        if b > 0:
            kept.extend(range(pos, pos + w))
        pos += w
    kept = np.asarray(kept)
    P = V[:, kept].T                      # kept PCA axes, plan order
    kw = [w for w, b in zip(widths, bits) if b > 0]
    kb = [b for b in bits if b > 0]
    # a random rotation per kept segment, as the encoder applies (Section 4.1)
    R = np.zeros((len(kept), len(kept)))
    a = 0
    for s, w in enumerate(kw):
        R[a:a + w, a:a + w] = synth.haar_rotation(w, 900 + s)
        a += w
    M = (R @ P).astype(np.float32)
    cf = c.astype(np.float32)
    e = oracle_mod.encode(X, M, cf, widths, bits, 4)
    plain = oracle_mod.estimate(Q, M, cf, widths, bits, e.codes, e.factors, e.norm2)
    return dict(ds=ds, X=X, Q=Q, c=cf, lam=lam[kept], P=P, M=M, widths=widths, bits=bits,
                kw=kw, kb=kb, e=e, plain=plain)


def _ms(oracle_mod, S, m, tau):
    e = S["e"]
    return oracle_mod.estimate_multistage(S["Q"], S["M"], S["c"], S["widths"], S["bits"],
                                          e.codes, e.factors, e.norm2, S["P"], S["lam"], m, tau)


def _truncated(oracle_mod, S, t):
    """Plain estimator over the first t kept segments (the others' factors 0)."""
    e = S["e"]
    f = e.factors.copy()
    f[:, t:] = 0.0
    return oracle_mod.estimate(S["Q"], S["M"], S["c"], S["widths"], S["bits"], e.codes, f,
                               e.norm2)


def test_no_threshold_is_the_plain_estimator(oracle_mod, setup):
    d2, stage, _ = _ms(oracle_mod, setup, 4.0, np.inf)
    assert np.all(stage == len(setup["kw"]))
    np.testing.assert_array_equal(d2, setup["plain"])


def test_sigma_is_the_std_of_the_segment_inner_product(oracle_mod, setup):
    """Var over the data of <o_s, q_s>, with o_s and q_s in the rotated basis
    the codes live in, measured on 40,000 held-out rows."""
    S = setup
    _, _, sigma = _ms(oracle_mod, S, 4.0, np.inf)
    Xh = S["ds"].rows(6000, 46000).astype(np.float64) - S["c"]
    Qc = S["Q"].astype(np.float64) - S["c"]
    M = S["M"].astype(np.float64)
    a = 0
    for s, w in enumerate(S["kw"]):
        Ms = M[a:a + w]
        ip = (Xh @ Ms.T) @ (Qc @ Ms.T).T          # [rows, queries]
        emp = ip.std(axis=0)
        rel = np.abs(emp / sigma[:, s] - 1.0)
        assert rel.max() < 0.06, (s, rel.max())
        assert np.median(rel) < 0.03, (s, np.median(rel))
        a += w


@pytest.mark.parametrize("m", [1.0, 2.0, 3.0])
def test_chebyshev_tail_on_gaussian_data(oracle_mod, setup, m):
    S = setup
    _, _, sigma = _ms(oracle_mod, S, m, np.inf)
    Xh = S["ds"].rows(6000, 36000).astype(np.float64) - S["c"]
    Qc = S["Q"].astype(np.float64) - S["c"]
    M = S["M"].astype(np.float64)
    normal_tail = math.erfc(m / math.sqrt(2.0))      # P(|Z| >= m)
    a = 0
    for s, w in enumerate(S["kw"]):
        Ms = M[a:a + w]
        ip = (Xh @ Ms.T) @ (Qc @ Ms.T).T
        frac = np.mean(np.abs(ip) >= m * sigma[None, :, s])
        assert frac <= 1.0 / m ** 2
        assert abs(frac - normal_tail) < 0.15 * normal_tail + 2e-3, (s, frac, normal_tail)
        a += w


def test_all_pruned_at_stage_zero(oracle_mod, setup):
    S = setup
    d2, stage, sigma = _ms(oracle_mod, S, 4.0, -np.inf)
    assert np.all(stage == 0)
    expect = _truncated(oracle_mod, S, 0) - 2.0 * 4.0 * sigma.sum(1)[:, None]
    np.testing.assert_allclose(d2, expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())


def test_stage_values_and_rule(oracle_mod, setup):
    S = setup
    k = len(S["kw"])
    m = 2.0
    tau = np.sort(S["plain"], axis=1)[:, 9]
    d2, stage, sigma = _ms(oracle_mod, S, m, tau)
    counts = np.bincount(stage.ravel(), minlength=k + 1)
    assert counts[:k].sum() > 0.5 * stage.size and counts[k] > 0   # pruning happens, not always
    scale = np.abs(S["plain"]).max()
    tol = 1e-10 * scale
    lbs = []
    for t in range(k):
        rest = sigma[:, t:].sum(1)[:, None]
        lbs.append(_truncated(oracle_mod, S, t) - 2.0 * m * rest)
    lbs = np.stack(lbs)                                     # [k, nq, n]
    for t in range(k + 1):
        sel = stage == t
        if not sel.any():
            continue
        for tp in range(t):
            assert np.all(lbs[tp][sel] <= (tau[:, None] + tol).repeat(sel.shape[1], 1)[sel])
        if t < k:
            assert np.all(lbs[t][sel] > (tau[:, None] - tol).repeat(sel.shape[1], 1)[sel])
            np.testing.assert_allclose(d2[sel], lbs[t][sel], rtol=0, atol=tol)
        else:
            np.testing.assert_array_equal(d2[sel], S["plain"][sel])


def test_stages_grow_with_m_and_threshold(oracle_mod, setup):
    S = setup
    tau = np.sort(S["plain"], axis=1)[:, 9]
    _, s1, _ = _ms(oracle_mod, S, 1.0, tau)
    _, s2, _ = _ms(oracle_mod, S, 2.0, tau)
    _, s4, _ = _ms(oracle_mod, S, 4.0, tau)
    assert np.all(s2 >= s1) and np.all(s4 >= s2)
    _, t2, _ = _ms(oracle_mod, S, 2.0, np.sort(S["plain"], axis=1)[:, 99])
    assert np.all(t2 >= s2) and (t2 > s2).any()


def test_default_m_keeps_neighbours_and_reads_fewer_bits(oracle_mod, setup):
    """Section 4.3 / 5: at m = 4 the recall is (almost) untouched and most
    candidates stop before all segments are read."""
    S = setup
    k = len(S["kw"])
    tau = np.sort(S["plain"], axis=1)[:, 9]
    _, stage, _ = _ms(oracle_mod, S, 4.0, tau)
    top = np.argsort(S["plain"], axis=1, kind="stable")[:, :10]
    kept = np.take_along_axis(stage, top, axis=1) == k
    assert kept.mean() >= 0.99
    seg_bits = np.asarray(S["kw"]) * np.asarray(S["kb"])
    read = np.concatenate([[0], np.cumsum(seg_bits)])[stage]
    assert read.mean() < 0.6 * seg_bits.sum()
