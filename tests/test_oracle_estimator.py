"""Pins for the oracle's distance estimator (Section 3.2) against the error
behaviour the paper states: E-RaBitQ's empirical bound (Section 2.3 remark),
error roughly halving per extra bit (Section 4.2), and near-exactness at
many bits."""
import numpy as np
import pytest

import synth


def _unit(rng, n, d):
    a = rng.standard_normal((n, d))
    return a / np.linalg.norm(a, axis=1, keepdims=True)


def _est_ip(oracle_mod, O, Qv, B, rounds=6):
    d = O.shape[1]
    eye = np.eye(d, dtype=np.float32)
    zero = np.zeros(d, np.float32)
    e = oracle_mod.encode(O.astype(np.float32), eye, zero, [d], [B], rounds)
    d2 = oracle_mod.estimate(Qv.astype(np.float32), eye, zero, [d], [B], e.codes, e.factors,
                             e.norm2)
    qn = (Qv.astype(np.float32).astype(np.float64) ** 2).sum(1)
    return (e.norm2[None, :] + qn[:, None] - d2) / 2.0


@pytest.mark.parametrize("B", [2, 4, 6])
def test_inner_product_error_within_erabitq_bound(oracle_mod, B):
    """CAQ shares E-RaBitQ's codebook (Section 3.3), so its estimates of
    <o, q> for unit vectors should satisfy the reported bound
    |err| < 2^-B * 5.75 / sqrt(D) for (almost) all pairs."""
    rng = np.random.default_rng(20 + B)
    D = 128
    O, Qv = _unit(rng, 400, D), _unit(rng, 25, D)
    est = _est_ip(oracle_mod, O, Qv, B)
    true = Qv.astype(np.float32).astype(np.float64) @ O.astype(np.float32).astype(np.float64).T
    frac = np.mean(np.abs(est - true) < 2.0 ** -B * 5.75 / np.sqrt(D))
    assert frac >= 0.995


def test_error_halves_per_bit(oracle_mod):
    rng = np.random.default_rng(30)
    D = 96
    O, Qv = _unit(rng, 300, D), _unit(rng, 20, D)
    true = Qv.astype(np.float32).astype(np.float64) @ O.astype(np.float32).astype(np.float64).T
    errs = []
    for B in range(2, 9):
        errs.append(np.mean(np.abs(_est_ip(oracle_mod, O, Qv, B) - true)))
    ratios = np.array(errs[1:]) / np.array(errs[:-1])
    assert np.all((ratios > 0.35) & (ratios < 0.65)), ratios


def test_many_bits_is_nearly_exact(oracle_mod):
    ds = synth.cfg1(200)
    X, Qr = ds.rows(), ds.queries(10)
    d = X.shape[1]
    eye = np.eye(d, dtype=np.float32)
    c = X.mean(0).astype(np.float32)
    e = oracle_mod.encode(X, eye, c, [d], [16], 4)
    d2 = oracle_mod.estimate(Qr, eye, c, [d], [16], e.codes, e.factors, e.norm2)
    true = oracle_mod.true_dist2(Qr, X)
    rel = oracle_mod.relative_error(d2, true)
    # the bound above at B=16, D=128 is ~8e-6 on a unit-vector inner product
    assert np.mean(rel) < 1e-5 and np.max(rel) < 1e-4


def test_dropped_segment_contributes_nothing(oracle_mod):
    """Dims of a 0-bit segment are left out of the inner product but their
    energy stays in ||o||^2 (the stored full norm)."""
    rng = np.random.default_rng(31)
    X = rng.standard_normal((50, 32)).astype(np.float32)
    Qv = rng.standard_normal((5, 32)).astype(np.float32)
    eye = np.eye(32, dtype=np.float32)
    zero = np.zeros(32, np.float32)
    e = oracle_mod.encode(X, eye[:16], zero, [16], [8], 4)
    d2 = oracle_mod.estimate(Qv, eye[:16], zero, [16], [8], e.codes, e.factors, e.norm2)
    X64, Q64 = X.astype(np.float64), Qv.astype(np.float64)
    ip_head = Q64[:, :16] @ X64[:, :16].T
    expect = (X64 ** 2).sum(1)[None, :] + (Q64 ** 2).sum(1)[:, None] - 2 * ip_head
    assert np.allclose(d2, expect, rtol=0, atol=0.05 * np.abs(ip_head).max())
