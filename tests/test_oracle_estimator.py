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


# -- progressive approximation from code prefixes (Section 3.2) --------------

def _ip(d2, norm2, Qv):
    qn = (Qv.astype(np.float32).astype(np.float64) ** 2).sum(1)
    return (norm2[None, :] + qn[:, None] - d2) / 2.0


def test_prefix_estimator_matches_the_paper_formula(oracle_mod):
    """With c_s = floor(c / 2^(B-b)) and Delta' = Delta 2^(B-b), Section 3.2
    estimates <o, q> as <o_s', q> / <o_a, o> * ||o||^2 with
    o_s' = Delta' (c_s + 1/2) - v_max.  Written out here from the encoder's
    own v_max, Delta and <o_a, o>, it must equal the oracle's factor form."""
    rng = np.random.default_rng(41)
    D, B = 24, 6
    O, Qv = _unit(rng, 60, D).astype(np.float32), _unit(rng, 7, D).astype(np.float32)
    eye, zero = np.eye(D, dtype=np.float32), np.zeros(D, np.float32)
    e = oracle_mod.encode(O, eye, zero, [D], [B], 4, instrument=True)
    v, delta, oao = e.seg_aux[:, 0, 0], e.seg_aux[:, 0, 1], e.seg_aux[:, 0, 2]
    for b in range(1, B + 1):
        d2 = oracle_mod.estimate(Qv, eye, zero, [D], [B], e.codes, e.factors, e.norm2,
                                 prefix_bits=b)
        cs = np.floor(e.codes / 2.0 ** (B - b))
        dp = delta * 2.0 ** (B - b)
        o_s = dp[:, None] * (cs + 0.5) - v[:, None]
        ref = (Qv.astype(np.float64) @ o_s.T) / oao[None, :] * e.norm2[None, :]
        assert np.allclose(_ip(d2, e.norm2, Qv), ref, rtol=1e-10, atol=1e-12), b


def test_prefix_codes_are_the_leading_bit_planes(oracle_mod):
    """The MSB-first record layout: the first b planes of a segment's B-bit
    record are exactly the packed b-bit prefix codes floor(c / 2^(B-b))."""
    rng = np.random.default_rng(42)
    widths, bits = [16, 24, 8], [7, 5, 3]
    codes = np.concatenate([rng.integers(0, 2 ** b, size=(50, w)) for w, b in zip(widths, bits)],
                           axis=1).astype(np.int32)
    packed = oracle_mod.pack(codes, widths, bits)
    off_c, off_b = 0, 0
    for w, B in zip(widths, bits):
        pb = (w + 7) // 8
        for b in range(1, B + 1):
            pre = codes[:, off_c:off_c + w] >> (B - b)
            assert np.array_equal(oracle_mod.pack(pre, [w], [b]), packed[:, off_b:off_b + b * pb])
        off_c += w
        off_b += B * pb


def test_prefix_error_is_close_to_a_native_encode(oracle_mod):
    """Section 3.2: the b-bit prefix of an 8-bit code estimates almost as well
    as a native b-bit code, and its error still halves per bit."""
    rng = np.random.default_rng(40)
    D = 128
    O, Qv = _unit(rng, 400, D).astype(np.float32), _unit(rng, 30, D).astype(np.float32)
    eye, zero = np.eye(D, dtype=np.float32), np.zeros(D, np.float32)
    true = Qv.astype(np.float64) @ O.astype(np.float64).T
    e8 = oracle_mod.encode(O, eye, zero, [D], [8], 6)
    pre_err = []
    for b in range(1, 8):
        pre = _ip(oracle_mod.estimate(Qv, eye, zero, [D], [8], e8.codes, e8.factors, e8.norm2,
                                      prefix_bits=b), e8.norm2, Qv)
        eb = oracle_mod.encode(O, eye, zero, [D], [b], 6)
        nat = _ip(oracle_mod.estimate(Qv, eye, zero, [D], [b], eb.codes, eb.factors, eb.norm2),
                  eb.norm2, Qv)
        ep, en = np.mean(np.abs(pre - true)), np.mean(np.abs(nat - true))
        assert 0.9 < ep / en < 1.25, (b, ep, en)
        pre_err.append(ep)
    ratios = np.array(pre_err[1:]) / np.array(pre_err[:-1])
    assert np.all((ratios > 0.35) & (ratios < 0.65)), ratios


def test_prefix_of_all_bits_is_the_full_estimator(oracle_mod):
    rng = np.random.default_rng(43)
    widths, bits = [16, 16, 16], [6, 4, 2]
    D = sum(widths)
    O, Qv = _unit(rng, 40, D).astype(np.float32), _unit(rng, 5, D).astype(np.float32)
    eye, zero = np.eye(D, dtype=np.float32), np.zeros(D, np.float32)
    e = oracle_mod.encode(O, eye, zero, widths, bits, 4)
    full = oracle_mod.estimate(Qv, eye, zero, widths, bits, e.codes, e.factors, e.norm2)
    for b in (6, 7, 16):
        assert np.array_equal(full, oracle_mod.estimate(Qv, eye, zero, widths, bits, e.codes,
                                                        e.factors, e.norm2, prefix_bits=b))
    # prefix 2: the 2-bit segment keeps all its bits, the others are truncated
    p2 = oracle_mod.estimate(Qv, eye, zero, widths, bits, e.codes, e.factors, e.norm2,
                             prefix_bits=2)
    assert not np.array_equal(full, p2)
