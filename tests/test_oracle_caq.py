"""Pins for the oracle's CAQ encoder (Section 3.1, Eq. find_nearest_code,
Eq. adj-obj, Algorithm 1) against facts that do not come from the oracle:
brute-force nearest midpoints, exhaustive code search, exact rational
arithmetic for the cosine objective, and special cases the paper states."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import synth


def exact_u(codes, B):
    h = Fraction(2 ** B - 1, 2)
    return [Fraction(int(c)) - h for c in codes]


def exact_ip_n(codes, B, o):
    u = exact_u(codes, B)
    ip = sum(ui * Fraction(float(oi)) for ui, oi in zip(u, o))
    n = sum(ui * ui for ui in u)
    return ip, n


def cos_cmp(a, b):
    """sign(L(a) - L(b)) for (ip, n) pairs, exactly (L = ip / sqrt(n) / |o|)."""
    (ia, na), (ib, nb) = a, b
    # compare ia/sqrt(na) with ib/sqrt(nb)
    if ia >= 0 and ib <= 0:
        return 0 if (ia == 0 and ib == 0) else 1
    if ia <= 0 and ib >= 0:
        return -1
    sa, sb = ia * ia * nb, ib * ib * na
    s = (sa > sb) - (sa < sb)
    return s if ia > 0 else -s


def L_float(codes, B, o):
    u = np.asarray(codes, np.float64) - (2 ** B - 1) / 2
    return float(u @ o / (np.linalg.norm(u) * np.linalg.norm(o)))


def test_init_code_is_nearest_midpoint(oracle_mod):
    """rounds=0 gives Eq. find_nearest_code: the nearest of the 2^B midpoints
    -v + Delta (k + 1/2) of the uniform grid on [-v, v] (brute force)."""
    rng = np.random.default_rng(1)
    for B in (1, 2, 3, 4, 6, 9):
        O = rng.standard_normal((200, 24))
        e = oracle_mod.quantize(O, [24], [B], rounds=0)
        for r in range(O.shape[0]):
            v = np.abs(O[r]).max()
            delta = 2 * v / 2 ** B
            mids = -v + delta * (np.arange(2 ** B) + 0.5)
            best = np.argmin(np.abs(O[r][:, None] - mids[None, :]), axis=1)
            assert np.array_equal(e.codes[r], best), (B, r)


def test_clamp_at_vmax_and_sign_agreement(oracle_mod):
    o = np.array([[1.5, -1.5, 0.0, 0.25, -0.75, 1.0]])
    for B in (1, 2, 3, 5):
        e = oracle_mod.quantize(o, [6], [B], rounds=4)
        c = e.codes[0]
        assert c[0] == 2 ** B - 1          # o = +v -> last cell (clamped)
        assert c[1] == 0                   # o = -v -> first cell
        u = c - (2 ** B - 1) / 2
        nz = o[0] != 0
        assert np.all(np.sign(u[nz]) == np.sign(o[0][nz]))
        assert u[2] == 0.5                 # o = 0 sits on the middle boundary


def test_zero_segment(oracle_mod):
    O = np.zeros((3, 32))
    O[1, 16:] = np.linspace(-1, 1, 16)
    e = oracle_mod.quantize(O, [16, 16], [4, 3], rounds=4)
    assert np.all(e.codes[0, :16] == 8) and np.all(e.codes[0, 16:] == 4)
    assert np.all(e.codes[1, :16] == 8)
    assert e.factors[0, 0] == 0.0 and e.factors[0, 1] == 0.0 and e.factors[1, 0] == 0.0
    assert e.factors[1, 1] > 0


def test_b1_adjustment_is_noop(oracle_mod):
    """With one bit every code is +-1/2 and sign-aligned with o; no +-1 move
    can raise the cosine (RaBitQ's sign code, Section 2.2)."""
    O = np.random.default_rng(2).standard_normal((300, 64))
    e0 = oracle_mod.quantize(O, [64], [1], rounds=0)
    e8 = oracle_mod.quantize(O, [64], [1], rounds=8, instrument=True)
    assert np.array_equal(e0.codes, e8.codes)
    assert np.array_equal(e0.codes, (O > 0).astype(np.int32) | (O == 0))
    assert e8.round_stats[:, :, 0].sum() == 0


@pytest.mark.parametrize("B", [2, 3, 4, 7])
def test_each_round_strictly_raises_cosine(oracle_mod, B):
    """Algorithm 1 only accepts strict improvements: the cosine after round
    r+1 is exactly (rational arithmetic) above the cosine after round r when
    round r+1 accepted something, and identical otherwise."""
    O = np.random.default_rng(3).standard_normal((40, 12)) * np.linspace(2, 0.1, 12)
    prev = oracle_mod.quantize(O, [12], [B], rounds=0)
    for r in range(1, 7):
        cur = oracle_mod.quantize(O, [12], [B], rounds=r, instrument=True)
        for i in range(O.shape[0]):
            acc = cur.round_stats[i, 0, r - 1] if cur.round_stats[i, 0, -1] >= r else 0
            a = exact_ip_n(cur.codes[i], B, O[i])
            b = exact_ip_n(prev.codes[i], B, O[i])
            if acc > 0:
                assert cos_cmp(a, b) == 1, (B, r, i)
            else:
                assert np.array_equal(cur.codes[i], prev.codes[i])
        prev = cur


@pytest.mark.parametrize("B", [2, 3, 5])
def test_converged_has_no_improving_move(oracle_mod, B):
    """rounds=-1 runs to a fixed point: no single +-1 change (inside the code
    range) raises the cosine, checked exactly from scratch."""
    O = np.random.default_rng(4).standard_normal((30, 10))
    e = oracle_mod.quantize(O, [10], [B], rounds=-1)
    for r in range(O.shape[0]):
        base = exact_ip_n(e.codes[r], B, O[r])
        for i in range(10):
            for s in (1, -1):
                c = e.codes[r].copy()
                c[i] += s
                if 0 <= c[i] <= 2 ** B - 1:
                    assert cos_cmp(exact_ip_n(c, B, O[r]), base) <= 0


@pytest.mark.parametrize("D,B", [(4, 3), (6, 2), (6, 3), (8, 2)])
def test_exhaustive_optimum_bounds_caq(oracle_mod, D, B):
    """The CAQ codebook equals E-RaBitQ's grid (Lemma in Section 3.3), so the
    exhaustive argmax of the cosine over all 2^(B*D) codes bounds the
    coordinate-descent result; CAQ should land close to it."""
    rng = np.random.default_rng(5 + D + B)
    O = rng.standard_normal((25, D))
    grid = np.array(list(itertools.product(range(2 ** B), repeat=D)), np.float64)
    U = grid - (2 ** B - 1) / 2
    Un = U / np.linalg.norm(U, axis=1, keepdims=True)
    e = oracle_mod.quantize(O, [D], [B], rounds=-1)
    gaps = []
    for r in range(O.shape[0]):
        opt = float((Un @ O[r]).max() / np.linalg.norm(O[r]))
        got = L_float(e.codes[r], B, O[r])
        assert got <= opt + 1e-12
        gaps.append(opt - got)
    assert np.mean(gaps) < 0.01


def test_adjustment_approaches_optimum_with_rounds(oracle_mod):
    """Section 5.3 (rounds ablation): the error gap to the optimum shrinks as
    the round limit grows."""
    rng = np.random.default_rng(9)
    O = rng.standard_normal((60, 6))
    B = 3
    grid = np.array(list(itertools.product(range(2 ** B), repeat=6)), np.float64)
    U = grid - (2 ** B - 1) / 2
    Un = U / np.linalg.norm(U, axis=1, keepdims=True)
    opt = (O @ Un.T).max(axis=1) / np.linalg.norm(O, axis=1)
    gap = []
    for r in (0, 1, 4):
        e = oracle_mod.quantize(O, [6], [B], rounds=r)
        got = np.array([L_float(e.codes[i], B, O[i]) for i in range(O.shape[0])])
        gap.append(float(np.mean(opt - got)))
    assert gap[0] > gap[1] >= gap[2] >= 0.0


def test_b1_cosine_concentrates_near_0_8(oracle_mod):
    """Section 2.2: the 1-bit code's <o_bar, o> for unit vectors concentrates
    around 0.8; for Gaussian o it is sqrt(2/pi) = 0.798 in the limit."""
    O = np.random.default_rng(6).standard_normal((400, 256))
    e = oracle_mod.quantize(O, [256], [1], rounds=4)
    cos = np.array([L_float(e.codes[i], 1, O[i]) for i in range(400)])
    assert abs(cos.mean() - math.sqrt(2 / math.pi)) < 0.01
    assert cos.std() < 0.02


def test_factor_matches_paper_estimator_form(oracle_mod):
    """Eq. (estimator_inner_product): <o_a, q> = Delta <c, q> + q_sum (-v + Delta/2),
    and <o, q> ~= <o_a, q> / <o_a, o> * ||o||^2.  The stored factor form
    f * <u, q> with f = ||o||^2 / <u, o> gives the same number."""
    rng = np.random.default_rng(7)
    O = rng.standard_normal((50, 32))
    Qv = rng.standard_normal((50, 32))
    e = oracle_mod.quantize(O, [32], [5], rounds=4, instrument=True)
    for r in range(50):
        v, delta, xo, oo = e.seg_aux[r, 0]
        q = Qv[r]
        oa_q = delta * (e.codes[r] @ q) + q.sum() * (-v + delta / 2)
        paper = oa_q / xo * oo
        u = e.codes[r] - (2 ** 5 - 1) / 2
        ours = e.factors[r, 0] * (u @ q)
        assert paper == pytest.approx(ours, rel=1e-12, abs=1e-12)
        # the stored <o_a, o> is the inner product of the final quantized vector
        oa = delta * (e.codes[r] + 0.5) - v
        assert xo == pytest.approx(oa @ O[r], rel=1e-12)
        assert oo == pytest.approx(O[r] @ O[r], rel=1e-12)


def test_multi_segment_is_per_segment(oracle_mod):
    """Section 4.2: each segment is quantized on its own, 'just as a normal
    vector' -- a plan of segments equals separate runs on the slices."""
    O = np.random.default_rng(8).standard_normal((20, 48)) * np.repeat([3.0, 1.0, 0.2], 16)
    whole = oracle_mod.quantize(O, [16, 16, 16], [6, 4, 2], rounds=4)
    for s, (lo, B) in enumerate([(0, 6), (16, 4), (32, 2)]):
        part = oracle_mod.quantize(O[:, lo:lo + 16], [16], [B], rounds=4)
        assert np.array_equal(part.codes, whole.codes[:, lo:lo + 16])
        assert np.array_equal(part.factors[:, 0], whole.factors[:, s])


def test_projection_and_norm(oracle_mod):
    """Eq. (rotate): o = P (o_r - c); an orthonormal P keeps ||o|| = ||o_r - c||
    (checked against numpy in FP64)."""
    ds = synth.cfg1(300)
    X = ds.rows()
    R = synth.haar_rotation(128, 99).astype(np.float32)
    c = X.mean(0).astype(np.float32)
    O, nn = oracle_mod.project(X, R, c)
    ref = (X.astype(np.float64) - c.astype(np.float64)) @ R.astype(np.float64).T
    assert np.allclose(O, ref, rtol=0, atol=1e-12)
    assert np.allclose(nn, (O ** 2).sum(1), rtol=1e-6)


def test_pack_layout_golden(oracle_mod):
    """Bit-plane layout, worked by hand: per segment, MSB plane first; dim i
    of a plane at byte i//8, bit i%8; a plane takes ceil(W/8) bytes."""
    # segment 1: W=10, B=3, codes 5 0 7 2 1 1 0 6 3 4 (binary 101 000 111 010
    # 001 001 000 110 011 100); segment 2: W=2, B=2, codes 2 1 (10 01)
    codes = np.array([[5, 0, 7, 2, 1, 1, 0, 6, 3, 4, 2, 1]], np.int32)
    got = oracle_mod.pack(codes, [10, 2], [3, 2])
    expect = [
        0b10000101, 0b00000010,   # bit 2: dims 0, 2, 7 | dim 9
        0b10001100, 0b00000001,   # bit 1: dims 2, 3, 7 | dim 8
        0b00110101, 0b00000001,   # bit 0: dims 0, 2, 4, 5 | dim 8
        0b00000001,               # segment 2, bit 1: dim 0
        0b00000010,               # segment 2, bit 0: dim 1
    ]
    assert list(got[0]) == expect


def test_pack_roundtrip(oracle_mod):
    rng = np.random.default_rng(10)
    widths, bits = [16, 48, 32, 24], [9, 4, 1, 3]
    codes = np.concatenate([rng.integers(0, 2 ** b, size=(7, w)) for w, b in zip(widths, bits)],
                           axis=1).astype(np.int32)
    packed = oracle_mod.pack(codes, widths, bits)
    assert packed.shape[1] == sum(b * ((w + 7) // 8) for w, b in zip(widths, bits))
    # unpack independently
    out = np.zeros_like(codes)
    pos = off = 0
    for w, b in zip(widths, bits):
        pb = (w + 7) // 8
        for p in range(b - 1, -1, -1):
            bitsarr = np.unpackbits(packed[:, pos:pos + pb], axis=1, bitorder="little")[:, :w]
            out[:, off:off + w] |= bitsarr.astype(np.int32) << p
            pos += pb
        off += w
    assert np.array_equal(out, codes)


def test_thread_count_argument_leaves_the_process_setting(oracle_mod):
    """A call with threads=1 runs on one thread and then restores the OpenMP
    thread count: the runtime is shared with every library in the process."""
    import ctypes
    gomp = ctypes.CDLL("libgomp.so.1")
    before = gomp.omp_get_max_threads()
    O = np.random.default_rng(0).standard_normal((50, 16))
    oracle_mod.quantize(O, [16], [4], rounds=2, threads=1)
    oracle_mod.project(O.astype(np.float32), np.eye(16, dtype=np.float32),
                       np.zeros(16, np.float32), threads=1)
    assert gomp.omp_get_max_threads() == before
