"""Pins for the oracle's plan search (Section 4.2, Eq. seg-err, Algorithm 2
and the fewest-segments selection) against brute force over every
segmentation and bit vector, the closed-form minimum of a separable convex
allocation (greedy marginal allocation), and the special cases the paper
states (uniform spectrum -> one segment)."""
import heapq
import itertools

import numpy as np
import pytest

import synth


def all_plans(units, max_bits, max_w_units):
    """Every composition of the unit list into contiguous segments, with every
    bit vector."""
    nu = len(units)
    for cuts in itertools.product([0, 1], repeat=nu - 1):
        bounds = [0] + [i + 1 for i, c in enumerate(cuts) if c] + [nu]
        segs = [(bounds[j], bounds[j + 1]) for j in range(len(bounds) - 1)]
        for bits in itertools.product(range(max_bits + 1), repeat=len(segs)):
            if max_w_units and any(b > 0 and (e - s) > max_w_units
                                   for (s, e), b in zip(segs, bits)):
                continue
            yield segs, bits


def brute(sig2, g, quota, max_bits, max_w_units=0, eps=1e-3):
    D = len(sig2)
    units = [g] * (D // g) + ([D % g] if D % g else [])
    pos = np.concatenate([[0], np.cumsum(units)])
    best = np.inf
    cands = []
    for segs, bits in all_plans(units, max_bits, max_w_units):
        cost = sum(b * (pos[e] - pos[s]) for (s, e), b in zip(segs, bits))
        if cost > quota:
            continue
        err = sum(sig2[pos[s]:pos[e]].sum() * 2.0 ** -b for (s, e), b in zip(segs, bits))
        cands.append((err, len(segs)))
        best = min(best, err)
    fewest = min(k for err, k in cands if err <= (1 + eps) * best)
    best_at_fewest = min(err for err, k in cands if k == fewest and err <= (1 + eps) * best)
    return best, fewest, best_at_fewest


def greedy_min(sig2, g, quota, max_bits):
    """Separable convex allocation with unit increments: repeatedly give one
    more bit to the unit with the largest error reduction per bit."""
    D = len(sig2)
    units = [g] * (D // g) + ([D % g] if D % g else [])
    pos = np.concatenate([[0], np.cumsum(units)])
    S = [sig2[pos[j]:pos[j + 1]].sum() for j in range(len(units))]
    b = [0] * len(units)
    used = 0
    heap = [(-S[j] * 0.5 / units[j], j) for j in range(len(units))]
    heapq.heapify(heap)
    while heap:
        gain, j = heapq.heappop(heap)
        if used + units[j] > quota or b[j] >= max_bits:
            continue
        b[j] += 1
        used += units[j]
        if b[j] < max_bits:
            heapq.heappush(heap, (-S[j] * 2.0 ** -(b[j] + 1) / units[j], j))
    return sum(S[j] * 2.0 ** -b[j] for j in range(len(units)))


def rand_spectrum(rng, d):
    return np.sort(rng.gamma(0.5, 1.0, size=d))[::-1] + 1e-3


@pytest.mark.parametrize("seed", range(6))
def test_plan_matches_brute_force(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    g = 4
    nu = 3 + seed % 3                      # 3..5 units
    D = g * nu - (seed % 2)                # a partial last unit on odd seeds
    sig2 = rand_spectrum(rng, D)
    bpd = [1.0, 1.5, 2.25, 3.0][seed % 4]
    max_bits = 4
    p = oracle_mod.plan_search(sig2, bpd, g=g, max_bits=max_bits)
    quota = oracle_mod.quota_bits(bpd, D)
    best, fewest, best_at = brute(sig2, g, quota, max_bits)
    assert p.min_error == pytest.approx(best, rel=1e-12)
    assert p.nseg == fewest
    assert p.error == pytest.approx(best_at, rel=1e-12)
    assert p.cost <= quota and sum(p.widths) == D


def test_plan_max_width_brute_force(oracle_mod):
    rng = np.random.default_rng(11)
    g, D = 4, 20
    sig2 = rand_spectrum(rng, D)
    p = oracle_mod.plan_search(sig2, 2.0, g=g, max_bits=3, max_width=8)
    best, fewest, best_at = brute(sig2, g, oracle_mod.quota_bits(2.0, D), 3, max_w_units=2)
    assert p.min_error == pytest.approx(best, rel=1e-12)
    assert p.nseg == fewest
    assert all(w <= 8 for w, b in zip(p.widths, p.bits) if b > 0)


@pytest.mark.parametrize("bpd", [0.5, 1.0, 2.0, 4.0, 5.5])
def test_min_error_equals_greedy(oracle_mod, bpd):
    """The error model is a per-dimension sum, so splitting or merging
    equal-bit neighbours changes neither error nor cost and the minimum over
    plans is the separable allocation over g-dim units (greedy is exact)."""
    rng = np.random.default_rng(int(bpd * 10))
    D, g = 96, 16
    sig2 = rand_spectrum(rng, D)
    err, _ = oracle_mod.alg2(sig2, bpd, g=g, max_bits=9)
    assert err == pytest.approx(greedy_min(sig2, g, oracle_mod.quota_bits(bpd, D), 9), rel=1e-12)
    p = oracle_mod.plan_search(sig2, bpd, g=g, max_bits=9)
    assert p.min_error == pytest.approx(err, rel=1e-12)
    assert p.error <= (1 + 1e-3) * err


def test_uniform_spectrum_gives_one_segment(oracle_mod):
    """Section 4.2: with a perfectly uniform eigenvalue distribution the plan
    is a single segment holding every dimension (CAQ)."""
    for bpd in (1.0, 3.0, 4.0):
        p = oracle_mod.plan_search(np.ones(128), bpd, g=16, max_bits=9)
        assert p.widths == [128] and p.bits == [int(bpd)]


def test_min_plan_bits_non_increasing(oracle_mod):
    rng = np.random.default_rng(12)
    for _ in range(5):
        sig2 = rand_spectrum(rng, 160)
        _, (w, b) = oracle_mod.alg2(sig2, 3.0, g=16, max_bits=9)
        assert all(b[i] >= b[i + 1] for i in range(len(b) - 1))


def test_exponential_spectrum_reverse_water_filling(oracle_mod):
    """With ERROR = sum sigma^2 2^-B the continuous optimum equalises the
    marginal gain sigma_j^2 2^-b_j, i.e. b_j = log2(sigma_j^2) + lambda clipped
    to [0, max_bits] (reverse water-filling); for sigma_i^2 = exp(-i/tau) the
    bits fall by one every tau*ln 2 dims.  The integer plan on 16-dim units
    stays within one bit of it everywhere."""
    tau, D, g = 24.0, 128, 16
    sig2 = synth.exp_spectrum(D, tau)
    p = oracle_mod.plan_search(sig2, 4.0, g=g, max_bits=9)
    per_dim = np.repeat(p.bits, p.widths).astype(float)
    unit_var = sig2.reshape(-1, g).mean(1)
    lo, hi = -60.0, 60.0
    for _ in range(200):
        lam = (lo + hi) / 2
        b = np.clip(np.log2(unit_var) + lam, 0, 9)
        lo, hi = (lam, hi) if b.sum() * g < 512 else (lo, lam)
    cont = np.repeat(np.clip(np.log2(unit_var) + lam, 0, 9), g)
    assert np.max(np.abs(per_dim - cont)) <= 1.0
    assert np.polyfit(np.arange(D), cont, 1)[0] == pytest.approx(-1 / (tau * np.log(2)), rel=0.1)
    assert p.cost == 512


def test_record_size_matches_paper_storage_table():
    """Section 5.3 storage table: 10M x 1024 at B=4 takes 5,114 MB (raw 39,100
    MB), i.e. about 536 bytes per vector = 512 bytes of code plus a few
    4-byte factors.  Our record is B*D/8 + 4*(kept segments + 1)."""
    path = __file__.replace("test_oracle_plan.py", "golden/quant_space_msmarco.txt")
    rows = dict(l.split("=") for l in open(path).read().split("\n") if "=" in l and l[0] != "#")
    n, d = int(rows["n"]), int(rows["d"])
    raw_mb, saq_mb = float(rows["raw_mb_reported"]), float(rows["saq_b4_mb_reported"])
    # the table's MB are MiB: raw = n*d*4 bytes
    assert raw_mb == pytest.approx(n * d * 4 / 2 ** 20, rel=2e-3)
    per_vec = saq_mb * 2 ** 20 / n
    code = 4 * d / 8
    extra_floats = (per_vec - code) / 4
    assert 4 <= extra_floats <= 8        # 5-7 factors, e.g. 5 segments + norm
