"""The parity harness's classifier of differing codes, checked on the CPU.

A stand-in for the device perturbs the oracle's FP64 projection by at most
eps per component and quantizes with the oracle: every code that then
differs must be explained (init cell edge, decision near-tie or cascade).
A code changed by one away from any boundary must come out unexplained."""
from types import SimpleNamespace

import numpy as np

import oracle
import synth
from gpu_util import classify_mismatches


def _setup(seed):
    ds = synth.cfg1(3000)
    X = ds.rows()
    c, _, lam, V = oracle.pca(X)
    plan = oracle.plan_search(lam, 4.0, 16, 9)
    kw = [w for w, b in zip(plan.widths, plan.bits) if b > 0]
    kb = [b for b in plan.bits if b > 0]
    M = V[:, :sum(kw)].T.astype(np.float32)
    ref = oracle.encode(X, M, c.astype(np.float32), kw, kb, 4, instrument=True)
    return SimpleNamespace(kept_widths=kw, kept_bits=kb), ref


def test_perturbed_projection_is_explained():
    plan, ref = _setup(0)
    rng = np.random.default_rng(1)
    # a far larger error than the device's, so that many codes move
    eps = 3e-4 * np.sqrt(ref.norm2)
    noisy = ref.O + rng.uniform(-1, 1, ref.O.shape) * eps[:, None]
    dev = oracle.quantize(noisy, plan.kept_widths, plan.kept_bits, 4)
    counts = classify_mismatches(plan, dev.codes, ref, np.abs(noisy - ref.O))
    moved = int(np.count_nonzero(dev.codes != ref.codes))
    assert moved > 50
    assert counts["unexplained"] == 0, counts
    assert counts["init"] + counts["decision"] + counts["cascade"] == moved
    assert counts["init"] > 0 and counts["decision"] > 0


def test_planted_off_by_one_is_unexplained():
    plan, ref = _setup(0)
    err = 1e-7 * np.sqrt(ref.norm2)[:, None]       # about the device's projection error
    codes = ref.codes.copy()
    # a code of the 4-bit segment (dims 48 .. 79) in a row whose segment has no
    # decision within 1e-4 of a tie and no value within 1e-4 cells of an edge
    s, lo, w, B = 3, 48, 32, 4
    v, delta = ref.seg_aux[:, s, 0], ref.seg_aux[:, s, 1]
    q = (ref.O[:, lo:lo + w] + v[:, None]) / delta[:, None]
    edge = np.abs(q - np.clip(np.rint(q), 1, 2 ** B - 1)).min(1)
    tie = ref.code_aux[:, lo:lo + w, 1].min(1)
    r = int(np.argmax(np.minimum(edge, tie)))
    assert min(edge[r], tie[r]) > 1e-4
    i = lo + 5
    codes[r, i] += 1 if codes[r, i] == 0 else -1
    counts = classify_mismatches(plan, codes, ref, err)
    assert counts["unexplained"] == 1, counts
