"""Planted mistakes in the oracle's Algorithm 1 (Section 3.1): each copy of
oracle/saq_oracle.c with one mistake is compiled on the CPU and run through
the code-adjustment pins; every mistake must fail at least one of them.

Trying -Delta before +Delta is not a mistake one can catch: it computes the
same function (with the other coordinates fixed the cosine is unimodal in one
code, so at most one of the two moves can raise it), and the last test shows
that on random data instead.
"""
import functools
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_caq as caq
import test_oracle_caq_order as order

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "saq_oracle.c")

# (name, text in the oracle, replacement)
MUTANTS = [
    ("dims visited in descending order",
     "        for (int i = 0; i < W; ++i) {\n            for (int k = 0; k < 2; ++k) {",
     "        for (int i = W - 1; i >= 0; --i) {\n            for (int k = 0; k < 2; ++k) {"),
    ("non-strict comparison (>=)",
     "                if (L2 > L) {",
     "                if (L2 >= L) {"),
    ("one round more than the limit",
     "for (int round = 0; rounds < 0 || round < rounds; ++round) {",
     "for (int round = 0; rounds < 0 || round <= rounds; ++round) {"),
    ("one round fewer than the limit",
     "for (int round = 0; rounds < 0 || round < rounds; ++round) {",
     "for (int round = 0; rounds < 0 || round + 1 < rounds; ++round) {"),
]

SWAPPED_DELTA = [
    ("                const double d = k == 0 ? delta : -delta;",
     "                const double d = k == 0 ? -delta : delta;"),
    ("                    code[i] += k == 0 ? 1 : -1;",
     "                    code[i] += k == 0 ? -1 : 1;"),
]


def _compile(tmp_path, name, edits):
    src = open(SRC, encoding="utf-8").read()
    for old, new in edits:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    cfile = tmp_path / (name.replace(" ", "_").replace("(", "").replace(")", "")
                        .replace(">=", "ge") + ".c")
    cfile.write_text(src)
    so = str(cfile) + ".so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                           "-ffp-contract=off", "-fno-fast-math", str(cfile), "-o", so, "-lm"])
    return oracle.load(so)


class _Shim:
    """The oracle module with quantize taken from another build."""

    def __init__(self, library):
        self.quantize = functools.partial(oracle.quantize, library=library)
        self.project = oracle.project
        self.pack = oracle.pack


def _pins():
    """Every code-adjustment pin, as (label, callable(oracle_like))."""
    p = [("hand trace", order.check_hand_trace),
         ("hand trace in a plan", order.check_hand_trace_in_a_plan),
         ("init = nearest midpoint", caq.test_init_code_is_nearest_midpoint),
         ("clamp and sign", caq.test_clamp_at_vmax_and_sign_agreement),
         ("zero segment", caq.test_zero_segment),
         ("B = 1 no-op", caq.test_b1_adjustment_is_noop),
         ("rounds approach optimum", caq.test_adjustment_approaches_optimum_with_rounds),
         ("factor form", caq.test_factor_matches_paper_estimator_form),
         ("per segment", caq.test_multi_segment_is_per_segment)]
    for B in (2, 3, 4, 7):
        p.append((f"rounds raise cosine B={B}",
                  functools.partial(caq.test_each_round_strictly_raises_cosine, B=B)))
    for B in (2, 3, 5):
        p.append((f"fixed point B={B}",
                  functools.partial(caq.test_converged_has_no_improving_move, B=B)))
    for D, B in ((4, 3), (6, 2)):
        p.append((f"exhaustive D={D} B={B}",
                  functools.partial(caq.test_exhaustive_optimum_bounds_caq, D=D, B=B)))
    return p


def test_every_pin_passes_on_the_oracle(oracle_mod):
    for label, pin in _pins():
        pin(oracle_mod)


@pytest.mark.parametrize("mutant", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, mutant, capsys):
    name, old, new = mutant
    shim = _Shim(_compile(tmp_path, name, [(old, new)]))
    caught = []
    for label, pin in _pins():
        try:
            pin(shim)
        except AssertionError:
            caught.append(label)
    with capsys.disabled():
        print(f"\n  [{name}] caught by: {', '.join(caught) or 'nothing'}")
    assert caught, name


def test_swapped_delta_order_is_the_same_function(tmp_path):
    """-Delta before +Delta gives bit-identical codes, factors and round
    counts on Gaussian and anisotropic rows at several budgets."""
    shim = _Shim(_compile(tmp_path, "minus delta first", SWAPPED_DELTA))
    rng = np.random.default_rng(77)
    O = rng.standard_normal((3000, 48)) * np.repeat([4.0, 1.5, 0.5], 16)
    O[:50, 5] = 0.0
    for B in ((2, 3, 4), (5, 7, 9), (1, 6, 2)):
        for r in (1, 4, -1):
            a = oracle.quantize(O, [16, 16, 16], list(B), r, instrument=True)
            b = shim.quantize(O, [16, 16, 16], list(B), r, instrument=True)
            assert np.array_equal(a.codes, b.codes), (B, r)
            assert np.array_equal(a.factors, b.factors), (B, r)
            assert np.array_equal(a.round_stats, b.round_stats), (B, r)
