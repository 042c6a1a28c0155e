"""Pins for the order in which Algorithm 1 visits its moves (Section 3.1):
rounds outer, the dimensions of a segment in ascending order inside a round,
+Delta tried before -Delta, a move kept only on a strict increase of the
cosine, and exactly r rounds.

The invariants in test_oracle_caq.py (each round raises the cosine, the
fixed point has no improving move, the exhaustive optimum bounds the result)
hold for any visiting order.  The trace below is worked by hand from the
algorithm with exact fractions, and its codes change under a descending
visiting order, a non-strict comparison, or one round more or less.

Swapping +Delta and -Delta cannot change any result, and the second test
shows why on random states: with the other coordinates fixed, the cosine as
a function of one code is unimodal, so the two neighbours of a code never
both raise it.
"""
from fractions import Fraction

import numpy as np
import pytest

# o = (1/2, -1, 3/4, 0), B = 3 (one segment).
#   v_max = 1, Delta = 2 v_max / 2^B = 1/4; the initial code is
#   floor((o_i + v_max) / Delta) = floor(4 (o_i + 1)), clamped to 7:
#   (6, 0, 7, 4).  With u = c - 7/2 the cosine is <u, o> / (|u| |o|), so a
#   move is compared through ip^2 / n, ip = <u, o>, n = |u|^2 (ip > 0).
#   start: u = (5/2, -7/2, 7/2, 1/2), ip = 59/8, n = 31, ip^2/n = 3481/1984 (1.75454)
# round 1 (dims 0, 1, 2, 3):
#   dim 0: +1 -> ip 63/8, n 37: 3969/2368 (1.67610) no;
#          -1 -> ip 55/8, n 27: 3025/1728 (1.75058) no
#   dim 1: +1 -> ip 51/8, n 25: 2601/1600 (1.62563) no; -1 leaves the grid (code -1)
#   dim 2: +1 leaves the grid (code 8);
#          -1 -> ip 53/8, n 25: 2809/1600 (1.75563) > 1.75454: ACCEPT, code 7 -> 6
#   dim 3: +1 -> ip 53/8, n 27: 2809/1728 (1.62558) no;
#          -1 -> ip 53/8, n 25: 2809/1600, equal, not strictly larger: no
#   after round 1: (6, 0, 6, 4), ip = 53/8, n = 25
# round 2:
#   dim 0: +1 -> ip 57/8, n 31: 3249/1984 (1.63760) no;
#          -1 -> ip 49/8, n 21: 343/192 (1.78646) > 1.75563: ACCEPT, code 6 -> 5
#   dim 1: +1 -> ip 41/8, n 15: 1681/960 (1.75104) no
#   dim 2: +1 -> ip 55/8, n 27: 3025/1728 (1.75058) no;
#          -1 -> ip 43/8, n 17: 1849/1088 (1.69945) no
#   dim 3: +1 -> ip 49/8, n 23: 2401/1472 (1.63111) no; -1 equal: no
#   after round 2: (5, 0, 6, 4), ip = 49/8, n = 21
# round 3:
#   dim 0: +1 -> back to 2809/1600 no; -1 -> ip 45/8, n 19: 2025/1216 (1.66530) no
#   dims 1, 2, 3: as in round 2 from the same ip, n: no
#   nothing accepted: (5, 0, 6, 4) is the fixed point.
TRACE_O = [0.5, -1.0, 0.75, 0.0]
TRACE_B = 3
TRACE_CODES = {
    0: [6, 0, 7, 4],
    1: [6, 0, 6, 4],
    2: [5, 0, 6, 4],
    3: [5, 0, 6, 4],
    -1: [5, 0, 6, 4],
}
# Under a descending order, round 1 visits dim 2 first (the same accept) and
# then dim 0 against ip 53/8, n 25, where -1 already wins: (5, 0, 6, 4) after
# one round.  Under ">=" the tie at dim 3 is taken: (6, 0, 6, 3).  One round
# more or less gives the round-2 or round-0 codes at r = 1.


def check_hand_trace(oracle_mod):
    O = np.array([TRACE_O])
    for r, want in TRACE_CODES.items():
        e = oracle_mod.quantize(O, [4], [TRACE_B], rounds=r)
        assert list(e.codes[0]) == want, (r, list(e.codes[0]), want)


def check_hand_trace_in_a_plan(oracle_mod):
    """The same trace as the second segment of a plan, behind a segment whose
    moves must not leak into it, and repeated over many rows."""
    first = [0.9, -0.3, 0.1, 0.6]
    O = np.tile(np.array([first + TRACE_O]), (37, 1))
    for r in (1, 2):
        e = oracle_mod.quantize(O, [4, 4], [2, TRACE_B], rounds=r)
        assert np.all(e.codes[:, 4:] == TRACE_CODES[r]), r


def test_hand_worked_trace(oracle_mod):
    check_hand_trace(oracle_mod)


def test_hand_worked_trace_in_a_plan(oracle_mod):
    check_hand_trace_in_a_plan(oracle_mod)


def test_round_statistics_follow_the_trace(oracle_mod):
    """One accept in round 1 (dim 2), one in round 2 (dim 0), none in round
    3, which ends the loop; with no round limit the same three rounds run."""
    O = np.array([TRACE_O])
    for r in (3, 8, -1):
        e = oracle_mod.quantize(O, [4], [TRACE_B], rounds=r, instrument=True)
        st = e.round_stats[0, 0]
        assert list(st[:3]) == [1, 1, 0], (r, st[:4])
        assert st[-1] == 3


def _exact_ratio(u, o):
    ip = sum(a * b for a, b in zip(u, o))
    n = sum(a * a for a in u)
    return ip, n


@pytest.mark.parametrize("B", [2, 3, 4, 6])
def test_plus_and_minus_never_both_raise_the_cosine(B):
    """Why the +Delta/-Delta order is immaterial.  Take any code whose terms
    u_j o_j are all >= 0 (the initial code has this property, and Algorithm 1
    keeps it, since a move that flips the sign of a term lowers <u, o>
    without lowering |u|).  For one coordinate t = u_i with the others fixed,
    L(t) = (a + t o_i) / sqrt(b + t^2) with a = <u, o> - u_i o_i >= 0 has the
    derivative sign of o_i b - a t: one sign change, so L rises and then
    falls and the two neighbours t - 1, t + 1 cannot both lie above L(t).
    Checked exactly on random sign-aligned codes."""
    rng = np.random.default_rng(40 + B)
    half = Fraction(2 ** B - 1, 2)
    cmax = 2 ** B - 1
    for _ in range(300):
        W = int(rng.integers(2, 9))
        o = [Fraction(int(k), 64) for k in rng.integers(-64, 65, size=W)]
        codes = []
        for oi in o:
            if oi > 0:
                codes.append(int(rng.integers(2 ** (B - 1), cmax + 1)))
            elif oi < 0:
                codes.append(int(rng.integers(0, 2 ** (B - 1))))
            else:
                codes.append(int(rng.integers(0, cmax + 1)))
        u = [Fraction(c) - half for c in codes]
        ip, n = _exact_ratio(u, o)
        if ip <= 0:
            continue
        for i in range(W):
            better = 0
            for s in (1, -1):
                if not 0 <= codes[i] + s <= cmax:
                    continue
                u2 = list(u)
                u2[i] += s
                ip2, n2 = _exact_ratio(u2, o)
                if ip2 > 0 and ip2 * ip2 * n > ip * ip * n2:
                    better += 1
            assert better <= 1, (o, codes, i)
