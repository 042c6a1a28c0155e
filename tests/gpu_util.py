"""Shared helpers for the GPU tests: run the device path through the C ABI and
compare its records with the oracle's."""
import sys

import numpy as np

import oracle
import paper_2509_12086_amd as saq


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def cuda():
    import torch
    return torch.device("cuda", 0)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(cuda())


def gpu_project(plan, X):
    """The device's projection of host rows X (row layout; the same values
    the encode quantizes): FP32 [n, D_kept]."""
    import torch
    O, _ = saq.project(plan, to_dev(np.asarray(X, np.float32)))
    torch.cuda.synchronize()
    return O.cpu().numpy()[:, :plan.D_kept]


def gpu_encode(plan, X, rounds=4):
    import torch
    codes, fac = saq.encode(plan, to_dev(X.astype(np.float32)), rounds)
    torch.cuda.synchronize()
    return codes.cpu().numpy(), fac.cpu().numpy()


def oracle_encode(plan, X, rounds=4, instrument=True):
    """The oracle's encode, instrumented (per-code init and decision margins,
    per-segment grid) so that compare() can classify differing codes."""
    M, c, _ = plan.arrays()
    return oracle.encode(X, M, c, plan.kept_widths, plan.kept_bits, rounds, instrument)


def oracle_records(plan, X, rounds=4):
    """Records encoded and packed by the oracle, for the scans' parity tests:
    (packed uint8 [n, code_bytes], factors float32 [n, k + 1], codes int32
    [n, D_kept]).  Both sides then read the same bytes and the same FP32
    factors, and nothing the oracle reads comes from the device."""
    enc = oracle_encode(plan, X, rounds, instrument=False)
    packed = oracle.pack(enc.codes, plan.kept_widths, plan.kept_bits)
    fac = np.concatenate([enc.factors, enc.norm2[:, None]], axis=1).astype(np.float32)
    return packed, fac, enc.codes


def oracle_scan(plan, Q, codes, fac, prefix_bits=0):
    """The oracle's Section 3.2 estimator on records given as in oracle_records."""
    M, c, _ = plan.arrays()
    return oracle.estimate(Q, M, c, plan.kept_widths, plan.kept_bits, codes,
                           fac[:, :-1].astype(np.float64), fac[:, -1].astype(np.float64),
                           prefix_bits=prefix_bits)


U32 = 2.0 ** -24


def classify_mismatches(plan, codes, ref, err):
    """Sort every code that differs from the oracle's into one of:
      init      -- the oracle's (o_i + v) / Delta lies within 4 e_s / Delta
                   of an edge between two cells (an integer 1 .. 2^B - 1; the
                   ends 0 and 2^B of the grid are not edges: the clamp keeps
                   the extreme codes there);
      decision  -- some trial of Algorithm 1 on that dim moved the cosine by
                   at most kappa = 5 |d_s| / (sqrt(W) L0 |o_s|), relative;
      cascade   -- neither, in a segment of that vector that holds a dim at
                   an init cell edge or a decision near-tie;
      unexplained -- everything else.
    err [n, D_kept] is the absolute difference between the device's and the
    oracle's projected components (0 where both quantized the same values),
    d_s its restriction to segment s and e_s = max |d_s|.  Derivation: a
    shift of every o_i by at most e_s moves v_max by at most e_s and Delta by
    2 e_s / 2^B, so (o_i + v) / Delta moves by at most
    (e_s + e_s + 2^B (2 e_s / 2^B)) / Delta = 4 e_s / Delta.  A decision
    compares L(u') with L(u) for the same o, u' one unit away from u: with
    g(o) = <u'/|u'| - u/|u|, o> the oracle's margin is |g| / <u/|u|, o>, and
    |g(o + d) - g(o)| <= 2 |d| / |u| (the normalised difference is at most
    2 |u' - u| / |u|), |u| >= sqrt(W) / 2 and <u, o> = L |u| |o| with L at
    least the cosine L0 of the initial code; so a flip needs a margin
    <= 4 |d_s| / (sqrt(W) L0 |o_s|), and kappa allows a quarter more for the
    change of the denominator.  The first place where the device's
    trajectory leaves the oracle's is such a dim; the moves that follow from
    it can differ far from any boundary, and the dim itself may end on the
    oracle's code again: those are the cascade.  Returns the counts."""
    counts = {"init": 0, "decision": 0, "cascade": 0, "unexplained": 0}
    diff = codes.astype(np.int64) - ref.codes
    if not np.any(diff):
        return counts
    assert ref.code_aux is not None and ref.seg_aux is not None, "instrumented oracle needed"
    err = np.broadcast_to(np.abs(np.asarray(err, np.float64)), ref.codes.shape)
    init0 = oracle.quantize(ref.O, plan.kept_widths, plan.kept_bits, 0).codes
    off = 0
    for s, (w, b) in enumerate(zip(plan.kept_widths, plan.kept_bits)):
        d = diff[:, off:off + w]
        rows = np.nonzero(np.any(d != 0, axis=1))[0]
        for r in rows:
            o = ref.O[r, off:off + w]
            es = err[r, off:off + w]
            on = float(np.sqrt(ref.seg_aux[r, s, 3]))
            delta = float(ref.seg_aux[r, s, 1])
            u0 = init0[r, off:off + w] - (2 ** b - 1) / 2
            L0 = float(u0 @ o / (np.linalg.norm(u0) * on)) if on > 0 else 1.0
            tau_i = 4.0 * float(es.max()) / delta if delta > 0 else np.inf
            kappa = (5.0 * float(np.linalg.norm(es)) / (np.sqrt(w) * max(L0, 1e-3) * on)
                     if on > 0 else np.inf)
            v = float(ref.seg_aux[r, s, 0])
            q = (o + v) / delta if delta > 0 else np.full(w, 0.5)
            im = np.abs(q - np.clip(np.rint(q), 1, 2 ** b - 1))
            dm = ref.code_aux[r, off:off + w, 1]
            at_init = im <= tau_i
            at_dec = dm <= kappa
            root = bool(np.any(at_init | at_dec))
            for i in np.nonzero(d[r])[0]:
                if at_init[i]:
                    counts["init"] += 1
                elif at_dec[i]:
                    counts["decision"] += 1
                elif root:
                    counts["cascade"] += 1
                else:
                    counts["unexplained"] += 1
        off += w
    return counts


def compare(plan, packed, fac, ref, max_rate=1e-4, factor_rtol=1e-5, label="",
            projected_input=False, dev_O=None):
    """The parity bar: >= 99.99 % identical codes; every difference exactly
    1 and at a rounding boundary of the oracle's computation (an init cell
    edge or a decision near-tie within the projection's error, or a cascade
    of one in the same segment; see classify_mismatches); factors within
    1e-5 relative where the segment's codes agree (else against the oracle's
    factor recomputed on the GPU's codes); the stored norm within 1e-6
    relative.  Returns the mismatch rate.

    With projected_input both sides quantized the same FP32 projected values,
    so no difference has a cause and the codes must agree.  End to end, the
    device's projected components of the same rows (dev_O [n, D_kept]) give
    the error the classification uses; without them the bound
    D u ||x - c|| per component that the projection tests check stands in
    (u = 2^-24)."""
    codes = saq.unpack_codes(plan, packed)
    # the packed record itself must be the oracle's packing of these codes
    assert np.array_equal(oracle.pack(codes, plan.kept_widths, plan.kept_bits), packed)
    diff = codes.astype(np.int64) - ref.codes
    rate = float(np.mean(diff != 0)) if diff.size else 0.0
    count = int(np.count_nonzero(diff))
    say(f"  [{label}] code mismatch rate {rate:.3e} ({count} of {diff.size})")
    assert rate <= max_rate or (max_rate > 0 and count <= 1), rate
    assert np.all(np.abs(diff) <= 1)
    if projected_input:
        err = np.zeros(1)
    elif dev_O is not None:
        err = np.abs(np.asarray(dev_O, np.float64)[:, :ref.codes.shape[1]] - ref.O)
    else:
        err = (plan.D * U32 * np.sqrt(ref.norm2))[:, None]
    cls = classify_mismatches(plan, codes, ref, err)
    if count:
        say(f"  [{label}] differing codes: {cls['init']} at an init cell edge, "
            f"{cls['decision']} at a decision near-tie, {cls['cascade']} cascaded, "
            f"{cls['unexplained']} unexplained")
    assert cls["unexplained"] == 0, cls
    k = len(plan.kept_widths)
    off = 0
    worst = 0.0
    for s, (w, b) in enumerate(zip(plan.kept_widths, plan.kept_bits)):
        same = np.all(diff[:, off:off + w] == 0, axis=1)
        f_ref = ref.factors[:, s]
        f_gpu = fac[:, s].astype(np.float64)
        err = np.abs(f_gpu[same] - f_ref[same])
        ok = err <= factor_rtol * np.abs(f_ref[same]) + 1e-30
        assert ok.all(), (s, np.max(err / np.maximum(np.abs(f_ref[same]), 1e-300)))
        if same.any():
            worst = max(worst, float(np.max(err / np.maximum(np.abs(f_ref[same]), 1e-300))))
        if (~same).any():
            o = ref.O[~same, off:off + w]
            u = codes[~same, off:off + w] - (2 ** b - 1) / 2
            f_rec = (o * o).sum(1) / (u * o).sum(1)
            assert np.all(np.abs(f_gpu[~same] - f_rec) <= factor_rtol * np.abs(f_rec))
        off += w
    say(f"  [{label}] worst factor relative error {worst:.2e}")
    assert np.allclose(fac[:, k], ref.norm2, rtol=1e-6, atol=0)
    return rate
