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


def gpu_encode(plan, X, rounds=4):
    import torch
    codes, fac = saq.encode(plan, to_dev(X.astype(np.float32)), rounds)
    torch.cuda.synchronize()
    return codes.cpu().numpy(), fac.cpu().numpy()


def oracle_encode(plan, X, rounds=4, instrument=False):
    M, c, _ = plan.arrays()
    return oracle.encode(X, M, c, plan.kept_widths, plan.kept_bits, rounds, instrument)


def oracle_records(plan, X, rounds=4):
    """Records encoded and packed by the oracle, for the scans' parity tests:
    (packed uint8 [n, code_bytes], factors float32 [n, k + 1], codes int32
    [n, D_kept]).  Both sides then read the same bytes and the same FP32
    factors, and nothing the oracle reads comes from the device."""
    enc = oracle_encode(plan, X, rounds)
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


def compare(plan, packed, fac, ref, max_rate=1e-4, factor_rtol=1e-5, label="",
            projected_input=False):
    """The parity bar: >= 99.99 % identical codes, every difference exactly
    1; factors within 1e-5 relative where the segment's codes agree (else
    against the oracle's factor recomputed on the GPU's codes); the stored
    norm within 1e-6 relative.  Returns the mismatch rate.

    With projected_input both sides quantized the same FP32 projected values
    and the factor bar is exactly 1e-5.  End to end, the device's o carries
    the rounding of its FP32 projection: under the probabilistic model of
    FP32 accumulation each component is off by about sqrt(D) u ||x - c||, and
    f_s = ||o_s||^2 / <u_s, o_s> moves by about twice that relative to
    ||o_s||, so that amount is allowed on top of 1e-5."""
    codes = saq.unpack_codes(plan, packed)
    # the packed record itself must be the oracle's packing of these codes
    assert np.array_equal(oracle.pack(codes, plan.kept_widths, plan.kept_bits), packed)
    diff = codes.astype(np.int64) - ref.codes
    rate = float(np.mean(diff != 0)) if diff.size else 0.0
    count = int(np.count_nonzero(diff))
    say(f"  [{label}] code mismatch rate {rate:.3e} ({count} of {diff.size})")
    assert rate <= max_rate or (max_rate > 0 and count <= 1), rate
    assert np.all(np.abs(diff) <= 1)
    k = len(plan.kept_widths)
    off = 0
    xn = np.sqrt(ref.norm2)
    worst = 0.0
    for s, (w, b) in enumerate(zip(plan.kept_widths, plan.kept_bits)):
        o_seg = ref.O[:, off:off + w]
        if projected_input:
            rtol = np.full(len(o_seg), factor_rtol)
        else:
            on = np.sqrt((o_seg ** 2).sum(1))
            with np.errstate(divide="ignore", invalid="ignore"):
                rtol = factor_rtol + np.where(on > 0, 2.0 * np.sqrt(plan.D) * U32 * xn / on, 0.0)
        same = np.all(diff[:, off:off + w] == 0, axis=1)
        f_ref = ref.factors[:, s]
        f_gpu = fac[:, s].astype(np.float64)
        err = np.abs(f_gpu[same] - f_ref[same])
        ok = err <= rtol[same] * np.abs(f_ref[same]) + 1e-30
        assert ok.all(), (s, np.max(err / np.maximum(np.abs(f_ref[same]), 1e-300)))
        if same.any():
            worst = max(worst, float(np.max(err / np.maximum(np.abs(f_ref[same]), 1e-300))))
        if (~same).any():
            o = ref.O[~same, off:off + w]
            u = codes[~same, off:off + w] - (2 ** b - 1) / 2
            f_rec = (o * o).sum(1) / (u * o).sum(1)
            assert np.all(np.abs(f_gpu[~same] - f_rec) <= rtol[~same] * np.abs(f_rec))
        off += w
    say(f"  [{label}] worst factor relative error {worst:.2e}")
    assert np.allclose(fac[:, k], ref.norm2, rtol=1e-6, atol=0)
    return rate
