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


def compare(plan, packed, fac, ref, max_rate=1e-4, factor_rtol=1e-5, label=""):
    """Spec bar: >= 99.99 % identical codes, every difference exactly
    1; factors within 1e-5 relative where the segment's codes agree (else
    against the oracle's factor recomputed on the GPU's codes); the stored
    norm within 1e-6 relative.  Returns the mismatch rate."""
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
    for s, (w, b) in enumerate(zip(plan.kept_widths, plan.kept_bits)):
        same = np.all(diff[:, off:off + w] == 0, axis=1)
        f_ref = ref.factors[:, s]
        f_gpu = fac[:, s].astype(np.float64)
        ok = np.abs(f_gpu[same] - f_ref[same]) <= factor_rtol * np.abs(f_ref[same]) + 1e-30
        assert ok.all(), (s, np.max(np.abs(f_gpu[same] - f_ref[same]) / np.abs(f_ref[same])))
        if (~same).any():
            o = ref.O[~same, off:off + w]
            u = codes[~same, off:off + w] - (2 ** b - 1) / 2
            f_rec = (o * o).sum(1) / (u * o).sum(1)
            assert np.all(np.abs(f_gpu[~same] - f_rec) <= factor_rtol * np.abs(f_rec))
        off += w
    assert np.allclose(fac[:, k], ref.norm2, rtol=1e-6, atol=0)
    return rate
