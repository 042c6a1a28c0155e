"""The pre-split projection matrix the split-operand GEMM reads.

With FP32 accumulation the projection forms each FP32 product from operands
written exactly as three bf16 terms.  The plan builds M's terms on the host
and uploads them beside M.  Read back from the device buffer, the terms of
every entry must sum to the FP32 entry exactly, and each term must be the
round-to-nearest-even bf16 of what the earlier terms leave (so the first
term is within 2^-8 and the first two within 2^-16 of the entry, relative:
bf16 keeps 8 significant bits).
The chunk order is the GEMM's: [n_pad/128][k_pad/16][term][k half][row],
8 entries of one row per 16-byte chunk."""
import numpy as np
import pytest

import oracle
import synth
import paper_2509_12086_amd as saq
from gpu_util import say, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _bf16_value(h):
    return (h.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _rne_bf16(x32):
    u = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


@pytest.mark.parametrize("D,bpd", [(960, 4.0), (99, 3.0)])
def test_plan_split_terms_sum_to_M(D, bpd):
    X = synth.cfg2(4000).rows() if D == 960 else (
        np.random.default_rng(3).standard_normal((4000, D)) * np.exp(-np.arange(D) / 25.0)
    ).astype(np.float32)
    plan = saq.Plan.fit(X, saq.PlanParams(bits_per_dim=bpd, fit_sample=0)).upload(0)
    torch.cuda.synchronize()
    M, _, _ = plan.arrays()
    dk = plan.D_kept
    n_pad = max(128, -(-dk // 128) * 128)
    k_pad = -(-D // 32) * 32
    say(f"split M: D={D} D_kept={dk} n_pad={n_pad} k_pad={k_pad}")
    buf = plan._dev.cpu().numpy()
    off = (-plan._dev.data_ptr()) % 256
    off_ms = off                     # the first region of the plan buffer
    nchunk = (n_pad // 128) * (k_pad // 16) * 768
    h = buf[off_ms:off_ms + nchunk * 16].view(np.uint16)
    # [tile][step][term][half][row][e] -> [term][tile*128 + row][step*16 + half*8 + e]
    h = h.reshape(n_pad // 128, k_pad // 16, 3, 2, 128, 8).transpose(2, 0, 4, 1, 3, 5)
    h = h.reshape(3, n_pad, k_pad)
    Mp = np.zeros((n_pad, k_pad), np.float32)
    Mp[:dk, :D] = M
    t0, t1, t2 = (_bf16_value(h[i]) for i in range(3))
    assert np.array_equal(t0 + t1 + t2, Mp.astype(np.float64))      # exact (FP64 sum)
    assert np.array_equal(h[0], _rne_bf16(Mp))
    r1 = (Mp.astype(np.float64) - t0).astype(np.float32)            # exact in FP32
    assert np.array_equal(h[1], _rne_bf16(r1))
    r2 = (r1.astype(np.float64) - t1).astype(np.float32)
    assert np.array_equal(h[2], _rne_bf16(r2))
    a = np.abs(Mp.astype(np.float64))
    assert np.all(np.abs(Mp - t0) <= 2.0 ** -8 * a)
    assert np.all(np.abs(Mp - t0 - t1) <= 2.0 ** -16 * a)


@pytest.mark.parametrize("e", [-50, 50])
def test_encode_is_exactly_scale_equivariant(e):
    """Scaling X and c by 2^e commutes with every step of the encode: the
    three-term split, the MFMA products and FP32 sums, the grid, the FP64
    adjustment decisions and the factors.  So the records must be the
    unscaled ones bit for bit, the factors exactly 2^e times and the norms
    2^(2e) times, on both accumulations (FP32, and FP64 k-tile totals), on a
    ragged row count."""
    X = synth.cfg2(6000).rows()[:4999]
    mean, _, lam, V = oracle.pca(X)
    c0 = mean.astype(np.float32).astype(np.float64)
    s = np.float32(2.0 ** e)
    for mode in (1, 2):
        params = saq.PlanParams(bits_per_dim=4.0, projection_accumulation=mode)
        p0 = saq.Plan.from_basis(c0, V, lam, params).upload(0)
        p1 = saq.Plan.from_basis(c0 * 2.0 ** e, V, lam, params).upload(0)
        assert p0.widths == p1.widths and p0.bits == p1.bits
        assert np.array_equal(p0.arrays()[0], p1.arrays()[0])
        say(f"scale 2^{e}, accumulation mode {mode}")
        r0, f0 = saq.encode(p0, to_dev(X), 4)
        r1, f1 = saq.encode(p1, to_dev(X * s), 4)
        torch.cuda.synchronize()
        assert torch.equal(r0, r1)
        f0, f1 = f0.cpu().numpy().astype(np.float64), f1.cpu().numpy().astype(np.float64)
        k = len(p0.kept_widths)
        assert np.array_equal(f1[:, :k], f0[:, :k] * 2.0 ** e)
        assert np.array_equal(f1[:, k], f0[:, k] * 2.0 ** (2 * e))


@pytest.mark.parametrize("bits", [4, 8])
@pytest.mark.parametrize("D", [16, 32, 48, 64, 80, 100, 132, 200, 515])
def test_projection_k_loop_boundaries(D, bits):
    """The projection's k-loop runs its bulk with unconditional 16-byte loads
    and the ragged end through element loads.  Input dimensions around those
    boundaries (no bulk trips below 48, a ragged 16-byte tail at 100, odd D),
    FP32 accumulation (4-bit segment) and FP64 k-tile totals (8-bit): the
    projection stays within D FP32 unit roundoffs (2^-24) of ||x - c|| of the
    FP64 one, the norm is the FP64 ||x - c||^2 rounded once, and a misaligned
    copy of the same rows (element loads only) gives the same bits.  The
    bound holds for D >= 16 with room: one rounding of x - c, the split's
    dropped products (below 2^-23 relative) and six accumulator roundings
    per 16-wide k-step, each at most u times a sum bounded by ||x - c||
    (the rows of M are orthonormal)."""
    rng = np.random.default_rng(10 * D + bits)
    n = 333
    X = (rng.standard_normal((n, D)) * 3.0 + 5.0).astype(np.float32)
    c = (5.0 + 0.1 * rng.standard_normal(D)).astype(np.float32)
    Q, _ = np.linalg.qr(rng.standard_normal((D, D)))
    M = Q.T.astype(np.float32)
    widths = [D] if D <= 512 else [512, D - 512]
    plan = saq.Plan.from_parts(widths, [bits] * len(widths), M, c).upload(0)
    assert plan.info["projection_fp64_totals"] == (bits >= 8)
    say(f"projection D={D} bits={bits} fp64_totals={bits >= 8}")
    Xd = to_dev(X)
    O, n2 = saq.project(plan, Xd)
    buf = torch.empty(n * D + 1, dtype=torch.float32, device=Xd.device)
    buf[1:].copy_(Xd.reshape(-1))
    Xm = buf[1:].view(n, D)
    assert Xm.data_ptr() % 16 != 0
    O2, n22 = saq.project(plan, Xm)
    torch.cuda.synchronize()
    assert torch.equal(O, O2) and torch.equal(n2, n22)
    x64 = X.astype(np.float64) - c.astype(np.float64)
    ref = x64 @ M.astype(np.float64).T
    nref = (x64 ** 2).sum(1)
    err = np.abs(O.cpu().numpy()[:, :D] - ref)
    assert np.all(err <= D * 2.0 ** -24 * np.sqrt(nref)[:, None])
    # FP64 sums in another order, one FP32 rounding
    assert np.all(np.abs(n2.cpu().numpy() - nref) <= 2.0 ** -24 * nref * (1 + 1e-9))
