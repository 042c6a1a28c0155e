"""Batched encode (many datasets with uneven segments, in one persistent
fused launch or in two grouped launches): every dataset's records are
bit-identical to its own plain saq_encode, for every launch shape the
autotuner may pick."""
import numpy as np
import pytest

import synth
import paper_2509_12086_amd as saq
from paper_2509_12086_amd import autotune
from gpu_util import compare, cuda, gpu_project, oracle_encode, say, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _basis_plan(ds, bpd, **kw):
    """Plan from the generating basis (rotation columns, spectrum)."""
    return saq.Plan.from_basis(np.zeros(ds.d), ds.rotation, ds.lam,
                               saq.PlanParams(bits_per_dim=bpd, **kw)).upload(0)


@pytest.fixture(scope="module")
def batch():
    sets = []
    ds = synth.cfg1(6000)
    X = ds.rows()
    sets.append((saq.Plan.fit(X, saq.PlanParams(bits_per_dim=4.0, fit_sample=0)).upload(0), X))
    ds = synth.cfg4(3000)
    sets.append((_basis_plan(ds, 6.0), ds.rows()))
    rng = np.random.default_rng(99)
    X = (rng.standard_normal((777, 99)) * np.exp(-np.arange(99) / 30.0)).astype(np.float32)
    sets.append((saq.Plan.fit(X, saq.PlanParams(bits_per_dim=2.0, granularity=8, max_width=32,
                                               fit_sample=0)).upload(0), X))
    ds = synth.cfg3(0, 1500)
    sets.append((_basis_plan(ds, 8.0), ds.rows()))
    ds = synth.cfg5(0, 1)
    sets.append((_basis_plan(ds, 3.0), ds.rows()))
    say("batch plans: " + "; ".join(f"D={p.D} W={p.kept_widths} B={p.kept_bits}" for p, _ in sets))
    return [(p, to_dev(X)) for p, X in sets]


def _plain(batch, rounds):
    out = []
    for p, X in batch:
        c, f = saq.encode(p, X, rounds)
        out.append((c, f))
    torch.cuda.synchronize()
    return [(c.cpu().numpy(), f.cpu().numpy()) for c, f in out]


@pytest.mark.parametrize("tuning", [
    saq.BatchTuning(),
    saq.BatchTuning(mode=saq.BATCH_FUSED, tile_rows=64),
    saq.BatchTuning(mode=saq.BATCH_GROUPED),
    saq.BatchTuning(mode=saq.BATCH_GROUPED, quant_waves=2, gemm_xcd_order=False),
    saq.BatchTuning(mode=saq.BATCH_GROUPED, quant_waves=4, gemm_xcd_order=True),
])
def test_batched_bit_identical_to_plain(batch, tuning):
    say(f"batched encode {tuning}")
    ref = _plain(batch, 4)
    ws = torch.empty(saq.batched_workspace_bytes(batch, tuning), dtype=torch.uint8, device=cuda())
    outs = saq.encode_batched(batch, 4, tuning, ws)
    torch.cuda.synchronize()
    for (c, f), (rc, rf), (p, _) in zip(outs, ref, batch):
        assert np.array_equal(c.cpu().numpy(), rc), p.D
        assert np.array_equal(f.cpu().numpy(), rf), p.D


@pytest.mark.parametrize("tuning", [
    saq.BatchTuning(),
    saq.BatchTuning(mode=saq.BATCH_FUSED, tile_rows=128),
    saq.BatchTuning(mode=saq.BATCH_FUSED, tile_rows=64),
    saq.BatchTuning(mode=saq.BATCH_GROUPED, tile_rows=128, quant_waves=2),
])
def test_batched_fp32_tiles_bit_identical_to_plain(batch, tuning):
    """Datasets that all accumulate in FP32 run the 128-row projection tile
    (two quantize waves per fused item) unless 64 rows are asked for."""
    ds = synth.cfg5(0, 2000)
    sub = [batch[0], batch[2], (_basis_plan(ds, 2.0), to_dev(ds.rows()))]
    assert not any(p.info["projection_fp64_totals"] for p, _ in sub)
    say(f"batched FP32-tile encode {tuning}")
    ref = _plain(sub, 4)
    for rep in range(2):          # the ticket is cleared before every launch
        outs = saq.encode_batched(sub, 4, tuning)
        torch.cuda.synchronize()
        for (c, f), (rc, rf), (p, _) in zip(outs, ref, sub):
            assert np.array_equal(c.cpu().numpy(), rc), (p.D, rep)
            assert np.array_equal(f.cpu().numpy(), rf), (p.D, rep)


def test_fused_launch_reuses_one_workspace(batch):
    """Back-to-back fused launches on one workspace (the ticket left at the
    item count by the first) and a graph-free stream order: the second
    launch's records are again the plain encoder's."""
    ws = torch.empty(saq.batched_workspace_bytes(batch), dtype=torch.uint8, device=cuda())
    ref = _plain(batch, 4)
    for _ in range(3):
        outs = saq.encode_batched(batch, 4, saq.BatchTuning(), ws)
    torch.cuda.synchronize()
    for (c, f), (rc, rf) in zip(outs, ref):
        assert np.array_equal(c.cpu().numpy(), rc) and np.array_equal(f.cpu().numpy(), rf)


def test_batched_with_empty_entry_and_rounds(batch):
    empty = (batch[0][0], batch[0][1][:0])
    sub = [batch[1], empty, batch[4]]
    for rounds in (0, 1, 7):
        ref = _plain([batch[1], batch[4]], rounds)
        outs = saq.encode_batched(sub, rounds)
        torch.cuda.synchronize()
        assert outs[1][0].shape[0] == 0
        for (c, f), (rc, rf) in zip([outs[0], outs[2]], ref):
            assert np.array_equal(c.cpu().numpy(), rc) and np.array_equal(f.cpu().numpy(), rf)


def test_batched_matches_oracle_wide_segments(batch):
    """The D=3072, 8 b/dim plan has 9-bit segments up to 512 wide (16-bit
    codes, one wave per quantize workgroup): compare with the oracle too."""
    p, X = batch[3]
    X = X[:300].contiguous()
    outs = saq.encode_batched([(p, X)], 4)
    torch.cuda.synchronize()
    c, f = outs[0]
    Xh = X.cpu().numpy()
    compare(p, c.cpu().numpy(), f.cpu().numpy(), oracle_encode(p, Xh, 4),
            label="batched D3072 b8", dev_O=gpu_project(p, Xh))


def test_batched_argument_errors(batch):
    with pytest.raises(ValueError):
        saq.encode_batched([batch[0]] * 17)
    p, X = batch[0]
    small = torch.empty(64, dtype=torch.uint8, device=cuda())
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.encode_batched([(p, X)], 4, workspace=small)
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.encode_batched([(p, X)], -2)
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.encode_batched([(p, X)], 4, saq.BatchTuning(quant_waves=3))
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.encode_batched([(p, X)], 4, saq.BatchTuning(mode=5))
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.encode_batched([(p, X)], 4, saq.BatchTuning(tile_rows=96))
    p8, X8 = batch[3]                     # FP64 k-tile totals take the 64-row tile
    assert p8.info["projection_fp64_totals"]
    with pytest.raises(saq.SaqError, match="SAQ_EINVAL"):
        saq.encode_batched([(p8, X8)], 4, saq.BatchTuning(tile_rows=128))
    # the reserved field of saq_batch_tuning must be 0
    import ctypes
    arr = saq._batch_struct([(p, X, None, None)])
    t = saq._Tuning(1, 1, 0, 0, 7)
    assert saq.lib().saq_encode_batched_workspace_bytes(arr, 1, ctypes.byref(t)) == -1


def test_autotuner_picks_a_valid_shape(batch):
    best, table = autotune.tune(batch[:3], rounds=4, reps=1, sample_rows=4096)
    assert len(table) == len(autotune.candidates(batch[:3]))
    assert best in [t for t, _ in table]
    again, table2 = autotune.tune(batch[:3], rounds=4)
    assert again == best and table2 == []           # cached
    outs = saq.encode_batched(batch[:3], 4, best)
    torch.cuda.synchronize()
    for (c, f), (rc, rf) in zip(outs, _plain(batch[:3], 4)):
        assert np.array_equal(c.cpu().numpy(), rc) and np.array_equal(f.cpu().numpy(), rf)


@pytest.mark.skip(reason="the single persistent launch with in-kernel waits between projection "
                         "and quantize work items did not finish on the GPU (twice); its cause "
                         "could not be shown on the CPU (a CPU model of its queue protocol is "
                         "deadlock-free), so that code path was removed and the batch runs as "
                         "two grouped launches instead")
def test_persistent_single_launch_pipeline():
    raise AssertionError("removed code path")


def test_cfg3_full_size_batched_sampled():
    """Four 1M x 3072 datasets (variance (i+1)^-1.2, budgets 1/2/4/8 b/dim,
    6-12 segments of widths 16-512 and 1-9 bits) through saq_encode_batched
    in the autotuned launch shape the benchmark times; 400 sampled records of
    each dataset compared with the oracle."""
    n = 1_000_000
    entries = []
    for i, b in enumerate((1.0, 2.0, 4.0, 8.0)):
        ds = synth.cfg3(i, n)
        say(f"cfg3 dataset {i}: generating {n} x 3072 on the device")
        entries.append((_basis_plan(ds, b, granularity=16, max_bits=9, max_width=512),
                        ds.rows_torch(n, cuda())))
    best, _ = autotune.tune(entries, rounds=4, reps=1)
    say(f"cfg3 batched encode, tuning {best}")
    outs = saq.encode_batched(entries, 4, best)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(5).choice(n, 400, replace=False))
    ti = torch.from_numpy(idx).to(cuda())
    for (p, X), (c, f) in zip(entries, outs):
        Xs = X[ti].cpu().numpy()
        compare(p, c[ti].cpu().numpy(), f[ti].cpu().numpy(), oracle_encode(p, Xs, 4),
                label=f"cfg3 D3072 {p.code_bytes * 8 // 3072} b/dim", dev_O=gpu_project(p, Xs))
    del entries, outs
    torch.cuda.empty_cache()
