"""Autotuner for the batched encode launches.

It picks the launch shape of saq_encode_batched for a batch by timing
candidates on the batch itself (or on its first rows):
  * mode            one persistent fused launch, or two grouped launches
  * tile_rows       projection tile rows: 128 (FP32 accumulation only) or 64
  * quant_waves     grouped mode: waves (64 vectors each) per quantize
                    workgroup: {1, 2, 4} (fewer when their LDS code buffers
                    would not fit)
  * gemm_xcd_order  grouped mode: XCD-aware or row-major order of the
                    projection tiles
Results are cached per batch signature (dimensions, plans, sizes rounded to a
power of two, round limit), in memory and optionally in a JSON file.
Every candidate gives bit-identical records; only the time differs.
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional, Sequence, Tuple

from . import BATCH_FUSED, BATCH_GROUPED, BatchTuning, encode_batched, batched_workspace_bytes

_CACHE: Dict[str, BatchTuning] = {}


def _cus() -> int:
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count


def signature(entries, rounds: int) -> str:
    parts = []
    for e in entries:
        plan, X = e[0], e[1]
        n = int(X.shape[0])
        parts.append((plan.D, tuple(plan.widths), tuple(plan.bits), 1 << max(n - 1, 0).bit_length()))
    return json.dumps([parts, rounds])


def candidates(entries=()) -> List[BatchTuning]:
    """Launch shapes for a batch: 128-row tiles only when no dataset takes
    FP64 k-tile totals (those run the 64-row tile)."""
    any64 = any(bool(e[0].info["projection_fp64_totals"]) for e in entries)
    rows = (64,) if any64 else (128, 64)
    out = [BatchTuning(mode=BATCH_FUSED, tile_rows=r) for r in rows]
    out += [BatchTuning(mode=BATCH_GROUPED, tile_rows=r, quant_waves=w, gemm_xcd_order=x)
            for r in rows for w in (1, 2, 4) for x in (True, False)]
    return out


def tune(entries, rounds: int = 4, reps: int = 2, sample_rows: int = 131072,
         cache_file: Optional[str] = None, verbose: bool = False
         ) -> Tuple[BatchTuning, List[Tuple[BatchTuning, float]]]:
    """Time every candidate on (the first ``sample_rows`` rows of) each
    dataset and return (best tuning, [(tuning, ms), ...])."""
    import torch
    sig = signature(entries, rounds)
    if sig in _CACHE:
        return _CACHE[sig], []
    if cache_file and os.path.exists(cache_file):
        stored = _read_cache(cache_file)
        if sig in stored:
            _CACHE[sig] = BatchTuning(**stored[sig])
            return _CACHE[sig], []
    sub = [(e[0], e[1][:sample_rows]) for e in entries]
    cands = candidates(entries)
    need = max(batched_workspace_bytes(sub, t) for t in cands)
    ws = torch.empty(need, dtype=torch.uint8, device=sub[0][1].device)
    outs = encode_batched(sub, rounds, cands[0], ws)         # allocate outputs once
    full = [(p, X, c, f) for (p, X), (c, f) in zip(sub, outs)]
    stream = torch.cuda.current_stream()
    table = []
    for t in cands:
        encode_batched(full, rounds, t, ws)                  # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            encode_batched(full, rounds, t, ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        table.append((t, ms))
        if verbose:
            print(f"  autotune {t} -> {ms:.3f} ms", flush=True)
    best = min(table, key=lambda r: r[1])[0]
    _CACHE[sig] = best
    if cache_file:
        stored = _read_cache(cache_file) if os.path.exists(cache_file) else {}
        stored[sig] = {"quant_waves": best.quant_waves, "gemm_xcd_order": best.gemm_xcd_order,
                       "mode": best.mode, "tile_rows": best.tile_rows}
        with open(cache_file, "w", encoding="utf-8") as f:
            json.dump(stored, f)
    return best, table


def _read_cache(path: str) -> dict:
    with open(path, encoding="utf-8") as f:
        return json.load(f)
