"""SAQ encode benchmark on one MI355X.

Workload (default): 1,000,000 x 960 FP32 vectors, a mixture of 1024 Gaussian
clusters with within-cluster std (i+1)^-0.5 under a random rotation (shaped
like the paper's 1M x 960 image-feature dataset, which is not available
here), 4 bits/dim average, 4 adjustment rounds.  One step = one full encode
of the whole batch (projection GEMM, quantization, adjustment, factors,
packing) with the input already resident in HBM.

Prints one JSON line: vectors/s, per-kernel roofline figures measured with
HIP events on the launch stream, and the FP64 oracle's CPU rate on a bounded
sample of the same rows.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3e12     # MI355X dense FP32 matrix FLOP/s
PEAK_HBM = 8.0e12             # MI355X HBM3E bytes/s
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock: lane-ops/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--bpd", type=float, default=4.0)
    ap.add_argument("--rounds", type=int, default=4)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the per-kernel loops (short runs under a profiler)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {a.gpus} is not supported "
              "(encoding shards by vectors with no exchange; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    import paper_2509_12086_amd as saq

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ds = synth.cfg2(a.n)
    t0 = time.time()
    X = ds.rows_torch(a.n, dev)
    fit_rows = X[: min(a.n, 65536)].cpu().numpy()
    plan = saq.Plan.fit(fit_rows, saq.PlanParams(bits_per_dim=a.bpd, fit_sample=0)).upload(0)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    n, D, dk = a.n, plan.D, plan.D_kept
    print(f"# setup {setup_s:.1f}s plan widths={plan.widths} bits={plan.bits} "
          f"D_kept={dk} code_bytes={plan.code_bytes}", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream(dev)
    codes = torch.empty((n, plan.code_bytes), dtype=torch.uint8, device=dev)
    fac = torch.empty((n, plan.n_factors), dtype=torch.float32, device=dev)
    ws = torch.empty(plan.encode_workspace_bytes(n), dtype=torch.uint8, device=dev)
    ld = (n + 3) // 4 * 4
    O = torch.empty((max(dk, 1), ld), dtype=torch.float32, device=dev)
    nrm = torch.empty(n, dtype=torch.float32, device=dev)

    def step():
        saq.encode(plan, X, a.rounds, codes, fac, ws, stream)

    ms_step = None
    if not a.kernels_only:
        for _ in range(a.warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(a.steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        ms_step = e0.elapsed_time(e1) / a.steps

    # per-kernel durations: the same two launches saq_encode makes, bracketed
    # by events on the launch stream
    def timed(fn, k):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        evs[0].record(stream)
        for i in range(k):
            fn()
            evs[i + 1].record(stream)
        torch.cuda.synchronize()
        d = [evs[i].elapsed_time(evs[i + 1]) for i in range(k)]
        return float(np.mean(d)), float(np.min(d))

    proj_ms, proj_min = timed(lambda: saq.project(plan, X, O, nrm, saq.LAYOUT_DIMS, stream),
                              a.steps)
    quant_ms, quant_min = timed(lambda: saq.quantize(plan, O, a.rounds, nrm, codes, fac,
                                                     saq.LAYOUT_DIMS, n, stream), a.steps)
    if ms_step is None:
        ms_step = proj_ms + quant_ms

    flops = 2.0 * D * dk * n
    proj_tflops = flops / (proj_ms * 1e-3) / 1e12
    q_bytes = n * (4.0 * dk + 4.0 + plan.code_bytes + 4.0 * plan.n_factors)
    q_gbs = q_bytes / (quant_ms * 1e-3) / 1e9
    e2e_bytes = n * (4.0 * D + plan.code_bytes + 4.0 * plan.n_factors)

    cpu = None
    if not a.no_cpu and not a.kernels_only:
        cpu = cpu_baseline(plan, X, a)

    out = {
        "metric": "SAQ encode vectors/s (D=960, 4 b/dim)" if a.bpd == 4.0 else
                  f"SAQ encode vectors/s (D=960, {a.bpd:g} b/dim)",
        "value": n / (ms_step * 1e-3),
        "unit": "vectors/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{n} x {D} FP32 cluster mixture (1024 centers, within-cluster std "
                        f"(i+1)^-0.5, random rotation), {a.bpd:g} b/dim, r={a.rounds}",
            "n": n, "D": D, "bits_per_dim": a.bpd, "rounds": a.rounds,
            "granularity": 16, "max_bits": 9, "max_width": 512,
            "segments": {"widths": plan.widths, "bits": plan.bits},
            "D_kept": dk, "code_bytes": plan.code_bytes,
        },
        "roofline": {
            "kernel": "project_kernel (FP32 MFMA GEMM, o = M (x - c))",
            "bound": "mfma",
            "achieved": proj_tflops,
            "peak": PEAK_FP32_MFMA / 1e12,
            "unit": "TFLOP/s",
            "frac": proj_tflops * 1e12 / PEAK_FP32_MFMA,
            "traffic": None,
            "algorithmic_per_launch": flops,
            "avg_ms": proj_ms,
        },
        "quantize_kernel": {
            "kernel": "quantize_kernel (grid code, adjustment, factors, packing)",
            "bound": "hbm",
            "achieved": q_gbs,
            "peak": PEAK_HBM / 1e9,
            "unit": "GB/s",
            "frac": q_gbs * 1e9 / PEAK_HBM,
            "algorithmic_per_launch": q_bytes,
            "avg_ms": quant_ms,
        },
        "end_to_end": {
            "bytes_per_vector": e2e_bytes / n,
            "hbm_frac": e2e_bytes / (ms_step * 1e-3) / PEAK_HBM,
            "binding_roofline_vectors_per_s": min(PEAK_HBM / (e2e_bytes / n),
                                                  PEAK_FP32_MFMA / (2.0 * D * dk)),
        },
        "cpu_baseline": cpu,
    }
    out["end_to_end"]["frac_of_binding"] = out["value"] / out["end_to_end"]["binding_roofline_vectors_per_s"]
    print(json.dumps(out), flush=True)


def cpu_baseline(plan, X, a):
    """The FP64 oracle on the host cores, on a bounded sample of the same rows."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    M, c, _ = plan.arrays()
    probe = X[:2000].cpu().numpy()
    t = time.time()
    oracle.encode(probe, M, c, plan.kept_widths, plan.kept_bits, a.rounds, threads=cores)
    rate = probe.shape[0] / (time.time() - t)
    m = int(min(a.n, max(2000, rate * a.cpu_seconds)))
    rows = X[:m].cpu().numpy()
    t = time.time()
    oracle.encode(rows, M, c, plan.kept_widths, plan.kept_bits, a.rounds, threads=cores)
    dt = time.time() - t
    return {"value": m / dt, "unit": "vectors/s", "cores": cores, "kind": "oracle",
            "sample": f"first {m} of the {a.n} rows, full encode (FP64 projection + Algorithm 1), "
                      f"{dt:.1f} s"}


if __name__ == "__main__":
    main()
