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
PEAK_BF16_MFMA = 2.5e15       # MI355X dense bf16 matrix FLOP/s
SPLIT_PRODUCTS = 6            # bf16 MFMA products per FP32 product in the projection
PEAK_HBM = 8.0e12             # MI355X HBM3E bytes/s
PEAK_FP64_MFMA = 78.6e12      # MI355X dense FP64 matrix FLOP/s
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock: lane-ops/s


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "encode_1Mx960_b4_hbm_counters.md")


def kernel_code_digest() -> str:
    """sha256 of the encode kernels' code: csrc/device.hip followed by
    csrc/plan.hpp with comments removed, every run of blanks in a line made
    one space and empty lines dropped, so that an edit of comments or of
    indentation keeps the digest and a change of code changes it."""
    return code_digest("\n".join(open(os.path.join(ROOT, "paper_2509_12086_amd", "csrc", f),
                                       encoding="utf-8").read()
                                  for f in ("device.hip", "plan.hpp")))


def code_digest(src: str) -> str:
    """sha256 of C++ source text with comments removed (string and character
    literals kept as written), blanks in a line collapsed and empty lines
    dropped."""
    import hashlib
    import re
    lexeme = re.compile(r'("(?:\\.|[^"\\\n])*"|\'(?:\\.|[^\'\\\n])*\')|//[^\n]*|/\*.*?\*/', re.S)
    code = lexeme.sub(lambda m: m.group(1) if m.group(1) else " ", src)
    lines = (" ".join(line.split()) for line in code.splitlines())
    return hashlib.sha256("\n".join(x for x in lines if x).encode()).hexdigest()


def _record(path: str, tag: str, workload: str):
    """The machine-readable record of a committed counter summary, or None
    when it is for another workload or for other kernel code than the code
    built here."""
    try:
        text = open(path, encoding="utf-8").read()
        rec = json.loads(text.split(f"<!-- {tag} ", 1)[1].split(" -->", 1)[0])
        digest = kernel_code_digest()
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("workload") != workload or digest != rec.get("code_sha256"):
        return None
    return rec


INSTR_RECORD = os.path.join(ROOT, "profiles", "encode_1Mx960_b4_instruction_mix.md")


def recorded_valu(kernel: str, workload: str):
    """Wave-level VALU instructions per launch of `kernel` (rocprofv3
    SQ_INSTS_VALU), under the same conditions as recorded_traffic."""
    rec = _record(INSTR_RECORD, "instruction-record", workload)
    k = None if rec is None else rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("SQ_INSTS_VALU")


def recorded_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by a plain-copy calibration), or
    None when the summary is for another workload or for other kernel
    sources than the ones built here."""
    rec = _record(TRAFFIC_RECORD, "traffic-record", workload)
    k = None if rec is None else rec.get("kernels", {}).get(kernel)
    return None if k is None else k["read_bytes"] + k["write_bytes"]


CLOCK_RECORD = os.path.join(ROOT, "profiles", "encode_1Mx960_b4_clock_occupancy.md")


def recorded_cycles(kernel: str, workload: str):
    """GPU clock cycles per launch of `kernel` (rocprofv3 GRBM_GUI_ACTIVE / 8)
    and the counter run's other clock figures, under the same conditions as
    recorded_traffic."""
    rec = _record(CLOCK_RECORD, "clock-record", workload)
    return None if rec is None else rec.get("kernels", {}).get(kernel)


def clock_figures(rec, ms: float):
    """The clock a kernel ran at in this run: its recorded cycles per launch
    (constant for given kernel code and shape) over this run's time per
    launch; with the matrix-core busy cycles, the fraction of those cycles the
    matrix cores worked."""
    if rec is None:
        return None
    c = float(rec["cycles_per_launch"])
    out = {"cycles_per_launch": c, "effective_clock_ghz": c / (ms * 1e-3) / 1e9,
           "resident_waves_per_cu": rec.get("resident_waves_per_cu"),
           "source": "profiles/encode_1Mx960_b4_clock_occupancy.md"}
    if "mfma_busy_cycles_per_launch" in rec:
        out["mfma_busy_frac_of_cycles"] = rec["mfma_busy_cycles_per_launch"] / 1024 / c
    return out


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
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="length of the served-ingestion trace (0 = skip the serving legs)")
    ap.add_argument("--overload-rate", type=float, default=24000.0,
                    help="request rate of the serving overload point")
    ap.add_argument("--overload-seconds", type=float, default=4.0,
                    help="length of the serving overload point (0 = skip)")
    ap.add_argument("--mix-seconds", type=float, default=5.0,
                    help="length of the served multi-dataset mix")
    ap.add_argument("--batched-n", type=int, default=1_000_000,
                    help="vectors per dataset in the batched leg (0 = skip)")
    ap.add_argument("--scan-only", action="store_true",
                    help="only the estimate-scan leg (short runs under a profiler)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched leg (short runs under a profiler)")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the serving legs")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the per-kernel loops (short runs under a profiler)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (calibrates the "
                         "profiler's byte counters)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {a.gpus} is not supported. The encode "
              "shards by vectors with no exchange between GPUs (each holds the plan and "
              "encodes its own rows), so N GPUs run at N times one GPU's rate.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    import paper_2509_12086_amd as saq

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if a.batched_only:
        print(json.dumps({"batched": batched_leg(a)}), flush=True)
        return
    if a.scan_only:
        print(json.dumps({"estimate_scan": scan_leg(a)}), flush=True)
        return
    if a.serve_only:
        print(json.dumps({"serving": serve_leg(a), "serving_mix": serve_mix_leg(a)}), flush=True)
        return
    ds = synth.cfg2(a.n)
    t0 = time.time()
    X = ds.rows_torch(a.n, dev)
    fit_rows = X[: min(a.n, 65536)].cpu().numpy()
    stream = torch.cuda.current_stream(dev)
    head = encode_leg(a, X, fit_rows, a.bpd, stream, t0)
    plan, ms_step = head["plan"], head["ms_step"]
    n, D, dk = a.n, plan.D, plan.D_kept
    if a.copy_probe:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        for _ in range(3):
            dst.copy_(src)          # reads 1 GiB, writes 1 GiB per call
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not a.no_cpu and not a.kernels_only:
        cpu = cpu_baseline(plan, X, a)
    fit = None if a.kernels_only else fit_leg(a, X, fit_rows, stream)
    refs = None if a.kernels_only else ref_leg(a, ds, plan, X, head["codes"], head["fac"],
                                                head["ws"], stream, ms_step)
    for k in ("codes", "fac", "ws"):
        head.pop(k)
    other = None
    if not a.kernels_only:
        # the second budget of the headline configuration (2 and 4 b/dim)
        ob = 2.0 if a.bpd != 2.0 else 4.0
        leg = encode_leg(a, X, fit_rows, ob, stream, time.time())
        other = {"bits_per_dim": ob, "value": n / (leg["ms_step"] * 1e-3), "unit": "vectors/s",
                 "ms_per_step": leg["ms_step"],
                 "segments": {"widths": leg["plan"].widths, "bits": leg["plan"].bits},
                 "D_kept": leg["plan"].D_kept, "code_bytes": leg["plan"].code_bytes,
                 **{k: v for k, v in kernel_records(a, leg).items()}}
        del leg
    del X
    torch.cuda.empty_cache()
    batched = scans = None
    if a.batched_n > 0 and not a.kernels_only:
        batched = batched_leg(a)
    if not a.kernels_only:
        scans = scan_leg(a)
    serving = serving_mix = None
    if a.serve_seconds > 0 and not a.kernels_only:
        serving = serve_leg(a)
        serving_mix = serve_mix_leg(a)

    recs = kernel_records(a, head)
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
        **recs,
        "other_budget": other,
        "cpu_baseline": cpu,
        "fit": fit,
        "reference_vectors": refs,
        "batched": batched,
        "estimate_scan": scans,
        "serving": serving,
        "serving_mix": serving_mix,
    }
    print(json.dumps(out), flush=True)


def encode_leg(a, X, fit_rows, bpd, stream, t0):
    """Fit the plan at `bpd` b/dim on the first 65,536 rows, then time the
    whole encode step (warm-up, then `steps` steps between two events on the
    launch stream) and each of its two kernels alone (the same launches,
    each bracketed by events on that stream)."""
    import torch
    import paper_2509_12086_amd as saq
    dev = X.device
    plan = saq.Plan.fit(fit_rows, saq.PlanParams(bits_per_dim=bpd, fit_sample=0)).upload(0)
    torch.cuda.synchronize()
    n, dk = X.shape[0], plan.D_kept
    print(f"# setup {time.time() - t0:.1f}s {bpd:g} b/dim plan widths={plan.widths} "
          f"bits={plan.bits} D_kept={dk} code_bytes={plan.code_bytes}", file=sys.stderr,
          flush=True)
    codes = torch.empty((n, plan.code_bytes), dtype=torch.uint8, device=dev)
    fac = torch.empty((n, plan.n_factors), dtype=torch.float32, device=dev)
    ws = torch.empty(plan.encode_workspace_bytes(n), dtype=torch.uint8, device=dev)

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

    O = torch.empty(((n + 63) // 64, max(dk, 1), 64), dtype=torch.float32, device=dev)
    nrm = torch.empty(n, dtype=torch.float32, device=dev)

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
        return float(np.mean(d))

    proj_ms = timed(lambda: saq.project(plan, X, O, nrm, saq.LAYOUT_TILES, stream), a.steps)
    quant_ms = timed(lambda: saq.quantize(plan, O, a.rounds, nrm, codes, fac, saq.LAYOUT_TILES,
                                          n, stream), a.steps)
    del O, nrm
    if ms_step is None:
        ms_step = proj_ms + quant_ms
    return {"plan": plan, "bpd": bpd, "n": n, "ms_step": ms_step, "proj_ms": proj_ms,
            "quant_ms": quant_ms, "codes": codes, "fac": fac, "ws": ws}


TRIAL_LANE_OPS = 6   # per Algorithm 1 trial with the division-free accept rule: two
                     # multiply-adds, two compares, two range compares


def kernel_records(a, leg):
    """Roofline records of one encode leg, every figure on the method's own
    work: the projection's 2 D D_kept FLOP per vector, the quantize kernel's
    algorithmic bytes, Algorithm 1's 2 r D_kept trials per vector."""
    plan, n = leg["plan"], leg["n"]
    D, dk = plan.D, plan.D_kept
    proj_ms, quant_ms, ms_step = leg["proj_ms"], leg["quant_ms"], leg["ms_step"]
    flops = 2.0 * D * dk * n
    proj_bytes = n * (4.0 * D + 4.0 * dk + 4.0)        # read X, write O and ||x - c||^2
    workload = f"{n:,} x {D}, {leg['bpd']:g} b/dim, r={a.rounds}"
    q_valu = recorded_valu("quantize_kernel", workload)
    achieved = flops / (proj_ms * 1e-3)
    acc64 = bool(plan.info["projection_fp64_totals"])
    q_bytes = n * (4.0 * dk + 4.0 + plan.code_bytes + 4.0 * plan.n_factors)
    q_rate = q_bytes / (quant_ms * 1e-3)
    e2e_bytes = n * (4.0 * D + plan.code_bytes + 4.0 * plan.n_factors)
    lane_ops = TRIAL_LANE_OPS * 2.0 * a.rounds * dk       # per vector
    bind = {"hbm": PEAK_HBM / (e2e_bytes / n),
            "mfma_bf16": PEAK_BF16_MFMA / (flops / n)}
    if lane_ops > 0:                                      # no trials at --rounds 0
        bind["valu"] = VALU_LANE_OPS / lane_ops
    bound = min(bind, key=bind.get)
    return {
        "roofline": {
            "kernel": ("project_kernel (o = M (x - c) on the bf16 matrix cores: FP32 products "
                       "as six bf16 products of exactly split operands, " +
                       ("FP64 k-tile totals)" if acc64 else "FP32 accumulation)")),
            "bound": "mfma",
            "achieved": achieved / 1e12,
            "peak": PEAK_BF16_MFMA / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_BF16_MFMA,
            "traffic": recorded_traffic("project_kernel", workload),
            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)",
            "work": "2 D D_kept FLOP per vector (the method's projection)",
            "algorithmic_per_launch": flops,
            "algorithmic_bytes_per_launch": proj_bytes,
            "avg_ms": proj_ms,
            "frac_of_fp32_mfma_peak": achieved / PEAK_FP32_MFMA,
            "clock": clock_figures(recorded_cycles("project_kernel", workload), proj_ms),
            "split_emulation": {
                "note": "matrix-core work issued by the six bf16 products per FP32 product: "
                        "MFMA utilisation, not the method's work",
                "bf16_products_per_fp32_product": SPLIT_PRODUCTS,
                "issued_tflops": SPLIT_PRODUCTS * achieved / 1e12,
                "frac_of_bf16_peak": SPLIT_PRODUCTS * achieved / PEAK_BF16_MFMA},
        },
        "quantize_kernel": {
            "kernel": "quantize_kernel (grid code, adjustment, factors, packing)",
            "bound": "alu",
            "hbm_target": {"figure": "HBM roofline fraction of the quantize kernel "
                                     "(algorithmic bytes / time / 8 TB/s)",
                           "value": q_rate / PEAK_HBM, "target": 0.6},
            "hbm": {"achieved": q_rate / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                    "frac": q_rate / PEAK_HBM, "algorithmic_per_launch": q_bytes,
                    "traffic": recorded_traffic("quantize_kernel", workload)},
            "valu": None if q_valu is None else {
                "achieved": q_valu * 64 / (quant_ms * 1e-3), "peak": VALU_LANE_OPS,
                "unit": "lane-ops/s", "frac": q_valu * 64 / (quant_ms * 1e-3) / VALU_LANE_OPS,
                "instructions_per_launch": q_valu},
            "clock": clock_figures(recorded_cycles("quantize_kernel", workload), quant_ms),
            "avg_ms": quant_ms,
        },
        "end_to_end": {
            "bytes_per_vector": e2e_bytes / n,
            "flops_per_vector": flops / n,
            "trial_lane_ops_per_vector": lane_ops,
            "hbm_frac": e2e_bytes / (ms_step * 1e-3) / PEAK_HBM,
            "binding_roofline_vectors_per_s": bind[bound],
            "binding_unit": bound,
            "roofline_vectors_per_s": bind,
            "frac_of_binding": n / (ms_step * 1e-3) / bind[bound],
        },
    }


def ref_leg(a, ds, plan, X, codes, fac, ws, stream, plain_ms):
    """Encode with a reference vector per record (saq_encode_ref): the 1,024
    cluster centers of the headline data as IVF list centroids, each record
    on its nearest one (assigned outside the timed region).  Same plan and
    launch shapes as the headline step; only the centering differs."""
    import torch
    import paper_2509_12086_amd as saq
    dev = X.device
    refs = torch.from_numpy((ds.centers @ ds.rotation.T).astype(np.float32)).to(dev)
    rn = (refs.double() ** 2).sum(1)
    rt = refs.double().T.contiguous()
    ids = torch.empty(X.shape[0], dtype=torch.int32, device=dev)
    for a0 in range(0, X.shape[0], 65536):
        xb = X[a0:a0 + 65536].double()
        ids[a0:a0 + xb.shape[0]] = torch.argmin(rn[None, :] - 2.0 * (xb @ rt), dim=1).to(torch.int32)
    del rt
    step = lambda: saq.encode(plan, X, a.rounds, codes, fac, ws, stream, refs=refs, ref_ids=ids)
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(a.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.steps
    del refs, ids
    return {"workload": f"{X.shape[0]} x {X.shape[1]}, 1024 list centroids, nearest per record, "
                        f"{a.bpd:g} b/dim, r={a.rounds}",
            "ms_per_step": ms, "vectors_per_s": X.shape[0] / (ms * 1e-3),
            "plain_ms_per_step": plain_ms}


def fit_leg(a, X, fit_rows, stream):
    """Section 4.1's fit with the rows on the device: mean and covariance on
    the FP64 matrix cores, the eigen-decomposition by device Jacobi, the plan
    search on the host. Timed on the 65,536 rows the headline plan is fitted
    on (D = 960), against the host fit of the same rows; the covariance and
    the eigen-decomposition alone at D = 960 and 3072."""
    import torch
    import synth
    import paper_2509_12086_amd as saq
    params = saq.PlanParams(bits_per_dim=a.bpd, fit_sample=0)
    m = fit_rows.shape[0]
    Xs = X[:m]
    t0 = time.time()
    saq.Plan.fit(fit_rows, params)
    host_s = time.time() - t0
    saq.Plan.fit_device(Xs, params, stream=stream)
    torch.cuda.synchronize()
    t0 = time.time()
    saq.Plan.fit_device(Xs, params, stream=stream)
    dev_s = time.time() - t0

    def cov_ms(Y, k=3):
        mean, cov = saq.covariance(Y, 0, stream=stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(k):
            saq.covariance(Y, 0, mean, cov, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    def eig_ms(Y):
        _, cov = saq.covariance(Y, 0, stream=stream)
        saq.sym_eigen(cov, stream=stream)
        torch.cuda.synchronize()
        t0 = time.time()
        saq.sym_eigen(cov, stream=stream)
        torch.cuda.synchronize()
        return (time.time() - t0) * 1e3

    rows = []
    for D, Y in ((Xs.shape[1], Xs), (3072, None)):
        if Y is None:
            Y = synth.cfg3(0, m).rows_torch(m, X.device)
        ms = cov_ms(Y)
        flop = float(m) * D * (D + 1)          # upper triangle, multiply and add
        rows.append({"D": D, "rows": m, "covariance_ms": ms,
                     "tflops_fp64": flop / (ms * 1e-3) / 1e12,
                     "frac_fp64_mfma": flop / (ms * 1e-3) / PEAK_FP64_MFMA,
                     "eigen_ms": eig_ms(Y)})
        del Y
    torch.cuda.empty_cache()
    return {"workload": f"fit on {m} rows: D = {Xs.shape[1]} (the headline plan's rows) and "
                        f"D = 3072 (covariance and eigen-decomposition only)",
            "host_fit_s": host_s, "device_fit_s": dev_s, "covariance": rows}


def batched_leg(a):
    """Batched uneven segments: 4 datasets of n x 3072 (variance (i+1)^-1.2,
    random rotation, one dataset per budget 1/2/4/8 b/dim), encoded by the
    two grouped launches of saq_encode_batched with the launch shape the
    autotuner picks, against the plain encoder run once per dataset."""
    import torch
    import synth
    import paper_2509_12086_amd as saq
    from paper_2509_12086_amd import autotune
    dev = torch.device("cuda", 0)
    n = a.batched_n
    budgets = (1.0, 2.0, 4.0, 8.0)
    entries = []
    for i, b in enumerate(budgets):
        ds = synth.cfg3(i, n)
        plan = saq.Plan.from_basis(np.zeros(ds.d), ds.rotation, ds.lam,
                                   saq.PlanParams(bits_per_dim=b, granularity=16, max_bits=9,
                                                  max_width=512)).upload(0)
        X = ds.rows_torch(n, dev)
        codes = torch.empty((n, plan.code_bytes), dtype=torch.uint8, device=dev)
        fac = torch.empty((n, plan.n_factors), dtype=torch.float32, device=dev)
        entries.append((plan, X, codes, fac))
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    print(f"# batched leg: {len(entries)} x {n} x 3072, plans "
          + "; ".join(f"{b:g}b: {len(p.kept_widths)} kept segs W {min(p.kept_widths)}-"
                      f"{max(p.kept_widths)} B {min(p.kept_bits)}-{max(p.kept_bits)}"
                      for b, (p, *_) in zip(budgets, entries)), file=sys.stderr, flush=True)

    def timed(fn, k, warm):
        for _ in range(warm):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    steps = max(1, min(a.steps, 3))
    # plain: one saq_encode per dataset, sharing one workspace
    ws = torch.empty(max(p.encode_workspace_bytes(n) for p, *_ in entries), dtype=torch.uint8,
                     device=dev)
    plain_ms = timed(lambda: [saq.encode(p, X, a.rounds, c, f, ws, stream)
                              for p, X, c, f in entries], steps, 1)
    ref = [(c.clone(), f.clone()) for _, _, c, f in entries]
    del ws
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    best, table = autotune.tune([(p, X) for p, X, _, _ in entries], rounds=a.rounds, reps=2)
    tune_s = time.perf_counter() - t0
    wsb = torch.empty(saq.batched_workspace_bytes(entries, best), dtype=torch.uint8, device=dev)
    batched_ms = timed(lambda: saq.encode_batched(entries, a.rounds, best, wsb, stream), steps, 1)
    identical = all(torch.equal(c, rc) and torch.equal(f, rf)
                    for (_, _, c, f), (rc, rf) in zip(entries, ref))
    flops = sum(2.0 * p.D * p.D_kept * n for p, *_ in entries)
    del wsb, ref
    torch.cuda.empty_cache()

    # many small datasets: 16 slices of 8,192 rows (4 per plan); here the
    # two grouped launches replace 32 plain ones
    small_n = 8192
    small = [(p, X[j * small_n:(j + 1) * small_n]) for p, X, _, _ in entries for j in range(4)]
    small = [(p, X, torch.empty((small_n, p.code_bytes), dtype=torch.uint8, device=dev),
              torch.empty((small_n, p.n_factors), dtype=torch.float32, device=dev))
             for p, X in small]
    ws = torch.empty(max(p.encode_workspace_bytes(small_n) for p, *_ in small), dtype=torch.uint8,
                     device=dev)
    s_plain = timed(lambda: [saq.encode(p, X, a.rounds, c, f, ws, stream)
                             for p, X, c, f in small], 10, 2)
    s_best, _ = autotune.tune([(p, X) for p, X, _, _ in small], rounds=a.rounds, reps=3)
    wss = torch.empty(saq.batched_workspace_bytes(small, s_best), dtype=torch.uint8, device=dev)
    s_batched = timed(lambda: saq.encode_batched(small, a.rounds, s_best, wss, stream), 10, 2)
    del small, ws, wss
    out = {
        "workload": f"{len(entries)} datasets x {n} x 3072, variance (i+1)^-1.2, random rotation; "
                    "budgets 1/2/4/8 b/dim (one per dataset), r=" + str(a.rounds),
        "plans": [{"bits_per_dim": b, "kept_widths": p.kept_widths, "kept_bits": p.kept_bits,
                   "segments": len(p.widths),
                   "fp64_k_tile_totals": bool(p.info["projection_fp64_totals"])}
                  for b, (p, *_) in zip(budgets, entries)],
        "plain_vectors_per_s": len(entries) * n / (plain_ms * 1e-3),
        "plain_ms": plain_ms,
        "batched_vectors_per_s": len(entries) * n / (batched_ms * 1e-3),
        "batched_ms": batched_ms,
        "batched_over_plain": plain_ms / batched_ms,
        "projection_tflops_batched": flops / (batched_ms * 1e-3) / 1e12,
        "records_identical_to_plain": identical,
        "small": {"datasets": 16, "rows_each": small_n,
                  "plain_ms": s_plain, "batched_ms": s_batched,
                  "plain_vectors_per_s": 16 * small_n / (s_plain * 1e-3),
                  "batched_vectors_per_s": 16 * small_n / (s_batched * 1e-3),
                  "batched_over_plain": s_plain / s_batched,
                  "tuning": _tuning_dict(s_best)},
        "autotune": {"best": _tuning_dict(best),
                     "seconds": tune_s,
                     "table_ms": [dict(_tuning_dict(t), ms=ms) for t, ms in table]},
    }
    del entries
    torch.cuda.empty_cache()
    return out


def _tuning_dict(t):
    import paper_2509_12086_amd as saq
    if t.mode == saq.BATCH_FUSED:
        return {"mode": "fused", "tile_rows": t.tile_rows}
    return {"mode": "grouped", "tile_rows": t.tile_rows, "quant_waves": t.quant_waves,
            "gemm_xcd_order": t.gemm_xcd_order}


def serve_leg(a):
    """Served ingestion: Poisson arrivals at 2,000 requests/s, D=768 rows
    with variance exp(-i/96), sizes lognormal (median 512, sigma 1.5)
    clipped to [1, 65536], budgets uniform over {2, 4, 6} bits/dim (three
    resident plans), for --serve-seconds.  Rows come from a pinned host
    pool; latency runs from arrival to the codes and factors being back on
    the host.  Then an overload point: the same stream at --overload-rate
    requests/s for --overload-seconds, past what the host link and the
    scheduler sustain, reporting the throughput actually served."""
    import torch
    import synth
    import paper_2509_12086_amd as saq
    from paper_2509_12086_amd.serve import ENCODE, GpuBackend, Server, replay
    dev = torch.device("cuda", 0)
    ds = synth.cfg4(262144)
    pool = ds.rows_torch(ds.n, dev).cpu().pin_memory()
    plans = {b: saq.Plan.from_basis(np.zeros(ds.d), ds.rotation, ds.lam,
                                    saq.PlanParams(bits_per_dim=float(b))).upload(0)
             for b in (2, 4, 6)}

    def make_trace(rate, seconds, seed):
        t, size, bud = synth.poisson_requests(rate, seconds, seed=seed)
        trace, off = [], 0
        for ti, n, b in zip(t, size, bud):
            n = int(n)
            if off + n > pool.shape[0]:
                off = 0
            trace.append((float(ti), int(b), pool[off:off + n], ENCODE))
            off += n
        return trace

    be = GpuBackend(0, slots=4, rounds=a.rounds)
    for b, p in plans.items():
        be.add_plan(b, p)
    # warm-up: one request per plan, and one split request
    server = Server(be, hbm_budget=32 << 30).start()
    for b in plans:
        server.submit(b, pool[:1024]).wait(60)
    server.submit(4, pool[:40000]).wait(60)
    server.drain()

    def run(trace, seconds):
        server = Server(be, hbm_budget=32 << 30, keep_results=False).start()
        replay(server, trace)
        server.drain(timeout=600)
        st = server.stats()
        offered = sum(x[2].shape[0] for x in trace) / seconds
        return st, offered

    trace = make_trace(2000.0, a.serve_seconds, 41)
    st, offered = run(trace, a.serve_seconds)
    over = None
    if a.overload_seconds > 0:
        otrace = make_trace(a.overload_rate, a.overload_seconds, 43)
        ost, ooff = run(otrace, a.overload_seconds)
        over = {"rate_req_per_s": a.overload_rate, "seconds": a.overload_seconds,
                "requests": ost["requests"], "offered_vectors_per_s": ooff,
                "sustained_vectors_per_s": ost["vectors_per_s"],
                "p50_ms": ost["p50_ms"], "p99_ms": ost["p99_ms"], "max_queue": ost["max_queue"]}
    # the plain single-launch encoder on the same vectors, already on the device
    per_b = {}
    for _, b, x, _ in trace:
        per_b[b] = per_b.get(b, 0) + x.shape[0]
    total = sum(per_b.values())
    Xd = pool[: min(pool.shape[0], max(per_b.values()))].to(dev)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for b, cnt in per_b.items():
        left = cnt
        while left > 0:
            m = min(left, Xd.shape[0])
            saq.encode(plans[b], Xd[:m], a.rounds)
            left -= m
    e1.record()
    torch.cuda.synchronize()
    plain = total / (e0.elapsed_time(e1) * 1e-3)
    del Xd, pool
    return {
        "workload": f"Poisson 2000 req/s for {a.serve_seconds:g} s, D=768 exp(-i/96), sizes "
                    "lognormal(median 512, sigma 1.5) clipped to [1, 65536], budgets {2,4,6} b/dim",
        "server": {"slots": be.slots, "max_batch_vectors": 262144, "split_vectors": 0,
                   "launch": "grouped", "buffers": "per slot, reused",
                   "gc": "paused while serving"},
        "requests": st["requests"], "rejected": st["rejected"], "batches": st["batches"],
        "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
        "served_vectors_per_s": st["vectors_per_s"],
        "offered_vectors_per_s": offered,
        "plain_encoder_vectors_per_s": plain,
        "max_queue": st["max_queue"],
        "overload": over,
    }


def multistage_timing(plan, Q, codes, fac, plain_out, ws, stream, k, m=4.0, sub=16384):
    """Multi-stage scan (Section 4.3) at the paper's default m = 4.  Each
    query's threshold is its 10th smallest estimate over the first 16,384
    records (a pruning threshold a search would hold after a first probe).
    Reports the time per scan, the code bits read per (query, record) pair,
    the share of pairs closed early, and the share of the full scan's 10
    nearest that stay open; then the same for a single query, where each
    workgroup holds one query's pairs and can stop early."""
    import torch
    import paper_2509_12086_amd as saq
    nq, n = plain_out.shape
    dev = plain_out.device
    part = torch.empty((nq, sub), dtype=torch.float32, device=dev)
    saq.estimate_dist(plan, Q, codes[:sub], fac[:sub], part, ws, stream)
    tau = torch.kthvalue(part, 10, dim=1).values.contiguous()
    saq.estimate_dist(plan, Q, codes, fac, plain_out, ws, stream)
    top = torch.topk(plain_out, 10, dim=1, largest=False).indices
    out = torch.empty_like(plain_out)
    stage = torch.empty((nq, n), dtype=torch.uint8, device=dev)
    seg_bits = [w * b for w, b in zip(plan.kept_widths, plan.kept_bits)]
    cum = torch.tensor(np.concatenate([[0], np.cumsum(seg_bits)]), dtype=torch.float64, device=dev)
    kk = len(seg_bits)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    ms = timed(lambda: saq.estimate_multistage(plan, Q, codes, fac, tau, m, out, stage, ws, stream))
    st = stage.long()
    res = {"m": m, "ms_per_scan": ms,
           "bits_per_pair": float(cum[st].mean()), "bits_full": int(sum(seg_bits)),
           "closed_frac": float((st < kk).double().mean()),
           "top10_open_frac": float((torch.gather(st, 1, top) == kk).double().mean())}
    q1, t1, o1, s1 = Q[:1], tau[:1], out[:1], stage[:1]
    res["nq1_plain_ms"] = timed(lambda: saq.estimate_dist(plan, q1, codes, fac, o1, ws, stream))
    res["nq1_ms"] = timed(lambda: saq.estimate_multistage(plan, q1, codes, fac, t1, m, o1, s1, ws,
                                                          stream))
    res["nq1_bits_per_pair"] = float(cum[s1.long()].mean())
    del part, out, stage, st
    return res


def scan_products_per_dim(plan, prefix_bits=0):
    """bf16 matrix-core products the plain scan issues per kept dim and
    query-record pair, averaged over the kept dims.  Plans whose kept widths
    are all multiples of 16 and whose 32-dim steps would leave at least a
    quarter of the steps to padding take packed steps with the scaled codes
    split in three terms: six products.  Every other plan steps segment by
    segment with the codes' c - h as one exact term (two above 8 bits read)
    against the query's three: three products, or five."""
    ws, bs = plan.kept_widths, plan.kept_bits
    if not ws:
        return 0.0
    steps = sum((w + 31) // 32 for w in ws)
    if all(w % 16 == 0 for w in ws) and 4 * ((sum(ws) + 31) // 32) <= 3 * steps:
        return float(SPLIT_PRODUCTS)
    used = [prefix_bits if 0 < prefix_bits < b else b for b in bs]
    return sum(w * (5 if u > 8 else 3) for w, u in zip(ws, used)) / sum(ws)


def scan_leg(a):
    """Estimate scans (Section 3.2): 64 queries against 1M stored records
    encoded at 4 b/dim, for D = 128, 768, 1536 and 3072 (variance
    exp(-8i/D)); the scan kernel contracts the records' codes with the
    projected queries on the bf16 matrix cores at FP32 accuracy (exact
    split operands; scan_products_per_dim gives the products issued)."""
    import torch
    import synth
    import paper_2509_12086_amd as saq
    dev = torch.device("cuda", 0)
    n, nq = 1_000_000, 64
    stream = torch.cuda.current_stream(dev)
    rows = []
    for i in (0, 2, 4, 6):
        ds = synth.cfg5(i, n)
        plan = saq.Plan.from_basis(np.zeros(ds.d), ds.rotation, ds.lam,
                                   saq.PlanParams(bits_per_dim=4.0)).upload(0)
        X = ds.rows_torch(n, dev)
        codes, fac = saq.encode(plan, X, a.rounds)
        del X
        Q = ds.rows_torch(nq, dev, seed_offset=2)
        out = torch.empty((nq, n), dtype=torch.float32, device=dev)
        ws = torch.empty(plan.estimate_workspace_bytes(nq), dtype=torch.uint8, device=dev)
        for _ in range(2):
            saq.estimate_dist(plan, Q, codes, fac, out, ws, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        k = 5
        for _ in range(k):
            saq.estimate_dist(plan, Q, codes, fac, out, ws, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / k
        flops = 2.0 * nq * plan.D_kept * n
        row = {"D": ds.d, "D_kept": plan.D_kept, "code_bytes": plan.code_bytes,
               "ms_per_scan": ms, "tflops": flops / (ms * 1e-3) / 1e12,
               "frac_bf16_mfma": flops / (ms * 1e-3) / PEAK_BF16_MFMA,
               "bf16_products_per_fp32_product": scan_products_per_dim(plan),
               "issued_frac_bf16_mfma": scan_products_per_dim(plan) * flops / (ms * 1e-3) / PEAK_BF16_MFMA,
               "frac_fp32_mfma": flops / (ms * 1e-3) / PEAK_FP32_MFMA,
               "record_GBps": n * (plan.code_bytes + 4 * plan.n_factors) / (ms * 1e-3) / 1e9}
        if ds.d == 3072:
            # progressive approximation: only the first b bit planes are read
            pre = {}
            for b in (1, 2, 4):
                saq.estimate_dist(plan, Q, codes, fac, out, ws, stream, prefix_bits=b)
                torch.cuda.synchronize()
                e0.record(stream)
                for _ in range(k):
                    saq.estimate_dist(plan, Q, codes, fac, out, ws, stream, prefix_bits=b)
                e1.record(stream)
                torch.cuda.synchronize()
                pre[str(b)] = e0.elapsed_time(e1) / k
            row["prefix_ms_per_scan"] = pre
        row["multistage"] = multistage_timing(plan, Q, codes, fac, out, ws, stream, k)
        rows.append(row)
        del codes, fac, out, ws
    torch.cuda.empty_cache()
    return {"workload": f"{nq} queries x {n} records, 4 b/dim, D in 128/768/1536/3072", "scans": rows}


def serve_mix_leg(a):
    """Served multi-dataset mix: 8 resident datasets (D = 128, 128, 768, 768,
    1536, 1536, 3072, 3072; variance exp(-8i/D); 4 b/dim plans), each with
    1M stored records.  Poisson arrivals at 100 requests/s: 80 % encode
    requests of log-uniform 1..131,072 vectors, 20 % estimate scans of 64
    queries over the dataset's 1M stored records; datasets uniform; HBM
    budget 64 GiB.  Latency runs from arrival to the results on the host."""
    import torch
    import synth
    import paper_2509_12086_amd as saq
    from paper_2509_12086_amd.serve import ENCODE, SCAN, GpuBackend, Server, replay
    dev = torch.device("cuda", 0)
    n_store, pool_n, rate = 1_000_000, 131_072, 100.0
    be = GpuBackend(0, slots=4, rounds=a.rounds)
    pools, queries = {}, {}
    for i in range(len(synth.CFG5_DIMS)):
        ds = synth.cfg5(i, n_store)
        pid = f"d{i}"
        plan = saq.Plan.from_basis(np.zeros(ds.d), ds.rotation, ds.lam,
                                   saq.PlanParams(bits_per_dim=4.0)).upload(0)
        be.add_plan(pid, plan)
        X = ds.rows_torch(n_store, dev)
        be.add_store(pid, *saq.encode(plan, X, a.rounds))
        del X
        pools[pid] = ds.rows_torch(pool_n, dev, seed_offset=1).cpu().pin_memory()
        queries[pid] = ds.rows_torch(64, dev, seed_offset=2).cpu().pin_memory()
    torch.cuda.synchronize()
    rng = np.random.default_rng(52)
    t = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * a.mix_seconds * 1.5) + 10))
    t = t[t < a.mix_seconds]
    trace, offs = [], {pid: 0 for pid in pools}
    for ti in t:
        pid = f"d{rng.integers(len(pools))}"
        if rng.random() < 0.2:
            trace.append((float(ti), pid, queries[pid], SCAN))
            continue
        n = int(min(pool_n, max(1, round(np.exp(rng.uniform(0.0, np.log(pool_n)))))))
        if offs[pid] + n > pool_n:
            offs[pid] = 0
        trace.append((float(ti), pid, pools[pid][offs[pid]:offs[pid] + n], ENCODE))
        offs[pid] += n
    budget = 64 << 30
    warm = Server(be, hbm_budget=budget, keep_results=False).start()
    for pid in pools:
        warm.submit(pid, pools[pid][:1024])
        warm.submit(pid, queries[pid], SCAN)
    warm.drain()
    server = Server(be, hbm_budget=budget, keep_results=False).start()
    replay(server, trace)
    server.drain(timeout=600)
    st = server.stats()
    scans = st["by_kind"][SCAN]["count"]
    out = {
        "workload": f"8 resident datasets (D {'/'.join(str(d) for d in synth.CFG5_DIMS)}, "
                    f"4 b/dim, 1M stored records each); Poisson {rate:g} req/s for "
                    f"{a.mix_seconds:g} s, 80 % encodes of log-uniform 1..131072 vectors, "
                    "20 % 64-query estimate scans over 1M records; HBM budget 64 GiB",
        "requests": st["requests"], "rejected": st["rejected"], "batches": st["batches"],
        "encode": st["by_kind"][ENCODE], "scan": st["by_kind"][SCAN],
        "encoded_vectors_per_s": st["vectors_per_s"],
        "scanned_query_record_pairs_per_s": scans * n_store * 64 / a.mix_seconds,
        "max_inflight_bytes": st["max_inflight_bytes"],
        "max_queue": st["max_queue"],
    }
    del be, pools, queries
    torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo", encoding="utf-8"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(plan, X, a):
    """The FP64 oracle on the host cores, on bounded samples of the same rows:
    every core the process may use (OpenMP over vectors), then one core."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    M, c, _ = plan.arrays()

    def rate_on(threads, seconds):
        probe = X[:2000].cpu().numpy() if threads > 1 else X[:300].cpu().numpy()
        t = time.time()
        oracle.encode(probe, M, c, plan.kept_widths, plan.kept_bits, a.rounds, threads=threads)
        r = probe.shape[0] / (time.time() - t)
        m = int(min(a.n, max(probe.shape[0], r * seconds)))
        rows = X[:m].cpu().numpy()
        t = time.time()
        oracle.encode(rows, M, c, plan.kept_widths, plan.kept_bits, a.rounds, threads=threads)
        dt = time.time() - t
        return m / dt, m, dt

    v, m, dt = rate_on(cores, a.cpu_seconds)
    v1, m1, dt1 = rate_on(1, a.cpu_seconds * 0.75)
    return {"value": v, "unit": "vectors/s", "cores": cores, "kind": "oracle",
            "sample": f"first {m} of the {a.n} rows, full encode (FP64 projection + Algorithm 1), "
                      f"{dt:.1f} s on {cores} threads",
            "cpu": cpu_model(),
            "one_core": {"value": v1, "unit": "vectors/s", "cores": 1,
                         "sample": f"first {m1} rows, {dt1:.1f} s on 1 thread"}}


if __name__ == "__main__":
    main()
