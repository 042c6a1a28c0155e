"""Host side of the benchmark (no GPU needed): its one-GPU contract and its
link to the committed counter records.

`roofline.traffic`, the VALU figures and the clock figures come from rocprofv3 counter runs kept
as text under profiles/.  They are reported only while the kernel code is the
code the counters were taken on, keyed by a digest of the code with comments
and blanks removed: an edit of comments must keep the digest, any edit of code
must change it."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEVICE = os.path.join(ROOT, "paper_2509_12086_amd", "csrc", "device.hip")


def test_comment_and_blank_edits_keep_the_digest():
    src = open(DEVICE, encoding="utf-8").read()
    base = bench.code_digest(src)
    assert bench.code_digest("// a new first line\n" + src) == base
    assert bench.code_digest(src.replace("\n", "\n\n")) == base
    assert bench.code_digest(src.replace("    ", "\t")) == base
    assert bench.code_digest(src + "\n/* a block comment\n   over two lines */\n") == base
    # a comment reflowed over more lines
    assert bench.code_digest("int a; // one two three\n") == bench.code_digest("int a; // one\n// two three\n")


def test_code_edits_change_the_digest():
    src = open(DEVICE, encoding="utf-8").read()
    base = bench.code_digest(src)
    assert "SK" in src
    assert bench.code_digest(src.replace("SK", "SK2", 1)) != base
    assert bench.code_digest(src + "\nstatic int unused_probe;\n") != base
    # comment markers inside literals are code, not comments
    assert bench.code_digest('const char* s = "a // b";\n') != bench.code_digest('const char* s = "a ";\n')
    assert bench.code_digest("char c = '/'; int d; // x\n") != bench.code_digest("char c = '*'; int d;\n")
    # line structure is kept (a preprocessor line must not absorb the next)
    assert bench.code_digest("#define A 1\nint b;\n") != bench.code_digest("#define A 1 int b;\n")


def test_records_are_keyed_by_the_code_digest():
    """Each committed record carries a code digest; a record for another
    digest or another workload is not reported."""
    for path, tag in ((bench.TRAFFIC_RECORD, "traffic-record"), (bench.INSTR_RECORD, "instruction-record"),
                      (bench.CLOCK_RECORD, "clock-record")):
        text = open(path, encoding="utf-8").read()
        assert f"<!-- {tag} " in text and '"code_sha256": "' in text
        assert bench._record(path, tag, "another workload") is None


def test_more_than_one_gpu_exits_with_a_message():
    """The benchmark measures one GPU: --gpus N > 1 exits with status 2 and a
    message on stderr, before touching a GPU, and prints no result line."""
    for n in (2, 8):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                           capture_output=True, text=True, timeout=60)
        assert r.returncode == 2
        assert f"--gpus {n} is not supported" in r.stderr
        assert r.stdout == ""


def test_roofline_fractions_price_the_methods_own_work():
    """roofline.frac is the projection's 2 D D_kept FLOP per vector over the
    measured time and the bf16 matrix-core peak; the six emulation products
    appear only in their own labelled record; the end-to-end binding
    roofline takes the method's bytes, FLOPs and trial lane-ops per vector."""
    from types import SimpleNamespace
    plan = SimpleNamespace(D=960, D_kept=864, code_bytes=480, n_factors=8,
                           info={"projection_fp64_totals": 0})
    a = SimpleNamespace(rounds=4)
    n = 1_000_000
    leg = {"plan": plan, "n": n, "bpd": 4.0, "proj_ms": 9.0, "quant_ms": 3.5, "ms_step": 12.8}
    r = bench.kernel_records(a, leg)
    flops = 2.0 * 960 * 864 * n
    assert abs(r["roofline"]["frac"] - flops / 9.0e-3 / 2.5e15) < 1e-12
    assert r["roofline"]["algorithmic_per_launch"] == flops
    assert abs(r["roofline"]["split_emulation"]["frac_of_bf16_peak"]
               - 6 * r["roofline"]["frac"]) < 1e-12
    q_bytes = n * (4.0 * 864 + 4.0 + 480 + 4.0 * 8)
    assert abs(r["quantize_kernel"]["hbm"]["frac"] - q_bytes / 3.5e-3 / 8e12) < 1e-12
    e = r["end_to_end"]
    assert e["bytes_per_vector"] == 4.0 * 960 + 480 + 32
    assert e["roofline_vectors_per_s"]["mfma_bf16"] == 2.5e15 / (2.0 * 960 * 864)
    assert e["binding_roofline_vectors_per_s"] == min(e["roofline_vectors_per_s"].values())
    assert abs(e["frac_of_binding"] - n / 12.8e-3 / e["binding_roofline_vectors_per_s"]) < 1e-12


def test_clock_figures_follow_the_recorded_cycles():
    """The effective clock is the recorded cycles per launch over this run's
    time per launch, and the matrix-core busy fraction is the busy cycles per
    SIMD (1,024 SIMDs) over those cycles; without a record there is no clock
    figure, and zero adjustment rounds leave the VALU bound out."""
    rec = {"cycles_per_launch": 1.6e7, "resident_waves_per_cu": 11.0,
           "mfma_busy_cycles_per_launch": 1024 * 8.0e6}
    c = bench.clock_figures(rec, 10.0)
    assert abs(c["effective_clock_ghz"] - 1.6) < 1e-12
    assert abs(c["mfma_busy_frac_of_cycles"] - 0.5) < 1e-12
    assert "mfma_busy_frac_of_cycles" not in bench.clock_figures({"cycles_per_launch": 1e6}, 1.0)
    assert bench.clock_figures(None, 1.0) is None
    from types import SimpleNamespace
    plan = SimpleNamespace(D=960, D_kept=864, code_bytes=480, n_factors=8,
                           info={"projection_fp64_totals": 0})
    leg = {"plan": plan, "n": 1000, "bpd": 4.0, "proj_ms": 1.0, "quant_ms": 1.0, "ms_step": 2.0}
    r = bench.kernel_records(SimpleNamespace(rounds=0), leg)
    assert "valu" not in r["end_to_end"]["roofline_vectors_per_s"]


def test_scan_products_per_dim_follows_the_scan_path():
    """The bf16 products the bench counts per FP32 product: six for plans the
    scan runs with packed k-steps (kept widths all multiples of 16, packing
    saving at least a quarter of the 32-dim steps), otherwise three per dim,
    five in segments with more than 8 bits read, averaged over the kept dims."""
    import numpy as np
    import paper_2509_12086_amd as saq

    def plan(widths, bits):
        D = sum(widths)
        k = sum(w for w, b in zip(widths, bits) if b > 0)
        return saq.Plan.from_parts(widths, bits, np.eye(D, dtype=np.float32)[:k], np.zeros(D, np.float32))

    # six 16-dim segments: 3 packed steps instead of 6
    assert bench.scan_products_per_dim(plan([16] * 6, [9, 7, 6, 5, 3, 2])) == 6.0
    # multiples of 16 where packing saves under a quarter: segment by segment
    p = plan([64, 48, 32], [9, 4, 2])
    assert bench.scan_products_per_dim(p) == (64 * 5 + 48 * 3 + 32 * 3) / 144
    # ragged widths; a prefix of 3 bits reads no segment above 8 bits
    p = plan([13, 37, 70, 9], [16, 9, 4, 2])
    assert bench.scan_products_per_dim(p) == (13 * 5 + 37 * 5 + 70 * 3 + 9 * 3) / 129
    assert bench.scan_products_per_dim(p, prefix_bits=3) == 3.0
    # a dropped trailing segment does not count
    assert bench.scan_products_per_dim(plan([20, 12], [3, 0])) == 3.0
