"""Host side of the benchmark (no GPU needed): its one-GPU contract and its
link to the committed counter records.

`roofline.traffic` and the VALU figures come from rocprofv3 counter runs kept
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
    for path, tag in ((bench.TRAFFIC_RECORD, "traffic-record"), (bench.INSTR_RECORD, "instruction-record")):
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
