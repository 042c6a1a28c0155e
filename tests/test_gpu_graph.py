"""The encode and scan entry points under HIP graph capture.

They allocate nothing, clear nothing with memset and never synchronize, so a
caller can capture them (torch's CUDA graph API drives hipGraph on ROCm).
The graph is replayed several times with the program's own eager work and
synchronizations between the replays, and every replay must give exactly the
eager results, including after the input buffer is refilled in place."""
import numpy as np
import pytest

import synth
import paper_2509_12086_amd as saq
from gpu_util import cuda, say, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_encode_and_scans_replay_in_a_graph():
    ds = synth.cfg1(12_000)
    X1, X2 = ds.rows(0, 5000), ds.rows(5000, 10_000)
    plan = saq.Plan.fit(ds.rows(0, 4000), saq.PlanParams(bits_per_dim=4.0, fit_sample=0)).upload(0)
    n, nq = X1.shape[0], 40
    dev = cuda()
    Xd = to_dev(X1)
    Qd = to_dev(ds.queries(nq))
    codes = torch.empty((n, plan.code_bytes), dtype=torch.uint8, device=dev)
    fac = torch.empty((n, plan.n_factors), dtype=torch.float32, device=dev)
    ws = torch.empty(plan.encode_workspace_bytes(n), dtype=torch.uint8, device=dev)
    out = torch.empty((nq, n), dtype=torch.float32, device=dev)
    out_ms = torch.empty((nq, n), dtype=torch.float32, device=dev)
    stage = torch.empty((nq, n), dtype=torch.uint8, device=dev)
    wse = torch.empty(plan.estimate_workspace_bytes(nq), dtype=torch.uint8, device=dev)
    tau = torch.full((nq,), float(np.inf), dtype=torch.float32, device=dev)

    def run(stream=None):
        saq.encode(plan, Xd, 4, codes, fac, ws, stream)
        saq.estimate_dist(plan, Qd, codes, fac, out, wse, stream)
        saq.estimate_multistage(plan, Qd, codes, fac, tau, 4.0, out_ms, stage, wse, stream)

    def eager():
        run()
        torch.cuda.synchronize()
        return [t.clone() for t in (codes, fac, out, out_ms, stage)]

    want1 = eager()
    # tau from the eager scan: the 10th smallest estimate per query
    tau.copy_(torch.kthvalue(want1[2], 10, dim=1).values)
    want1 = eager()
    assert (want1[4] < len(plan.kept_widths)).any()            # the pruning is exercised
    Xd.copy_(to_dev(X2))
    want2 = eager()
    Xd.copy_(to_dev(X1))

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run(side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for i, (src, want) in enumerate(((X1, want1), (X1, want1), (X2, want2), (X1, want1))):
        say(f"graph replay {i}")
        for t in (codes, fac, out, out_ms, stage):
            t.zero_()                        # eager work between the replays
        Xd.copy_(to_dev(src))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for got, ref in zip((codes, fac, out, out_ms, stage), want):
            assert torch.equal(got, ref), i
