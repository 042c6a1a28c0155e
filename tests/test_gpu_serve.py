"""Serving loop on the GPU: requests of uneven sizes and budgets arrive while
others run; every request's result equals its result alone (bit for bit),
for encode requests and for estimate scans, and in-flight device memory
stays within the admission budget."""
import numpy as np
import pytest

import synth
import paper_2509_12086_amd as saq
from paper_2509_12086_amd.serve import ENCODE, SCAN, GpuBackend, Server, replay
from gpu_util import cuda, say, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    ds = synth.cfg4(60000)
    X = ds.rows()
    plans = {f"b{b}": saq.Plan.from_basis(np.zeros(ds.d), ds.rotation, ds.lam,
                                          saq.PlanParams(bits_per_dim=float(b))).upload(0)
             for b in (2, 4, 6)}
    return ds, X, plans


@pytest.mark.parametrize("split", [0, 1024])
def test_served_encodes_equal_alone(setup, split):
    """With split = 1024 every request above 1,024 vectors runs as chunks on
    several slots; its joined result must still be its result alone."""
    ds, X, plans = setup
    be = GpuBackend(0, slots=3)
    for pid, p in plans.items():
        be.add_plan(pid, p)
    budget = 512 << 20
    server = Server(be, hbm_budget=budget, max_batch_vectors=32768, split_vectors=split).start()
    t, size, bud = synth.poisson_requests(2000.0, 0.05, seed=7, hi=8192)
    trace, off = [], 0
    for ti, n, b in zip(t, size, bud):
        n = int(min(n, X.shape[0] - off))
        trace.append((float(ti), f"b{int(b)}", X[off:off + n], ENCODE))
        off = (off + n) % (X.shape[0] - 8192)
    say(f"serving {len(trace)} encode requests, {sum(len(x[2]) for x in trace)} vectors")
    reqs = replay(server, trace)
    server.drain(timeout=120)
    st = server.stats()
    say(f"  {st}")
    assert st["requests"] == len(trace) and st["rejected"] == 0
    assert st["max_inflight_bytes"] <= budget
    assert st["batches"] < len(trace)            # requests were batched together
    for r in reqs:
        codes, fac = r.wait(0)
        ac, af = saq.encode(plans[r.plan_id], to_dev(r.data), 4)
        torch.cuda.synchronize()
        assert np.array_equal(codes, ac.cpu().numpy()) and np.array_equal(fac, af.cpu().numpy())


def test_served_scans_mixed_with_encodes(setup):
    ds, X, plans = setup
    p = plans["b4"]
    store_c, store_f = saq.encode(p, to_dev(X[:20000]), 4)
    be = GpuBackend(0, slots=2)
    for pid, pl in plans.items():
        be.add_plan(pid, pl)
    be.add_store("b4", store_c, store_f)
    server = Server(be, hbm_budget=1 << 30).start()
    Q = ds.queries(64 * 4)
    trace = []
    for i in range(8):
        if i % 2 == 0:
            trace.append((0.001 * i, "b4", Q[64 * (i // 2): 64 * (i // 2 + 1)], SCAN))
        else:
            trace.append((0.001 * i, "b2", X[30000 + 100 * i: 30000 + 100 * i + 700], ENCODE))
    reqs = replay(server, trace)
    server.drain(timeout=120)
    for r in reqs:
        res = r.wait(0)
        if r.kind == SCAN:
            alone = saq.estimate_dist(p, to_dev(r.data), store_c, store_f)
            torch.cuda.synchronize()
            assert np.array_equal(res[0], alone.cpu().numpy())
        else:
            ac, af = saq.encode(plans["b2"], to_dev(r.data), 4)
            torch.cuda.synchronize()
            assert np.array_equal(res[0], ac.cpu().numpy()) and np.array_equal(res[1], af.cpu().numpy())
