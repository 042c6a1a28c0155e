"""Scheduling and admission logic of the serving loop, on the CPU, with a
stand-in backend and a manual clock (the GPU path is in test_gpu_serve.py)."""
import numpy as np
import pytest

from paper_2509_12086_amd.serve import ENCODE, Rejected, Server


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeBatch:
    def __init__(self, be, groups):
        self.be, self.groups = be, groups
        self.t_done = be.clock() + be.duration
        be.launches.append(groups)

    def done(self):
        return self.be.clock() >= self.t_done

    def finish(self):
        out = []
        for kind, pid, reqs in self.groups:
            for r in reqs:
                # a per-row function: each row's result depends on that row only
                out.append((r, (r.data.sum(axis=1) * self.be.scale[pid],)))
        return out


class FakeBackend:
    def __init__(self, clock, slots=2, bytes_per_row=100, duration=1.0, fail_plan=None):
        self.clock, self.slots = clock, slots
        self.bytes_per_row, self.duration = bytes_per_row, duration
        self.scale = {"a": 1.0, "b": 2.0, "c": 3.0}
        self.launches = []
        self.fail_plan = fail_plan

    def footprint(self, kind, pid, n):
        return n * self.bytes_per_row

    def launch(self, slot, groups):
        if self.fail_plan and any(pid == self.fail_plan for _, pid, _ in groups):
            raise RuntimeError("device error")
        return FakeBatch(self, groups)


def rows(n, seed):
    return np.random.default_rng(seed).standard_normal((n, 4)).astype(np.float32)


def test_admission_by_memory_and_continuous_batching():
    clk = Clock()
    be = FakeBackend(clk, slots=2, duration=1.0)
    s = Server(be, hbm_budget=1000, clock=clk)
    r1 = s.submit("a", rows(4, 1))      # 400 B
    r2 = s.submit("a", rows(4, 2))      # 400 B
    r3 = s.submit("b", rows(4, 3))      # 400 B: would exceed 1000
    s.step()
    assert r1.batch_id == r2.batch_id == 0 and r3.batch_id is None
    assert s.used == 800 and len(be.launches) == 1
    assert len(be.launches[0]) == 1 and be.launches[0][0][1] == "a"   # one entry per plan
    clk.t = 0.5
    r4 = s.submit("c", rows(1, 4))      # arrives while the first batch runs
    s.step()
    # the head request r3 does not fit the free 200 B; r4 must not overtake it
    assert r3.batch_id is None and r4.batch_id is None
    clk.t = 1.0
    s.step()
    assert r1.finished == 1.0 and r1.latency == 1.0
    assert r3.batch_id == 1 and r4.batch_id == 1 and s.used == 500
    clk.t = 2.0
    s.step()
    for r in (r1, r2, r3, r4):
        np.testing.assert_array_equal(r.wait(0)[0], r.data.sum(axis=1) * be.scale[r.plan_id])


def test_oversize_request_rejected_at_submission():
    clk = Clock()
    s = Server(FakeBackend(clk), hbm_budget=1000, clock=clk)
    r = s.submit("a", rows(11, 0))
    with pytest.raises(Rejected):
        r.wait(0)
    assert s.rejected == 1 and not s.queue


def test_batch_limits_plans_and_vectors():
    clk = Clock()
    be = FakeBackend(clk, slots=1, bytes_per_row=1)
    s = Server(be, hbm_budget=10 ** 9, max_batch_vectors=10, clock=clk)
    reqs = [s.submit("a", rows(4, i)) for i in range(3)]   # 12 vectors > 10
    s.step()
    assert [r.batch_id for r in reqs] == [0, 0, None]
    many = Server(FakeBackend(clk, slots=1, bytes_per_row=1), hbm_budget=10 ** 9, clock=clk)
    many.be.scale = {f"p{i}": 1.0 for i in range(20)}
    rs = [many.submit(f"p{i}", rows(1, i)) for i in range(20)]
    many.step()
    assert sum(r.batch_id == 0 for r in rs) == 16           # at most 16 plans per batch


def test_cancel_while_queued_and_failed_batch_isolated():
    clk = Clock()
    be = FakeBackend(clk, slots=1, fail_plan="b")
    s = Server(be, hbm_budget=10 ** 6, max_batch_vectors=4, clock=clk)
    ra = s.submit("a", rows(4, 0))
    rb = s.submit("b", rows(4, 1))
    rc = s.submit("a", rows(4, 2))
    assert s.cancel(rc) and rc.cancelled
    s.step()                       # ra launches
    clk.t = 1.0
    s.step()                       # ra done; rb's launch fails, only rb
    assert ra.wait(0) is not None
    with pytest.raises(RuntimeError, match="device error"):
        rb.wait(0)
    with pytest.raises(RuntimeError, match="cancelled"):
        rc.wait(0)
    assert s.used == 0 and not s.inflight


def test_threaded_loop_drains_and_reports():
    import time
    be = FakeBackend(time.monotonic, slots=3, duration=0.002)
    s = Server(be, hbm_budget=10 ** 6, clock=time.monotonic).start()
    reqs = [s.submit("abc"[i % 3], rows(1 + i % 5, i)) for i in range(60)]
    s.drain(timeout=30)
    st = s.stats()
    assert st["requests"] == 60 and st["rejected"] == 0 and st["batches"] >= 1
    assert st["p99_ms"] >= st["p50_ms"] >= 0
    for r in reqs:
        np.testing.assert_array_equal(r.wait(0)[0], r.data.sum(axis=1) * be.scale[r.plan_id])
