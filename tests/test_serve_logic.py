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

    def finish(self, keep=True):
        out = []
        for kind, pid, reqs in self.groups:
            for r in reqs:
                # a per-row function: each row's result depends on that row only
                out.append((r, (r.data.sum(axis=1) * self.be.scale[pid],) if keep else None))
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


def test_large_request_split_into_chunks_across_slots():
    """An encode request above split_vectors goes out as chunks, in arrival
    order with the other requests, on several slots at once; it completes
    with its last chunk and its result is its rows' results in order."""
    clk = Clock()
    be = FakeBackend(clk, slots=3, bytes_per_row=1, duration=1.0)
    s = Server(be, hbm_budget=10 ** 6, max_batch_vectors=4, split_vectors=4, clock=clk)
    big = s.submit("a", rows(10, 1))          # chunks of 4, 4, 2
    small = s.submit("b", rows(2, 2))
    assert len(s.queue) == 4 and s.max_queue == 4
    s.step()                                   # three slots: two chunks, then chunk 3 + small
    assert [c.batch_id for c in big.chunks] == [0, 1, 2] and small.batch_id == 2
    clk.t = 1.0
    s.step()
    assert big.finished == 1.0 and small.finished == 1.0
    np.testing.assert_array_equal(big.wait(0)[0], big.data.sum(axis=1))
    st = s.stats()
    assert st["requests"] == 2 and st["encoded_vectors"] == 12


def test_split_request_cancel_and_failure():
    clk = Clock()
    be = FakeBackend(clk, slots=1, bytes_per_row=1, fail_plan="b")
    s = Server(be, hbm_budget=10 ** 6, max_batch_vectors=4, split_vectors=4, clock=clk)
    blocker = s.submit("a", rows(4, 0))
    r = s.submit("a", rows(9, 1))
    assert s.cancel(r) and r.cancelled and len(s.queue) == 1
    with pytest.raises(RuntimeError, match="cancelled"):
        r.wait(0)
    s.step()                                   # blocker runs
    bad = s.submit("b", rows(9, 2))            # every chunk's launch fails
    assert not s.cancel(blocker)               # already on the device
    for t in (1.0, 2.0, 3.0, 4.0):
        clk.t = t
        s.step()
    with pytest.raises(RuntimeError, match="device error"):
        bad.wait(0)
    assert blocker.wait(0) is not None and s.used == 0 and not s.queue
    assert s.stats()["requests"] == 1


def test_chunk_footprint_decides_rejection():
    """A request that fits the budget only chunk by chunk is admitted."""
    clk = Clock()
    s = Server(FakeBackend(clk, bytes_per_row=100), hbm_budget=1000, split_vectors=5, clock=clk)
    r = s.submit("a", rows(20, 0))             # 2000 B whole, 500 B per chunk
    assert r.error is None and len(r.chunks) == 4
    s2 = Server(FakeBackend(clk, bytes_per_row=100), hbm_budget=1000, split_vectors=0, clock=clk)
    with pytest.raises(Rejected):
        s2.submit("a", rows(20, 0)).wait(0)


def test_size_classes_keep_small_requests_off_the_large_slot():
    clk = Clock()
    be = FakeBackend(clk, slots=3, bytes_per_row=1, duration=1.0)
    s = Server(be, hbm_budget=10 ** 6, max_batch_vectors=100, large_vectors=8,
               large_slots=1, clock=clk)
    big1 = s.submit("a", rows(20, 1))
    big2 = s.submit("a", rows(90, 2))
    small = [s.submit("b", rows(3, i)) for i in range(3)]
    s.step()
    # slot 0 takes the large ones (20 + 90 > 100: one of them), slots 1-2 the small
    assert big1.batch_id == 0 and big2.batch_id is None
    assert {r.batch_id for r in small} == {1}
    clk.t = 1.0
    s.step()
    assert big2.batch_id is not None and big2.batch_id >= 2
    # no large request queued: slot 0 serves small ones too
    clk.t = 2.0
    s.step()
    more = [s.submit("b", rows(2, 10 + i)) for i in range(2)]
    s.step()
    assert all(r.batch_id is not None for r in more)


def test_collector_paused_while_serving_and_restored():
    import gc
    import time
    was = gc.isenabled()
    be = FakeBackend(time.monotonic, slots=2, duration=0.001)
    s = Server(be, hbm_budget=10 ** 6, clock=time.monotonic).start()
    assert not gc.isenabled()
    s.submit("a", rows(3, 0))
    s.drain(timeout=30)
    assert gc.isenabled() == was


def test_loop_failure_fails_requests_instead_of_hanging():
    import time

    class Broken(FakeBackend):
        def footprint(self, kind, pid, n):
            return n

        def launch(self, slot, groups):
            raise KeyboardInterrupt("not an Exception: escapes the per-batch handler")

    s = Server(Broken(time.monotonic, slots=1), hbm_budget=10 ** 6, clock=time.monotonic,
               pause_gc=False).start()
    r = s.submit("a", rows(2, 0))
    with pytest.raises(RuntimeError, match="serving loop failed"):
        s.drain(timeout=30)
    with pytest.raises(KeyboardInterrupt):
        r.wait(1)
