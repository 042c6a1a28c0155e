"""Serving loop for SAQ encode requests (continuous batching on one GPU).

Requests -- a block of FP32 vectors for one resident dataset (plan), or a
64-query estimate scan over a dataset's stored records -- arrive at any time.
A scheduler thread keeps them in arrival order and, whenever a launch slot
(a HIP stream) is free, forms the next batch from the queued requests that
fit the HBM budget:

  * admission   a request is admitted only while the device bytes of all
                in-flight work plus its own stay within ``hbm_budget``; one
                that can never fit is rejected at submission;
  * batching    encode requests of the same plan are concatenated into one
                dataset entry, up to BATCH_MAX plans and ``max_batch_vectors``
                vectors per batch, and the batch runs as one
                saq_encode_batched call (two grouped launches);
  * overlap     every slot has its own stream: host-to-device copies, the
                launches and the device-to-host copies of one batch overlap
                with other slots' batches;
  * completion  batches finish through events; per-request latency is the
                time from arrival to the results being on the host.

Each vector's record depends only on that vector and its plan, so a request
gets exactly the same records alone or in any mix.

The device work goes through a backend object; ``GpuBackend`` drives libsaq
with PyTorch streams and pinned host memory.  Tests of the scheduling and
admission logic can plug in a backend and a clock of their own.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import BATCH_MAX

ENCODE, SCAN = "encode", "scan"


class Rejected(RuntimeError):
    pass


@dataclasses.dataclass(eq=False)
class Request:
    rid: int
    kind: str                      # ENCODE or SCAN
    plan_id: str
    data: object                   # encode: [n, D] rows; scan: [nq, D] queries
    arrival: float
    footprint: int = 0
    admitted: Optional[float] = None
    finished: Optional[float] = None
    result: Optional[Tuple] = None     # encode: (codes, factors); scan: (dist2,)
    error: Optional[BaseException] = None
    cancelled: bool = False
    batch_id: Optional[int] = None
    _event: threading.Event = dataclasses.field(default_factory=threading.Event, repr=False)

    @property
    def n(self) -> int:
        return int(self.data.shape[0])

    def wait(self, timeout: Optional[float] = None):
        if not self._event.wait(timeout):
            raise TimeoutError(f"request {self.rid} not finished")
        if self.error is not None:
            raise self.error
        return self.result

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


def _is_pinned(a) -> bool:
    return hasattr(a, "is_pinned") and a.is_pinned()


class GpuBackend:
    """libsaq on one GPU: one stream per slot, pinned staging buffers."""

    def __init__(self, device: int = 0, slots: int = 4, rounds: int = 4):
        import torch
        self.torch = torch
        self.rounds = rounds
        self.device = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]
        self.plans: Dict[str, object] = {}
        self.stores: Dict[str, Tuple[object, object]] = {}

    @property
    def slots(self) -> int:
        return len(self.streams)

    def add_plan(self, plan_id: str, plan):
        if plan.info is not None and getattr(plan, "_dev", None) is None:
            plan.upload(self.device.index)
        self.plans[plan_id] = plan

    def add_store(self, plan_id: str, codes, factors):
        """Stored records (device tensors) that scan requests read."""
        self.stores[plan_id] = (codes, factors)

    def footprint(self, kind: str, plan_id: str, n: int) -> int:
        """Device bytes a request occupies while in flight."""
        p = self.plans[plan_id]
        if kind == ENCODE:
            return n * (4 * p.D + p.code_bytes + 4 * p.n_factors) + p.encode_workspace_bytes(n)
        nstore = self.stores[plan_id][0].shape[0]
        return n * 4 * p.D + 4 * n * nstore + p.estimate_workspace_bytes(n)

    def launch(self, slot: int, groups):
        """Start one batch on a slot.  groups: [(kind, plan_id, [Request])].
        Returns an object with done() and finish() -> per-request results."""
        return _GpuBatch(self, slot, groups)


class _GpuBatch:
    def __init__(self, be: GpuBackend, slot: int, groups):
        from . import encode_batched, estimate_dist
        torch = be.torch
        self.torch = torch
        st = be.streams[slot]
        self.parts = []            # (request, host result tensors, row slice)
        entries = []
        copies = []                # (device result, pinned host copy)
        self.keep = []             # tensors that must live until the batch is done
        with torch.cuda.stream(st):
            for kind, pid, reqs in groups:
                plan = be.plans[pid]
                n = sum(r.n for r in reqs)
                X = torch.empty((n, plan.D), dtype=torch.float32, device=be.device)
                staged = [r for r in reqs if not _is_pinned(r.data)]
                if staged:
                    host = torch.empty((sum(r.n for r in staged), plan.D), dtype=torch.float32,
                                       pin_memory=True)
                    self.keep.append(host)
                row, srow = 0, 0
                for r in reqs:
                    if _is_pinned(r.data):          # straight from the caller's pinned rows
                        X[row:row + r.n].copy_(r.data, non_blocking=True)
                    else:
                        host[srow:srow + r.n].numpy()[:] = r.data
                        X[row:row + r.n].copy_(host[srow:srow + r.n], non_blocking=True)
                        srow += r.n
                    row += r.n
                self.keep.append(X)
                if kind == ENCODE:
                    codes = torch.empty((n, plan.code_bytes), dtype=torch.uint8, device=be.device)
                    fac = torch.empty((n, plan.n_factors), dtype=torch.float32, device=be.device)
                    entries.append((plan, X, codes, fac))
                    hc = torch.empty(codes.shape, dtype=torch.uint8, pin_memory=True)
                    hf = torch.empty(fac.shape, dtype=torch.float32, pin_memory=True)
                    self.keep += [codes, fac]
                    copies += [(codes, hc), (fac, hf)]
                    row = 0
                    for r in reqs:
                        self.parts.append((r, (hc, hf), slice(row, row + r.n)))
                        row += r.n
                else:
                    codes, fac = be.stores[pid]
                    out = estimate_dist(plan, X, codes, fac, stream=st)
                    ho = torch.empty(out.shape, dtype=torch.float32, pin_memory=True)
                    self.keep.append(out)
                    copies.append((out, ho))
                    row = 0
                    for r in reqs:
                        self.parts.append((r, (ho,), slice(row, row + r.n)))
                        row += r.n
            if entries:
                encode_batched(entries, be.rounds, stream=st)
            for dev_t, host_t in copies:
                host_t.copy_(dev_t, non_blocking=True)
            self.event = torch.cuda.Event()
            self.event.record(st)

    def done(self) -> bool:
        return self.event.query()

    def finish(self):
        # results are views of the batch's pinned host buffers (each view
        # keeps its buffer alive); no host-side copy in the scheduler thread
        self.event.synchronize()
        out = []
        for r, hosts, sl in self.parts:
            out.append((r, tuple(h.numpy()[sl] for h in hosts)))
        self.keep = None
        return out


class Server:
    """Continuous-batching encode/scan server over a backend."""

    def __init__(self, backend, hbm_budget: int, max_batch_vectors: int = 262144,
                 clock: Callable[[], float] = time.monotonic, poll_s: float = 2e-4,
                 keep_results: bool = True):
        self.be = backend
        self.keep_results = keep_results      # False: record timings, drop results
        self.budget = int(hbm_budget)
        self.max_batch = int(max_batch_vectors)
        self.clock = clock
        self.poll_s = poll_s
        self.queue: collections.deque = collections.deque()
        self.inflight: Dict[int, Tuple[object, List[Request], int]] = {}   # slot -> (batch, reqs, bytes)
        self.used = 0
        self.lock = threading.Condition()
        self.done: List[Request] = []
        self.rejected = 0
        self.next_rid = 0
        self.next_batch = 0
        self.batches = 0
        self.max_queue = 0
        self.max_used = 0
        self._stop = False
        self._thread: Optional[threading.Thread] = None

    # -- submission ---------------------------------------------------------
    def submit(self, plan_id: str, data, kind: str = ENCODE,
               arrival: Optional[float] = None) -> Request:
        """data: [n, D] FP32 rows (numpy, or a pinned host torch tensor that
        is copied to the device without staging)."""
        if not _is_pinned(data):
            data = np.ascontiguousarray(data, np.float32)
        with self.lock:
            r = Request(self.next_rid, kind, plan_id, data,
                        self.clock() if arrival is None else arrival)
            self.next_rid += 1
            r.footprint = self.be.footprint(kind, plan_id, r.n)
            if r.footprint > self.budget:
                self.rejected += 1
                r.error = Rejected(f"request {r.rid} needs {r.footprint} device bytes, "
                                   f"more than the budget {self.budget}")
                r.finished = r.arrival
                r._event.set()
                return r
            self.queue.append(r)
            self.max_queue = max(self.max_queue, len(self.queue))
            self.lock.notify_all()
            return r

    def cancel(self, r: Request) -> bool:
        """Cancel a request that is still queued (not yet on the device)."""
        with self.lock:
            if r in self.queue:
                self.queue.remove(r)
                r.cancelled = True
                r.error = RuntimeError(f"request {r.rid} cancelled")
                r.finished = self.clock()
                r._event.set()
                return True
            return False

    # -- scheduling ---------------------------------------------------------
    def _form_batch(self) -> Optional[Tuple[list, List[Request], int]]:
        """Take queued requests in arrival order into one batch: same-kind
        entries per plan, at most BATCH_MAX plans, max_batch vectors, and the
        free HBM budget.  The first queued request always starts the batch if
        it fits the free budget (it is never overtaken indefinitely)."""
        free = self.budget - self.used
        picked: List[Request] = []
        groups: Dict[Tuple[str, str], List[Request]] = {}
        vectors = 0
        bytes_ = 0
        for r in list(self.queue):
            key = (r.kind, r.plan_id)
            if key not in groups and len(groups) >= BATCH_MAX:
                continue
            if picked and vectors + r.n > self.max_batch:
                continue
            if bytes_ + r.footprint > free:
                if not picked:
                    return None          # head of the queue waits for memory
                continue
            groups.setdefault(key, []).append(r)
            picked.append(r)
            vectors += r.n
            bytes_ += r.footprint
        if not picked:
            return None
        for r in picked:
            self.queue.remove(r)
        return [(k, pid, rs) for (k, pid), rs in groups.items()], picked, bytes_

    def step(self) -> bool:
        """One scheduler pass: retire finished batches, then fill free slots.
        Returns True when anything happened."""
        acted = False
        for slot, (batch, reqs, nbytes) in list(self.inflight.items()):
            if batch.done():
                results = batch.finish()
                now = self.clock()
                with self.lock:
                    del self.inflight[slot]
                    self.used -= nbytes
                    for r, res in results:
                        r.result = res if self.keep_results else None
                        r.finished = now
                        self.done.append(r)
                        r._event.set()
                    self.lock.notify_all()
                acted = True
        for slot in range(self.be.slots):
            if slot in self.inflight:
                continue
            with self.lock:
                formed = self._form_batch()
                if formed is None:
                    break
                groups, reqs, nbytes = formed
                self.used += nbytes
                self.max_used = max(self.max_used, self.used)
                now = self.clock()
                bid = self.next_batch
                self.next_batch += 1
                for r in reqs:
                    r.admitted = now
                    r.batch_id = bid
            try:
                batch = self.be.launch(slot, groups)
            except Exception as exc:                  # fail only this batch
                with self.lock:
                    self.used -= nbytes
                    for r in reqs:
                        r.error = exc
                        r.finished = self.clock()
                        r._event.set()
                continue
            with self.lock:
                self.inflight[slot] = (batch, reqs, nbytes)
                self.batches += 1
            acted = True
        return acted

    def _loop(self):
        while True:
            with self.lock:
                if self._stop and not self.queue and not self.inflight:
                    return
            if not self.step():
                time.sleep(self.poll_s)

    def start(self) -> "Server":
        self._thread = threading.Thread(target=self._loop, name="saq-serve", daemon=True)
        self._thread.start()
        return self

    def drain(self, timeout: float = 600.0):
        """Wait until everything submitted so far has finished, then stop."""
        with self.lock:
            self._stop = True
            self.lock.notify_all()
        if self._thread is not None:
            self._thread.join(timeout)
            if self._thread.is_alive():
                raise TimeoutError("server did not drain")

    # -- metrics --------------------------------------------------------------
    def stats(self) -> dict:
        lat = np.array([r.latency for r in self.done if r.error is None])
        enc = [r for r in self.done if r.kind == ENCODE and r.error is None]
        vec = sum(r.n for r in enc)
        span = (max(r.finished for r in self.done) - min(r.arrival for r in self.done)) \
            if self.done else 0.0
        return {
            "requests": len(self.done), "rejected": self.rejected, "batches": self.batches,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "mean_ms": float(lat.mean() * 1e3) if lat.size else None,
            "encoded_vectors": int(vec),
            "vectors_per_s": vec / span if span > 0 else None,
            "max_queue": self.max_queue,
            "max_inflight_bytes": self.max_used,
            "by_kind": {k: _percentiles([r.latency for r in self.done
                                         if r.kind == k and r.error is None])
                        for k in (ENCODE, SCAN)},
        }


def _percentiles(lat) -> dict:
    a = np.asarray(lat, dtype=np.float64)
    if a.size == 0:
        return {"count": 0}
    return {"count": int(a.size), "p50_ms": float(np.percentile(a, 50) * 1e3),
            "p99_ms": float(np.percentile(a, 99) * 1e3), "mean_ms": float(a.mean() * 1e3)}


def replay(server: Server, trace: Sequence[Tuple[float, str, np.ndarray, str]],
           clock: Callable[[], float] = time.monotonic) -> List[Request]:
    """Submit (t_offset_s, plan_id, data, kind) requests at their offsets in
    real time (open loop) and return the requests."""
    t0 = clock()
    out = []
    for t, pid, data, kind in trace:
        wait = t0 + t - clock()
        if wait > 0:
            time.sleep(wait)
        out.append(server.submit(pid, data, kind, arrival=t0 + t))
    return out
