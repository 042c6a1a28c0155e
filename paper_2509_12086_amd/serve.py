"""Serving loop for SAQ encode requests (continuous batching on one GPU).

Requests -- a block of FP32 vectors for one resident dataset (plan), or a
64-query estimate scan over a dataset's stored records -- arrive at any time.
A scheduler thread keeps them in arrival order and, whenever a launch slot
(a HIP stream) is free, forms the next batch from the queued requests that
fit the HBM budget:

  * admission   a request is admitted only while the device bytes of all
                in-flight work plus its own stay within ``hbm_budget``; one
                that can never fit is rejected at submission;
  * splitting   an encode request of more than ``split_vectors`` vectors is
                queued as chunks of that size, which go out in arrival order
                like any request and can run on several slots at once; the
                request completes when its last chunk is on the host, so a
                large request neither waits for one slot's whole copy nor
                holds small requests behind it;
  * classes     with ``large_vectors`` set, requests above it run only on
                the first ``large_slots`` slots (which take small requests
                while no large one waits), so a small request never queues
                behind the host-to-device copy of a large one;
  * batching    encode requests (or chunks) of the same plan are
                concatenated into one dataset entry, up to BATCH_MAX plans and
                ``max_batch_vectors`` vectors per batch, and the batch runs as
                one saq_encode_batched call (the two grouped launches, whose
                projection tiles spread a small batch over many compute
                units);
  * overlap     every slot has its own stream: host-to-device copies, the
                launches and the device-to-host copies of one batch overlap
                with other slots' batches;
  * completion  batches finish through events; per-request latency is the
                time from arrival to the results being on the host;
  * steady state every slot reuses device and pinned buffers sized at start
                for max_batch_vectors, and Python's garbage collector is
                paused while the loop runs (a full collection stalls the
                interpreter, and so every request, for tens of ms).

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
    parent: Optional["Request"] = dataclasses.field(default=None, repr=False)
    chunk: int = 0                     # index of this chunk in its parent
    chunks: Optional[List["Request"]] = dataclasses.field(default=None, repr=False)
    parts: Optional[list] = dataclasses.field(default=None, repr=False)
    pending: int = 0
    _event: threading.Event = dataclasses.field(default_factory=threading.Event, repr=False)

    @property
    def n(self) -> int:
        return int(self.data.shape[0])

    def wait(self, timeout: Optional[float] = None):
        if not self._event.wait(timeout):
            raise TimeoutError(f"request {self.rid} not finished")
        if self.error is not None:
            raise self.error
        if self.result is None and self.parts is not None:
            # a split request: its chunks' results, joined on the caller's thread
            self.result = tuple(np.concatenate([p[i] for p in self.parts])
                                for i in range(len(self.parts[0])))
            self.parts = None
        return self.result

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


def _is_pinned(a) -> bool:
    return hasattr(a, "is_pinned") and a.is_pinned()


class _SlotBuffers:
    """Device and pinned host buffers of one slot, grown only when a batch
    needs more than any before it, so that in steady state a batch
    allocates nothing: a fresh device or pinned allocation can stall the
    scheduler thread for tens of milliseconds."""

    def __init__(self, torch, device):
        self.torch, self.device = torch, device
        self.bufs: Dict[str, object] = {}
        self.grown = 0                    # allocations made (for diagnostics)

    def get(self, name: str, nbytes: int, pinned: bool = False):
        torch = self.torch
        cur = self.bufs.get(name)
        if cur is None or cur.numel() < nbytes:
            size = max(int(nbytes), 1 << 20)
            if cur is not None:
                size = max(size, 2 * cur.numel())
            cur = (torch.empty(size, dtype=torch.uint8, pin_memory=True) if pinned else
                   torch.empty(size, dtype=torch.uint8, device=self.device))
            self.bufs[name] = cur
            self.grown += 1
        return cur


def _carve(buf, off: int, shape, dtype):
    """A [shape] view of dtype at byte offset off (256-byte aligned) of a
    flat uint8 buffer; returns (view, next offset)."""
    import math
    n = int(math.prod(shape))
    itemsize = dtype.itemsize if hasattr(dtype, "itemsize") else 4
    off = (off + 255) & ~255
    view = buf[off:off + n * itemsize].view(dtype).view(*shape)
    return view, off + n * itemsize


class GpuBackend:
    """libsaq on one GPU: one stream per slot, each with its own reused
    device and pinned host buffers for encode batches."""

    def __init__(self, device: int = 0, slots: int = 4, rounds: int = 4, tuning=None):
        import torch
        from . import BATCH_GROUPED, BatchTuning
        self.torch = torch
        self.rounds = rounds
        self.tuning = tuning if tuning is not None else BatchTuning(mode=BATCH_GROUPED)
        self.device = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]
        self.buffers = [_SlotBuffers(torch, self.device) for _ in range(slots)]
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

    def reserve(self, rows: int):
        """Size every slot's encode buffers for batches of up to `rows`
        vectors of any resident plan, so that no batch allocates (the pinned
        staging of rows given as numpy arrays still grows on first use)."""
        from . import BatchTuning  # noqa: F401  (the tuning decides the workspace)
        if not self.plans:
            return
        ps = list(self.plans.values())
        x = rows * 4 * max(p.D for p in ps) + 256 * 16
        out = rows * max(p.code_bytes + 4 * p.n_factors for p in ps) + 512 * 16
        # one dataset per plan of a batch: each rounds its rows up to whole
        # 64-row tiles and its regions up to 256 bytes
        ws = max(p.encode_workspace_bytes(rows) for p in ps) + \
            16 * (64 * 4 * max(max(p.D_kept, 1) for p in ps) + 64 * 4 + 1024)
        for b in self.buffers:
            b.get("X", x)
            b.get("dev_out", out)
            b.get("host_out", out, pinned=True)
            b.get("ws", ws)

    def launch(self, slot: int, groups):
        """Start one batch on a slot.  groups: [(kind, plan_id, [Request])].
        Returns an object with done() and finish() -> per-request results."""
        return _GpuBatch(self, slot, groups)


class _GpuBatch:
    def __init__(self, be: GpuBackend, slot: int, groups):
        from . import batched_workspace_bytes, encode_batched, estimate_dist
        torch = be.torch
        self.torch = torch
        st = be.streams[slot]
        buf = be.buffers[slot]
        self.parts = []            # (request, host result tensors, row slice, copy out)
        entries = []
        copies = []                # (device result, pinned host copy)
        self.keep = []             # tensors that must live until the batch is done
        enc = [(k, pid, reqs) for k, pid, reqs in groups if k == ENCODE]
        # byte sizes of the slot's flat buffers for this batch's encodes
        need = {"X": 0, "stage": 0, "dev_out": 0, "host_out": 0}
        for _, pid, reqs in enc:
            p = be.plans[pid]
            n = sum(r.n for r in reqs)
            need["X"] += n * 4 * p.D + 256
            need["stage"] += sum(r.n for r in reqs if not _is_pinned(r.data)) * 4 * p.D + 256
            need["dev_out"] += n * (p.code_bytes + 4 * p.n_factors) + 512
        need["host_out"] = need["dev_out"]
        bX = buf.get("X", need["X"]) if enc else None
        bS = buf.get("stage", need["stage"], pinned=True) if need["stage"] else None
        bO = buf.get("dev_out", need["dev_out"]) if enc else None
        bH = buf.get("host_out", need["host_out"], pinned=True) if enc else None
        oX = oS = oO = oH = 0
        with torch.cuda.stream(st):
            for kind, pid, reqs in groups:
                plan = be.plans[pid]
                n = sum(r.n for r in reqs)
                if kind == ENCODE:
                    X, oX = _carve(bX, oX, (n, plan.D), torch.float32)
                else:
                    X = torch.empty((n, plan.D), dtype=torch.float32, device=be.device)
                    self.keep.append(X)
                staged = [r for r in reqs if not _is_pinned(r.data)]
                if staged:
                    if kind == ENCODE:
                        host, oS = _carve(bS, oS, (sum(r.n for r in staged), plan.D), torch.float32)
                    else:
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
                if kind == ENCODE:
                    codes, oO = _carve(bO, oO, (n, plan.code_bytes), torch.uint8)
                    fac, oO = _carve(bO, oO, (n, plan.n_factors), torch.float32)
                    hc, oH = _carve(bH, oH, (n, plan.code_bytes), torch.uint8)
                    hf, oH = _carve(bH, oH, (n, plan.n_factors), torch.float32)
                    entries.append((plan, X, codes, fac))
                    copies += [(codes, hc), (fac, hf)]
                    row = 0
                    for r in reqs:
                        # the slot's host buffer is reused: results are copied out
                        self.parts.append((r, (hc, hf), slice(row, row + r.n), True))
                        row += r.n
                else:
                    codes, fac = be.stores[pid]
                    out = estimate_dist(plan, X, codes, fac, stream=st)
                    ho = torch.empty(out.shape, dtype=torch.float32, pin_memory=True)
                    self.keep.append(out)
                    copies.append((out, ho))
                    row = 0
                    for r in reqs:
                        self.parts.append((r, (ho,), slice(row, row + r.n), False))
                        row += r.n
            if entries:
                wsb = buf.get("ws", batched_workspace_bytes(entries, be.tuning))
                encode_batched(entries, be.rounds, be.tuning, wsb, stream=st)
            for dev_t, host_t in copies:
                host_t.copy_(dev_t, non_blocking=True)
            self.event = torch.cuda.Event()
            self.event.record(st)

    def done(self) -> bool:
        return self.event.query()

    def finish(self, keep: bool = True):
        # scan results are views of the batch's own pinned buffers (each view
        # keeps its buffer alive); encode results leave the slot's reused
        # buffer as copies, or not at all when the caller keeps no results
        self.event.synchronize()
        out = []
        for r, hosts, sl, copy in self.parts:
            if copy:
                out.append((r, tuple(h.numpy()[sl].copy() for h in hosts) if keep else None))
            else:
                out.append((r, tuple(h.numpy()[sl] for h in hosts)))
        self.keep = None
        return out


class Server:
    """Continuous-batching encode/scan server over a backend."""

    def __init__(self, backend, hbm_budget: int, max_batch_vectors: int = 262144,
                 clock: Callable[[], float] = time.monotonic, poll_s: float = 2e-4,
                 keep_results: bool = True, split_vectors: int = 0,
                 large_vectors: int = 0, large_slots: int = 1, pause_gc: bool = True):
        self.be = backend
        self.keep_results = keep_results      # False: record timings, drop results
        self.budget = int(hbm_budget)
        self.max_batch = int(max_batch_vectors)
        self.split = int(split_vectors)       # 0: never split
        # size classes: requests above large_vectors run only on the first
        # large_slots slots, which take small requests only while no large
        # one is queued (0: one class)
        self.large = int(large_vectors)
        self.large_slots = int(large_slots) if self.large > 0 else 0
        # Python's cyclic garbage collector holds the interpreter lock for
        # tens of milliseconds in a full collection, and every request in
        # flight inherits that stall: while the loop runs, objects that exist
        # are frozen and automatic collection is paused; drain() restores it
        self.pause_gc = pause_gc
        self._gc_was_enabled = None
        self.failure: Optional[BaseException] = None
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
            split = kind == ENCODE and self.split > 0 and r.n > self.split
            step = self.split if split else r.n
            r.footprint = self.be.footprint(kind, plan_id, min(r.n, step) if r.n else 0)
            if r.footprint > self.budget:
                self.rejected += 1
                r.error = Rejected(f"request {r.rid} needs {r.footprint} device bytes, "
                                   f"more than the budget {self.budget}")
                r.finished = r.arrival
                r._event.set()
                return r
            if not split:
                self.queue.append(r)
            else:
                r.chunks = []
                for i, a in enumerate(range(0, r.n, step)):
                    c = Request(r.rid, kind, plan_id, data[a:a + step], r.arrival, parent=r,
                                chunk=i)
                    c.footprint = self.be.footprint(kind, plan_id, c.n)
                    r.chunks.append(c)
                r.parts = [None] * len(r.chunks)
                r.pending = len(r.chunks)
                self.queue.extend(r.chunks)
            self.max_queue = max(self.max_queue, len(self.queue))
            self.lock.notify_all()
            return r

    def cancel(self, r: Request) -> bool:
        """Cancel a request that is still queued (not yet on the device); a
        split request only while none of its chunks has left the queue."""
        with self.lock:
            members = r.chunks if r.chunks is not None else [r]
            if all(any(m is q for q in self.queue) for m in members):
                for m in members:
                    self.queue.remove(m)
                r.cancelled = True
                r.error = RuntimeError(f"request {r.rid} cancelled")
                r.finished = self.clock()
                r.parts = None
                r._event.set()
                return True
            return False

    def _complete(self, r: Request, result, error, now):
        """Record one finished request or chunk (lock held)."""
        p = r.parent
        if p is None:
            r.result = result if (self.keep_results and error is None) else None
            r.error = error
            r.finished = now
            if error is None:
                self.done.append(r)
            r._event.set()
            return
        if error is not None and p.error is None:
            p.error = error
        if p.parts is not None:
            p.parts[r.chunk] = result if self.keep_results else None
        p.pending -= 1
        if p.pending == 0:
            if not self.keep_results or p.error is not None:
                p.parts = None
            p.finished = now
            if p.error is None:
                self.done.append(p)
            p._event.set()

    # -- scheduling ---------------------------------------------------------
    def _is_large(self, r: Request) -> bool:
        return self.large > 0 and r.n > self.large

    def _form_batch(self, slot: int = 0) -> Optional[Tuple[list, List[Request], int]]:
        """Take queued requests in arrival order into one batch: same-kind
        entries per plan, at most BATCH_MAX plans, max_batch vectors, and the
        free HBM budget.  The first queued request of the slot's class
        always starts the batch if it fits the free budget (it is never
        overtaken indefinitely).  With size classes, a slot below
        large_slots serves the large requests (the small ones only while no
        large one waits), the other slots only the small ones."""
        free = self.budget - self.used
        picked: List[Request] = []
        groups: Dict[Tuple[str, str], List[Request]] = {}
        vectors = 0
        bytes_ = 0
        cands = list(self.queue)
        if self.large_slots:
            if slot < self.large_slots:
                big = [r for r in cands if self._is_large(r)]
                cands = big if big else cands
            else:
                cands = [r for r in cands if not self._is_large(r)]
        for r in cands:
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
                results = batch.finish(self.keep_results)
                now = self.clock()
                with self.lock:
                    del self.inflight[slot]
                    self.used -= nbytes
                    for r, res in results:
                        self._complete(r, res, None, now)
                    self.lock.notify_all()
                acted = True
        for slot in range(self.be.slots):
            if slot in self.inflight:
                continue
            with self.lock:
                formed = self._form_batch(slot)
                if formed is None:
                    continue
                groups, reqs, nbytes = formed
                self.used += nbytes
                self.max_used = max(self.max_used, self.used)
                now = self.clock()
                bid = self.next_batch
                self.next_batch += 1
                for r in reqs:
                    r.admitted = now
                    r.batch_id = bid
                    if r.parent is not None and r.parent.admitted is None:
                        r.parent.admitted = now
            try:
                batch = self.be.launch(slot, groups)
            except BaseException as exc:              # fail only this batch
                with self.lock:
                    self.used -= nbytes
                    now = self.clock()
                    for r in reqs:
                        self._complete(r, None, exc, now)
                if not isinstance(exc, Exception):
                    raise                             # and stop the loop
                continue
            with self.lock:
                self.inflight[slot] = (batch, reqs, nbytes)
                self.batches += 1
            acted = True
        return acted

    def _loop(self):
        try:
            while True:
                with self.lock:
                    if self._stop and not self.queue and not self.inflight:
                        return
                if not self.step():
                    time.sleep(self.poll_s)
        except BaseException as exc:          # the loop must not die silently
            self._fail_all(exc)

    def _fail_all(self, exc: BaseException):
        """Fail every queued and in-flight request with exc and stop."""
        with self.lock:
            self.failure = exc
            now = self.clock()
            for r in list(self.queue):
                self._complete(r, None, exc, now)
            self.queue.clear()
            for slot, (_, reqs, nbytes) in list(self.inflight.items()):
                for r in reqs:
                    self._complete(r, None, exc, now)
                self.used -= nbytes
            self.inflight.clear()
            self.lock.notify_all()

    def start(self) -> "Server":
        if hasattr(self.be, "reserve"):
            self.be.reserve(self.max_batch)
        if self.pause_gc:
            import gc
            self._gc_was_enabled = gc.isenabled()
            gc.collect()
            gc.freeze()
            gc.disable()
        self._thread = threading.Thread(target=self._loop, name="saq-serve", daemon=True)
        self._thread.start()
        return self

    def drain(self, timeout: float = 600.0):
        """Wait until everything submitted so far has finished, then stop."""
        with self.lock:
            self._stop = True
            self.lock.notify_all()
        try:
            if self._thread is not None:
                self._thread.join(timeout)
                if self._thread.is_alive():
                    raise TimeoutError("server did not drain")
        finally:
            if self.pause_gc and self._gc_was_enabled is not None:
                import gc
                gc.unfreeze()
                if self._gc_was_enabled:
                    gc.enable()
                self._gc_was_enabled = None
        if self.failure is not None:
            raise RuntimeError("serving loop failed") from self.failure

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
            # arrival to the first launch of the request (or of its first
            # chunk), and from there to its results on the host
            "queue_wait": _percentiles([r.admitted - r.arrival for r in self.done
                                        if r.admitted is not None]),
            "service": _percentiles([r.finished - r.admitted for r in self.done
                                     if r.admitted is not None]),
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
