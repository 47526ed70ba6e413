"""Serving loop: query x database Jaccard against a resident encoded database.

Requests (each 1..64 query sets) arrive over time.  A fixed number of slots
(one HIP stream and one host thread each) take work from a FIFO queue:
whenever a slot frees up it takes the oldest waiting request and, while they
fit, the next ones too (continuous batching: requests that arrived while
others were on the GPU join the next call), up to ``max_batch_sets`` query
sets and within the HBM budget.  A call is admitted only when its device
workspace (jas_query_workspace_bytes plus outputs) fits in the budget left by
the calls in flight; calls on different slots overlap on the device.

Each request's result is the same bytes whether it runs alone or batched with
others: a query row depends only on its own set and the database.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import List, Optional

import numpy as np

from . import jas as cabi


@dataclasses.dataclass
class Request:
    rid: int
    ids: np.ndarray       # uint64, CSR entries of its query sets
    offsets: np.ndarray   # uint64[nq + 1]
    arrival: float = 0.0  # seconds, relative to the start of the run
    start: float = 0.0
    done: float = 0.0
    batch_size: int = 0   # requests in the call that served it
    B: Optional[np.ndarray] = None
    q_card: Optional[np.ndarray] = None
    den: Optional[np.ndarray] = None
    J: Optional[np.ndarray] = None

    @property
    def nq(self) -> int:
        return self.offsets.size - 1

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Server:
    """keep_results: hand every request its rows of B, |Q|, C and J (copied out
    of the slot's output buffers); False keeps only the timings (long runs)."""

    def __init__(self, db, slots: int = 4, budget_bytes: int = 8 << 30, max_batch_sets: int = 64,
                 device: int = 0, keep_results: bool = True):
        self.db = db
        self.n = db.n
        self.slots = slots
        self.budget = budget_bytes
        self.max_batch_sets = max_batch_sets
        self.device = device
        self.keep_results = keep_results
        self.streams = None  # created on the first run (one default-priority stream per slot)
        self.outbufs = None  # per slot: page-locked B, |Q|, C, J for max_batch_sets query rows
        self.queue: collections.deque = collections.deque()
        self.cv = threading.Condition()
        self.in_use = 0
        self.closed = False
        self.calls = 0
        self.errors: List[BaseException] = []

    # -- admission ------------------------------------------------------------
    def cost(self, reqs) -> int:
        nq = sum(r.nq for r in reqs)
        nid = sum(int(r.offsets[-1]) for r in reqs)
        return cabi.jas_query_workspace_bytes(self.db, nq, nid) + nq * self.n * (4 + 8 + 8) + nid * 8

    def _take(self):
        """Called with the lock held: the next batch that fits, or None."""
        if not self.queue:
            return None
        batch = [self.queue[0]]
        sets = batch[0].nq
        for r in list(self.queue)[1:]:
            if sets + r.nq > self.max_batch_sets:
                break
            batch.append(r)
            sets += r.nq
        while batch:
            c = self.cost(batch)
            if self.in_use + c <= self.budget or (self.in_use == 0 and len(batch) == 1):
                for _ in batch:
                    self.queue.popleft()
                self.in_use += c
                return batch, c
            batch.pop()
        return None

    def submit(self, req: Request):
        with self.cv:
            self.queue.append(req)
            self.cv.notify_all()

    def close(self):
        with self.cv:
            self.closed = True
            self.cv.notify_all()

    # -- one call ---------------------------------------------------------------
    def _outputs(self, slot, nq):
        """The slot's page-locked output buffers (allocated once, at the largest
        call size), viewed at nq rows; a larger call gets buffers of its own."""
        import torch
        cap = self.max_batch_sets
        if nq > cap:
            return (np.empty((nq, self.n), np.int32), np.empty(nq, np.int64), np.empty((nq, self.n), np.int64),
                    np.empty((nq, self.n), np.float64))
        if self.outbufs[slot] is None:
            self.outbufs[slot] = tuple(torch.empty(shape, dtype=dt, pin_memory=True).numpy() for shape, dt in
                                       [((cap, self.n), torch.int32), ((cap,), torch.int64),
                                        ((cap, self.n), torch.int64), ((cap, self.n), torch.float64)])
        B, qc, den, J = self.outbufs[slot]
        return B[:nq], qc[:nq], den[:nq], J[:nq]

    def _run_batch(self, batch, stream, t0, slot=0):
        import torch
        sizes = [r.nq for r in batch]
        nq = sum(sizes)
        ids = np.concatenate([r.ids for r in batch]) if len(batch) > 1 else batch[0].ids
        off = np.zeros(nq + 1, dtype=np.uint64)
        k = 0
        base = 0
        for r in batch:
            off[k + 1:k + 1 + r.nq] = r.offsets[1:] + np.uint64(base)
            base += int(r.offsets[-1])
            k += r.nq
        B, qc, den, J = self._outputs(slot, nq)
        start = time.perf_counter() - t0
        with torch.cuda.device(self.device):
            cabi.jas_query(self.db, ids, off, nq, cabi.JAS_HOST_PTRS, stream, B, qc, den, J)
        done = time.perf_counter() - t0
        k = 0
        for r in batch:
            if self.keep_results:
                r.B, r.q_card = B[k:k + r.nq].copy(), qc[k:k + r.nq].copy()
                r.den, r.J = den[k:k + r.nq].copy(), J[k:k + r.nq].copy()
            r.start, r.done, r.batch_size = start, done, len(batch)
            k += r.nq

    def _worker(self, slot, t0, finished):
        stream = self.streams[slot]
        while True:
            with self.cv:
                got = None
                while got is None:
                    got = self._take()
                    if got is None:
                        if self.closed and not self.queue:
                            return
                        self.cv.wait(0.05)
                batch, c = got
            try:
                self._run_batch(batch, stream, t0, slot)
            except BaseException as e:  # noqa: BLE001 - surfaced by run()
                self.errors.append(e)
            finally:
                with self.cv:
                    self.in_use -= c
                    self.calls += 1
                    finished.extend(batch)
                    self.cv.notify_all()

    def run(self, requests: List[Request], arrivals: Optional[List[float]] = None) -> List[Request]:
        """Serve the requests; arrivals[i] (seconds) is when request i enters the queue
        (None: all at time 0, i.e. a closed batch measuring saturation)."""
        if self.streams is None:
            import torch
            self.streams = [torch.cuda.Stream(device=self.device) for _ in range(self.slots)]
            self.outbufs = [None] * self.slots
        self.closed = False
        self.errors = []
        finished: List[Request] = []
        t0 = time.perf_counter()
        workers = [threading.Thread(target=self._worker, args=(s, t0, finished), daemon=True)
                   for s in range(self.slots)]
        if arrivals is None:  # the whole batch is queued before any slot takes work
            for r in requests:
                r.arrival = 0.0
                self.queue.append(r)
        for w in workers:
            w.start()
        if arrivals is not None:
            for i, r in enumerate(requests):
                r.arrival = arrivals[i]
                now = time.perf_counter() - t0
                if r.arrival > now:
                    time.sleep(r.arrival - now)
                self.submit(r)
        self.close()
        for w in workers:
            w.join()
        if self.errors:
            raise self.errors[0]
        return finished


def percentile(x, p):
    return float(np.percentile(np.asarray(x, dtype=np.float64), p)) if len(x) else None


def summarize(reqs: List[Request], n: int, wall: float) -> dict:
    lat = [r.latency for r in reqs]
    sets = sum(r.nq for r in reqs)
    return {"requests": len(reqs), "query_sets": sets, "wall_s": wall,
            "requests_per_s": len(reqs) / wall, "query_sets_per_s": sets / wall,
            "pair_intersections_per_s": sets * n / wall,
            "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
            "mean_batch_requests": float(np.mean([r.batch_size for r in reqs])) if reqs else None,
            "p999_ms": 1e3 * percentile(lat, 99.9),
            "requests_by_call_size": {int(k): int(v) for k, v in
                                      zip(*np.unique([r.batch_size for r in reqs], return_counts=True))}
            if reqs else {}}


def make_requests(db_spec, count: int, seed: int, max_sets: int = 64, size_scale: float = 1.0,
                  first_id: int = 0, pinned: bool = False, pool: int = 0) -> List[Request]:
    """Seeded synthetic requests: 1..max_sets query sets each (sizes and sharing as synth.query_spec).

    pinned: the IDs are received into page-locked host memory (as a server's
    receive buffers would be), so their copy to the device is a plain DMA.
    pool > 0: only `pool` distinct payloads are drawn and request k carries
    payload k % pool (a long stream without holding every payload in memory)."""
    import synth
    if pool and pool < count:
        base = make_requests(db_spec, pool, seed, max_sets, size_scale, first_id, pinned)
        out = []
        for k in range(count):
            src = base[k % pool]
            req = Request(first_id + k, src.ids, src.offsets)
            req._payload = src  # keeps a page-locked payload alive
            out.append(req)
        return out
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        nq = int(rng.integers(1, max_sets + 1))
        spec = synth.query_spec(db_spec, first_id + k, nq)
        if size_scale != 1.0:
            spec = synth.scaled(spec, size_scale=size_scale)
        if pinned:
            import torch
            off = synth.offsets(spec)
            buf = torch.empty(max(int(off[-1]), 1), dtype=torch.int64, pin_memory=True)
            ids = buf.numpy().view(np.uint64)[:int(off[-1])]
            synth.generate(spec, out=ids)
            req = Request(first_id + k, ids, off)
            req._pinned = buf  # keeps the page-locked buffer alive
        else:
            ids, off = synth.generate(spec)
            req = Request(first_id + k, ids, off)
        out.append(req)
    return out


def poisson_arrivals(count: int, rate: float, seed: int) -> List[float]:
    rng = np.random.default_rng(seed)
    return list(np.cumsum(rng.exponential(1.0 / rate, size=count)))
