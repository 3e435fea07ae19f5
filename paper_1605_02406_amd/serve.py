"""Serving many filter streams on one GPU.

Every stream owns one device-resident grid (its whole state lives in one arena, so its HBM
footprint is known exactly before it is created). A stream is admitted only if its arena fits
the remaining HBM budget. Requests (one measurement grid = one filter cycle of one stream) are
batched continuously: whenever fewer than `max_inflight` batches are queued on the device, the
oldest pending request of every stream with work waiting (at most `max_batch` streams, oldest
first) is stepped in one `dogm_step_batch` launch set. All batches go to one HIP stream, so a
stream's cycles run in arrival order even when consecutive ones sit in consecutive batches, and
each grid's result is bit-identical to stepping it alone.

Latency of a request = the host time at which its batch is seen complete - its arrival time.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

from . import dogm

MAX_BATCH = 32  # grids per launch set (the library's limit)


class Admission:
    """HBM budget bookkeeping (host only)."""

    def __init__(self, budget_bytes: int):
        if budget_bytes < 0:
            raise ValueError("budget must be >= 0")
        self.budget = int(budget_bytes)
        self.held = {}

    @property
    def used(self) -> int:
        return sum(self.held.values())

    @property
    def free(self) -> int:
        return self.budget - self.used

    def try_reserve(self, key, nbytes: int) -> bool:
        if key in self.held:
            raise KeyError(f"{key!r} already holds a reservation")
        if nbytes < 0:
            raise ValueError("nbytes must be >= 0")
        if nbytes > self.free:
            return False
        self.held[key] = int(nbytes)
        return True

    def release(self, key) -> int:
        return self.held.pop(key)


@dataclass
class Request:
    sid: object
    meas: dogm.Meas
    t_arrival: float
    seq: int
    t_launch: float = float("nan")
    t_done: float = float("nan")

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


def select_batch(pending, max_batch: int) -> list:
    """The streams of the next batch: the oldest pending request of each stream with work,
    oldest first (ties by the stream's request number, then insertion order), at most
    `max_batch` of them."""
    heads = [(q[0].t_arrival, q[0].seq, i, sid) for i, (sid, q) in enumerate(pending.items()) if q]
    heads.sort(key=lambda h: h[:3])
    return [sid for *_, sid in heads[:max_batch]]


@dataclass
class _Batch:
    event: object
    reqs: list
    t_launch: float


@dataclass
class Stats:
    done: list = field(default_factory=list)
    batches: int = 0
    batched_requests: int = 0
    rejected_streams: int = 0
    batch_sizes: collections.Counter = field(default_factory=collections.Counter)  # size -> count


class Server:
    """Admission, device-resident grids and continuous batching over one HIP stream."""

    def __init__(self, budget_bytes: int, max_batch: int = MAX_BATCH, max_inflight: int = 2,
                 stream=None, clock=time.perf_counter):
        import torch

        if not 1 <= max_batch <= MAX_BATCH:
            raise ValueError(f"max_batch must be in 1..{MAX_BATCH}")
        if max_inflight < 1:
            raise ValueError("max_inflight must be >= 1")
        self.torch = torch
        self.admission = Admission(budget_bytes)
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.clock = clock
        self.grids = {}
        self.pending = collections.OrderedDict()  # sid -> deque of requests
        self.inflight = collections.deque()
        self.stats = Stats()
        self._seq = collections.Counter()

    # -- streams --------------------------------------------------------------------------------
    def open(self, sid, params: dogm.CParams) -> bool:
        """Admits stream `sid` if its arena fits the remaining budget; creates its grid."""
        if sid in self.grids:
            raise KeyError(f"stream {sid!r} is already open")
        if not self.admission.try_reserve(sid, dogm.arena_bytes(params)):
            self.stats.rejected_streams += 1
            return False
        try:
            self.grids[sid] = dogm.Grid(params, stream=self.stream)
        except Exception:
            self.admission.release(sid)
            raise
        return True

    def close(self, sid):
        """Ends a stream: waits for the batches that still run its cycles (other streams' work is
        left queued), then frees its grid and its budget."""
        if sid not in self.grids:
            raise KeyError(f"stream {sid!r} is not open")
        if self.pending.get(sid):
            raise RuntimeError(f"stream {sid!r} still has pending requests")
        while any(r.sid == sid for b in self.inflight for r in b.reqs):
            self.inflight[0].event.synchronize()
            self.poll()
        del self.grids[sid]
        self.admission.release(sid)

    # -- requests -------------------------------------------------------------------------------
    def submit(self, sid, meas: dogm.Meas, t_arrival: float | None = None) -> Request:
        if sid not in self.grids:
            raise KeyError(f"stream {sid!r} is not open")
        r = Request(sid, meas, self.clock() if t_arrival is None else t_arrival, self._seq[sid])
        self._seq[sid] += 1
        self.pending.setdefault(sid, collections.deque()).append(r)
        return r

    def poll(self) -> int:
        """Retires the batches the device has finished (in launch order)."""
        n = 0
        while self.inflight and self.inflight[0].event.query():
            b = self.inflight.popleft()
            t = self.clock()
            for r in b.reqs:
                r.t_done = t
            self.stats.done.extend(b.reqs)
            n += 1
        return n

    def pump(self) -> int:
        """Retires finished batches, then launches one batch if there is room and work.
        Returns the number of requests launched."""
        self.poll()
        if len(self.inflight) >= self.max_inflight or not self.pending:
            return 0
        chosen = select_batch(self.pending, self.max_batch)
        reqs = []
        for sid in chosen:
            q = self.pending[sid]
            reqs.append(q.popleft())
            if not q:
                del self.pending[sid]
        t = self.clock()
        for r in reqs:
            r.t_launch = t
        with self.torch.cuda.stream(self.stream):
            dogm.step_batch([self.grids[r.sid] for r in reqs], [r.meas for r in reqs],
                            stream=self.stream)
            ev = self.torch.cuda.Event()
            ev.record(self.stream)
        self.inflight.append(_Batch(ev, reqs, t))
        self.stats.batches += 1
        self.stats.batched_requests += len(reqs)
        self.stats.batch_sizes[len(reqs)] += 1
        return len(reqs)

    def drain(self):
        """Launches and completes everything submitted so far."""
        while self.pending or self.inflight:
            if not self.pump() and self.inflight:
                self.inflight[0].event.synchronize()
