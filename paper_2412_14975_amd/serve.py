"""Continuous-batching recognition server over resident automata.

Requests (an automaton of the pool and a text in host memory) may arrive at
any time.  Each scheduler step

1. collects the batches that have finished (their events), returning every
   request's result with its arrival-to-result latency;
2. admits waiting requests in arrival order while their device footprint
   (``ri_request_footprint``: text plus the batch buffers it needs) fits in
   the HBM budget left by the batches in flight;
3. copies the admitted texts to the device in one transfer (pinned staging
   buffer -> device arena, 16-byte aligned offsets), re-plans the slot's
   fused batch for them (``ri_batch_update``: no device allocation once the
   buffers are large enough) and launches it on the slot's stream.

Slots (streams) let consecutive steps overlap on the device: requests that
arrive while others are running are admitted as soon as a slot and memory
are free.  The automata stay resident: their tables are uploaded once.
Every recognition step runs in the library's kernels; this module only
schedules.
"""

from __future__ import annotations

import collections
import time

import numpy as np
import torch

from . import binding as B


class _Request:
    __slots__ = ("rid", "auto", "text", "arrival", "footprint")

    def __init__(self, rid, auto, text, arrival, footprint):
        self.rid, self.auto, self.text, self.arrival, self.footprint = rid, auto, text, arrival, footprint


class _Slot:
    def __init__(self, device):
        self.device = device
        self.stream = torch.cuda.Stream(device=device)
        self.batch = None
        self.results = torch.empty(2, dtype=torch.int32, device=device)
        self.arena = torch.empty(16, dtype=torch.uint8, device=device)
        self.staging = torch.empty(16, dtype=torch.uint8).pin_memory()
        self.event = None
        self.reqs = []
        self.bytes = 0


def _grow_device(t, n, dtype, device):
    if t.numel() >= n:
        return t
    return torch.empty(max(n, 2 * t.numel()), dtype=dtype, device=device)


class Server:
    """``Server(recognizers, algo="rid", hbm_budget=..., slots=2)``; then
    ``submit(automaton_index, text)`` and ``step()`` (or ``drain()``)."""

    def __init__(self, recognizers, algo="rid", hbm_budget=8 << 30, slots=2, chunk_bytes=0, warmup_bytes=0,
                 max_batch=4096, device="cuda"):
        self.handles = [r.handle if isinstance(r, B.Recognizer) else r for r in recognizers]
        self.algo = algo
        self.budget = int(hbm_budget)
        self.chunk_bytes = int(chunk_bytes)
        self.warmup_bytes = int(warmup_bytes)
        self.max_batch = int(max_batch)
        self.device = torch.device(device)
        self.slots = [_Slot(self.device) for _ in range(int(slots))]
        self.queue = collections.deque()
        self.used = 0
        self.max_used = 0
        self.next_id = 0
        self.steps = 0
        # tables resident on the device before the first request
        empty = torch.empty(0, dtype=torch.uint8, device=self.device)
        warm = B.ri_batch_create_ex([(h, empty, algo) for h in self.handles], self.chunk_bytes, "fused",
                                    self.warmup_bytes)
        B.ri_batch_free(warm)

    def submit(self, automaton: int, text, arrival: float | None = None) -> int:
        """Queue a request; text is host bytes (numpy uint8 or bytes).
        Returns the request id."""
        x = np.ascontiguousarray(np.frombuffer(text, np.uint8) if isinstance(text, (bytes, bytearray)) else text,
                                 dtype=np.uint8)
        fp = B.ri_request_footprint(self.handles[automaton], self.algo, len(x), self.chunk_bytes)
        rid = self.next_id
        self.next_id += 1
        self.queue.append(_Request(rid, automaton, x, time.perf_counter() if arrival is None else arrival, fp))
        return rid

    def pending(self) -> int:
        return len(self.queue)

    def inflight(self) -> int:
        return sum(len(s.reqs) for s in self.slots)

    def _collect(self, done):
        for sl in self.slots:
            if sl.reqs and sl.event.query():
                res = sl.results[: 2 * len(sl.reqs)].view(-1, 2).cpu().numpy()
                now = time.perf_counter()
                for r, (acc, fin) in zip(sl.reqs, res):
                    done.append(dict(id=r.rid, automaton=r.auto, n=len(r.text), accept=bool(acc),
                                     final_state=int(fin), arrival=r.arrival, done=now, latency=now - r.arrival))
                self.used -= sl.bytes
                sl.reqs, sl.bytes, sl.event = [], 0, None

    def _admit(self):
        take, fp = [], 0
        while self.queue and len(take) < self.max_batch:
            r = self.queue[0]
            fits = self.used + fp + r.footprint <= self.budget
            if not fits and (take or self.used > 0):
                break      # wait for memory; a lone oversized request runs when nothing else does
            take.append(self.queue.popleft())
            fp += r.footprint
        return take, fp

    def _launch(self, sl, take, fp):
        offs, total = [], 0
        for r in take:
            offs.append(total)
            total += (len(r.text) + 15) // 16 * 16
        total = max(total, 16)
        if sl.staging.numel() < total:
            sl.staging = torch.empty(max(total, 2 * sl.staging.numel()), dtype=torch.uint8).pin_memory()
        sl.arena = _grow_device(sl.arena, total, torch.uint8, self.device)
        sl.results = _grow_device(sl.results, 2 * len(take), torch.int32, self.device)
        host = sl.staging.numpy()
        for r, o in zip(take, offs):
            host[o:o + len(r.text)] = r.text
        with torch.cuda.stream(sl.stream):
            sl.arena[:total].copy_(sl.staging[:total], non_blocking=True)
        reqs = [(self.handles[r.auto], sl.arena[o:o + len(r.text)], self.algo) for r, o in zip(take, offs)]
        if sl.batch is None:
            sl.batch = B.ri_batch_create_ex(reqs, self.chunk_bytes, "fused", self.warmup_bytes)
        else:
            B.ri_batch_update(sl.batch, reqs)
        B.ri_batch_run(sl.batch, sl.results, stream=sl.stream)
        sl.event = torch.cuda.Event()
        sl.event.record(sl.stream)
        sl.reqs, sl.bytes = take, fp
        self.used += fp
        self.max_used = max(self.max_used, self.used)
        self.steps += 1

    def step(self) -> list:
        """One scheduler step; returns the requests completed in it."""
        done = []
        self._collect(done)
        for sl in self.slots:
            if not self.queue:
                break
            if sl.reqs:
                continue
            take, fp = self._admit()
            if not take:
                break
            self._launch(sl, take, fp)
        return done

    def drain(self) -> list:
        """Run steps until every submitted request has completed."""
        out = []
        while self.queue or self.inflight():
            out += self.step()
        return out

    def close(self):
        for sl in self.slots:
            if sl.event is not None:
                sl.event.synchronize()
            if sl.batch is not None:
                B.ri_batch_free(sl.batch)
                sl.batch = None


def run_open_loop(server: Server, schedule):
    """Drive the server with arrivals: schedule is a list of (arrival offset in
    seconds, automaton, text) sorted by offset.  Requests are submitted when
    their arrival time has passed (latency counts from the arrival time).
    Returns (completed requests, wall seconds)."""
    t0 = time.perf_counter()
    i, out = 0, []
    n = len(schedule)
    while i < n or server.pending() or server.inflight():
        now = time.perf_counter()
        while i < n and t0 + schedule[i][0] <= now:
            off, auto, text = schedule[i]
            server.submit(auto, text, arrival=t0 + off)
            i += 1
        got = server.step()
        out += got
        if not got and i < n and not server.pending() and not server.inflight():
            wait = t0 + schedule[i][0] - time.perf_counter()
            if wait > 0:
                time.sleep(min(wait, 1e-3))
    return out, time.perf_counter() - t0
