"""Continuous-batching request loop over the batched entry point.

Requests (a plan, a resident complex64 input, an arrival time) are admitted
by device-memory footprint: a request needs its plan's per-transform
workspace in the batch workspace plus its outputs, and the requests in
flight may hold at most `budget_bytes` of it.  Whenever an executor slot is
free, everything admitted and waiting goes out as one `sft_execute_many`
batch (at most `max_batch` transforms, and at most `slot_budget` bytes when
the slots' workspaces are sized up front); requests that arrive while
batches run wait for the next free slot, so their work overlaps the batches
already on the device.  A request whose footprint alone exceeds the budget
(or a slot) is rejected.

The executor is pluggable: `GpuExecutor` runs each batch on its own HIP
stream (default priority), each stream with the library's batch workspace
reserved once for `reserve_bytes` (so the device memory of serving is the
slots' reservations, and no batch allocates), and detects completion with
an event; any object with the same three methods (launch, done, finish) can
stand in for it.  A transform whose device-side capacities overflowed gets
an error message and its (still filled) outputs.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any, Callable, Optional


@dataclasses.dataclass
class Request:
    rid: int
    plan: Any                   # paper_1706_02740_amd.Plan (or what the executor understands)
    f: Any                      # input, resident where the executor runs
    arrival: float              # seconds, on the server's clock
    nbytes: int = 0             # workspace the request holds while in flight
    start: Optional[float] = None
    done: Optional[float] = None
    result: Any = None          # (freqs, coefs, count) once done
    error: Optional[str] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class GpuExecutor:
    """One `sft_execute_many` per batch, each on its own stream."""

    def __init__(self, slots: int = 2, reserve_bytes: int = 0, max_batch: int = 256):
        import torch

        from . import execute_many, execute_many_release, execute_many_reserve, execute_many_status
        self._torch = torch
        self._execute_many = execute_many
        self._status = execute_many_status
        self._release = execute_many_release
        self.slots = slots
        self._streams = [torch.cuda.Stream() for _ in range(slots)]   # default priority
        self._busy = [False] * slots
        if reserve_bytes:
            for st in self._streams:
                execute_many_reserve(st, reserve_bytes, max_batch)

    def free_slot(self) -> Optional[int]:
        for i, b in enumerate(self._busy):
            if not b:
                return i
        return None

    def launch(self, batch: list) -> Any:
        torch = self._torch
        i = self.free_slot()
        if i is None:
            raise RuntimeError("no free executor slot")
        st = self._streams[i]
        # the inputs were written on the current stream: order this stream after it
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            outs = [(torch.empty(r.plan.s, dtype=torch.int64, device="cuda"),
                     torch.empty(r.plan.s, dtype=torch.complex64, device="cuda")) for r in batch]
            counts = torch.empty(len(batch), dtype=torch.int32, device="cuda")
            self._execute_many([r.plan for r in batch], [r.f for r in batch], outs, counts, st)
            ev = torch.cuda.Event()
            ev.record(st)
        self._busy[i] = True
        return (i, ev, outs, counts)

    def done(self, handle) -> bool:
        return handle[1].query()

    def finish(self, handle, batch: list) -> None:
        i, ev, outs, counts = handle
        ev.synchronize()
        flags = self._status(self._streams[i], len(batch))
        for k, r in enumerate(batch):
            r.result = (outs[k][0], outs[k][1], counts[k:k + 1])
            if flags[k]:
                r.error = f"device-side capacity exceeded (status flags {flags[k]})"
        self._busy[i] = False

    def close(self) -> None:
        """Free the slots' batch workspaces (waits for their work)."""
        for st in self._streams:
            self._release(st)


def footprint_bytes(plan) -> int:
    """Device bytes charged to one in-flight transform of `plan`: its slice
    of the batch workspace plus its outputs (int64 and complex64 per slot, an
    int32 count).  The plan's tables are resident for as long as the plan
    and are not charged per request."""
    return int(plan.workspace_bytes()) + 16 * int(plan.s) + 4


class Server:
    def __init__(self, executor, budget_bytes: int, max_batch: int = 256,
                 clock: Callable[[], float] = time.perf_counter, slot_budget: Optional[int] = None):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.slot_budget = self.budget if slot_budget is None else min(int(slot_budget), self.budget)
        self.max_batch = int(max_batch)
        self.clock = clock
        self.waiting = collections.deque()
        self.inflight = []            # (handle, batch)
        self.held = 0                 # bytes held by requests in flight
        self.completed = []
        self.rejected = []
        self.batches = 0
        self.max_inflight = 0         # most batches on the device at once
        self.max_held = 0

    def submit(self, r: Request) -> bool:
        if r.nbytes > self.slot_budget:
            r.error = "footprint exceeds the serving budget"
            self.rejected.append(r)
            return False
        self.waiting.append(r)
        return True

    def poll(self) -> int:
        """Collect finished batches; returns how many requests completed."""
        n = 0
        keep = []
        for h, batch in self.inflight:
            if self.ex.done(h):
                self.ex.finish(h, batch)
                now = self.clock()
                for r in batch:
                    r.done = now
                    self.held -= r.nbytes
                self.completed.extend(batch)
                n += len(batch)
            else:
                keep.append((h, batch))
        self.inflight = keep
        return n

    def launch(self) -> int:
        """Send the admitted waiting requests out as one batch if a slot is free."""
        if not self.waiting or self.ex.free_slot() is None:
            return 0
        batch = []
        held = self.held
        in_batch = 0
        while self.waiting and len(batch) < self.max_batch and held + self.waiting[0].nbytes <= self.budget \
                and in_batch + self.waiting[0].nbytes <= self.slot_budget:
            r = self.waiting.popleft()
            held += r.nbytes
            in_batch += r.nbytes
            batch.append(r)
        if not batch:
            return 0
        now = self.clock()
        for r in batch:
            r.start = now
        h = self.ex.launch(batch)
        self.held = held
        self.inflight.append((h, batch))
        self.batches += 1
        self.max_inflight = max(self.max_inflight, len(self.inflight))
        self.max_held = max(self.max_held, held)
        return len(batch)

    def step(self) -> None:
        self.poll()
        self.launch()

    def idle(self) -> bool:
        return not self.waiting and not self.inflight


def run_trace(server: Server, requests: list, t0: Optional[float] = None) -> list:
    """Replay requests (sorted by `arrival`, seconds from the start) against
    the server's clock until every admitted request has completed."""
    clock = server.clock
    t0 = clock() if t0 is None else t0
    order = sorted(requests, key=lambda r: r.arrival)
    for r in order:
        r.arrival += t0
    i = 0
    while i < len(order) or not server.idle():
        now = clock()
        while i < len(order) and order[i].arrival <= now:
            server.submit(order[i])
            i += 1
        server.step()
    return order
