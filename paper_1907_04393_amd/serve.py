"""Serving loop: continuous batching of camera frames from many streams.

Streams (camera sessions) arrive and leave; each sends its user-free frames
first (the paper's initialisation phase, Section 2) and then hand frames at
its own rate. The server keeps every admitted stream's background model
resident on the device, in a slot sized for its resolution. Slots come from
a pool sized by an HBM budget; a stream that finds no free slot of its class
waits (its frames queue, none is dropped) until a slot frees up.

Device work is issued in steps: a step takes at most one pending frame from
each admitted stream that has no frame in flight and runs them together
(one batched pipeline pass). Slots are spread over `lanes` independent
batches, each on its own HIP stream, so a step can be issued on one lane
while another lane's step is still on the device: frames that arrive while
others are being processed are admitted as soon as a lane is free. A
frame's latency is the time its pointer reached host memory minus its
arrival time.

Backends: GpuBackend (fizi.Batch per lane, HIP streams, pinned pointer
copies) and, for tests of the scheduling logic on a machine without a GPU,
any object with the same methods (see OracleBackend in the tests).
"""
from __future__ import annotations

import collections
import dataclasses
import gc
import heapq
import time

import numpy as np


@dataclasses.dataclass
class Session:
    """One camera stream's visit: learning frames, then hand frames at the
    given arrival times (seconds from the start of the run)."""
    sid: int
    width: int
    height: int
    bg: object                     # callable() -> learning frames, or the frames
    frames: object                 # callable(k) -> hand frame k
    arrivals: list                 # arrival time of each hand frame
    start: float = 0.0             # when the session asks to be admitted
    params: object = None


@dataclasses.dataclass
class FrameResult:
    sid: int
    seq: int
    t_arrival: float
    t_done: float
    pointer: dict

    @property
    def latency(self):
        return self.t_done - self.t_arrival


def poisson_arrivals(rate, t0, t1, rng):
    """Arrival times of a Poisson process of the given rate on [t0, t1)."""
    out, t = [], t0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= t1:
            return out
        out.append(t)


def plan_slots(classes, counts, bytes_per_class, budget):
    """Slots per resolution class: as many as the budget allows, in
    proportion to the demand (streams per class), at least one per class
    with demand when it fits. Returns {class: n_slots}."""
    demand = {c: counts.get(c, 0) for c in classes}
    slots = {c: 0 for c in classes}
    # whole demand if it fits
    need = sum(demand[c] * bytes_per_class[c] for c in classes)
    if need <= budget:
        return dict(demand)
    total = sum(demand.values())
    left = budget
    for c in classes:                       # one slot for every class in use
        if demand[c] and bytes_per_class[c] <= left:
            slots[c] = 1
            left -= bytes_per_class[c]
    # then proportional shares, largest remaining deficit first
    while True:
        best, best_def = None, 0.0
        for c in classes:
            if slots[c] >= demand[c] or bytes_per_class[c] > left:
                continue
            deficit = demand[c] / total - slots[c] / max(1, sum(slots.values()))
            if best is None or deficit > best_def:
                best, best_def = c, deficit
        if best is None:
            return slots
        slots[best] += 1
        left -= bytes_per_class[best]


class Server:
    def __init__(self, backend, clock=time.perf_counter):
        self.be = backend
        self.clock = clock
        self.results = []
        self.deferred = set()      # sessions that had to wait for a slot
        self.max_waiting = 0
        self.steps = 0
        self.max_step = 0          # most frames in one step
        self.max_queue = 0

    def run(self, sessions, duration, t_max=None, admitted=None):
        """Serves the sessions' frames that arrive before `duration` seconds,
        then drains the queues. `admitted` maps sessions already bound (and
        learned) before the run to their slots. Returns the FrameResults."""
        # the cyclic garbage collector pauses for tens of milliseconds once many
        # result objects exist; the loop creates no reference cycles
        gc_on = gc.isenabled()
        gc.disable()
        try:
            return self._run(sessions, duration, t_max, admitted)
        finally:
            if gc_on:
                gc.enable()

    def _run(self, sessions, duration, t_max, admitted):
        be = self.be
        if hasattr(be, "begin"):
            be.begin()
        t0 = self.clock()
        now = lambda: self.clock() - t0                        # noqa: E731
        by_sid = {s.sid: s for s in sessions}
        admitted = dict(admitted or {})
        pending = sorted((s for s in sessions if s.sid not in admitted), key=lambda s: s.start)
        waiting = collections.deque()                          # asking, no slot yet
        bound = dict(admitted)                                 # sid -> slot
        queues = {s.sid: collections.deque() for s in sessions}
        nxt = {s.sid: 0 for s in sessions}
        heap = [(s.arrivals[0], s.sid) for s in sessions if s.arrivals and s.arrivals[0] < duration]
        heapq.heapify(heap)
        ended = {s.sid for s in sessions if not s.arrivals or s.arrivals[0] >= duration}
        ready = [set() for _ in be.lanes()]                    # bound, queued, not busy
        inflight = {}                                          # lane -> (handle, items)
        busy = set()
        t_limit = t_max if t_max is not None else duration * 4 + 10
        while True:
            t = now()
            while pending and pending[0].start <= t:
                waiting.append(pending.pop(0))
            while heap and heap[0][0] <= t:
                ta, sid = heapq.heappop(heap)
                k = nxt[sid]
                queues[sid].append((k, ta))
                arr = by_sid[sid].arrivals
                nxt[sid] = k + 1
                if k + 1 < len(arr) and arr[k + 1] < duration:
                    heapq.heappush(heap, (arr[k + 1], sid))
                else:
                    ended.add(sid)
                if sid in bound and sid not in busy:
                    ready[be.lane_of(bound[sid])].add(sid)
            # admission: a free slot of the session's class
            if waiting:
                still = collections.deque()
                for s in waiting:
                    slot = be.acquire(s.width, s.height)
                    if slot is None:
                        still.append(s)
                        continue
                    be.learn(slot, s.bg() if callable(s.bg) else s.bg, s.params)
                    bound[s.sid] = slot
                    if queues[s.sid]:
                        ready[be.lane_of(slot)].add(s.sid)
                self.deferred.update(x.sid for x in still)
                self.max_waiting = max(self.max_waiting, len(still))
                waiting = still
            # completions
            for lane, (h, items) in list(inflight.items()):
                if be.done(h):
                    ptrs = be.pointers(h)
                    td = now()
                    for sid, seq, ta, slot in items:
                        self.results.append(FrameResult(sid, seq, ta, td, ptrs[slot]))
                        busy.discard(sid)
                        if queues[sid]:
                            ready[lane].add(sid)
                        elif sid in ended:
                            be.release(bound.pop(sid))
                    del inflight[lane]
            # sessions whose frames are over and served leave
            for sid in [x for x in ended if x in bound and x not in busy and not queues[x]]:
                be.release(bound.pop(sid))
            # issue steps on idle lanes
            for lane in be.lanes():
                if lane in inflight or not ready[lane]:
                    continue
                items = []
                for sid in ready[lane]:
                    seq, ta = queues[sid].popleft()
                    items.append((sid, seq, ta, bound[sid]))
                ready[lane] = set()
                frames = {slot: by_sid[sid].frames(seq) for sid, seq, ta, slot in items}
                inflight[lane] = (be.step(lane, frames), items)
                busy.update(sid for sid, *_ in items)
                self.steps += 1
                self.max_step = max(self.max_step, len(items))
            qlen = sum(len(q) for q in queues.values()) if self.steps % 64 == 0 else 0
            self.max_queue = max(self.max_queue, qlen)
            if t >= duration and not heap and not pending and not waiting and not inflight \
                    and not any(queues[s] for s in queues):
                break
            if t > t_limit:
                break
        return self.results


def summarize(results, px_of, wall):
    lat = np.array([r.latency for r in results]) * 1e3 if results else np.zeros(1)
    px = sum(px_of[r.sid] for r in results)
    return {"frames": len(results), "Mpixel_per_s": round(px / wall / 1e6, 1),
            "frames_per_s": round(len(results) / wall, 1),
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                           "p99": round(float(np.percentile(lat, 99)), 3),
                           "max": round(float(lat.max()), 3)}}


class GpuBackend:
    """Slot pool over `lanes` fizi.Batch objects, each on its own HIP stream."""

    def __init__(self, slot_geoms, lanes=2, device="cuda", mode=None):
        import torch
        from . import fizi
        self.torch, self.fizi = torch, fizi
        self.device = torch.device(device)
        self.n_lanes = lanes
        # slot i lives in lane i % lanes
        self.slot_geom = list(slot_geoms)
        self.lane_slots = [[i for i in range(len(self.slot_geom)) if i % lanes == L] for L in range(lanes)]
        self.batches, self.streams, self.ptrs, self.host, self.events = [], [], [], [], []
        for L in range(lanes):
            geoms = [self.slot_geom[i] for i in self.lane_slots[L]] or [(64, 1)]
            b = fizi.Batch(geoms, device=self.device)
            b.set_mode(fizi.BATCH_GRAPH if mode is None else mode)
            self.batches.append(b)
            self.streams.append(torch.cuda.Stream(device=self.device))
            self.ptrs.append(torch.empty((len(geoms), 56), dtype=torch.uint8, device=self.device))
            self.host.append(torch.empty((len(geoms), 56), dtype=torch.uint8, pin_memory=True))
            self.events.append(None)
        self.free = collections.defaultdict(list)
        for i, g in enumerate(self.slot_geom):
            self.free[g].append(i)
        self.learn_stream = torch.cuda.Stream(device=self.device)

    @staticmethod
    def state_bytes(geom, params=None):
        from . import fizi
        return fizi.Batch.stream_bytes(geom, params)

    def lanes(self):
        return range(self.n_lanes)

    def lane_of(self, slot):
        return slot % self.n_lanes

    def acquire(self, w, h):
        f = self.free.get((w, h))
        return f.pop() if f else None

    def release(self, slot):
        self.free[self.slot_geom[slot]].append(slot)

    def begin(self):
        """Frames made on other streams before the run are complete."""
        self.torch.cuda.synchronize()

    def learn(self, slot, frames, params=None):
        L = self.lane_of(slot)
        j = self.lane_slots[L].index(slot)
        s = self.streams[L]
        # the frames come from the current stream; the lane reads them, and the
        # allocator must not hand their memory out before the lane is done
        s.wait_stream(self.torch.cuda.current_stream())
        frames.record_stream(s)
        self.batches[L].learn(j, frames, reset=True, stream=s)

    def step(self, lane, frames):
        torch = self.torch
        b, s = self.batches[lane], self.streams[lane]
        idx = self.lane_slots[lane]
        fr = [frames.get(i) for i in idx]
        # frames may have been made on the current stream just now: the lane
        # waits for them, and the allocator keeps their memory until the lane
        # is done with it
        s.wait_stream(torch.cuda.current_stream(self.device))
        for f in fr:
            if f is not None:
                f.record_stream(s)
        b.step(fr, self.ptrs[lane], stream=s)
        with torch.cuda.stream(s):
            self.host[lane].copy_(self.ptrs[lane], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return (lane, ev, list(frames))

    def done(self, h):
        return h[1].query()

    def pointers(self, h):
        lane, _, slots = h
        recs = self.fizi.pointers_to_numpy(self.host[lane])
        idx = self.lane_slots[lane]
        return {slot: self.fizi.pointer_dict(recs[idx.index(slot)]) for slot in slots}

    def close(self):
        for b in self.batches:
            b.close()
