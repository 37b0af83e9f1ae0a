"""Continuous-batching request loop for many independent frame streams.

Requests (one frame of one stream each) arrive over time.  Whenever fewer
than ``max_inflight`` batches are on the GPU, every request that has arrived,
is not yet running, and fits the HBM budget is admitted (oldest first) and
launched as ONE ``wskp_denoise_batch`` call on the next stream.  Requests
that arrive while batches run are admitted as soon as a slot and memory free
up, so their work overlaps with the batches already on the device.  No
arithmetic crosses frames, so each result is the same alone and in any mix.

The scheduling policy is independent of the GPU: an ``Executor`` launches a
batch and reports when it is done.  ``GpuExecutor`` drives libwskp through
the binding; tests use a fake executor with a programmable latency model.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    stream: int
    t_arrival: float
    H: int
    W: int
    seq: int = 0                 # index of the frame within its stream
    t_start: float = float("nan")
    t_done: float = float("nan")
    error: Optional[str] = None


def poisson_trace(n_streams: int, frames_per_stream: int, rate_total: float,
                  resolutions: Sequence[Tuple[int, int]], seed: int = 7):
    """Per-stream Poisson arrivals (rate_total / n_streams each); each stream
    draws its resolution uniformly from ``resolutions``.  Returns
    (stream_sizes [(H, W)], requests sorted by arrival)."""
    rng = np.random.default_rng(seed)
    per = rate_total / n_streams
    sizes = [tuple(resolutions[i]) for i in rng.integers(0, len(resolutions), size=n_streams)]
    reqs = []
    for s in range(n_streams):
        t = np.cumsum(rng.exponential(1.0 / per, size=frames_per_stream))
        for k in range(frames_per_stream):
            reqs.append((float(t[k]), s, k))
    reqs.sort()
    out = [Request(i, s, t, *sizes[s], seq=k) for i, (t, s, k) in enumerate(reqs)]
    return sizes, out


class Arena:
    """First-fit allocator of byte ranges inside the workspace budget."""

    def __init__(self, size: int, align: int = 256):
        self.size = int(size)
        self.align = align
        self.live: List[Tuple[int, int]] = []   # (offset, size), sorted

    def alloc(self, n: int) -> Optional[int]:
        n = (int(n) + self.align - 1) // self.align * self.align
        off = 0
        for o, sz in self.live:
            if o - off >= n:
                break
            off = o + sz
        else:
            if self.size - off < n:
                return None
        self.live.append((off, n))
        self.live.sort()
        return off

    def free(self, off: int) -> None:
        self.live = [(o, s) for o, s in self.live if o != off]

    @property
    def used(self) -> int:
        return sum(s for _, s in self.live)


class Executor:
    """Interface: launch(batch, slot, ws_offset) -> token; done(token) -> bool.

    ``request_bytes(r)`` is the workspace of ``r`` alone; a batch needs at
    most the sum of its requests' values (``workspace_bytes(batch)``), so the
    scheduler can account memory per request without re-sizing whole
    batches.

    ``per_stream_cap``: at most this many frames of one stream may be in
    flight at once (None: no limit), e.g. the size of a stream's output ring.
    """

    per_stream_cap: Optional[int] = None

    def workspace_bytes(self, reqs: List[Request]) -> int:
        raise NotImplementedError

    def request_bytes(self, r: Request) -> int:
        return self.workspace_bytes([r])

    def launch(self, reqs: List[Request], slot: int, ws_offset: int = 0):
        raise NotImplementedError

    def done(self, token) -> bool:
        raise NotImplementedError

    def wait(self, token) -> None:
        while not self.done(token):
            pass


@dataclasses.dataclass
class ServeStats:
    frames: int
    errors: int
    wall_s: float
    frames_per_s: float
    p50_ms: float
    p99_ms: float
    mean_batch: float
    max_batch: int
    batches: int


class Server:
    """Continuous batching with an HBM admission budget.

    budget_bytes bounds the workspace of all in-flight batches together; a
    single request larger than the budget is rejected (error "budget").
    Frames of one stream start in arrival order, and no more than the
    executor's ``per_stream_cap`` of them are in flight together; a stream
    at its cap waits while other streams' requests pass.
    """

    def __init__(self, executor: Executor, budget_bytes: int, max_inflight: int = 2,
                 max_batch: int = 64, clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_inflight = max_inflight
        self.max_batch = max_batch
        self.clock = clock

    def run(self, requests: List[Request], realtime: bool = True) -> ServeStats:
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        pending: List[Request] = []          # arrived, not started (oldest first)
        inflight: List[Tuple[object, List[Request], int]] = []  # (token, batch, ws offset)
        arena = Arena(self.budget)
        nxt = 0
        slot = 0
        batches = []
        cap = self.ex.per_stream_cap
        live: Dict[int, int] = {}            # frames in flight per stream
        self.max_stream_inflight = 0
        t0 = self.clock()
        now = lambda: self.clock() - t0
        while nxt < len(reqs) or pending or inflight:
            t = now()
            # arrivals up to now (offline: everything); a request larger than
            # the whole budget can never run and is rejected on arrival
            while nxt < len(reqs) and (not realtime or reqs[nxt].t_arrival <= t):
                r = reqs[nxt]
                nxt += 1
                if self.ex.request_bytes(r) > self.budget:
                    r.error = "budget"
                    r.t_start = r.t_done = now()
                else:
                    pending.append(r)
            # completions free their slot and their memory
            still = []
            for tok, b, off in inflight:
                if self.ex.done(tok):
                    td = now()
                    for r in b:
                        r.t_done = td
                        live[r.stream] -= 1
                    arena.free(off)
                else:
                    still.append((tok, b, off))
            inflight = still
            # admission: oldest first, while a slot is free and memory fits;
            # a request that does not fit lets younger, smaller ones pass
            if pending and len(inflight) < self.max_inflight:
                free = self.budget - arena.used
                batch, rest, need = [], [], 0
                taken: Dict[int, int] = {}       # frames of each stream in this batch
                blocked = set()                  # streams whose next frame waits
                for i, r in enumerate(pending):
                    if len(batch) == self.max_batch:
                        rest.extend(pending[i:])
                        break
                    n_s = live.get(r.stream, 0) + taken.get(r.stream, 0)
                    if r.stream in blocked or (cap is not None and n_s >= cap):
                        blocked.add(r.stream)    # keeps the stream's frames in order
                        rest.append(r)
                        continue
                    rb = self.ex.request_bytes(r)
                    if need + rb <= free:
                        batch.append(r)
                        taken[r.stream] = taken.get(r.stream, 0) + 1
                        need += rb
                    else:
                        blocked.add(r.stream)
                        rest.append(r)
                pending = rest
                off = arena.alloc(need) if batch else None
                if batch and off is None:       # fragmented: retry after a completion
                    pending = sorted(batch + pending, key=lambda r: (r.t_arrival, r.rid))
                    batch = []
                if batch:
                    ts = now()
                    try:
                        tok = self.ex.launch(batch, slot, off)
                    except Exception as e:  # executor failure: this batch errors out
                        arena.free(off)
                        for r in batch:
                            r.error = f"launch: {e}"
                            r.t_start = r.t_done = now()
                        continue
                    slot = (slot + 1) % self.max_inflight
                    for r in batch:
                        r.t_start = ts
                        live[r.stream] = live.get(r.stream, 0) + 1
                        self.max_stream_inflight = max(self.max_stream_inflight, live[r.stream])
                    inflight.append((tok, batch, off))
                    batches.append(len(batch))
            if realtime and not pending and not inflight and nxt < len(reqs):
                # idle until the next arrival
                dt = reqs[nxt].t_arrival - now()
                if dt > 2e-4:
                    time.sleep(dt - 1e-4)
        wall = now()
        ok = [r for r in reqs if r.error is None]
        lat = np.array([(r.t_done - r.t_arrival) * 1e3 for r in ok]) if ok else np.array([np.nan])
        span = (max(r.t_done for r in ok) - min(r.t_arrival for r in ok)) if ok else 0.0
        return ServeStats(
            frames=len(ok), errors=len(reqs) - len(ok), wall_s=wall,
            frames_per_s=len(ok) / span if span > 0 else float("nan"),
            p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
            mean_batch=float(np.mean(batches)) if batches else 0.0,
            max_batch=max(batches) if batches else 0, batches=len(batches))


def fifo_single(executor: Executor, requests: List[Request], realtime: bool = True,
                clock: Callable[[], float] = time.perf_counter) -> ServeStats:
    """The plain loop: one frame at a time in arrival order, each waited for."""
    reqs = sorted(requests, key=lambda r: r.t_arrival)
    t0 = clock()
    now = lambda: clock() - t0
    for r in reqs:
        if realtime:
            dt = r.t_arrival - now()
            if dt > 2e-4:
                time.sleep(dt - 1e-4)
            while now() < r.t_arrival:
                pass
        r.t_start = now()
        tok = executor.launch([r], 0, 0)
        executor.wait(tok)
        r.t_done = now()
    lat = np.array([(r.t_done - r.t_arrival) * 1e3 for r in reqs])
    span = max(r.t_done for r in reqs) - min(r.t_arrival for r in reqs)
    return ServeStats(frames=len(reqs), errors=0, wall_s=now(), frames_per_s=len(reqs) / span,
                      p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                      mean_batch=1.0, max_batch=1, batches=len(reqs))


class GpuExecutor(Executor):
    """Runs batches through libwskp on ``slots`` HIP streams (with
    ``graph``, each batch replays the graph of its stream and capacity
    bucket).

    Every stream of the trace owns resident device buffers: its input frames
    (one frame, or a list that frame ``seq`` of the stream reads at index
    seq % len) and an output ring of ``ring`` frames (default slots + 1):
    frame ``seq`` writes ring slot seq % ring, and at most ``ring`` frames of
    a stream are in flight at once (``per_stream_cap``), so no two frames in
    flight share an output.  One workspace of ``ws_bytes`` (the admission
    budget) is shared by the in-flight batches; the server hands each batch a
    disjoint range of it.
    """

    def __init__(self, denoiser, stream_inputs: Dict[int, "object"], ws_bytes: int,
                 slots: int = 2, ring: Optional[int] = None, graph: bool = False,
                 temporal: bool = False):
        import torch
        from . import wskp
        self.torch = torch
        self.wskp = wskp
        self.dn = denoiser
        self.inputs = {s: (f if isinstance(f, (list, tuple)) else [f])
                       for s, f in stream_inputs.items()}
        ring = slots + 1 if ring is None else ring
        self.per_stream_cap = ring
        # temporal accumulation (Sec. 4.1): each stream keeps its accumulated
        # radiance and history length on the device, in two slots that
        # consecutive frames alternate between; a frame reads the previous
        # frame's slot, so a stream has one frame in flight at a time
        self.temporal = temporal
        if temporal:
            self.per_stream_cap = 1
            self.state = {s: [(torch.empty_like(f[0]["radiance"]),
                               torch.empty(f[0]["radiance"].shape[:2], dtype=torch.float32,
                                           device=f[0]["radiance"].device)) for _ in range(2)]
                          for s, f in self.inputs.items()}
        # graph replay: one HIP graph per stream and capacity bucket
        self.flags = wskp.BATCH_GRAPH if graph else 0
        self.outputs = {s: [torch.empty_like(f[0]["radiance"]) for _ in range(ring)]
                        for s, f in self.inputs.items()}
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        self._one: Dict[Tuple[int, int], int] = {}

    def workspace_bytes(self, reqs: List[Request]) -> int:
        return self.wskp.wskp_workspace_size(self.dn.h, [r.H for r in reqs], [r.W for r in reqs])

    def request_bytes(self, r: Request) -> int:
        key = (r.H, r.W)
        if key not in self._one:
            self._one[key] = self.workspace_bytes([r])
        return self._one[key]

    def output_of(self, stream: int, k: int):
        ring = self.outputs[stream]
        return ring[k % len(ring)]

    def input_of(self, stream: int, k: int):
        ins = self.inputs[stream]
        return ins[k % len(ins)]

    def launch(self, reqs: List[Request], slot: int, ws_offset: int = 0):
        s = self.streams[slot]
        frames = []
        for r in reqs:
            src = self.input_of(r.stream, r.seq)
            f = {k: src[k] for k in ("radiance", "albedo", "normal", "depth")}
            if self.temporal:
                acc, ln = self.state[r.stream][r.seq % 2]
                prev = None
                if r.seq > 0:
                    pa, pl = self.state[r.stream][(r.seq - 1) % 2]
                    ps = self.input_of(r.stream, r.seq - 1)
                    prev = {"radiance": pa, "length": pl, "normal": ps["normal"], "wpos": ps["wpos"]}
                self.wskp.wskp_temporal(self.dn.h, src["radiance"], src["normal"], src["wpos"],
                                        src["motion"], prev, acc, ln, stream=s)
                f["radiance"] = acc
            f["out"] = self.output_of(r.stream, r.seq)
            frames.append(f)
        need = self.workspace_bytes(reqs)
        self.wskp.wskp_denoise_batch(self.dn.h, frames, self.ws[ws_offset:ws_offset + need],
                                     self.flags, s)
        ev = self.torch.cuda.Event()
        ev.record(s)
        return ev

    def done(self, token) -> bool:
        return token.query()

    def wait(self, token) -> None:
        token.synchronize()
