"""Request loop over the library's continuous-batching calls.

A request is an image, its lambda and adjacency.  Requests wait in a FIFO
until the device-side serving budget has room for them (Context.serve_admit,
admission by the twin and tile-state footprint); every iteration then runs a
few rounds over all resident images at once (Context.serve_step), so
requests that arrive while others are in flight join the running batch at
the next round, and each image leaves as soon as it is stable.

A request may come from host memory: its pinned host input is copied to its
device buffer on a copy stream when it arrives (it is admitted once that
copy is done), and its result is copied back to a pinned host output on the
same stream as soon as it retires.  The copies run on the GPU's copy engines
while other images' rounds run.  Latency is taken on the host, from a
request's arrival time to the moment its result is visible on the host (the
copy back observed complete), or, for a device-only request, to the return
of the step that retired it (its result is then final in its own device
buffer).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from .thin import Context, Stats


@dataclass
class Request:
    tag: int
    image: object          # 2-D uint8/uint16 device tensor, thinned in place
    lam: int
    adj: object = "8,4"
    arrival: float = 0.0   # seconds from the start of the replay
    host_in: object = None   # pinned host tensor copied into `image` on arrival
    host_out: object = None  # pinned host tensor that receives the result


@dataclass
class Report:
    images: int
    pixels: int
    wall_s: float
    steps: int
    latencies_s: np.ndarray
    stats: dict = field(default_factory=dict)      # tag -> Stats
    max_resident: int = 0

    @property
    def images_per_s(self) -> float:
        return self.images / self.wall_s if self.wall_s > 0 else 0.0

    @property
    def mpixel_per_s(self) -> float:
        return self.pixels / self.wall_s / 1e6 if self.wall_s > 0 else 0.0

    def percentile_ms(self, q: float) -> float:
        return float(np.percentile(self.latencies_s, q) * 1e3) if len(self.latencies_s) else 0.0


class Server:
    """FIFO admission in front of one Context's serving calls, with the
    host-to-device and device-to-host copies of host requests on
    `copy_stream` (a torch CUDA stream of default priority)."""

    def __init__(self, ctx: Context, rounds_per_step: int = 2, copy_stream=None):
        self.ctx = ctx
        self.rounds = rounds_per_step
        self.copy_stream = copy_stream
        self.queue: collections.deque[Request] = collections.deque()
        self.in_flight: dict[int, Request] = {}
        self.copy_in: dict[int, object] = {}    # tag -> event of its input copy
        self.copy_out: list = []                # (Request, Stats, event of its output copy)
        self.steps = 0

    def submit(self, req: Request):
        if req.host_in is not None:
            import torch
            with torch.cuda.stream(self.copy_stream):
                req.image.copy_(req.host_in, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(self.copy_stream)
            self.copy_in[req.tag] = ev
        self.queue.append(req)

    def _admit(self):
        while self.queue:
            req = self.queue[0]
            ev = self.copy_in.get(req.tag)
            if ev is not None and not ev.query():
                return                      # its input is still on the way
            if not self.ctx.serve_admit(req.image, req.lam, req.adj, req.tag):
                if not self.in_flight:
                    raise RuntimeError(f"request {req.tag} ({tuple(req.image.shape)}) can never "
                                       "fit the serving budget")
                return
            self.copy_in.pop(req.tag, None)
            self.queue.popleft()
            self.in_flight[req.tag] = req

    def step(self):
        """Admits what fits, runs one step; returns [(Request, Stats)] whose
        results are final: on the device for device requests, on the host
        for host requests (their copies back are polled here)."""
        self._admit()
        done, _ = self.ctx.serve_step(self.rounds if self.in_flight else 0)
        self.steps += 1
        out = []
        for tag, st in done:
            req = self.in_flight.pop(tag)
            if req.host_out is None:
                out.append((req, st))
                continue
            import torch
            # serve_step returned, so the result is final in req.image
            with torch.cuda.stream(self.copy_stream):
                req.host_out.copy_(req.image, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(self.copy_stream)
            self.copy_out.append((req, st, ev))
        return out + self.poll()

    def poll(self):
        """Host requests whose results have reached the host since the last call."""
        ready = [(r, st) for r, st, ev in self.copy_out if ev.query()]
        if ready:
            tags = {r.tag for r, _ in ready}
            self.copy_out = [x for x in self.copy_out if x[0].tag not in tags]
        return ready

    @property
    def idle(self) -> bool:
        return not self.queue and not self.in_flight and not self.copy_out


def replay(ctx: Context, requests, rounds_per_step: int = 2, clock=time.perf_counter,
           copy_stream=None) -> Report:
    """Feeds `requests` (sorted by arrival) to a Server in real time and
    returns throughput and per-request latency.  Device requests must already
    be on the device; host requests are copied in and out on copy_stream.
    The clock starts at the first arrival."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    srv = Server(ctx, rounds_per_step, copy_stream)
    lat = {}
    stats = {}
    nxt = 0
    t0 = clock() - (reqs[0].arrival if reqs else 0.0)
    last = t0
    max_res = 0
    while nxt < len(reqs) or not srv.idle:
        now = clock() - t0
        while nxt < len(reqs) and reqs[nxt].arrival <= now:
            srv.submit(reqs[nxt])
            nxt += 1
        if srv.idle:
            # Nothing to do before the next arrival.
            while clock() - t0 < reqs[nxt].arrival:
                pass
            continue
        if not srv.in_flight and not srv.queue:
            finished = srv.poll()        # only copies back are left
        else:
            finished = srv.step()
        for req, st in finished:
            last = clock()
            lat[req.tag] = (last - t0) - req.arrival
            stats[req.tag] = st
        max_res = max(max_res, len(srv.in_flight))
    wall = last - t0 - (reqs[0].arrival if reqs else 0.0)
    pixels = sum(int(r.image.shape[0]) * int(r.image.shape[1]) for r in reqs)
    return Report(images=len(reqs), pixels=pixels, wall_s=wall, steps=srv.steps,
                  latencies_s=np.array([lat[r.tag] for r in reqs]), stats=stats,
                  max_resident=max_res)
