"""Request loop over the library's continuous-batching calls.

A request is a device image, its lambda and adjacency.  Requests wait in a
FIFO until the device-side serving budget has room for them
(Context.serve_admit, admission by the twin and tile-state footprint); every
iteration then runs a few rounds over all resident images at once
(Context.serve_step), so requests that arrive while others are in flight
join the running batch at the next round, and each image leaves as soon as
it is stable.  Latency is taken on the host, from a request's arrival time
to the return of the step that retired it (its result is then final in its
own device buffer).
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
    """FIFO admission in front of one Context's serving calls."""

    def __init__(self, ctx: Context, rounds_per_step: int = 2):
        self.ctx = ctx
        self.rounds = rounds_per_step
        self.queue: collections.deque[Request] = collections.deque()
        self.in_flight: dict[int, Request] = {}
        self.steps = 0

    def submit(self, req: Request):
        self.queue.append(req)

    def _admit(self):
        while self.queue:
            req = self.queue[0]
            if not self.ctx.serve_admit(req.image, req.lam, req.adj, req.tag):
                if not self.in_flight:
                    raise RuntimeError(f"request {req.tag} ({tuple(req.image.shape)}) can never "
                                       "fit the serving budget")
                return
            self.queue.popleft()
            self.in_flight[req.tag] = req

    def step(self):
        """Admits what fits, runs one step; returns [(Request, Stats)] retired."""
        self._admit()
        done, _ = self.ctx.serve_step(self.rounds if self.in_flight else 0)
        self.steps += 1
        return [(self.in_flight.pop(tag), st) for tag, st in done]

    @property
    def idle(self) -> bool:
        return not self.queue and not self.in_flight


def replay(ctx: Context, requests, rounds_per_step: int = 2, clock=time.perf_counter) -> Report:
    """Feeds `requests` (sorted by arrival) to a Server in real time and
    returns throughput and per-request latency.  Inputs must already be on
    the device; the clock starts at the first arrival."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    srv = Server(ctx, rounds_per_step)
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
        for req, st in srv.step():
            last = clock()
            lat[req.tag] = (last - t0) - req.arrival
            stats[req.tag] = st
        max_res = max(max_res, len(srv.in_flight))
    wall = last - t0 - (reqs[0].arrival if reqs else 0.0)
    pixels = sum(int(r.image.shape[0]) * int(r.image.shape[1]) for r in reqs)
    return Report(images=len(reqs), pixels=pixels, wall_s=wall, steps=srv.steps,
                  latencies_s=np.array([lat[r.tag] for r in reqs]), stats=stats,
                  max_resident=max_res)
