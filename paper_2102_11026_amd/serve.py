"""Served form: a request loop over slot pools (continuous batching).

Each request is one simulation instance of a request class (its own seeded
initial state) that asks for a number of implicit-Euler steps.  Requests arrive
as a seeded Poisson stream, wait in a FIFO, and are admitted while the context's
HBM budget and the class pool have room.  Every tick advances all live
instances by one step with one graph launch per class pool; a request that
arrives while others are on the GPU joins at the next tick, and a finished one
leaves its slot (its instance is kept for reuse by the next request of the
class).  Per-step latency is the wall time of the tick that advanced the
instance.  All compute runs in the library's kernels; this module only
schedules.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Dict, List

import numpy as np

from . import nmr, synth


@dataclass
class RequestClass:
    name: str
    problem: "synth.Problem"
    capacity: int
    decoder: object = None
    pool: object = None
    free: List[object] = field(default_factory=list)   # retired instances kept for reuse


@dataclass
class Request:
    rid: int
    cls: str
    t_arrive: float
    steps_left: int
    r0: np.ndarray
    inst: object = None
    slot: int = -1
    t_admit: float = 0.0


def poisson_arrivals(rate: float, horizon: float, class_names, steps: int, problems: Dict[str, object],
                     seed: int = synth.MASTER_SEED) -> List[Request]:
    """Seeded Poisson arrivals over [0, horizon) with a uniform class mix;
    each request seeds only its own q0 ~ N(0, 0.1^2)."""
    n_max = int(rate * horizon * 2 + 50)
    gaps = -np.log(synth.uniform("arrivals", n_max, seed)) / rate
    times = np.cumsum(gaps)
    times = times[times < horizon]
    cls_draw = synth.raw64("class", times.size, seed) % np.uint64(len(class_names))
    reqs = []
    for k, (t, c) in enumerate(zip(times, cls_draw)):
        name = class_names[int(c)]
        p = problems[name]
        r0 = np.zeros(p.R)
        r0[p.n_p:] = 0.1 * synth.normal(f"serve/q0/{k}", p.n_q, seed)
        reqs.append(Request(rid=k, cls=name, t_arrive=float(t), steps_left=steps, r0=r0))
    return reqs


class Server:
    def __init__(self, ctx: "nmr.Context", classes: List[RequestClass], prec: str, n_iters: int,
                 keep_results: bool = False):
        self.ctx, self.prec, self.n_iters = ctx, prec, n_iters
        self.results = {} if keep_results else None
        self.classes = {c.name: c for c in classes}
        for c in classes:
            p = c.problem
            c.decoder = nmr.Decoder(ctx, p.weights, p.biases, p.act, prec)
            c.pool = nmr.Pool(ctx, c.capacity)

    def _admit(self, req: Request) -> bool:
        c = self.classes[req.cls]
        if len(c.free):
            inst = c.free.pop()
        else:
            try:
                inst = nmr.Instance(self.ctx, c.problem, self.prec, shared=c.decoder)
            except nmr.NmrError as e:
                if nmr.STATUS.get(e.code) in ("budget", "oom"):
                    return False
                raise
        inst.set_state(req.r0, np.zeros_like(req.r0))
        try:
            req.slot = c.pool.attach(inst)
        except nmr.NmrError as e:
            if nmr.STATUS.get(e.code) != "budget":
                raise
            c.free.append(inst)
            return False
        req.inst = inst
        return True

    def _retire(self, req: Request):
        c = self.classes[req.cls]
        if self.results is not None and req.steps_left == 0:
            self.results[req.rid] = req.inst.get_state()
        c.pool.detach(req.slot)
        c.free.append(req.inst)
        req.inst = None

    def run(self, requests: List[Request], max_seconds: float, log=None) -> dict:
        import torch
        pending = sorted(requests, key=lambda r: r.t_arrive)
        fifo: List[Request] = []
        live: List[Request] = []
        step_ms: List[float] = []
        wait_ms: List[float] = []
        done = 0
        iters = 0
        max_live = 0
        t0 = time.perf_counter()
        nxt = 0
        ticks = 0
        while (nxt < len(pending) or fifo or live) and time.perf_counter() - t0 < max_seconds:
            now = time.perf_counter() - t0
            while nxt < len(pending) and pending[nxt].t_arrive <= now:
                fifo.append(pending[nxt])
                nxt += 1
            while fifo:
                if not self._admit(fifo[0]):
                    break
                req = fifo.pop(0)
                req.t_admit = time.perf_counter() - t0
                wait_ms.append(1000.0 * (req.t_admit - req.t_arrive))
                live.append(req)
            if not live:
                if nxt < len(pending):
                    time.sleep(max(0.0, min(pending[nxt].t_arrive - (time.perf_counter() - t0), 0.01)))
                continue
            max_live = max(max_live, len(live))
            ta = time.perf_counter()
            for c in self.classes.values():
                if any(r.cls == c.name for r in live):
                    c.pool.step(self.n_iters, status=False, timing=False)
            torch.cuda.synchronize()
            tick_ms = 1000.0 * (time.perf_counter() - ta)
            ticks += 1
            still = []
            for r in live:
                step_ms.append(tick_ms)
                iters += self.n_iters
                r.steps_left -= 1
                if r.steps_left == 0:
                    self._retire(r)
                    done += 1
                else:
                    still.append(r)
            live = still
            if log and ticks % 200 == 0:
                log(f"serve t={time.perf_counter() - t0:.1f}s live={len(live)} fifo={len(fifo)} done={done}")
        elapsed = time.perf_counter() - t0
        for r in live:  # time cap reached: release the slots of unfinished requests
            self._retire(r)
        sm = np.asarray(step_ms) if step_ms else np.zeros(1)
        wm = np.asarray(wait_ms) if wait_ms else np.zeros(1)
        return dict(requests=len(pending), arrived=nxt, admitted=len(wait_ms), completed=done, ticks=ticks,
                    max_live=max_live, elapsed_s=round(elapsed, 3),
                    newton_iters_per_s=round(iters / elapsed, 1),
                    p50_step_ms=round(float(np.percentile(sm, 50)), 4),
                    p99_step_ms=round(float(np.percentile(sm, 99)), 4),
                    p50_admission_wait_ms=round(float(np.percentile(wm, 50)), 2),
                    p99_admission_wait_ms=round(float(np.percentile(wm, 99)), 2))

    def close(self):
        for c in self.classes.values():
            for x in c.free:
                x.close()
            c.free.clear()
            c.pool.close()
            c.decoder.close()
