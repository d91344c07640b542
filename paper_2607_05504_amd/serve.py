"""Served form: continuous batching of SIDM steps from many independent haloes.

Requests (one isolated halo each: particles, cross-section, seed, a number of
steps) arrive over time.  A request is admitted when a slot is free and its
device memory -- a library context sized to it plus its particle state --
fits the HBM budget; its state then stays resident on the device until its
last step.  Every slot has its own HIP stream (default priority) and its own
context, so the steps of different requests run concurrently on the GPU; the
host loop keeps at most ``depth`` steps of each slot in flight and refills a
slot as soon as one of its steps completes, so requests that arrive while
others run start without waiting for them to finish.

One step of a request is the scattering step through the C ABI
(sidm_build_tree, sidm_find_ngb, sidm_scatter_step, sidm_pair_timestep) and
then sidm_advance_hernquist, the leapfrog step in the halo's potential that
stands in for gravity and sets the next global step length from the
per-pair bounds; the first step's length comes from the bounds of the
initial state, computed at admission.  The step latency reported is the device time of the
scattering part, from events on the slot's stream; request latency is
arrival to completion on the host clock.

Contexts are pooled by capacity class (powers of two) and reused; an idle
context is destroyed only when the budget needs its memory.
"""
from __future__ import annotations

import collections
import dataclasses
import sys
import time
from typing import Callable, Optional

import numpy as np

from . import FP64, Context, footprint, runner

STATE_BYTES_PER_PARTICLE = 6 * 8 + 4 + 1 + 4 + 8 + 8 + 8   # x, v, id, state, active, dt, h, dt_sidm


def state_bytes(n: int, k: int) -> int:
    return n * (STATE_BYTES_PER_PARTICLE + 4 * k)


def capacity_class(n: int) -> int:
    c = 16384
    while c < n:
        c *= 2
    return c


@dataclasses.dataclass
class ServeConfig:
    n_slots: int = 8
    hbm_budget: int = 4 << 30
    depth: int = 2                 # steps of one slot in flight
    precision: int = FP64
    dt_cap: float = 0.25           # t_dyn(a) / 8 of the G = M = a = 1 halo
    gm: float = 1.0
    a: float = 1.0
    keep_results: bool = False     # copy each request's final state to the host
    progress_s: float = 0.0        # > 0: a progress line on stderr this often


@dataclasses.dataclass
class _Active:
    req: object
    w: object
    ds: object
    out: object
    ctx: Context
    cap: int
    mem: int
    admitted: float
    issued: int = 0
    done_steps: int = 0
    inflight: collections.deque = dataclasses.field(default_factory=collections.deque)
    step_ms: list = dataclasses.field(default_factory=list)
    stats: Optional[dict] = None


class Server:
    def __init__(self, cfg: ServeConfig):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.streams = [torch.cuda.Stream() for _ in range(cfg.n_slots)]   # default priority
        self.pool = collections.defaultdict(list)      # capacity -> idle contexts
        self.pool_mem = 0
        self.used = 0                                    # bytes held by running requests

    # -- memory --------------------------------------------------------------
    def _config(self, w, cap):
        # every step's length keeps all P(i|j) below C_SIDM (the first one's
        # from the bound at admission), so a step lists far fewer candidates
        # than there are particles; half of them is room to spare
        return runner.config_for(w, precision=self.cfg.precision,
                                 max_accept=max(cap // 2, 1 << 16))

    def _ctx_bytes(self, w, cap):
        return footprint(self._config(w, cap), cap, cap)

    def _take_ctx(self, w, cap, stream):
        """A context of capacity cap bound to stream, from the pool if one is idle."""
        if self.pool[cap]:
            ctx = self.pool[cap].pop()
            self.pool_mem -= ctx._serve_bytes
            ctx.set_stream(stream)
            ctx.reconfigure(self._config(w, cap))
            return ctx
        ctx = Context(self._config(w, cap), cap, cap, stream=stream)
        ctx._serve_bytes = self._ctx_bytes(w, cap)
        return ctx

    def _fits(self, need, cap):
        """Free idle contexts (largest first, keeping one of class cap) until
        need bytes fit the budget; False if they cannot."""
        reuse = self.pool[cap][-1]._serve_bytes if self.pool[cap] else 0
        while self.used + self.pool_mem + need - reuse > self.cfg.hbm_budget:
            victims = [c for c, lst in self.pool.items() if lst and not (c == cap and len(lst) == 1)]
            if not victims:
                return False
            c = max(victims)
            ctx = self.pool[c].pop()
            self.pool_mem -= ctx._serve_bytes
            ctx.close()
        return True

    # -- the loop --------------------------------------------------------------
    def run(self, requests, make_workload: Callable, on_admit: Optional[Callable] = None):
        """Serve ``requests`` (objects with rid, arrival, n, steps) whose
        workloads ``make_workload(req)`` builds; returns a report dict."""
        torch = self.torch
        cfg = self.cfg
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        slots = [None] * cfg.n_slots
        results, step_ms, req_lat, waits = {}, [], [], []
        particle_steps = 0
        head = None                       # (request, workload) at the head of the queue
        t0 = time.perf_counter()
        first_arrival = pending[0].arrival if pending else 0.0
        n_total, t_report = len(pending), 0.0
        while pending or any(s is not None for s in slots):
            now = time.perf_counter() - t0
            progressed = False
            if cfg.progress_s > 0 and now - t_report >= cfg.progress_s:
                t_report = now
                busy = sum(s is not None for s in slots)
                print(f"[serve] t={now:.0f}s done={len(results)}/{n_total} running={busy} "
                      f"particle-steps={particle_steps:.3g}", file=sys.stderr, flush=True)
            # admission: first come, first served, as slots and memory free up
            while pending and pending[0].arrival <= now:
                free = [k for k, s in enumerate(slots) if s is None]
                if not free:
                    break
                req = pending[0]
                if head is None or head[0] is not req:
                    head = (req, make_workload(req))
                w = head[1]
                cap = capacity_class(w.n)
                need = self._ctx_bytes(w, cap) + state_bytes(w.n, w.n_ngb)
                if need > cfg.hbm_budget:
                    raise ValueError(f"request {req.rid} needs {need} bytes > budget")
                if not self._fits(need, cap):
                    break
                pending.popleft()
                k = free[0]
                stream = self.streams[k]
                with torch.cuda.stream(stream):
                    ds = runner.upload(w, "cuda")
                    out = runner.alloc_out(ds, w.n_ngb)
                    ctx = self._take_ctx(w, cap, stream)
                    self._first_step_length(ctx, ds, out)
                mem = ctx._serve_bytes + state_bytes(w.n, w.n_ngb)
                self.used += mem
                slots[k] = _Active(req, w, ds, out, ctx, cap, mem, admitted=time.perf_counter() - t0)
                waits.append(slots[k].admitted - req.arrival)
                if on_admit:
                    on_admit(req, k)
                progressed = True
            # retire completed steps, refill slots
            for k, s in enumerate(slots):
                if s is None:
                    continue
                while s.inflight and s.inflight[0][2].query():
                    e0, e1, e2 = s.inflight.popleft()
                    s.step_ms.append(e0.elapsed_time(e1))
                    s.done_steps += 1
                    progressed = True
                if s.done_steps == s.req.steps:
                    s.stats = s.ctx.sync()
                    t_end = time.perf_counter() - t0
                    req_lat.append(t_end - s.req.arrival)
                    step_ms.extend(s.step_ms)
                    particle_steps += s.w.n * s.req.steps
                    res = dict(stats=s.stats, step_ms=s.step_ms, n=s.w.n, slot=k,
                               admitted=s.admitted, finished=t_end)
                    if cfg.keep_results:
                        res.update({f: getattr(s.ds, f).cpu().numpy()
                                    for f in ("x", "y", "z", "vx", "vy", "vz", "state")})
                    results[s.req.rid] = res
                    self.used -= s.mem
                    self.pool[s.cap].append(s.ctx)
                    self.pool_mem += s.ctx._serve_bytes
                    slots[k] = None
                    progressed = True
                    continue
                while s.issued < s.req.steps and len(s.inflight) < cfg.depth:
                    self._issue(s, self.streams[k])
                    progressed = True
            if not progressed:
                time.sleep(0.0002)
        wall = time.perf_counter() - t0 - first_arrival
        sm = np.array(step_ms) if step_ms else np.zeros(1)
        return dict(results=results, wall_s=wall, particle_steps=particle_steps,
                    throughput=particle_steps / wall if wall > 0 else 0.0,
                    p50_step_ms=float(np.percentile(sm, 50)), p99_step_ms=float(np.percentile(sm, 99)),
                    p50_request_s=float(np.percentile(req_lat, 50)) if req_lat else 0.0,
                    p99_request_s=float(np.percentile(req_lat, 99)) if req_lat else 0.0,
                    mean_admission_wait_s=float(np.mean(waits)) if waits else 0.0,
                    max_admission_wait_s=float(np.max(waits)) if waits else 0.0,
                    n_requests=len(results))

    def _first_step_length(self, ctx, ds, out):
        """The first step's length, as every later one's: the largest
        dt_cap / 2^b not above the smallest per-pair bound (sec. 4.4) of the
        request's initial state (one host round trip at admission)."""
        ctx.build_tree(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, ds.ids, state=ds.state,
                       m_scalar=ds.mass)
        ctx.find_ngb(ds.active, out.ngb, out.h)
        ctx.pair_timestep(ds.active, out.ngb, out.h, out.dt_sidm, reuse_active=True)
        m = float(out.dt_sidm.min().item()) if out.dt_sidm.numel() else float("inf")
        d, b = float(self.cfg.dt_cap), 0
        while not d <= m and b < 62:
            d *= 0.5
            b += 1
        ds.dt.fill_(d)

    def _issue(self, s: _Active, stream):
        torch = self.torch
        w, ds, out, ctx = s.w, s.ds, s.out, s.ctx
        t = s.issued
        with torch.cuda.stream(stream):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e2 = torch.cuda.Event()
            e0.record(stream)
            runner.run_step(ctx, ds, out, w.seed, w.step + t)
            e1.record(stream)
            ctx.advance_hernquist(ds.x, ds.y, ds.z, ds.vx, ds.vy, ds.vz, out.dt_sidm,
                                  w.n_active, self.cfg.dt_cap, self.cfg.gm, self.cfg.a,
                                  dt_next=ds.dt)
            e2.record(stream)
        s.inflight.append((e0, e1, e2))
        s.issued += 1

    def close(self):
        for lst in self.pool.values():
            for ctx in lst:
                ctx.close()
        self.pool.clear()
        self.pool_mem = 0
