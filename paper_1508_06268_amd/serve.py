"""Serving loop: continuous batching of realization requests.

Requests (one disorder realization each, with the paper's adaptive schedule:
short trial runs with temperature insertion, Sec. 4, then production sweeps)
arrive over time.  The loop admits waiting requests whenever the engine's
device-memory budget can hold them, advances every admitted realization
together in quanta of whole exchange intervals, runs each request's
insertion step in place when its trial run ends, and collects and releases
requests as they finish; requests that arrive while others run join the
running set at the next quantum boundary.  It reports per-request latency
(completion - arrival) with p50/p99, throughput and utilization.

The loop talks to an engine (admit / step / poll / result / release):
admit hands over a request with its whole schedule, the engine runs the
insertion steps and reports finished requests through poll.  `PoolEngine`
drives the GPU pool of librfim through rfim_pool_admit_job,
rfim_pool_step, rfim_pool_poll and rfim_pool_result.  Any object with the
same methods works (the tests use a CPU engine and a virtual clock).
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float      # seconds after the start of the run
    spec: object        # workloads.Realization (with .adapt and .sweeps)


@dataclasses.dataclass
class Outcome:
    rid: int
    arrival: float
    admitted: Optional[float] = None
    finished: Optional[float] = None
    error: Optional[str] = None
    R: int = 0
    temps: Optional[np.ndarray] = None
    energies: Optional[np.ndarray] = None
    perm: Optional[np.ndarray] = None
    magnetizations: Optional[np.ndarray] = None
    attempts: int = 0

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


class PoolEngine:
    """Engine over the librfim pool (GPU)."""

    def __init__(self, budget_bytes: int, stream=None, shapes=None):
        from .rfim import Pool

        self.pool = Pool(budget_bytes, stream=stream)
        for (L, kind), shape in (shapes or {}).items():
            self.pool.set_shape(L, kind, *shape)

    def bytes_needed(self, spec) -> int:
        return self.pool.bytes_needed(spec)

    def admit(self, spec):
        """Slot id with the request's schedule, or None if the budget is full."""
        return self.pool.admit_job(spec)

    def step(self, quantum: int, every: int) -> None:
        self.pool.step(quantum, every)

    def sync(self) -> None:
        self.pool.synchronize()

    def poll(self):
        return self.pool.poll()

    def result(self, slot) -> dict:
        return self.pool.result(slot)

    def release(self, slot) -> None:
        self.pool.release(slot)

    def close(self):
        self.pool.close()


def schedule(spec):
    """(trials, sweeps per trial, production sweeps, every) of a request."""
    a = getattr(spec, "adapt", None) or {}
    return (int(a.get("trials", 0)), int(a.get("sweeps_per_trial", 0)), int(spec.sweeps),
            int(a.get("every", spec.every)))


class Server:
    def __init__(self, engine, quantum: int = 50, every: int = 10,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, log=None):
        if quantum % every:
            raise ValueError("quantum must be a multiple of the exchange interval")
        self.engine = engine
        self.quantum = quantum
        self.every = every
        self.clock = clock
        self.sleep = sleep
        self.log = log

    def _check(self, spec):
        trials, S, P, every = schedule(spec)
        if every != self.every:
            raise ValueError("request exchange interval %d differs from the server's %d" % (every, self.every))
        if trials < 0 or (trials > 0 and S < 1) or P < 1:
            raise ValueError("a request needs production sweeps >= 1 and, with trial runs, trial sweeps >= 1")
        if S % self.quantum or P % self.quantum:
            raise ValueError("trial and production sweeps must be multiples of the quantum %d" % self.quantum)

    def run(self, requests: List[Request]) -> Dict[str, object]:
        eng = self.engine
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque = collections.deque()
        active: Dict[int, Outcome] = {}
        outcomes: Dict[int, Outcome] = {}
        t0 = self.clock()
        busy_steps = 0
        max_active = 0
        while pending or waiting or active:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admit in arrival order while the budget holds them
            while waiting:
                req = waiting[0]
                out = Outcome(req.rid, req.arrival)
                try:
                    self._check(req.spec)
                    slot = eng.admit(req.spec)
                except (ValueError, RuntimeError) as exc:   # this request only
                    waiting.popleft()
                    out.error = str(exc)
                    outcomes[req.rid] = out
                    continue
                if slot is None:
                    if not active:      # cannot fit even into an empty pool
                        waiting.popleft()
                        out.error = "larger than the device-memory budget"
                        outcomes[req.rid] = out
                        continue
                    break
                waiting.popleft()
                out.admitted = now
                active[slot] = out
            if not active:
                if pending:
                    self.sleep(max(0.0, pending[0].arrival - (self.clock() - t0)))
                continue
            max_active = max(max_active, len(active))
            eng.step(self.quantum, self.every)
            eng.sync()
            busy_steps += 1
            # the engine runs each request's schedule (insertion steps after
            # its trial runs) and reports the finished ones
            for slot in eng.poll():
                out = active.pop(slot)
                res = eng.result(slot)
                eng.release(slot)
                out.finished = self.clock() - t0
                for k in ("R", "temps", "energies", "perm", "magnetizations", "attempts"):
                    setattr(out, k, res[k])
                out.attempts = int(out.attempts)
                outcomes[out.rid] = out
        wall = self.clock() - t0
        done = [o for o in outcomes.values() if o.finished is not None]
        lat = np.array([o.latency for o in done]) if done else np.zeros(0)
        stats = {
            "requests": len(requests), "completed": len(done),
            "failed": sum(1 for o in outcomes.values() if o.error),
            "wall_s": wall, "realizations_per_s": len(done) / wall if wall > 0 else 0.0,
            "latency_p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "latency_p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "latency_mean_s": float(lat.mean()) if len(lat) else None,
            "steps": busy_steps, "max_active": max_active,
            "attempts": int(sum(o.attempts for o in done)),
        }
        return {"outcomes": outcomes, "stats": stats}


def run_alone(engine_factory, req: Request, quantum: int, every: int) -> Outcome:
    """The same request through an engine holding nothing else."""
    eng = engine_factory()
    srv = Server(eng, quantum=quantum, every=every, clock=_VirtualClock(), sleep=lambda s: None)
    out = srv.run([Request(req.rid, 0.0, req.spec)])["outcomes"][req.rid]
    return out


class _VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3
        return self.t
