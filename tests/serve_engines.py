"""A CPU engine for the serving loop, built on the oracle (test
infrastructure): the same admit / step / poll / result / release protocol as
the GPU pool (which runs each request's schedule itself: the insertion step
after every trial run, completion after the production sweeps), with a byte
budget and a virtual clock that advances with the work done."""
import numpy as np

from oracle.oracle import Oracle


class _Job:
    def __init__(self, o, need, spec):
        a = getattr(spec, "adapt", None) or {}
        self.o, self.need, self.spec = o, need, spec
        self.trials = int(a.get("trials", 0))
        self.S = int(a.get("sweeps_per_trial", 0)) if self.trials else 0
        self.P = int(spec.sweeps)
        self.threshold = float(a.get("rate_threshold", 0.0))
        self.max_insert = int(a.get("max_insert_per_trial", 0))
        self.R_cap = int(getattr(spec, "R_cap", 0) or spec.R)
        self.done = 0
        self.trials_done = 0
        self.finished = False
        self.attempts = 0


class OracleEngine:
    def __init__(self, budget_bytes, clock=None, ns_per_attempt=1.0, fail_alloc=False):
        self.budget = budget_bytes
        self.reserved = 0
        self.slots = {}
        self.clock = clock
        self.ns_per_attempt = ns_per_attempt
        self.fail_alloc = fail_alloc
        self.log = []

    def bytes_needed(self, spec):
        R_cap = int(getattr(spec, "R_cap", 0) or spec.R)
        return R_cap * spec.L ** 3 + 4 * spec.L ** 3

    def admit(self, spec):
        if self.fail_alloc:
            raise RuntimeError("device allocation failed")
        need = self.bytes_needed(spec)
        if self.reserved + need > self.budget:
            return None
        o = Oracle(spec.L, spec.R, spec.J, spec.h, spec.fields, spec.temps, seed=spec.seed,
                   realization=spec.realization, R_cap=int(getattr(spec, "R_cap", 0) or 0))
        slot = 0
        while slot in self.slots:
            slot += 1
        self.slots[slot] = _Job(o, need, spec)
        self.reserved += need
        self.log.append(("admit", slot))
        return slot

    def step(self, quantum, every):
        work = 0
        running = 0
        for slot, j in sorted(self.slots.items()):
            if j.finished:
                continue
            running += 1
            j.o.sweep(quantum, every)
            n = j.o.R * j.spec.L ** 3 * quantum
            j.attempts += n
            work += n
            j.done += quantum
            if j.trials_done < j.trials and j.done == (j.trials_done + 1) * j.S:
                j.o.insert_step(j.threshold, j.max_insert, j.R_cap)
                j.trials_done += 1
            if j.trials_done == j.trials and j.done == j.trials * j.S + j.P:
                j.finished = True
        if self.clock is not None:
            self.clock.advance(work * self.ns_per_attempt * 1e-9)
        self.log.append(("step", running))

    def sync(self):
        pass

    def poll(self):
        return [s for s, j in sorted(self.slots.items()) if j.finished]

    def result(self, slot):
        j = self.slots[slot]
        o = j.o
        return dict(R=o.R, temps=o.temps(), energies=o.energies(), perm=o.perm(),
                    magnetizations=o.magnetizations(), attempts=j.attempts, finished=j.finished)

    def release(self, slot):
        j = self.slots.pop(slot)
        self.reserved -= j.need
        j.o.close()
        self.log.append(("release", slot))


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt):
        self.t += dt

    def sleep(self, dt):
        self.t += max(dt, 1e-6)
