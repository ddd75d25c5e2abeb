"""A CPU engine for the serving loop, built on the oracle (test
infrastructure): same admit / step / adapt / collect / release protocol as
the GPU pool, with a byte budget and a virtual clock that advances with the
work done."""
import numpy as np

from oracle.oracle import Oracle


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
        self.slots[slot] = (o, need, spec)
        self.reserved += need
        self.log.append(("admit", slot))
        return slot

    def step(self, quantum, every):
        work = 0
        for slot, (o, _, spec) in sorted(self.slots.items()):
            o.sweep(quantum, every)
            work += o.R * spec.L ** 3 * quantum
        if self.clock is not None:
            self.clock.advance(work * self.ns_per_attempt * 1e-9)
        self.log.append(("step", len(self.slots)))

    def sync(self):
        pass

    def adapt(self, slot, rate_threshold, max_insert, R_cap):
        return self.slots[slot][0].insert_step(rate_threshold, max_insert, R_cap)

    def collect(self, slot):
        o = self.slots[slot][0]
        return dict(R=o.R, temps=o.temps(), energies=o.energies(), perm=o.perm(),
                    magnetizations=o.magnetizations())

    def release(self, slot):
        o, need, _ = self.slots.pop(slot)
        self.reserved -= need
        o.close()
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
