"""Shared setup for the GPU parity tests: the same seeded inputs go to the
HIP path (through the C ABI binding) and to the CPU oracle."""
import numpy as np


def make_pair(rfim_mod, oracle_mod, L, R, J, h, fields, temps, seed=0, realization=0, R_cap=0,
              field_kind=-1):
    g = rfim_mod.Rfim(L, R, J, h, fields, temps, seed=seed, realization=realization,
                      field_kind=field_kind, R_cap=R_cap)
    o = oracle_mod.Oracle(L, R, J, h, fields, temps, seed=seed, realization=realization,
                          field_kind=field_kind, R_cap=R_cap)
    return g, o


def assert_same_state(g, o, what=""):
    """Bit-exact comparison of the whole chain state."""
    gs, os_ = g.spins(), o.spins()
    if not np.array_equal(gs, os_):
        diff = np.argwhere(gs != os_)
        raise AssertionError("%s spins differ at %d places, first %s" % (what, len(diff), diff[:5].tolist()))
    assert np.array_equal(g.perm(), o.perm()), what + " t2r"
    assert g.counters() == o.counters(), what + " counters"
    ga, gc = g.exchange_stats()
    oa, oc = o.exchange_stats()
    assert np.array_equal(ga, oa) and np.array_equal(gc, oc), what + " exchange stats"
    assert np.array_equal(g.temps(), o.temps()), what + " temps"
    assert np.array_equal(g.energies(), o.energies()), what + " energies"
    assert np.array_equal(g.magnetizations(), o.magnetizations()), what + " magnetizations"
