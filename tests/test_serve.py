"""The serving loop (continuous batching) on the CPU: an oracle-backed
engine with a byte budget and a virtual clock.  Covers admission against the
budget, admission while others run, per-request isolation of failures, and
that every request's result is the same alone and in the mix."""
import numpy as np
import pytest

from paper_1508_06268_amd import workloads as W
from paper_1508_06268_amd.serve import Request, Server, run_alone
from serve_engines import OracleEngine, VirtualClock


def _req(rid, arrival, L=4, R=4, kind="g", trial=20, prod=40, every=5, seed=3):
    f = W.gaussian_fields(L, [40, rid]) if kind == "g" else W.bimodal_fields(L, [40, rid])
    R_cap = R + 3
    spec = W.Realization(L=L, R=R, J=1.0, h=1.5, fields=f, temps=W.linear_temps(R, 1.0, 6.0), seed=seed,
                         realization=rid, sweeps=prod, every=every, R_cap=R_cap,
                         adapt=dict(trials=1 if trial else 0, sweeps_per_trial=trial, every=every,
                                    rate_threshold=0.5, max_insert_per_trial=3, R_cap=R_cap))
    return Request(rid, arrival, spec)


def _server(budget, clock=None, **kw):
    clock = clock or VirtualClock()
    eng = OracleEngine(budget, clock=clock, **kw)
    return Server(eng, quantum=10, every=5, clock=clock, sleep=clock.sleep), eng, clock


def _mix():
    return [_req(0, 0.0, L=4, R=4), _req(1, 1e-6, L=6, R=3, kind="b"), _req(2, 2e-5, L=4, R=5, prod=60),
            _req(3, 3e-5, L=2, R=4, kind="b", trial=0), _req(4, 1e-4, L=6, R=4)]


def test_each_result_same_alone_and_in_the_mix():
    srv, eng, _ = _server(10 ** 9)
    res = srv.run(_mix())
    assert res["stats"]["completed"] == 5
    assert res["stats"]["max_active"] >= 3
    for rq in _mix():
        got = res["outcomes"][rq.rid]
        alone = run_alone(lambda: OracleEngine(10 ** 9), rq, 10, 5)
        assert got.R == alone.R
        assert np.array_equal(got.temps, alone.temps)
        assert np.array_equal(got.perm, alone.perm)
        assert np.array_equal(got.energies, alone.energies)


def test_in_the_mix_equals_the_plain_api():
    """A served request equals create + adapt_temps(1 trial) + sweep on the
    oracle directly."""
    from oracle.oracle import Oracle

    srv, _, _ = _server(10 ** 9)
    reqs = _mix()
    res = srv.run(reqs)
    for rq in reqs:
        w = rq.spec
        o = Oracle(w.L, w.R, w.J, w.h, w.fields, w.temps, seed=w.seed, realization=w.realization,
                   R_cap=w.R_cap)
        a = w.adapt
        if a["trials"]:
            o.adapt_temps(a["trials"], a["sweeps_per_trial"], a["every"], a["rate_threshold"],
                          a["max_insert_per_trial"], a["R_cap"])
        o.sweep(w.sweeps, w.every)
        got = res["outcomes"][rq.rid]
        assert np.array_equal(got.energies, o.energies())
        assert np.array_equal(got.perm, o.perm())


def test_admission_waits_for_budget_and_never_exceeds_it():
    reqs = [_req(q, 1e-7 * q, L=4, R=4) for q in range(6)]
    per = OracleEngine(0).bytes_needed(reqs[0].spec)
    srv, eng, _ = _server(2 * per + 1)
    seen = []
    orig_step = eng.step

    def step(quantum, every):
        seen.append(eng.reserved)
        orig_step(quantum, every)

    eng.step = step
    res = srv.run(reqs)
    assert res["stats"]["completed"] == 6
    assert max(seen) <= 2 * per + 1
    assert res["stats"]["max_active"] == 2


def test_requests_join_while_others_run():
    # a long request first, short ones arriving during its run
    reqs = [_req(0, 0.0, L=6, R=4, prod=200)] + [_req(q, 2e-5 * q, L=4, R=3, prod=20) for q in range(1, 4)]
    srv, eng, _ = _server(10 ** 9, ns_per_attempt=5.0)
    res = srv.run(reqs)
    admits = [i for i, e in enumerate(eng.log) if e[0] == "admit"]
    steps = [i for i, e in enumerate(eng.log) if e[0] == "step"]
    assert admits[1] > steps[0]            # admitted after the first request started
    out = res["outcomes"]
    assert all(out[q].finished < out[0].finished for q in (1, 2, 3))


def test_bad_requests_fail_alone():
    reqs = _mix()
    bad = _req(9, 0.0, L=4, R=4)
    bad.spec = bad.spec.__class__(**{**bad.spec.__dict__, "temps": np.array([3.0, 2.0, 1.0, 0.5])})
    odd = _req(10, 0.0, L=4, R=4, prod=33)            # not a multiple of the quantum
    srv, _, _ = _server(10 ** 9)
    res = srv.run(reqs + [bad, odd])
    out = res["outcomes"]
    assert out[9].error and out[10].error
    assert res["stats"]["completed"] == len(reqs)


def test_request_larger_than_budget_fails_and_alloc_failure_is_isolated():
    reqs = [_req(0, 0.0, L=6, R=4)]
    srv, _, _ = _server(100)
    res = srv.run(reqs)
    assert "budget" in res["outcomes"][0].error
    srv, _, _ = _server(10 ** 9, fail_alloc=True)
    res = srv.run(_mix())
    assert res["stats"]["failed"] == 5 and res["stats"]["completed"] == 0


def test_empty_schedules_are_rejected():
    """A request whose schedule can never finish (an empty trial run, no
    production sweeps) fails at admission instead of running forever."""
    no_trial = _req(20, 0.0, L=4, R=4, trial=0)
    no_trial.spec.adapt["trials"] = 1            # one trial run of 0 sweeps
    no_prod = _req(21, 0.0, L=4, R=4, prod=0)
    srv, eng, _ = _server(10 ** 9)
    res = srv.run([no_trial, no_prod] + _mix())
    out = res["outcomes"]
    assert out[20].error and out[21].error
    assert res["stats"]["completed"] == len(_mix())


def test_latency_statistics():
    srv, _, _ = _server(10 ** 9)
    st = srv.run(_mix())["stats"]
    assert st["latency_p50_s"] <= st["latency_p99_s"]
    assert st["realizations_per_s"] > 0
