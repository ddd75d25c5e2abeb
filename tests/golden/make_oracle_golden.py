"""Writes oracle_chain_digest.json beside this file: the oracle's final state
after a few fixed short runs (both field kinds, an adaptive trial, exchange
steps and a ragged interval).  It calls only the oracle and the seeded input
generators, so the digest guards the oracle against unintended change; it
is not a pin against the paper (the pins are the tests named
test_oracle_*).  A change to the digest must come with the reason the
oracle's chain changed.

    python tests/golden/make_oracle_golden.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DIGEST = os.path.join(HERE, "oracle_chain_digest.json")

CASES = [
    dict(name="bimodal_l4_ragged", L=4, R=6, J=1.0, h=1.0, kind="b", fkey=[60, 4], temps=("linear", 3.5, 4.5),
         seed=12345, realization=7, adapt=None, calls=[(13, 5), (24, 5)]),
    dict(name="bimodal_l8_adaptive", L=8, R=4, J=1.0, h=2.0, kind="b", fkey=[61, 8], temps=("linear", 3.0, 6.0),
         seed=777, realization=3, adapt=(2, 40, 5, 0.9, 2, 8), calls=[(40, 5)]),
    dict(name="gaussian_l6", L=6, R=4, J=1.0, h=2.0, kind="g", fkey=[62, 6], temps=("geometric", 2.5, 6.0),
         seed=99, realization=0, adapt=None, calls=[(23, 4)]),
]


def run_case(oracle_mod, case):
    from paper_1508_06268_amd import workloads as W

    L, R = case["L"], case["R"]
    f = W.bimodal_fields(L, case["fkey"]) if case["kind"] == "b" else W.gaussian_fields(L, case["fkey"])
    kind, lo, hi = case["temps"]
    T = W.linear_temps(R, lo, hi) if kind == "linear" else W.geometric_temps(R, lo, hi)
    R_cap = case["adapt"][5] if case["adapt"] else 0
    o = oracle_mod.Oracle(L, R, case["J"], case["h"], f, T, seed=case["seed"], realization=case["realization"],
                          R_cap=R_cap)
    if case["adapt"]:
        o.adapt_temps(*case["adapt"])
    for n, every in case["calls"]:
        o.sweep(n, every)
    att, acc = o.exchange_stats()
    out = {
        "R": int(o.R),
        "spins_sha256": hashlib.sha256(o.spins().tobytes()).hexdigest(),
        "perm": [int(x) for x in o.perm()],
        "counters": [int(x) for x in o.counters()],
        "att": [int(x) for x in att],
        "acc": [int(x) for x in acc],
        "temps": [float(x).hex() for x in o.temps()],
        "energies": [float(x).hex() for x in o.energies()],
        "magnetizations": [int(x) for x in o.magnetizations()],
    }
    o.close()
    return out


def main():
    from oracle import oracle

    oracle.build()
    digest = {c["name"]: run_case(oracle, c) for c in CASES}
    with open(DIGEST, "w") as fh:
        json.dump(digest, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print("wrote", DIGEST)


if __name__ == "__main__":
    main()
