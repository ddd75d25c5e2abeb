"""Writes gaussian_two_sample.json beside this file: the oracle's per-slot
statistics of time-averaged energy and |M| over independent seeds, for the
continuous-field (Gaussian) two-sample parity test.  It calls only the
oracle and the seeded input generators.

Each run: the fixed disorder realization and ladder of its case, `burn`
sweeps with an exchange every 10, then `meas` sweeps in intervals of 10;
after every exchange step of the window the energy and |M| of the replica at
each temperature slot are sampled, and their time averages over the window
are the run's values.  Sets:
  l32_null   L=32, R=64 (the paper-scale shape), seeds 2000..2031
  l32_null2  same, seeds 4000..4031 (a second null sample: the test must
             not reject it against l32_null)
  l32_beta   same, seeds 3000..3031, every temperature divided by 1.01
             (beta scaled by 1.01: the test must reject it)
  l64_null   L=64, R=8 (the streaming shape), seeds 2000..2031

    python tests/golden/make_gaussian_stats.py [--procs 8]
"""
import argparse
import json
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.dirname(HERE)):
    if p not in sys.path:
        sys.path.insert(0, p)

OUT = os.path.join(HERE, "gaussian_two_sample.json")
NSEEDS = 32
CASES = {
    "l32": dict(L=32, R=64, J=1.0, h=2.0, fkey=[24, 32], lo=1.0, hi=6.0, burn=200, meas=200, every=10),
    "l64": dict(L=64, R=8, J=1.0, h=2.0, fkey=[24, 64], lo=1.0, hi=6.0, burn=200, meas=200, every=10),
}
SETS = {
    "l32_null": ("l32", 2000, 1.0),
    "l32_null2": ("l32", 4000, 1.0),
    "l32_beta": ("l32", 3000, 1.01),
    "l64_null": ("l64", 2000, 1.0),
}


def case_inputs(name):
    from paper_1508_06268_amd import workloads as W

    c = CASES[name]
    return W.gaussian_fields(c["L"], c["fkey"]), W.geometric_temps(c["R"], c["lo"], c["hi"])


def oracle_run(args):
    """Time averages (E by slot, |M| by slot) of one oracle run."""
    import numpy as np

    from oracle.oracle import Oracle

    case, seed, beta_scale = args
    c = CASES[case]
    f, T = case_inputs(case)
    o = Oracle(c["L"], c["R"], c["J"], c["h"], f, T / beta_scale, seed=seed)
    o.sweep(c["burn"], c["every"])
    n = c["meas"] // c["every"]
    E = np.zeros(c["R"])
    M = np.zeros(c["R"])
    for _ in range(n):
        o.sweep(c["every"], c["every"])
        E += o.energies()
        M += np.abs(o.magnetizations())
    o.close()
    return (E / n).tolist(), (M / n).tolist()


def main():
    import numpy as np

    from two_sample import summary, to_json

    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    args = ap.parse_args()
    jobs = [(name, SETS[name][0], SETS[name][1] + i, SETS[name][2]) for name in SETS for i in range(NSEEDS)]
    with Pool(args.procs) as pool:
        res = pool.map(oracle_run, [j[1:] for j in jobs])
    out = {"cases": CASES, "nseeds": NSEEDS, "sets": {}}
    for name in SETS:
        rows = [r for j, r in zip(jobs, res) if j[0] == name]
        E = np.array([r[0] for r in rows])
        M = np.array([r[1] for r in rows])
        case, seed0, scale = SETS[name]
        out["sets"][name] = {"case": case, "seed0": seed0, "beta_scale": scale,
                             "E": to_json(summary(E)), "absM": to_json(summary(M)),
                             "first_seed": {"E": rows[0][0], "absM": rows[0][1]}}
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=0)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
