"""The two-sample statistic for the continuous-field (Gaussian) parity check.

With continuous fields the device evaluates the Metropolis bound in FP32 and
the oracle in FP64, so a rare decision differs and the two chains of one
seed part ways; only their statistics must agree.  Each side runs its own
set of independent seeds on the same disorder realization and temperature
ladder, and records, per temperature slot, the time average of the energy
and of |M| over the exchange steps of a fixed window (one sample after every
exchange step).  Per slot and observable, Welch's t compares the two sample
means; the family of 2R comparisons is read at three sigma as a whole: it
rejects when any comparison's two-sided p-value is below 0.0027 / (2R)
(Bonferroni), so that the chance of a false rejection of the whole family
is at most that of one three-sigma comparison."""
import numpy as np
from scipy import stats

FAMILY_ALPHA = 0.0027          # two-sided three sigma


def summary(x):
    """Per-column mean, sample variance (ddof 1) and count of an n x m array."""
    x = np.asarray(x, dtype=np.float64)
    return {"mean": x.mean(axis=0), "var": x.var(axis=0, ddof=1), "n": x.shape[0]}


def welch(a, b):
    """Welch's t and its Welch-Satterthwaite degrees of freedom, per column,
    from two summaries."""
    va, vb = a["var"] / a["n"], b["var"] / b["n"]
    se = np.sqrt(va + vb)
    t = (a["mean"] - b["mean"]) / np.where(se > 0, se, np.inf)
    df = (va + vb) ** 2 / np.where(va + vb > 0, va ** 2 / (a["n"] - 1) + vb ** 2 / (b["n"] - 1), 1.0)
    return t, df


def compare(a_E, a_M, b_E, b_M):
    """Family test over the slots of both observables.  Returns (reject,
    smallest p-value, per-comparison threshold, largest |t|)."""
    ps, ts = [], []
    for a, b in ((a_E, b_E), (a_M, b_M)):
        t, df = welch(a, b)
        ps.append(2.0 * stats.t.sf(np.abs(t), df))
        ts.append(np.abs(t))
    p = np.concatenate(ps)
    thr = FAMILY_ALPHA / p.size
    return bool(p.min() < thr), float(p.min()), thr, float(np.concatenate(ts).max())


def from_json(d):
    return {"mean": np.asarray(d["mean"], dtype=np.float64), "var": np.asarray(d["var"], dtype=np.float64),
            "n": int(d["n"])}


def to_json(s):
    return {"mean": [float(v) for v in s["mean"]], "var": [float(v) for v in s["var"]], "n": int(s["n"])}
