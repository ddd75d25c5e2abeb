"""Physical observables from the per-slot sums the exchange kernel keeps
(one sample per exchange step, Sec. 7): thermal averages per realization and
the disorder averages [.] of Eq. 11-13.

Per slot the device holds [count, sum E, sum E^2, sum |M|, sum M^2, sum M^4]
(see rfim_observables).  With N = L^3 sites and e = E/N:
  <|m|> = <|M|>/N                                  (Eq. 11, inside [.])
  C     = N/T^2 (<e^2> - <e>^2) = (<E^2> - <E>^2)/(N T^2)   (Eq. 12)
  g     = (3 - [<M^4>]/[<M^2>]^2)/2                (Eq. 13, disorder averages)
With the optional Fourier measurement (rfim_set_measure) the device also
holds [count, sum F] per slot, F = (1/(3N)) sum over the axes of
|sum_i s_i e^{i K x_mu,i}|^2 at K = 2 pi / L (Eq. 15-17 read with s_i), and
  xi_paper = sqrt((<M^2>/N) / <F> - 1)             (Eq. 14, inside [.])
  xi       = xi_paper / (2 sin(K/2))                (the usual second-moment
             correlation length; the printed Eq. 14 omits this factor).
"""
from __future__ import annotations

from typing import Dict, Iterable

import numpy as np


def thermal(obs: np.ndarray, temps: np.ndarray, N: int, fourier=None) -> Dict[str, np.ndarray]:
    """Per-slot thermal averages of one realization from its [R][6] sums
    (and, if given, the [R][2] Fourier sums: adds xi and xi_paper)."""
    obs = np.asarray(obs, dtype=np.float64)
    n = obs[:, 0]
    if np.any(n <= 0):
        raise ValueError("a slot has no samples")
    E, E2, aM, M2, M4 = (obs[:, q] / n for q in range(1, 6))
    T = np.asarray(temps, dtype=np.float64)
    out = {"T": T, "E": E / N, "C": (E2 - E * E) / (N * T * T), "absm": aM / N,
           "M2": M2, "M4": M4, "samples": n}
    if fourier is not None:
        fo = np.asarray(fourier, dtype=np.float64)
        if np.any(fo[:, 0] <= 0):
            raise ValueError("a slot has no Fourier samples")
        F = fo[:, 1] / fo[:, 0]
        L = round(N ** (1.0 / 3.0))
        with np.errstate(invalid="ignore", divide="ignore"):
            xi_p = np.sqrt(np.maximum((M2 / N) / F - 1.0, 0.0))
        out.update({"F": F, "xi_paper": xi_p, "xi": xi_p / (2.0 * np.sin(np.pi / L))})
    return out


def disorder_average(per_realization: Iterable[Dict[str, np.ndarray]]) -> Dict[str, np.ndarray]:
    """[.] over realizations that share one temperature set."""
    rs = list(per_realization)
    if not rs:
        raise ValueError("no realizations")
    T = rs[0]["T"]
    for r in rs[1:]:
        if r["T"].shape != T.shape or not np.allclose(r["T"], T):
            raise ValueError("realizations must share the temperature set")
    mean = lambda key: np.mean([r[key] for r in rs], axis=0)
    M2, M4 = mean("M2"), mean("M4")
    out = {"T": T, "E": mean("E"), "C": mean("C"), "absm": mean("absm"),
           "g": 0.5 * (3.0 - M4 / (M2 * M2)), "realizations": len(rs)}
    if all("xi" in r for r in rs):
        out["xi"] = mean("xi")
        out["xi_paper"] = mean("xi_paper")
    return out


def crossing(T: np.ndarray, a: np.ndarray, b: np.ndarray):
    """First temperature where a - b changes sign, by linear interpolation."""
    d = np.asarray(a) - np.asarray(b)
    for q in range(len(d) - 1):
        if d[q] == 0.0:
            return float(T[q])
        if d[q] * d[q + 1] < 0:
            return float(T[q] + (T[q + 1] - T[q]) * d[q] / (d[q] - d[q + 1]))
    return None
