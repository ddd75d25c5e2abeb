"""Disorder-averaged observables from batched realizations.

The paper's physics runs (Sec. 7) average thermal observables over many
disorder realizations at several lattice sizes and read the transition
temperature from where the Binder factors of different L cross.  This module
runs such a study through the batched path: every realization of every size
in one batch, one measurement per exchange step on the device, then the
estimators of `observables`.
"""
from __future__ import annotations

from typing import Dict, Sequence

import numpy as np

from . import observables as ob
from . import workloads as W
from .rfim import FIELDS_BIMODAL, MEASURE_FOURIER, Batch


def binder_study(Ls: Sequence[int], realizations, temps: np.ndarray, h: float = 1.0,
                 J: float = 1.0, equilibration: int = 2000, measure: int = 4000, every: int = 10,
                 seed: int = 0, stream=None, correlation: bool = False) -> Dict[int, Dict[str, np.ndarray]]:
    """[<|m|>], [C], [g] per size for +-1 fields of strength h (and [xi],
    [xi_paper] with `correlation`).  `realizations` is one count for every
    size or a dict size -> count."""
    counts = realizations if isinstance(realizations, dict) else {L: realizations for L in Ls}
    specs = []
    for L in Ls:
        for q in range(counts[L]):
            specs.append(W.Realization(L=L, R=len(temps), J=J, h=h, fields=W.bimodal_fields(L, [7, L, q]),
                                       temps=np.asarray(temps, dtype=np.float64), seed=seed,
                                       realization=(L << 16) | q, sweeps=equilibration + measure,
                                       every=every))
    b = Batch(specs, stream=stream)
    if correlation:
        # the Fourier measurement reads byte spins: classes that start in
        # bit storage (L = 64, 128, 256) take the streaming byte shape
        for L in Ls:
            if L in (64, 128, 256):
                b.set_shape(L, FIELDS_BIMODAL, 0, 4, 128)
    b.sweep(equilibration, every)
    b.synchronize()
    for q in range(len(specs)):
        b.item(q).reset_observables()
        if correlation:
            b.item(q).set_measure(MEASURE_FOURIER)
    b.sweep(measure, every)
    b.synchronize()
    out = {}
    q = 0
    for L in Ls:
        per = []
        for _ in range(counts[L]):
            it = b.item(q)
            per.append(ob.thermal(it.observables(), it.temps(), L ** 3,
                                  fourier=it.fourier() if correlation else None))
            q += 1
        out[L] = ob.disorder_average(per)
    b.close()
    return out
