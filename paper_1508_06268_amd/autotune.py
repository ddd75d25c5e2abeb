"""Launch-shape autotuner for batches.

Every launch shape gives bit-identical chains, so the tuner only measures
time.  For each class (L, field kind) of a batch it times a probe batch built
from the same realization specs (so the real chains are not advanced) over a
few exchange intervals per candidate shape, each class alone, then refines the
choice on the whole batch (the classes run concurrently, and a shape that is
fastest alone can lose beside the others).  Results are cached in a JSON file
keyed by (L, field kind, replicas of the class, members of the class).

The paper picks its block by minimising the halo surface of a w x x x y box
of fixed volume V (Sec. 3.2, Eq. 4-5): x = y = sqrt(V/w), giving
B_opt = (32, 4, 8) threads for V = 2 x 1024 spins and 32-wide warps.
`halo_optimal_block` restates that rule; it orders the candidates here (the
closest-to-optimal thread count first) but the measurement decides.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, List, Optional, Tuple

from .rfim import FIELDS_BIMODAL, FIELDS_CONTINUOUS, MODE_BITS, Batch

DEFAULT_CACHE = os.environ.get(
    "RFIM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "rfim_mi355x_tune.json"))


def halo_optimal_block(V: int, w: int) -> Tuple[int, int, int]:
    """Eq. 4-5: minimise S = 2(wy + xy + wx) at fixed V = wxy -> x = y =
    sqrt(V/w).  Returns the (w, y, x) box in spins; with two spins per
    thread (checkerboard) the thread block is (w, y/2, x)."""
    x = math.sqrt(V / w)
    return (w, int(round(x)), int(round(x)))


def halo_surface(w: int, x: float, y: float) -> float:
    return 2.0 * (w * y + x * y + w * x)


def candidate_shapes(L: int) -> List[Tuple[int, int, int]]:
    """Valid (mode, dwords per thread, threads per workgroup) for L; at
    L = 64, 128 and 256 also one bit per spin, (MODE_BITS, 0, 0), tried
    first."""
    out = []
    for nw in (1, 2, 4, 8):
        if 4 * nw > L // 2:
            continue
        chunks = L ** 3 // 8 // nw
        for wg in (64, 128, 256):
            if chunks % wg == 0 or chunks < wg:
                out.append((0, nw, wg))
        if L <= 32 and nw <= 4:
            for wg in (64, 128, 256, 512, 1024):
                out.append((1, nw, wg))
    # wave64 analogue of the paper's rule: a wave covers a 64-site row
    # segment, so order by distance of the thread count from the optimum box
    _, y, x = halo_optimal_block(2 * 1024, 64)
    opt = 64 * y * x // 2
    out.sort(key=lambda s: (abs(math.log2(s[2] * 4 * s[1]) - math.log2(max(opt, 1))), s))
    if L in (64, 128, 256):
        out.insert(0, (MODE_BITS, 0, 0))
    return out


def _kind_of(w) -> int:
    import numpy as np

    fk = getattr(w, "field_kind", -1)
    if fk in (FIELDS_BIMODAL, FIELDS_CONTINUOUS):
        return fk
    f = np.asarray(w.fields)
    return FIELDS_BIMODAL if np.all((f == 1.0) | (f == -1.0)) else FIELDS_CONTINUOUS


# Bumped whenever the kernels or the timing method change, so that shapes
# cached by an older build are measured again.
CACHE_VERSION = 4


def class_key(L: int, kind: int, items) -> str:
    return "v%d_L%d_k%d_R%d_n%d" % (CACHE_VERSION, L, kind, sum(int(w.R) for w in items), len(items))


def load_cache(path: str = DEFAULT_CACHE) -> Dict[str, list]:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def save_cache(cache: Dict[str, list], path: str = DEFAULT_CACHE) -> None:
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _time_batch(torch, batch, stream, every: int, intervals: int) -> float:
    batch.sweep(every, every)          # warm the shape (and capture its graph)
    batch.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    batch.sweep(every * intervals, every)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1)


def tune(specs, every: int = 10, intervals: int = 3, cache_path: Optional[str] = DEFAULT_CACHE,
         log=None, refine_top: int = 3, whole_intervals: int = 10) -> Dict[Tuple[int, int], Tuple[int, int, int]]:
    """Best shape per (L, field kind) class of the given realization specs.

    Two stages.  Each class alone: every candidate shape on a probe batch of
    that class's specs, best of two passes.  Then the whole batch, because
    the classes of a batch run concurrently on their lanes and a shape that
    wins alone can lose beside the others (a streaming shape's many short
    launches against the other lanes' work): class by class, largest first,
    its `refine_top` fastest shapes alone are timed in the full batch with
    the other classes fixed (over `whole_intervals` exchange intervals,
    starting from the better of the batch's default shapes and the shapes
    fastest alone), and the fastest there is kept."""
    import torch

    classes: Dict[Tuple[int, int], list] = {}
    for w in specs:
        classes.setdefault((int(w.L), _kind_of(w)), []).append(w)
    cache = load_cache(cache_path) if cache_path else {}
    best: Dict[Tuple[int, int], Tuple[int, int, int]] = {}
    todo = []
    for key, items in classes.items():
        ck = class_key(key[0], key[1], items)
        if ck in cache:
            best[key] = tuple(cache[ck])
        else:
            todo.append(key)
    if todo:
        stream = torch.cuda.Stream()
        alone: Dict[Tuple[int, int], Dict[Tuple[int, int, int], float]] = {}
        for key in todo:
            L, kind = key
            probe = Batch(classes[key], stream=stream)
            timings = {}
            for _ in range(2):
                for shape in candidate_shapes(L):
                    probe.set_shape(L, kind, *shape)
                    ms = _time_batch(torch, probe, stream, every, intervals)
                    timings[shape] = min(ms, timings.get(shape, ms))
                    if log:
                        log("tune L=%d kind=%d shape %s: %.3f ms" % (L, kind, shape, ms))
            probe.close()
            alone[key] = timings
            best[key] = min(timings, key=lambda sh: (timings[sh], sh))
        if refine_top > 1 and len(classes) > 1:
            full = Batch(specs, stream=stream)
            first = {}
            for q, w in enumerate(specs):
                first.setdefault((int(w.L), _kind_of(w)), tuple(full.item(q).launch_shape()))

            def whole():
                return min(_time_batch(torch, full, stream, every, whole_intervals) for _ in range(2))

            # start from the better of the batch's default shapes and the
            # shapes that won alone (a class-by-class search from the latter
            # can miss a combination the defaults already hold)
            t_default = whole()
            apply(full, best)
            base = whole()
            if log:
                log("tune whole batch: default shapes %.3f ms, shapes fastest alone %.3f ms" % (t_default, base))
            if t_default < base:
                for key in todo:
                    best[key] = first[key]
                apply(full, best)
                base = t_default
            work = {k: sum(int(w.R) * int(w.L) ** 3 for w in classes[k]) for k in todo}
            for key in sorted(todo, key=lambda k: -work[k]):
                L, kind = key
                cands = sorted(alone[key], key=lambda sh: (alone[key][sh], sh))[:refine_top]
                for shape in cands:
                    if shape == best[key]:
                        continue
                    full.set_shape(L, kind, *shape)
                    ms = whole()
                    if log:
                        log("tune whole batch, L=%d kind=%d shape %s: %.3f ms (best %.3f)" % (L, kind, shape, ms,
                                                                                           base))
                    if ms < base:
                        base = ms
                        best[key] = shape
                    else:
                        full.set_shape(L, kind, *best[key])
            full.close()
        for key in todo:
            cache[class_key(key[0], key[1], classes[key])] = list(best[key])
        if cache_path:
            save_cache(cache, cache_path)
    return best


def apply(batch: Batch, shapes: Dict[Tuple[int, int], Tuple[int, int, int]]) -> None:
    for (L, kind), shape in shapes.items():
        batch.set_shape(L, kind, *shape)
