"""Benchmark: Exchange Monte Carlo for the 3D RFIM on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload adaptive_l64]

One step is one whole disorder realization of the named workload run through
the hot path: checkerboard Metropolis sweeps over all replicas, the
per-replica energy reduction and the replica exchange every 10 sweeps, with
the adaptive temperature trials in front (Sec. 3.1, 3.3, 4).  The default
workload is L=64 with bimodal fields h=2.25, 128 replicas linear in T [1, 6],
4 trial runs of 2000 sweeps inserting temperatures where the adjacent rate
is below 0.2 (cap 192, at most 16 per trial), then 2x10^4 sweeps.

Inputs (fields, temperatures, the realization's handle) are resident on
the GPU before the timed region.  Prints one JSON line on stdout; progress
goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "spin-flip attempts/ns & % HBM roofline at L=64; realizations/s + p99 latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_1508_06268_amd", "csrc", "rfim_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_pow2_l64_r192_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "sweep_pow2_l64_r192_valu.txt")
# Algorithmic HBM bytes per spin-flip attempt of one half-sweep with one-byte
# spins: read the site (1), read the other colour once (1), read the field
# (1 for +-1 fields, 4 for FP32 fields), write the site (1).  The field is
# shared by every replica of a realization, so a launch over R replicas
# needs it once: 3 + f/R bytes per attempt is the floor with perfect reuse.
BYTES_PER_ATTEMPT = {0: 4.0, 1: 7.0}
# One bit per spin: the site, the other colour and the +-1 field are 1/8
# byte each, and the site is written: 0.5 B per attempt.
BITS_BYTES_PER_ATTEMPT = 0.5
TRAFFIC_BITS_FILE = os.path.join(ROOT, "profiles", "sweep_bits_l64_r192_traffic.txt")
VALU_BITS_FILE = os.path.join(ROOT, "profiles", "sweep_bits_l64_r192_valu.txt")
FIELD_BYTES = {0: 1.0, 1: 4.0}
# Vector ALU issue: 256 CUs x 4 SIMDs at 2.4 GHz.  The published fp32 vector
# peak, 157.3 TFLOP/s = 256 x 4 x 2.4e9 x 64 FLOP per cycle, is 32 fused
# multiply-adds per SIMD and cycle: one wave64 32-bit instruction every two
# cycles, 1.229e12 wave-instruction slots per second.  The fp64 peak (78.6)
# is half that: an instruction with a 64-bit result (the Philox product,
# v_mad_u64_u32) takes two slots; a transcendental (v_exp_f32) four.  A
# kernel's slots per attempt: its VALU instructions from the committed
# counters, plus one more per 64-bit product and three more per exponential
# (both counted in the kernel's instruction stream, stated in the same
# summary).
CUS, SIMDS, CLOCK_HZ = 256, 4, 2.4e9
WAVE_SLOTS_PER_S = CUS * SIMDS * CLOCK_HZ / 2.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def _profile_value(path, pattern):
    """A figure from a committed rocprofv3 summary, if it was taken on the
    current kernel source (same hash), else None."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    m_val = re.search(pattern, text)
    if not m_hash or not m_val or m_hash.group(1) != kernel_hash():
        return None
    return float(m_val.group(1))


def measured_traffic(path):
    """HBM bytes per launch of a sweep kernel (FETCH_SIZE + WRITE_SIZE)."""
    return _profile_value(path, r"hbm_bytes_per_launch:\s*([0-9.eE+]+)")


def measured_valu_per_1024(path):
    """VALU issue slots per 1024 attempts of a sweep kernel (see
    WAVE_SLOTS_PER_S): its VALU wave-instructions, one more slot per 64-bit
    product and three more per exponential."""
    ins = _profile_value(path, r"VALU instructions per 1024 attempts:\s*([0-9.]+)")
    mad = _profile_value(path, r"64-bit products \(v_mad_u64_u32\) per 1024 attempts:\s*([0-9.]+)")
    exp = _profile_value(path, r"exponentials \(v_exp_f32\) per 1024 attempts:\s*([0-9.]+)")
    if ins is None or mad is None or exp is None:
        return None
    return ins + mad + 3.0 * exp


def run_realization(h, w, stream, torch):
    """One realization: adaptive trials then the production sweeps.
    Returns the number of spin-flip attempts issued."""
    N = w.L ** 3
    attempts = 0
    a = w.adapt
    for _ in range(a["trials"]):
        attempts += h.R * N * a["sweeps_per_trial"]
        h.adapt_temps(1, a["sweeps_per_trial"], a["every"], a["rate_threshold"],
                      a["max_insert_per_trial"], a["R_cap"])
    attempts += h.R * N * w.sweeps
    h.sweep(w.sweeps, w.every)
    return attempts


def host_info():
    """What the CPU baseline ran on: model name, nproc and the CPUs this
    process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_allowed": allowed}


def oracle_timed_build():
    """The oracle built for timing on this host (-O3 -march=native
    -ffp-contract=off) in a private directory."""
    import tempfile

    from oracle import oracle as O

    return O.timed_build(tempfile.mkdtemp(prefix="rfim_oracle_"))


def cpu_baseline(w, lib_path, sweeps=20):
    """The CPU oracle on a bounded sample of the same workload: the initial
    replica set for `sweeps` sweeps with exchange every 10, one thread."""
    from oracle import oracle as O

    O.use_library(lib_path)
    o = O.Oracle(w.L, w.R, w.J, w.h, w.fields, w.temps, seed=w.seed)
    t0 = time.perf_counter()
    o.sweep(sweeps, w.every)
    dt = time.perf_counter() - t0
    att = w.R * w.L ** 3 * sweeps
    return {"value": att / (dt * 1e9), "unit": "spin-flip attempts/ns", "cores": 1, "kind": "oracle",
            "sample": "L=%d, R=%d, %d sweeps with exchange every %d (%.2e attempts, %.1f s, 1 thread; "
                      "gcc -O3 -march=native -ffp-contract=off)" % (w.L, w.R, sweeps, w.every, att, dt)}


def kernel_only(torch, P, W, sweeps, storage):
    """Only a sweep kernel at the production shape (L=64, R=192, +-1
    fields; byte or bit storage): `sweeps` sweeps without exchange on one
    stream, for counter collection."""
    w = W.adaptive_l64()
    stream = torch.cuda.Stream()
    h = P.Rfim(w.L, w.R_cap, w.J, w.h, w.fields, W.linear_temps(w.R_cap, 1.0, 6.0), seed=w.seed,
               stream=stream)
    h.set_spin_storage(storage)
    h.set_concurrency(1)
    h.sweep(sweeps, 0)
    h.synchronize()
    log("kernel mode: %d half-sweep launches at L=%d R=%d, %s" % (2 * sweeps, w.L, w.R_cap,
                                                                 "bits" if storage else "bytes"))


def gauss_kernel_only(torch, P, W, which, sweeps=20):
    """Only a continuous-field sweep, for counters: `streaming` is L=64,
    R=128 (Gaussian fields, h=2) in byte storage on one stream, `bits` the
    same in bit storage (its default), `paper_scale` the L=32, R=64 shape on
    its default slab launch, `resident` the same on the LDS-resident launch
    (1, 4, 1024); `sweeps` sweeps with an exchange every 10."""
    if which in ("streaming", "bits"):
        L, R = 64, 128
    else:
        L, R = 32, 64
    stream = torch.cuda.Stream()
    h = P.Rfim(L, R, 1.0, 2.0, W.gaussian_fields(L, [5, L]), W.geometric_temps(R, 1.0, 6.0), seed=5,
               stream=stream)
    if which == "resident":
        h.set_launch_shape(1, 4, 1024)
    h.set_spin_storage(P.rfim.SPINS_BITS if which == "bits" else P.rfim.SPINS_BYTES)
    h.set_concurrency(1)
    h.sweep(sweeps, 10)
    h.synchronize()
    log("gauss %s mode: L=%d R=%d shape %s, storage %d, %d sweeps" % (which, L, R, h.launch_shape(),
                                                                       h.spin_storage(), sweeps))


def hbm_bits_leg(torch, P, W, n=128, R=128, sweeps=100, every=10):
    """One bit per spin on data of the HBM-streaming leg's byte size: n
    realizations x R=128 at L=64 (512 MiB of spin bits at n = 128), each a
    handle in bit storage, swept one after another on one stream."""
    stream = torch.cuda.Stream()
    hs = []
    for q in range(n):
        g = P.Rfim(64, R, 1.0, 2.25, W.bimodal_fields(64, [9, q]), W.linear_temps(R, 1.0, 6.0), seed=0,
                   realization=q, stream=stream)
        assert g.spin_storage() == P.rfim.SPINS_BITS
        g.sweep(every, every)
        hs.append(g)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for g in hs:
        g.sweep(sweeps, every)
    e1.record(stream)
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) / 1e3
    for g in hs:
        g.close()
    attempts = n * R * 64 ** 3 * sweeps
    rate = attempts / dt / 1e9
    mib = n * R * 64 ** 3 / 8 / 2 ** 20
    log("hbm-size bits: %d x L=64 R=%d (%.0f MiB of spin bits), %d sweeps each: %.1f attempts/ns"
        % (n, R, mib, sweeps, rate))
    return {"workload": "hbm_size_bits_l64", "realizations": n, "L": 64, "R": R, "spin_bits_mib": round(mib, 1),
            "sweeps": sweeps, "exchange_every": every, "attempts_per_ns": round(rate, 1),
            "hbm_gbs_algorithmic": round(rate * BITS_BYTES_PER_ATTEMPT, 1)}


def tiles_only(torch, P, W, sweeps=2, hits=100, tiles=(32, 8, 8)):
    """Only the multi-hit tile kernel at the production shape (L=64, R=192,
    +-1 fields, 100 hits): `sweeps` sweeps without exchange, for counters."""
    w = W.adaptive_l64()
    stream = torch.cuda.Stream()
    h = P.Rfim(w.L, w.R_cap, w.J, w.h, w.fields, W.linear_temps(w.R_cap, 1.0, 6.0), seed=w.seed,
               stream=stream)
    h.set_update_order(P.rfim.ORDER_TILES, tiles, hits)
    h.sweep(sweeps, 0)
    h.synchronize()
    log("tiles mode: %d tile launches at L=%d R=%d, %d hits" % (2 * sweeps, w.L, w.R_cap, hits))


def copy_only(torch, nbytes, reps=5):
    """A plain device-to-device copy of known size (counter calibration)."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy mode: %d copies of %d bytes (read %d, write %d per copy)" % (reps, nbytes, nbytes, nbytes))


def cpu_worker(q, lib_path, sweeps=20):
    """Child process of the all-cores figure: the oracle on realization q of
    the L=64 workload (no GPU, no torch), one JSON line on stdout."""
    from paper_1508_06268_amd import workloads as W
    from oracle import oracle as O

    O.use_library(lib_path)
    w = W.adaptive_l64()
    o = O.Oracle(w.L, w.R, w.J, w.h, W.bimodal_fields(w.L, [9, q]), w.temps, seed=w.seed, realization=q)
    t0 = time.perf_counter()
    o.sweep(sweeps, w.every)
    dt = time.perf_counter() - t0
    print(json.dumps({"attempts": w.R * w.L ** 3 * sweeps, "seconds": dt}), flush=True)


def cpu_all_cores(procs, lib_path):
    """`procs` independent oracle processes on different realizations at
    once (child processes of a fresh interpreter that never touch the GPU);
    aggregate attempts over the wall time of the slowest."""
    import subprocess

    t0 = time.perf_counter()
    ps = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(q),
                            "--cpu-worker-lib", lib_path], stdout=subprocess.PIPE, cwd=ROOT)
          for q in range(procs)]
    outs = [json.loads(p.communicate()[0].decode().strip().splitlines()[-1]) for p in ps]
    wall = time.perf_counter() - t0
    if any(p.returncode != 0 for p in ps):
        raise RuntimeError("an oracle worker failed")
    att = sum(o["attempts"] for o in outs)
    return {"value": att / (wall * 1e9), "unit": "spin-flip attempts/ns", "cores": procs,
            "sample": "%d processes x (L=64, R=128, 20 sweeps, exchange every 10), %.1f s wall" % (procs, wall)}


def hbm_streaming_leg(torch, P, W, every=10, sweeps=200, reps=5, blocked=True):
    """The byte sweep on data that does not fit the on-package cache: 16
    realizations x R=128 at L=64 (512 MiB of spins) in one batch.  With the
    batch's temporal blocking off, each half-sweep launch covers 2048
    replicas and streams them through HBM (the HBM-roofline figure); with
    it on (the default of batches), groups of items run whole exchange
    intervals inside the on-package cache."""
    specs = W.hbm_streaming_l64(sweeps=sweeps)
    stream = torch.cuda.Stream()

    def run(group_bytes):
        b = P.Batch(specs, stream=stream)
        b.set_shape(64, P.FIELDS_BIMODAL, 0, 4, 128)     # byte spins (L=64 classes start in bits)
        if group_bytes is not None:
            b.set_group_bytes(group_bytes)
        # graph capture and the first pass over the 512 MiB outside the
        # timed region (a single warm-up interval left the first timed pass
        # ~13 % slow); median of `reps` timed passes
        b.sweep(5 * every, every)
        b.synchronize()
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            b.sweep(sweeps, every)
            e1.record(stream)
            b.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
        b.close()
        return float(np.median(times))

    dt = run(0)
    attempts = sum(w.R * w.L ** 3 for w in specs) * sweeps
    spins_bytes = sum(w.R * w.L ** 3 for w in specs)
    rate = attempts / dt / 1e9
    gbs = BYTES_PER_ATTEMPT[0] * attempts / dt / 1e9
    log("hbm streaming: %d x L=64 R=%d (%.0f MiB of spins), %d sweeps: %.1f attempts/ns, %.0f GB/s "
        "algorithmic (%.1f%% of HBM)" % (len(specs), specs[0].R, spins_bytes / 2 ** 20, sweeps, rate, gbs,
                                          100 * gbs / HBM_PEAK_GBS))
    out = {"workload": "hbm_streaming_l64", "realizations": len(specs), "L": 64, "R": specs[0].R,
           "spins_mib": round(spins_bytes / 2 ** 20, 1), "sweeps": sweeps, "exchange_every": every, "reps": reps,
           "attempts_per_ns": round(rate, 1), "hbm_gbs_algorithmic": round(gbs, 1),
           "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    if blocked:
        dtb = run(None)
        out["temporal_blocking"] = {"group_mib": 96, "attempts_per_ns": round(attempts / dtb / 1e9, 1)}
        log("hbm streaming with temporal blocking (groups of <= 96 MiB): %.1f attempts/ns" % (attempts / dtb / 1e9))
    return out


def batched_leg(torch, P, W, n=256, sweeps=5000, every=10):
    """Many realizations of uneven L and R in one batch (one launch per
    class and half-sweep or interval, graph-replayed intervals, autotuned
    shapes) against the same realizations run one at a time through
    rfim_create/rfim_sweep on the same GPU.  Handles and batch are created
    before the timed regions; each timed region ends when every result
    (energies by slot) is back on the host."""
    from paper_1508_06268_amd import autotune

    specs = W.batched_mix(n, sweeps)
    attempts = sum(w.R * w.L ** 3 for w in specs) * sweeps
    log("batched: %d realizations, %.2e attempts; tuning shapes" % (n, attempts))
    shapes = autotune.tune(specs, every=every, log=None)
    stream = torch.cuda.Stream()
    b = P.Batch(specs, stream=stream)
    autotune.apply(b, shapes)
    b.sweep(every, every)                  # graph capture outside the timed region
    b.synchronize()
    t0 = time.perf_counter()
    b.sweep(sweeps - every, every)
    b.synchronize()
    E = [b.item(q).energies() for q in range(n)]
    t_batch = time.perf_counter() - t0
    att_batch = sum(w.R * w.L ** 3 for w in specs) * (sweeps - every)
    b.close()
    log("batched: %.3f s -> %.1f realizations/s" % (t_batch, n / t_batch))
    singles = [P.Rfim(w.L, w.R, w.J, w.h, w.fields, w.temps, seed=w.seed, realization=w.realization,
                      stream=stream) for w in specs]
    for h in singles:
        h.sweep(every, every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for h in singles:
        h.sweep(sweeps - every, every)
        h.energies()
    t_single = time.perf_counter() - t0
    for h in singles:
        h.close()
    log("one at a time: %.3f s -> %.1f realizations/s" % (t_single, n / t_single))
    assert len(E) == n
    return {"workload": "batched_mix", "realizations": n, "sweeps": sweeps - every,
            "exchange_every": every, "L": [8, 16, 32], "R": [16, 32, 64],
            "batched_realizations_per_s": round(n / t_batch, 2),
            "batched_attempts_per_ns": round(att_batch / t_batch / 1e9, 1),
            "single_loop_realizations_per_s": round(n / t_single, 2),
            "speedup_vs_single_loop": round(t_single / t_batch, 2),
            "shapes": {"L%d_%s" % (L, "pm1" if k == 0 else "gauss"): list(s)
                       for (L, k), s in sorted(shapes.items())}}


def served_leg(torch, P, W, n=2000, rate=50.0, budget=200 << 30, quantum=50, single_sample=200):
    """The served workload: a Poisson stream of realization requests through
    the continuous-batching pool (admission against the device budget, one
    adaptive trial in place, then the production sweeps), paced by the
    arrival times; then the same requests all at once (capacity); then a
    sample of them one at a time through rfim_create/adapt/sweep."""
    from paper_1508_06268_amd.serve import PoolEngine, Request, Server

    stream = torch.cuda.Stream()
    reqs = [Request(q, t, w) for q, (t, w) in enumerate(W.served_stream(n, rate))]
    offered = sum(w.R * w.L ** 3 * (w.sweeps + w.adapt["sweeps_per_trial"]) for _, w in
                  [(r.arrival, r.spec) for r in reqs])
    log("served: %d requests at %.0f/s, offered >= %.2e attempts/s" % (n, rate, offered / reqs[-1].arrival))
    # launch shapes per (L, field kind) from the autotuner (cached)
    from paper_1508_06268_amd import autotune

    probe = []
    for L in (8, 16, 32, 64):
        probe += [r.spec for r in reqs if r.spec.L == L][:8]
    shapes = autotune.tune(probe, every=10)
    log("served: shapes %s" % {k: v for k, v in sorted(shapes.items())})
    # warm up the pool and its kernels on a few requests
    warm = Server(PoolEngine(budget, stream=stream, shapes=shapes), quantum=quantum, every=10)
    warm.run([Request(r.rid, 0.0, r.spec) for r in reqs[:8]])
    warm.engine.close()
    eng = PoolEngine(budget, stream=stream, shapes=shapes)
    res = Server(eng, quantum=quantum, every=10).run(reqs)
    eng.close()
    st = res["stats"]
    log("served (paced): %d done in %.2f s, p50 %.3f s, p99 %.3f s, max active %d"
        % (st["completed"], st["wall_s"], st["latency_p50_s"], st["latency_p99_s"], st["max_active"]))
    eng = PoolEngine(budget, stream=stream, shapes=shapes)
    cap = Server(eng, quantum=quantum, every=10).run([Request(r.rid, 0.0, r.spec) for r in reqs])["stats"]
    eng.close()
    log("served (all at once): %.1f realizations/s, %.1f attempts/ns" % (cap["realizations_per_s"],
                                                                         cap["attempts"] / cap["wall_s"] / 1e9))
    sample = reqs[:single_sample]
    t0 = time.perf_counter()
    for r in sample:
        w = r.spec
        a = w.adapt
        g = P.Rfim(w.L, w.R, w.J, w.h, w.fields, w.temps, seed=w.seed, realization=w.realization,
                   R_cap=w.R_cap, stream=stream)
        g.adapt_temps(a["trials"], a["sweeps_per_trial"], a["every"], a["rate_threshold"],
                      a["max_insert_per_trial"], a["R_cap"])
        g.sweep(w.sweeps, w.every)
        g.energies()
        g.close()
    t_single = time.perf_counter() - t0
    log("one at a time (first %d requests): %.2f s -> %.1f realizations/s"
        % (len(sample), t_single, len(sample) / t_single))
    capacity = cap["realizations_per_s"]
    return {"workload": "served_stream", "requests": n, "arrival_rate_per_s": rate,
            "budget_bytes": budget, "quantum_sweeps": quantum,
            "paced": {"realizations_per_s": round(st["realizations_per_s"], 2),
                      "latency_p50_s": round(st["latency_p50_s"], 4),
                      "latency_p99_s": round(st["latency_p99_s"], 4),
                      "latency_mean_s": round(st["latency_mean_s"], 4), "wall_s": round(st["wall_s"], 2),
                      "max_active": st["max_active"], "failed": st["failed"], "quanta": st["steps"],
                      "mean_quantum_ms": round(1e3 * st["wall_s"] / max(1, st["steps"]), 3)},
            "capacity_realizations_per_s": round(capacity, 2),
            "capacity_attempts_per_ns": round(cap["attempts"] / cap["wall_s"] / 1e9, 1),
            "utilization": round(rate / capacity, 3) if capacity else None,
            "single_loop_realizations_per_s": round(len(sample) / t_single, 2),
            "single_loop_sample": len(sample),
            "capacity_vs_single_loop": round(capacity * t_single / len(sample), 2),
            "shapes": {"L%d_%s" % (L, "pm1" if k == 0 else "gauss"): list(v) for (L, k), v in sorted(shapes.items())}}


def paper_scale_leg(torch, P, W, reps=3):
    """Plain method at paper scale: L=32, Gaussian FP32 fields h=2, R=64
    geometric in [1, 6], 10^4 sweeps with an exchange every 10, on the
    handle's default shape; median of `reps` whole runs, each timed with
    events on the handle's stream."""
    w = W.paper_scale_l32()
    stream = torch.cuda.Stream()
    times = []
    shape = None
    for _ in range(reps):
        h = P.Rfim(w.L, w.R, w.J, w.h, w.fields, w.temps, seed=w.seed, stream=stream)
        shape = h.launch_shape()
        h.sweep(10, 10)
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        h.sweep(w.sweeps, w.every)
        e1.record(stream)
        stream.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
        h.close()
    dt = float(np.median(times))
    attempts = w.R * w.L ** 3 * w.sweeps
    rate = attempts / dt / 1e9
    bpa = 3.0 + FIELD_BYTES[1] / w.R
    log("paper scale (L=32, R=64, Gaussian, 10^4 sweeps): %.1f ms -> %.1f attempts/ns" % (dt * 1e3, rate))
    return {"workload": "paper_scale_l32", "L": w.L, "R": w.R, "fields": "gaussian fp32", "h": w.h,
            "sweeps": w.sweeps, "exchange_every": w.every, "launch_shape": list(shape),
            "seconds": round(dt, 5), "attempts_per_ns": round(rate, 1),
            "hbm_gbs_at_7B": round(rate * 7.0, 1), "hbm_gbs_at_shared_field_bytes": round(rate * bpa, 1),
            "bytes_per_attempt_shared_field": round(bpa, 4)}


def multi_hit_leg(torch, P, W, hits=100, tiles=(32, 8, 8), sweeps=4, reps=5):
    """The double-checkerboard order with multi-hit updates (Sec. 3.2; the
    mh = 100 runs of Sec. 5.2) on the L=64 workload's realization at its
    production size (R=192, +-1 fields h=2.25): `hits` local sweeps per tile
    visit, tiles staged in LDS.  Median of `reps` event-timed runs of
    `sweeps` sweeps with an exchange every 2."""
    w = W.adaptive_l64()
    stream = torch.cuda.Stream()
    h = P.Rfim(w.L, w.R_cap, w.J, w.h, w.fields, W.linear_temps(w.R_cap, 1.0, 6.0), seed=w.seed, stream=stream)
    h.set_update_order(P.rfim.ORDER_TILES, tiles, hits)
    h.sweep(2, 2)
    h.synchronize()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        h.sweep(sweeps, 2)
        e1.record(stream)
        stream.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    h.close()
    dt = float(np.median(times))
    attempts = w.R_cap * w.L ** 3 * hits * sweeps
    rate = attempts / dt / 1e9
    log("multi-hit: L=64 R=%d tiles %s, %d hits: %.1f attempts/ns" % (w.R_cap, tiles, hits, rate))
    return {"workload": "multi_hit_l64", "L": w.L, "R": w.R_cap, "fields": "bimodal +-1", "h": w.h,
            "tiles": list(tiles), "hits": hits, "sweeps": sweeps, "exchange_every": 2, "reps": reps,
            "seconds": round(dt, 6), "attempts_per_ns": round(rate, 1)}


def trace_summary(path, top=40):
    """Per (kernel, grid, workgroup) launch statistics of a rocprofv3 kernel
    trace (csv output), longest total first: the same kernel at different
    grid sizes (e.g. the roofline leg's launches over all replicas and the
    production path's half-size launches) is listed separately."""
    import csv
    from collections import defaultdict

    def size(row, what):
        if what in row:
            return int(row[what])
        return int(row[what + "_X"]) * int(row[what + "_Y"]) * int(row[what + "_Z"])

    acc = defaultdict(list)
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            name = row["Kernel_Name"]
            key = (name[:90], size(row, "Grid_Size"), size(row, "Workgroup_Size"))
            acc[key].append(int(row["End_Timestamp"]) - int(row["Start_Timestamp"]))
    total = sum(sum(v) for v in acc.values())
    lines = ["%-90s %10s %6s %8s %12s %10s %10s %10s %7s" % ("kernel", "grid", "wg", "calls", "total ms",
                                                            "avg us", "min us", "max us", "%")]
    for key, v in sorted(acc.items(), key=lambda kv: -sum(kv[1]))[:top]:
        lines.append("%-90s %10d %6d %8d %12.1f %10.3f %10.3f %10.3f %7.2f" % (
            key[0], key[1], key[2], len(v), sum(v) / 1e6, np.mean(v) / 1e3, min(v) / 1e3, max(v) / 1e3,
            100.0 * sum(v) / total))
    return "\n".join(lines)


def counter_summary(kernel_csv, copy_csv, counter, kernel_match="sweep_pow2"):
    """Mean of `counter` (KiB per dispatch) over the dispatches of the
    kernel, and the factor that makes a plain device copy of 1 GiB read
    (FETCH_SIZE) or write (WRITE_SIZE) 1 GiB."""
    import csv

    k = [float(r["Counter_Value"]) for r in csv.DictReader(open(kernel_csv, newline=""))
         if kernel_match in r["Kernel_Name"]]
    c = [float(r["Counter_Value"]) for r in csv.DictReader(open(copy_csv, newline=""))
         if "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) > 1000]
    factor = (1 << 20) / float(np.mean(c))
    return {"counter": counter, "dispatches": len(k), "mean_kib": float(np.mean(k)), "min_kib": float(min(k)),
            "max_kib": float(max(k)), "copy_dispatches": len(c), "copy_mean_kib": float(np.mean(c)),
            "factor": factor, "bytes": float(np.mean(k)) * factor * 1024.0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="adaptive_l64", choices=["adaptive_l64", "served_stream"],
                    help="served_stream: only the continuous-batching serving run (its own JSON line)")
    ap.add_argument("--production-sweeps", type=int, default=20000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="bench", choices=["bench", "kernel", "kernel_bits", "kernel_gauss",
                                                     "bits_gauss", "paper_scale_gauss", "resident_gauss", "tiles",
                                                     "streaming", "copy"],
                    help="kernel / kernel_bits: only the byte / bit sweep kernel (for counters); kernel_gauss / "
                         "bits_gauss / paper_scale_gauss / resident_gauss: only the continuous-field streaming "
                         "sweep (L=64, R=128) in bytes / in bits / the L=32, R=64 sweep on its default slab "
                         "shape / on the LDS-resident shape; "
                         "tiles: only "
                         "the multi-hit "
                         "tile kernel (for counters); streaming: only the "
                         "HBM-streaming leg; copy: a plain copy of --copy-bytes (counter calibration)")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-realizations leg")
    ap.add_argument("--no-served", action="store_true", help="skip the served-stream leg")
    ap.add_argument("--trace-summary", default=None, metavar="KERNEL_TRACE_CSV",
                    help="print per (kernel, grid) statistics of a rocprofv3 kernel trace and exit")
    ap.add_argument("--kernel-match", default="sweep_pow2",
                    help="with --traffic-summary: the kernel name to match (sweep_pow2, sweep_bits)")
    ap.add_argument("--traffic-summary", nargs=4, default=None,
                    metavar=("FETCH_KERNEL_CSV", "FETCH_COPY_CSV", "WRITE_KERNEL_CSV", "WRITE_COPY_CSV"),
                    help="print the calibrated FETCH_SIZE + WRITE_SIZE bytes per sweep launch and exit")
    ap.add_argument("--cpu-worker", type=int, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-worker-lib", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker is not None:
        cpu_worker(args.cpu_worker, args.cpu_worker_lib)
        return
    if args.trace_summary:
        print(trace_summary(args.trace_summary))
        return
    if args.traffic_summary:
        fk, fc, wk, wc = args.traffic_summary
        a = counter_summary(fk, fc, "FETCH_SIZE", args.kernel_match)
        b = counter_summary(wk, wc, "WRITE_SIZE", args.kernel_match)
        for d in (a, b):
            print("%s: %d dispatches, mean %.1f KiB (min %.1f, max %.1f); copy calibration %.1f KiB per 1 GiB "
                  "-> factor %.4f -> %.4e bytes" % (d["counter"], d["dispatches"], d["mean_kib"], d["min_kib"],
                                                    d["max_kib"], d["copy_mean_kib"], d["factor"], d["bytes"]))
        print("hbm_bytes_per_launch: %.6e" % (a["bytes"] + b["bytes"]))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: a realization runs on a single MI355X and sharding "
              "across GPUs is not built; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1508_06268_amd as P
    from paper_1508_06268_amd import workloads as W

    torch.cuda.set_device(0)
    if args.mode in ("kernel", "kernel_bits"):
        kernel_only(torch, P, W, 20, P.rfim.SPINS_BITS if args.mode == "kernel_bits" else P.rfim.SPINS_BYTES)
        return
    if args.mode in ("kernel_gauss", "bits_gauss", "paper_scale_gauss", "resident_gauss"):
        gauss_kernel_only(torch, P, W, {"kernel_gauss": "streaming", "bits_gauss": "bits",
                                        "paper_scale_gauss": "paper_scale", "resident_gauss": "resident"}[args.mode])
        return
    if args.mode == "tiles":
        tiles_only(torch, P, W)
        return
    if args.mode == "copy":
        copy_only(torch, args.copy_bytes)
        return
    if args.mode == "streaming":
        hbm_streaming_leg(torch, P, W, sweeps=20, reps=1, blocked=False)
        return
    if args.workload == "served_stream":
        served = served_leg(torch, P, W)
        print(json.dumps({"metric": METRIC, "value": served["paced"]["realizations_per_s"],
                          "unit": "realizations/s", "n_gpus": 1, "higher_is_better": True,
                          "dtype": "u8", "data": "synthetic",
                          "config": {"workload": "served_stream"}, "served": served}), flush=True)
        return
    w = W.adaptive_l64(sweeps=args.production_sweeps)
    stream = torch.cuda.Stream()
    log("creating %d handles: L=%d R=%d R_cap=%d" % (args.warmup + args.steps, w.L, w.R, w.R_cap))
    handles = [P.Rfim(w.L, w.R, w.J, w.h, w.fields, w.temps, seed=w.seed, R_cap=w.R_cap, stream=stream)
               for _ in range(args.warmup + args.steps)]
    torch.cuda.synchronize()

    warm_ms = []
    for q in range(args.warmup):
        t0 = time.perf_counter()
        run_realization(handles[q], w, stream, torch)
        handles[q].synchronize()
        warm_ms.append((time.perf_counter() - t0) * 1e3)
        log("warmup %d: %.1f ms, R=%d" % (q, warm_ms[-1], handles[q].R))

    # Timed region: K whole realizations back to back on one stream; an
    # event after each one gives the per-step times without synchronizing.
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    attempts = 0
    step_R = []
    evs[0].record(stream)
    t0 = time.perf_counter()
    for q in range(args.steps):
        h = handles[args.warmup + q]
        attempts += run_realization(h, w, stream, torch)
        evs[q + 1].record(stream)
        step_R.append(h.R)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = evs[0].elapsed_time(evs[-1])
    step_ms = [evs[q].elapsed_time(evs[q + 1]) for q in range(args.steps)]
    elapsed_s = max(wall, gpu_ms / 1e3)
    value = attempts / (elapsed_s * 1e9)
    R_final = handles[-1].R
    log("timed: %d steps, %.2e attempts, %.3f s wall, %.3f s events -> %.1f attempts/ns"
        % (args.steps, attempts, wall, gpu_ms / 1e3, value))
    log("step ms: %s" % " ".join("%.1f" % t for t in step_ms))

    # Roofline legs, timed with events on the handle's stream: one launch
    # over every replica (one stream), median of 10 repetitions of 40
    # sweeps (80 launches); and the production path's two-stream half-sweep
    # in its steady state, median of 10 repetitions of 200 sweeps.  The
    # workload's handles keep one bit per spin (the default for +-1 fields
    # at L = 64), so its dominant kernel is the bit sweep; the byte sweep is
    # measured on the same handle beside it.
    h = handles[-1]
    reps = 10

    def half_sweep_us(streams, n_roof):
        h.set_concurrency(streams)
        h.sweep(10, 0)
        stream.synchronize()
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            h.sweep(n_roof, 0)
            e1.record(stream)
            stream.synchronize()
            times.append(e0.elapsed_time(e1) * 1e3 / (2 * n_roof))
        return float(np.median(times))

    kind = h.field_kind
    attempts_per_launch = R_final * w.L ** 3 // 2
    waves_per_launch = attempts_per_launch / 1024.0

    def alu_of(valu_per_1024, us):
        rate = valu_per_1024 * waves_per_launch / (us * 1e-6)
        return rate, rate / WAVE_SLOTS_PER_S

    storage = h.spin_storage()
    bits_legs = None
    if storage == P.rfim.SPINS_BITS:
        bits_us = half_sweep_us(1, 40)
        bits_split_us = half_sweep_us(2, 200)
        valu_bits = measured_valu_per_1024(VALU_BITS_FILE)
        b_bytes = BITS_BYTES_PER_ATTEMPT * attempts_per_launch
        b_gbs = b_bytes / (bits_us * 1e-6) / 1e9
        bits_legs = {"launch_us": bits_us, "split_us": bits_split_us, "valu": valu_bits, "bytes": b_bytes,
                     "gbs": b_gbs}
        log("bit sweep: %.2f us per half-sweep launch (%.1f attempts/ns); two streams: %.2f us"
            % (bits_us, attempts_per_launch / (bits_us * 1e3), bits_split_us))
    h.set_spin_storage(P.rfim.SPINS_BYTES)
    launch_us = half_sweep_us(1, 40)
    split_us = half_sweep_us(2, 200)
    h.set_concurrency(0)
    mode, nw, wg = h.launch_shape()
    bytes_per_launch = BYTES_PER_ATTEMPT[kind] * attempts_per_launch
    hbm_gbs = bytes_per_launch / (launch_us * 1e-6) / 1e9
    valu_bytes = measured_valu_per_1024(VALU_FILE)
    byte_kernel = {"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": round(hbm_gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(TRAFFIC_FILE),
                   "kernel": "sweep_pow2<bimodal, %d dwords x %d threads>, one launch over R=%d" % (nw, wg, R_final),
                   "launch_us": round(launch_us, 3), "attempts_per_launch": attempts_per_launch,
                   "bytes_per_attempt": BYTES_PER_ATTEMPT[kind], "bytes_per_launch": bytes_per_launch,
                   "attempts_per_ns_kernel": round(attempts_per_launch / (launch_us * 1e3), 1),
                   "valu_frac": round(alu_of(valu_bytes, launch_us)[1], 4) if valu_bytes else None,
                   "two_streams": {"half_sweep_us": round(split_us, 3),
                                   "attempts_per_ns": round(attempts_per_launch / (split_us * 1e3), 1),
                                   "hbm_frac": round(bytes_per_launch / (split_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}}
    log("byte sweep: %.2f us per half-sweep launch, %.0f GB/s algorithmic (%.1f%% of HBM); "
        "two streams: %.2f us per half-sweep" % (launch_us, hbm_gbs, 100 * hbm_gbs / HBM_PEAK_GBS, split_us))
    if bits_legs and bits_legs["valu"]:
        rate, frac = alu_of(bits_legs["valu"], bits_legs["launch_us"])
        roofline = {"bound": "alu", "achieved": round(rate / 1e12, 4), "peak": round(WAVE_SLOTS_PER_S / 1e12, 4),
                    "unit": "T wave64 VALU slots/s", "frac": round(frac, 4),
                    "traffic": measured_traffic(TRAFFIC_BITS_FILE),
                    "kernel": "sweep_bits<bimodal>, one launch over R=%d" % R_final,
                    "launch_us": round(bits_legs["launch_us"], 3), "attempts_per_launch": attempts_per_launch,
                    "valu_slots_per_1024_attempts": bits_legs["valu"],
                    "attempts_per_ns_kernel": round(attempts_per_launch / (bits_legs["launch_us"] * 1e3), 1),
                    "hbm": {"achieved": round(bits_legs["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(bits_legs["gbs"] / HBM_PEAK_GBS, 4),
                            "bytes_per_attempt": BITS_BYTES_PER_ATTEMPT, "bytes_per_launch": bits_legs["bytes"]},
                    "two_streams": {"half_sweep_us": round(bits_legs["split_us"], 3),
                                    "attempts_per_ns": round(attempts_per_launch / (bits_legs["split_us"] * 1e3), 1),
                                    "alu_frac": round(alu_of(bits_legs["valu"], bits_legs["split_us"])[1], 4)},
                    "byte_kernel": byte_kernel}
        log("VALU of the bit sweep: %.1f%% of the issue peak (one launch), %.1f%% (two streams)"
            % (100 * frac, 100 * roofline["two_streams"]["alu_frac"]))
    else:
        roofline = dict(byte_kernel)
        if bits_legs:
            roofline["bit_kernel"] = {"launch_us": round(bits_legs["launch_us"], 3),
                                      "two_streams_half_sweep_us": round(bits_legs["split_us"], 3),
                                      "hbm_gbs_algorithmic": round(bits_legs["gbs"], 1)}

    for hh in handles:
        hh.close()
    # the realization-level legs first: a batch's concurrent lanes and a
    # pool's ran slower in a process that had already run the HBM-size legs
    # (the hardware queues its streams land on follow from how many streams
    # the process made before)
    batched = None if args.no_batched else batched_leg(torch, P, W)
    served = None if args.no_served else served_leg(torch, P, W)
    streaming = hbm_streaming_leg(torch, P, W)
    roofline["hbm_streaming"] = streaming
    roofline["hbm_size_bits"] = hbm_bits_leg(torch, P, W)
    paper_scale = paper_scale_leg(torch, P, W)
    # last of the GPU legs: its sustained VALU load can lower the clock for
    # what follows
    multi_hit = multi_hit_leg(torch, P, W)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: building the oracle for this host")
        lib_path = oracle_timed_build()
        log("cpu baseline: oracle on a bounded sample")
        cpu = cpu_baseline(w, lib_path)
        info = host_info()
        # the GPU's host share is 16 cores: one process per core of it
        procs = max(1, min(16, info["cpus_allowed"]))
        log("cpu baseline: %d oracle processes at once" % procs)
        cpu["all_cores"] = cpu_all_cores(procs, lib_path)
        cpu["host"] = info

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "spin-flip attempts/ns", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elapsed_s * 1e3 / args.steps, 3),
        "step_ms": [round(t, 2) for t in step_ms], "step_R": step_R,
        "warmup_ms": [round(t, 2) for t in warm_ms],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "adaptive_l64", "L": w.L, "R0": w.R, "R_final": R_final,
                   "fields": "bimodal +-1", "spin_storage": "bits", "J": w.J, "h": w.h, "T": [1.0, 6.0],
                   "trial_runs": w.adapt["trials"], "trial_sweeps": w.adapt["sweeps_per_trial"],
                   "rate_threshold": w.adapt["rate_threshold"], "R_cap": w.R_cap,
                   "production_sweeps": w.sweeps, "exchange_every": w.every,
                   "attempts_per_step": attempts // args.steps},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "paper_scale_l32": paper_scale,
        "multi_hit_l64": multi_hit,
        "batched": batched,
        "served": served,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
