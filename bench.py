#!/usr/bin/env python3
"""Benchmark of the transport hot path on one MI355X.

Workload (one step): one batch of 2e7 histories of the lookup-bound scale
case -- a 255x255 pin lattice (15x15 assemblies of 17x17 pins, reflective
faces), one material of 300 synthetic nuclides on 20k-150k point grids
(605 MB of tables), 8192-bin hash grid, uniform 2 MeV source, event-based,
100x100x10 mesh flux tally on (an active batch).  value = active particles/s
over the timed steps (inputs resident in HBM, no per-launch timing inside the
timed region).

The lookup kernel, the dominant one, is timed with HIP events on the stream it
runs on, in a separate batch on one event loop.  Its roofline entry prices the
bytes it moves from DRAM per lookup (rocprofv3 counters, committed under
profiles/ for this kernel source) against the HBM peak; the algorithmic
gather rate (36 + 56 n_nuclides bytes per macroscopic lookup, which neighbours
in a sorted queue share through the caches) is reported beside it.  The
oracle (plain C, history-based) is timed on the host on a bounded sample of
the same workload.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# particle state one event kernel streams per event (position, direction,
# energy, weight, cross sections, ids, counters and flags: ~130 B per slot in
# the bank, plus the queue index and the fields written back)
STATE_BYTES_PER_EVENT = 150
METRIC = "active particles/s and macro-XS lookups/s (HBM GB/s % peak); FOM learned vs analog"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lookup_traffic_c3.json")
# launch shapes found by the library's autotuner on an MI355X (its cache format:
# one line per problem signature); missing or stale entries are tuned afresh
TUNING_CACHE = os.path.join(ROOT, "paper_2403_12345_amd", "tuning_cache.txt")


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for f in ("mc_kernels.hip", "mc_device.h"):
        with open(os.path.join(ROOT, "paper_2403_12345_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """DRAM bytes per macroscopic lookup of the transport's lookup kernel (read
    and written, from the committed rocprofv3 counter runs), valid only for
    the kernel source they were taken on; None otherwise."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_digest") != kernel_source_digest():
        return None
    return d


def streaming_rooflines(one, glob):
    """HBM rooflines of the event kernels that stream particle state, from a
    batch run with every launch timed: per event STATE_BYTES_PER_EVENT bytes;
    events are flights (k_advance), surface crossings (queue split and
    k_cross) and collisions (k_collide with its re-gathers), the last two as
    the batch's shares of its flights."""
    from paper_2403_12345_amd import mc
    flights = one["flights"]
    if not flights:
        return None
    ncoll, ncross = float(glob[mc.MC_G_NCOLL]), float(glob[mc.MC_G_NCROSS])
    f_coll = ncoll / (ncoll + ncross) if ncoll + ncross > 0 else 0.0
    out = {"bytes_per_event": STATE_BYTES_PER_EVENT, "flights": flights, "launches": one["iterations"],
           "collision_share_of_flights": f_coll}
    for name, ms, events in (("k_advance", one["advance_ms"], flights),
                             ("k_split+k_cross", one["cross_ms"], flights * (1.0 - f_coll)),
                             ("k_collide", one["collide_ms"], flights * f_coll)):
        if ms <= 0:
            continue
        gbs = STATE_BYTES_PER_EVENT * events / (ms / 1e3) / 1e9
        out[name] = {"ms": ms, "events": events, "ns_per_event": ms * 1e6 / events if events else None,
                     "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, seed: int, target_s: float = 15.0, n1: int = 2000):
    """The oracle on the host: the first pids of the same batch, sized to
    about target_s seconds."""
    import oracle
    op = oracle.OracleProblem(prob)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.run(op, seed, 0, n1)
    t1 = time.perf_counter() - t0
    n2 = int(min(prob.histories, max(n1, n1 * target_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    oracle.run(op, seed, 0, n2)
    t2 = time.perf_counter() - t0
    return {"value": n2 / t2, "unit": "particles/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"histories [0, {n2}) of one batch of the same problem, seed {seed}, "
                      f"history-based OpenMP over {threads} threads, {t2:.1f} s",
            "per_core": n2 / t2 / threads}


def cpu_oracle_extra(c2, c3, target_s: float = 5.0):
    """The oracle's other rates on the host: the 17x17 lattice on the first
    pids of its batch and macroscopic lookups/s on log-uniform energies for
    the 30-nuclide fuel and the 300-nuclide material."""
    import numpy as np

    import mcsynth
    import oracle
    threads = oracle.max_threads()
    op2 = oracle.OracleProblem(c2)
    n1 = 20_000
    t0 = time.perf_counter()
    oracle.run(op2, c2.seed, 0, n1)
    t1 = time.perf_counter() - t0
    n2 = int(min(c2.histories, max(n1, n1 * target_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    oracle.run(op2, c2.seed, 0, n2)
    t2 = time.perf_counter() - t0
    rng = np.random.default_rng(12345)
    out = {"cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
           "c2_subset": {"particles_per_s": n2 / t2, "per_core": n2 / t2 / threads,
                         "sample": f"histories [0, {n2}) of the 17x17 lattice batch, seed {c2.seed}, "
                                   f"{t2:.1f} s"}}
    op3 = oracle.OracleProblem(c3)
    for name, prob, n in (("c2_fuel_lookups_per_s", c2, 200_000), ("c3_lookups_per_s", c3, 20_000)):
        op = op3 if prob is c3 else op2
        E = mcsynth.lookup_energies(rng, n)
        t0 = time.perf_counter()
        oracle.macro_xs(op, np.zeros(n, np.int32), E)
        out[name] = n / (time.perf_counter() - t0)
    return out


def c2_transport(tuning_cache: str, prob=None, warmup: int = 3, steps: int = 12):
    """The 17x17 pin lattice (materials of 30/3/5 nuclides, 28 MB of tables
    that sit in the on-chip caches): batches of 1e6 histories through
    mc_run_batches with the tuned event loops, then one batch on one loop with
    its lookup launches timed."""
    import torch

    import mcsynth
    from paper_2403_12345_amd import mc
    from paper_2403_12345_amd.transport import Transport

    prob = prob if prob is not None else mcsynth.c2_problem()
    n, seed = prob.histories, prob.seed
    with Transport(prob, device=0) as t:
        tuning = mc.mc_autotune(t.ctx, seed, 1 << 40, n, tuning_cache)
        t.run_batches(seed, 0, n, warmup)
        t.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t.run_batches(seed, warmup * n, n, steps)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        tot = t.stats()
        mc.mc_set_tuning(t.ctx, **{**tuning, "loops": 1})
        t.run_batch(seed, (warmup + steps) * n, n, time_kernels=True)
        one = t.stats()
    launches = max(one["lookup_launches"], 1)
    avg_s = one["lookup_ms"] / 1e3 / launches
    gbs = one["lookup_bytes"] / launches / avg_s / 1e9 if avg_s > 0 else 0.0
    return {"workload": "17x17 pin lattice (r 0.41, pitch 1.26, h 1 cm, reflective), materials of 30/3/5 "
                        "synthetic nuclides on 10k-60k point fp64 grids (28 MB, cache-resident), 8192 hash "
                        "bins, uniform 2 MeV source, 1e6 histories per batch, per-pin flux tally",
            "particles_per_s": steps * n / elapsed, "ms_per_batch": elapsed / steps * 1e3,
            "warmup": warmup, "steps": steps, "tuning": tuning,
            "lookups_per_s_insitu": tot["lookups"] / elapsed,
            "nuclide_lookups_per_lookup": tot["nuclide_lookups"] / max(tot["lookups"], 1),
            "iterations_per_batch": tot["iterations"] / steps,
            "one_loop_batch_ms": one["batch_ms"],
            "lookup": {"avg_launch_us": avg_s * 1e6, "launches": one["lookup_launches"],
                       "effective_gather_GBs": gbs, "effective_gather_frac": gbs / HBM_PEAK_GBS,
                       "bound": "on-chip caches (tables in the Infinity Cache), not HBM"}}


def c3_channels(tuning: dict, n_chan: int = 10, histories: int = 20_000_000, prob=None):
    """The 300-nuclide lattice with n_chan reaction channels per nuclide (the
    per-nuclide reaction data of a depletion tally; ~2.6 GB of tables for 10):
    every lookup assembles them, every flight scores per-material
    track-length reaction rates.  One batch of 2e7 histories with the launch
    shapes tuned for the same lattice without channels, on one event loop (so
    the lookup kernel's time is its own)."""
    import mcsynth
    from paper_2403_12345_amd import mc
    from paper_2403_12345_amd.transport import Transport

    prob = prob if prob is not None else mcsynth.c3_problem()
    prob = mcsynth.with_channels(prob, n_chan)
    table_bytes = prob.data_bytes()
    try:
        with Transport(prob, device=0) as t:
            tuning = {**tuning, "loops": 1}
            mc.mc_set_tuning(t.ctx, **tuning)
            t.run_batch(prob.seed, 0, histories, time_kernels=True)
            s = t.stats()
            rr, _, _ = t.tallies(mc.MC_T_REACTION)
    finally:
        prob.channels = None
    sec = s["batch_ms"] / 1e3
    lk = s["lookup_ms"] / 1e3
    gbs = s["lookup_bytes"] / lk / 1e9 if lk > 0 else 0.0
    return {"workload": f"the 300-nuclide lattice with {n_chan} reaction channels per nuclide "
                        f"({table_bytes / 1e9:.2f} GB of tables), per-material track-length reaction "
                        f"rates, 2e7 histories per batch, one event loop",
            "xs_bytes": table_bytes,
            "n_chan": n_chan, "histories": histories, "particles_per_s": histories / sec, "batch_s": sec,
            "lookups_per_s_insitu": s["lookups"] / sec, "bytes_per_lookup": 36 + 8 * n_chan + (56 + 16 * n_chan) * 300,
            "lookup_kernel_s": lk, "lookup_GBs": gbs, "lookup_frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
            "reaction_rates_per_source": [float(x) for x in rr], "tuning": tuning}


def c2_union(tuning: dict, steps: int = 5, n_lookups: int = 10_000_000):
    """What the hash grid gives up against unionized grids on the 17x17
    lattice: the C2 transport (same tuning, 1e6 histories per batch) and 1e7
    stand-alone lookups on the 30-nuclide fuel, with per-nuclide hash searches
    and with one union-grid search per lookup (same results bit for bit)."""
    import numpy as np
    import torch

    import mcsynth
    from paper_2403_12345_amd import mc
    from paper_2403_12345_amd.transport import Transport

    prob = mcsynth.c2_problem()
    n = prob.histories
    out = {"workload": "17x17 lattice transport (1e6 histories per batch) and 1e7 log-uniform lookups on its "
                       "30-nuclide fuel, hash-grid against unionized-grid search"}
    rng = np.random.default_rng(4321)
    E = torch.from_numpy(mcsynth.lookup_energies(rng, n_lookups)).cuda()
    M = torch.zeros(n_lookups, dtype=torch.int32, device="cuda")
    Sa = torch.empty(n_lookups, dtype=torch.float64, device="cuda")
    Ss = torch.empty(n_lookups, dtype=torch.float64, device="cuda")
    with Transport(prob, device=0) as t:
        mc.mc_set_tuning(t.ctx, **tuning)
        for mode in ("hash", "union"):
            if mode == "union":
                out["union_table_bytes"] = mc.mc_set_union_grid(t.ctx, True)
            t.run_batches(prob.seed, 0, n, 1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t.run_batches(prob.seed, n, n, steps)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            r = {"particles_per_s": steps * n / sec}
            for srt in (False, True):
                mc.mc_lookup_macro(t.ctx, E, M, Sa, Ss, srt)
                mc.mc_set_timing(t.ctx, True)
                for _ in range(3):
                    mc.mc_lookup_macro(t.ctx, E, M, Sa, Ss, srt)
                s = t.stats()
                mc.mc_set_timing(t.ctx, False)
                r["sorted_lookups_per_s" if srt else "unsorted_lookups_per_s"] = s["lookups"] / (s["lookup_ms"] / 1e3)
            out[mode] = r
        mc.mc_set_union_grid(t.ctx, False)
    return out


FLOPS_PER_POLE = 280  # fp64 operations of one pole term (Faddeeva series of 32 terms, residues)


def multipole_microbench(n: int = 1_000_000, reps: int = 3):
    """Windowed-multipole lookups with Doppler broadening on the fly: 300
    synthetic nuclides of 200 resonances (poles) each, 1024 windows in
    sqrt(E), one material at 600 K, 1e6 log-uniform energies.  Bound by fp64
    arithmetic: FLOPS_PER_POLE per pole term summed against the 78.6 TFLOP/s
    fp64 vector peak."""
    import numpy as np
    import torch

    import mcsynth
    from paper_2403_12345_amd import mc

    nucs, ids, dens = mcsynth.multipole_material()
    rng = np.random.default_rng(99)
    E = torch.from_numpy(mcsynth.lookup_energies(rng, n)).cuda()
    M = torch.zeros(n, dtype=torch.int32, device="cuda")
    Sa = torch.empty(n, dtype=torch.float64, device="cuda")
    Ss = torch.empty(n, dtype=torch.float64, device="cuda")
    c = mc.mc_create(0)
    try:
        mc.mc_init_multipole(c, nucs, [len(ids)], ids, dens, [600.0])
        poles = mc.mc_lookup_multipole(c, E, M, Sa, Ss, count_poles=True)
        mc.mc_set_timing(c, True)
        for _ in range(reps):
            mc.mc_lookup_multipole(c, E, M, Sa, Ss)
        s = mc.mc_get_stats(c).as_dict()
        mc.mc_set_timing(c, False)
    finally:
        mc.mc_destroy(c)
    sec = s["lookup_ms"] / 1e3 / s["lookup_launches"]
    tflops = poles * FLOPS_PER_POLE / sec / 1e12
    return {"workload": "1e6 log-uniform energies, one material of 300 multipole nuclides (200 poles, 1024 windows "
                        "each) at 600 K", "lookups_per_s": n / sec, "pole_terms_per_lookup": poles / n,
            "launch_ms": sec * 1e3, "roofline": {"bound": "alu", "achieved": tflops, "peak": 78.6,
                                                  "unit": "TFLOP/s", "frac": tflops / 78.6,
                                                  "flops_per_pole": FLOPS_PER_POLE}}


def lookup_microbench(n: int = 10_000_000, reps: int = 3, ilps=(2,), prob=None):
    """Stand-alone lookup of n (energy, material) pairs on the 300-nuclide
    material (grids of 20k-150k points, ~0.6 GB of tables, far above the
    on-chip caches): the lookup-bound case, unsorted and sorted, for each
    number of nuclides looked up in lockstep per lane."""
    import numpy as np
    import torch

    import mcsynth
    from paper_2403_12345_amd import mc
    from paper_2403_12345_amd.transport import Transport

    prob = prob if prob is not None else mcsynth.c3_problem()
    rng = np.random.default_rng(12345)
    E = torch.from_numpy(mcsynth.lookup_energies(rng, n)).cuda()
    M = torch.zeros(n, dtype=torch.int32, device="cuda")
    Sa = torch.empty(n, dtype=torch.float64, device="cuda")
    Ss = torch.empty(n, dtype=torch.float64, device="cuda")
    out = {"workload": "macroscopic lookups of 1e7 log-uniform energies in [1e-5, 2e7] eV on one material "
                       "of 300 synthetic nuclides (clustered grids of 20k-150k points)",
           "n": n, "xs_bytes": prob.data_bytes(), "bytes_per_lookup": 36 + 56 * 300}
    with Transport(prob, device=0) as t:
        for ilp in ilps:
            mc.mc_set_tuning(t.ctx, lookup_ilp=ilp)
            for name, srt in (("unsorted", False), ("sorted", True)):
                mc.mc_lookup_macro(t.ctx, E, M, Sa, Ss, srt)  # warm-up
                mc.mc_set_timing(t.ctx, True)
                for _ in range(reps):
                    mc.mc_lookup_macro(t.ctx, E, M, Sa, Ss, srt)
                s = t.stats()
                mc.mc_set_timing(t.ctx, False)
                sec = s["lookup_ms"] / 1e3
                gbs = s["lookup_bytes"] / sec / 1e9
                out[f"{name}_ilp{ilp}"] = {
                    "lookups_per_s": s["lookups"] / sec, "achieved_GBs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
                    "avg_launch_ms": s["lookup_ms"] / s["lookup_launches"]}
        mc.mc_set_tuning(t.ctx)
    return out


def problem_set_bench(batches: int = 3):
    """The 64 uneven problems run together (persistent kernel, graph replay,
    autotuned work-item size and grid) against the same problems run one after
    another through the single-problem event loop."""
    import torch

    import mcsynth
    from paper_2403_12345_amd import mc
    from paper_2403_12345_amd.transport import ProblemSet, Transport

    probs = mcsynth.c4_problem_set()
    total = sum(p.histories for p in probs)
    with ProblemSet(probs, device=0) as ps:
        best = mc.mc_autotune_problem_set(ps.ctx)
        ps.run_batch(use_graph=True)  # capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(batches):
            ps.run_batch(use_graph=True)
        torch.cuda.synchronize()
        set_s = (time.perf_counter() - t0) / batches
    seq_s = 0.0
    for p in probs:
        with Transport(p, device=0) as t:
            t.run_batch(p.seed, 0, p.histories)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t.run_batch(p.seed, p.histories, p.histories)
            torch.cuda.synchronize()
            seq_s += time.perf_counter() - t0
    return {"workload": "64 independent fixed-source problems, histories log-uniform in [1e3, 1e5] "
                        f"({total} in all), 2-80 synthetic nuclides, infinite media and reflective pin cells",
            "histories_per_batch": total, "set_particles_per_s": total / set_s,
            "sequential_particles_per_s": total / seq_s, "speedup": seq_s / set_s,
            "set_ms_per_batch": set_s * 1e3, "sequential_ms_per_batch": seq_s * 1e3, "tuning": best}


def fom_bench(analog_histories: int = 40_000_000, learned_histories: int = 4_000_000, analog_batches: int = 40,
              batches: int = 20, shield: bool = False, linear_histories: int = 0):
    """Deep-penetration slab: figure of merit 1/(R^2 T) of the far-face leakage
    with windows from the learned importance map (bootstrap, training, one
    refinement round) against analog transport, the two estimates checked for
    agreement within 3 sigma.  Also the linear bootstrap windows, and the
    learned FOM with the generation and training time added to T.  shield:
    the slab whose attenuation sits in a thin dense shield deep inside, where
    the importance is far from linear in depth."""
    import math

    import mcsynth
    from paper_2403_12345_amd import importance
    from paper_2403_12345_amd.transport import Transport

    prob = mcsynth.c5_shield_problem() if shield else mcsynth.c5_problem()
    seed = prob.seed
    linear_histories = linear_histories or learned_histories
    layers = "160/12/28 cm, Sigma_t(2 MeV) 0.05/3.0/0.05" if shield else "100/10/90 cm, Sigma_t(2 MeV) 0.2/1.5/0.2"
    out = {"workload": f"3-layer slab {layers} per cm, synthetic absorber/scatterers (10 nuclides), normal "
                       f"2 MeV beam, detector = leakage through x = 200",
           "analog_histories": analog_histories, "learned_histories": learned_histories,
           "linear_histories": linear_histories, "analog_batches": analog_batches, "batches": batches}
    with Transport(prob) as t:
        t.run_batch(seed, 0, 100_000)  # warm-up (allocation, first launches)
        tic = time.perf_counter()
        li = importance.learn(t, seed=seed, pilot=1_000_000, boot=250_000, steps=2000, refine=1)
        t_learn = time.perf_counter() - tic
        an = importance.production(t, seed=seed + 1, histories=analog_histories, batches=analog_batches,
                                   windows="analog")
        lin = importance.production(t, seed=seed + 2, histories=linear_histories, batches=batches,
                                    windows="linear", lin=(0.0, li.slope, 0.0))
        ml = importance.production(t, seed=seed + 3, histories=learned_histories, batches=batches,
                                   windows="mlp", ln_range=li.ln_range)

    def entry(p):
        return {"mean": p.mean, "rel_err": p.rel, "seconds": p.seconds, "fom": p.fom,
                "histories": p.histories, "splits_per_history": p.splits, "roulette_per_history": p.roulette}

    out["analog"] = entry(an)
    out["linear_bootstrap"] = entry(lin)
    out["learned"] = entry(ml)
    out["learn_seconds"] = t_learn
    out["learn_breakdown"] = li.seconds
    out["training_samples"] = li.n_samples[-1]
    out["final_loss"] = float(li.loss_curves[-1][-1])
    out["ln_importance_span"] = li.ln_range
    out["gain_vs_analog"] = ml.fom / an.fom if an.fom > 0 else None
    out["gain_vs_linear"] = ml.fom / lin.fom if lin.fom > 0 else None
    rel = ml.rel
    out["learned_fom_incl_training"] = 1.0 / (rel * rel * (ml.seconds + t_learn)) if ml.mean > 0 else 0.0
    out["agree_3sigma"] = bool(abs(ml.mean - an.mean) <= 3 * math.hypot(ml.stderr, an.stderr))
    return out


def copy_calibration(n_doubles: int = 1 << 28, reps: int = 5):
    """A plain device copy of known size (2 GiB read + 2 GiB written per launch),
    the reference for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    x = torch.ones(n_doubles, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) / 1e3 / reps
    return {"bytes_read_per_launch": n_doubles * 8, "bytes_written_per_launch": n_doubles * 8,
            "copy_GBs": 2 * n_doubles * 8 / sec / 1e9}


def pmc_per_dispatch(dirs, kernel_regex: str):
    """Counter values of the dispatches whose kernel name matches kernel_regex,
    from rocprofv3 --pmc CSV output (every *counter_collection.csv under the
    given directories): {counter: [value per dispatch]}, dispatches in id order."""
    import csv
    import glob
    import re
    pat = re.compile(kernel_regex)
    per = {}
    for d in dirs:
        for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
            with open(f, newline="") as fh:
                for row in csv.DictReader(fh):
                    if not pat.search(row.get("Kernel_Name", "")):
                        continue
                    key = (f, int(row.get("Dispatch_Id", 0)))
                    per.setdefault(row["Counter_Name"], {})
                    per[row["Counter_Name"]][key] = per[row["Counter_Name"]].get(key, 0.0) + float(row["Counter_Value"])
    return {c: [v[k] for k in sorted(v)] for c, v in per.items()}


def traffic_summary(lookup_dirs, copy_dirs, roof_json: str, out_path: str, stream_dirs=None):
    """Bytes the lookup kernel moves between L2 and memory, per macroscopic
    lookup, from rocprofv3 counter runs of the roofline batch (bench.py --mode
    c3roof, whose JSON line gives the batch's lookups), and the same counters
    on the copy calibration (bench.py --mode copy: 2 GiB read + 2 GiB written
    per launch) as the scale check.  Read bytes by request size: 32 B x
    TCC_EA0_RDREQ_32B + 64 B x _64B + 128 B x _128B; bytes to DRAM: 32 B x
    TCC_EA0_RDREQ_DRAM_32B (a 64-byte request counts 2, a 128-byte one 4) and
    32 B x TCC_EA0_WRREQ_WRITE_DRAM_32B; FETCH_SIZE and WRITE_SIZE (KiB) as
    the counter definitions compute them, with the copy's ratio of true to
    counted bytes."""
    with open(roof_json) as f:
        roof = json.loads(f.read().strip().splitlines()[-1])["c3_roofline_batch"]
    lk = pmc_per_dispatch(lookup_dirs, r"k_lookup")
    cp = pmc_per_dispatch(copy_dirs, r"(?i)copy|elementwise") if copy_dirs else {}

    def tot(d, c):
        return float(sum(d.get(c, []))) if c in d else None

    n_lookups = roof["lookups"]
    launches = roof["lookup_launches"]
    out = {"kernel_digest": roof["kernel_digest"], "source": "profiles/k_lookup_c3_transport.md",
           "lookups": n_lookups, "launches": launches,
           "dispatches_counted": {c: len(v) for c, v in lk.items()}}
    rd = {b: tot(lk, f"TCC_EA0_RDREQ_{b}B_sum") for b in (32, 64, 128)}
    if all(v is not None for v in rd.values()):
        rbytes = 32 * rd[32] + 64 * rd[64] + 128 * rd[128]
        out["read_requests"] = {f"{b}B": rd[b] for b in rd}
        out["read_bytes_per_lookup"] = rbytes / n_lookups
    dram = tot(lk, "TCC_EA0_RDREQ_DRAM_32B_sum")
    dramw = tot(lk, "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum")
    if dram is not None:
        out["dram_read_bytes_per_lookup"] = 32 * dram / n_lookups
    if dramw is not None:
        out["dram_write_bytes_per_lookup"] = 32 * dramw / n_lookups
    if dram is not None and dramw is not None:
        out["dram_bytes_per_lookup"] = 32 * (dram + dramw) / n_lookups
    hit, miss = tot(lk, "TCC_HIT_sum"), tot(lk, "TCC_MISS_sum")
    if hit is not None and miss is not None and hit + miss > 0:
        out["l2_hit"] = hit / (hit + miss)
    fetch, write = tot(lk, "FETCH_SIZE"), tot(lk, "WRITE_SIZE")
    cal = {}
    copy_bytes = float(1 << 31)
    if cp:
        n_copy = max(len(cp.get("FETCH_SIZE", [])), len(cp.get("WRITE_SIZE", [])), 1)
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            if c in cp and cp[c]:
                cal[c] = copy_bytes / (max(cp[c]) * 1024.0)  # true bytes per counted byte, largest dispatch = the copy
        rdc = {b: cp.get(f"TCC_EA0_RDREQ_{b}B_sum") for b in (32, 64, 128)}
        if all(rdc.values()):
            k = max(range(len(rdc[128])), key=lambda j: rdc[128][j])
            cal["read_by_size"] = copy_bytes / (32 * rdc[32][k] + 64 * rdc[64][k] + 128 * rdc[128][k])
        if cp.get("TCC_EA0_RDREQ_DRAM_32B_sum"):
            cal["dram_read"] = copy_bytes / (32 * max(cp["TCC_EA0_RDREQ_DRAM_32B_sum"]))
        if cp.get("TCC_EA0_WRREQ_WRITE_DRAM_32B_sum"):
            cal["dram_write"] = copy_bytes / (32 * max(cp["TCC_EA0_WRREQ_WRITE_DRAM_32B_sum"]))
        out["copy_dispatches"] = n_copy
    out["copy_scale"] = cal
    if dram is not None and dramw is not None:
        # the DRAM-side bytes with the copy's ratio of true to counted bytes
        out["dram_bytes_per_lookup_scaled"] = 32 * (dram * cal.get("dram_read", 1.0) +
                                                    dramw * cal.get("dram_write", 1.0)) / n_lookups
    if fetch is not None:
        out["fetch_kib_per_launch"] = fetch / launches
    if write is not None:
        out["write_kib_per_launch"] = write / launches
    if fetch is not None and write is not None and "FETCH_SIZE" in cal and "WRITE_SIZE" in cal:
        out["traffic_bytes_per_lookup"] = (fetch * cal["FETCH_SIZE"] + write * cal["WRITE_SIZE"]) * 1024 / n_lookups
    sq = {c: tot(lk, c) for c in ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_INSTS_SMEM",
                                  "SQ_INSTS_VMEM_RD", "SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES",
                                  "SQ_INST_CYCLES_VALU", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_BRANCH",
                                  "SQ_LDS_BANK_CONFLICT", "SQ_WAIT_INST_LDS", "SQ_INSTS_VALU_INT32",
                                  "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
                                  "SQ_INSTS_VALU_TRANS_F64", "GRBM_GUI_ACTIVE") if c in lk}
    if sq:
        wave_nuc = roof["nuclide_lookups"] / 64.0
        out["per_wave_nuclide"] = {c: v / wave_nuc for c, v in sq.items()
                                   if c.startswith("SQ_INSTS") or c.startswith("SQ_INST_")}
        out["sq_totals"] = sq
    # the event kernels that stream particle state: DRAM-side bytes per flight
    if stream_dirs:
        st_out = {}
        for name, rx in (("k_advance", r"k_advance"), ("k_split", r"k_split_"), ("k_cross", r"k_cross"),
                         ("k_collide", r"k_collide"), ("k_slots", r"k_slots_")):
            d = pmc_per_dispatch(stream_dirs, rx)
            r, w = tot(d, "TCC_EA0_RDREQ_DRAM_32B_sum"), tot(d, "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum")
            if r is None or w is None or not roof.get("flights"):
                continue
            st_out[name] = {"dispatches": len(d["TCC_EA0_RDREQ_DRAM_32B_sum"]),
                            "dram_read_bytes_per_flight": 32 * r / roof["flights"],
                            "dram_write_bytes_per_flight": 32 * w / roof["flights"]}
        out["streaming_per_flight"] = st_out
    out["source_runs"] = {"lookup": list(lookup_dirs), "copy": list(copy_dirs or []), "roofline_batch": roof_json,
                          "streaming": list(stream_dirs or [])}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1, help="untimed batches first")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-inactive", action="store_true", help="skip the tally-off contrast batch")
    ap.add_argument("--no-lookup-bench", action="store_true", help="skip the 300-nuclide lookup benchmark")
    ap.add_argument("--no-problem-set", action="store_true", help="skip the 64-problem batching benchmark")
    ap.add_argument("--no-fom", action="store_true", help="skip the learned-importance figure-of-merit benchmark")
    ap.add_argument("--no-c2", action="store_true", help="skip the 17x17 lattice transport batches")
    ap.add_argument("--no-channels", action="store_true", help="skip the 300-nuclide lattice with reaction channels")
    ap.add_argument("--tuning-cache", default=TUNING_CACHE, help="autotuner cache file")
    ap.add_argument("--no-union", action="store_true", help="skip the hash-grid against union-grid comparison")
    ap.add_argument("--no-multipole", action="store_true", help="skip the windowed-multipole lookup benchmark")
    ap.add_argument("--loops", type=int, default=0, help="event loops of the timed steps (0: the tuned count)")
    ap.add_argument("--tune", nargs="*", default=[], metavar="KEY=VALUE",
                    help="override tuned launch shapes of the headline workload (mc_tuning fields)")
    ap.add_argument("--pmc-dirs", nargs="*", default=[], help="traffic mode: rocprofv3 --pmc output directories "
                                                              "of the roofline batch")
    ap.add_argument("--copy-dirs", nargs="*", default=[], help="traffic mode: the same counters on --mode copy")
    ap.add_argument("--roof-json", default="", help="traffic mode: the JSON line printed by --mode c3roof")
    ap.add_argument("--stream-dirs", nargs="*", default=[], help="traffic mode: DRAM counter runs of the event "
                                                                 "kernels that stream particle state")
    ap.add_argument("--traffic-out", default=TRAFFIC_FILE, help="traffic mode: where to write the summary")
    ap.add_argument("--mode", choices=("full", "c3", "c3roof", "traffic", "lookup", "copy", "set", "fom", "c2", "union",
                                       "multipole"),
                    default="full",
                    help="c3: the headline steps only (no other benchmark, no CPU baseline); c3roof: only the "
                         "roofline batch (one batch of the headline workload on one event loop, every lookup "
                         "launch timed; for counter runs); lookup: only the 300-nuclide lookup benchmark; copy: "
                         "only the copy calibration")
    args = ap.parse_args()
    if args.mode == "c3":
        for k in ("no_cpu_baseline", "no_inactive", "no_lookup_bench", "no_problem_set", "no_fom", "no_c2",
                  "no_channels", "no_union", "no_multipole"):
            setattr(args, k, True)
    if args.mode == "traffic":  # host only: summarise counter runs
        print(json.dumps(traffic_summary(args.pmc_dirs, args.copy_dirs, args.roof_json, args.traffic_out,
                                         args.stream_dirs)))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on a single MI355X and has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import mcsynth
    from paper_2403_12345_amd.transport import Transport

    torch.cuda.set_device(0)
    if args.mode == "copy":
        print(json.dumps({"copy_calibration": copy_calibration()}), flush=True)
        return
    if args.mode == "lookup":
        print(json.dumps({"lookup_microbench": lookup_microbench(ilps=(1, 2, 4))}), flush=True)
        return
    if args.mode == "set":
        print(json.dumps({"problem_set": problem_set_bench()}), flush=True)
        return
    if args.mode == "fom":
        print(json.dumps({"fom": fom_bench(),
                          "fom_shield": fom_bench(shield=True, learned_histories=4_000_000,
                                                  linear_histories=400_000)}), flush=True)
        return
    if args.mode == "multipole":
        print(json.dumps({"multipole": multipole_microbench()}), flush=True)
        return
    if args.mode == "union":
        from paper_2403_12345_amd import mc
        p = mcsynth.c2_problem()
        with Transport(p, device=0) as t:
            tuning = mc.mc_autotune(t.ctx, p.seed, 1 << 40, p.histories, args.tuning_cache)
        print(json.dumps({"c2_union": c2_union(tuning)}), flush=True)
        return
    if args.mode == "c2":
        print(json.dumps({"c2_transport": c2_transport(args.tuning_cache)}), flush=True)
        return
    from paper_2403_12345_amd import mc

    prob = mcsynth.c3_problem()
    n = prob.histories
    seed = prob.seed
    if args.mode == "c3roof":
        with Transport(prob, device=0) as t:
            tuning = mc.mc_autotune(t.ctx, seed, 1 << 40, n, args.tuning_cache)
            tuning = {**tuning, **{k: int(v) for k, v in (kv.split("=", 1) for kv in args.tune)}}
            mc.mc_set_tuning(t.ctx, **{**tuning, "loops": 1})
            t.run_batch(seed, 0, n, time_kernels=True)
            one = t.stats()
        print(json.dumps({"c3_roofline_batch": {
            "histories": n, "tuning": {**tuning, "loops": 1}, "lookups": one["lookups"],
            "nuclide_lookups": one["nuclide_lookups"], "lookup_launches": one["lookup_launches"],
            "lookup_ms": one["lookup_ms"], "lookup_bytes": one["lookup_bytes"], "batch_ms": one["batch_ms"],
            "flights": one["flights"], "advance_ms": one["advance_ms"], "cross_ms": one["cross_ms"],
            "collide_ms": one["collide_ms"], "iterations": one["iterations"],
            "kernel_digest": kernel_source_digest()}}), flush=True)
        return
    t = Transport(prob, device=0)
    # launch shapes from the library's autotuner (from its cache when this
    # problem was tuned on this device kind, else timed on batches of other pids)
    tuning = mc.mc_autotune(t.ctx, seed, 1 << 40, n, args.tuning_cache)
    if args.loops or args.tune:
        over = {k: int(v) for k, v in (kv.split("=", 1) for kv in args.tune)}
        tuning = {**tuning, **over, **({"loops": args.loops} if args.loops else {})}
        mc.mc_set_tuning(t.ctx, **tuning)
    if args.warmup:
        t.run_batches(seed, 0, n, args.warmup)
    t.reset()
    # the K steps: K batches through mc_run_batches, no per-launch timing
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t.run_batches(seed, args.warmup * n, n, args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = args.steps * n / elapsed
    steps_stats = t.stats()
    mesh, _, _ = t.tallies(mc.MC_T_FLUX_TRACK)
    glob, _, _ = t.tallies(mc.MC_T_GLOBAL)

    # the roofline of the lookup kernel: one more batch on one event loop with
    # every lookup launch bracketed by HIP events on its stream (with several
    # loops a launch shares the GPU with the other loops' kernels)
    mc.mc_set_tuning(t.ctx, **{**tuning, "loops": 1})
    t.reset()
    t.run_batch(seed, (args.warmup + args.steps) * n, n, time_kernels=True)
    one = t.stats()
    glob_one, _, _ = t.tallies(mc.MC_T_GLOBAL)
    mc.mc_set_tuning(t.ctx, **tuning)

    inactive = None
    if not args.no_inactive:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        t.run_batch(seed, (args.warmup + args.steps + 1) * n, n, no_tally=True)
        torch.cuda.synchronize()
        inactive = n / (time.perf_counter() - t1)
    t.close()

    streaming = streaming_rooflines(one, glob_one)
    launches = max(one["lookup_launches"], 1)
    avg_launch_s = one["lookup_ms"] / 1e3 / launches
    lookups_per_launch = one["lookups"] / launches
    alg_bytes_per_launch = one["lookup_bytes"] / launches
    alg_gbs = alg_bytes_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    traffic = measured_traffic()
    if traffic is not None:
        dram_per_launch = traffic.get("dram_bytes_per_lookup_scaled", traffic["dram_bytes_per_lookup"]) * \
            lookups_per_launch
        achieved = dram_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
        roof_bytes = "DRAM bytes per lookup from the committed counter runs x lookups per launch"
    else:
        dram_per_launch = None
        achieved = None
        roof_bytes = "no counter data for this kernel source: DRAM traffic unmeasured"
    roofline = {
        "kernel": "k_lookup (sorted-queue window path)",
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS if achieved is not None else None,
        "traffic": dram_per_launch,
        "bytes": roof_bytes,
        "avg_launch_us": avg_launch_s * 1e6,
        "launches": one["lookup_launches"],
        "lookups_per_launch": lookups_per_launch,
        "measured_on": "one batch on one event loop, every lookup launch timed with HIP events",
        "algorithmic_bytes_per_launch": alg_bytes_per_launch,
        "effective_gather_GBs": alg_gbs,
        "effective_gather_frac": alg_gbs / HBM_PEAK_GBS,
    }
    if traffic is not None:
        roofline["counter_profile"] = traffic.get("source")
        roofline["l2_hit"] = traffic.get("l2_hit")
        if traffic.get("valu_insts_per_nuclide_wave") is not None:
            roofline["valu_insts_per_nuclide_wave"] = traffic["valu_insts_per_nuclide_wave"]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "255x255 pin lattice (15x15 assemblies of 17x17 pins, r 0.41, pitch 1.26, h 1 cm, "
                        "reflective), one material of 300 synthetic nuclides on 20k-150k point fp64 grids "
                        "(605 MB of tables), 8192 hash bins, uniform 2 MeV source, 2e7 histories per batch "
                        "event-based, 100x100x10 mesh flux tally",
            "histories_per_step": n,
            "in_flight": tuning["in_flight"],
            "tuning": tuning,
            "nuclides": len(prob.nuclides),
            "xs_bytes": prob.data_bytes(),
        },
        "roofline": roofline,
        "one_loop_batch_ms": one["batch_ms"],
        "one_loop_particles_per_s": n / (one["batch_ms"] / 1e3),
        "lookups_per_s_kernel": one["lookups"] / (one["lookup_ms"] / 1e3) if one["lookup_ms"] else None,
        "lookups_per_s_insitu": steps_stats["lookups"] / elapsed,
        "lookup_kernel_share_one_loop": one["lookup_ms"] / one["batch_ms"] if one["batch_ms"] else None,
        "iterations_per_step": steps_stats["iterations"] / args.steps,
        "mesh_track_sum": float(mesh.sum()),
        "total_track": float(glob[mc.MC_G_TRACK]),
        "mesh_underflow": steps_stats["mesh_underflow"],
        "inactive_particles_per_s": inactive,
        "streaming_kernels": streaming,
    }
    c2 = mcsynth.c2_problem()
    if not args.no_c2:
        line["c2_transport"] = c2_transport(args.tuning_cache, prob=c2)
    if not args.no_lookup_bench:
        line["lookup_microbench"] = lookup_microbench(prob=prob)
    if not args.no_channels:
        line["c3_channels"] = c3_channels(tuning, prob=prob)
    # rates quoted against the measured copy bandwidth too
    cal = copy_calibration() if args.mode != "c3" else None
    if cal is not None:
        line["copy_GBs"] = cal["copy_GBs"]
        line["roofline"]["effective_gather_frac_of_copy_bw"] = alg_gbs / cal["copy_GBs"]
    if not args.no_lookup_bench:
        for k, v in line["lookup_microbench"].items():
            if isinstance(v, dict) and "achieved_GBs" in v:
                v["frac_of_copy_bw"] = v["achieved_GBs"] / cal["copy_GBs"]
    if not args.no_union:
        c2_tuning = line["c2_transport"]["tuning"] if "c2_transport" in line else {}
        line["c2_union"] = c2_union(c2_tuning)
    if not args.no_multipole:
        line["multipole"] = multipole_microbench()
    if not args.no_problem_set:
        line["problem_set"] = problem_set_bench()
    if not args.no_fom:
        line["fom"] = fom_bench()
        # linear windows split ~500 times per history in the shielded slab:
        # fewer histories for them
        line["fom_shield"] = fom_bench(shield=True, learned_histories=4_000_000, linear_histories=400_000)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob, seed)
        line["cpu_oracle"] = cpu_oracle_extra(c2, prob)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
