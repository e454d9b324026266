#!/usr/bin/env python3
"""Benchmark: replica-exchange Metropolis sweeps of a bead-spring homopolymer
on one MI355X, mixed precision (FP32 Lennard-Jones terms and pair sums from
FP64 separations; FP64 bond terms, energies and decisions) beside plain FP64,
on the same seeded synthetic input.

A step is one pass of the whole hot path over the batch: every slot does one
sweep of N single-monomer moves (each scored against all N-1 other monomers
plus its bonds), records E, Ree^2 and Rg^2, and one neighbour-temperature
exchange step follows.  The timed region is K such steps enqueued with HIP
events around every sweep-kernel launch, bracketed by a synchronize.  Where
all replicas fit on the chip at once, one persistent launch runs all K steps;
where they do not, one task-flow launch does.

Prints one JSON line.  Default workload: one chain of N = 100 monomers,
64 temperatures geometric in [0.1, 1.5], random-walk start, seed 2; the line
also holds sub-records of the long-chain workload (N = 500, 128 slots) and of
the two batched workloads (48 uneven chains; 16 chains of N = 2000 with 256
slots each), each on its own step counts.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_PAIR = 27          # two LJ evaluations (13 each) + their difference
# Arithmetic of the mixed path (the `dtype` field): Lennard-Jones brackets in
# FP32 from FP64 separations, summed in FP32; bond terms, running energies and
# every decision in FP64; moves inside the guard band re-scored in FP64.
MIXED_DTYPE = "f32 pair terms and pair sums, f64 separations, bonds, energies and decisions"
PEAK_FP32 = 157.3e12        # MI355X FP32 vector, FLOP/s
PEAK_FP64 = 78.6e12         # MI355X FP64 vector, FLOP/s

WORKLOADS = {
    "c2": "1 chain, N=100, 64 slots, T geometric in [0.1,1.5], random-walk start, seed 2",
    "c3": "1 chain, N=500, 128 slots, T geometric in [0.2,2.0], random-walk start, seed 3",
    "c4": "48 chains, N uniform over {13,30,55,100,200,500}, 32 slots each, T in [0.1,1.5], seed 4",
    "c5": "16 chains, N=2000, 256 slots each, T geometric in [0.3,2.5], random-walk start, seed 5",
    "c1": "1 chain, N=30, 16 slots, T geometric in [0.1,1.5], straight start, seed 1",
}


_T0 = time.perf_counter()


def progress(msg):
    """A progress line on stderr (stdout carries the JSON line alone)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def run_gpu(w, precision, steps, warmup, schedule=0, tune=True, by_n=None):
    import torch
    from paper_1107_3490_amd import pt

    # The mapping autotuner (outside the timed region), or the caller's mapping
    # per chain length (by_n); results do not depend on it.
    if by_n is not None:
        mapping = np.array([by_n[int(n)] for n in w.n_beads], dtype=np.int32)
    else:
        mapping = pt.autotune(w, precision, schedule, trial_sweeps=20) if tune else None
    sim = pt.Simulation(w, precision=precision, schedule=schedule, mapping=mapping)
    bpl, wpr, _ = sim.mapping()
    codes = list(mapping) if mapping is not None else [0] * len(w.n_beads)
    def flag(c):
        c = int(c)
        return (("lane",) if c & pt.PT_MAP_LANE else ("pack2",) if c & pt.PT_MAP_PACK2
                else ("pack4",) if c & pt.PT_MAP_PACK4 else ())

    tuned = sorted({(int(n), int(b), int(v)) + flag(c) for n, b, v, c in zip(w.n_beads, bpl, wpr, codes)})
    classes = sorted({(int(b), int(v)) for b, v in zip(bpl, wpr)})
    modes = sim.mapping()[2]
    persistent = bool(np.all(modes == 1))
    # schedule of each (B, W) class: 1 persistent, 2 task flow, 0 per sweep
    class_mode = {(int(b), int(v)): int(m) for b, v, m in zip(bpl, wpr, modes)}
    sim.sweep(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sweep_ms, total_ms, launches = sim.time_sweeps(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    obs = sim.observables()
    # Stability of the figure: five more segments of K/5 steps (after the
    # timed region, not part of it).
    seg = max(1, steps // 5)
    repeats = [sim.time_sweeps(seg)[1] / seg for _ in range(5)]
    sim.close()
    pairs = w.pair_interactions_per_sweep() * steps
    return dict(pairs=pairs, wall_s=wall, event_total_ms=total_ms, sweep_kernel_ms=sweep_ms,
                launches=launches, rescored=int(obs["counts"][:, 3].sum()),
                moves=int(obs["counts"][:, 5].sum()), exch_recompute=int(obs["counts"][:, 4].sum()),
                persistent=persistent, class_mode=class_mode, mapping=tuned, classes=classes,
                resyncs=int(obs["counts"][:, 6].sum()), repeats_ms_per_step=repeats)


def kernel_sources_sha256():
    """SHA-256 over every device source of the library (kernels, device
    helpers, the persistent and task-flow instantiations), in name order."""
    csrc = os.path.join(ROOT, "paper_1107_3490_amd", "csrc")
    h = hashlib.sha256()
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith((".hip", ".hpp", ".inc")):
            with open(os.path.join(csrc, fn), "rb") as f:
                h.update(fn.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(workload, kernel, sweeps_per_launch):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes (copy-calibrated, per sweep), or None when they were
    taken on other kernel sources or another kernel."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    e = t.get(workload)
    entries = e if isinstance(e, list) else [e] if e is not None else []
    for x in entries:
        if x.get("kernel") == kernel:
            return (x["read_bytes_per_sweep"] + x["write_bytes_per_sweep"]) * sweeps_per_launch
    return None


def with_transfers(w, steps):
    """Mixed path with the host-side costs the paper's timings include: handle
    set-up (validation, swizzle, host-to-device copies, starting energies), the
    K sweeps, and the read-back of every conformation and observable."""
    import torch
    from paper_1107_3490_amd import pt

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim = pt.Simulation(w, precision="mixed")
    sim.sweep(steps)
    sim.coords()
    sim.observables()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.close()
    return dict(value=w.pair_interactions_per_sweep() * steps / wall, unit="pair interactions/s",
                wall_s=wall, note="pt_init with uploads + K sweeps + read-back, default mapping")


def cpu_baseline(w, budget_s=12.0, threads=None):
    """The CPU oracle as it stands, on a bounded sample of the same workload:
    a first short run gives the rate, a second run fills about budget_s."""
    from oracle import oracle as O

    threads = threads or int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    sim = O.Simulation(w, n_threads=threads)
    t0 = time.perf_counter()
    sim.run(2)
    dt = time.perf_counter() - t0
    per_sweep = max(dt / 2, 1e-6)
    n = max(2, min(w.sweeps, int(budget_s / per_sweep)))
    t0 = time.perf_counter()
    sim.run(n)
    dt = time.perf_counter() - t0
    pairs = w.pair_interactions_per_sweep() * n
    return dict(value=pairs / dt, unit="pair interactions/s", cores=threads, cpu_model=cpu_model(), kind="oracle",
                sample=f"{n} sweeps of the full workload ({pairs:.3e} pair interactions, "
                       f"{dt:.1f} s, OpenMP over slots, FP64 incl. per-sweep canonical energy)")


def paper_protocol(n_beads=55, sweeps=4000, every=1000, edge=0.02,
                   replicas=(1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096)):
    """The benchmark of the paper's Sec. 4.2 on this GPU: one chain of N = 55,
    displacement edge 0.02, 4000 sweeps, an exchange step every 1000 sweeps, as
    a function of the number of replicas n_r.  t_GPU includes set-up, the
    host-to-device copies, the sweeps and the read-back of every conformation
    (the paper's timing includes its copies); S_p = t_CPU / t_GPU with t_CPU the
    oracle on one core, timed on a few replicas and scaled by n_r (its cost is
    linear in n_r).  The mapping is the autotuner's (chosen before the timed run:
    one or several replicas per wavefront), and the default one is timed beside
    it.  Context only: the paper's hardware and numbers differ."""
    import torch
    from oracle import oracle as O
    from paper_1107_3490_amd import inputs as I
    from paper_1107_3490_amd import pt

    def workload(nr):
        return I.make_workload([n_beads], [nr], [(0.1, 1.5)], "straight", 55, sweeps, "mixed",
                               name="paper-protocol", step_edge=edge, exchange_every=every)

    # one oracle core: 4 replicas, 1000 sweeps
    wc = workload(4)
    sim = O.Simulation(wc, n_threads=1)
    t0 = time.perf_counter()
    sim.run(1000)
    cpu_per_replica_sweep = (time.perf_counter() - t0) / (4 * 1000)
    rows = []
    def t_run(w, prec, mapping):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = pt.Simulation(w, precision=prec, mapping=mapping)
        s.sweep(sweeps)
        s.coords()
        s.observables()
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        s.close()
        return t

    for nr in replicas:
        w = workload(nr)
        for prec in ("mixed", "fp64"):
            progress(f"paper protocol: n_r = {nr}, {prec}")
            code = int(pt.autotune(w, prec, trial_sweeps=20)[0])
            t_gpu = t_run(w, prec, [code])
            t_default = t_run(w, prec, None)
            t_cpu = cpu_per_replica_sweep * nr * sweeps
            rows.append({"n_r": nr, "precision": prec, "mapping": hex(code), "t_gpu_s": t_gpu,
                         "t_gpu_default_mapping_s": t_default, "t_cpu_1core_s": t_cpu,
                         "S_p": t_cpu / t_gpu,
                         "pair_per_s": w.pair_interactions_per_sweep() * sweeps / t_gpu})
    return {"protocol": f"N={n_beads}, edge {edge}, {sweeps} sweeps, exchange every {every}, "
                        "straight start, T geometric in [0.1, 1.5]; t_GPU incl. set-up, copies, read-back",
            "cpu_1core_s_per_replica_sweep": cpu_per_replica_sweep, "rows": rows}


def ablations(sweeps=40, warmup=5):
    """The paper's alternative designs, timed on this GPU beside the main path
    (sweep-kernel event time, same inputs, identical results):
      * one lane per replica (the paper's first design: a thread runs a whole
        sweep) against the wavefront-per-replica kernels, FP64, on the paper's
        N = 55 chain as a function of the number of replicas;
      * the full FP64-order energy recomputed after every sweep (the paper's
        per-sweep energy) against the running energy, on the N = 100 and
        N = 500 workloads and the N = 55 chain at 4096 replicas;
      * mixed precision with every accepted move re-scored in the FP64 order
        (a running energy as accurate as the FP64 path's) against plain mixed
        and plain FP64;
      * the paper's one-pair-per-thread energy kernel against the FP64-order
        one (one wavefront per conformation, a row per lane)."""
    import torch
    from paper_1107_3490_amd import inputs as I
    from paper_1107_3490_amd import pt

    def timed(w, prec, schedule=0, mapping=None):
        s = pt.Simulation(w, precision=prec, schedule=schedule, mapping=mapping)
        s.sweep(warmup)
        torch.cuda.synchronize()
        _, total_ms, _ = s.time_sweeps(sweeps)
        persistent = bool(np.all(s.mapping()[2] != 0))
        s.close()
        return total_ms / sweeps, persistent

    def chain55(nr):
        return I.make_workload([55], [nr], [(0.1, 1.5)], "straight", 55, sweeps, "fp64",
                               name="N=55", step_edge=0.02)

    lane_rows = []
    for nr in (64, 256, 1024, 4096, 16384):
        progress(f"ablations: one lane per replica, n_r = {nr}")
        w = chain55(nr)
        wave_ms, pers = timed(w, "fp64")
        lane_ms, _ = timed(w, "fp64", mapping=[pt.PT_MAP_LANE | 0x11])
        pps = w.pair_interactions_per_sweep() * 1e3
        lane_rows.append({"n_r": nr, "wavefront_ms_per_sweep": wave_ms, "wavefront_persistent": pers,
                          "lane_ms_per_sweep": lane_ms, "wavefront_pair_per_s": pps / wave_ms,
                          "lane_pair_per_s": pps / lane_ms, "lane_over_wavefront_time": lane_ms / wave_ms})
    energy_rows = []
    for name, w in (("c2", I.named("c2")), ("c3", I.named("c3")), ("N=55 x 4096", chain55(4096))):
        for prec in ("mixed", "fp64"):
            progress(f"ablations: full energy every sweep, {name}, {prec}")
            run_ms, pers = timed(w, prec)
            full_ms, _ = timed(w, prec, schedule=pt.PT_SCHED_FULL_ENERGY)
            energy_rows.append({"workload": name, "precision": prec, "persistent": pers,
                                "running_energy_ms_per_sweep": run_ms,
                                "full_energy_ms_per_sweep": full_ms,
                                "full_over_running": full_ms / run_ms})
    accept_rows = []
    for name, w in (("c2", I.named("c2")), ("c3", I.named("c3")), ("N=55 x 4096", chain55(4096))):
        run_ms, pers = timed(w, "mixed")
        on_ms, _ = timed(w, "mixed", schedule=pt.PT_SCHED_FP64_ON_ACCEPT)
        fp64_ms, _ = timed(w, "fp64")
        accept_rows.append({"workload": name, "persistent": pers, "mixed_ms_per_sweep": run_ms,
                            "mixed_fp64_on_accept_ms_per_sweep": on_ms, "fp64_ms_per_sweep": fp64_ms,
                            "on_accept_over_mixed": on_ms / run_ms})
    method_rows = []
    for name, w in (("c2", I.named("c2")), ("c3", I.named("c3")), ("N=55 x 4096", chain55(4096)),
                    ("c5 chain 0 (N=2000 x 256)", I.subset(I.named("c5"), [0]))):
        s = pt.Simulation(w, precision="fp64")
        row = {"workload": name}
        for key, method in (("fp64_order", pt.PT_ENERGY_FP64_ORDER),
                            ("pair_per_thread", pt.PT_ENERGY_PAIR_PER_THREAD)):
            times = []
            for _ in range(3):
                e, b, ms = s.energy_method(method)
                times.append(ms)
            row[key + "_ms"] = min(times)
            row[key + "_max_bound"] = float(np.max(b))
        exact = s.energy()
        row["pair_per_thread_max_abs_diff"] = float(np.max(np.abs(e - exact)))
        row["pair_energies_per_s_fp64_order"] = 0.5 * sum(
            r * n * (n - 1) for n, r in zip(w.n_beads, w.n_slots)) / (row["fp64_order_ms"] / 1e3)
        row["pair_over_fp64_order_time"] = row["pair_per_thread_ms"] / row["fp64_order_ms"]
        s.close()
        method_rows.append(row)
    return {"ablations": "paper's alternative designs vs this library's, one MI355X, identical results "
                         "(the pair-per-thread energy: within its rigorous bound)",
            "sweeps": sweeps, "one_lane_per_replica_fp64_N55_edge0.02": lane_rows,
            "full_energy_every_sweep": energy_rows, "fp64_on_accept": accept_rows,
            "energy_kernels": method_rows}


def cpu_model():
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def dominant_kernel(run):
    """Name of the kernel that dominates the sweep time of a measured run: the
    persistent launch of the widest class, else its task flow, else the
    per-sweep kernel of the most expensive class."""
    b_, w_ = max(run["classes"], key=lambda c: c[0] * c[1])
    mode = run["class_mode"][(b_, w_)]
    if mode == 1:
        return f"k_run<{w_}, true>"
    if mode == 2:
        return f"k_flow<{b_}, {w_}, true>"
    return f"k_sweep<{b_}, {w_}, true>"


def roofline(w, run, steps, workload=None):
    """Algorithmic FP32 FLOP/s of the sweep launches (27 per pair interaction)
    over the average launch duration, against the FP32 vector peak."""
    avg_kernel_s = run["sweep_kernel_ms"] / 1e3 / run["launches"]
    flop_per_launch = FLOP_PER_PAIR * w.pair_interactions_per_sweep() * steps / run["launches"]
    achieved = flop_per_launch / avg_kernel_s
    kernel = dominant_kernel(run)
    waves_of_n = {int(m[0]): int(m[2]) for m in run["mapping"]}
    occupied = min(1024, sum(int(r) * waves_of_n[int(n)] for n, r in zip(w.n_beads, w.n_slots)))
    # A persistent or task-flow launch runs all the timed sweeps of its group
    # (one launch per group); a per-sweep launch one sweep.
    b_, w_ = max(run["classes"], key=lambda c: c[0] * c[1])
    per_launch = steps if run["class_mode"][(b_, w_)] in (1, 2) else steps / run["launches"]
    traffic = measured_traffic(workload, kernel, per_launch) if workload else None
    return {"bound": "alu", "kernel": kernel, "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": traffic,
            "traffic_unit": "bytes per launch (HBM read + write, rocprofv3 FETCH_SIZE/WRITE_SIZE x copy calibration)",
            "occupied_simds": occupied, "frac_of_occupied_simds": achieved / (PEAK_FP32 * occupied / 1024.0),
            "avg_launch_ms": avg_kernel_s * 1e3, "flop_per_launch": flop_per_launch}


def sub_record(name, steps, warmup, cpu_budget_s, with_cpu, cpu_chains=None):
    """One of the batched workloads, both precisions on the same input, with its
    own step counts (its first sweeps relax random-walk starts: the warm-up
    keeps most of that out of the timed steps)."""
    from paper_1107_3490_amd import inputs as I

    w = I.named(name)
    progress(f"{name}: mixed")
    mixed = run_gpu(w, "mixed", steps, warmup)
    progress(f"{name}: fp64")
    fp64 = run_gpu(w, "fp64", steps, warmup)
    pps = w.pair_interactions_per_sweep()
    rec = {"workload": f"{name}: {WORKLOADS[name]}", "steps": steps, "warmup": warmup,
           "pairs_per_step": pps, "slots": w.total_slots,
           "mixed": {"value": mixed["pairs"] / (mixed["event_total_ms"] / 1e3), "unit": "pair interactions/s",
                     "ms_per_step": mixed["event_total_ms"] / steps,
                     "replica_sweeps_per_s": steps * w.total_slots / (mixed["event_total_ms"] / 1e3),
                     "mapping_N_B_W": mixed["mapping"], "launches": mixed["launches"],
                     "schedule": "+".join(sorted({("per-sweep", "persistent", "task flow")[m]
                                                  for m in mixed["class_mode"].values()})),
                     "rescored_moves": mixed["rescored"], "moves": mixed["moves"],
                     "energy_resyncs": mixed["resyncs"], "exchange_fp64_recomputes": mixed["exch_recompute"],
                     "roofline": roofline(w, mixed, steps, name)},
           "fp64": {"value": fp64["pairs"] / (fp64["event_total_ms"] / 1e3), "unit": "pair interactions/s",
                    "ms_per_step": fp64["event_total_ms"] / steps, "mapping_N_B_W": fp64["mapping"],
                    "launches": fp64["launches"]}}
    rec["mixed_over_fp64"] = rec["mixed"]["value"] / rec["fp64"]["value"]
    if with_cpu:
        progress(f"{name}: CPU oracle")
        ws = I.subset(w, cpu_chains) if cpu_chains is not None else w
        cb = cpu_baseline(ws, budget_s=cpu_budget_s)
        if cpu_chains is not None:
            cb["sample"] = (f"extrapolated: chain(s) {list(cpu_chains)} of {w.n_chains} with all their slots "
                            f"({cb['sample']}); the oracle's cost is linear in pair interactions, so its "
                            "rate on the whole workload is this rate")
            cb["extrapolated"] = True
        rec["cpu_baseline"] = cb
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the sub-records of the other workloads (c3, c4, c5)")
    ap.add_argument("--schedule", type=int, default=0, choices=[0, 1, 2, 3],
                    help="0 auto, 1 one sweep launch per sweep, 2 persistent, 3 task flow")
    ap.add_argument("--no-tune", action="store_true", help="default mapping instead of the autotuner's")
    ap.add_argument("--mapping", default=None,
                    help="mapping per chain length instead of the autotuner's, e.g. "
                         "'13:0x11,30:0x11,55:0x11,100:0x21,200:0x14,500:0x24' (code 16 B + W)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy (scale for FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--paper-protocol", action="store_true",
                    help="the paper's benchmark: N = 55, edge 0.02, 4000 sweeps, exchange every 1000, "
                         "replica-count scan with speed-ups over one oracle core")
    ap.add_argument("--ablations", action="store_true",
                    help="the paper's alternative designs (one lane per replica, full energy every "
                         "sweep) timed beside this library's")
    args = ap.parse_args()
    if args.ablations:
        print(json.dumps(ablations()), flush=True)
        return
    if args.paper_protocol:
        print(json.dumps(paper_protocol()), flush=True)
        return
    if args.calibrate_copy:
        import torch
        n = 256 * 1024 * 1024 // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": n * 4, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): sharding chains and "
              "ladders over GPUs is designed but not built in this library.", file=sys.stderr)
        sys.exit(2)

    from paper_1107_3490_amd import inputs as I

    w = I.named(args.workload)
    by_n = None
    if args.mapping:
        by_n = {int(n): int(c, 0) for n, c in (x.split(":") for x in args.mapping.split(","))}
        missing = sorted(set(int(n) for n in w.n_beads) - set(by_n))
        if missing:
            print(f"--mapping has no code for chain length(s) {missing}", file=sys.stderr)
            sys.exit(2)
    progress(f"{args.workload}: mixed")
    mixed = run_gpu(w, "mixed", args.steps, args.warmup, args.schedule, not args.no_tune, by_n)
    progress(f"{args.workload}: fp64")
    fp64 = run_gpu(w, "fp64", args.steps, args.warmup, args.schedule, not args.no_tune, by_n)

    slots = w.total_slots
    value = mixed["pairs"] / (mixed["event_total_ms"] / 1e3)
    ms_per_step = mixed["event_total_ms"] / args.steps
    fp64_value = fp64["pairs"] / (fp64["event_total_ms"] / 1e3)
    fp64_sweep_s = fp64["sweep_kernel_ms"] / 1e3 / args.steps

    out = {
        "metric": "pair interactions/sec and sweeps/sec, mixed vs plain FP64 GPU",
        "value": value,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": MIXED_DTYPE,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}",
                   "slots": slots, "n_beads": sorted(set(w.n_beads)),
                   "pairs_per_step": w.pair_interactions_per_sweep(), "precision": "mixed",
                   "schedule": "+".join(sorted({("per-sweep", "persistent", "task flow")[m]
                                                for m in mixed["class_mode"].values()})),
                   "mapping_N_B_W": mixed["mapping"]},
        "repeat_segments": {"steps_each": max(1, args.steps // 5),
                            "ms_per_step": mixed["repeats_ms_per_step"],
                            "median_ms_per_step": float(np.median(mixed["repeats_ms_per_step"]))},
        "sweeps_per_s": args.steps / (mixed["event_total_ms"] / 1e3),
        "replica_sweeps_per_s": args.steps * slots / (mixed["event_total_ms"] / 1e3),
        "wall_s": mixed["wall_s"],
        "rescored_moves": mixed["rescored"],
        "energy_resyncs": mixed["resyncs"],
        "moves": mixed["moves"],
        "exchange_fp64_recomputes": mixed["exch_recompute"],
        "fp64_path": {
            "value": fp64_value,
            "unit": "pair interactions/s",
            "sweeps_per_s": args.steps / (fp64["event_total_ms"] / 1e3),
            "ms_per_step": fp64["event_total_ms"] / args.steps,
            "sweep_kernel_ms_per_step": fp64_sweep_s * 1e3,
            "mapping_N_B_W": fp64["mapping"],
            "fp64_flops_frac": FLOP_PER_PAIR * w.pair_interactions_per_sweep() / fp64_sweep_s / PEAK_FP64,
        },
        "mixed_over_fp64": value / fp64_value,
        "roofline": roofline(w, mixed, args.steps, args.workload),
    }
    # The mixed path with every accepted move also re-scored in the FP64 order:
    # same decisions, running energies within 1e-9 like the FP64 path's.
    from paper_1107_3490_amd import pt as _pt
    progress(f"{args.workload}: mixed, FP64 re-score of accepted moves")
    acc64 = run_gpu(w, "mixed", args.steps, args.warmup, args.schedule | _pt.PT_SCHED_FP64_ON_ACCEPT,
                    not args.no_tune, by_n)
    acc64_value = acc64["pairs"] / (acc64["event_total_ms"] / 1e3)
    out["mixed_fp64_on_accept"] = {"value": acc64_value, "unit": "pair interactions/s",
                                   "ms_per_step": acc64["event_total_ms"] / args.steps,
                                   "over_fp64": acc64_value / fp64_value,
                                   "mapping_N_B_W": acc64["mapping"]}
    out["incl_init_and_readback"] = with_transfers(w, args.steps)
    if not args.no_cpu:
        progress(f"{args.workload}: CPU oracle")
        out["cpu_baseline"] = cpu_baseline(w)
        # one core, the convention of the paper's speed-ups (context only)
        out["cpu_baseline_1core"] = cpu_baseline(w, budget_s=5.0, threads=1)
    if not args.no_batched and args.workload == "c2":
        # The batched workloads the throughput targets are stated for, on their
        # own step counts (see sub_record).
        out["workloads"] = {
            "c3": sub_record("c3", 200, 100, 10.0, not args.no_cpu),
            "c4": sub_record("c4", 500, 100, 10.0, not args.no_cpu),
            "c5": sub_record("c5", 30, 100, 10.0, not args.no_cpu, cpu_chains=[0]),
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
