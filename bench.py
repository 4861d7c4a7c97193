#!/usr/bin/env python3
"""Benchmark of the single-variable update sweep on one MI355X.

Default workload (the headline configuration): sparse Erdos-Renyi QUIO, N = 10,000 integer
variables in [-50, 50], mean degree 8, heat bath, automatic schedule, 2000 sweeps, 256 reads.
One step = one complete annealing run of all reads (random initial states, energy, every sweep,
final states and energies) = one kernel launch on device-resident inputs.

Prints ONE JSON line: metric/value (updates per second), roofline of the annealing kernel, and the
CPU oracle's rate on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(ROOT, "paper_2511_17245_amd", "csrc")
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# The heat bath's algorithmic FP64 work per weight w = exp(-beta * dE), as the method states it:
# one multiply, one exponential evaluated directly (the FP64 operations of the gfx950 exp sequence,
# FMA = 2 flops) and the additions of the cumulative sum.  The kernel's factored weights for
# linear variables execute far fewer (two exponentials per lane and one fused multiply-add per
# weight); the counter record gives the executed instructions.
FP64_FLOPS_PER_WEIGHT = 30.0
# VALU issue: a wave64 VALU instruction occupies one of the 4 SIMDs of a compute unit for 4 cycles
VALU_ISSUE_PEAK_G = 256 * 4 * 2.4 / 4   # 10^9 wave instructions/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="cfg2",
                    choices=["cfg1", "cfg2", "cfg2-closed", "cfg3-otm", "cfg3-metropolis", "cfg4",
                             "cfg5"])
    ap.add_argument("--requests", type=int, default=300, help="cfg5: requests in the stream")
    ap.add_argument("--load", type=float, default=0.8, help="cfg5: arrival rate / saturated rate")
    ap.add_argument("--plain-sample", type=int, default=48,
                    help="cfg4: problems timed with plain per-instance launches")
    ap.add_argument("--sweeps", type=int, default=0, help="override the number of sweeps")
    ap.add_argument("--reads", type=int, default=0, help="override the number of reads")
    ap.add_argument("--waves-per-replica", type=int, default=0,
                    help="wavefronts cooperating on one replica (0: automatic)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only copy a device buffer of this many MiB (counter calibration) and exit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--suite", action="store_true",
                    help="the paper's experiments (FC, ML, RI models at N = 100) instead of updates/s")
    ap.add_argument("--figures", default="",
                    help="the paper's Figs. 3-8 configurations at its sample counts: comma-separated "
                         "list of fig3,fig4,fig5,fig6,fig7,fig8 (or all)")
    ap.add_argument("--figures-md", default="", help="--figures: also write a markdown summary here")
    ap.add_argument("--ttt", action="store_true",
                    help="time to target energy instead of updates/s (cfg1, cfg2, cfg2-closed, cfg3-*)")
    ap.add_argument("--ttt-oracle-reads", type=int, default=0,
                    help="oracle reads behind the target energy and the CPU time (0: automatic)")
    ap.add_argument("--no-closed-form", action="store_true",
                    help="cfg2: skip timing the closed-form heat-bath draw beside the enumeration")
    ap.add_argument("--no-ttt", action="store_true",
                    help="cfg2: skip the time-to-target grid in the default line")
    ap.add_argument("--no-batch", action="store_true",
                    help="cfg2: skip the batched-versus-plain measurement in the default line")
    ap.add_argument("--lanes-per-update", type=int, default=0,
                    help="heat bath: 4 (quad kernel), 64 (one wavefront per update) or 0 (automatic)")
    ap.add_argument("--cpu-reads", type=int, default=16)
    ap.add_argument("--cpu-sweeps", type=int, default=0, help="0: the whole schedule")
    return ap.parse_args()


def workload(args):
    from paper_2511_17245_amd import inputs as I
    if args.config == "cfg1":
        w = I.cfg1_dense_quio()
    elif args.config in ("cfg2", "cfg2-closed"):
        w = I.cfg2_sparse_quio()
        if args.config == "cfg2-closed":
            # the same workload with the closed-form heat-bath draw (every variable is linear)
            w.rule = I.RULES["heat_bath_closed"]
            w.name = w.name.replace("heat bath", "heat bath (closed-form draw)")
    else:
        w = I.cfg3_huio(rule=args.config.split("-")[1])
    if args.sweeps:
        w.n_sweeps = args.sweeps
        w.beta = None if w.beta is None else w.beta[: args.sweeps]
    if args.reads:
        w.n_reads = args.reads
    return w


# the sources that define the device program and the data it reads: kernels, their argument
# layout, the instance packing and the launch choice (geometry and waves per replica)
KERNEL_SOURCES = ("sa_device.h", "sa_quad.h", "sa_quad_mo.h", "sa_kernels_quad.hip", "sa_kernels_quad_mo.hip",
                  "sa_kernels.hip", "sa_kernels_heat_bath.hip", "sa_kernels_heat_bath_closed.hip",
                  "sa_kernels_metropolis.hip", "sa_kernels_otm.hip", "sa_kernels_batch.hip",
                  "sa_kernels_batch16.hip", "sa_kernel_table.h", "sa_internal.h", "sa_host.cpp",
                  "sa_api.cpp")


def kernel_source_hash() -> str:
    """Hash of the kernel sources' code: HBM traffic measured with counters applies only to the
    kernels built from exactly this code.  Line comments and blank space are left out (no source
    holds "//" inside a string), so that editing a comment keeps the counter records."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(CSRC, name), "r", encoding="utf-8") as f:
            code = re.sub(r"//[^\n]*", "", f.read())
        code = "\n".join(line.strip() for line in code.splitlines() if line.strip())
        h.update(name.encode() + b"\0" + code.encode())
    return h.hexdigest()[:16]


def counter_record(workload_key):
    """The committed counter summary of a workload's kernel, or None when the kernels changed
    since it was taken (or none exists)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(workload_key)
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec


def measured_traffic(workload_key):
    """HBM bytes per launch from the committed counter summary (None as counter_record)."""
    rec = counter_record(workload_key)
    return None if rec is None else rec["hbm_bytes_per_launch"]


def copy_probe(mib):
    import torch
    a = torch.ones(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": mib << 20}), flush=True)


def host_cpu():
    """The host's CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable}


def cpu_baseline(w, beta, n_reads, n_sweeps, one_core_sweeps=0):
    """The oracle (paper's coefficient-cache mode), as it stands, on a bounded sample: all usable
    host threads over n_reads reads, and one thread over one read (the first one_core_sweeps
    sweeps of the schedule)."""
    import numpy as np
    import oracle
    P = oracle.Poly(w.problem)
    threads = oracle.default_threads()
    b = np.ascontiguousarray(beta[:n_sweeps])
    # the sample runs the first n_sweeps of the real schedule (by default all of it), so every
    # temperature phase is represented
    t0 = time.perf_counter()
    P.anneal(w.rule, b, n_reads, w.seed, w.instance_id, cache_mode=1, n_threads=threads)
    dt = time.perf_counter() - t0
    upd = n_reads * n_sweeps * w.problem.n_vars
    out = {"value": upd / dt, "unit": "updates/s", "cores": min(threads, n_reads), "kind": "oracle",
           "sample": f"{n_reads} reads x {'all' if n_sweeps == w.n_sweeps else 'first ' + str(n_sweeps) + ' of'} "
                     f"{w.n_sweeps} sweeps of the same workload "
                     f"({upd:.3g} updates, {dt:.1f} s, coefficient-cache mode, {min(threads, n_reads)} threads)"}
    out.update(host_cpu())
    if one_core_sweeps > 0:
        s1 = min(one_core_sweeps, w.n_sweeps)
        t0 = time.perf_counter()
        P.anneal(w.rule, np.ascontiguousarray(beta[:s1]), 1, w.seed, w.instance_id, cache_mode=1, n_threads=1)
        d1 = time.perf_counter() - t0
        u1 = s1 * w.problem.n_vars
        out["one_core"] = {"value": u1 / d1, "unit": "updates/s", "cores": 1,
                           "sample": f"1 read x first {s1} of {w.n_sweeps} sweeps ({u1:.3g} updates, {d1:.1f} s)"}
    return out


def stored_oracle_energies(name):
    """Final energies of every read that the oracle recorded for a full-size workload
    (tests/golden/full_size_<name>.txt, written by the oracle alone), or None."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"full_size_{name}.txt")
    if not os.path.exists(path):
        return None
    e = []
    with open(path) as f:
        for line in f:
            if line.startswith("#") or line.startswith("workload"):
                continue
            e.append(int(line.split()[1]))
    return np.array(e, np.int64)


def ttt_grid(plan, w, R, lanes, e_target, e_best):
    """GPU runs of all reads at 1/8 .. 2 times the sweeps (automatic schedule of each length): the
    time to target is the kernel time of the shortest run whose median final energy reaches
    e_target; TTS99 to e_best is t_run ln(0.01) / ln(1 - p_hit), minimised over the grid."""
    import numpy as np
    import torch
    from paper_2511_17245_amd import sa
    prob, S = w.problem, w.n_sweeps
    stream = torch.cuda.current_stream()
    z = torch.empty((R, prob.n_vars), dtype=torch.int32, device="cuda")
    e = torch.empty(R, dtype=torch.int64, device="cuda")
    grid = []
    for f in (0.125, 0.25, 0.5, 1.0, 2.0):
        Sg = max(2, int(round(f * S)))
        beta = sa.auto_schedule(prob, Sg)
        plan.run_device(Sg, R, w.seed, z, e, beta=beta, stream=stream.cuda_stream, instance_id=w.instance_id,
                        lanes_per_update=lanes)
        torch.cuda.synchronize()   # warm (also stages beta)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.run_device(Sg, R, w.seed, z, e, beta=beta, stream=stream.cuda_stream, instance_id=w.instance_id,
                        lanes_per_update=lanes)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        eh = e.cpu().numpy()
        p_hit = float(np.mean(eh <= e_best))
        tts99 = (ms / 1e3) * (math.log(0.01) / math.log(1.0 - p_hit)) if 0.0 < p_hit < 1.0 else \
            (ms / 1e3 if p_hit >= 1.0 else None)
        grid.append({"sweeps": Sg, "gpu_ms": ms, "median_energy": float(np.median(eh)), "min_energy": int(eh.min()),
                     "p_hit_best": p_hit, "tts99_s": tts99})
        print(f"[bench] ttt grid {Sg} sweeps: {ms:.1f} ms, median {np.median(eh):.0f}", file=sys.stderr, flush=True)
    hit = next((g for g in grid if g["median_energy"] <= e_target), None)
    tts = [g["tts99_s"] for g in grid if g["tts99_s"] is not None]
    return {"target_median_energy": e_target, "best_energy": e_best,
            "ttt_s": hit["gpu_ms"] / 1e3 if hit else None, "ttt_sweeps": hit["sweeps"] if hit else None,
            "tts99_best_s": min(tts) if tts else None, "grid": grid}


def bench_ttt(args):
    """Time to target energy (the paper's energy-versus-annealing-time protocol, Sec. 4.4): the
    target is the median final energy of the oracle over a seeded sample of reads at the
    configuration's sweep count; the GPU runs the full read count at sweep counts 1/8 .. 2 times
    that, and the time to target is the kernel time of the shortest run whose median final energy
    reaches the target.  The oracle's time for that run is measured on a sample of its reads and
    scaled to the full read count."""
    import numpy as np
    import torch
    import oracle
    from paper_2511_17245_amd import inputs as I
    from paper_2511_17245_amd import sa

    w = workload(args)
    prob, S, R = w.problem, w.n_sweeps, w.n_reads
    P = oracle.Poly(prob)
    threads = oracle.default_threads()

    def schedule(n_sweeps):
        if args.config == "cfg1":
            return I.cfg1_beta(n_sweeps)
        return P.schedule(n_sweeps)[0]

    n_or = args.ttt_oracle_reads
    if n_or <= 0:   # every read when the oracle finishes in about a minute, else a sample of 32
        n_or = R if R * S * prob.n_vars <= 3e9 else 32
    ids = np.sort(np.random.Generator(np.random.PCG64(77)).choice(R, size=min(n_or, R),
                                                                   replace=False)).astype(np.uint32)
    print(f"[bench] oracle target: {len(ids)} reads x {S} sweeps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    _, e_or = P.anneal_reads(w.rule, schedule(S), ids, w.seed, w.instance_id, cache_mode=1,
                             n_threads=threads)
    oracle_target_s = time.perf_counter() - t0
    e_tgt = float(np.median(e_or))
    e_best = int(e_or.min())

    plan = sa.Plan(prob, w.rule)
    stream = torch.cuda.current_stream()
    z = torch.empty((R, prob.n_vars), dtype=torch.int32, device="cuda")
    e = torch.empty(R, dtype=torch.int64, device="cuda")
    grid = []
    for f in (0.125, 0.25, 0.5, 1.0, 2.0):
        Sg = max(2, int(round(f * S)))
        beta = schedule(Sg)
        plan.run_device(Sg, R, w.seed, z, e, beta=beta, stream=stream.cuda_stream, instance_id=w.instance_id)
        torch.cuda.synchronize()   # warm (also stages beta)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.run_device(Sg, R, w.seed, z, e, beta=beta, stream=stream.cuda_stream, instance_id=w.instance_id)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        eh = e.cpu().numpy()
        p_hit = float(np.mean(eh <= e_best))
        tts99 = (ms / 1e3) * (math.log(0.01) / math.log(1.0 - p_hit)) if 0.0 < p_hit < 1.0 else \
            (ms / 1e3 if p_hit >= 1.0 else None)
        grid.append({"sweeps": Sg, "gpu_ms": ms, "median_energy": float(np.median(eh)),
                     "min_energy": int(eh.min()), "p_hit_best": p_hit, "tts99_s": tts99})
        print(f"[bench] ttt grid {Sg} sweeps: {ms:.1f} ms, median {np.median(eh):.0f}", file=sys.stderr,
              flush=True)
    plan.close()
    hit = next((g for g in grid if g["median_energy"] <= e_tgt), None)
    out_cpu = None
    if hit is not None and not args.no_cpu_baseline:
        n_cpu = int(len(ids))
        t0 = time.perf_counter()
        P.anneal(w.rule, schedule(hit["sweeps"]), n_cpu, w.seed, w.instance_id, cache_mode=1, n_threads=threads)
        dt = time.perf_counter() - t0
        out_cpu = {"value": dt * R / n_cpu, "unit": "s", "cores": threads, "kind": "oracle",
                   "sample": f"{n_cpu} of {R} reads at {hit['sweeps']} sweeps ({dt:.1f} s), scaled to {R} reads"}
    tts = [g["tts99_s"] for g in grid if g["tts99_s"] is not None]
    out = {
        "metric": "time-to-target energy at 1 GPU",
        "value": hit["gpu_ms"] / 1e3 if hit else None, "unit": "s", "n_gpus": 1, "higher_is_better": False,
        "dtype": "int64+f64", "data": "synthetic",
        "config": {"workload": w.name, "n_vars": prob.n_vars, "n_reads": R, "n_sweeps": S,
                   "rule": sa.RULE_NAMES[w.rule]},
        "target": {"median_energy": e_tgt, "best_energy": e_best, "oracle_reads": int(len(ids)),
                   "oracle_s": oracle_target_s},
        "grid": grid, "ttt_sweeps": hit["sweeps"] if hit else None,
        "tts99_best_s": min(tts) if tts else None,
        "cpu_baseline": out_cpu,
    }
    print(json.dumps(out), flush=True)


def bench_suite(args):
    """The paper's experiments (Sec. 4) on the GPU with its three models at N = 100 (integer-scaled
    fixtures, synthetic random-interaction realizations): annealing time against the range 2u+1
    and the degree p at 1000 sweeps and 100 reads (Figs. 1-2), energy against temperature within
    one anneal (Figs. 3-4), against the sweep count (Figs. 5-6) and against annealing time for wide
    ranges (Figs. 7-8).  The heat bath is the paper's: closed-form draws where the energy
    difference is linear, enumeration elsewhere.  Times are GPU kernel times of one launch that
    runs all reads at once."""
    import numpy as np
    import torch
    from paper_2511_17245_amd import inputs as I
    from paper_2511_17245_amd import sa

    stream = torch.cuda.current_stream()
    HB = sa.HEAT_BATH_CLOSED
    names = {sa.METROPOLIS: "metropolis", HB: "heat_bath", sa.OPT_METROPOLIS: "otm",
             sa.HEAT_BATH: "heat_bath_enumerated"}
    otm_enum_max = 64   # wider ranges take the forward-difference argmin (logarithmic in the range)

    def run(prob, rule, n_sweeps, n_reads=100, seed=2511, beta=None, reps=2):
        plan = sa.Plan(prob, rule)
        beta = sa.auto_schedule(prob, n_sweeps) if beta is None else beta
        z = torch.empty((n_reads, prob.n_vars), dtype=torch.int32, device="cuda")
        e = torch.empty(n_reads, dtype=torch.int64, device="cuda")
        best = None
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            plan.run_device(n_sweeps, n_reads, seed, z, e, beta=beta, stream=stream.cuda_stream,
                            otm_enum_max=otm_enum_max)
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            best = ms if best is None else min(best, ms)
        out = e.cpu().numpy()
        plan.close()
        return best, out

    res = {}
    # Figs. 1-2: time against 2u+1 (FC, p = 1, 2) and against p (FC u = 1; ML u = 10)
    t_range = []
    for p_ in (1, 2):
        for u in (1, 10, 100, 1000):
            prob = I.fully_connected(100, p_, u)
            rules = [sa.METROPOLIS, HB, sa.OPT_METROPOLIS] + ([sa.HEAT_BATH] if p_ == 1 else [])
            for rule in rules:
                ms, e = run(prob, rule, 1000)
                t_range.append({"model": "FC", "p": p_, "u": u, "range": 2 * u + 1, "rule": names[rule],
                                "ms": ms, "mean_energy_over_gs": float(np.mean(e)) /
                                (I.fully_connected_scale(p_, u) * 100 * 101 / 2)})
        print(f"[bench] suite: time vs range p={p_} done", file=sys.stderr, flush=True)
    res["time_vs_range"] = t_range
    t_p = []
    for p_ in (1, 2, 3, 4, 6, 8):
        prob = I.fully_connected(100, p_, 1)
        for rule in [sa.METROPOLIS, HB] + ([sa.OPT_METROPOLIS] if p_ <= 4 else []):
            ms, _ = run(prob, rule, 1000)
            t_p.append({"model": "FC", "u": 1, "p": p_, "rule": names[rule], "ms": ms})
    for p_ in (2, 3, 4, 6, 8, 10):
        prob = I.multilinear(100, p_, 10)
        for rule in (sa.METROPOLIS, HB, sa.OPT_METROPOLIS):
            ms, _ = run(prob, rule, 1000)
            t_p.append({"model": "ML", "u": 10, "p": p_, "rule": names[rule], "ms": ms})
    res["time_vs_p"] = t_p
    print("[bench] suite: time vs p done", file=sys.stderr, flush=True)

    # Figs. 3-4: energy against temperature inside one 1000-sweep anneal (chunks of 50 sweeps)
    e_T = []
    for label, prob, gs in (("FC p=2 u=10", I.fully_connected(100, 2, 10), 100 * 100 * 101 / 2),
                            ("ML p=3 u=10", I.multilinear(100, 3, 10), 100 * 1000)):
        for rule in (sa.METROPOLIS, HB, sa.OPT_METROPOLIS):
            plan = sa.Plan(prob, rule)
            S = 1000
            beta = sa.auto_schedule(prob, S)
            z = torch.empty((100, prob.n_vars), dtype=torch.int32, device="cuda")
            e = torch.empty(100, dtype=torch.int64, device="cuda")
            pts = []
            for s0 in range(0, S, 50):
                plan.run_device(S, 100, 7, z, e, beta=beta, stream=stream.cuda_stream, sweep_begin=s0,
                                sweep_end=s0 + 50, init_states=None if s0 == 0 else z)
                torch.cuda.synchronize()
                pts.append({"T": 1.0 / float(beta[s0 + 49]), "mean_energy_over_gs":
                            float(e.float().mean().item()) / gs})
            plan.close()
            e_T.append({"model": label, "rule": names[rule], "points": pts})
    res["energy_vs_temperature"] = e_T
    print("[bench] suite: energy vs temperature done", file=sys.stderr, flush=True)

    # Figs. 5-8: energy against sweeps and annealing time
    e_s = []
    rng = np.random.Generator(np.random.PCG64(2511))
    models = [("FC p=2 u=10", I.fully_connected(100, 2, 10), 100 * 100 * 101 / 2),
              ("ML p=3 u=10", I.multilinear(100, 3, 10), 100 * 1000)]
    for u in (10, 1000):
        for r_ in range(3):
            models.append((f"RI p=2 u={u} #{r_}", I.random_interaction(100, 2, u, 1000, rng), None))
    for label, prob, gs in models:
        rows = []
        for S in (10, 30, 100, 300, 1000):
            for rule in (sa.METROPOLIS, HB, sa.OPT_METROPOLIS):
                ms, e = run(prob, rule, S)
                rows.append({"sweeps": S, "rule": names[rule], "ms": ms, "mean_energy": float(np.mean(e)),
                             "min_energy": int(e.min()), "p_ground": None if gs is None else
                             float(np.mean(e <= -gs))})
        best = min(r["min_energy"] for r in rows)
        for r in rows:
            r["mean_energy_over_best"] = r["mean_energy"] / abs(best)
        e_s.append({"model": label, "ground_energy": None if gs is None else -gs, "rows": rows})
        print(f"[bench] suite: energy vs sweeps {label} done", file=sys.stderr, flush=True)
    res["energy_vs_sweeps_and_time"] = e_s

    # the paper's qualitative statements, evaluated on these numbers
    def t(model, p_, u, rule):
        return next(r["ms"] for r in t_range if r["p"] == p_ and r["u"] == u and r["rule"] == rule)
    checks = {
        "p1_time_flat_in_range": {r: t("FC", 1, 1000, r) / t("FC", 1, 1, r)
                                  for r in ("metropolis", "heat_bath", "otm")},
        "p1_enumerated_heat_bath_growth": t("FC", 1, 1000, "heat_bath_enumerated") / t("FC", 1, 1, "heat_bath_enumerated"),
        "p2_heat_bath_growth_u1000_over_u10": t("FC", 2, 1000, "heat_bath") / t("FC", 2, 10, "heat_bath"),
        "p2_metropolis_otm_growth_u1000_over_u10": {r: t("FC", 2, 1000, r) / t("FC", 2, 10, r)
                                                   for r in ("metropolis", "otm")},
        "ml_time_ratio_p10_over_p2": {r: next(x["ms"] for x in t_p if x["model"] == "ML" and x["p"] == 10 and x["rule"] == r)
                                      / next(x["ms"] for x in t_p if x["model"] == "ML" and x["p"] == 2 and x["rule"] == r)
                                      for r in ("metropolis", "heat_bath", "otm")},
    }
    wide = [m for m in e_s if m["model"].startswith("RI p=2 u=1000")]
    short = {r: float(np.mean([next(x["mean_energy_over_best"] for x in m["rows"] if x["sweeps"] == 10 and x["rule"] == r)
                               for m in wide])) for r in ("metropolis", "heat_bath", "otm")}
    checks["ri_wide_mean_energy_over_best_at_10_sweeps"] = short
    out = {"metric": "paper experiment suite (Sec. 4) on 1 GPU", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "FC / ML / RI models, N = 100, 100 reads", "otm_enum_max": otm_enum_max},
           "checks": checks, "results": res}
    print(json.dumps(out), flush=True)
    if args.figures_md:
        write_suite_md(out, args.figures_md)


def write_suite_md(out, path):
    """A short text summary of a --suite run: its command, the checks, and the timing tables of
    Figs. 1 and 2."""
    res = out["results"]
    lines = ["# Paper experiment suite (Sec. 4, Figs. 1-2): annealing time against range and degree, N = 100",
             "", "Command: `python " + " ".join(sys.argv) + "`", "",
             "1000 sweeps, 100 reads, automatic schedule; times are GPU kernel times of the launch that runs",
             "all reads (best of two).", "", "## Checks", ""]
    for k, v in out["checks"].items():
        lines.append(f"- `{k}`: {json.dumps(v)}")
    lines += ["", "## Time against the range 2u+1 (FC)", "", "| p | u | rule | ms | mean energy / ground state |",
              "|---|---|---|---|---|"]
    lines += [f"| {r['p']} | {r['u']} | {r['rule']} | {r['ms']:.2f} | {r['mean_energy_over_gs']:.4f} |"
              for r in res["time_vs_range"]]
    lines += ["", "## Time against the degree p (FC u = 1, ML u = 10)", "", "| model | p | rule | ms |", "|---|---|---|---|"]
    lines += [f"| {r['model']} | {r['p']} | {r['rule']} | {r['ms']:.2f} |" for r in res["time_vs_p"]]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")

def bench_figures(args):
    """The configurations of the paper's Figs. 3-8 (Secs. 4.2-4.4) at N = 100 and its sample
    counts: energy against temperature inside one anneal (Figs. 3, 4), against the number of sweeps
    (Figs. 5, 6) and against annealing time (Figs. 7, 8), for Metropolis, the paper's heat bath
    (closed-form draws where dE is linear, enumeration of the range elsewhere) and OTM, each with
    the automatic schedule of Sec. 3.4.  Random-interaction realizations are seeded synthetic
    stand-ins (the paper's are not published): 100 realizations x 100 reads run as one batched
    launch.  Times are GPU kernel times of the launch that runs every read of a point.  Each
    figure's qualitative statement is evaluated on the numbers ("checks")."""
    import numpy as np
    import torch
    from paper_2511_17245_amd import inputs as I
    from paper_2511_17245_amd import sa

    allf = [f"fig{i}" for i in range(3, 9)]
    want = set(allf) if args.figures == "all" else set(args.figures.split(","))
    bad = want - set(allf)
    if bad:
        raise SystemExit(f"unknown figures {sorted(bad)}")
    stream = torch.cuda.Stream()   # plans and batches run here, and the timing events are recorded here
    RULES = [(sa.METROPOLIS, "metropolis"), (sa.HEAT_BATH_CLOSED, "heat_bath"), (sa.OPT_METROPOLIS, "otm")]
    NAMES = [name for _, name in RULES]
    otm_enum_max = 64
    N, SEED = 100, 2511

    def progress(*a):
        print("[figures]", *a, file=sys.stderr, flush=True)

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    def anneal(prob, rule, S, R, cuts):
        """One S-sweep anneal of R reads, stopped after each sweep count in `cuts` (the run resumes
        from the device state, which equals one uninterrupted run): the mean energy and the
        temperature at each cut, the summed kernel time and the final energies."""
        plan = sa.Plan(prob, rule)
        beta = sa.auto_schedule(prob, S)
        z = torch.empty((R, prob.n_vars), dtype=torch.int32, device="cuda")
        e = torch.empty(R, dtype=torch.int64, device="cuda")
        pts, s0, ms = [], 0, 0.0
        torch.cuda.synchronize()
        for s1 in cuts:
            ms += timed(lambda: plan.run_device(S, R, SEED, z, e, beta=beta, stream=stream.cuda_stream,  # noqa: B023
                                                sweep_begin=s0, sweep_end=s1, init_states=None if s0 == 0 else z,
                                                otm_enum_max=otm_enum_max))
            pts.append({"sweep": s1, "T": 1.0 / float(beta[s1 - 1]), "mean_energy": float(e.double().mean().item())})
            s0 = s1
            if S >= 100000:
                progress(f"{prob.name} {sa.RULE_NAMES[rule]} S={S}: sweep {s1}")
        out = e.cpu().numpy()
        plan.close()
        return {"curve": pts, "ms": ms, "e": out}

    def batch(probs, rule, S, cut=None, R=100):
        """Every realization with R reads in one batched launch of the S-sweep schedule, or of its
        first `cut` sweeps (the state of the S-sweep anneal after `cut` sweeps): kernel time, mean
        energy over all reads, mean over realizations of the lowest energy, and the schedule's
        temperature at the last sweep (mean over realizations)."""
        n = S if cut is None else cut
        betas = [sa.auto_schedule(pr, S)[:n].copy() for pr in probs]
        items = [I.Workload(pr, rule, n, R, SEED, i, b, pr.name) for i, (pr, b) in enumerate(zip(probs, betas))]
        b = sa.Batch(items, use_graph=False, stream=stream.cuda_stream)
        if n < 1000:   # an untimed run first where launch costs are not negligible
            b.run()
            b.wait()
        ms = timed(b.run)
        res = b.results()
        b.close()
        return {"ms": ms, "mean_energy": float(np.mean([r[1].mean() for r in res])),
                "mean_min_energy": float(np.mean([r[1].min() for r in res])),
                "T": float(np.mean([1.0 / bb[-1] for bb in betas]))}

    def ri_set(p_, u, seed):
        rng = np.random.Generator(np.random.PCG64(seed))
        return [I.random_interaction(N, p_, u, 1000, rng, name=f"ri_p{p_}_u{u}_{i}") for i in range(100)]

    def at(rows, S, rule):
        return next(r["mean_energy"] for r in rows if r["sweeps"] == S and r["rule"] == rule)

    def energy_at_time(rows, rule, t):
        """Mean energy of `rule` at time t, interpolated linearly in log time between its points."""
        pts = sorted((r["ms"], r["mean_energy"]) for r in rows if r["rule"] == rule)
        if t <= pts[0][0]:
            return pts[0][1]
        for (t0, e0), (t1, e1) in zip(pts, pts[1:]):
            if t <= t1:
                f = (np.log(t) - np.log(t0)) / (np.log(t1) - np.log(t0))
                return float(e0 + f * (e1 - e0))
        return pts[-1][1]

    def by_time(rows):
        """The rule with the lowest interpolated mean energy at three common time budgets: the
        largest of the rules' shortest times, the smallest of their longest times, and the
        geometric mean of the two."""
        lo = max(min(r["ms"] for r in rows if r["rule"] == n) for n in NAMES)
        hi = min(max(r["ms"] for r in rows if r["rule"] == n) for n in NAMES)
        out = {}
        for label, t in (("short", lo), ("middle", float(np.sqrt(lo * hi))), ("long", hi)):
            es = {n: energy_at_time(rows, n, t) for n in NAMES}
            out[label] = {"ms": t, "lowest": min(es, key=es.get), "mean_energy": es}
        return out

    figs, checks, cache = {}, {}, {}

    def ml_anneal(p_, u, rule, name, S, R, cuts):
        # the 10^6-sweep anneals of Fig. 4 are the 10^6-sweep points of Figs. 6 and 8
        key = (p_, u, name, S, R, tuple(cuts))
        if key not in cache:
            cache[key] = anneal(I.multilinear(N, p_, u), rule, S, R, cuts)
        return cache[key]

    def fifths(S):
        return sorted(set([max(1, S // 20), max(1, S // 10)] + [S * i // 5 for i in range(1, 6)]))

    # ---- Fig. 3: FC p=2 u=100 (1000 reads) and RI p=4 u=100 (100 realizations x 100 reads) ----
    if "fig3" in want:
        fc = I.fully_connected(N, 2, 100)
        scale = I.fully_connected_scale(2, 100)
        ri = ri_set(4, 100, 3)
        out = {"fc_p2_u100": {}, "ri_p4_u100": {}}
        for S in (100, 1000, 10000):
            cuts = sorted(set(int(round(S * (i + 1) / 20)) for i in range(20)))
            for rule, name in RULES:
                r = anneal(fc, rule, S, 1000, cuts)
                out["fc_p2_u100"][f"{name}/{S}"] = [dict(p, mean_energy=p["mean_energy"] / scale) for p in r["curve"]]
                out["ri_p4_u100"][f"{name}/{S}"] = [dict(batch(ri, rule, S, c), sweep=c) for c in fifths(S)]
                progress(f"fig3 {name} {S} sweeps done")
        figs["fig3"] = out
        fc_c, ri_c = out["fc_p2_u100"], out["ri_p4_u100"]

        def below_at_equal_T(curves, a, b, S):
            # the share of cuts after the first tenth of the schedule where rule a is at or below b
            A, B = curves[f"{a}/{S}"], curves[f"{b}/{S}"]
            pairs = [(x["mean_energy"], y["mean_energy"]) for x, y in zip(A, B) if x["sweep"] > S // 10]
            return float(np.mean([x <= y for x, y in pairs]))

        def last_fifth_drop(c):
            # decrease of the mean energy over the last fifth of the schedule, relative to the final value
            e_end = c[-1]["mean_energy"]
            e_4 = next(x["mean_energy"] for x in c if x["sweep"] >= c[-1]["sweep"] * 4 // 5)
            return (e_4 - e_end) / abs(e_end)

        for model, curves in (("fc", fc_c), ("ri", ri_c)):
            checks[f"fig3_{model}_heat_bath_at_or_below_metropolis_at_equal_T"] = {
                S: below_at_equal_T(curves, "heat_bath", "metropolis", S) for S in (100, 1000, 10000)}
            checks[f"fig3_{model}_otm_at_or_below_metropolis_at_equal_T"] = {
                S: below_at_equal_T(curves, "otm", "metropolis", S) for S in (100, 1000, 10000)}
            checks[f"fig3_{model}_drop_over_last_fifth"] = {k: last_fifth_drop(v) for k, v in curves.items()}
            drops = checks[f"fig3_{model}_drop_over_last_fifth"]
            checks[f"fig3_{model}_metropolis_100_still_falling_most_at_the_end"] = drops["metropolis/100"] == max(drops.values())
            gaps = {S: abs(curves[f"metropolis/{S}"][-1]["mean_energy"] - curves[f"heat_bath/{S}"][-1]["mean_energy"]) /
                    abs(curves[f"heat_bath/{S}"][-1]["mean_energy"]) for S in (100, 1000, 10000)}
            checks[f"fig3_{model}_final_metropolis_heat_bath_gap"] = gaps
            checks[f"fig3_{model}_gap_shrinks_with_sweeps"] = gaps[100] > gaps[1000] > gaps[10000]
        checks["fig3_fc_final_mean_energy_over_ground_state_-5050"] = {
            k: v[-1]["mean_energy"] / -5050.0 for k, v in fc_c.items()}
        checks["fig3_ri_otm_final_above_heat_bath"] = {
            S: ri_c[f"otm/{S}"][-1]["mean_energy"] > ri_c[f"heat_bath/{S}"][-1]["mean_energy"] for S in (100, 1000, 10000)}

    # ---- Fig. 4 (and the 10^6-sweep points of Figs. 6b, 8b): ML p=30 u=1, 1000 reads ----
    if "fig4" in want:
        out = {}
        for S in (100, 10000, 1000000):
            cuts = sorted(set(int(round(S * (i + 1) / 20)) for i in range(20)))
            for rule, name in RULES:
                out[f"{name}/{S}"] = ml_anneal(30, 1, rule, name, S, 1000, cuts)["curve"]
            progress(f"fig4 {S} sweeps done")
        figs["fig4"] = {"ml_p30_u1": out, "reads": 1000}
        drop = {k: (v[-5]["mean_energy"] - v[-1]["mean_energy"]) / N for k, v in out.items()}
        checks["fig4_drop_over_last_fifth_per_variable"] = drop
        checks["fig4_still_falling_at_10^2_and_10^4_flatter_at_10^6"] = {
            name: drop[f"{name}/100"] > drop[f"{name}/1000000"] and drop[f"{name}/10000"] > drop[f"{name}/1000000"]
            for name in NAMES}
        checks["fig4_final_mean_energy_above_ground_state_-100"] = {
            k: v[-1]["mean_energy"] for k, v in out.items() if k.endswith("/1000000")}

    # ---- Figs. 5 and 7: RI batches at fixed sweep counts ----
    ri_models = []
    if "fig5" in want:
        ri_models += [(2, 1), (2, 1000)]
    if "fig7" in want:
        ri_models += [(2, 1), (2, 100), (4, 1), (4, 100)]
    ri_rows = {}
    for p_, u in dict.fromkeys(ri_models):
        ri = ri_set(p_, u, 5 + p_ + u)
        rows = []
        for S in (10, 30, 100, 300, 1000, 3000):
            for rule, name in RULES:
                r = batch(ri, rule, S)
                rows.append({"sweeps": S, "rule": name, "ms": r["ms"], "mean_energy": r["mean_energy"],
                             "mean_min_energy": r["mean_min_energy"]})
            progress(f"RI p={p_} u={u} {S} sweeps done")
        ri_rows[f"ri_p{p_}_u{u}"] = rows
    if ri_rows:
        figs["fig5_fig7"] = ri_rows
    if "fig5" in want:
        a, b = ri_rows["ri_p2_u1"], ri_rows["ri_p2_u1000"]

        def spread(rows, S):
            es = [at(rows, S, n) for n in NAMES]
            return (max(es) - min(es)) / abs(min(es))
        checks["fig5a_u1_relative_spread_of_the_rules"] = {S: spread(a, S) for S in (10, 100, 1000, 3000)}
        checks["fig5b_u1000_relative_spread_of_the_rules"] = {S: spread(b, S) for S in (10, 100, 1000, 3000)}
        checks["fig5b_u1000_metropolis_highest"] = {S: at(b, S, "metropolis") == max(at(b, S, n) for n in NAMES)
                                                    for S in (10, 30, 100, 300, 1000, 3000)}
        checks["fig5b_u1000_heat_bath_below_otm"] = {S: at(b, S, "heat_bath") < at(b, S, "otm")
                                                     for S in (10, 30, 100, 300, 1000, 3000)}
    if "fig7" in want:
        for key in ("ri_p2_u1", "ri_p2_u100", "ri_p4_u1", "ri_p4_u100"):
            rows = ri_rows[key]
            checks[f"fig7_{key}_lowest_rule_at_equal_time"] = by_time(rows)
            checks[f"fig7_{key}_time_per_sweep_heat_bath_over_metropolis"] = float(np.mean(
                [next(r["ms"] for r in rows if r["sweeps"] == S and r["rule"] == "heat_bath") /
                 next(r["ms"] for r in rows if r["sweeps"] == S and r["rule"] == "metropolis") for S in (1000, 3000)]))

    # ---- Figs. 6 and 8: ML p=2 u=10^6 and ML p=30 u=1 at fixed sweep counts, 1000 reads ----
    if "fig6" in want or "fig8" in want:
        out = {}
        for label, p_, u, grid in (("ml_p2_u1e6", 2, 10 ** 6, (10, 30, 100, 300, 1000, 3000, 10000)),
                                   ("ml_p30_u1", 30, 1, (10, 100, 1000, 10000, 100000, 1000000))):
            rows = []
            for S in grid:
                for rule, name in RULES:
                    cuts = sorted(set(int(round(S * (i + 1) / 20)) for i in range(20))) if S >= 100000 else [S]
                    r = ml_anneal(p_, u, rule, name, S, 1000, cuts)
                    e = r["e"] / float(u ** p_)
                    rows.append({"sweeps": S, "rule": name, "ms": r["ms"], "mean_energy": float(e.mean()),
                                 "stderr": float(e.std(ddof=1) / np.sqrt(e.size)), "min_energy": float(e.min()),
                                 "p_ground": float(np.mean(e <= -N))})
                progress(f"{label} {S} sweeps done")
            out[label] = rows
        figs["fig6_fig8"] = out
        a, b = out["ml_p2_u1e6"], out["ml_p30_u1"]
        checks["fig6a_ml_p2_u1e6_metropolis_highest"] = {S: at(a, S, "metropolis") == max(at(a, S, n) for n in NAMES)
                                                         for S in (10, 30, 100, 300, 1000, 3000, 10000)}
        hb = [at(a, S, "heat_bath") for S in (10, 30, 100, 300, 1000, 3000, 10000)]
        checks["fig6a_ml_p2_u1e6_heat_bath_not_monotone_or_above_otm_at_small_sweeps"] = {
            "heat_bath_rises_somewhere": any(y > x for x, y in zip(hb, hb[1:])),
            "heat_bath_above_otm": {S: at(a, S, "heat_bath") > at(a, S, "otm") for S in (10, 30, 100)}}
        checks["fig6b_ml_p30_no_rule_reaches_ground_state_on_average_at_10^6"] = all(
            r["mean_energy"] > -N for r in b if r["sweeps"] == 1000000)
        checks["fig6b_ml_p30_lowest_rule_by_sweeps"] = {S: min(NAMES, key=lambda n: at(b, S, n))
                                                        for S in (10, 100, 1000, 10000, 100000, 1000000)}
        checks["fig8a_ml_p2_u1e6_lowest_rule_at_equal_time"] = by_time(a)
        checks["fig8b_ml_p30_lowest_rule_at_equal_time"] = by_time(b)

    out = {"metric": "paper figures 3-8 configurations on 1 GPU", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "FC / ML / RI models, N = 100", "otm_enum_max": otm_enum_max,
                      "figures": sorted(want)},
           "checks": checks, "figures": figs}
    print(json.dumps(out), flush=True)
    if args.figures_md:
        write_figures_md(out, args.figures_md)


def write_figures_md(out, path):
    """A short text summary of a --figures run: its command, the checks, and one table per
    sweep-count or time series."""
    lines = ["# Paper figure configurations (Secs. 4.2-4.4), N = 100, one MI355X", "",
             "Command: `python " + " ".join(sys.argv) + "`", "",
             "Energies of FC are divided by u^2 (ground state -5050), of ML by u^p (ground state -100);",
             "RI energies are the integer-coefficient stand-ins' own. Times are kernel times of the launch",
             "that runs every read of a point (1000 reads, or 100 realizations x 100 reads).", "",
             "## Checks", ""]
    for k, v in out["checks"].items():
        lines.append(f"- `{k}`: {json.dumps(v)}")
    figs = out["figures"]
    for key in ("fig5_fig7", "fig6_fig8"):
        for label, rows in figs.get(key, {}).items():
            lines += ["", f"## {key} {label}", "", "| sweeps | rule | ms | mean energy |", "|---|---|---|---|"]
            lines += [f"| {r['sweeps']} | {r['rule']} | {r['ms']:.2f} | {r['mean_energy']:.6g} |" for r in rows]
    for key in ("fig3", "fig4"):
        if key not in figs:
            continue
        groups = figs[key] if key == "fig3" else {"ml_p30_u1": figs[key]["ml_p30_u1"]}
        for label, curves in groups.items():
            lines += ["", f"## {key} {label}: mean energy at the cuts of each anneal", "",
                      "| rule/sweeps | (sweep, T, mean energy) at the first, middle and last cut |", "|---|---|"]
            for k, c in curves.items():
                sel = [c[0], c[len(c) // 2], c[-1]]
                lines.append(f"| {k} | " + "; ".join(f"({p['sweep']}, {p['T']:.4g}, {p['mean_energy']:.6g})"
                                                     for p in sel) + " |")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def batched_vs_plain(steps, warmup, plain_sample, sweeps=0):
    """512 problems of uneven size, width, order and rule in one persistent (graph-replayed,
    autotuned) launch, against plain per-instance launches of a seeded sample of the same problems
    (one wavefront per update: the update code the batch runs, so the outputs must be identical)."""
    import numpy as np
    import torch
    from paper_2511_17245_amd import inputs as I
    from paper_2511_17245_amd import sa

    items = I.cfg4_batch()
    if sweeps:
        for w in items:
            w.n_sweeps = sweeps
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        batch = sa.Batch(items, autotune=True, use_graph=True, stream=stream.cuda_stream)
        create_s = time.perf_counter() - t0
        info = batch.info()
        for _ in range(warmup):
            batch.run()
        batch.wait()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for i in range(steps):
            batch.run()
            print(f"[bench] queued batch {i + 1}/{steps}", file=sys.stderr, flush=True)
        stop.record(stream)
        stream.synchronize()
        ms = start.elapsed_time(stop) / steps
        batched = batch.results()
        value = info["total_updates"] / (ms / 1e3)

        # plain launches, one problem at a time, on a seeded sample
        rng = np.random.Generator(np.random.PCG64(4242))
        sample = np.sort(rng.choice(len(items), size=min(plain_sample, len(items)), replace=False))
        plain_ms, plain_upd, same = 0.0, 0, True
        for i in sample:
            w = items[i]
            plan = sa.Plan(w.problem, w.rule)
            z = torch.empty((w.n_reads, w.problem.n_vars), dtype=torch.int32, device="cuda")
            e = torch.empty(w.n_reads, dtype=torch.int64, device="cuda")
            beta = w.beta if w.beta is not None else sa.auto_schedule(w.problem, w.n_sweeps)
            plan.run_device(w.n_sweeps, w.n_reads, w.seed, z, e, beta=beta, stream=stream.cuda_stream,
                            instance_id=w.instance_id, lanes_per_update=64)   # stages beta; not timed
            stream.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            plan.run_device(w.n_sweeps, w.n_reads, w.seed, z, e, beta=beta, stream=stream.cuda_stream,
                            instance_id=w.instance_id, lanes_per_update=64)
            b.record(stream)
            stream.synchronize()
            plain_ms += a.elapsed_time(b)
            plain_upd += w.n_reads * w.n_sweeps * w.problem.n_vars
            same = same and np.array_equal(z.cpu().numpy(), batched[i][0]) and \
                np.array_equal(e.cpu().numpy(), batched[i][1])
            plan.close()
        plain = plain_upd / (plain_ms / 1e3)
        batch.close()
    return {"value": value, "unit": "updates/s", "ms_per_step": ms, "steps": steps,
            "workload": "512 mixed QUIO/HUIO problems, N 50-5000, widths 2-1000, 32 reads, "
                        f"{sweeps or 1000} sweeps, one persistent graph-replayed launch",
            "batch": info, "create_s": create_s,
            "plain": {"value": plain, "unit": "updates/s", "sample_problems": int(len(sample)),
                      "sample_ms": plain_ms, "identical_outputs": bool(same)},
            "batched_over_plain": value / plain}


def bench_batch(args):
    r = batched_vs_plain(args.steps, args.warmup, args.plain_sample, args.sweeps)
    out = {
        "metric": "single-variable updates/sec at 1 GPU (batched form)",
        "value": r["value"], "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64+f64", "data": "synthetic",
        "config": {"workload": r["workload"], "batch": r["batch"], "create_s": r["create_s"]},
        "plain": r["plain"],
        "batched_over_plain": r["batched_over_plain"],
    }
    print(json.dumps(out), flush=True)


def bench_serving(args):
    """Poisson stream of requests to the continuous-batching server: p50/p99 latency and updates/s
    at a load below saturation, after a saturation pass that measures the request rate."""
    import threading
    import numpy as np
    import torch
    from paper_2511_17245_amd import inputs as I
    from paper_2511_17245_amd import sa

    n = args.requests
    t0 = time.perf_counter()
    reqs = [I.cfg5_request(i) for i in range(n)]
    gen_s = time.perf_counter() - t0
    kinds = sum(1 for w in reqs if w.rule == sa.HEAT_BATH)
    print(f"[bench] generated {n} requests ({kinds} dense heat-bath) in {gen_s:.1f}s", file=sys.stderr, flush=True)

    def stream(server, items, arrivals):
        tickets = [None] * len(items)

        def client():
            start = time.perf_counter()
            for i, w in enumerate(items):
                delay = arrivals[i] - (time.perf_counter() - start)
                if delay > 0:
                    time.sleep(delay)
                tickets[i] = server.submit(w)
                if (i + 1) % 25 == 0:
                    print(f"[bench] submitted {i + 1}/{len(items)}: {server.stats()}", file=sys.stderr, flush=True)

        th = threading.Thread(target=client)
        th.start()
        th.join()
        tim = []
        for k, t in enumerate(tickets):
            tim.append(server.wait(t))
            if (k + 1) % 25 == 0:
                print(f"[bench] completed {k + 1}/{len(items)}", file=sys.stderr, flush=True)
        return tickets, tim

    # saturation: everything submitted at once
    m = min(n, max(60, n // 5))
    srv = sa.Server(chunk_sweeps=50)
    _, tim = stream(srv, reqs[:m], np.zeros(m))
    span = max(t["t_done"] for t in tim) - min(t["t_submit"] for t in tim)
    sat_rate = m / span
    srv.close()
    print(f"[bench] saturated: {m} requests in {span:.1f}s = {sat_rate:.2f} req/s", file=sys.stderr, flush=True)

    rate = args.load * sat_rate
    arrivals = I.cfg5_arrivals(n, rate)
    srv = sa.Server(chunk_sweeps=50)
    tickets, tim = stream(srv, reqs, arrivals)
    stats = srv.stats()
    ok = [t for t in tim if t["status"] == sa.OK]
    lat = np.array([t["t_done"] - t["t_submit"] for t in ok])
    span = max(t["t_done"] for t in ok) - min(t["t_submit"] for t in ok)
    upd = float(sum(t["updates"] for t in ok))
    # where the time goes, per request kind: waiting (preparation and admission) and running
    by_kind = {}
    for kind, sel in (("huio", lambda w: w.rule != sa.HEAT_BATH), ("dense_heat_bath", lambda w: w.rule == sa.HEAT_BATH)):
        idx = [i for i, w in enumerate(reqs) if sel(w) and tim[i]["status"] == sa.OK]
        if not idx:
            continue
        wait = np.array([tim[i]["t_admit"] - tim[i]["t_submit"] for i in idx])
        run = np.array([tim[i]["t_done"] - tim[i]["t_admit"] for i in idx])
        tot = wait + run
        by_kind[kind] = {"count": len(idx), "p50": float(np.percentile(tot, 50)), "p99": float(np.percentile(tot, 99)),
                         "wait_p50": float(np.percentile(wait, 50)), "wait_p99": float(np.percentile(wait, 99)),
                         "run_p50": float(np.percentile(run, 50)), "run_p99": float(np.percentile(run, 99))}
    # alone-versus-mix identity on a sample of requests
    rng = np.random.Generator(np.random.PCG64(555))
    sample = rng.choice(n, size=min(12, n), replace=False)
    same = True
    for i in sample:
        w = reqs[i]
        plan = sa.Plan(w.problem, w.rule)
        z = torch.empty((w.n_reads, w.problem.n_vars), dtype=torch.int32, device="cuda")
        e = torch.empty(w.n_reads, dtype=torch.int64, device="cuda")
        plan.run_device(w.n_sweeps, w.n_reads, w.seed, z, e, stream=torch.cuda.current_stream().cuda_stream,
                        instance_id=w.instance_id)
        torch.cuda.synchronize()
        zs, es = srv.result(tickets[i])
        same = same and np.array_equal(z.cpu().numpy(), zs) and np.array_equal(e.cpu().numpy(), es)
        plan.close()
    srv.close()
    out = {
        "metric": "single-variable updates/sec at 1 GPU (served stream)",
        "value": upd / span, "unit": "updates/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": span * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64+f64", "data": "synthetic",
        "config": {"workload": f"Poisson stream of {n} requests: 90% HUIO N=2000 (OTM/Metropolis, 16 reads, "
                               f"1000 sweeps), 10% dense QUIO N=4096 [-1000,1000] heat bath (16 reads, 100 sweeps)",
                   "arrival_rate_req_s": rate, "saturated_req_s": sat_rate, "load": args.load,
                   "chunk_sweeps": 50},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "mean": float(lat.mean()), "max": float(lat.max())},
        "latency_by_kind_s": by_kind,
        "completed": len(ok), "server": stats, "alone_vs_mix_identical": bool(same),
    }
    if n < 10_000:
        # the stream is 10^4 requests with a distinct dense instance per dense request; a shorter
        # stream, whose dense requests share a pool of four instances (so that the served plan
        # cache skips their preparation), is not that configuration
        out["status"] = (f"UNMEASURED-at-config: {n} of 10^4 requests; dense requests share a pool of 4 "
                         "instances")
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus_requested": args.gpus}), flush=True)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2511_17245_amd import sa

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        return copy_probe(args.copy_probe_mib)
    if args.ttt:
        return bench_ttt(args)
    if args.suite:
        return bench_suite(args)
    if args.figures:
        return bench_figures(args)
    if args.config == "cfg4":
        return bench_batch(args)
    if args.config == "cfg5":
        return bench_serving(args)
    w = workload(args)
    prob = w.problem
    n, S, R = prob.n_vars, w.n_sweeps, w.n_reads
    beta = w.beta if w.beta is not None else sa.auto_schedule(prob, S)
    plan = sa.Plan(prob, w.rule)
    info = plan.info()
    z = torch.empty((R, n), dtype=torch.int32, device="cuda")
    e = torch.empty(R, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()

    lanes = args.lanes_per_update

    def step():
        plan.run_device(S, R, w.seed, z, e, beta=beta, stream=stream.cuda_stream,
                        instance_id=w.instance_id, waves_per_replica=args.waves_per_replica,
                        lanes_per_update=lanes)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for i in range(args.steps):
        step()
        print(f"[bench] queued step {i + 1}/{args.steps}", file=sys.stderr, flush=True)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop) / args.steps   # one kernel per step on this stream
    launch = plan.last_launch()
    updates = R * S * n
    value = updates / (ms / 1e3)

    e_host = e.cpu().numpy()
    W_mean = float(np.mean(prob.upper.astype(np.int64) - prob.lower + 1))
    traffic = measured_traffic(f"{args.config}:{S}:{R}")
    if w.rule == sa.HEAT_BATH:
        # the method's work: W weights per update, one direct exponential each (the kernel's
        # factored weights execute fewer instructions; the executed VALU issue is reported in
        # valu_issue below)
        flops = updates * W_mean * FP64_FLOPS_PER_WEIGHT
        achieved = flops / (ms / 1e3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                "basis": "algorithmic: W weights x 30 FP64 flops per update (one direct exponential each); "
                         "executed instructions in valu_issue"}
    else:
        # Metropolis / OTM: the incidence records come from the caches (measured HBM traffic is a
        # small fraction of them), and the counters show VALU issue as the busy resource: the
        # bound reported is VALU issue, from the counted instructions per update (committed
        # counter record of the same kernel sources) at this run's rate; null without a record
        crec = counter_record(f"{args.config}:{S}:{R}")
        vi = crec["valu_insts_per_update"] * value / 1e9 if crec and crec.get("valu_insts_per_update") else None
        roof = {"bound": "alu", "achieved": vi, "peak": VALU_ISSUE_PEAK_G, "unit": "G wave-instructions/s",
                "frac": vi / VALU_ISSUE_PEAK_G if vi is not None else None, "traffic": traffic,
                "basis": "counted VALU instructions per update x update rate (issue-bound)"}

    out = {
        "metric": "single-variable updates/sec at 1 GPU",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"int{info['arith_bits']}+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_vars": n, "n_sweeps": S, "n_reads": R,
                   "kernel_source_hash": kernel_source_hash(),
                   "rule": sa.RULE_NAMES[w.rule], "n_terms": info["n_terms"],
                   "n_incidences": info["n_incidences"], "launch": launch,
                   "mean_final_energy": float(np.mean(e_host)), "min_final_energy": int(e_host.min()),
                   "wall_s": wall},
        "roofline": roof,
    }
    crec = counter_record(f"{args.config}:{S}:{R}")
    if crec and crec.get("valu_insts_per_update"):
        # the binding resource of the heat bath: VALU instructions per update (counters, same
        # kernel sources) at this run's update rate, against the issue peak of the chip
        vi = crec["valu_insts_per_update"] * value / 1e9
        out["valu_issue"] = {"achieved": vi, "peak": VALU_ISSUE_PEAK_G, "unit": "G wave-instructions/s",
                             "frac": vi / VALU_ISSUE_PEAK_G, "insts_per_update": crec["valu_insts_per_update"],
                             "fp64_insts_per_update": crec.get("fp64_insts_per_update"),
                             "source": crec.get("profile")}
    if args.config == "cfg2" and not args.no_closed_form:
        # the paper's O(1) heat-bath draw on the same workload (its variables are all linear)
        cplan = sa.Plan(prob, sa.HEAT_BATH_CLOSED)

        def cstep():
            cplan.run_device(S, R, w.seed, z, e, beta=beta, stream=stream.cuda_stream,
                             instance_id=w.instance_id, waves_per_replica=args.waves_per_replica,
                             lanes_per_update=lanes)

        cstep()
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(args.steps):
            cstep()
        stop.record(stream)
        torch.cuda.synchronize()
        cms = start.elapsed_time(stop) / args.steps
        ce = e.cpu().numpy()
        out["heat_bath_closed_form"] = {"value": updates / (cms / 1e3), "unit": "updates/s", "ms_per_step": cms,
                                        "speedup_over_enumeration": ms / cms, "launch": cplan.last_launch(),
                                        "mean_final_energy": float(np.mean(ce)), "min_final_energy": int(ce.min())}
        cplan.close()
    if args.config == "cfg2" and not args.no_ttt and S == 2000 and R == 256:
        # time to target (the paper's energy-versus-time protocol, Sec. 4.4): the target is the
        # median of the oracle's final energies over all reads of this workload (stored by the
        # oracle alone, tests/golden/full_size_cfg2.txt), the best of them for TTS99
        eo = stored_oracle_energies("cfg2")
        if eo is not None and len(eo) == R:
            print("[bench] time-to-target grid", file=sys.stderr, flush=True)
            out["time_to_target"] = ttt_grid(plan, w, R, lanes, float(np.median(eo)), int(eo.min()))
    plan.close()
    if args.config == "cfg2" and not args.no_batch:
        print("[bench] batched versus plain (512 problems)", file=sys.stderr, flush=True)
        out["batched_vs_plain"] = batched_vs_plain(1, 1, 24)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, beta, min(args.cpu_reads, R),
                                           S if args.cpu_sweeps <= 0 else min(args.cpu_sweeps, S),
                                           one_core_sweeps=500 if args.config.startswith("cfg2") else 1000)
        tt = out.get("time_to_target")
        if tt and tt.get("ttt_sweeps"):
            # the oracle's time for the same grid run (its own median is the target at S sweeps),
            # at its all-core rate
            tt["oracle_s_at_ttt_sweeps"] = R * tt["ttt_sweeps"] * n / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
