"""Throughput of PT + isoenergetic cluster moves on one MI355X.

A step is SWEEPS_PER_STEP simulation steps (Metropolis sweep, cluster moves at
the cold temperatures, PT) over the whole batch of the workload -- by default
1024 3D L=8 Gaussian instances, 20 temperatures x 4 replicas -- issued as
launches of the fused sweep-block kernel replayed from a captured hipGraph.
Inputs are synthetic and resident in HBM before timing starts.

Prints one JSON line: value = spin-flip attempts/s over the whole job; also
cluster moves/s, the same kernels with plain per-instance launches, the
roofline of the fused kernel (effective HBM: algorithmic bytes over the
kernel's launch time; beside it the VALU issue fraction from measured
instruction counts), a short served run (continuous batching of the serving
mix: p50/p99 latency and attempts/s against per-instance launches of the same
requests) and the CPU oracle's rate on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s (one
# non-packed 32-bit or FP64 operation per lane per cycle)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Launch shape of the headline line unless the autotuner finds a faster one:
# 256 threads per workgroup, 16 cluster moves in flight per workgroup, tables
# placed by the library (in LDS for this workload), 256-sweep launches
# replayed from a captured graph, four launches per step.
DEFAULT_LAUNCH = dict(threads=256, icm_slots=16, sweeps_per_launch=256, use_graph=1, table_placement=0)
SWEEPS_PER_STEP = 1024


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="3d_L8_gauss_1024inst")
    ap.add_argument("--instances", type=int, default=0,
                    help="run the first N instances of the workload (0: all; for the Table I workloads "
                         "the first ones are all of the smallest size)")
    ap.add_argument("--sweeps-per-step", type=int, default=SWEEPS_PER_STEP)
    ap.add_argument("--sweeps-per-launch", type=int, default=DEFAULT_LAUNCH["sweeps_per_launch"])
    ap.add_argument("--threads", type=int, default=DEFAULT_LAUNCH["threads"])
    ap.add_argument("--icm-slots", type=int, default=DEFAULT_LAUNCH["icm_slots"])
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the launch shape of the flags instead of autotuning it")
    ap.add_argument("--tune-cache", default="", help="autotuner cache file (default: search every run)")
    ap.add_argument("--per-instance-sample", type=int, default=32)
    ap.add_argument("--served-requests", type=int, default=240,
                    help="requests of the short served run in the default line (0: none)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-instance", action="store_true")
    ap.add_argument("--serve", type=int, default=0,
                    help="run the serving workload with this many requests instead")
    ap.add_argument("--serve-sweeps", type=int, default=1 << 13)
    ap.add_argument("--serve-block", type=int, default=256)
    ap.add_argument("--serve-load", type=float, default=0.8)
    ap.add_argument("--arena-mib", type=int, default=1024)
    ap.add_argument("--thermalization", type=int, default=0,
                    help="run this many sweeps with and without ICM and report Delta(t) (Eq. 2) instead")
    ap.add_argument("--table1", type=int, default=0,
                    help="run the thermalization study at the paper's Table I parameters for this many "
                         "sweeps instead (PT vs PT + ICM per topology and size)")
    ap.add_argument("--table1-instances", type=int, default=128, help="disorder instances per size")
    ap.add_argument("--table1-topologies", default="2d,chimera,3d")
    ap.add_argument("--anneal", type=int, default=0,
                    help="run simulated annealing with and without cluster moves for this many sweeps instead")
    ap.add_argument("--anneal-instances", type=int, default=256)
    ap.add_argument("--percolation", type=int, default=0,
                    help="run the site-percolation Binder study with this many samples per (size, p) instead")
    return ap.parse_args()


def algorithmic_bytes_per_sweep(spec, N, n_bonds, jbytes):
    """2 bytes (int8 spin read + write) per attempt plus the couplings once."""
    S = spec["n_temps"] * spec["n_replicas"]
    return 2 * S * N + n_bonds * jbytes


# The sources the fused sweep kernel is compiled from.
SWEEP_KERNEL_SOURCES = ("icm_kernels.hip", "icm_device.h", "icm_internal.h")


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for name in SWEEP_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1501_05630_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def launch_tag(cfg):
    return "t{threads}_s{icm_slots}_spl{sweeps_per_launch}".format(**cfg)


# Counters of one launch of the fused kernel on a workload, from rocprofv3
# --pmc runs of this bench (the summaries under profiles/): HBM bytes =
# FETCH_SIZE + WRITE_SIZE, each scaled by what the counter reads for a plain
# 256 MiB device copy, and SQ_INSTS_VALU (wave instructions).  Valid only for
# the kernel source (digest) and launch shape they were measured on; the line
# reports null otherwise.
PROFILED = {
    "3d_L8_gauss_1024inst": {"kernel": "deabc0ef5d7c9f14", "launch": "t256_s16_spl256",
                             "hbm_bytes_per_launch": 102604222, "valu_insts_per_launch": 8.9388e9,
                             "profile": "profiles/sweep_block_kernel_3d_L8_gauss_1024inst.md"},
    "chimera_C12_int3_512inst": {"kernel": "deabc0ef5d7c9f14", "launch": "t512_s16_spl256",
                                 "hbm_bytes_per_launch": 1467544054, "valu_insts_per_launch": 8.0294e9,
                                 "profile": "profiles/sweep_block_kernel_chimera_C12_int3_512inst.md"},
}


def profiled(name, cfg):
    p = PROFILED.get(name)
    if p and p["kernel"] == kernel_source_digest() and p["launch"] == launch_tag(cfg):
        return p
    return None


def copy_bandwidth_gbs(nbytes=1 << 30, reps=8):
    """Measured device-to-device copy bandwidth (read + write bytes / time) of
    one GiB, timed with HIP events: the practical HBM ceiling beside the
    vendor peak."""
    import torch
    a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def cpu_baseline(name, spec, seconds):
    """The CPU oracle on the host cores, over a bounded sample of the workload."""
    import concurrent.futures as cf

    import oracle
    from paper_1501_05630_amd import inputs

    cores = os.cpu_count() or 1
    cores = min(cores, 16)
    S = spec["n_temps"] * spec["n_replicas"]
    n_inst = cores
    # sampled instances spread evenly over the batch (every size class of an
    # uneven batch is represented)
    picks = [b * spec["n_instances"] // n_inst for b in range(n_inst)]

    def sim(b, flags=oracle.FLAG_2A | oracle.FLAG_PT):
        J, temps, kc, sp = inputs.workload_instance(name, b)
        o = oracle.Sim(sp["topology"], sp["L"], J, temps, spec["n_replicas"], kc, flags=flags,
                       seed=inputs.MASTER_SEED, instance_key=b, j_scale=spec["j_scale"])
        o.init_hot()
        return o, inputs.n_sites(sp["topology"], sp["L"])

    # calibrate on the largest sampled instance: sweeps so that the sample takes ~`seconds`
    o, _ = sim(picks[-1])
    t0 = time.perf_counter()
    o.run(4)
    per_sweep = (time.perf_counter() - t0) / 4
    sweeps = max(4, int(seconds / max(per_sweep, 1e-9)))

    def job(b):
        o, N = sim(b)
        o.run(sweeps)
        return o.stats()["icm_moves"], S * N * sweeps

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        res = list(ex.map(job, picks))
    dt = time.perf_counter() - t0
    # one thread alone: a quarter of one instance's sweeps
    o, N1 = sim(picks[0])
    s1 = max(2, sweeps // 4)
    t1 = time.perf_counter()
    o.run(s1)
    dt1 = time.perf_counter() - t1
    # the cluster moves alone, on the states the single-thread run left:
    # Metropolis and PT switched off (steps 2a and 2b only), one thread
    ic, _ = sim(picks[0], flags=oracle.FLAG_2A | oracle.FLAG_SKIP_METRO)
    ic.set_states(o.states())
    m0 = ic.stats()["icm_moves"]
    s_icm = max(8, 4 * s1)
    t2 = time.perf_counter()
    ic.run(s_icm)
    dt2 = time.perf_counter() - t2
    icm_only = (ic.stats()["icm_moves"] - m0) / dt2
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": sum(r[1] for r in res) / dt, "unit": "spin-flip attempts/s", "cores": cores,
            "kind": "oracle", "icm_moves_per_s": sum(r[0] for r in res) / dt,
            "single_thread_value": S * N1 * s1 / dt1, "cpu_model": model, "host_cpus": os.cpu_count(),
            "icm_only_moves_per_s": icm_only,
            "sample": f"{n_inst} instances x {sweeps} sweeps of {name}, one oracle per thread; "
                      f"single thread: {s1} sweeps of one instance; cluster moves alone (no Metropolis, "
                      f"no PT) on that instance's states: {s_icm} steps, one thread"}


def serve_request(x, rng):
    """One request of the serving mix: 2D +-J L in {16,32,64}, 3D Gaussian L in
    {6,8,12}, chimera C in 4..16, uniformly."""
    from paper_1501_05630_amd import icm, inputs
    cls = int(rng.integers(0, 3))
    if cls == 0:
        L = int(rng.choice([16, 32, 64]))
        J = inputs.pm_j_couplings(inputs.SQUARE2D, L, rng)
        temps = inputs.geometric_temps(0.2, 1.6, 16)
        d = dict(topology=inputs.SQUARE2D, L=L, couplings=J, temps=temps, n_replicas=2, j_scale=1)
    elif cls == 1:
        L = int(rng.choice([6, 8, 12]))
        J = inputs.gaussian_couplings(inputs.CUBIC3D, L, rng)
        temps = inputs.geometric_temps(0.2, 2.0, 20)
        d = dict(topology=inputs.CUBIC3D, L=L, couplings=J, temps=temps, n_replicas=4, j_scale=1)
    else:
        C = int(rng.integers(4, 17))
        J = inputs.int_couplings(inputs.CHIMERA, C, rng)
        temps = inputs.geometric_temps(0.2, 3.0, 30)
        d = dict(topology=inputs.CHIMERA, L=C, couplings=J, temps=temps, n_replicas=2, j_scale=3)
    d["icm_ntemps"] = inputs.icm_cutoff(d["temps"])
    d["instance_key"] = x
    d["flags"] = icm.FLAG_2A | icm.FLAG_PT
    N = inputs.n_sites(d["topology"], d["L"])
    return d, len(d["temps"]) * d["n_replicas"] * N


def serve_mix(n_requests, sweeps, block, load, arena_mib, n_sat=None, per_instance=0):
    """Continuous batching of the serving mix: the saturated request rate (n_sat
    requests submitted at once), then n_requests Poisson arrivals at `load`
    times that rate: p50/p99 latency, sweeps/s and attempts/s.  With
    per_instance > 0, the same kernels with plain per-instance launches on that
    many requests of the mix (256 sweeps each) for comparison."""
    import numpy as np
    import torch

    from paper_1501_05630_amd import icm, inputs
    rng = inputs.make_rng(4, 0)
    reqs = [serve_request(x, rng) for x in range(n_requests)]
    ctx = icm.Context(arena_bytes=arena_mib << 20, seed=inputs.MASTER_SEED)
    out = {"requests": n_requests, "sweeps_per_request": sweeps, "block": block, "arena_mib": arena_mib}
    if per_instance:
        # plain per-instance launches: one request's instance per launch, no graph
        pick = reqs[:per_instance]
        hs = []
        for d, _ in pick:
            hs.append(ctx.icm_add_instance(**{k: v for k, v in d.items()}))
            ctx.icm_init_states(hs[-1])
        ctx.icm_set_run_config(sweeps_per_launch=256, use_graph=0)
        ctx.icm_run_per_instance(hs, 256)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        ctx.icm_run_per_instance(hs, 256)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        secs = e0.elapsed_time(e1) / 1e3
        out["per_instance"] = {"attempts_per_s": sum(w for _, w in pick) * 256 / secs,
                               "sample": f"{len(pick)} requests of the mix, 256 sweeps, one launch each"}
        for h in hs:
            ctx.icm_remove_instance(h)
    ctx.icm_serve_start(block)

    def drain(tickets):
        lat = []
        for t, (d, _) in tickets:
            while True:
                done, us = ctx.icm_poll(t)
                if done:
                    break
                time.sleep(0.0005)
            K, R = len(d["temps"]), d["n_replicas"]
            ctx.icm_take_result(t, K, R, inputs.n_sites(d["topology"], d["L"]))
            lat.append(us)
        return lat

    # saturated rate: a batch of requests submitted at once
    n_sat = n_sat or max(8, n_requests // 4)
    t0 = time.perf_counter()
    tickets = [(ctx.icm_submit(sweeps, **d), (d, w)) for d, w in reqs[:n_sat]]
    drain(tickets)
    sat_wall = time.perf_counter() - t0
    sat_rate = n_sat / sat_wall
    out["saturated_rate_per_s"] = sat_rate
    out["saturated_attempts_per_s"] = sum(w for _, w in reqs[:n_sat]) * sweeps / sat_wall
    # Poisson arrivals at a fraction of the saturated rate
    rate = load * sat_rate
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t0 = time.perf_counter()
    tickets = []
    next_t = t0
    for (d, w), g in zip(reqs, gaps):
        next_t += g
        while time.perf_counter() < next_t:
            time.sleep(0.0002)
        tickets.append((ctx.icm_submit(sweeps, **d), (d, w)))
    lat = drain(tickets)
    wall = time.perf_counter() - t0
    ctx.icm_serve_stop()
    ctx.close()
    attempts = sum(w for _, w in reqs) * sweeps
    lat = np.array(lat) / 1e3
    out.update({"load": load, "arrival_rate_per_s": rate,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "sweeps_per_s": n_requests * sweeps / wall, "attempts_per_s": attempts / wall})
    if "per_instance" in out:
        out["saturated_over_per_instance"] = out["saturated_attempts_per_s"] / out["per_instance"]["attempts_per_s"]
    return out


def run_serving(args):
    """Continuous batching under Poisson arrivals: p50/p99 latency and sweeps/s."""
    return serve_mix(args.serve, args.serve_sweeps, args.serve_block, args.serve_load, args.arena_mib,
                     per_instance=12)


def run_thermalization(args):
    """Delta(t) of Eq. 2, disorder-averaged per logarithmic time bin, for PT
    alone and PT + ICM on the same instances, seeds and temperatures."""
    import numpy as np
    import torch

    from paper_1501_05630_amd import analysis, icm, inputs
    name = args.workload
    spec = inputs.WORKLOADS[name]
    n_inst = spec["n_instances"]
    out = {"metric": "thermalization: disorder-averaged Delta (Eq. 2) per time bin t in [2^b, 2^(b+1))",
           "workload": name, "instances": n_inst, "sweeps": args.thermalization}
    for mode in ("pt", "pt_icm"):
        ctx = icm.Context(arena_bytes=4 << 30, seed=inputs.MASTER_SEED)
        ctx.icm_set_run_config(threads=args.threads, sweeps_per_launch=args.sweeps_per_step, use_graph=1,
                               icm_slots=args.icm_slots)
        hs, meta = [], []
        for b in range(n_inst):
            J, temps, kc, sp = inputs.workload_instance(name, b)
            hs.append(ctx.icm_add_instance(sp["topology"], sp["L"], J, temps, spec["n_replicas"],
                                           kc if mode == "pt_icm" else 0,
                                           flags=icm.FLAG_2A | icm.FLAG_PT | icm.FLAG_MEASURE,
                                           instance_key=b, j_scale=spec["j_scale"]))
            ctx.icm_init_states(hs[-1])
            N = inputs.n_sites(sp["topology"], sp["L"])
            nb = {inputs.SQUARE2D: 2 * N, inputs.CUBIC3D: 3 * N,
                  inputs.CHIMERA: 16 * sp["L"] ** 2 + 8 * sp["L"] * (sp["L"] - 1)}[sp["topology"]]
            meta.append((temps, N, nb))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.icm_run(hs, args.thermalization)
        ctx.icm_sync()
        wall = time.perf_counter() - t0
        unit = analysis.OBS_ENERGY_UNIT_FLOAT if spec["kind"] == "gauss" else 1.0 / spec["j_scale"]
        deltas = []
        for h, (temps, N, nb) in zip(hs, meta):
            sums, counts = ctx.icm_read_observables(h)
            deltas.append(analysis.delta_per_bin(sums, counts, temps, N, nb, unit)[2])
        d = np.array(deltas)                                   # [instances][bins][K]
        nbins = int(np.floor(np.log2(args.thermalization))) + 1
        mean = d[:, :nbins, :].mean(axis=0)
        se = d[:, :nbins, :].std(axis=0, ddof=1) / np.sqrt(len(d))
        out[mode] = {"wall_s": wall, "temps": [float(x) for x in meta[0][0]],
                     "delta_coldest": [float(x) for x in mean[:, 0]],
                     "se_coldest": [float(x) for x in se[:, 0]],
                     "delta_all_temps_last_bin": [float(x) for x in mean[-1]]}
        ctx.close()
    return out


def run_table1(args):
    """The thermalization study at the paper's Table I parameters with fewer
    disorder instances and sweeps: per topology and size, Delta (Eq. 2) at the
    lowest temperature per time bin for PT alone and PT + ICM on the same
    instances, the thermalization bin of each (analysis.thermalization_bin), their
    ratio, and the fraction p of potential cluster sites against T in the last
    complete bin."""
    import numpy as np
    import torch

    from paper_1501_05630_amd import analysis, icm, inputs
    names = {"2d": "table1_2d_gauss", "chimera": "table1_chimera_gauss", "3d": "table1_3d_gauss"}
    M = args.table1_instances
    out = {"metric": "thermalization at the Table I parameters: Delta (Eq. 2) at T_min per time bin "
                     "t in [2^b, 2^(b+1)), PT vs PT + ICM; cluster-site fraction p(T)",
           "sweeps": args.table1, "instances_per_size": M, "data": "synthetic Gaussian disorder, hot start"}
    for top in args.table1_topologies.split(","):
        name = names[top]
        spec = inputs.WORKLOADS[name]
        per = {}
        for mode in ("pt", "pt_icm"):
            ctx = icm.Context(arena_bytes=6 << 30, seed=inputs.MASTER_SEED)
            ctx.icm_set_run_config(threads=args.threads, sweeps_per_launch=args.sweeps_per_step,
                                   use_graph=1, icm_slots=args.icm_slots)
            hs = []
            for si, L in enumerate(spec["sides"]):
                for m in range(M):
                    b = si * spec["per_side"] + m
                    J, temps, kc, sp = inputs.workload_instance(name, b)
                    hs.append((L, ctx.icm_add_instance(sp["topology"], L, J, temps, spec["n_replicas"],
                                                       kc if mode == "pt_icm" else 0,
                                                       flags=icm.FLAG_2A | icm.FLAG_PT | icm.FLAG_MEASURE,
                                                       instance_key=b, j_scale=1)))
                    ctx.icm_init_states(hs[-1][1])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            done, shown = 0, t0
            while done < args.table1:      # in chunks, with a progress line every 30 s
                n = min(1 << 14, args.table1 - done)
                ctx.icm_run([h for _, h in hs], n)
                ctx.icm_sync()
                done += n
                if time.perf_counter() - shown > 30:
                    shown = time.perf_counter()
                    print(f"table1 {top} {mode}: {done} sweeps", file=sys.stderr, flush=True)
            wall = time.perf_counter() - t0
            print(f"table1 {top} {mode}: {len(hs)} instances x {args.table1} sweeps in {wall:.1f} s",
                  file=sys.stderr, flush=True)
            for L in spec["sides"]:
                N = inputs.n_sites(spec["topology"], L)
                nb = {inputs.SQUARE2D: 2 * N, inputs.CUBIC3D: 3 * N,
                      inputs.CHIMERA: 16 * L * L + 8 * L * (L - 1)}[spec["topology"]]
                d, p = [], []
                for L2, h in hs:
                    if L2 != L:
                        continue
                    sums, counts = ctx.icm_read_observables(h)
                    d.append(analysis.delta_per_bin(sums, counts, temps, N, nb, analysis.OBS_ENERGY_UNIT_FLOAT)[2][:, 0])
                    p.append(analysis.cluster_fraction_per_bin(sums, counts, N))
                complete = [int(c) == (1 << b) for b, c in enumerate(counts)]
                last = max(b for b in range(len(complete)) if complete[b])
                d = np.array(d)                                   # [instances][bins]
                d = d[:, :last + 1]
                mean = d.mean(axis=0)
                se = d.std(axis=0, ddof=1) / np.sqrt(len(d))
                tb = analysis.thermalization_bin(mean, se, complete)
                per.setdefault(L, {"N": N})[mode] = {
                    "wall_s": wall, "delta_tmin": [float(x) for x in mean[:last + 1]],
                    "se_tmin": [float(x) for x in se[:last + 1]], "thermalized_bin": tb}
                if mode == "pt_icm":
                    per[L]["temps"] = [float(x) for x in temps]
                    per[L]["p_last_bin"] = [float(x) for x in np.mean(np.array(p), axis=0)[last]]
            ctx.close()
        for L, r in per.items():
            a, b = r["pt"]["thermalized_bin"], r["pt_icm"]["thermalized_bin"]
            r["speedup"] = (2.0 ** (a - b) if a is not None and b is not None else
                            (f">= 2^{len(r['pt']['delta_tmin']) - b}" if b is not None else None))
        out[top] = {"workload": name, "t_min": spec["t_min"], "n_icm": spec["n_icm"],
                    "sizes": {str(L): r for L, r in per.items()}}
    return out


# Site-percolation study: sizes and occupation probabilities around the
# thresholds (chimera: the paper's own estimate; square and cubic lattices: the
# values the paper quotes from the literature)
PERCOLATION = {
    "chimera": dict(topology=2, sides=(4, 8, 12, 16, 22, 32, 45), p=(0.37, 0.40), p_ref=0.3866, nu_ref=1.39,
                    fit_from=16),
    "2d": dict(topology=0, sides=(16, 32, 64, 128), p=(0.58, 0.61), p_ref=0.592, nu_ref=4 / 3, fit_from=32),
    # cubic lattice: with sqrt(N) as the length the exponent is 3/2 of the usual nu
    "3d": dict(topology=1, sides=(8, 12, 16, 24), p=(0.30, 0.325), p_ref=0.311, nu_ref=1.3, fit_from=12),
}


def run_percolation(args):
    """The Binder ratio g(p, N) of the largest cluster of random site
    configurations on a grid of p for several sizes per topology, the p where
    the curves of consecutive sizes cross (estimates of p_c), and the
    throughput of the percolation kernel in samples/s."""
    import numpy as np
    import torch

    from paper_1501_05630_amd import analysis, icm, inputs
    n = args.percolation
    ctx = icm.Context(arena_bytes=64 << 20, seed=inputs.MASTER_SEED)
    out = {"metric": "site percolation: Binder ratio g = (3 - <s^4>/<s^2>^2)/2 of the largest cluster",
           "samples_per_point": n}
    buf = torch.empty(n, dtype=torch.int32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for name, cfg in PERCOLATION.items():
        ps = np.linspace(cfg["p"][0], cfg["p"][1], 11)
        res, g_all, sides = {}, [], []
        for L in cfg["sides"]:
            N = inputs.n_sites(cfg["topology"], L)
            try:
                ctx.icm_percolation_smax(cfg["topology"], L, 0.5, 1, key=L, out=buf)
            except icm.IcmError as e:      # larger than the device's LDS per workgroup allows
                res[str(L)] = {"N": N, "skipped": str(e)}
                continue
            sides.append(L)
            gs, ses, ms = [], [], 0.0
            for pi, p in enumerate(ps):
                e0.record(ctx.stream)
                ctx.icm_percolation_smax(cfg["topology"], L, float(p), n, sample0=pi * n, key=L, out=buf)
                e1.record(ctx.stream)
                s = buf.cpu().numpy()
                ms += e0.elapsed_time(e1)
                gs.append(float(analysis.binder_ratio(s)))
                # standard error from 16 blocks of samples
                blocks = [analysis.binder_ratio(b) for b in np.array_split(s, 16)]
                ses.append(float(np.std(blocks, ddof=1) / 4.0))
            g_all.append(np.array(gs))
            res[str(L)] = {"N": N, "g": gs, "se": ses,
                           "samples_per_s": len(ps) * n / (ms * 1e-3)}
            print(f"percolation {name} L={L}: {len(ps) * n / (ms * 1e-3):.3g} samples/s",
                  file=sys.stderr, flush=True)
        crossings = []
        for a in range(len(sides) - 1):
            d = g_all[a + 1] - g_all[a]
            x = None
            for i in range(len(ps) - 1):
                if d[i] <= 0 < d[i + 1] or d[i] >= 0 > d[i + 1]:
                    x = float(ps[i] + (ps[i + 1] - ps[i]) * d[i] / (d[i] - d[i + 1]))
                    break
            crossings.append({"sizes": [sides[a], sides[a + 1]], "p_cross": x})
        fit = [L for L in sides if L >= cfg["fit_from"]]
        pc, nu, chi2 = analysis.binder_collapse(ps, [res[str(L)]["N"] for L in fit], [res[str(L)]["g"] for L in fit],
                                           [res[str(L)]["se"] for L in fit], cfg["p_ref"], cfg["nu_ref"])
        out[name] = {"p": [float(x) for x in ps], "p_ref": cfg["p_ref"], "sizes": res, "crossings": crossings,
                     "collapse": {"sides": fit, "p_c": pc, "nu_sqrtN": nu, "chi2_per_dof": chi2}}
    ctx.close()
    return out


def run_anneal(args):
    """Simulated annealing as a ground-state heuristic with and without
    isoenergetic cluster moves at every temperature step (the introduction's
    proposal), on the same chimera instances and schedule: the fraction of
    replicas that end at the lowest energy any method found and the mean
    residual energy per spin; then zero-temperature dynamics from the annealed
    states, with and without cluster moves, counting the distinct
    lowest-energy configurations visited (hopping through a degenerate
    ground-state manifold, discussion of Fig. 1)."""
    import numpy as np
    import torch

    from paper_1501_05630_amd import analysis, icm, inputs
    C, R, steps = 8, 16, 64
    M = args.anneal_instances
    per_step = max(1, args.anneal // steps)
    schedule = np.geomspace(3.0, 0.1, steps)
    N = inputs.n_sites(inputs.CHIMERA, C)
    Js = [inputs.pm_j_couplings(inputs.CHIMERA, C, inputs.make_rng(8, b)) for b in range(M)]
    out = {"metric": "annealing: success fraction and residual energy, SA vs SA + ICM",
           "instances": M, "topology": "chimera", "C": C, "N": N, "replicas": R,
           "schedule": {"t_start": 3.0, "t_end": 0.1, "steps": steps, "sweeps_per_step": per_step}}
    ctx = icm.Context(arena_bytes=2 << 30, seed=inputs.MASTER_SEED)
    ctx.icm_set_run_config(threads=args.threads, sweeps_per_launch=per_step, use_graph=1, icm_slots=args.icm_slots)
    finals, states = {}, {}
    for mode, kc in (("sa", 0), ("sa_icm", 1)):
        hs = [ctx.icm_add_instance(inputs.CHIMERA, C, J, [3.0], R, kc, flags=icm.FLAG_2A, instance_key=b,
                                   j_scale=1) for b, J in enumerate(Js)]
        for h in hs:
            ctx.icm_init_states(h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for T in schedule:
            for h in hs:
                ctx.icm_set_temperatures(h, [T])
            ctx.icm_run(hs, per_step)
        ctx.icm_sync()
        wall = time.perf_counter() - t0
        finals[mode] = np.array([ctx.icm_read_energies(h)[0][0] for h in hs])       # [M][R], units of J
        states[mode] = [ctx.icm_read_states(h)[0] for h in hs]
        for h in hs:
            ctx.icm_remove_instance(h)
        out[mode] = {"wall_s": wall}
        print(f"anneal {mode}: {M} instances in {wall:.1f} s", file=sys.stderr, flush=True)
    # reference: parallel tempering with cluster moves, 2^14 sweeps, coldest walkers
    temps = inputs.geometric_temps(0.1, 3.0, 30)
    hs = [ctx.icm_add_instance(inputs.CHIMERA, C, J, temps, 2, inputs.icm_cutoff(temps),
                               flags=icm.FLAG_2A | icm.FLAG_PT, instance_key=b, j_scale=1) for b, J in enumerate(Js)]
    for h in hs:
        ctx.icm_init_states(h)
    ctx.icm_set_run_config(threads=args.threads, sweeps_per_launch=256, use_graph=1, icm_slots=args.icm_slots)
    ctx.icm_run(hs, 1 << 14)
    ctx.icm_sync()
    pt_best = np.array([ctx.icm_read_energies(h)[0].min() for h in hs])
    for h in hs:
        ctx.icm_remove_instance(h)
    best = np.minimum(pt_best, np.minimum(finals["sa"].min(axis=1), finals["sa_icm"].min(axis=1)))
    out["reference"] = "lowest energy of SA, SA + ICM and 2^14 sweeps of PT + ICM (30 temperatures)"
    for mode in ("sa", "sa_icm"):
        f = finals[mode]
        out[mode].update({"success_fraction": float(np.mean(f == best[:, None])),
                          "instances_solved": float(np.mean((f == best[:, None]).any(axis=1))),
                          "residual_per_spin": float(np.mean(f - best[:, None]) / N)})
    out["pt_icm_reaches_best"] = float(np.mean(pt_best == best))
    # zero temperature from the SA + ICM states
    for mode, kc in (("t0_metropolis", 0), ("t0_icm", 1)):
        hs = [ctx.icm_add_instance(inputs.CHIMERA, C, J, [1e-3], R, kc, flags=icm.FLAG_2A, instance_key=b,
                                   j_scale=1) for b, J in enumerate(Js)]
        seen = [set() for _ in hs]
        for h, st in zip(hs, states["sa_icm"]):
            ctx.icm_set_states(h, st.reshape(1, R, N))
        ctx.icm_set_run_config(threads=args.threads, sweeps_per_launch=16, use_graph=1, icm_slots=args.icm_slots)
        for _ in range(16):
            ctx.icm_run(hs, 16)
            for b, h in enumerate(hs):
                e = ctx.icm_read_energies(h)[0][0]
                st = ctx.icm_read_states(h)[0]
                for r in np.flatnonzero(e == best[b]):
                    x = st[r] if st[r][0] > 0 else -st[r]
                    seen[b].add(x.tobytes())
        for h in hs:
            ctx.icm_remove_instance(h)
        out[mode] = {"sweeps": 256, "distinct_ground_states_mean": float(np.mean([len(s) for s in seen])),
                     "instances_with_several": float(np.mean([len(s) > 1 for s in seen]))}
    ctx.close()
    return out


def main():
    args = parse()
    if args.anneal:
        if args.gpus != 1:
            print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
            sys.exit(2)
        print(json.dumps(run_anneal(args)), flush=True)
        return
    if args.percolation:
        if args.gpus != 1:
            print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
            sys.exit(2)
        print(json.dumps(run_percolation(args)), flush=True)
        return
    if args.table1:
        if args.gpus != 1:
            print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
            sys.exit(2)
        print(json.dumps(run_table1(args)), flush=True)
        return
    if args.thermalization:
        if args.gpus != 1:
            print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
            sys.exit(2)
        print(json.dumps(run_thermalization(args)), flush=True)
        return
    if args.serve:
        if args.gpus != 1:
            print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
            sys.exit(2)
        print(json.dumps({"metric": "serving: p50/p99 latency and sweeps/s",
                          "serving": run_serving(args)}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1501_05630_amd import analysis, icm, inputs

    name = args.workload
    spec = dict(inputs.WORKLOADS[name])
    if args.instances:
        spec["n_instances"] = min(args.instances, spec["n_instances"])
    n_inst = spec["n_instances"]
    S = spec["n_temps"] * spec["n_replicas"]
    ctx = icm.Context(arena_bytes=4 << 30, seed=inputs.MASTER_SEED)
    hs, sizes, moves_per_sweep, bonds = [], [], [], []
    for b in range(n_inst):
        J, temps, kc, sp = inputs.workload_instance(name, b)
        hs.append(ctx.icm_add_instance(sp["topology"], sp["L"], J, temps, spec["n_replicas"], kc,
                                       instance_key=b, j_scale=spec["j_scale"]))
        ctx.icm_init_states(hs[-1])
        N = inputs.n_sites(sp["topology"], sp["L"])
        sizes.append(N)
        moves_per_sweep.append(kc * spec["n_replicas"] // 2)
        bonds.append({inputs.SQUARE2D: 2 * N, inputs.CUBIC3D: 3 * N,
                      inputs.CHIMERA: 16 * sp["L"] ** 2 + 8 * sp["L"] * (sp["L"] - 1)}[sp["topology"]])
    jbytes = 4 if spec["kind"] == "gauss" else 1
    spsw = args.sweeps_per_step
    launch = dict(threads=args.threads, icm_slots=args.icm_slots, sweeps_per_launch=args.sweeps_per_launch,
                  use_graph=args.graph, table_placement=0, class_threads=(-1, -1, -1, -1))
    tuned = {"source": "flags"}
    if not args.no_tune:
        # the autotuner times every candidate shape on this batch (advancing
        # it), then the batch restarts from its hot start
        from paper_1501_05630_amd import autotune
        cands = [c for c in autotune.candidates() if spsw % c["sweeps_per_launch"] == 0]
        best, info = autotune.tune(ctx, hs, cache_path=args.tune_cache or None, cands=cands)
        launch.update(best)
        tuned = {"source": info["source"], "key": info["key"], "candidates": len(cands)}
        if "ms_per_sweep" in info:
            tuned["best_ms_per_sweep"] = min(info["ms_per_sweep"].values())
            dflt = json.dumps(dict(threads=DEFAULT_LAUNCH["threads"], icm_slots=DEFAULT_LAUNCH["icm_slots"],
                                   sweeps_per_launch=DEFAULT_LAUNCH["sweeps_per_launch"], use_graph=1,
                                   class_threads=autotune.NO_CLASS_THREADS), sort_keys=True)
            if dflt in info["ms_per_sweep"]:
                tuned["default_ms_per_sweep"] = info["ms_per_sweep"][dflt]
        for h in hs:
            ctx.icm_init_states(h)
    ctx.icm_set_run_config(**launch)
    spl = launch["sweeps_per_launch"]
    # one launch per size class of units (sites <= 512, <= 1024, <= 2048, more)
    n_groups = len({0 if n <= 512 else (1 if n <= 1024 else (2 if n <= 2048 else 3)) for n in sizes})
    launches_per_step = n_groups * ((spsw + spl - 1) // spl)
    stream = ctx.stream
    for _ in range(args.warmup):
        ctx.icm_run(hs, spsw)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        ctx.icm_run(hs, spsw)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    sweeps = spsw * args.steps
    attempts_per_sweep = S * sum(sizes)
    secs = ms / 1e3
    value = attempts_per_sweep * sweeps / secs
    icm_moves = sum(moves_per_sweep) * sweeps
    step_ms = ms / args.steps
    bytes_per_sweep = sum(2 * S * N + nb * jbytes for N, nb in zip(sizes, bonds))
    sides = sorted({inputs.instance_side(spec, b) for b in range(n_inst)})
    uneven = len(sides) > 1
    # the roofline of the fused kernel: one size class -> launches back to
    # back on the context stream, so a launch lasts step time / launches;
    # several classes (uneven batch) -> taken over the whole step
    launch_ms = step_ms / launches_per_step if n_groups == 1 else step_ms
    per_launch_bytes = bytes_per_sweep * (spl if n_groups == 1 else spsw)
    achieved_gbs = per_launch_bytes / (launch_ms / 1e3) / 1e9
    prof = profiled(name, launch) if n_groups == 1 else None
    alu = None
    if prof:
        lane_ops = prof["valu_insts_per_launch"] * 64
        alu = {"valu_lane_ops_per_attempt": lane_ops / (attempts_per_sweep * spl),
               "achieved": lane_ops / (launch_ms / 1e3) / 1e12, "peak": VALU_PEAK_TOPS, "unit": "T lane-op/s"}
        alu["frac"] = alu["achieved"] / VALU_PEAK_TOPS

    out = {
        "metric": "spin-flip attempts/s + ICM moves/s, batched vs per-instance; % HBM roofline",
        "value": value, "unit": "spin-flip attempts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i32",
        "dtype_detail": ("bit-packed spins; int32 fields of 24-bit fixed-point couplings (2^-20 grid); fp32 "
                         "acceptance filter with an exact fp64 decision near the boundary; fp64 energies"
                         if spec["kind"] == "gauss" else
                         "bit-packed spins; int32 fields and energies; u32 threshold tables"),
        "data": "synthetic (seeded disorder, hot start)",
        "config": {"workload": name, "instances": n_inst, "topology": inputs.TOPOLOGY_NAMES[spec["topology"]],
                   "L": sides if uneven else sides[0],
                   "N": sorted(set(sizes)) if uneven else sizes[0], "temps": spec["n_temps"],
                   "replicas": spec["n_replicas"], "icm_temps": moves_per_sweep[0] * 2 // spec["n_replicas"],
                   "sweeps_per_step": spsw, "sweeps_per_launch": spl, "launches_per_step": launches_per_step,
                   "threads": sorted({icm.launch_threads(n, launch["threads"], launch["class_threads"])
                                      for n in sizes}),
                   "class_threads": [int(x) for x in launch["class_threads"]],
                   "threads_requested": launch["threads"], "icm_slots": launch["icm_slots"],
                   "graph": bool(launch["use_graph"]) and spsw // spl > 1, "launch_shape": tuned,
                   "parallelism": "single GPU, one workgroup per instance"},
        "icm_moves_per_s": icm_moves / secs,
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved_gbs / HBM_PEAK_GBS,
                     "traffic": prof["hbm_bytes_per_launch"] if prof else None,
                     "kind": "effective (algorithmic bytes / kernel time)",
                     "bytes_per_attempt": bytes_per_sweep / attempts_per_sweep,
                     "algorithmic_bytes_per_launch": per_launch_bytes, "launch_ms": launch_ms,
                     "alu": alu},
    }
    # the practical HBM ceiling beside the vendor peak (outside the timed region)
    copy_gbs = copy_bandwidth_gbs()
    out["roofline"]["measured_copy_gbs"] = copy_gbs
    out["roofline"]["frac_of_measured_copy"] = achieved_gbs / copy_gbs
    # the cluster moves' own accounting: a move reads both replicas' N spins and
    # writes the |C| flipped sites in both (2 N + 2 <|C|> bytes as int8)
    st = [ctx.icm_read_stats(h) for h in hs]
    moves = sum(x["icm_moves"] for x in st)
    if moves:
        mean_c = sum(x["icm_cluster_sites"] for x in st) / moves
        out["icm"] = {"mean_cluster_sites": mean_c,
                      "nontrivial_fraction": sum(x["icm_nontrivial"] for x in st) / moves,
                      "bytes_per_move": 2 * sum(sizes) / len(sizes) + 2 * mean_c}
    if not args.no_per_instance:
        # plain per-instance launches over a sample spread evenly over the batch
        k = min(args.per_instance_sample, n_inst)
        pick = [b * n_inst // k for b in range(k)]
        sample = [hs[b] for b in pick]
        ctx.icm_set_run_config(use_graph=0, sweeps_per_launch=spl)
        ctx.icm_run_per_instance(sample, spl)
        torch.cuda.synchronize()
        ev0.record(stream)
        ctx.icm_run_per_instance(sample, spl)
        ev1.record(stream)
        torch.cuda.synchronize()
        pms = ev0.elapsed_time(ev1)
        out["per_instance"] = {"value": S * sum(sizes[b] for b in pick) * spl / (pms / 1e3),
                               "icm_moves_per_s": sum(moves_per_sweep[b] for b in pick) * spl / (pms / 1e3),
                               "sample": f"{k} instances, one launch of {spl} sweeps each, no graph"}
        out["batched_over_per_instance"] = value / out["per_instance"]["value"]
    ctx.close()
    if args.served_requests:
        out["served"] = serve_mix(args.served_requests, args.serve_sweeps, args.serve_block, args.serve_load,
                                  args.arena_mib, n_sat=args.served_requests, per_instance=12)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(name, spec, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
