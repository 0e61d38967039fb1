#!/usr/bin/env python3
"""Benchmark: attempted swaps/s of link-cell parallel swap Metropolis on one
MI355X, with the HBM roofline of the mini-step kernel and the CPU oracle timed
beside it.

Workload (default): BCC 800^3 conventional cells (1.024e9 sites, uint8), 4
species equiatomic, EPI on 4 shells (V ~ N(0, 0.02 eV), seed 5), 1200 K,
link-cell edge 4 (128 mini-steps per sweep).  One step = 10 sweeps followed by
one short-range-order reduction (pair counts -> Warren-Cowley SRO); 5 steps =
the 50-sweep run with SRO every 10 sweeps.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# 32-bit VALU lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
Z_SHELLS = {0: (8, 6, 12, 24), 1: (12, 6, 24, 12)}


def algorithmic_ops_per_trial(lattice, K, S):
    """32-bit ALU operations one trial needs in the counted-neighbour form:
    Philox4x32-10 (10 rounds of two 32x32->64 products = 4 multiplies, and 4
    xors) 80; partner index and uniform 4; one shift-add per neighbour of
    either site 2*sum(Z); per (shell, species) term extract, convert, multiply
    and add 4*S*K; decision 4."""
    return 80 + 4 + 2 * sum(Z_SHELLS[lattice][:S]) + 4 * S * K + 4


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps-per-step", type=int, default=10)
    ap.add_argument("--edge", type=int, default=800, help="conventional cells per axis")
    ap.add_argument("--dims", type=str, default="",
                    help="X,Y,Z conventional cells (overrides --edge; not the headline workload)")
    ap.add_argument("--ell", type=int, default=4, help="link-cell edge")
    ap.add_argument("--tile", type=str, default="0,0,0")
    ap.add_argument("--mode", default="stream", choices=["stream", "persistent", "plain", "auto"])
    ap.add_argument("--tiles", action="store_true",
                    help="stage per-offset tile windows even where whole-row windows fit")
    ap.add_argument("--double-buffer", action="store_true",
                    help="stream the next tile window in while the current one runs")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU time budget of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ladder", action="store_true",
                    help="skip the batched-ladder vs plain-loop comparison")
    ap.add_argument("--ladder-sweeps", type=int, default=20)
    ap.add_argument("--legs", type=str, default="all",
                    help="comma list of legs to run, for profiling one at a time: main (the BCC lattice "
                         "above), ladder, tempering, anneal, qsro, fcc128, backward, paper795, clusters, cpu; "
                         "the JSON line is printed only when main runs")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--profile-name", type=str, default="",
                    help="with --summarize trace: file stem and title of the summary (default: the "
                         "benchmark lattice's sweep trace)")
    ap.add_argument("--summarize", nargs="+", metavar="ARG",
                    help="write profiles/ summaries from rocprofv3 csv output and exit: "
                         "'trace DIR CMD' (kernel-trace --stats) or "
                         "'traffic FETCH_DIR WRITE_DIR COPYF_DIR COPYW_DIR CMD' (--pmc passes)")
    return ap.parse_args()


def copy_probe():
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n, "launches": 3}))


def host_cpu():
    """CPU model (first "model name" of /proc/cpuinfo), the CPUs the machine
    reports and the CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count() or 1
    return model, os.cpu_count() or 1, allowed


def cpu_baseline(lattice, dims, K, S, cells, occ_host, V, seed, beta, budget_s):
    """The oracle on a bounded sample of the same workload: the first mini-steps
    of sweep 0 on the same lattice, on the threads the host grants this job
    (OMP_NUM_THREADS, else every CPU the process may use), and the next
    mini-step on one thread."""
    from oracle import oracle as O
    model, ncpu, allowed = host_cpu()
    env = os.environ.get("OMP_NUM_THREADS", "")
    nthreads = int(env) if env.isdigit() and int(env) > 0 else allowed
    occ = occ_host.copy()
    t0 = time.perf_counter()
    r = O.run_ministeps(lattice, dims, K, S, cells, occ, V, seed, beta, 0, 0, 1, nthreads=nthreads)
    t1 = time.perf_counter() - t0
    trials = int(r.stats[0])
    n_more = max(0, int(budget_s / max(t1, 1e-3)) - 1)
    nA = int(np.prod([max(c) for c in cells])) * (2 if lattice == 0 else 4)
    n_more = min(n_more, nA - 2)
    if n_more > 0:
        t0 = time.perf_counter()
        r2 = O.run_ministeps(lattice, dims, K, S, cells, occ, V, seed, beta, 0, 1, 1 + n_more,
                             nthreads=nthreads)
        t1 += time.perf_counter() - t0
        trials += int(r2.stats[0])
    # one thread: the next mini-step of the same sweep
    t0 = time.perf_counter()
    r1 = O.run_ministeps(lattice, dims, K, S, cells, occ, V, seed, beta, 0, 1 + n_more, 2 + n_more, nthreads=1)
    ts = time.perf_counter() - t0
    return {"value": trials / t1, "unit": "attempted swaps/s", "cores": nthreads, "kind": "oracle",
            "sample": f"mini-steps 0..{n_more} of sweep 0 on the same {dims[0]}x{dims[1]}x{dims[2]} "
                      f"lattice ({trials} trials, {t1:.1f} s)",
            "cpu_model": model, "host_cpus": ncpu, "cpus_allowed": allowed,
            "single_thread": {"value": int(r1.stats[0]) / ts, "unit": "attempted swaps/s",
                              "sample": f"mini-step {1 + n_more} of sweep 0 ({int(r1.stats[0])} trials, "
                                        f"{ts:.1f} s)"}}


def main():
    args = parse()
    if args.summarize:
        summarize(args)
        return
    legs = set(args.legs.split(",")) if args.legs != "all" else None
    if legs is not None and "main" not in legs:
        side_legs(args, legs)
        return
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; --gpus N > 1 is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_probe:
        copy_probe()
        return
    from paper_2503_12591_amd import inputs as I
    from paper_2503_12591_amd import smcx

    lattice, K, S = I.BCC, 4, 4
    dims = tuple(int(x) for x in args.dims.split(",")) if args.dims else (args.edge,) * 3
    N = I.n_sites(lattice, dims)
    V = I.epi(K, S, 0.02, seed=5)
    T = 1200.0
    beta = float(I.beta_of_T(T))
    seed = 0
    tile = tuple(int(x) for x in args.tile.split(","))
    print(f"[bench] generating {N} sites", file=sys.stderr, flush=True)
    occ = I.occupancy_device(I.equiatomic(K, N), seed=0)
    occ_host = occ.cpu().numpy() if not args.no_cpu_baseline and (legs is None or "cpu" in legs) else None
    lat = smcx.Lattice(lattice, dims, K, S, occ, ell=args.ell, tile=tile, double_buffer=args.double_buffer,
                       rows=not args.tiles)
    lat.set_epi(V)
    cells, nA = lat.schedule(0)
    nC = int(np.prod([len(c) for c in cells]))
    spst = args.sweeps_per_step
    betas = torch.full((spst, 1), beta, dtype=torch.float64, device="cuda")
    stats = torch.zeros(3, dtype=torch.int64, device="cuda")
    ties = torch.zeros(4096 * 24, dtype=torch.uint8, device="cuda")
    tie_count = torch.zeros(1, dtype=torch.int32, device="cuda")

    sweep_no = 0

    def step():
        nonlocal sweep_no
        lat.sweep(spst, seed, betas, first_sweep=sweep_no, mode=args.mode, stats=stats, ties=ties,
                  tie_count=tie_count)
        sweep_no += spst
        return lat.sro()

    print(f"[bench] warmup {args.warmup} step(s)", file=sys.stderr, flush=True)
    lat.sro()  # SRO of the initial configuration (sweep 0)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st0 = stats.cpu().numpy().copy()
    print(f"[bench] timing {args.steps} step(s)", file=sys.stderr, flush=True)
    lat.timing(True)
    lat.timing_read()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    kern_ms, launches = lat.timing_read()
    lat.timing(False)
    st1 = stats.cpu().numpy()
    attempted = int(st1[0] - st0[0])
    assert attempted == args.steps * spst * N, (attempted, args.steps * spst * N)
    secs = ms / 1e3
    value = attempted / secs
    avg_launch_s = kern_ms / 1e3 / max(launches, 1)
    launches_per_sweep = launches / (args.steps * spst)
    M = [int(max(c)) for c in cells]
    kernel = "k_rows" if abs(launches_per_sweep - M[1] * M[2]) < 1e-9 else "k_ministep"
    bytes_per_launch = algorithmic_bytes_per_launch(cells, N, 2, launches_per_sweep)
    achieved = bytes_per_launch / avg_launch_s / 1e9 if args.mode == "stream" else None
    trials_per_launch = N * args.steps * spst / max(launches, 1)
    ops = algorithmic_ops_per_trial(lattice, K, S)
    alu_achieved = trials_per_launch * ops / avg_launch_s / 1e12
    traffic = None
    dtag = "x".join(str(d) for d in dims) if len(set(dims)) > 1 else str(dims[0])
    tfile = os.path.join(ROOT, "profiles", f"traffic_{kernel[2:]}_bcc{dtag}_ell{args.ell}.json")
    if os.path.exists(tfile):
        with open(tfile) as f:
            tr = json.load(f)
        if tr.get("kernel_build") == kernel_fingerprint():
            traffic = tr["bytes_per_launch"]
    out = {
        "metric": "attempted swaps/sec and HBM GB/s fraction; batched ladder vs plain sweep",
        "value": value,
        "unit": "attempted swaps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp64",
        "data": "synthetic",
        "config": {"workload": f"bcc{dtag}_k4_s4_T1200_sro10", "lattice": "BCC",
                   "arithmetic": "fp64 dE, E and SRO; integer pair counts",
                   "storage": "u8 occupancy (one byte per site)",
                   "dims": list(dims), "sites": N, "species": K, "shells": S, "T_K": T,
                   "sweeps_per_step": spst, "link_cell": args.ell, "n_ministeps": nA,
                   "n_cells": nC, "mode": args.mode, "tile": list(tile),
                   "window_buffers": 2 if args.double_buffer else 1,
                   "accepted_frac": float(st1[1] - st0[1]) / attempted,
                   "near_ties": int(tie_count.item())},
        "roofline": roofline(kernel, achieved, alu_achieved, traffic, avg_launch_s, launches, bytes_per_launch,
                             trials_per_launch, ops, value, nA),
        "wall_s": wall,
    }
    want = lambda name: legs is None or name in legs
    if not args.no_ladder:
        for name, fn in (("ladder", ladder_bench), ("tempering", tempering_bench), ("anneal", anneal_bench),
                         ("qsro", qsro_bench), ("fcc128", fcc128_bench), ("backward", backward_bench),
                         ("paper795", paper795_bench)):
            if want(name):
                print(f"[bench] {name}", file=sys.stderr, flush=True)
                out[name] = fn(args)
        if want("clusters"):
            print("[bench] clusters", file=sys.stderr, flush=True)
            out["clusters"] = clusters_bench(lat, N)
    if not args.no_cpu_baseline and want("cpu"):
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(lattice, dims, K, S, cells, occ_host, V, seed, beta,
                                           args.cpu_seconds)
    lat.close()
    print(json.dumps(out), flush=True)


def side_legs(args, legs):
    """The workloads beside the headline one, each alone (for profiling)."""
    out = {}
    for name, fn in (("ladder", ladder_bench), ("tempering", tempering_bench), ("anneal", anneal_bench),
                     ("qsro", qsro_bench), ("fcc128", fcc128_bench), ("backward", backward_bench),
                     ("paper795", paper795_bench)):
        if name in legs:
            print(f"[bench] {name}", file=sys.stderr, flush=True)
            out[name] = fn(args)
    print(json.dumps({"legs": out}), flush=True)


def roofline(kernel, hbm_gbs, alu_tops, traffic, avg_launch_s, launches, bytes_per_launch, trials_per_launch,
             ops, swaps_per_s, n_ministeps):
    """The sweep kernel's bound.  The tile kernel re-reads every link cell of
    the lattice once per offset (HBM-bound); the row kernel reads it once per
    (o_y, o_z) group and is limited by its ALU work, so it is priced against
    the chip's 32-bit ALU lane-operation rate with the algorithmic operations
    per trial; the HBM figures are kept beside it."""
    hbm = {"achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": None if hbm_gbs is None else hbm_gbs / HBM_PEAK_GBS,
           "algorithmic_bytes_per_launch": bytes_per_launch,
           # bandwidth a one-launch-per-mini-step schedule (every byte re-read per
           # mini-step, 2 bytes written per trial) would need for this throughput
           "per_ministep_schedule_equivalent": swaps_per_s * (n_ministeps + 2.0) / 1e9}
    if traffic and avg_launch_s:
        # measured HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)
        hbm["measured_gbs"] = traffic / avg_launch_s / 1e9
        hbm["measured_frac"] = hbm["measured_gbs"] / HBM_PEAK_GBS
    hbm["half_peak_met"] = bool(hbm["frac"] is not None and hbm["frac"] >= 0.5)
    common = {"kernel": kernel, "avg_launch_us": avg_launch_s * 1e6, "launches": launches, "traffic": traffic}
    if kernel == "k_rows":
        return {"bound": "alu", "achieved": alu_tops, "peak": ALU_PEAK_TOPS, "unit": "Tops/s",
                "frac": alu_tops / ALU_PEAK_TOPS, "ops_per_trial": ops, "trials_per_launch": trials_per_launch,
                **common, "hbm": hbm}
    return {"bound": "hbm", "achieved": hbm["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm["frac"],
            "algorithmic_bytes_per_launch": bytes_per_launch, **common,
            "alu": {"achieved": alu_tops, "peak": ALU_PEAK_TOPS, "unit": "Tops/s", "ops_per_trial": ops}}


def ladder_bench(args):
    """Temperature ladder of 256 cubic BCC replicas with edges drawn from
    16..48 (4 species, 4 shells, T_r = 300 * 10^(r/255) K): attempted swaps/s
    of the batched launches (stream: one launch per mini-step group over all
    replicas; persistent: one launch for all sweeps; graph / stream_graph:
    those captured once and replayed; tuned: the autotuner's pick) against the
    plain loop that launches every replica's mini-steps one replica at a time
    (plain_graph: that loop captured and replayed)."""
    import torch
    from paper_2503_12591_amd import inputs as I
    from paper_2503_12591_amd import smcx
    lad = I.c4a_ladder()
    occ = np.concatenate([lad.occ(r) for r in range(lad.R)])
    N = int(occ.size)
    dims = lad.dims()
    occ_dev = torch.from_numpy(occ).cuda()

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    res = {}
    n = args.ladder_sweeps
    work = occ_dev.clone()
    lat = smcx.Lattice(I.BCC, dims, lad.K, lad.S, work, ell=4)
    lat.set_epi(lad.V)
    sweep_no = 0
    for mode, ns in (("plain", 2), ("stream", n), ("persistent", n)):  # stream: row windows where they apply
        bt = np.tile(lad.betas, (ns, 1))
        lat.sweep(1, 0, lad.betas.reshape(1, -1), first_sweep=sweep_no, mode=mode)  # warm-up
        sweep_no += 1
        secs = timed(lambda: lat.sweep(ns, 0, bt, first_sweep=sweep_no, mode=mode))
        sweep_no += ns
        res[mode] = ns * N / secs
    for key, mode, ns in (("graph", "persistent", n), ("stream_graph", "stream", n), ("plain_graph", "plain", 2)):
        g = smcx.LadderGraph(lat, ns, 0, lad.betas, first_sweep=sweep_no, mode=mode)
        g.launch()  # warm-up replay
        secs = timed(g.launch)
        res[key] = ns * N / secs
        sweep_no = int(g.counter.item())
        g.close()
    lat.close()
    # the batched stream launch of the plain loop's own kernel (tile windows,
    # one launch per mini-step group over all replicas): the gain of batching
    # alone, with the kernel held fixed
    work = occ_dev.clone()
    lat = smcx.Lattice(I.BCC, dims, lad.K, lad.S, work, ell=4, rows=False)
    lat.set_epi(lad.V)
    bt = np.tile(lad.betas, (n, 1))
    lat.sweep(1, 0, lad.betas.reshape(1, -1), mode="stream")
    res["stream_tiles"] = n * N / timed(lambda: lat.sweep(n, 0, bt, first_sweep=1, mode="stream"))
    lat.close()
    best = smcx.autotune(I.BCC, dims, lad.K, lad.S, occ_dev, lad.V, lad.betas, sweeps=2)
    work = occ_dev.clone()
    lat = smcx.Lattice(I.BCC, dims, lad.K, lad.S, work, ell=best["ell"], tile=best["tile"], rows=best["rows"])
    lat.set_epi(lad.V)
    bt = np.tile(lad.betas, (n, 1))
    lat.sweep(1, 0, lad.betas.reshape(1, -1), mode=best["mode"])
    secs = timed(lambda: lat.sweep(n, 0, bt, first_sweep=1, mode=best["mode"]))
    res["tuned"] = n * N / secs
    lat.close()
    batched = max(res["stream"], res["persistent"], res["graph"], res["stream_graph"], res["tuned"])
    return {"workload": "bcc_ladder256_L16to48_k4_s4", "sites": N, "sweeps": n,
            "unit": "attempted swaps/s", "swaps_per_s": res,
            "tuned_config": {"tile": best["tile"], "mode": best["mode"], "ell": best["ell"], "rows": best["rows"]},
            "batched_over_plain": batched / res["plain"],
            "batched_over_plain_graph": batched / res["plain_graph"],
            # same kernel (tile windows) in both: batching alone
            "batching_gain_same_kernel": res["stream_tiles"] / res["plain"]}


def tempering_bench(args, rounds: int = 4, sweeps_per_round: int = 5):
    """Replica exchange on 256 BCC 32^3 replicas (the ladder's temperatures
    and EPI): attempted swaps/s of whole rounds (sweeps of every replica at
    its slot's temperature, then smcx_exchange: pair counts, energies and one
    round of slot trades), the time of one exchange round on its own, and the
    fraction of slot trades taken."""
    import torch
    from paper_2503_12591_amd import inputs as I
    from paper_2503_12591_amd import smcx
    lad = I.tempering_ladder()
    occ = torch.from_numpy(np.concatenate([lad.occ(r) for r in range(lad.R)])).cuda()
    N = int(occ.numel())
    lat = smcx.Lattice(I.BCC, lad.dims(), lad.K, lad.S, occ, ell=4)
    lat.set_epi(lad.V)
    pt = smcx.Tempering(lat, lad.betas, seed=0, sweeps_per_round=sweeps_per_round, mode="stream")
    pt.run(1)  # warm-up round

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    secs = timed(lambda: pt.run(rounds))
    x0 = pt.xstats.cpu().numpy().reshape(-1, 2).sum(axis=0)
    # one exchange round alone (it only permutes slots; the next sweeps would read its betas)
    ex = timed(lambda: smcx._check(smcx.lib().smcx_exchange(
        lat.h, pt.round, 0, smcx._ptr(pt.beta_slot), smcx._ptr(pt.rep_at), smcx._ptr(pt.beta_rows),
        pt.n, smcx._ptr(lat.counts), smcx._ptr(pt.E), smcx._ptr(pt.xstats), smcx._ptr(pt.ties),
        pt.tie_cap, smcx._ptr(pt.tie_count), smcx._stream(torch))))
    lat.close()
    return {"workload": "bcc_tempering256_L32_k4_s4", "sites": N, "rounds": rounds,
            "sweeps_per_round": sweeps_per_round, "unit": "attempted swaps/s",
            "swaps_per_s": rounds * sweeps_per_round * N / secs, "exchange_round_us": ex * 1e6,
            "trade_fraction": float(x0[1] / max(x0[0], 1))}


def anneal_bench(args, warmup: int = 5, record: int = 5):
    """Stepwise anneal of the BCC 64^3 lattice (4 species, 4 shells) from
    2000 K down to 300 K in 50 K steps, `warmup` sweeps then `record` sweeps
    with energies per temperature and the heat capacity of every step
    (smcx_anneal): attempted swaps/s of the whole protocol and the time of the
    same sweeps in one call without recording (the difference is the cost of
    the energy records).  A throughput measurement: with a few sweeps per
    temperature the heat capacities are not equilibrium values."""
    import torch
    from paper_2503_12591_amd import inputs as I
    from paper_2503_12591_amd import smcx
    wl = I.c2_anneal_bcc()
    T = I.stepwise_temperatures(2000.0, 300.0, 50.0)
    beta = I.beta_of_T(T)
    occ = torch.from_numpy(wl.occ()).cuda()
    lat = smcx.Lattice(wl.lattice, wl.dims, wl.K, wl.S, occ, ell=4)
    lat.set_epi(wl.V)
    lat.anneal(beta[:1], 1, 1, seed=0, mode="stream")  # warm-up

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        r = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3, r

    per = warmup + record
    secs, out = timed(lambda: lat.anneal(beta, warmup, record, seed=0, first_sweep=2, mode="stream"))
    bt = np.repeat(beta, per).reshape(-1, 1)
    plain, _ = timed(lambda: lat.sweep(len(bt), 0, bt, first_sweep=2 + len(bt), mode="stream"))
    lat.close()
    n_sweeps = len(T) * per
    return {"workload": "bcc64_k4_s4_anneal2000to300_step50", "sites": wl.N, "temperatures": len(T),
            "warmup": warmup, "record": record, "unit": "attempted swaps/s",
            "swaps_per_s": n_sweeps * wl.N / secs, "ms": secs * 1e3,
            "sweeps_only_ms": plain * 1e3, "records": len(T) * record}


def clusters_bench(lat, N):
    """The paper's analysis step on the benchmark lattice as the timed steps
    left it: per-site local energies (smcx_local_energy), then the clusters of
    the sites at or below the 15 % quantile of the local energy
    (smcx_clusters: union-find over nearest neighbours).  Local energies move
    9 algorithmic bytes per site (1 read, 8 written)."""
    import torch

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        r = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3, r

    e = lat.local_energy()  # warm-up
    t_e, e = timed(lambda: lat.local_energy(e=e))
    thr = float(torch.quantile(e[::4096].float(), 0.15).item())
    lat.clusters(thr, e=e)  # warm-up
    t_c, (label, size, nc) = timed(lambda: lat.clusters(thr, e=e))
    out = {"workload": "local energies and clusters of the benchmark lattice (threshold: 15 % quantile)",
           "sites": N, "local_energy_ms": t_e * 1e3, "local_energy_GBps": 9.0 * N / t_e / 1e9,
           "clusters_ms": t_c * 1e3, "sites_per_s": N / t_c,
           "marked_fraction": float((label >= 0).sum().item()) / N, "clusters": int(nc.item()),
           "largest": int(size.max().item())}
    del e, label, size
    return out


def qsro_bench(args, sweeps: int = 2):
    """The qSRO model on FCC 64^3 (5 species, 2 shells, 1000 K, link cells of
    4, the interaction-zone minimum): attempted swaps/s of qSRO sweeps
    (smcx_sweep_qsro: a wave per trial over its affected set) beside EPI
    sweeps of the same lattice and partition; their ratio is the cost of
    the nonlinear model per trial."""
    import torch
    from paper_2503_12591_amd import inputs as I
    from paper_2503_12591_amd import smcx
    dims, counts, V, W, beta = I.qsro_fcc()
    occ = I.occupancy(counts, seed=0)
    N = len(occ)
    lat = smcx.Lattice(I.FCC, dims, 5, 2, occ, ell=4)
    lat.set_qsro(V, W)
    lat.set_epi(V)

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    lat.sweep_qsro(1, 0, [beta])  # warm-up
    tq = timed(lambda: lat.sweep_qsro(sweeps, 0, [beta] * sweeps, first_sweep=1))
    bt = np.full((sweeps, 1), beta)
    lat.sweep(1, 0, bt[:1], first_sweep=1 + sweeps)
    te = timed(lambda: lat.sweep(sweeps, 0, bt, first_sweep=2 + sweeps))
    lat.close()
    return {"workload": "fcc64_k5_s2_T1000_qsro", "sites": N, "sweeps": sweeps, "unit": "attempted swaps/s",
            "qsro_swaps_per_s": sweeps * N / tq, "epi_swaps_per_s_same_lattice": sweeps * N / te,
            "qsro_cost_over_epi": te and tq / te}


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    r = fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3, r


def fcc128_bench(args, sweeps: int = 10):
    """FCC 128^3 (8.4e6 sites, 5 species 0.28/0.28/0.28/0.08/0.08, 4 shells,
    800 K): attempted swaps/s of 10 sweeps followed by the energy and SRO
    measurement the workload takes every 10 sweeps."""
    import torch
    from paper_2503_12591_amd import inputs as I
    from paper_2503_12591_amd import smcx
    w = I.c3_fcc()
    lat = smcx.Lattice(w.lattice, w.dims, w.K, w.S, w.occ(), ell=4)
    lat.set_epi(w.V)
    bt = w.betas[:sweeps].reshape(-1, 1)
    lat.sweep(1, 0, bt[:1])
    lat.sro()

    def step():
        lat.sweep(sweeps, 0, bt, first_sweep=1)
        return lat.sro()

    secs, _ = _timed(step)
    lat.close()
    return {"workload": w.name, "sites": w.N, "sweeps": sweeps, "unit": "attempted swaps/s",
            "swaps_per_s": sweeps * w.N / secs, "ms": secs * 1e3}


def paper795_bench(args, sweeps: int = 4):
    """The paper's own large lattice shape (Tab. 4, MoNbTaW_1B_EPI: BCC 795^3,
    1.005e9 sites) with synthetic inputs (4 species equiatomic, V ~ N(0,
    0.02 eV), 1200 K): (a) the paper's link cells of 3 with 2 shells (54
    mini-steps per sweep), (b) 4 shells, whose link cells must be at least 4
    (795 = 195 x 4 + 3 x 5: uneven cells, 250 mini-steps).  Attempted swaps/s
    of `sweeps` timed sweeps after one warm-up sweep, and the row kernel's
    average launch."""
    import torch
    from paper_2503_12591_amd import inputs as I
    from paper_2503_12591_amd import smcx
    out = {"unit": "attempted swaps/s", "sweeps": sweeps}
    occ = None
    for name, S, ell in (("s2_ell3", 2, 3), ("s4_ell4", 4, 4)):
        w = I.paper_large_bcc(S)
        if occ is None:
            occ = I.occupancy_device(w.counts, seed=w.occ_seed)
            out["sites"] = w.N
        lat = smcx.Lattice(w.lattice, w.dims, w.K, w.S, occ.clone(), ell=ell)
        lat.set_epi(w.V)
        cells, nA = lat.schedule(0)
        betas = torch.full((sweeps, 1), float(w.betas[0]), dtype=torch.float64, device="cuda")
        lat.sweep(1, 0, betas[:1], mode="stream")
        lat.timing(True)
        lat.timing_read()
        secs, _ = _timed(lambda: lat.sweep(sweeps, 0, betas, first_sweep=1, mode="stream"))
        kern_ms, launches = lat.timing_read()
        lat.timing(False)
        avg_s = kern_ms / 1e3 / max(launches, 1)
        trials_per_launch = w.N * sweeps / max(launches, 1)
        ops = algorithmic_ops_per_trial(w.lattice, w.K, w.S)
        out[name] = {"workload": w.name, "shells": S, "link_cell": ell, "n_ministeps": nA,
                     "cells_per_axis": [len(c) for c in cells], "swaps_per_s": sweeps * w.N / secs,
                     "ms_per_sweep": secs * 1e3 / sweeps, "launches_per_sweep": launches / sweeps,
                     "avg_launch_us": avg_s * 1e6, "ops_per_trial": ops,
                     "alu_frac": trials_per_launch * ops / avg_s / 1e12 / ALU_PEAK_TOPS}
        lat.close()
    return out


def backward_bench(args):
    """energy_backward (batched pair counts, dE/dV = C / 2) at the workloads'
    batch sizes: 64 snapshots of BCC 64^3 (3.4e7 sites) and 4096
    configurations of BCC 16^3 (the fit set, 3.4e7 sites); one byte per site
    read, so the rate is in sites/s and GB/s."""
    import torch
    from paper_2503_12591_amd import inputs as I
    from paper_2503_12591_amd import smcx
    out = {"unit": "sites/s"}
    for name, dims, B in (("bcc64_snapshots64", (64, 64, 64), 64), ("bcc16_fit4096", (16, 16, 16), 4096)):
        N = I.n_sites(I.BCC, dims)
        g = torch.Generator(device="cuda")
        g.manual_seed(7)
        batch = torch.randint(0, 4, (B, N), dtype=torch.uint8, device="cuda", generator=g)
        smcx.energy_backward_counts(I.BCC, dims, 4, 4, batch)  # warm-up
        secs, _ = _timed(lambda: smcx.energy_backward_counts(I.BCC, dims, 4, 4, batch))
        out[name] = {"sites": B * N, "ms": secs * 1e3, "sites_per_s": B * N / secs, "GBps": B * N / secs / 1e9}
        del batch
    return out


def algorithmic_bytes_per_launch(cells, N, m, launches_per_sweep):
    """Average algorithmic HBM bytes of one sweep launch.  The mini-steps of
    one offset o read every occupancy byte of the link cells that have o (the
    LIZ+ regions of their active sites cover those cells) -- once per launch,
    since a launch covers consecutive basis sites of one o -- and every trial
    writes at most 2 bytes (2N per sweep).  With uniform cells and all m basis
    sites in one launch that is N + 2 m n_C."""
    M = [int(max(c)) for c in cells]
    n_o = M[0] * M[1] * M[2]
    reads = 0.0
    for oz in range(M[2]):
        for oy in range(M[1]):
            for ox in range(M[0]):
                act = [(np.asarray(cells[a]) > o).sum() for a, o in enumerate((ox, oy, oz))]
                reads += np.prod([act[a] / len(cells[a]) for a in range(3)]) * N
    per_sweep = reads * (launches_per_sweep / n_o) + 2 * N
    return per_sweep / launches_per_sweep


def kernel_fingerprint() -> str:
    """Hash of the kernel sources; counter data is only valid for the build it
    was taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("smcx_kernels.hip", "smcx_internal.h"):
        with open(os.path.join(ROOT, "paper_2503_12591_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# --------------------------------------------------------------------------
# rocprofv3 csv -> short text summaries under profiles/
# --------------------------------------------------------------------------
def _csv(d, suffix):
    import csv
    import glob
    fs = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not fs:
        raise SystemExit(f"no *{suffix} under {d}")
    with open(fs[0]) as f:
        return list(csv.DictReader(f))


def _per_dispatch(d, counter, match):
    """Average value of a counter over the dispatches whose kernel name contains
    `match` (one row per dispatch and counter)."""
    vals = [float(r["Counter_Value"]) for r in _csv(d, "counter_collection.csv")
            if r["Counter_Name"] == counter and match(r["Kernel_Name"])]
    if not vals:
        raise SystemExit(f"no {counter} rows in {d}")
    return sum(vals) / len(vals), len(vals)


def _copy_factor(d, counter, nbytes=1 << 30):
    """True bytes per counted byte, from the largest dispatch of the copy probe."""
    rows = [r for r in _csv(d, "counter_collection.csv") if r["Counter_Name"] == counter]
    kib = max(float(r["Counter_Value"]) for r in rows)
    return nbytes / (kib * 1024.0), kib


def summarize(args):
    kind, rest = args.summarize[0], args.summarize[1:]
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    tag = f"bcc{args.edge}_ell{args.ell}"
    if kind == "trace":
        d, cmd = rest[0], " ".join(rest[1:])
        rows = _csv(d, "kernel_stats.csv")
        rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
        title = args.profile_name or f"BCC {args.edge}^3 benchmark, link cell {args.ell}"
        lines = [f"# rocprofv3 kernel trace: {title}",
                 f"# command: {cmd}", "",
                 f"{'calls':>7} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'total_ms':>10} {'pct':>6}  kernel"]
        for r in rows:
            name = r["Name"]
            if len(name) > 110:
                name = name[:107] + "..."
            lines.append(f"{int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.1f} "
                         f"{float(r['MinNs']) / 1e3:10.1f} {float(r['MaxNs']) / 1e3:10.1f} "
                         f"{float(r['TotalDurationNs']) / 1e6:10.2f} {float(r['Percentage']):6.2f}  {name}")
        stem = args.profile_name.replace(" ", "_") if args.profile_name else f"sweep_{tag}"
        with open(os.path.join(ROOT, "profiles", f"{stem}_kernel_trace.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")
    elif kind == "traffic":
        fd, wd, cfd, cwd, cmd = rest[0], rest[1], rest[2], rest[3], " ".join(rest[4:])
        names = {r["Kernel_Name"] for r in _csv(fd, "counter_collection.csv")}
        kname = "k_rows" if any("k_rows" in n for n in names) else "k_ministep"
        tag = f"{kname[2:]}_bcc{args.edge}_ell{args.ell}"
        is_k = lambda n: kname in n
        fk, nf = _per_dispatch(fd, "FETCH_SIZE", is_k)
        wk, nw = _per_dispatch(wd, "WRITE_SIZE", is_k)
        ff, fcopy = _copy_factor(cfd, "FETCH_SIZE")
        fw, wcopy = _copy_factor(cwd, "WRITE_SIZE")
        rd = fk * 1024 * ff
        wr = wk * 1024 * fw
        lines = [f"# HBM traffic of {kname}: BCC {args.edge}^3 benchmark, link cell {args.ell}",
                 f"# command (one pass per counter): {cmd}",
                 "# calibration: bench.py --copy-probe (torch copy of 1 GiB) under the same counters", "",
                 f"FETCH_SIZE per dispatch (KiB, avg over {nf}): {fk:.1f}",
                 f"WRITE_SIZE per dispatch (KiB, avg over {nw}): {wk:.1f}",
                 f"copy probe FETCH_SIZE (KiB) for 1 GiB read: {fcopy:.1f} -> factor {ff:.4f}",
                 f"copy probe WRITE_SIZE (KiB) for 1 GiB written: {wcopy:.1f} -> factor {fw:.4f}",
                 f"scaled read bytes per launch: {rd:.4e}",
                 f"scaled write bytes per launch: {wr:.4e}",
                 f"scaled HBM bytes per launch: {rd + wr:.4e}"]
        with open(os.path.join(ROOT, "profiles", f"{tag}_traffic.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")
        with open(os.path.join(ROOT, "profiles", f"traffic_{tag}.json"), "w") as f:
            json.dump({"bytes_per_launch": rd + wr, "read_bytes": rd, "write_bytes": wr,
                       "kernel_build": kernel_fingerprint(), "command": cmd}, f, indent=1)
    elif kind == "traffic-all":
        # HBM traffic of every library kernel in the same counter runs, with
        # its algorithmic bytes where they have a plain definition
        fd, wd, cfd, cwd, cmd = rest[0], rest[1], rest[2], rest[3], " ".join(rest[4:])
        ff, _ = _copy_factor(cfd, "FETCH_SIZE")
        fw, _ = _copy_factor(cwd, "WRITE_SIZE")
        names = sorted({r["Kernel_Name"] for r in _csv(fd, "counter_collection.csv") if "smcx::" in r["Kernel_Name"]})
        N = 2 * args.edge ** 3
        algo = {"k_pair_counts_slab": (N, 0), "k_pair_counts_tiled": (N, 0), "k_pack": (N, None), "k_unpack": (None, N),
                "k_validate": (N, 0)}
        lines = [f"# HBM traffic of every library kernel: BCC {args.edge}^3 benchmark, link cell {args.ell}",
                 f"# command (one pass per counter): {cmd}",
                 "# FETCH_SIZE x 2.0 and WRITE_SIZE x 1.0 (copy-probe calibration), per dispatch; algorithmic",
                 "# bytes: the lattice read (pair counts, pack, validate) or written (unpack), N = sites", "",
                 f"{'kernel':58s} {'read GB':>9s} {'write GB':>9s} {'read / N':>9s}"]
        for n in names:
            short = n.split("(")[0].replace("void ", "")
            rd = _per_dispatch(fd, "FETCH_SIZE", lambda k, n=n: k == n)[0] * 1024 * ff
            wr = _per_dispatch(wd, "WRITE_SIZE", lambda k, n=n: k == n)[0] * 1024 * fw
            base = short.split("::")[-1].split("<")[0]
            ratio = f"{rd / N:9.2f}" if base in algo and algo[base][0] else f"{'':9s}"
            lines.append(f"{short[:58]:58s} {rd / 1e9:9.3f} {wr / 1e9:9.3f} {ratio}")
        with open(os.path.join(ROOT, "profiles", f"kernels_{tag}_traffic.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")
    elif kind == "counters":
        # rest: counter-pass directories, then the command
        dirs = [d for d in rest if os.path.isdir(d)]
        cmd = " ".join(r for r in rest if r not in dirs)
        vals, kname, ndisp = {}, None, 0
        for d in dirs:
            rows = _csv(d, "counter_collection.csv")
            names = {r["Kernel_Name"] for r in rows}
            kname = "k_rows" if any("k_rows" in n for n in names) else "k_ministep"
            per = {}
            for r in rows:
                if kname in r["Kernel_Name"]:
                    per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
            for c, v in per.items():
                vals[c] = sum(v) / len(v)
                ndisp = len(v)
        trials = args.edge ** 3 * 2  # one sweep of the benchmark lattice
        lines = [f"# SQ counters of {kname}: BCC {args.edge}^3 benchmark, link cell {args.ell}",
                 f"# command (one pass per group of counters): {cmd}",
                 "# device totals per dispatch; 'per wave-trial' divides by the dispatch's trials / 64", "",
                 f"{'counter':28s} {'per dispatch':>16s} {'per wave-trial':>15s}"]
        for c in sorted(vals):
            per_wt = vals[c] / (trials / ndisp / 64) if ndisp else float("nan")
            lines.append(f"{c:28s} {vals[c]:16.1f} {per_wt:15.2f}")
        if "SQ_LDS_BANK_CONFLICT" in vals and "SQ_LDS_IDX_ACTIVE" in vals:
            lines.append(f"\nLDS bank-conflict cycles / LDS active cycles: "
                         f"{vals['SQ_LDS_BANK_CONFLICT'] / vals['SQ_LDS_IDX_ACTIVE']:.3f}")
        with open(os.path.join(ROOT, "profiles", f"{kname[2:]}_{tag}_sq_counters.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")
    elif kind == "counters-all":
        # rest: counter-pass directories, then the command; every library
        # kernel of the run, counters averaged per dispatch and per wave
        dirs = [d for d in rest if os.path.isdir(d)]
        cmd = " ".join(r for r in rest if r not in dirs)
        per = {}
        for d in dirs:
            for r in _csv(d, "counter_collection.csv"):
                if "smcx::" not in r["Kernel_Name"]:
                    continue
                k = r["Kernel_Name"].split("(")[0].replace("void ", "")
                per.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        title = args.profile_name or "library kernels"
        lines = [f"# SQ counters of every library kernel: {title}",
                 f"# command (one pass per group of counters): {cmd}",
                 "# per dispatch: device totals averaged over the kernel's dispatches; per wave: divided by SQ_WAVES", ""]
        for k in sorted(per):
            c = {n: sum(v) / len(v) for n, v in per[k].items()}
            nd = max(len(v) for v in per[k].values())
            waves = c.get("SQ_WAVES", 0.0)
            lines.append(f"{k}  ({nd} dispatches)")
            for n in sorted(c):
                pw = f"{c[n] / waves:14.2f}" if waves else ""
                lines.append(f"  {n:26s} {c[n]:16.1f} {pw}")
            if "SQ_LDS_BANK_CONFLICT" in c and c.get("SQ_LDS_IDX_ACTIVE"):
                lines.append(f"  LDS bank-conflict cycles / LDS active cycles: "
                             f"{c['SQ_LDS_BANK_CONFLICT'] / c['SQ_LDS_IDX_ACTIVE']:.3f}")
            lines.append("")
        stem = args.profile_name.replace(" ", "_") if args.profile_name else "kernels"
        with open(os.path.join(ROOT, "profiles", f"{stem}_sq_counters.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")
    else:
        raise SystemExit(f"unknown summary kind {kind}")


if __name__ == "__main__":
    main()
