#!/usr/bin/env python3
"""Benchmark of the all-pairs N-body hot path on one MI355X.

Headline workload: softened gravity on a Plummer sphere, N = 1,048,576
(seed 5, eps = 0.005, G = 1, equal masses 1/N), FP32 pair arithmetic with
Kahan-compensated accumulation.  One timed step is one kick-drift-kick
leapfrog step in FP64 (pack + kick/drift, the all-pairs force and potential
evaluation with its FP64 finalize, and the closing kick) -- N^2 ordered pair
interactions.  The launch configuration comes from the autotuner, run before
the timed region (the rule's choice at this size: the symmetric pair tiles, which
evaluate each unordered pair once and apply it to both particles).

Printed (one JSON line on stdout):
  * interactions per second of the headline step;
  * the roofline of the all-pairs kernel (algorithmic flops per launch / its mean
    launch time, measured with HIP events on the launch stream) and its HBM traffic
    from the committed counter record;
  * the issue-rate ceiling of the pair sequence from the library's probes;
  * the oracle timed on a bounded row sample on the host cores;
  * the accuracy of the timed path against the FP64 GPU pass and the oracle;
and, by default, secondary legs: one GPU's share of the headline evaluation if its
rows were sharded over 8 GPUs (N/8 rows against all N j records); the batched
ensemble (256 LJC systems, N_s in
[500, 5000], one persistent launch vs one launch per system, each side autotuned);
the position adjoint at N = 262,144 (FP32 vs FP64); every pair law of Table 1 at
N = 65,536; the acceleration-and-jerk kernel and the block-time-step Hermite
integrator on a Plummer sphere of 65,536; bonded chains with exclusion lists
(N = 8192); the batched adjoint of the 256-system ensemble; 100 leapfrog steps at
N = 65,536 with their energy drift; and the oracle timed in full on the small
configurations.
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

PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector: 256 CUs x 256 flops/cycle/CU x 2.4 GHz
N_MAIN = 1 << 20
EPS_MAIN = 0.005
DT = 1e-3
N_LAWS = 65536
# sigmoidal dielectric zeta(r) = exp(a r^3 + b r^2 + c r + d): 4.6 at 5 A, about 100 at 20 A
ZETA_SIGMOIDAL = (2e-4, -6e-3, 0.25, 0.4)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=N_MAIN, help="particles of the headline workload")
    ap.add_argument("--legs", default="all", choices=["all", "main", "laws", "batched", "jerk", "backward"],
                    help="'main' runs only the headline workload (for counter runs), 'laws' the "
                         "headline workload and the per-law leg, 'batched' the headline workload "
                         "and the batched forward and backward legs, 'jerk' the headline workload "
                         "and the acceleration-and-jerk leg, 'backward' the headline workload and "
                         "the single-system adjoints")
    ap.add_argument("--no-tune", action="store_true", help="use the heuristic configuration")
    ap.add_argument("--launch", default=None, metavar="BLOCK,IPL,JTILE,SPLIT,STAGE",
                    help="force the headline kernel's launch configuration (for counter runs of one "
                         "configuration); implies no autotuning")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target host time of the oracle sample")
    ap.add_argument("--save-inputs", default=None, metavar="DIR",
                    help="also write the drawn inputs (headline Plummer sphere; with the default "
                         "legs the ensemble and the per-law MD box) as .npy files into DIR")
    ap.add_argument("--make-traffic", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "BENCH_JSON"),
                    help="no GPU work: write the traffic record of the headline kernel from the "
                         "counter CSVs of two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "'bench.py --legs main' and the JSON line one of them printed")
    args = ap.parse_args()
    if args.make_traffic:
        make_traffic(*args.make_traffic)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        msg = ("bench.py measures one GPU: the library has no multi-GPU path (the forward would "
               "shard the i range and all-gather the FP32 j records; the shard_share leg times "
               "one GPU's share). Run with --gpus 1.")
        log(msg)
        if int(os.environ.get("RANK", "0")) == 0:
            print(json.dumps({"error": msg, "n_gpus": args.gpus}))
        sys.exit(2)

    from paper_0706_3060_amd import workloads as W

    # ---- inputs drawn before any GPU work (the ensemble uses a fork pool)
    t0 = time.time()
    pos, vel, mass = W.plummer(args.n, 5)
    ens = W.batched_md(256, seed=4) if args.legs in ("all", "batched") else None
    md = (W.md_system(N_LAWS, 3, box=(32.0 * N_LAWS) ** (1.0 / 3.0)) if args.legs in ("all", "laws", "backward")
          else None)
    chains = W.bonded_chains(256, 32, 3) if args.legs == "all" else None
    log("inputs drawn in %.1f s" % (time.time() - t0))
    if args.save_inputs:
        save_inputs(args.save_inputs, args.n, pos, vel, mass, ens, md)

    import torch
    from paper_0706_3060_amd import nbody as nb

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    props = torch.cuda.get_device_properties(dev)
    log("device:", props.name, "CUs:", props.multi_processor_count)

    # calibration copy of known size (bytes moved are known exactly; used to
    # scale hardware traffic counters in counter runs)
    cal = torch.empty(64 << 20, dtype=torch.float32, device=dev)   # 256 MiB
    cal2 = cal.clone()
    del cal, cal2

    n = args.n
    x = torch.tensor(pos, device=dev)
    v = torch.tensor(vel, device=dev)
    m = torch.tensor(mass, device=dev)
    law = nb.gravity("fp32_kahan", softening=EPS_MAIN)
    law64 = nb.gravity("fp64", softening=EPS_MAIN)

    # ---- accuracy of the timed precision at t = 0 (FP64 GPU pass over all N,
    #      oracle on a random row sample)
    if args.launch:
        b, ipl, jt, sp, js = (int(v) for v in args.launch.split(","))
        for api in (nb.API_FORCES, nb.API_LEAPFROG):
            nb.set_config(api, b, ipl, jt, sp, js)
        log("forced forces config:", args.launch)
    elif not args.no_tune:
        cfg, tune_ms = nb.autotune(x, m, law, potential=True)
        log("autotuned forces config:", cfg, "%.2f ms" % tune_ms)
    a32, p32 = nb.forces(x, m, law)
    a64, p64 = nb.forces(x, m, law64)
    torch.cuda.synchronize()
    e = (torch.linalg.norm(a32 - a64, dim=1) / torch.linalg.norm(a64, dim=1)).cpu().numpy()
    ep = ((p32 - p64).abs() / p64.abs()).cpu().numpy()
    acc = {"fp32_kahan_vs_fp64_gpu": {"median": float(np.median(e)), "p99": float(np.quantile(e, 0.99)),
                                      "max": float(e.max()), "potential_median": float(np.median(ep)),
                                      "potential_max": float(ep.max())}}
    log("fp32 vs fp64 gpu:", acc["fp32_kahan_vs_fp64_gpu"])

    # ---- timed region: K leapfrog steps (inputs resident in HBM)
    acc_t = a32.clone()
    for _ in range(args.warmup):
        nb.leapfrog(x, v, acc_t, m, law, DT, 1, potential=True)     # the timed step's own work
    torch.cuda.synchronize()
    nb.timing_read(reset=True)
    nb.timing_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        nb.leapfrog(x, v, acc_t, m, law, DT, 1, potential=True)
    torch.cuda.synchronize()
    t_el = time.perf_counter() - t_start
    nb.timing_enable(False)
    k_ms, k_launches = nb.timing_read(reset=True)
    ms_step = 1e3 * t_el / args.steps
    pairs = float(n) * float(n)
    value = pairs / (t_el / args.steps) / 1e9
    flops_pair = nb.flops_per_pair(nb.API_FORCES, nb.GRAVITY, True)
    k_avg_s = (k_ms / max(k_launches, 1)) * 1e-3
    achieved = flops_pair * pairs / k_avg_s / 1e12
    cfg_used = nb.get_config(nb.API_LEAPFROG, n, law)
    log("step %.3f ms, %.1f G pairs/s; all-pairs kernel %.3f ms/launch over %d launches, %.2f TFLOP/s"
        % (ms_step, value, k_ms / max(k_launches, 1), k_launches, achieved))

    # issue-rate ceiling of the timed kernel's instruction sequence, measured on this GPU,
    # per interaction-wave (64 interactions of 20 flops against 64 flops per SIMD-cycle at
    # peak; 157.3 TFLOP/s is that at 2.4 GHz).  Symmetric pair tiles (j_stage 2): one
    # unordered pair-wave is 18 ordinary FP32 VALU instructions, one v_rsq_f32 and half a
    # DPP move (the potential's j sum; the force sums move through the LDS crossbar, off
    # the VALU) for two interactions; one-sided kernels: 13 ordinary instructions and one
    # v_rsq_f32 for one interaction.  The clock under the pair kernel
    # is not visible here: clock_for_kernel_ghz is the clock at which the measured launch
    # time equals the modelled cycles.
    rates = nb.probe_issue_rates(dev)
    if cfg_used["j_stage"] == 2:
        inter_cycles = (18 * rates["fma_cycles"] + rates["rsq_cycles"] + 0.5 * rates["dpp_mov_cycles"]) / 2.0
        model = "symmetric: (18 VALU + 1 rsq + 0.5 DPP move) per unordered pair-wave, two interactions"
    else:
        inter_cycles = 13 * rates["fma_cycles"] + rates["rsq_cycles"]
        model = "one-sided: 13 VALU + 1 rsq per interaction-wave"
    inter_waves_per_simd = pairs / 64.0 / (4 * props.multi_processor_count)
    ceiling = {"probe": rates, "model": model, "interaction_wave_cycles_model": inter_cycles,
               "cap_frac_of_clock_peak": 20.0 / inter_cycles,
               "clock_for_kernel_ghz": inter_cycles * inter_waves_per_simd / k_avg_s / 1e9}
    log("ceiling:", ceiling)

    # oracle on a row sample of the same (t = 0) workload, same FP32-rounded inputs
    import oracle
    rng = np.random.default_rng(55)
    rows = np.sort(rng.choice(n, 256, replace=False))
    xr = W.round_to_f32(pos)
    mr = W.round_to_f32(mass)
    t1 = time.perf_counter()
    a_ref, phi_ref = oracle.gravity(xr, mr, eps=EPS_MAIN, ilist=rows)
    t_cal = time.perf_counter() - t1
    e_or = np.linalg.norm(a32.cpu().numpy()[rows] - a_ref, axis=1) / np.linalg.norm(a_ref, axis=1)
    a64_or, _ = oracle.gravity(pos, mass, eps=EPS_MAIN, ilist=rows)
    e64_or = np.linalg.norm(a64.cpu().numpy()[rows] - a64_or, axis=1) / np.linalg.norm(a64_or, axis=1)
    acc["fp32_kahan_vs_oracle_sample"] = {"rows": int(rows.size), "median": float(np.median(e_or)),
                                          "max": float(e_or.max())}
    acc["fp64_gpu_vs_oracle_sample"] = {"rows": int(rows.size), "max": float(e64_or.max())}

    # cpu baseline: the oracle as it stands, on a bounded row sample sized to ~cpu_seconds
    rate = rows.size * n / t_cal
    k_rows = int(max(256, min(n, args.cpu_seconds * rate / n)))
    sample = np.sort(rng.choice(n, k_rows, replace=False))
    threads = oracle.threads(0)
    t1 = time.perf_counter()
    oracle.gravity(pos, mass, eps=EPS_MAIN, ilist=sample)
    t_cpu = time.perf_counter() - t1
    cpu_value = k_rows * n / t_cpu / 1e9
    log("oracle: %d rows x %d in %.1f s on %d threads = %.3f G pairs/s" % (k_rows, n, t_cpu, threads, cpu_value))
    # the same oracle on one thread, on a sample of about a tenth of the time
    k1 = int(max(16, min(n, 0.1 * args.cpu_seconds * rate / n / max(threads, 1))))
    t1 = time.perf_counter()
    oracle.gravity(pos, mass, eps=EPS_MAIN, ilist=sample[:k1], nthreads=1)
    t_one = time.perf_counter() - t1
    one_value = k1 * n / t_one / 1e9
    host = {"nproc": os.cpu_count(), "cpu_model": _cpu_model()}
    log("oracle on one thread: %d rows in %.1f s = %.4f G pairs/s; host %s" % (k1, t_one, one_value, host))

    traffic = measured_traffic(n, cfg_used)
    out = {
        "metric": "G pair-interactions/s & %FP32 VALU peak, N=1M; batched vs loop @1e-5 err",
        "value": value,
        "unit": "G pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plummer_gravity_kdk_step", "n": n, "softening": EPS_MAIN,
                   "G": 1.0, "dt": DT, "seed": 5, "precision": "fp32_kahan",
                   "pairs_per_step": pairs, "flops_per_pair": flops_pair,
                   "launch": cfg_used, "parallelism": "single_gpu"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "kernel_ms": k_ms / max(k_launches, 1), "launches": k_launches},
        "ceiling": ceiling,
        "cpu_baseline": {"value": cpu_value, "unit": "G pair-interactions/s", "cores": threads,
                         "kind": "oracle",
                         "sample": "%d random rows of the N=%d Plummer workload against all N "
                                   "(FP64 oracle, compensated sums), %.1f s" % (k_rows, n, t_cpu),
                         "one_thread_value": one_value, "one_thread_sample_rows": k1, "host": host,
                         "extrapolated_full_evaluation_s": pairs / (cpu_value * 1e9),
                         "extrapolated_full_evaluation_note": "N^2 pairs at the sampled rate, "
                                                              "extrapolated, not timed"},
        "accuracy": acc,
    }

    if args.legs == "all":
        out["shard_share"] = shard_leg(nb, torch, dev, x, m, law, k_ms / max(k_launches, 1))
        out["batched"] = batched_leg(nb, torch, dev, ens)
        out["backward"] = backward_leg(nb, torch, dev, W, md)
        out["laws"] = laws_leg(nb, torch, dev, W, md)
        out["jerk"] = jerk_leg(nb, torch, dev, W, not args.no_tune)
        out["bonded"] = bonded_leg(nb, torch, dev, W, chains)
        out["batched_backward"] = batched_backward_leg(nb, torch, dev, ens)
        out["leapfrog_100"] = leapfrog_leg(nb, torch, dev, W)
        out["oracle_configs"] = oracle_configs_leg(nb, torch, dev, W, ens, out)
    elif args.legs == "laws":
        out["laws"] = laws_leg(nb, torch, dev, W, md)
    elif args.legs == "batched":
        out["batched"] = batched_leg(nb, torch, dev, ens)
        out["batched_backward"] = batched_backward_leg(nb, torch, dev, ens)
    elif args.legs == "jerk":
        out["jerk"] = jerk_leg(nb, torch, dev, W, not args.no_tune)
    elif args.legs == "backward":
        out["backward"] = backward_leg(nb, torch, dev, W, md)
    print(json.dumps(out), flush=True)


TRAFFIC_SOURCES = ["paper_0706_3060_amd/csrc/forward.hip", "paper_0706_3060_amd/csrc/device.h",
                   "paper_0706_3060_amd/csrc/allpairs.h", "paper_0706_3060_amd/csrc/kernels.h",
                   "paper_0706_3060_amd/csrc/symmetric.hip"]


def timed_kernel(n, cfg):
    """Name and grid (work-items) of the all-pairs launch of the headline configuration:
    the symmetric pair tiles (j_stage 2; one 512-thread workgroup per tile of the block
    grid's upper triangle, the count padded to a multiple of the 8 XCDs) or the one-sided
    forces kernel."""
    if cfg["j_stage"] == 2:
        rec = cfg["j_tile"]
        nblk = -(-n // rec)
        tiles = nblk * (nblk + 1) // 2
        waves = cfg["block"] // 64
        return ("k_sym<0, 1, true, %d, %d>" % (waves, cfg["i_per_lane"]),
                str(-(-tiles // 8) * 8 * cfg["block"]))              # padded to the 8 XCDs
    waves = -(-n // (64 * cfg["i_per_lane"]))
    wpb = cfg["block"] // 64
    return ("k_forces<0, 1, %d, true, %d>" % (cfg["i_per_lane"], cfg["j_stage"]),
            str(-(-waves // wpb) * cfg["block"] * cfg["j_split"]))


def make_traffic(fetch_csv, write_csv, bench_json):
    """Traffic record of the timed all-pairs launch: the mean FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch) of its launches in the counter runs, each scaled by bytes moved /
    counter reading of the 256 MiB calibration copy the bench makes first, with a hash
    of the kernel sources and the launch configuration they were taken on."""
    import csv
    import hashlib
    import re
    import statistics
    line = [ln for ln in open(bench_json).read().splitlines() if ln.startswith("{")][-1]
    cfg_run = json.loads(line)["config"]
    n, cfg = cfg_run["n"], cfg_run["launch"]
    name, grid = timed_kernel(n, cfg)
    copy_bytes = 256 << 20
    copy_grid = "131072"                        # the grid rocprofv3 reports for the 256 MiB copy

    def vals(path, counter, pred):
        out = []
        for r in csv.DictReader(open(path)):
            kn = re.sub(r"\(.*", "", r["Kernel_Name"])
            if r["Counter_Name"] == counter and pred(kn, r["Grid_Size"]):
                out.append(float(r["Counter_Value"]))
        return out

    f = vals(fetch_csv, "FETCH_SIZE", lambda k, g: name in k and g == grid)
    w = vals(write_csv, "WRITE_SIZE", lambda k, g: name in k and g == grid)
    cf = vals(fetch_csv, "FETCH_SIZE", lambda k, g: "copyBuffer" in k and g == copy_grid)
    cw = vals(write_csv, "WRITE_SIZE", lambda k, g: "copyBuffer" in k and g == copy_grid)
    if not (f and w and cf and cw):
        raise SystemExit("counter rows not found (kernel %s grid %s, copy grid %s)" % (name, grid, copy_grid))
    fs, ws = copy_bytes / 1024 / cf[0], copy_bytes / 1024 / cw[0]
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, p), "rb").read() for p in TRAFFIC_SOURCES)).hexdigest()
    fk, wk = statistics.mean(f), statistics.mean(w)
    rec = {"kernel": name,
           "workload": "gravity N=%d FP32+Kahan with potential, block %d, i_per_lane %d, j_tile %d, "
                       "j_split %d, j_stage %d" % (n, cfg["block"], cfg["i_per_lane"], cfg["j_tile"],
                                                  cfg["j_split"], cfg["j_stage"]),
           "sources": TRAFFIC_SOURCES, "sources_sha256": h, "dispatches": len(f),
           "fetch_kib": fk, "write_kib": wk, "copy_fetch_kib": cf[0], "copy_write_kib": cw[0],
           "copy_bytes": copy_bytes, "fetch_scale": fs, "write_scale": ws,
           "bytes_per_launch": fk * 1024 * fs + wk * 1024 * ws, "config": cfg, "n": n}
    # one record per launch configuration, all on the same kernel sources
    path = os.path.join(ROOT, "profiles", "traffic_allpairs_gravity_fp32kahan_n%d.json" % n)
    records = []
    try:
        with open(path) as fh:
            records = [r for r in json.load(fh).get("records", []) if r.get("sources_sha256") == h]
    except (OSError, ValueError, AttributeError):
        records = []
    records = [r for r in records if r.get("config") != cfg] + [rec]
    records.sort(key=lambda r: sorted(r["config"].items()))
    with open(path, "w") as fh:
        json.dump({"records": records}, fh, indent=1)
    print(json.dumps(rec, indent=1))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measured_traffic(n, cfg):
    """HBM bytes per launch of the all-pairs kernel from the committed counter runs
    (FETCH_SIZE and WRITE_SIZE, copy-calibrated), or None when the kernel sources or
    the launch configuration differ from the ones the counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_allpairs_gravity_fp32kahan_n1048576.json")
    try:
        with open(path) as fh:
            records = json.load(fh)["records"]
        h = hashlib.sha256(b"".join(open(os.path.join(ROOT, s), "rb").read()
                                    for s in TRAFFIC_SOURCES)).hexdigest()
    except (OSError, KeyError, ValueError, TypeError):
        return None
    for rec in records:
        if rec.get("sources_sha256") == h and rec.get("config") == cfg and rec.get("n") == n:
            return rec["bytes_per_launch"]
    return None


def save_inputs(out_dir, n, pos, vel, mass, ens, md):
    """The seeded inputs of the run as .npy files (plain arrays, no pickles)."""
    os.makedirs(out_dir, exist_ok=True)
    arrays = {"plummer_n%d_seed5_pos" % n: pos, "plummer_n%d_seed5_vel" % n: vel,
              "plummer_n%d_seed5_mass" % n: mass}
    if ens is not None:
        off, epos, epar, _ = ens
        arrays.update({"ensemble256_seed4_offsets": np.asarray(off, dtype=np.int64),
                       "ensemble256_seed4_pos": epos, "ensemble256_seed4_params": epar})
    if md is not None:
        arrays.update({"md_n%d_seed3_pos" % md.n: md.pos, "md_n%d_seed3_params" % md.n: md.params(),
                       "md_n%d_seed3_types" % md.n: md.types})
    for name, a in arrays.items():
        np.save(os.path.join(out_dir, name + ".npy"), np.asarray(a), allow_pickle=False)
    log("inputs written to %s (%d arrays)" % (out_dir, len(arrays)))


def shard_leg(nb, torch, dev, x, m, law, full_kernel_ms, n_gpus=8):
    """One GPU's share of the headline evaluation if it were spread over n_gpus GPUs.
    Symmetric tiles (nbody_forces_share): share k of n_gpus equal ranges of the tile
    triangle, per-row partial sums of all rows (which a reduce-scatter would add across the
    GPUs), for the first and the last share.  One-sided rows (nbody_forces_subset): a
    contiguous block of N / n_gpus rows against all N records, for the first and the last
    block.  Each kernel time is set against 1 / n_gpus of the full symmetric launch."""
    n = x.shape[0]
    rows = n // n_gpus
    res = {"n": n, "gpus": n_gpus, "full_kernel_ms": full_kernel_ms}

    def kernel_ms(fn):
        fn()
        torch.cuda.synchronize()
        nb.timing_read(reset=True)
        nb.timing_enable(True)
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        nb.timing_enable(False)
        k_ms, k_n = nb.timing_read(reset=True)
        return k_ms / max(k_n, 1)

    pairs_share = float(n) * n / n_gpus
    for name, sh in (("tiles_first", 0), ("tiles_last", n_gpus - 1)):
        ms = kernel_ms(lambda: nb.forces_share(x, m, law, sh, n_gpus))
        res[name] = {"share": sh, "kernel_ms": ms, "g_pairs_per_s": pairs_share / (ms * 1e-3) / 1e9,
                     "efficiency_vs_full": full_kernel_ms / n_gpus / ms}
    for name, r0 in (("rows_first", 0), ("rows_last", n - rows)):
        il = torch.arange(r0, r0 + rows, dtype=torch.int64, device=dev)
        ms = kernel_ms(lambda: nb.forces_subset(x, m, il, law))
        res[name] = {"rows": rows, "kernel_ms": ms, "g_pairs_per_s": float(rows) * n / (ms * 1e-3) / 1e9,
                     "efficiency_vs_full": full_kernel_ms / n_gpus / ms}
    log("shard share:", res)
    return res


def batched_leg(nb, torch, dev, ens):
    """256 LJC systems: one persistent FP32+Kahan launch vs one FP64 launch per system."""
    off, pos, par, systems = ens
    S = len(systems)
    x = torch.tensor(pos, device=dev)
    p = torch.tensor(par, device=dev)
    law = nb.ljc_linear("fp32_kahan")
    law64 = nb.ljc_linear("fp64")
    cfg, _ = nb.autotune(x, p, law, offsets=off, potential=True)
    log("autotuned batched config:", cfg)
    pairs = float(sum(int(off[s + 1] - off[s]) ** 2 for s in range(S)))
    fpp = nb.flops_per_pair(nb.API_FORCES, nb.LJC_LINEAR, True)

    def run_batched():
        return nb.forces_batched(off, x, p, law)

    views = [(x[off[s]:off[s + 1]], p[off[s]:off[s + 1]]) for s in range(S)]

    # the per-system baselines get the same treatment as the batched launch: the
    # autotuner picks their configuration, once per power-of-two size bucket (the
    # granularity at which tuned configurations are remembered), on the largest
    # system of the bucket
    sizes = np.diff(off)
    buckets = {}
    for s in range(S):
        if sizes[s] > 0:
            b = int(np.ceil(np.log2(sizes[s])))
            if b not in buckets or sizes[s] > sizes[buckets[b]]:
                buckets[b] = s
    for l in (law64, law):
        for b, s in sorted(buckets.items()):
            nb.autotune(views[s][0], views[s][1], l, potential=True)
    log("autotuned per-system loop baselines for size buckets", sorted(buckets))

    def run_loop(l):
        outs = []
        for xs, ps in views:
            outs.append(nb.forces(xs, ps, l))
        return outs

    def timeit(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            t = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        return best, r

    tb, (fb, ub) = timeit(run_batched, reps=20)
    # per call, in the same calls: the wall time from Python and the persistent kernel's own
    # time (HIP events around it); their difference is the call's work outside that kernel
    # (host marshalling, the pack and the part sums)
    nb.timing_read(reset=True)
    nb.timing_enable(True)
    walls, kerns = [], []
    for _ in range(20):
        t = time.perf_counter()
        run_batched()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t)
        k_ms, k_n = nb.timing_read(reset=True)
        kerns.append(k_ms / max(k_n, 1))
    nb.timing_enable(False)
    kb_ms = float(np.median(kerns))
    outside_us = sorted((w * 1e3 - k) * 1e3 for w, k in zip(walls, kerns))
    # the whole call replayed from a captured graph (its pack, kernel and part-sum launches,
    # without the host's part)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run_batched()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fg, _ = run_batched()
    graph.replay()
    torch.cuda.synchronize()
    graph_ok = bool(torch.equal(fg, fb))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    tg_ms = e0.elapsed_time(e1) / 20
    del graph
    tl64, outs64 = timeit(lambda: run_loop(law64))
    tl32, _ = timeit(lambda: run_loop(law))
    f64 = torch.cat([o[0] for o in outs64])
    e = (torch.linalg.norm(fb - f64, dim=1) / torch.linalg.norm(f64, dim=1)).cpu().numpy()
    med_sys = [float(np.median(e[off[s]:off[s + 1]])) for s in range(S) if off[s + 1] > off[s]]
    res = {"systems": S, "atoms": int(off[-1]), "pairs": pairs, "config": cfg,
           "batched_fp32_kahan_ms": tb * 1e3, "batched_kernel_ms": kb_ms,
           "batched_wall_minus_kernel_us": {"min": outside_us[0], "median": float(np.median(outside_us))},
           "batched_graph_replay_ms": tg_ms, "graph_replay_equals_eager": graph_ok,
           "flops_per_pair": fpp, "batched_kernel_tflops": fpp * pairs / (kb_ms * 1e-3) / 1e12,
           "batched_wall_tflops": fpp * pairs / tb / 1e12,
           "loop_fp64_ms": tl64 * 1e3, "loop_fp32_kahan_ms": tl32 * 1e3,
           "speedup_vs_loop_fp64": tl64 / tb, "speedup_vs_loop_fp32": tl32 / tb,
           "batched_g_pairs_per_s": pairs / tb / 1e9,
           "err_vs_fp64_per_system_median_max": max(med_sys), "err_vs_fp64_max": float(e.max())}
    log("batched:", res)
    return res


def backward_leg(nb, torch, dev, W, md=None):
    """Position adjoint (Hessian-vector product) of gravity at N = 262,144, FP32 vs FP64; with
    the per-law leg's MD box (65,536 atoms), LJC(linear)'s adjoint (positions, charges, sigma and
    epsilon) in FP32 + Kahan by the rule (unordered pairs), one-sided, and in FP64."""
    n = 262144
    pos, _, m = W.plummer(n, 6)
    g = W.unit_cotangent(n, 56)
    x = torch.tensor(pos, device=dev)
    mm = torch.tensor(m, device=dev)
    gg = torch.tensor(g, device=dev)
    res = {"n": n}
    outs = {}
    for name in ("fp32_fp64acc", "fp64"):
        law = nb.gravity(name, softening=EPS_MAIN)
        nb.forces_backward(x, mm, gg, law)
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(3):
            t = time.perf_counter()
            gp, _, _ = nb.forces_backward(x, mm, gg, law)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        outs[name] = gp
        res[name + "_ms"] = best * 1e3
    e = (torch.linalg.norm(outs["fp32_fp64acc"] - outs["fp64"], dim=1)
         / torch.linalg.norm(outs["fp64"], dim=1)).cpu().numpy()
    res["speedup_fp32_vs_fp64"] = res["fp64_ms"] / res["fp32_fp64acc_ms"]
    res["flops_per_pair"] = nb.flops_per_pair(nb.API_BACKWARD, nb.GRAVITY, False)
    res["fp32_tflops"] = res["flops_per_pair"] * float(n) ** 2 / (res["fp32_fp64acc_ms"] * 1e-3) / 1e12
    res["err_vs_fp64"] = {"median": float(np.median(e)), "max": float(e.max())}
    if md is not None:
        res["ljc_linear"] = ljc_backward(nb, torch, dev, W, md)
    log("backward:", res)
    return res


def ljc_backward(nb, torch, dev, W, md):
    n = md.n
    x = torch.tensor(md.pos, device=dev)
    p = torch.tensor(md.params(), device=dev)
    gg = torch.tensor(W.unit_cotangent(n, 57), device=dev)
    res = {"n": n, "flops_per_pair": nb.flops_per_pair(nb.API_BACKWARD, nb.LJC_LINEAR, False)}
    outs = {}
    for name, prec, cfg in (("fp32_kahan", "fp32_kahan", None), ("fp32_kahan_one_sided", "fp32_kahan", (256, 1, 256, 8, 1)),
                            ("fp64", "fp64", None)):
        law = nb.ljc_linear(prec)
        if cfg:
            nb.set_config(nb.API_BACKWARD, *cfg)
        try:
            c = nb.get_config(nb.API_BACKWARD, n, law)
            nb.forces_backward(x, p, gg, law)
            torch.cuda.synchronize()
            best = 1e30
            for _ in range(3):
                t = time.perf_counter()
                out = nb.forces_backward(x, p, gg, law)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t)
        finally:
            if cfg:
                nb.clear_config(nb.API_BACKWARD)
        outs[name] = out
        res[name] = {"ms": best * 1e3, "config": c,
                     "tflops": res["flops_per_pair"] * float(n) ** 2 / best / 1e12}
    ref = outs["fp64"]
    e = (torch.linalg.norm(outs["fp32_kahan"][0] - ref[0], dim=1) / torch.linalg.norm(ref[0], dim=1)).cpu().numpy()
    ep = ((outs["fp32_kahan"][1] - ref[1]).abs() / ref[1].abs().max(dim=0).values).cpu().numpy()
    res["speedup_vs_one_sided"] = res["fp32_kahan_one_sided"]["ms"] / res["fp32_kahan"]["ms"]
    res["speedup_vs_fp64"] = res["fp64"]["ms"] / res["fp32_kahan"]["ms"]
    res["err_vs_fp64"] = {"pos_median": float(np.median(e)), "pos_max": float(e.max()),
                          "params_median": float(np.median(ep)), "params_max": float(ep.max())}
    return res


def laws_leg(nb, torch, dev, W, md):
    """Every pair law of Table 1 at N = 65,536 (Plummer sphere for gravity, the MD box at
    density 1/32 A^-3 for the LJC laws), FP32 + Kahan with the potential: throughput, the
    all-pairs kernel's FLOP/s against the FP32 vector peak, and the error against an FP64
    pass over the same inputs."""
    n = md.n
    x = torch.tensor(md.pos, device=dev)
    p = torch.tensor(md.params(), device=dev)
    pg, _, mg = W.plummer(n, 2)
    xg = torch.tensor(pg, device=dev)
    mgt = torch.tensor(mg, device=dev)
    laws = [("gravity", nb.GRAVITY, xg, mgt, lambda pr: nb.gravity(pr, softening=0.01)),
            ("ljc_linear", nb.LJC_LINEAR, x, p, lambda pr: nb.ljc_linear(pr)),
            ("ljc_constant", nb.LJC_CONSTANT, x, p, lambda pr: nb.ljc_constant(pr)),
            ("ljc_sigmoidal", nb.LJC_SIGMOIDAL, x, p, lambda pr: nb.ljc_sigmoidal(ZETA_SIGMOIDAL, pr))]
    res = {"n": n, "pairs": float(n) * n, "zeta_sigmoidal": list(ZETA_SIGMOIDAL)}
    reps = 10
    for name, kind, xx, pp, mk in laws:
        law = mk("fp32_kahan")
        cfg, _ = nb.autotune(xx, pp, law, potential=True)
        f32, u32 = nb.forces(xx, pp, law)
        torch.cuda.synchronize()
        nb.timing_read(reset=True)
        nb.timing_enable(True)
        t = time.perf_counter()
        for _ in range(reps):
            nb.forces(xx, pp, law)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / reps
        nb.timing_enable(False)
        k_ms, k_n = nb.timing_read(reset=True)
        k_s = k_ms / max(k_n, 1) * 1e-3
        fpp = nb.flops_per_pair(nb.API_FORCES, kind, True)
        f64, u64 = nb.forces(xx, pp, mk("fp64"))
        e = (torch.linalg.norm(f32 - f64, dim=1) / torch.linalg.norm(f64, dim=1)).cpu().numpy()
        tf = fpp * float(n) * n / k_s / 1e12
        res[name] = {"config": cfg, "ms": wall * 1e3, "kernel_ms": k_s * 1e3,
                     "g_pairs_per_s": float(n) * n / wall / 1e9, "flops_per_pair": fpp,
                     "kernel_tflops": tf, "frac_fp32_peak": tf / PEAK_FP32_TFLOPS,
                     "err_vs_fp64": {"median": float(np.median(e)), "max": float(e.max())}}
        log("law %s:" % name, res[name])
    return res


def jerk_leg(nb, torch, dev, W, tune=True):
    """Acceleration + jerk (Table 1 "Gravity (accel & jerk)") on a Plummer sphere with
    N = 65,536, FP32 + Kahan with the potential (the autotuned configuration, or the rule's
    with tune False); then the Hermite scheme with block individual steps (FP32 + FP64
    accumulation, eta = 0.02, dt_max = 1/16) run from t = 0 to the first synchronisation
    point t = 1/16, with its energy error."""
    n = 65536
    eps = 0.01
    x, v, m = W.plummer(n, 2)
    X = torch.tensor(x, device=dev)
    V = torch.tensor(v, device=dev)
    M = torch.tensor(m, device=dev)
    law = nb.gravity("fp32_kahan", softening=eps)
    cfg = nb.autotune_jerk(X, V, M, law, potential=True)[0] if tune else nb.get_config(nb.API_JERK, n, law)
    a32, j32, _ = nb.forces_jerk(X, V, M, law)
    for _ in range(5):                                    # untimed: the clock settles
        nb.forces_jerk(X, V, M, law)
    torch.cuda.synchronize()
    reps = 10
    nb.timing_read(reset=True)
    nb.timing_enable(True)
    t = time.perf_counter()
    for _ in range(reps):
        nb.forces_jerk(X, V, M, law)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / reps
    nb.timing_enable(False)
    k_ms, k_n = nb.timing_read(reset=True)
    k_s = k_ms / max(k_n, 1) * 1e-3
    fpp = nb.flops_per_pair(nb.API_JERK, nb.GRAVITY, True)
    a64, j64, _ = nb.forces_jerk(X, V, M, nb.gravity("fp64", softening=eps))
    ea = (torch.linalg.norm(a32 - a64, dim=1) / torch.linalg.norm(a64, dim=1)).cpu().numpy()
    ej = (torch.linalg.norm(j32 - j64, dim=1) / torch.linalg.norm(j64, dim=1)).cpu().numpy()
    tf = fpp * float(n) * n / k_s / 1e12
    res = {"n": n, "config": cfg, "ms": wall * 1e3, "kernel_ms": k_s * 1e3,
           "g_pairs_per_s": float(n) * n / wall / 1e9, "flops_per_pair": fpp,
           "kernel_tflops": tf, "frac_fp32_peak": tf / PEAK_FP32_TFLOPS,
           "acc_err_vs_fp64": {"median": float(np.median(ea)), "max": float(ea.max())},
           "jerk_err_vs_fp64": {"median": float(np.median(ej)), "max": float(ej.max())}}
    log("jerk:", res)

    # block individual time steps to the first synchronisation point
    lawb = nb.gravity("fp32_fp64acc", softening=eps)
    law64 = nb.gravity("fp64", softening=eps)
    dt_max, eta = 1.0 / 16, 0.02

    def energy():
        _, phi = nb.forces(X, M, law64)
        return float((0.5 * (M * (V * V).sum(1)).sum() + 0.5 * (M * phi).sum()).item())

    A, J, _ = nb.forces_jerk(X, V, M, lawb, potential=False)
    T, DT = nb.hermite_block_init(A, J, 0.01, dt_max)
    e0 = energy()
    torch.cuda.synchronize()
    t = time.perf_counter()
    # one call: block steps are enqueued without host waits and end exactly at t = dt_max
    counts, t_now = nb.hermite_block(X, V, A, J, T, DT, M, lawb, eta, dt_max, 1 << 20, t_end=dt_max)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    e1 = energy()
    steps = counts[counts > 0]
    assert t_now == dt_max and bool(torch.all(T == dt_max)), "block steps did not reach t_end"
    pairs = float(steps.sum()) * n
    res["block_steps"] = {"law": "fp32_fp64acc", "eta": eta, "dt_max": dt_max, "t_end": t_now,
                          "block_steps": int(steps.size), "particle_steps": int(steps.sum()),
                          "mean_active": float(steps.mean()), "min_active": int(steps.min()),
                          "max_active": int(steps.max()), "wall_s": wall,
                          "g_pairs_per_s": pairs / wall / 1e9,
                          "rel_energy_error": abs(e1 - e0) / abs(e0)}
    log("block steps:", res["block_steps"])
    return res


def _time(torch, fn, reps=5):
    fn()
    torch.cuda.synchronize()
    best = 1e30
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best


def bonded_leg(nb, torch, dev, W, chains):
    """Bonded molecules with exclusion lists (Section 5): 256 chains of 32 atoms (N = 8192,
    1-2 and 1-3 pairs excluded), LJC(linear), FP32 + Kahan with the energy: forces with
    and without the lists, and the force-matching adjoint with them."""
    sy, eo, ei = chains
    x = torch.tensor(sy.pos, device=dev)
    p = torch.tensor(sy.params(), device=dev)
    ex = nb.Exclusions(torch.tensor(eo, device=dev), torch.tensor(ei, device=dev))
    law = nb.ljc_linear("fp32_kahan")
    law64 = nb.ljc_linear("fp64")
    t_ex = _time(torch, lambda: nb.forces(x, p, law, exclusions=ex))
    t_plain = _time(torch, lambda: nb.forces(x, p, law))
    f32, _ = nb.forces(x, p, law, exclusions=ex)
    f64, _ = nb.forces(x, p, law64, exclusions=ex)
    e = (torch.linalg.norm(f32 - f64, dim=1) / torch.linalg.norm(f64, dim=1)).cpu().numpy()
    g = torch.tensor(W.unit_cotangent(sy.n, 57), device=dev)
    t_adj = _time(torch, lambda: nb.forces_backward(x, p, g, law, exclusions=ex))
    t_adj64 = _time(torch, lambda: nb.forces_backward(x, p, g, law64, exclusions=ex))
    n = sy.n
    res = {"n": n, "chains": 256, "chain_len": 32, "excluded_pairs": int(eo[-1]),
           "forces_ms": t_ex * 1e3, "forces_no_exclusions_ms": t_plain * 1e3,
           "g_pairs_per_s": float(n) * n / t_ex / 1e9,
           "err_vs_fp64": {"median": float(np.median(e)), "max": float(e.max())},
           "adjoint_fp32_ms": t_adj * 1e3, "adjoint_fp64_ms": t_adj64 * 1e3,
           "adjoint_speedup_fp32_vs_fp64": t_adj64 / t_adj}
    log("bonded:", res)
    return res


def batched_backward_leg(nb, torch, dev, ens):
    """The adjoint of the 256-system LJC ensemble in one persistent FP32 launch against one
    FP64 adjoint launch per system (both with per-type sums)."""
    off, pos, par, systems = ens
    S = len(systems)
    x = torch.tensor(pos, device=dev)
    p = torch.tensor(par, device=dev)
    n = x.shape[0]
    rng = np.random.default_rng(58)
    g = torch.tensor(rng.standard_normal((n, 3)) / np.sqrt(3 * n), device=dev)
    types = torch.tensor(np.concatenate([s.types for s in systems]), device=dev)
    law = nb.ljc_linear("fp32_kahan")
    law64 = nb.ljc_linear("fp64")
    t_b = _time(torch, lambda: nb.forces_backward_batched(off, x, p, g, law, types=types, n_types=4))
    views = [(x[off[s]:off[s + 1]], p[off[s]:off[s + 1]], g[off[s]:off[s + 1]],
              types[off[s]:off[s + 1]]) for s in range(S)]

    def loop(l):
        return [nb.forces_backward(xs, ps, gs, l, types=ts, n_types=4) for xs, ps, gs, ts in views]

    t_l64 = _time(torch, lambda: loop(law64), reps=3)
    gb, qb, _ = nb.forces_backward_batched(off, x, p, g, law, types=types, n_types=4)
    outs = loop(law64)
    g64 = torch.cat([o[0] for o in outs])
    e = (torch.linalg.norm(gb - g64, dim=1) / torch.linalg.norm(g64, dim=1)).cpu().numpy()
    med_sys = [float(np.median(e[off[s]:off[s + 1]])) for s in range(S) if off[s + 1] > off[s]]
    pairs = float(sum(int(off[s + 1] - off[s]) ** 2 for s in range(S)))
    res = {"systems": S, "atoms": int(n), "pairs": pairs, "batched_fp32_kahan_ms": t_b * 1e3,
           "loop_fp64_ms": t_l64 * 1e3, "speedup_vs_loop_fp64": t_l64 / t_b,
           "flops_per_pair": nb.flops_per_pair(nb.API_BACKWARD_BATCHED, nb.LJC_LINEAR, False),
           "batched_tflops": 68 * pairs / t_b / 1e12,
           "err_vs_fp64_per_system_median_max": max(med_sys), "err_vs_fp64_max": float(e.max())}
    log("batched backward:", res)
    return res


def leapfrog_leg(nb, torch, dev, W):
    """100 KDK leapfrog steps of the N = 65,536 Plummer sphere (eps = 0.01, dt = 1e-3): wall time
    of the FP32 + Kahan and FP64 trajectories, and their relative energy drift with E from the
    FP64 potential pass in both cases."""
    n, eps, dt, steps = 65536, 0.01, 1e-3, 100
    pos, vel, m = W.plummer(n, 2)
    M = torch.tensor(m, device=dev)
    law64 = nb.gravity("fp64", softening=eps)

    def energy(x, v):
        _, phi = nb.forces(x, M, law64)
        return float((0.5 * M * (v * v).sum(1)).sum() + 0.5 * (M * phi).sum())

    res = {"n": n, "steps": steps, "dt": dt, "softening": eps}
    e0 = None
    for name in ("fp32_kahan", "fp64"):
        law = nb.gravity(name, softening=eps)
        X, V = torch.tensor(pos, device=dev), torch.tensor(vel, device=dev)
        A, _ = nb.forces(X, M, law)
        if e0 is None:
            e0 = energy(X, V)
        torch.cuda.synchronize()
        t = time.perf_counter()
        nb.leapfrog(X, V, A, M, law, dt, steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        res[name] = {"wall_s": wall, "ms_per_step": wall / steps * 1e3,
                     "g_pairs_per_s": float(n) * n * steps / wall / 1e9,
                     "rel_energy_drift": abs(energy(X, V) - e0) / abs(e0)}
    log("leapfrog 100 steps:", res)
    return res


def oracle_configs_leg(nb, torch, dev, W, ens, out):
    """The FP64 oracle, as it stands, timed in full on the host cores for the small
    configurations (N = 4096 gravity forces; the t = 0 force evaluation at N = 65,536; the
    N = 8192 MD forward and its force-matching adjoint; the 256-system ensemble), next to
    the GPU path on the same work.  A different kind of baseline from the paper's
    hand-vectorised CPU code: the plain double loop with compensated sums."""
    import oracle
    res = {"threads": oracle.threads(0)}

    def clock(fn):
        t = time.perf_counter()
        fn()
        return time.perf_counter() - t

    def gpu(fn, reps=5):
        return _time(torch, fn, reps=reps)

    # config 1: gravity N = 4096, FP64
    x1, _, m1 = W.plummer(4096, 1)
    t_or = clock(lambda: oracle.gravity(x1, m1, eps=0.01))
    X1, M1 = torch.tensor(x1, device=dev), torch.tensor(m1, device=dev)
    t_gpu = gpu(lambda: nb.forces(X1, M1, nb.gravity("fp64", softening=0.01)))
    res["gravity_4096_fp64"] = {"oracle_s": t_or, "gpu_s": t_gpu, "speedup": t_or / t_gpu}
    # config 2 at t = 0: gravity N = 65536, FP32 + Kahan on the GPU
    x2, _, m2 = W.plummer(65536, 2)
    t_or = clock(lambda: oracle.gravity(x2, m2, eps=0.01))
    X2, M2 = torch.tensor(x2, device=dev), torch.tensor(m2, device=dev)
    t_gpu = gpu(lambda: nb.forces(X2, M2, nb.gravity("fp32_kahan", softening=0.01)))
    res["gravity_65536_t0"] = {"oracle_s": t_or, "gpu_s": t_gpu, "speedup": t_or / t_gpu}
    # config 3: MD N = 8192 (64 A box), forward and force-matching adjoint
    s3 = W.md_system(8192, 3)
    g3 = W.unit_cotangent(s3.n, 57)
    t_f = clock(lambda: oracle.ljc_linear(s3.pos, s3.q, s3.sigma, s3.epsilon))
    t_b = clock(lambda: oracle.ljc_adjoint(s3.pos, s3.q, s3.sigma, s3.epsilon, g3))
    X3, P3, G3 = (torch.tensor(a, device=dev) for a in (s3.pos, s3.params(), g3))
    law3 = nb.ljc_linear("fp32_fp64acc")
    t_gf = gpu(lambda: nb.forces(X3, P3, law3))
    t_gb = gpu(lambda: nb.forces_backward(X3, P3, G3, law3))
    res["md_8192_forward"] = {"oracle_s": t_f, "gpu_s": t_gf, "speedup": t_f / t_gf}
    res["md_8192_adjoint"] = {"oracle_s": t_b, "gpu_s": t_gb, "speedup": t_b / t_gb}
    # config 4: the ensemble, one oracle call per system
    off, pos, par, systems = ens
    t_or = clock(lambda: [oracle.ljc_linear(sy.pos, sy.q, sy.sigma, sy.epsilon) for sy in systems])
    t_gpu = out["batched"]["batched_fp32_kahan_ms"] * 1e-3
    res["ensemble_256"] = {"oracle_s": t_or, "gpu_s": t_gpu, "speedup": t_or / t_gpu}
    log("oracle on the configurations:", res)
    return res


if __name__ == "__main__":
    main()
