"""Benchmark of the batched explicit asymptotic integrator on one MI355X.

One step = one asy_integrate_batch call that integrates every zone of the
workload from t = 0 to t_end (rates, fluxes, creation/depletion sums,
kappa-switched updates and step control), starting from the same initial
state each time.  Inputs are resident in HBM before the timed region; the
launch configuration is chosen by asy_autotune before it (--no-autotune keeps
the network's default).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.  value = accepted zone-steps per second over the K timed
steps of the 150-species, 4096-zone Arrhenius workload.  Further keys:
  roofline      the integrator is bound by LDS traffic: achieved = algorithmic
                LDS bytes per attempted zone-step x attempted zone-steps per
                launch / average launch time (HIP events on the launch stream);
                peak = the larger of the nominal LDS bandwidth (256 CUs x 128
                B/clock x 2.4 GHz) and the read bandwidth measured on the device
                with conflict-free 8- and 16-byte LDS reads; counter figures
                from the committed rocprofv3 summary of the same kernel sources
  c4            the 365-species, 1024-zone workload, timed the same way
  f32           the main workload in single precision
  zone_count_sweep  Z identical zones, Z = 1 .. 3073 (the concurrent-network
                staircase)
  launch_study  the main workload under several launch configurations
  learned       the learned step proposer against the plain controller
                (learned_leg)
  cpu_baseline  the oracle on the host cores (cpu_baseline_leg)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs at 2.4 GHz; an LDS delivers 128 bytes per clock per CU.
N_CU = 256
CLOCK_HZ = 2.4e9
LDS_BYTES_PER_CLK_CU = 128
LDS_PEAK_GBS = N_CU * LDS_BYTES_PER_CLK_CU * CLOCK_HZ / 1e9


def kernel_source_sha256() -> str:
    """Hash of the HIP sources, to tie a profile summary to the kernel it measured."""
    import glob
    import hashlib

    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1409_5826_amd", "csrc", "*"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_counters(workload: str) -> dict:
    """Counter figures per launch from the committed rocprofv3 summary of this workload
    (HBM bytes: FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size; LDS load
    bytes), or {} when there is no summary or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"integrate_strat_{workload}.md")
    if not os.path.exists(path):
        return {}
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("|", "*", "#", "`")):
                key, _, val = line.partition(":")
                fields[key.strip()] = val.strip()
    if fields.get("kernel_source_sha256") != kernel_source_sha256():
        return {}
    out = {}
    for key in ("traffic_bytes_per_launch", "lds_load_bytes_per_launch"):
        try:
            out[key] = float(fields[key])
        except (KeyError, ValueError):
            pass
    return out


def profiled_traffic(workload: str):
    """HBM bytes per launch from the committed profile summary, or None (see profiled_counters)."""
    return profiled_counters(workload).get("traffic_bytes_per_launch")


def algorithmic_bytes_per_zone_step(n_species: int, n_reactions: int, n_destruction: int,
                                    value_bytes: int = 8, rates_in_registers: bool = True) -> int:
    """LDS bytes one attempted step of one zone must move (value = 8 B in double, 4 B in
    single precision; index = 2 B).

    Per reaction: read k_j, write the flux, read it back with its product
    index (3 values + 2 B).  Per destruction incidence: gather the partner
    abundance with its index, write the partial rate, read it back (3 values
    + 2 B).  Per species: five reads/writes of Y, F+, k, Yn (5 values).  When
    the kernel holds the zone's rates in registers for the whole interval (the
    packed-rows kernel does), the per-reaction read of k_j is not LDS traffic:
    one value per reaction less.
    """
    v = value_bytes
    b = (3 * v + 2) * (n_reactions + n_destruction) + 5 * v * n_species
    if rates_in_registers:
        b -= v * n_reactions
    return b


def time_launches(net, buf, Y0, dt0, stream, steps, warmup, opts=None):
    """Warm up, then time `steps` whole-batch integrations from the same initial state.

    Returns (wall seconds of the timed loop, per-launch milliseconds from HIP events recorded
    on the launch stream)."""
    import torch

    for _ in range(warmup):
        buf["Y"].copy_(Y0)
        buf["dt"].copy_(dt0)
        net.integrate(buf, opts, stream=stream)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        buf["Y"].copy_(Y0)
        buf["dt"].copy_(dt0)
        starts[i].record(stream)
        net.integrate(buf, opts, stream=stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, [s.elapsed_time(e) for s, e in zip(starts, ends)]


def mass_drift(wl, Y):
    """Percentiles over the zones of sum_i w_i Y_i(t_end) / sum_i w_i Y_i(0): the explicit
    asymptotic update does not conserve the weighted sum (Eq. asySophia), so this reports how
    far each workload drifts."""
    import numpy as np

    w = wl.network.weight.astype(np.float64)
    ratio = (Y @ w) / (wl.zones.Y0 @ w)
    q = np.percentile(ratio, [1, 10, 50, 90, 99])
    return {"p1": q[0], "p10": q[1], "p50": q[2], "p90": q[3], "p99": q[4],
            "min": float(ratio.min()), "max": float(ratio.max())}


def run_workload(name, steps, warmup, peak, launch=None, autotune=True, n_zones=None):
    """One workload on the GPU: launch chosen (autotuned outside the timed region, or given),
    `steps` timed whole-batch integrations.  Returns (network handle, buffers, summary)."""
    import numpy as np
    import torch

    from paper_1409_5826_amd import binding, workloads

    wl = workloads.preset(name, n_zones=n_zones)
    net = binding.Network(wl.network)
    if launch:
        net.set_launch(**launch)
    buf = net.zone_buffers(wl.zones)
    Y0 = buf["Y"].clone()
    dt0 = buf["dt"].clone()
    tuned = None
    if autotune and not launch:
        t0 = time.perf_counter()
        binding.asy_autotune(net.handle, net.n_species, net.n_reactions, Y0, buf["t_end"], dt0,
                             T=buf["T"], k_zone=buf["k_zone"])
        tuned = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    elapsed, launch_ms = time_launches(net, buf, Y0, dt0, stream, steps, warmup)
    n_acc = buf["n_accepted"].cpu().numpy()
    n_rej = buf["n_rejected"].cpu().numpy()
    status = buf["zone_status"].cpu().numpy()
    if not (status == binding.ZONE_OK).all():
        print(f"warning: {name}: {int((status != 0).sum())} zones did not reach t_end",
              file=sys.stderr)
    n = wl.network
    acc, att = int(n_acc.sum()), int(n_acc.sum() + n_rej.sum())
    cfg = net.get_launch()
    b_step = algorithmic_bytes_per_zone_step(n.n_species, n.n_reactions, n.n_destruction, 8,
                                             cfg["variant"] == 1)
    ms = float(np.median(launch_ms))  # median of the timed launches
    achieved = b_step * att / (ms / 1e3) / 1e9
    summary = {
        "workload": wl.name, "description": wl.description, "zones": wl.zones.n_zones,
        "n_species": n.n_species, "n_reactions": n.n_reactions, "tol": wl.tol,
        "wall_s": elapsed, "time_to_t_end_ms": ms,
        "time_to_t_end_ms_min": float(np.min(launch_ms)),
        "time_to_t_end_ms_mean": float(np.mean(launch_ms)),
        "zone_steps_per_s": acc / (ms / 1e3), "attempted_steps_per_s": att / (ms / 1e3),
        "accepted_zone_steps": acc, "rejected_zone_steps": att - acc,
        "bytes_per_zone_step": b_step, "achieved_GBs": achieved, "frac": achieved / peak,
        "launch": cfg, "autotune_s": tuned,
        "layout": net.layout_info(cfg["threads_per_zone"]) if cfg["variant"] == 1 else None,
        "mass_drift": mass_drift(wl, buf["Y"].cpu().numpy()),
    }
    return wl, net, buf, (Y0, dt0, stream), summary


def zone_count_sweep(name, counts, reps=3):
    """Time to t_end of Z identical zones (one mid-range zone of the workload, copied) for each
    Z in counts: flat while every zone has a resident workgroup slot, then a step up each time
    Z passes a multiple of the slots (the staircase of the paper's concurrent-network runs)."""
    import numpy as np
    import torch

    from paper_1409_5826_amd import binding, workloads

    wl = workloads.preset(name)
    z = wl.zones
    pick = int(np.argsort(z.T if z.T is not None else z.k.sum(1))[z.n_zones // 2])
    net = binding.Network(wl.network)
    out = []
    try:
        stream = torch.cuda.current_stream()
        for Z in counts:
            zones = z.subset(np.full(Z, pick))
            buf = net.zone_buffers(zones)
            Y0, dt0 = buf["Y"].clone(), buf["dt"].clone()
            _, ms = time_launches(net, buf, Y0, dt0, stream, reps, 1)
            out.append({"zones": Z, "ms": float(np.median(ms)),
                        "accepted_per_zone": int(buf["n_accepted"][0].item())})
        launch = net.get_launch()
    finally:
        net.close()
    return {"workload": f"{name}, zone {pick} (median T) repeated", "launch": launch,
            "points": out}


def cpu_baseline_leg(wl, stride, repeats=3, one_core_stride=64):
    """The oracle (test infrastructure, plain C) on the host cores of this machine: a copy
    built here with -O3 -march=native (same arithmetic), OpenMP over zones; median of
    `repeats` runs on every `stride`-th zone with all threads, and on every
    `one_core_stride`-th zone with one thread."""
    import platform
    import tempfile

    import numpy as np

    import oracle

    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    tmp = tempfile.mkdtemp(prefix="oracle_native_")
    oracle.use_library(oracle.build_for_this_host(os.path.join(tmp, "liboracle_native.so")))

    def timed(idx, n_threads):
        sub = wl.zones.subset(idx)
        times, acc = [], 0
        for _ in range(repeats):
            tc = time.perf_counter()
            ref = oracle.integrate_batch(wl.network, sub, n_threads=n_threads)
            times.append(time.perf_counter() - tc)
            acc = int(ref["n_acc"].sum())
        return acc, float(np.median(times))

    threads = oracle.max_threads()
    idx_all = np.arange(0, wl.zones.n_zones, stride)
    acc, t_all = timed(idx_all, threads)
    idx_one = np.arange(0, wl.zones.n_zones, one_core_stride)
    acc1, t_one = timed(idx_one, 1)
    return {
        "value": acc / t_all,
        "unit": "zone-steps/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"{len(idx_all)} of {wl.zones.n_zones} zones (every {stride}th), {acc} accepted "
                  f"zone-steps, median of {repeats} runs {t_all:.2f} s",
        "one_core": {"value": acc1 / t_one, "unit": "zone-steps/s",
                     "sample": f"{len(idx_one)} zones (every {one_core_stride}th), {acc1} accepted "
                               f"zone-steps, median of {repeats} runs {t_one:.2f} s"},
        "cpu_model": model, "logical_cpus": os.cpu_count(),
        "build": "gcc -O3 -march=native -ffp-contract=off -fno-fast-math -fopenmp, "
                 "schedule(dynamic,1) over zones",
    }


def log(msg):
    """Progress on stderr (the JSON line is the only stdout output)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


SWEEP_COUNTS = (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 1536, 1537, 2048, 3072, 3073)

LAUNCH_STUDY = (
    dict(variant=1, threads_per_zone=64, groups_per_cu=0, use_graph=0, zone_order=1),
    dict(variant=1, threads_per_zone=128, groups_per_cu=0, use_graph=0, zone_order=0),
    dict(variant=1, threads_per_zone=128, groups_per_cu=0, use_graph=0, zone_order=1),
    dict(variant=1, threads_per_zone=128, groups_per_cu=0, use_graph=1, zone_order=1),
    dict(variant=1, threads_per_zone=128, groups_per_cu=3, use_graph=0, zone_order=1),
    dict(variant=1, threads_per_zone=128, groups_per_cu=6, use_graph=0, zone_order=1),
    dict(variant=1, threads_per_zone=128, groups_per_cu=6, use_graph=1, zone_order=1),
    dict(variant=1, threads_per_zone=256, groups_per_cu=0, use_graph=0, zone_order=1),
)


def launch_study(net, buf, Y0, dt0, stream, configs=LAUNCH_STUDY, reps=2):
    """Time to t_end of the batch under several launch configurations (the table behind the
    default and the autotuner's choice); the network's launch is restored afterwards."""
    import numpy as np

    from paper_1409_5826_amd import binding

    keep = net.get_launch()
    rows = []
    try:
        for cfg in configs:
            try:
                net.set_launch(**cfg)
            except binding.AsyError as e:
                rows.append(dict(cfg, ms=None, note=str(e)))
                continue
            _, ms = time_launches(net, buf, Y0, dt0, stream, reps, 1)
            rows.append(dict(cfg, ms=float(np.median(ms))))
    finally:
        net.set_launch(**keep)
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="n150_r1604_arrhenius")
    ap.add_argument("--zones", type=int, default=None)
    ap.add_argument("--cpu-sample-stride", type=int, default=4,
                    help="oracle baseline integrates every Nth zone")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", default=None, help="JSON dict of asy_launch fields (no autotune)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the network's default launch instead of timing the candidates")
    ap.add_argument("--no-f32", action="store_true",
                    help="skip the single-precision measurement of the same workload")
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the 365-species, 1024-zone workload")
    ap.add_argument("--no-sweep", action="store_true", help="skip the zone-count sweep")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-proposer comparison")
    ap.add_argument("--learned-zones", type=int, default=4096)
    ap.add_argument("--learned-step-probe", action="store_true",
                    help="time learned against plain zone-steps with a fixed network and exit")
    ap.add_argument("--mlp-train-probe", type=int, default=0,
                    help="only time this many epochs of MLP training (batch 1024) on 64 seeded "
                         "synthetic batches, for profiling the training kernels")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (calibrates HBM counters)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(zones are independent: they would shard across GPUs with no exchange)", file=sys.stderr)
        return 2

    import torch

    from paper_1409_5826_amd import binding

    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                          "launches": 3}), flush=True)
        return 0
    if args.mlp_train_probe:
        print(json.dumps(mlp_train_probe(args.mlp_train_probe)), flush=True)
        return 0
    if args.learned_step_probe:
        print(json.dumps(learned_step_probe()), flush=True)
        return 0
    lds_measured = {w: binding.asy_probe_lds_bandwidth(w) / 1e9 for w in (8, 16)}
    peak = max(LDS_PEAK_GBS, *lds_measured.values())
    launch = json.loads(args.launch) if args.launch else None
    log(f"LDS probe {lds_measured}")
    wl, net, buf, (Y0, dt0, stream), main_run = run_workload(
        args.workload, args.steps, args.warmup, peak, launch=launch,
        autotune=not args.no_autotune, n_zones=args.zones)
    log(f"{wl.name}: {main_run['time_to_t_end_ms']:.2f} ms, launch {main_run['launch']}")
    prof = profiled_counters(wl.name)
    n = wl.network

    out = {
        "metric": "zone-steps/sec and time-to-t_end for 4096 zones",
        "value": main_run["accepted_zone_steps"] * args.steps / main_run["wall_s"],
        "unit": "zone-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["wall_s"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": dict(main_run, parallelism="1 GPU"),
        "roofline": {
            "bound": "lds",
            "achieved": main_run["achieved_GBs"],
            "peak": peak,
            "unit": "GB/s",
            "frac": main_run["frac"],
            "peak_nominal": LDS_PEAK_GBS,
            "peak_measured": {f"ds_read_{8 * w}bit": v for w, v in lds_measured.items()},
            "traffic": prof.get("traffic_bytes_per_launch"),
            "bytes_per_zone_step": main_run["bytes_per_zone_step"],
            "attempted_zone_steps_per_launch": main_run["accepted_zone_steps"] +
                                               main_run["rejected_zone_steps"],
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1)",
            "lds_load_bytes_counter": prof.get("lds_load_bytes_per_launch"),
            "lds_load_bytes_counter_unit": "LDS load bytes per launch (rocprofv3 "
                                           "SQ_INSTS_LDS_LOAD_BANDWIDTH x 64 B), null if the "
                                           "profile predates the current kernel sources",
        },
        "cpu_baseline": None,
    }
    if not args.no_sweep and args.workload == "n150_r1604_arrhenius":
        out["launch_study"] = launch_study(net, buf, Y0, dt0, stream)
        log("launch study done")
    if not args.no_f32:
        out["f32"] = f32_leg(net, buf, Y0, dt0, stream, args.steps, b_step_fn=lambda: (
            algorithmic_bytes_per_zone_step(n.n_species, n.n_reactions, n.n_destruction, 4,
                                            net.get_launch()["variant"] == 1)), peak=peak,
            autotune=not args.no_autotune and launch is None)
    net.close()
    if not args.no_c4 and args.workload != "n365_r4400_arrhenius":
        _, net4, _, _, c4 = run_workload("n365_r4400_arrhenius", args.steps, args.warmup, peak,
                                         autotune=not args.no_autotune)
        net4.close()
        out["c4"] = c4
        log(f"365 species: {c4['time_to_t_end_ms']:.2f} ms")
    if not args.no_sweep:
        out["zone_count_sweep"] = zone_count_sweep(args.workload, SWEEP_COUNTS)
        log("zone-count sweep done")
    if not args.no_learned:
        out["learned"] = learned_leg(args.learned_zones)
        log("learned leg done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_leg(wl, args.cpu_sample_stride)
        log("cpu baseline done")
    print(json.dumps(out), flush=True)
    return 0


def learned_step_probe() -> dict:
    """Device cost of a learned zone-step against a plain one: 1024 zones of the 150-species
    constant-rate distribution (seed offset 1003) at tol 1e-2; the learned controller is driven
    by a fixed seeded network (untrained: its proposals are poor, so every zone runs to the
    200,000-attempt budget, which makes the count of attempted steps exact), each form timed as
    the median of 2 launches (HIP events on the launch stream)."""
    from paper_1409_5826_amd import binding, learned, workloads

    wl = workloads.preset("n150_r1604_const", n_zones=1024, seed_offset=1003)
    net = binding.Network(wl.network)
    mlp = binding.Mlp(1024)
    try:
        mlp.set_params(learned.initial_params(4005))
        net.set_mlp(mlp)
        rl = learned.integrate(net, wl.zones, 1e-2, True, repeats=2, max_steps=200_000)
        rp = learned.integrate(net, wl.zones, 1e-2, False, repeats=2)
    finally:
        mlp.close()
        net.close()
    att_l = int(rl.n_acc.sum() + rl.n_rej.sum())
    att_p = int(rp.n_acc.sum() + rp.n_rej.sum())
    return {"zones": 1024, "tol": 1e-2,
            "learned_ms": rl.ms, "learned_attempted_zone_steps": att_l,
            "learned_ns_per_zone_step": rl.ms * 1e6 / att_l,
            "plain_ms": rp.ms, "plain_attempted_zone_steps": att_p,
            "plain_ns_per_zone_step": rp.ms * 1e6 / att_p}


def mlp_train_probe(epochs: int) -> dict:
    """The learned leg's training loop (batch 1024, Adam) on 64 batches of seeded synthetic
    features and labels, after one untimed warm-up epoch: device time per step and samples per
    second."""
    import numpy as np
    import torch

    from paper_1409_5826_amd import learned

    rng = np.random.Generator(np.random.PCG64(5))
    n = 1024 * 64
    x = torch.tensor(rng.uniform(-1.0, 1.0, (n, learned.N_FEATURES)), dtype=torch.float32,
                     device="cuda")
    y = torch.tensor(rng.normal(size=n), dtype=torch.float32, device="cuda")
    tr = learned.Traces(x=x, y=y, zone=np.arange(n) // 1024, n_acc=np.zeros(n, np.int64), taken=n)
    va = learned.Traces(x=x[:1024], y=y[:1024], zone=np.zeros(1024, np.int64),
                        n_acc=np.zeros(1024, np.int64), taken=1024)
    learned.train(tr, va, epochs=1, batch=1024, lr=1e-3, seed=5).mlp.close()  # warm-up: code loading
    res = learned.train(tr, va, epochs=epochs, batch=1024, lr=1e-3, seed=5)
    res.mlp.close()
    steps = res.samples // 1024
    return {"mlp_train_steps": steps, "batch": 1024, "seconds": res.seconds,
            "us_per_step": res.seconds / steps * 1e6, "samples_per_s": res.samples / res.seconds,
            "achieved_tflops": res.samples * MLP_FLOP_PER_SAMPLE / res.seconds / 1e12}


def f32_leg(net, buf, Y0, dt0, stream, steps, b_step_fn, peak, autotune=True) -> dict:
    """The same workload integrated in single precision (HIP events).  The launch is tuned
    for single precision (outside the timed region) unless autotune is off, in which case the
    double-precision launch is kept."""
    import numpy as np
    import torch

    from paper_1409_5826_amd import binding

    opts = binding.options_default(precision=binding.PREC_F32)
    tuned = None
    if autotune:
        t0 = time.perf_counter()
        binding.asy_autotune(net.handle, net.n_species, net.n_reactions, Y0, buf["t_end"], dt0,
                             T=buf["T"], k_zone=buf["k_zone"], opts=opts)
        tuned = time.perf_counter() - t0
    times = []
    for i in range(steps + 1):
        buf["Y"].copy_(Y0)
        buf["dt"].copy_(dt0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        net.integrate(buf, opts, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        if i > 0:  # the first run warms up
            times.append(e0.elapsed_time(e1))
    acc = int(buf["n_accepted"].sum().item())
    att = acc + int(buf["n_rejected"].sum().item())
    ms = float(np.mean(times))
    b32 = b_step_fn()
    achieved = b32 * att / (ms / 1e3) / 1e9
    return {"time_to_t_end_ms": ms, "zone_steps_per_s": acc / (ms / 1e3),
            "accepted_zone_steps": acc, "rejected_zone_steps": att - acc,
            "bytes_per_zone_step": b32, "achieved_GBs": achieved, "frac": achieved / peak,
            "launch": net.get_launch(), "autotune_s": tuned}


# Algorithmic flops of the network per sample: forward 2 (166*128 + 128*128 + 128);
# backward (input and weight gradients) twice that.
MLP_FLOP_PER_SAMPLE = 3 * 2 * (166 * 128 + 128 * 128 + 128)
BF16_DENSE_PEAK_TFLOPS = 2500.0


C5_REFERENCE = os.path.join(ROOT, "tests", "golden", "c5_radau_reference.json")


def time_at_equal_error(curve_a, curve_b):
    """Each curve: [(error, ms), ...] from several tolerances.  Interpolates log(ms) against
    log(error) piecewise linearly and returns (error, ms_a, ms_b) at the smallest error both
    curves reach, or None when their error ranges do not overlap."""
    import numpy as np

    def interp(curve, e):
        pts = sorted(curve)
        le = np.log([p[0] for p in pts])
        lt = np.log([p[1] for p in pts])
        return float(np.exp(np.interp(np.log(e), le, lt)))

    if not curve_a or not curve_b:
        return None
    lo = max(min(p[0] for p in curve_a), min(p[0] for p in curve_b))
    hi = min(max(p[0] for p in curve_a), max(p[0] for p in curve_b))
    if not (lo <= hi):
        return None
    return lo, interp(curve_a, lo), interp(curve_b, lo)


def learned_leg(n_eval_zones: int, tols=(1e-2, 3e-3, 1e-3), tight_tols=(3e-4, 1e-4)) -> dict:
    """The learned step proposer against the plain controller on held-out zones of the
    150-species constant-rate distribution.

    Training: plain traces (boundary labels) at each tolerance on 128 training zones,
    2e5 pairs, each also for hypothetical last steps h 2^d (learned.augment_step_scale),
    20 epochs on the device.  Evaluation: both forms on n_eval_zones held-out
    zones at each tolerance; time to t_end of the whole batch; final-abundance error
    (mass-fraction L1) on the zones of the committed Radau reference; the time ratio at
    equal error interpolated from the two error-vs-time curves.  The plain form also runs at
    tight_tols, and the slope of its error against tol gives the tol a 1e-6 error would need."""
    import json as _json

    import numpy as np

    from paper_1409_5826_amd import binding, learned, workloads

    with open(C5_REFERENCE) as fh:
        ref = _json.load(fh)
    ev = workloads.preset(ref["workload"], n_zones=n_eval_zones, seed_offset=ref["seed_offset"])
    ref_idx = np.asarray(ref["zones"])
    ref_Y = np.asarray(ref["Y"])
    tr_wl = workloads.preset("n150_r1604_const", n_zones=128, seed_offset=2003)
    w = ev.network.weight.astype(np.float64)
    net = binding.Network(ev.network)
    try:
        per_tol = 200000 // len(tols)
        parts = []
        for tol in tols:
            stride = max(1, int(round(12 * 1e-2 / tol)))  # about as many records per tolerance
            # room for every record (about 230,000 per tolerance), so that which records are
            # kept does not depend on the order in which zones finish
            tr = learned.generate_traces(net, tr_wl.zones, tol, stride=stride, capacity=1 << 19)
            if tr.taken > (1 << 19):
                raise RuntimeError(f"trace buffer overflow at tol {tol}: {tr.taken} records")
            parts.append(learned.subsample(tr, per_tol, 4005))
        pairs = learned.augment_step_scale(learned.concat(parts), ev.network.n_species)
        tr_set, va_set = learned.split_by_zone(pairs, 0.1, 4005)
        log(f"learned: {len(pairs.zone)} training pairs")
        res = learned.train(tr_set, va_set, epochs=20, batch=1024, lr=1e-3, seed=4005)
        log(f"learned: trained, val loss {res.val_loss[-1]:.3e}")
        net.set_mlp(res.mlp)
        rows, curves = [], {"plain": [], "learned": []}
        drift = None
        for tol in tols:
            row = {"tol": tol}
            budget = None
            for form, is_learned in (("plain", False), ("learned", True)):
                # the learned form gets 4x the plain form's largest attempt count per zone: a
                # network that keeps shrinking the step ends there (status MAX_STEPS, counted)
                r = learned.integrate(net, ev.zones, tol, is_learned, repeats=1,
                                      max_steps=budget or 10_000_000)
                if budget is None:
                    budget = 4 * int((r.n_acc + r.n_rej).max())
                # a reference zone that did not reach t_end (the learned form's step budget)
                # counts as an infinite error
                done = r.status[ref_idx] == binding.ZONE_OK
                err = np.where(done, learned.mass_error(r.Y[ref_idx], ref_Y, w), np.inf)
                med = float(np.median(err))
                row[form] = {"ms": r.ms, "accepted_per_zone": float(r.n_acc.mean()),
                             "rejected_per_zone": float(r.n_rej.mean()),
                             "err_max_finished": float(err[done].max()) if done.any() else None,
                             "err_median": med if np.isfinite(med) else None,
                             "ref_zones_unfinished": int((~done).sum()),
                             "zones_ok": int((r.status == binding.ZONE_OK).sum()),
                             "max_steps": budget if is_learned else None}
                if np.isfinite(med):
                    curves[form].append((med, r.ms))
                log(f"learned: tol {tol:g} {form} {r.ms:.0f} ms, median error "
                    f"{np.median(err):.3g}")
                if form == "plain" and drift is None:
                    ratio = (r.Y @ w) / (ev.zones.Y0 @ w)
                    q = np.percentile(ratio, [10, 50, 90])
                    drift = {"tol": tol, "p10": q[0], "p50": q[1], "p90": q[2],
                             "max": float(ratio.max())}
            row["time_ratio_learned_over_plain"] = row["learned"]["ms"] / row["plain"]["ms"]
            rows.append(row)
        eq = time_at_equal_error(curves["plain"], curves["learned"])
        # the plain form alone at tighter tolerances: how its error falls toward the 1e-6 target
        tight = []
        for tol in tight_tols:
            r = learned.integrate(net, ev.zones, tol, False, repeats=1)
            done = r.status[ref_idx] == binding.ZONE_OK
            err = np.where(done, learned.mass_error(r.Y[ref_idx], ref_Y, w), np.inf)
            tight.append({"tol": tol, "ms": r.ms, "accepted_per_zone": float(r.n_acc.mean()),
                          "err_median": float(np.median(err))})
            log(f"learned: plain at tol {tol:g} {r.ms:.0f} ms, median error {np.median(err):.3g}")
        pts = [(row["tol"], row["plain"]["err_median"]) for row in rows] + \
              [(t["tol"], t["err_median"]) for t in tight]
        pts = [(t, e) for t, e in pts if e is not None and np.isfinite(e) and e > 0]
        order = tol_for_target = None
        if len(pts) >= 2:
            # least-squares slope of log error against log tol, and the tol it implies for 1e-6
            lt, le = np.log10([p[0] for p in pts]), np.log10([p[1] for p in pts])
            order, icpt = np.polyfit(lt, le, 1)
            tol_for_target = float(10.0 ** ((-6.0 - icpt) / order))
        sps = res.samples / res.seconds if res.seconds > 0 else None
        out = {
            "workload": f"{ev.name} held-out zones (seed offset {ref['seed_offset']}), "
                        f"{n_eval_zones} zones",
            "train": {"zones": 128, "tols": list(tols), "pairs": int(len(pairs.zone)),
                      "train_pairs": int(len(tr_set.zone)), "val_pairs": int(len(va_set.zone)),
                      "epochs": 20, "batch": 1024,
                      "train_loss": res.train_loss[-1], "val_loss": res.val_loss[-1],
                      "val_loss_mean_predictor": res.baseline_val_loss,
                      "samples_per_s": sps,
                      "achieved_tflops": None if sps is None else sps * MLP_FLOP_PER_SAMPLE / 1e12,
                      "peak_tflops_bf16": BF16_DENSE_PEAK_TFLOPS},
            "error_reference": f"scipy Radau (rtol {ref['rtol']:g}, atol {ref['atol']:g}) on "
                               f"zones {ref_idx[0]}..{ref_idx[-1]}, committed reference "
                               f"(estimated error {ref['error_estimate_mass_fraction_l1']:.1e})",
            "error_measure": "mass-fraction L1, sum_i w_i |Y_i - Y_ref_i|, median over the "
                             "reference zones (a zone that did not reach t_end counts as "
                             "infinite)",
            "curves": rows,
            "equal_error": None if eq is None else {
                "err_median": eq[0], "plain_ms": eq[1], "learned_ms": eq[2],
                "time_ratio_learned_over_plain": eq[2] / eq[1]},
            "target_err_1e-6_reached": bool(any(p[0] <= 1e-6 for p in curves["plain"] +
                                                curves["learned"])),
            "plain_tight_tols": tight,
            "plain_error_order_in_tol": None if order is None else float(order),
            "plain_tol_for_err_1e-6_extrapolated": tol_for_target,
            "plain_mass_drift": drift,
        }
        res.mlp.close()
        return out
    finally:
        net.close()


if __name__ == "__main__":
    sys.exit(main())
