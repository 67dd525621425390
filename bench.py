"""Benchmark of the batched explicit asymptotic integrator on one MI355X.

One step = one asy_integrate_batch call that integrates every zone of the
workload from t = 0 to t_end (rates, fluxes, creation/depletion sums,
kappa-switched updates and step control), starting from the same initial
state each time.  Inputs are resident in HBM before the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.  value = accepted zone-steps per second over the K
timed steps.  The "learned" object (skipped with --no-learned) compares the
learned step proposer with the plain controller on held-out zones of the
150-species constant-rate distribution: traces of the plain integrator on 128
training zones, 2e5 (features, label) pairs, training on the device, then
time-to-t_end and final-abundance error (mass-fraction L1 against the plain
integrator at tol 1e-4) of both forms at several tolerances.  roofline: the integrator is bound by LDS traffic; achieved =
algorithmic LDS bytes per attempted zone-step x attempted zone-steps per
launch / average launch time (HIP events on the launch stream); peak = the
larger of the nominal LDS bandwidth (256 CUs x 128 B/clock x 2.4 GHz) and the
read bandwidth measured on the device with conflict-free 8- and 16-byte LDS
reads.
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


def profiled_traffic(workload: str):
    """HBM bytes per launch from the committed rocprofv3 summary of this workload
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size), or None
    when there is no summary or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"integrate_strat_{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("|", "*", "#", "`")):
                key, _, val = line.partition(":")
                fields[key.strip()] = val.strip()
    if fields.get("kernel_source_sha256") != kernel_source_sha256():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def algorithmic_bytes_per_zone_step(n_species: int, n_reactions: int, n_destruction: int,
                                    value_bytes: int = 8) -> int:
    """LDS bytes one attempted step of one zone must move (value = 8 B in double, 4 B in
    single precision; index = 2 B).

    Per reaction: read k_j, write the flux, read it back with its product
    index (3 values + 2 B).  Per destruction incidence: gather the partner
    abundance with its index, write the partial rate, read it back (3 values
    + 2 B).  Per species: five reads/writes of Y, F+, k, Yn (5 values).
    """
    v = value_bytes
    return (3 * v + 2) * (n_reactions + n_destruction) + 5 * v * n_species


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
    ap.add_argument("--launch", default=None, help="JSON dict of asy_launch fields")
    ap.add_argument("--autotune", action="store_true",
                    help="time the candidate launch configurations on the workload first")
    ap.add_argument("--no-f32", action="store_true",
                    help="skip the single-precision measurement of the same workload")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-proposer comparison")
    ap.add_argument("--learned-zones", type=int, default=4096)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (calibrates HBM counters)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(zones are independent: they would shard across GPUs with no exchange)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1409_5826_amd import binding, workloads

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
    wl = workloads.preset(args.workload, n_zones=args.zones)
    net = binding.Network(wl.network)
    if args.launch:
        net.set_launch(**json.loads(args.launch))
    buf = net.zone_buffers(wl.zones)
    Y0 = buf["Y"].clone()
    dt0 = buf["dt"].clone()
    if args.autotune:
        binding.asy_autotune(net.handle, net.n_species, net.n_reactions, Y0, buf["t_end"], dt0,
                             T=buf["T"], k_zone=buf["k_zone"])
    stream = torch.cuda.current_stream()

    def step():
        buf["Y"].copy_(Y0)
        buf["dt"].copy_(dt0)
        net.integrate(buf, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        buf["Y"].copy_(Y0)
        buf["dt"].copy_(dt0)
        starts[i].record(stream)
        net.integrate(buf, stream=stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launch_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]

    n_acc = buf["n_accepted"].cpu().numpy()
    n_rej = buf["n_rejected"].cpu().numpy()
    status = buf["zone_status"].cpu().numpy()
    if not (status == binding.ZONE_OK).all():
        print(f"warning: {int((status != 0).sum())} zones did not reach t_end", file=sys.stderr)
    acc_per_step = int(n_acc.sum())
    att_per_step = int(n_acc.sum() + n_rej.sum())
    value = acc_per_step * args.steps / elapsed
    n = wl.network
    b_step = algorithmic_bytes_per_zone_step(n.n_species, n.n_reactions, n.n_destruction)
    avg_launch_s = float(np.mean(launch_ms)) / 1e3
    achieved = b_step * att_per_step / avg_launch_s / 1e9
    lds_measured = {w: binding.asy_probe_lds_bandwidth(w) / 1e9 for w in (8, 16)}
    peak = max(LDS_PEAK_GBS, *lds_measured.values())

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        idx = np.arange(0, wl.zones.n_zones, args.cpu_sample_stride)
        sub = wl.zones.subset(idx)
        threads = oracle.max_threads()
        tc = time.perf_counter()
        ref = oracle.integrate_batch(n, sub, n_threads=threads)
        tcpu = time.perf_counter() - tc
        cpu = {
            "value": float(ref["n_acc"].sum() / tcpu),
            "unit": "zone-steps/s",
            "cores": int(threads),
            "kind": "oracle",
            "sample": f"{len(idx)} of {wl.zones.n_zones} zones (every {args.cpu_sample_stride}th), "
                      f"{int(ref['n_acc'].sum())} accepted zone-steps in {tcpu:.2f} s",
        }

    out = {
        "metric": "zone-steps/sec and time-to-t_end for 4096 zones",
        "value": value,
        "unit": "zone-steps/s",
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
            "workload": wl.name,
            "description": wl.description,
            "zones": wl.zones.n_zones,
            "n_species": n.n_species,
            "n_reactions": n.n_reactions,
            "tol": wl.tol,
            "time_to_t_end_ms": float(np.mean(launch_ms)),
            "accepted_zone_steps": acc_per_step,
            "rejected_zone_steps": att_per_step - acc_per_step,
            "launch": net.get_launch(),
            "layout": (net.layout_info(net.get_launch()["threads_per_zone"])
                       if net.get_launch()["variant"] == 1 else None),
            "parallelism": "1 GPU",
        },
        "roofline": {
            "bound": "lds",
            "achieved": achieved,
            "peak": peak,
            "unit": "GB/s",
            "frac": achieved / peak,
            "peak_nominal": LDS_PEAK_GBS,
            "peak_measured": {f"ds_read_{8 * w}bit": v for w, v in lds_measured.items()},
            "traffic": profiled_traffic(wl.name),
            "bytes_per_zone_step": b_step,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1)",
        },
        "cpu_baseline": cpu,
    }
    if not args.no_f32:
        out["f32"] = f32_leg(net, buf, Y0, dt0, stream, args.steps, b_step_fn=lambda: (
            algorithmic_bytes_per_zone_step(n.n_species, n.n_reactions, n.n_destruction, 4)),
            peak=peak)
    net.close()
    if not args.no_learned:
        out["learned"] = learned_leg(args.learned_zones)
    print(json.dumps(out), flush=True)
    return 0


def f32_leg(net, buf, Y0, dt0, stream, steps, b_step_fn, peak) -> dict:
    """The same workload integrated in single precision (HIP events, same launch)."""
    import numpy as np
    import torch

    from paper_1409_5826_amd import binding

    opts = binding.options_default(precision=binding.PREC_F32)
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
            "launch": net.get_launch()}


# Algorithmic flops of the network per sample: forward 2 (166*128 + 128*128 + 128);
# backward (input and weight gradients) twice that.
MLP_FLOP_PER_SAMPLE = 3 * 2 * (166 * 128 + 128 * 128 + 128)
BF16_DENSE_PEAK_TFLOPS = 2500.0


def learned_leg(n_eval_zones: int, tols=(1e-2, 3e-3, 1e-3), tol_ref=1e-4) -> dict:
    """Learned step proposer against the plain controller (time and error at equal tol)."""
    import numpy as np

    from paper_1409_5826_amd import binding, learned, workloads

    ev = workloads.preset("n150_r1604_const", n_zones=n_eval_zones, seed_offset=1003)
    tr_wl = workloads.preset("n150_r1604_const", n_zones=128, seed_offset=2003)
    w = ev.network.weight.astype(np.float64)
    net = binding.Network(ev.network)
    try:
        traces = learned.generate_traces(net, tr_wl.zones, 1e-2, stride=12, capacity=400000)
        pairs = learned.subsample(traces, 200000, 4005)
        tr_set, va_set = learned.split_by_zone(pairs, 0.1, 4005)
        res = learned.train(tr_set, va_set, epochs=20, batch=1024, lr=1e-3, seed=4005)
        net.set_mlp(res.mlp)
        ref = learned.integrate(net, ev.zones, tol_ref, False, repeats=1)
        curves = []
        for tol in tols:
            row = {"tol": tol}
            for form, is_learned in (("plain", False), ("learned", True)):
                r = learned.integrate(net, ev.zones, tol, is_learned, repeats=1)
                err = learned.mass_error(r.Y, ref.Y, w)
                row[form] = {"ms": r.ms, "accepted_per_zone": float(r.n_acc.mean()),
                             "rejected_per_zone": float(r.n_rej.mean()),
                             "err_max": float(err.max()), "err_median": float(np.median(err)),
                             "zones_ok": int((r.status == binding.ZONE_OK).sum())}
            row["time_ratio_learned_over_plain"] = row["learned"]["ms"] / row["plain"]["ms"]
            curves.append(row)
        sps = res.samples / res.seconds if res.seconds > 0 else None
        out = {
            "workload": f"n150_r1604_const held-out zones (seed 3005), {n_eval_zones} zones",
            "train": {"zones": 128, "tol": 1e-2, "pairs": int(len(pairs.zone)),
                      "train_pairs": int(len(tr_set.zone)), "val_pairs": int(len(va_set.zone)),
                      "epochs": 20, "batch": 1024,
                      "train_loss": res.train_loss[-1], "val_loss": res.val_loss[-1],
                      "val_loss_mean_predictor": res.baseline_val_loss,
                      "samples_per_s": sps,
                      "achieved_tflops": None if sps is None else sps * MLP_FLOP_PER_SAMPLE / 1e12,
                      "peak_tflops_bf16": BF16_DENSE_PEAK_TFLOPS},
            "error_reference": f"plain integrator at tol {tol_ref:g}",
            "reference_accepted_per_zone": float(ref.n_acc.mean()),
            "curves": curves,
        }
        res.mlp.close()
        return out
    finally:
        net.close()


if __name__ == "__main__":
    sys.exit(main())
