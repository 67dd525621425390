"""The learned step proposer: traces, training and evaluation, all through the C ABI.

* Traces: the plain integrator run with trace output (asy_integrate_batch_trace)
  records, at sampled accepted states, the network input (166 features) and the
  boundary label: log2 of 0.9 times the largest step h 2^(q/32), q in [-96, 96],
  that the controller would accept from the state, over h (found in the kernel
  by bisection on q without changing the integration).
* Training: mean squared error on the labels, Adam on FP32 master weights, with
  the library's BF16-in / FP32-accumulate forward and backward kernels
  (asy_mlp_train_step).  Train / validation split by zone.
* Evaluation: the same zones integrated with the plain controller and with the
  learned one (asy_set_mlp + controller ASY_CTRL_LEARNED), timed with HIP events
  on the launch stream.

torch supplies device memory, streams, events and index shuffles; every step of
the method runs in the library's kernels.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import binding

N_FEATURES = binding.MLP_N_IN
N_IN_PAD, N_HID = 192, 128


def initial_params(seed: int) -> np.ndarray:
    """Seeded starting point in the ABI's flat layout (W1 [192x128], b1, W2 [128x128], b2,
    W3 [128], b3): He-uniform hidden layers (rows of W1 past 166 zero), a small output
    layer, zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w1 = np.zeros((N_IN_PAD, N_HID))
    w1[:N_FEATURES] = rng.uniform(-1.0, 1.0, size=(N_FEATURES, N_HID)) * np.sqrt(6.0 / N_FEATURES)
    w2 = rng.uniform(-1.0, 1.0, size=(N_HID, N_HID)) * np.sqrt(6.0 / N_HID)
    w3 = rng.uniform(-0.01, 0.01, size=N_HID)
    p = np.concatenate([w1.ravel(), np.zeros(N_HID), w2.ravel(), np.zeros(N_HID), w3, np.zeros(1)])
    assert p.size == binding.MLP_N_PARAMS
    return p.astype(np.float32)


@dataclass
class Traces:
    x: "object"        # torch float32 [n, 166] on the device
    y: "object"        # torch float32 [n]
    zone: np.ndarray   # int64 [n] zone index of each record
    n_acc: np.ndarray  # int64 [n] accepted-step index of each record
    taken: int         # records the kernel counted (before capacity and label filtering)


def generate_traces(net: binding.Network, zones, tol: float, stride: int = 1,
                    capacity: int = 1 << 20, max_steps: int = 10_000_000, stream=None) -> Traces:
    """Run the plain controller on `zones` with trace output; keep records with a label."""
    import torch

    buf = net.zone_buffers(zones)
    trace = torch.full((capacity, binding.TRACE_REC), float("nan"), dtype=torch.float32,
                       device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    opts = binding.options_default(tol=tol, max_steps=max_steps)
    net.integrate_trace(buf, trace, count, stride=stride, opts=opts, stream=stream)
    torch.cuda.synchronize()
    taken = int(count.item())
    rec = trace[:min(taken, capacity)]
    rec = rec[torch.isfinite(rec[:, 166])]
    # the kernel takes record slots in completion order; sort by (zone, step) so that
    # everything downstream (subsampling, splits, training) is deterministic
    zone = rec[:, 168].cpu().numpy().astype(np.int64)
    n_acc = rec[:, 169].cpu().numpy().astype(np.int64)
    order = np.lexsort((n_acc, zone))
    rec = rec.index_select(0, torch.as_tensor(order, device=rec.device))
    return Traces(x=rec[:, :N_FEATURES].contiguous(), y=rec[:, 166].contiguous(),
                  zone=zone[order], n_acc=n_acc[order], taken=taken)


# Octave shifts of the hypothetical last step used by augment_step_scale.
STEP_SHIFTS = (-10, -6, -3, -1, 1)
LABEL_CLIP = 3.0  # the proposal clamps the network output to [-3, 3]


def augment_step_scale(tr: Traces, n_species: int, shifts=STEP_SHIFTS) -> Traces:
    """Each record again for hypothetical last steps h 2^d, d in shifts.

    The label's boundary step h_b is a property of the state alone (its sums do not
    depend on the step that reached it), so for a last step h' = h 2^d the label is
    exactly log2(safety h_b / h') = label - d (clipped to the proposal's range), and
    the three step features log10(max k h)/10, log10(mean k h)/10, log10(h)/10 move
    by d log10(2) / 10; the abundances and the tolerance feature stay.  Plain traces
    only hold states whose last step sits just below the boundary; these records show
    the network where the boundary lies from every step size, so that its proposals
    return to it instead of drifting."""
    import torch

    xs, ys = [tr.x], [tr.y]
    for d in shifts:
        x = tr.x.clone()
        x[:, n_species:n_species + 3] += float(d) * float(np.log10(2.0)) / 10.0
        xs.append(x)
        ys.append((tr.y - float(d)).clamp(-LABEL_CLIP, LABEL_CLIP))
    k = 1 + len(shifts)
    return Traces(x=torch.cat(xs).contiguous(), y=torch.cat(ys).contiguous(),
                  zone=np.tile(tr.zone, k), n_acc=np.tile(tr.n_acc, k), taken=tr.taken)


def _select(tr: Traces, idx: np.ndarray) -> Traces:
    import torch

    it = torch.as_tensor(idx, device=tr.x.device)
    return Traces(x=tr.x.index_select(0, it).contiguous(), y=tr.y.index_select(0, it).contiguous(),
                  zone=tr.zone[idx], n_acc=tr.n_acc[idx], taken=tr.taken)


def concat(parts) -> Traces:
    import torch

    return Traces(x=torch.cat([p.x for p in parts]), y=torch.cat([p.y for p in parts]),
                  zone=np.concatenate([p.zone for p in parts]),
                  n_acc=np.concatenate([p.n_acc for p in parts]),
                  taken=sum(p.taken for p in parts))


def subsample(tr: Traces, n: int, seed: int) -> Traces:
    """n records drawn without replacement (seeded), in their original order."""
    if n >= len(tr.zone):
        return tr
    rng = np.random.Generator(np.random.PCG64(seed))
    return _select(tr, np.sort(rng.choice(len(tr.zone), n, replace=False)))


def split_by_zone(tr: Traces, val_frac: float, seed: int):
    """(train, validation): each zone's records all go to one side."""
    zones = np.unique(tr.zone)
    rng = np.random.Generator(np.random.PCG64(seed))
    n_val = max(1, int(round(val_frac * len(zones))))
    is_val = np.isin(tr.zone, rng.choice(zones, n_val, replace=False))
    return _select(tr, np.nonzero(~is_val)[0]), _select(tr, np.nonzero(is_val)[0])


@dataclass
class TrainResult:
    mlp: binding.Mlp
    train_loss: list = field(default_factory=list)   # per epoch, mean over its batches
    val_loss: list = field(default_factory=list)     # per epoch
    baseline_val_loss: float = 0.0                   # predicting the mean training label
    seconds: float = 0.0                             # device time of the training steps
    samples: int = 0                                 # samples processed


def mean_loss(mlp: binding.Mlp, x, y, batch: int) -> float:
    """Mean squared error over (x, y), from the library's loss, in batches of `batch`."""
    total, n = 0.0, int(x.shape[0])
    for i in range(0, n, batch):
        xb, yb = x[i:i + batch], y[i:i + batch]
        loss, _ = mlp.gradient(xb, yb)
        total += float(loss.item()) * int(xb.shape[0])
    return total / max(n, 1)


def train(train_set: Traces, val_set: Traces, epochs: int = 20, batch: int = 1024,
          lr: float = 1e-3, seed: int = 4005, params: Optional[np.ndarray] = None) -> TrainResult:
    """Adam on mean squared error, mini-batches of `batch` in a seeded order every epoch."""
    import torch

    mlp = binding.Mlp(batch)
    mlp.set_params(initial_params(seed) if params is None else params)
    res = TrainResult(mlp=mlp)
    y_mean = float(train_set.y.mean().item())
    yv = val_set.y.double()
    res.baseline_val_loss = float(((yv - y_mean) ** 2).mean().item())
    n = int(train_set.x.shape[0])
    rng = np.random.Generator(np.random.PCG64(seed))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(epochs):
        perm = torch.as_tensor(rng.permutation(n), device=train_set.x.device)
        xs, ys = train_set.x.index_select(0, perm), train_set.y.index_select(0, perm)
        losses = torch.zeros(n // batch, dtype=torch.float32, device="cuda")
        ev0.record()
        mlp.train_epoch(xs, ys, batch, lr=lr, losses=losses)  # n // batch steps, one call
        ev1.record()
        torch.cuda.synchronize()
        res.seconds += ev0.elapsed_time(ev1) / 1e3
        res.samples += (n // batch) * batch
        res.train_loss.append(float(losses.mean().item()))
        res.val_loss.append(mean_loss(mlp, val_set.x, val_set.y, batch))
    return res


@dataclass
class RunResult:
    Y: np.ndarray
    n_acc: np.ndarray
    n_rej: np.ndarray
    status: np.ndarray
    ms: float          # device time of one integration of the batch (HIP events, median)


def integrate(net: binding.Network, zones, tol: float, learned: bool, repeats: int = 3,
              max_steps: int = 10_000_000) -> RunResult:
    """Integrate `zones` from the same start `repeats` times; outputs of the last run and the
    median device time.  The learned controller needs net.set_mlp(...) first."""
    import torch

    buf = net.zone_buffers(zones)
    Y0, dt0 = buf["Y"].clone(), buf["dt"].clone()
    opts = binding.options_default(tol=tol, max_steps=max_steps,
                                   controller=binding.CTRL_LEARNED if learned else binding.CTRL_PLAIN)
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(repeats):
        buf["Y"].copy_(Y0)
        buf["dt"].copy_(dt0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        net.integrate(buf, opts, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return RunResult(Y=buf["Y"].cpu().numpy(), n_acc=buf["n_accepted"].cpu().numpy(),
                     n_rej=buf["n_rejected"].cpu().numpy(), status=buf["zone_status"].cpu().numpy(),
                     ms=float(np.median(times)))


def mass_error(Y: np.ndarray, Y_ref: np.ndarray, weight: np.ndarray) -> np.ndarray:
    """Per zone, the mass-fraction L1 distance sum_i w_i |Y_i - Y_ref_i|."""
    return np.abs(Y - Y_ref) @ np.asarray(weight, dtype=np.float64)
