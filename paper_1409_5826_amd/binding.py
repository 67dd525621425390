"""ctypes binding of the asynet C ABI (include/asynet.h).

Argument marshalling only: every step of the integration runs in the HIP
library.  torch supplies device memory and streams.  Importing this module
does not touch the GPU; loading the library does, and it raises if the
library has not been built (python -m paper_1409_5826_amd.build) -- there is
no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libasynet.so")

ASY_OK, ASY_EINVAL, ASY_ENOMEM, ASY_EDEVICE, ASY_ENOTSUP, ASY_ESTATE = 0, -1, -2, -3, -4, -5
ZONE_OK, ZONE_MAX_STEPS, ZONE_DT_UNDERFLOW, ZONE_NONFINITE, ZONE_BAD_INPUT = range(5)
RATES_PER_ZONE, RATES_ARRHENIUS = 0, 1
CTRL_PLAIN, CTRL_LEARNED = 0, 1
PREC_F64, PREC_F32 = 0, 1

# Every symbol include/asynet.h declares.
EXPORTS = (
    "asy_options_default",
    "asy_network_create",
    "asy_network_destroy",
    "asy_integrate_batch",
    "asy_integrate_batch_noalloc",
    "asy_get_launch",
    "asy_set_launch",
    "asy_autotune",
    "asy_last_error",
    "asy_version",
    "asy_mlp_create",
    "asy_mlp_destroy",
    "asy_mlp_set_params",
    "asy_mlp_get_params",
    "asy_mlp_forward",
    "asy_mlp_gradient",
    "asy_mlp_train_step",
    "asy_mlp_train_epoch",
    "asy_mlp_infer",
    "asy_set_mlp",
    "asy_integrate_batch_trace",
    "asy_probe_lds_bandwidth",
    "asy_integrate_schedule",
    "asy_network_layout_info",
)

MLP_N_IN = 166
MLP_N_PARAMS = 41345
TRACE_REC = 170


class AsyError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


class asy_network_desc(C.Structure):
    _fields_ = [
        ("n_species", C.c_int32),
        ("n_reactions", C.c_int32),
        ("reactant0", C.c_void_p),
        ("reactant1", C.c_void_p),
        ("product", C.c_void_p),
        ("weight", C.c_void_p),
        ("rate_form", C.c_int32),
        ("A", C.c_void_p),
        ("E", C.c_void_p),
        ("split_above", C.c_int32),
    ]


class asy_options(C.Structure):
    _fields_ = [
        ("kappa", C.c_double),
        ("tol", C.c_double),
        ("y_floor", C.c_double),
        ("grow_max", C.c_double),
        ("safety", C.c_double),
        ("shrink_min", C.c_double),
        ("dt_min", C.c_double),
        ("max_steps", C.c_int64),
        ("controller", C.c_int32),
        ("precision", C.c_int32),
    ]


class asy_launch(C.Structure):
    _fields_ = [
        ("variant", C.c_int32),
        ("threads_per_zone", C.c_int32),
        ("zones_per_group", C.c_int32),
        ("groups_per_cu", C.c_int32),
        ("use_graph", C.c_int32),
        ("zone_order", C.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class asy_layout_info(C.Structure):
    _fields_ = [
        ("available", C.c_int32),
        ("slots", C.c_int32),
        ("slots_used", C.c_int32),
        ("species_per_lane", C.c_int32),
        ("split_rows", C.c_int32),
        ("one_factor_waves", C.c_uint32),
        ("gather_cycles_packed", C.c_int64),
        ("gather_cycles_placed", C.c_int64),
        ("one_factor_slots", C.c_int32),
        ("one_factor_slots_run", C.c_int32),
        ("two_factor_wave_slots", C.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib():
    """Load libasynet.so (raises if it is missing: there is no other path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1409_5826_amd.build")
        L = C.CDLL(LIB_PATH)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        L.asy_options_default.argtypes = [C.POINTER(asy_options)]
        L.asy_options_default.restype = None
        L.asy_network_create.argtypes = [C.POINTER(asy_network_desc), C.POINTER(P)]
        L.asy_network_create.restype = I32
        L.asy_network_destroy.argtypes = [P]
        L.asy_network_destroy.restype = None
        L.asy_integrate_batch.argtypes = [P, C.POINTER(asy_options), I32, P, P, P, P, P, P, P, P, P]
        L.asy_integrate_batch.restype = I32
        L.asy_integrate_batch_noalloc.argtypes = [P, C.POINTER(asy_options), I32, P, P, P, P, P, P,
                                                  P, P, P]
        L.asy_integrate_batch_noalloc.restype = I32
        L.asy_get_launch.argtypes = [P, C.POINTER(asy_launch)]
        L.asy_get_launch.restype = I32
        L.asy_network_layout_info.argtypes = [P, I32, C.POINTER(asy_layout_info)]
        L.asy_network_layout_info.restype = I32
        L.asy_set_launch.argtypes = [P, C.POINTER(asy_launch)]
        L.asy_set_launch.restype = I32
        L.asy_autotune.argtypes = [P, C.POINTER(asy_options), I32, P, P, P, P, P, C.POINTER(asy_launch)]
        L.asy_autotune.restype = I32
        L.asy_last_error.argtypes = []
        L.asy_last_error.restype = C.c_char_p
        L.asy_version.argtypes = []
        L.asy_version.restype = C.c_char_p
        F = C.c_float
        L.asy_mlp_create.argtypes = [I32, C.POINTER(P)]
        L.asy_mlp_destroy.argtypes = [P]
        L.asy_mlp_destroy.restype = None
        L.asy_mlp_set_params.argtypes = [P, P]
        L.asy_mlp_get_params.argtypes = [P, P]
        L.asy_mlp_forward.argtypes = [P, I32, P, P, P]
        L.asy_mlp_gradient.argtypes = [P, I32, P, P, P, P, P]
        L.asy_mlp_train_step.argtypes = [P, I32, P, P, F, P, P]
        L.asy_mlp_train_epoch.argtypes = [P, I32, I32, P, P, F, P, P]
        L.asy_mlp_infer.argtypes = [P, I32, P, P, P]
        L.asy_set_mlp.argtypes = [P, P]
        L.asy_integrate_schedule.argtypes = [P, C.POINTER(asy_options), I32, I32, P, P, P, P, P, P,
                                             P, P, P, P, P]
        L.asy_probe_lds_bandwidth.argtypes = [I32, C.POINTER(C.c_double)]
        L.asy_probe_lds_bandwidth.restype = I32
        L.asy_integrate_batch_trace.argtypes = [P, C.POINTER(asy_options), I32, P, P, P, P, P, P,
                                                P, P, P, C.c_int64, P, I32, I32, P]
        for name in ("asy_mlp_create", "asy_mlp_set_params", "asy_mlp_get_params", "asy_mlp_forward",
                     "asy_mlp_gradient", "asy_mlp_train_step", "asy_mlp_train_epoch", "asy_mlp_infer",
                     "asy_set_mlp"):
            getattr(L, name).restype = I32
        _ = I64
        _lib = L
    return _lib


def last_error() -> str:
    return lib().asy_last_error().decode()


def _check(st: int, where: str):
    if st != ASY_OK:
        raise AsyError(st, where, last_error())


def options_default(**overrides) -> asy_options:
    o = asy_options()
    lib().asy_options_default(C.byref(o))
    for key, val in overrides.items():
        setattr(o, key, val)
    return o


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def asy_network_create(n_species, reactant0, reactant1, product, weight=None, A=None, E=None,
                       split_above=0):
    """Create a handle from host arrays; returns the opaque pointer (int)."""
    r0, r1, pr = _i32(reactant0), _i32(reactant1), _i32(product)
    w = None if weight is None else _i32(weight)
    a = None if A is None else _f64(A)
    e = None if E is None else _f64(E)
    d = asy_network_desc(
        n_species=int(n_species), n_reactions=len(r0),
        reactant0=r0.ctypes.data, reactant1=r1.ctypes.data, product=pr.ctypes.data,
        weight=None if w is None else w.ctypes.data,
        rate_form=RATES_ARRHENIUS if (a is not None or e is not None) else RATES_PER_ZONE,
        A=None if a is None else a.ctypes.data, E=None if e is None else e.ctypes.data,
        split_above=int(split_above))
    h = C.c_void_p()
    _check(lib().asy_network_create(C.byref(d), C.byref(h)), "asy_network_create")
    return h.value


def asy_network_destroy(handle):
    lib().asy_network_destroy(handle)


def _dev_ptr(t, dtype, shape, name):
    import torch

    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream_ptr(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


NOALLOC_MAX_ZONES = 1 << 18
NOALLOC_RATE_BYTES = 65011456  # rate-table part of the no-alloc scratch (Arrhenius networks)


def asy_integrate_batch(handle, n_species, n_reactions, Y, t_end, dt, n_accepted, n_rejected,
                        zone_status, T=None, k_zone=None, opts: Optional[asy_options] = None,
                        stream=None, noalloc: bool = False):
    """Queue the integration of Y.shape[0] zones on `stream` (default: torch's current).
    noalloc=True calls asy_integrate_batch_noalloc (static device scratch, no allocation)."""
    import torch

    Z = int(Y.shape[0])
    args = [
        _dev_ptr(Y, torch.float64, (Z, n_species), "Y"),
        _dev_ptr(T, torch.float64, (Z,), "T"),
        _dev_ptr(k_zone, torch.float64, (Z, n_reactions), "k_zone"),
        _dev_ptr(t_end, torch.float64, (Z,), "t_end"),
        _dev_ptr(dt, torch.float64, (Z,), "dt"),
        _dev_ptr(n_accepted, torch.int64, (Z,), "n_accepted"),
        _dev_ptr(n_rejected, torch.int64, (Z,), "n_rejected"),
        _dev_ptr(zone_status, torch.int32, (Z,), "zone_status"),
    ]
    fn = lib().asy_integrate_batch_noalloc if noalloc else lib().asy_integrate_batch
    st = fn(handle, None if opts is None else C.byref(opts), Z, *args, _stream_ptr(stream))
    _check(st, "asy_integrate_batch_noalloc" if noalloc else "asy_integrate_batch")


def asy_integrate_batch_trace(handle, n_species, n_reactions, Y, t_end, dt, n_accepted, n_rejected,
                              zone_status, trace, count, stride, trace_zones, T=None, k_zone=None,
                              opts: Optional[asy_options] = None, stream=None):
    """asy_integrate_batch that also writes training records into trace [capacity, TRACE_REC]."""
    import torch

    Z = int(Y.shape[0])
    cap = int(trace.shape[0])
    args = [
        _dev_ptr(Y, torch.float64, (Z, n_species), "Y"),
        _dev_ptr(T, torch.float64, (Z,), "T"),
        _dev_ptr(k_zone, torch.float64, (Z, n_reactions), "k_zone"),
        _dev_ptr(t_end, torch.float64, (Z,), "t_end"),
        _dev_ptr(dt, torch.float64, (Z,), "dt"),
        _dev_ptr(n_accepted, torch.int64, (Z,), "n_accepted"),
        _dev_ptr(n_rejected, torch.int64, (Z,), "n_rejected"),
        _dev_ptr(zone_status, torch.int32, (Z,), "zone_status"),
        _dev_ptr(trace, torch.float32, (cap, TRACE_REC), "trace"),
        cap,
        _dev_ptr(count, torch.int64, (1,), "count"),
        int(stride), int(trace_zones),
    ]
    st = lib().asy_integrate_batch_trace(handle, None if opts is None else C.byref(opts), Z, *args,
                                         _stream_ptr(stream))
    _check(st, "asy_integrate_batch_trace")


def asy_integrate_schedule(handle, n_species, n_reactions, Y, dt_hydro, dt, n_accepted,
                           n_rejected, zone_status, T=None, k_zone=None, q=None, energy=None,
                           opts: Optional[asy_options] = None, stream=None):
    """Queue len(dt_hydro) operator-split hydro steps (device [n_steps, Z] schedule arrays)."""
    import torch

    Z = int(Y.shape[0])
    S = int(dt_hydro.shape[0])
    args = [
        _dev_ptr(Y, torch.float64, (Z, n_species), "Y"),
        _dev_ptr(T, torch.float64, (S, Z), "T"),
        _dev_ptr(k_zone, torch.float64, (Z, n_reactions), "k_zone"),
        _dev_ptr(dt_hydro, torch.float64, (S, Z), "dt_hydro"),
        _dev_ptr(dt, torch.float64, (Z,), "dt"),
        _dev_ptr(q, torch.float64, (n_species,), "q"),
        _dev_ptr(energy, torch.float64, (S, Z), "energy"),
        _dev_ptr(n_accepted, torch.int64, (Z,), "n_accepted"),
        _dev_ptr(n_rejected, torch.int64, (Z,), "n_rejected"),
        _dev_ptr(zone_status, torch.int32, (Z,), "zone_status"),
    ]
    st = lib().asy_integrate_schedule(handle, None if opts is None else C.byref(opts), Z, S,
                                      *args, _stream_ptr(stream))
    _check(st, "asy_integrate_schedule")


def asy_get_launch(handle) -> asy_launch:
    c = asy_launch()
    _check(lib().asy_get_launch(handle, C.byref(c)), "asy_get_launch")
    return c


def asy_set_launch(handle, **fields):
    c = asy_get_launch(handle)
    for key, val in fields.items():
        setattr(c, key, int(val))
    _check(lib().asy_set_launch(handle, C.byref(c)), "asy_set_launch")


def asy_autotune(handle, n_species, n_reactions, Y, t_end, dt, T=None, k_zone=None,
                 sample_zones=None, opts: Optional[asy_options] = None) -> asy_launch:
    import torch

    Z = int(Y.shape[0])
    n_sample = Z if sample_zones is None else int(sample_zones)
    if not 1 <= n_sample <= Z:
        # the library copies sample_zones zones out of each array
        raise ValueError(f"sample_zones must be in [1, {Z}] (the zones in Y), got {n_sample}")
    best = asy_launch()
    st = lib().asy_autotune(
        handle, None if opts is None else C.byref(opts), n_sample,
        _dev_ptr(Y, torch.float64, (Z, n_species), "Y"), _dev_ptr(T, torch.float64, (Z,), "T"),
        _dev_ptr(k_zone, torch.float64, (Z, n_reactions), "k_zone"),
        _dev_ptr(t_end, torch.float64, (Z,), "t_end"), _dev_ptr(dt, torch.float64, (Z,), "dt"),
        C.byref(best))
    _check(st, "asy_autotune")
    return best


def asy_probe_lds_bandwidth(width_bytes: int = 16) -> float:
    """Measured LDS read bandwidth of the current device, bytes per second."""
    out = C.c_double()
    _check(lib().asy_probe_lds_bandwidth(int(width_bytes), C.byref(out)), "asy_probe_lds_bandwidth")
    return out.value


def asy_version() -> str:
    return lib().asy_version().decode()


class Network:
    """Convenience owner of a handle built from a workloads.Network."""

    def __init__(self, net, split_above=0):
        self.n_species = int(net.n_species)
        self.n_reactions = int(net.n_reactions)
        self.arrhenius = net.A is not None
        self.handle = asy_network_create(net.n_species, net.reactant0, net.reactant1, net.product,
                                         net.weight, net.A, net.E, split_above)

    def close(self):
        if self.handle:
            asy_network_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def zone_buffers(self, zones, device="cuda"):
        """Device copies of a workloads.Zones batch plus output buffers."""
        import torch

        Z = zones.n_zones
        buf = dict(
            Y=torch.as_tensor(zones.Y0, dtype=torch.float64, device=device).contiguous(),
            t_end=torch.as_tensor(zones.t_end, dtype=torch.float64, device=device),
            dt=torch.as_tensor(zones.dt0, dtype=torch.float64, device=device).clone(),
            n_accepted=torch.zeros(Z, dtype=torch.int64, device=device),
            n_rejected=torch.zeros(Z, dtype=torch.int64, device=device),
            zone_status=torch.full((Z,), -1, dtype=torch.int32, device=device),
            T=None if zones.T is None else torch.as_tensor(zones.T, dtype=torch.float64, device=device),
            k_zone=None if zones.k is None else torch.as_tensor(zones.k, dtype=torch.float64,
                                                                  device=device).contiguous(),
        )
        return buf

    def integrate(self, buf, opts=None, stream=None, noalloc=False):
        asy_integrate_batch(self.handle, self.n_species, self.n_reactions, buf["Y"], buf["t_end"],
                            buf["dt"], buf["n_accepted"], buf["n_rejected"], buf["zone_status"],
                            T=buf["T"], k_zone=buf["k_zone"], opts=opts, stream=stream,
                            noalloc=noalloc)

    def integrate_trace(self, buf, trace, count, stride=1, trace_zones=None, opts=None,
                        stream=None):
        Z = int(buf["Y"].shape[0])
        asy_integrate_batch_trace(self.handle, self.n_species, self.n_reactions, buf["Y"],
                                  buf["t_end"], buf["dt"], buf["n_accepted"], buf["n_rejected"],
                                  buf["zone_status"], trace, count, stride,
                                  Z if trace_zones is None else trace_zones, T=buf["T"],
                                  k_zone=buf["k_zone"], opts=opts, stream=stream)

    def integrate_schedule(self, buf, sched, opts=None, stream=None, with_energy=True):
        """Run a workloads.Schedule on the zones in buf; returns the energy [n_steps, Z] (device)."""
        import torch

        dev = buf["Y"].device
        S, Z = sched.dt_hydro.shape
        dt_h = torch.as_tensor(sched.dt_hydro, dtype=torch.float64, device=dev).contiguous()
        T = None if sched.T is None else torch.as_tensor(sched.T, dtype=torch.float64,
                                                         device=dev).contiguous()
        q = torch.as_tensor(sched.q, dtype=torch.float64, device=dev)
        energy = torch.zeros((S, Z), dtype=torch.float64, device=dev) if with_energy else None
        asy_integrate_schedule(self.handle, self.n_species, self.n_reactions, buf["Y"], dt_h,
                               buf["dt"], buf["n_accepted"], buf["n_rejected"], buf["zone_status"],
                               T=T, k_zone=buf["k_zone"], q=q, energy=energy, opts=opts,
                               stream=stream)
        return energy

    def set_mlp(self, mlp: "Mlp"):
        asy_set_mlp(self.handle, mlp)

    def set_launch(self, **fields):
        asy_set_launch(self.handle, **fields)

    def get_launch(self) -> dict:
        return asy_get_launch(self.handle).as_dict()

    def layout_info(self, threads_per_zone: int) -> dict:
        info = asy_layout_info()
        _check(lib().asy_network_layout_info(self.handle, int(threads_per_zone), C.byref(info)),
               "asy_network_layout_info")
        return info.as_dict()


class Mlp:
    """Owner of an asy_mlp training context (device memory for batches of batch_max)."""

    def __init__(self, batch_max: int):
        h = C.c_void_p()
        _check(lib().asy_mlp_create(int(batch_max), C.byref(h)), "asy_mlp_create")
        self.handle = h.value
        self.batch_max = int(batch_max)

    def close(self):
        if self.handle:
            lib().asy_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (MLP_N_PARAMS,):
            raise ValueError(f"params must have {MLP_N_PARAMS} values")
        _check(lib().asy_mlp_set_params(self.handle, p.ctypes.data), "asy_mlp_set_params")

    def get_params(self) -> np.ndarray:
        p = np.empty(MLP_N_PARAMS, dtype=np.float32)
        _check(lib().asy_mlp_get_params(self.handle, p.ctypes.data), "asy_mlp_get_params")
        return p

    def _xy(self, x, y=None):
        import torch

        n = int(x.shape[0])
        xp = _dev_ptr(x, torch.float32, (n, MLP_N_IN), "x")
        yp = None if y is None else _dev_ptr(y, torch.float32, (n,), "y")
        return n, xp, yp

    def forward(self, x, stream=None):
        import torch

        n, xp, _ = self._xy(x)
        o = torch.empty(n, dtype=torch.float32, device=x.device)
        _check(lib().asy_mlp_forward(self.handle, n, xp, o.data_ptr(), _stream_ptr(stream)),
               "asy_mlp_forward")
        return o

    def infer(self, x, stream=None):
        import torch

        n, xp, _ = self._xy(x)
        o = torch.empty(n, dtype=torch.float32, device=x.device)
        _check(lib().asy_mlp_infer(self.handle, n, xp, o.data_ptr(), _stream_ptr(stream)),
               "asy_mlp_infer")
        return o

    def gradient(self, x, y, stream=None):
        import torch

        n, xp, yp = self._xy(x, y)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        grad = torch.empty(MLP_N_PARAMS, dtype=torch.float32, device=x.device)
        _check(lib().asy_mlp_gradient(self.handle, n, xp, yp, loss.data_ptr(), grad.data_ptr(),
                                      _stream_ptr(stream)), "asy_mlp_gradient")
        return loss, grad

    def train_step(self, x, y, lr=1e-3, loss=None, stream=None):
        n, xp, yp = self._xy(x, y)
        _check(lib().asy_mlp_train_step(self.handle, n, xp, yp, float(lr),
                                        None if loss is None else loss.data_ptr(),
                                        _stream_ptr(stream)), "asy_mlp_train_step")

    def train_epoch(self, x, y, batch: int, lr=1e-3, losses=None, stream=None):
        """x.shape[0] // batch Adam steps over consecutive batches of (x, y) in one call;
        losses (device float32 [steps], optional) receives each step's loss."""
        import torch

        steps = int(x.shape[0]) // int(batch)
        if steps == 0:
            return 0
        n = steps * int(batch)
        xp = _dev_ptr(x[:n], torch.float32, (n, MLP_N_IN), "x")
        yp = _dev_ptr(y[:n], torch.float32, (n,), "y")
        lp = None
        if losses is not None:
            lp = _dev_ptr(losses, torch.float32, (steps,), "losses")
        _check(lib().asy_mlp_train_epoch(self.handle, steps, int(batch), xp, yp, float(lr), lp,
                                         _stream_ptr(stream)), "asy_mlp_train_epoch")
        return steps


def asy_set_mlp(net_handle, mlp: "Mlp"):
    _check(lib().asy_set_mlp(net_handle, mlp.handle), "asy_set_mlp")
