"""CPU oracle of the explicit asymptotic integrator (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It never imports the product package and the product
never imports it; the two share only the seeded input arrays.

The integrator itself is plain C (oracle.c), compiled with gcc and loaded here
through ctypes; `build()` compiles it.  The MLP reference of the learned
controller lives in `oracle.mlp` (numpy, FP64).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ZONE_OK, ZONE_MAX_STEPS, ZONE_DT_UNDERFLOW, ZONE_NONFINITE, ZONE_BAD_INPUT = range(5)


class Options(C.Structure):
    _fields_ = [
        ("kappa", C.c_double),
        ("tol", C.c_double),
        ("y_floor", C.c_double),
        ("grow_max", C.c_double),
        ("safety", C.c_double),
        ("shrink_min", C.c_double),
        ("dt_min", C.c_double),
        ("max_steps", C.c_int64),
        ("split_above", C.c_int32),
    ]


def options(**kw) -> Options:
    """Controller settings; defaults are the readings of the unspecified controller.
    split_above > 0 sums rows of more terms in chunks (see rhs); 0 sums every row in one pass."""
    d = dict(kappa=1.0, tol=0.01, y_floor=1e-10, grow_max=2.0, safety=0.9,
             shrink_min=0.1, dt_min=1e-20, max_steps=10_000_000, split_above=0)
    d.update(kw)
    return Options(**d)


# gcc flags of every build: no fused multiply-add contraction, no value-changing
# optimisation (the arithmetic is evaluated as written, in order)
_CFLAGS = ["-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fopenmp"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", *_CFLAGS, _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def build_for_this_host(path: str) -> str:
    """Compile a copy of the oracle for timing on the machine that runs it: -O3 and
    -march=native on top of the flags above (same arithmetic, same results), written to path."""
    cmd = ["gcc", "-O3", "-march=native", *_CFLAGS, _SRC, "-o", path + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(path + ".tmp", path)
    return path


_lib = None
_lib_path = _LIB


def use_library(path: str) -> None:
    """Load the oracle from path (a build_for_this_host copy) from now on."""
    global _lib, _lib_path
    _lib, _lib_path = None, path


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_lib_path):
            build()
        L = C.CDLL(_lib_path)
        P = C.c_void_p
        L.orc_rates_arrhenius.argtypes = [C.c_int32, P, P, C.c_double, P]
        L.orc_exp_for_tests.argtypes = [C.c_double]
        L.orc_exp_for_tests.restype = C.c_double
        L.orc_rhs.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P, P, P]
        L.orc_rhs_rows.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P, C.c_int32, P, P]
        L.orc_rhs_rows_f32.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P, C.c_int32, P, P]
        L.orc_update.argtypes = [C.c_int32, P, P, P, C.c_double, C.c_double, P, P]
        L.orc_change.argtypes = [C.c_int32, P, P, C.c_double]
        L.orc_change.restype = C.c_double
        L.orc_integrate_zone.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P, C.c_double, P,
                                         C.POINTER(Options), P, P, P]
        L.orc_integrate_zone.restype = C.c_int32
        L.orc_integrate_batch.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P, C.c_int32, P, P, P,
                                          P, P, P, P, P, C.POINTER(Options), C.c_int32]
        L.orc_max_threads.restype = C.c_int32
        L.orc_integrate_schedule.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P,
                                             C.c_int32, C.c_int32, P, P, P, P, P, P, P, P, P, P,
                                             C.POINTER(Options), C.c_int32]
        L.orc_rhs_f32.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P, P, P]
        L.orc_update_f32.argtypes = [C.c_int32, P, P, P, C.c_float, C.c_float, P]
        L.orc_integrate_zone_f32.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P, C.c_double, P,
                                             C.POINTER(Options), P, P]
        L.orc_integrate_zone_f32.restype = C.c_int32
        L.orc_integrate_batch_prec.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P,
                                               C.c_int32, P, P, P, P, P, P, P, P,
                                               C.POINTER(Options), C.c_int32]
        L.orc_mlp_forward.argtypes = [P, P]
        L.orc_mlp_forward.restype = C.c_double
        L.orc_mlp_forward_mfma.argtypes = [P, P]
        L.orc_mlp_forward_mfma.restype = C.c_float
        L.orc_mfma_dot.argtypes = [C.c_float, P, P, C.c_int32]
        L.orc_mfma_dot.restype = C.c_float
        L.orc_mlp_features.argtypes = [C.c_int32, P, P, C.c_double, C.c_double, P]
        L.orc_integrate_zone_learned.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P, C.c_double, P,
                                                 C.POINTER(Options), C.c_int32, P, P, C.c_int64,
                                                 C.POINTER(_LearnLog), P, P]
        L.orc_integrate_zone_learned.restype = C.c_int32
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class _Trace(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("count", C.c_int64), ("h", C.c_void_p),
                ("r", C.c_void_p), ("accepted", C.c_void_p)]


class _LearnLog(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("count", C.c_int64), ("q", C.c_void_p),
                ("feat", C.c_void_p), ("label", C.c_void_p), ("n_acc", C.c_void_p),
                ("label_stride", C.c_int64)]


def exp_cw(x: float) -> float:
    """The oracle's exponential of the Arrhenius factor (Cody-Waite reduction, Taylor degree 13)."""
    return float(lib().orc_exp_for_tests(float(x)))


def rates_arrhenius(A, E, T) -> np.ndarray:
    A, E = _f64(A), _f64(E)
    k = np.empty_like(A)
    lib().orc_rates_arrhenius(len(A), _p(A), _p(E), float(T), _p(k))
    return k


def rhs(net, k, Y, split_above: int = 0):
    """(F+, k_depletion) of Eq. eq1.1 at state Y.  split_above > 0: rows (the F+ or the k of
    one species) of more terms are summed in chunks of split_above / 2 terms (rounded down to a
    multiple of 4), whose sums are then added in order; otherwise every row in one pass."""
    a, b, c = _i32(net.reactant0), _i32(net.reactant1), _i32(net.product)
    k, Y = _f64(k), _f64(Y)
    n = net.n_species
    Fp, kd = np.empty(n), np.empty(n)
    if split_above > 0:
        lib().orc_rhs_rows(n, len(a), _p(a), _p(b), _p(c), _p(k), _p(Y), int(split_above),
                           _p(Fp), _p(kd))
    else:
        lib().orc_rhs(n, len(a), _p(a), _p(b), _p(c), _p(k), _p(Y), _p(Fp), _p(kd))
    return Fp, kd


def update(Y, Fp, kd, h, kappa=1.0):
    """(Yn, branch) of one kappa-switched step; branch 1 = asymptotic form."""
    Y, Fp, kd = _f64(Y), _f64(Fp), _f64(kd)
    Yn = np.empty_like(Y)
    br = np.empty(len(Y), dtype=np.int32)
    lib().orc_update(len(Y), _p(Y), _p(Fp), _p(kd), float(h), float(kappa), _p(Yn), _p(br))
    return Yn, br


def change(Y, Yn, y_floor=1e-10) -> float:
    Y, Yn = _f64(Y), _f64(Yn)
    return lib().orc_change(len(Y), _p(Y), _p(Yn), float(y_floor))


def integrate_zone(net, k, Y0, t_end, dt0, opts: Optional[Options] = None, trace_capacity=0):
    """Integrate one zone; returns dict(Y, dt, n_acc, n_rej, status[, trace])."""
    opts = opts or options()
    a, b, c = _i32(net.reactant0), _i32(net.reactant1), _i32(net.product)
    k = _f64(k)
    Y = _f64(Y0).copy()
    dt = np.array([dt0], dtype=np.float64)
    na = np.zeros(1, np.int64)
    nr = np.zeros(1, np.int64)
    tr = None
    trp = None
    if trace_capacity:
        th = np.zeros(trace_capacity)
        trr = np.zeros(trace_capacity)
        tacc = np.zeros(trace_capacity, np.int32)
        tr = _Trace(trace_capacity, 0, th.ctypes.data, trr.ctypes.data, tacc.ctypes.data)
        trp = C.byref(tr)
    st = lib().orc_integrate_zone(net.n_species, len(a), _p(a), _p(b), _p(c), _p(k), _p(Y),
                                  float(t_end), _p(dt), C.byref(opts), _p(na), _p(nr), trp)
    out = dict(Y=Y, dt=float(dt[0]), n_acc=int(na[0]), n_rej=int(nr[0]), status=int(st))
    if tr is not None:
        n = min(tr.count, trace_capacity)
        out["trace"] = dict(h=th[:n].copy(), r=trr[:n].copy(), accepted=tacc[:n].astype(bool),
                            count=int(tr.count))
    return out


def rhs_f32(net, k, Y, split_above: int = 0):
    """(F+, k_depletion) in float (inputs rounded to float first); split_above as in rhs."""
    a, b, c = _i32(net.reactant0), _i32(net.reactant1), _i32(net.product)
    k, Y = np.ascontiguousarray(k, np.float32), np.ascontiguousarray(Y, np.float32)
    n = net.n_species
    Fp, kd = np.empty(n, np.float32), np.empty(n, np.float32)
    if split_above > 0:
        lib().orc_rhs_rows_f32(n, len(a), _p(a), _p(b), _p(c), _p(k), _p(Y), int(split_above),
                               _p(Fp), _p(kd))
    else:
        lib().orc_rhs_f32(n, len(a), _p(a), _p(b), _p(c), _p(k), _p(Y), _p(Fp), _p(kd))
    return Fp, kd


def update_f32(Y, Fp, kd, h, kappa=1.0):
    Y, Fp, kd = (np.ascontiguousarray(v, np.float32) for v in (Y, Fp, kd))
    Yn = np.empty_like(Y)
    lib().orc_update_f32(len(Y), _p(Y), _p(Fp), _p(kd), float(h), float(kappa), _p(Yn))
    return Yn


def integrate_zone_f32(net, k, Y0, t_end, dt0, opts: Optional[Options] = None):
    """Integrate one zone in single precision (float state and arithmetic, double time)."""
    opts = opts or options()
    a, b, c = _i32(net.reactant0), _i32(net.reactant1), _i32(net.product)
    k = _f64(k)
    Y = _f64(Y0).copy()
    dt = np.array([dt0], dtype=np.float64)
    na, nr = np.zeros(1, np.int64), np.zeros(1, np.int64)
    st = lib().orc_integrate_zone_f32(net.n_species, len(a), _p(a), _p(b), _p(c), _p(k), _p(Y),
                                      float(t_end), _p(dt), C.byref(opts), _p(na), _p(nr))
    return dict(Y=Y, dt=float(dt[0]), n_acc=int(na[0]), n_rej=int(nr[0]), status=int(st))


def integrate_batch(net, zones, opts: Optional[Options] = None, n_threads: int = 0,
                    precision: int = 0):
    """Integrate every zone of a workloads.Zones batch; returns dict of arrays.

    precision 0: double; 1: single (see integrate_zone_f32)."""
    opts = opts or options()
    a, b, c = _i32(net.reactant0), _i32(net.reactant1), _i32(net.product)
    Z, n = zones.Y0.shape
    Y = _f64(zones.Y0).copy()
    dt = _f64(zones.dt0).copy()
    t_end = _f64(zones.t_end)
    na = np.zeros(Z, np.int64)
    nr = np.zeros(Z, np.int64)
    st = np.zeros(Z, np.int32)
    T = None if zones.T is None else _f64(zones.T)
    kz = None if zones.k is None else _f64(zones.k)
    A = None if net.A is None else _f64(net.A)
    E = None if net.E is None else _f64(net.E)
    if (T is None) == (kz is None):
        raise ValueError("zones need exactly one of T and k")
    if T is not None and (A is None or E is None):
        raise ValueError("Arrhenius zones need a network with A and E")
    lib().orc_integrate_batch_prec(int(precision), n, len(a), _p(a), _p(b), _p(c), _p(A), _p(E),
                                   Z, _p(Y), _p(T), _p(kz), _p(t_end), _p(dt), _p(na), _p(nr),
                                   _p(st), C.byref(opts), int(n_threads))
    return dict(Y=Y, dt=dt, n_acc=na, n_rej=nr, status=st)


def max_threads() -> int:
    return int(lib().orc_max_threads())


def mlp_forward_c(params, x) -> float:
    """The C reference's network output for one feature vector (166 floats)."""
    p = np.ascontiguousarray(params, dtype=np.float32)
    xv = np.ascontiguousarray(x, dtype=np.float32)
    return float(lib().orc_mlp_forward(_p(p), _p(xv)))


def mlp_forward_mfma(params, x) -> float:
    """The network output in the device's matrix-core arithmetic (FP32 accumulation by the
    measured gfx950 rule), the value that decides the proposal q."""
    p = np.ascontiguousarray(params, dtype=np.float32)
    xv = np.ascontiguousarray(x, dtype=np.float32)
    return float(lib().orc_mlp_forward_mfma(_p(p), _p(xv)))


def mfma_dot(acc, a, b) -> float:
    """acc + a.b accumulated by the matrix-core rule (len(a) a multiple of 8; a, b values
    representable in bfloat16)."""
    a, b = _f64(a), _f64(b)
    assert len(a) == len(b) and len(a) % 8 == 0
    return float(lib().orc_mfma_dot(float(np.float32(acc)), _p(a), _p(b), len(a)))


def mlp_features(Y, kd, h, tol) -> np.ndarray:
    Y, kd = _f64(Y), _f64(kd)
    x = np.zeros(166, dtype=np.float32)
    lib().orc_mlp_features(len(Y), _p(Y), _p(kd), float(h), float(tol), _p(x))
    return x


def integrate_zone_learned(net, k, Y0, t_end, dt0, params=None, opts: Optional[Options] = None,
                           learned=True, q_replay=None, log_capacity=0, label_stride=1):
    """One zone with the learned (or, learned=False, the plain) controller.

    q_replay (optional) supplies the first 32 q values in place of the network.
    With log_capacity > 0 the result holds, per proposal point, q (None for the
    plain controller), the features, the label (the boundary-step label, computed
    at points whose accepted-step count is a multiple of label_stride, else NaN)
    and the accepted-step count.
    """
    opts = opts or options()
    a, b, c = _i32(net.reactant0), _i32(net.reactant1), _i32(net.product)
    k = _f64(k)
    Y = _f64(Y0).copy()
    dt = np.array([dt0], dtype=np.float64)
    if learned and params is None:
        raise ValueError("the learned controller needs params")
    p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
    qr = None if q_replay is None else _i32(q_replay)
    cap = int(log_capacity)
    lq = np.zeros(max(cap, 1), np.int32)
    lf = np.zeros((max(cap, 1), 166), np.float32)
    ll = np.zeros(max(cap, 1), np.float64)
    ln = np.zeros(max(cap, 1), np.int64)
    lg = _LearnLog(cap, 0, lq.ctypes.data, lf.ctypes.data, ll.ctypes.data, ln.ctypes.data,
                   int(label_stride))
    na, nr = np.zeros(1, np.int64), np.zeros(1, np.int64)
    st = lib().orc_integrate_zone_learned(net.n_species, len(a), _p(a), _p(b), _p(c), _p(k), _p(Y),
                                          float(t_end), _p(dt), C.byref(opts), int(bool(learned)),
                                          _p(p), _p(qr), 0 if qr is None else len(qr), C.byref(lg),
                                          _p(na), _p(nr))
    n = min(int(lg.count), cap)
    out = dict(Y=Y, dt=float(dt[0]), n_acc=int(na[0]), n_rej=int(nr[0]), status=int(st),
               n_prop=int(lg.count))
    if cap:
        out["log"] = dict(q=lq[:n].copy() if learned else None, feat=lf[:n].copy(),
                          label=ll[:n].copy(), n_acc=ln[:n].copy())
    return out


def integrate_schedule(net, zones, sched, opts: Optional[Options] = None, n_threads: int = 0,
                       precision: int = 0, with_energy: bool = True):
    """Run the operator-split steps of a workloads.Schedule; returns dict of arrays
    (Y, dt, n_acc, n_rej, status, energy [n_steps, Z])."""
    opts = opts or options()
    a, b, c = _i32(net.reactant0), _i32(net.reactant1), _i32(net.product)
    Z, n = zones.Y0.shape
    S = sched.n_steps
    Y = _f64(zones.Y0).copy()
    dt = _f64(zones.dt0).copy()
    na, nr = np.zeros(Z, np.int64), np.zeros(Z, np.int64)
    st = np.zeros(Z, np.int32)
    energy = np.zeros((S, Z)) if with_energy else None
    T = None if sched.T is None else _f64(sched.T)
    kz = None if zones.k is None else _f64(zones.k)
    A = None if net.A is None else _f64(net.A)
    E = None if net.E is None else _f64(net.E)
    lib().orc_integrate_schedule(int(precision), n, len(a), _p(a), _p(b), _p(c), _p(A), _p(E), Z, S,
                                 _p(Y), _p(T), _p(kz), _p(_f64(sched.dt_hydro)), _p(dt),
                                 _p(_f64(sched.q)), _p(energy), _p(na), _p(nr), _p(st),
                                 C.byref(opts), int(n_threads))
    return dict(Y=Y, dt=dt, n_acc=na, n_rej=nr, status=st, energy=energy)
