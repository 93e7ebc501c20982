"""Thin ctypes binding of libqla.so (the C ABI declared in include/qla.h).

Argument marshalling only: every step of the QLA path runs in the library's HIP
kernels. Functions keep the C names; a non-zero status raises QlaError carrying
qla_last_error(). Host arrays are numpy float64; device arrays may be anything
exposing a device pointer (torch tensors via .data_ptr()).

Importing this module loads the built library and fails loudly if it is missing:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqla.so")

QLA_OK, QLA_EINVAL, QLA_ENOMEM, QLA_EDEVICE, QLA_ESTATE = 0, -1, -2, -3, -4
QLA_F64, QLA_F32 = 0, 1
QLA_V_SKEW_HALF, QLA_V_PAPER, QLA_V_NONE, QLA_V_BSTREAM = 0, 1, 2, 3
QLA_TRIPLE_EZ, QLA_TRIPLE_BZ = 0, 1

# Every symbol include/qla.h declares.
EXPORTED = (
    "qla_create", "qla_create_triple", "qla_divergence", "qla_set_index_ellipse",
    "qla_set_index", "qla_set_index_device", "qla_init_packet",
    "qla_set_fields", "qla_advance", "qla_get_fields", "qla_get_fields_device",
    "qla_energy", "qla_energy_device", "qla_energy_noalloc", "qla_get_coefficients",
    "qla_step_count",
    "qla_set_tuning", "qla_autotune", "qla_get_tuning", "qla_set_lane_columns",
    "qla_get_lane_columns", "qla_destroy", "qla_strerror",
    "qla_last_error", "qla_batch_create", "qla_batch_context", "qla_batch_plan", "qla_batch_run",
    "qla_batch_plan_info", "qla_batch_plan_fixed", "qla_batch_segment_rows",
    "qla_batch_destroy", "qla_fno_create", "qla_fno_destroy",
    "qla_fno_param_count", "qla_fno_get_params", "qla_fno_set_params", "qla_fno_get_grads",
    "qla_fno_forward", "qla_fno_loss_grad", "qla_fno_adam_step", "qla_fno_train_step",
    "qla_fno_output_energy", "qla_fno_band_fraction", "qla_fno_pack",
)


class QlaError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where} failed with status {status}: {message}")
        self.status = status


class qla_ellipse(ctypes.Structure):
    _fields_ = [(name, ctypes.c_double) for name in
                ("xc", "yc", "a", "b", "rot", "n_in", "n_out", "width")]


class qla_packet(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("sigma", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("phi", ctypes.c_double), ("amp", ctypes.c_double),
                ("planar", ctypes.c_int)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libqla.so and declare every prototype. Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2604_21128_amd.build`")
    lib = ctypes.CDLL(path)
    vp, dp, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64
    fp = ctypes.POINTER(ctypes.c_float)
    st = ctypes.c_int
    proto = {
        "qla_create": (st, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                            ctypes.c_int, vp, ctypes.POINTER(vp)]),
        "qla_create_triple": (st, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(vp)]),
        "qla_divergence": (st, [vp, dp, dp, dp]),
        "qla_set_index_ellipse": (st, [vp, ctypes.POINTER(qla_ellipse)]),
        "qla_set_index": (st, [vp, dp, ctypes.c_size_t]),
        "qla_set_index_device": (st, [vp, vp, ctypes.c_size_t]),
        "qla_init_packet": (st, [vp, ctypes.POINTER(qla_packet)]),
        "qla_set_fields": (st, [vp, dp, i64]),
        "qla_advance": (st, [vp, i64]),
        "qla_get_fields": (st, [vp, dp, ctypes.c_int]),
        "qla_get_fields_device": (st, [vp, vp, ctypes.c_int]),
        "qla_energy": (st, [vp, dp]),
        "qla_energy_device": (st, [vp, vp]),
        "qla_energy_noalloc": (st, [vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_size_t,
                                    ctypes.c_int, vp, vp]),
        "qla_get_coefficients": (st, [vp, dp, dp, dp]),
        "qla_step_count": (st, [vp, ctypes.POINTER(i64)]),
        "qla_set_tuning": (st, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "qla_autotune": (st, [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                              ctypes.POINTER(ctypes.c_int)]),
        "qla_get_tuning": (st, [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int)]),
        "qla_set_lane_columns": (st, [vp, ctypes.c_int]),
        "qla_get_lane_columns": (st, [vp, ctypes.POINTER(ctypes.c_int)]),
        "qla_destroy": (st, [vp]),
        "qla_batch_create": (st, [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_int), dp, ctypes.c_int, ctypes.c_int,
                                  vp, ctypes.POINTER(vp)]),
        "qla_batch_context": (st, [vp, ctypes.c_int, ctypes.POINTER(vp)]),
        "qla_batch_plan": (st, [vp, ctypes.POINTER(i64), ctypes.c_int]),
        "qla_batch_run": (st, [vp]),
        "qla_batch_plan_info": (st, [vp] + [ctypes.POINTER(ctypes.c_int)] * 5
                                + [ctypes.POINTER(i64)]),
        "qla_batch_plan_fixed": (st, [vp, ctypes.POINTER(i64)] + [ctypes.c_int] * 4),
        "qla_batch_segment_rows": (st, [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
        "qla_batch_destroy": (st, [vp]),
        "qla_fno_create": (st, [ctypes.c_int] * 9 + [ctypes.c_uint64, vp, ctypes.POINTER(vp)]),
        "qla_fno_destroy": (st, [vp]),
        "qla_fno_param_count": (st, [vp, ctypes.POINTER(i64)]),
        "qla_fno_get_params": (st, [vp, fp]),
        "qla_fno_set_params": (st, [vp, fp]),
        "qla_fno_get_grads": (st, [vp, fp]),
        "qla_fno_forward": (st, [vp, vp, ctypes.c_int, vp]),
        "qla_fno_loss_grad": (st, [vp, vp, vp, ctypes.c_int, fp]),
        "qla_fno_adam_step": (st, [vp] + [ctypes.c_float] * 4),
        "qla_fno_train_step": (st, [vp, vp, vp, ctypes.c_int, ctypes.c_float, vp]),
        "qla_fno_output_energy": (st, [vp, ctypes.c_int, vp]),
        "qla_fno_band_fraction": (st, [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]),
        "qla_fno_pack": (st, [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_double, vp, vp, vp]),
        "qla_strerror": (ctypes.c_char_p, [st]),
        "qla_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in proto.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != QLA_OK:
        msg = load().qla_last_error().decode(errors="replace")
        raise QlaError(status, where, msg)


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _devptr(x) -> int:
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    return int(x)


def _host_planes(a: np.ndarray, count: int, name: str) -> np.ndarray:
    if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous
            and a.size == count):
        raise ValueError(f"{name} must be a C-contiguous float64 array of {count} elements")
    return a


def qla_create(nx: int, ny: int, delta: float, precision: int = QLA_F64,
               potential: int = QLA_V_SKEW_HALF, hip_stream: Optional[int] = None) -> int:
    """Returns the context handle (an integer address)."""
    out = ctypes.c_void_p()
    _check(load().qla_create(int(nx), int(ny), float(delta), int(precision), int(potential),
                             ctypes.c_void_p(hip_stream) if hip_stream else None,
                             ctypes.byref(out)), "qla_create")
    return int(out.value)


def qla_create_triple(nx: int, ny: int, delta: float, precision: int = QLA_F64,
                      potential: int = QLA_V_SKEW_HALF, triple: int = QLA_TRIPLE_EZ,
                      hip_stream: Optional[int] = None) -> int:
    out = ctypes.c_void_p()
    _check(load().qla_create_triple(int(nx), int(ny), float(delta), int(precision),
                                    int(potential), int(triple),
                                    ctypes.c_void_p(hip_stream) if hip_stream else None,
                                    ctypes.byref(out)), "qla_create_triple")
    return int(out.value)


def qla_divergence(ctx: int):
    """(l2, max_abs, scale) of the in-plane field's discrete divergence."""
    v = [ctypes.c_double() for _ in range(3)]
    _check(load().qla_divergence(ctypes.c_void_p(ctx), *[ctypes.byref(x) for x in v]),
           "qla_divergence")
    return v[0].value, v[1].value, v[2].value


def qla_destroy(ctx: int) -> None:
    _check(load().qla_destroy(ctypes.c_void_p(ctx)), "qla_destroy")


def qla_set_index(ctx: int, n: np.ndarray) -> None:
    n = np.ascontiguousarray(n, dtype=np.float64)
    if n.ndim != 2:
        raise ValueError("n must be [ny, nx]")
    _check(load().qla_set_index(ctypes.c_void_p(ctx), _dptr(n), n.shape[1]), "qla_set_index")


def qla_set_index_ellipse(ctx: int, xc: float, yc: float, a: float, b: float, rot: float,
                          n_in: float, n_out: float, width: float) -> None:
    e = qla_ellipse(float(xc), float(yc), float(a), float(b), float(rot), float(n_in),
                    float(n_out), float(width))
    _check(load().qla_set_index_ellipse(ctypes.c_void_p(ctx), ctypes.byref(e)),
           "qla_set_index_ellipse")


def qla_set_index_device(ctx: int, n_device, ld: int) -> None:
    _check(load().qla_set_index_device(ctypes.c_void_p(ctx), ctypes.c_void_p(_devptr(n_device)),
                                       int(ld)), "qla_set_index_device")


def qla_init_packet(ctx: int, x0: float, y0: float, sigma: float, lam: float, phi: float = 0.0,
                    amp: float = 1.0, planar: bool = True) -> None:
    p = qla_packet(float(x0), float(y0), float(sigma), float(lam), float(phi), float(amp),
                   int(bool(planar)))
    _check(load().qla_init_packet(ctypes.c_void_p(ctx), ctypes.byref(p)), "qla_init_packet")


def qla_set_fields(ctx: int, q: np.ndarray, step: int = 0) -> None:
    """q: float64 [3, ny, nx] planes (q2, q3, q4)."""
    q = _host_planes(q, q.size, "q")
    _check(load().qla_set_fields(ctypes.c_void_p(ctx), _dptr(q), int(step)), "qla_set_fields")


def qla_advance(ctx: int, k: int) -> None:
    _check(load().qla_advance(ctypes.c_void_p(ctx), int(k)), "qla_advance")


def qla_get_fields(ctx: int, nx: int, ny: int, physical: bool = False) -> np.ndarray:
    out = np.empty((3, ny, nx), dtype=np.float64)
    _check(load().qla_get_fields(ctypes.c_void_p(ctx), _dptr(out), int(bool(physical))),
           "qla_get_fields")
    return out


def qla_get_fields_device(ctx: int, out_device, physical: bool = False) -> None:
    _check(load().qla_get_fields_device(ctypes.c_void_p(ctx), ctypes.c_void_p(_devptr(out_device)),
                                        int(bool(physical))), "qla_get_fields_device")


def qla_energy(ctx: int) -> float:
    e = ctypes.c_double()
    _check(load().qla_energy(ctypes.c_void_p(ctx), ctypes.byref(e)), "qla_energy")
    return float(e.value)


def qla_energy_device(ctx: int, out_device) -> None:
    _check(load().qla_energy_device(ctypes.c_void_p(ctx), ctypes.c_void_p(_devptr(out_device))),
           "qla_energy_device")


def qla_energy_noalloc(q_a, q_b, q_c, nx: int, ny: int, pitch: int, precision: int,
                       out_device, stream=None) -> None:
    """Energy of three caller-owned device planes (pointers or tensors) into one device
    double, with no allocation (the library's file-scope scratch holds the partials)."""
    _check(load().qla_energy_noalloc(ctypes.c_void_p(_devptr(q_a)), ctypes.c_void_p(_devptr(q_b)),
                                     ctypes.c_void_p(_devptr(q_c)), int(nx), int(ny), int(pitch),
                                     int(precision), ctypes.c_void_p(_devptr(out_device)),
                                     ctypes.c_void_p(_devptr(stream) if stream else None)),
           "qla_energy_noalloc")


def qla_get_coefficients(ctx: int, nx: int, ny: int):
    th, bx, by = (np.empty((ny, nx), dtype=np.float64) for _ in range(3))
    _check(load().qla_get_coefficients(ctypes.c_void_p(ctx), _dptr(th), _dptr(bx), _dptr(by)),
           "qla_get_coefficients")
    return th, bx, by


def qla_step_count(ctx: int) -> int:
    v = ctypes.c_int64()
    _check(load().qla_step_count(ctypes.c_void_p(ctx), ctypes.byref(v)), "qla_step_count")
    return int(v.value)


def qla_set_tuning(ctx: int, rows_per_segment: int = 0, prefetch_rows: int = 0,
                   steps_per_pass: int = 0) -> None:
    _check(load().qla_set_tuning(ctypes.c_void_p(ctx), int(rows_per_segment), int(prefetch_rows),
                                 int(steps_per_pass)), "qla_set_tuning")


def qla_autotune(ctx: int):
    """Returns the chosen (rows_per_segment, prefetch_rows, steps_per_pass)."""
    r, p, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load().qla_autotune(ctypes.c_void_p(ctx), ctypes.byref(r), ctypes.byref(p),
                               ctypes.byref(t)), "qla_autotune")
    return r.value, p.value, t.value


def qla_get_tuning(ctx: int):
    r, p, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load().qla_get_tuning(ctypes.c_void_p(ctx), ctypes.byref(r), ctypes.byref(p),
                                 ctypes.byref(t)), "qla_get_tuning")
    return r.value, p.value, t.value


def qla_set_lane_columns(ctx: int, columns: int = 0) -> None:
    _check(load().qla_set_lane_columns(ctypes.c_void_p(ctx), int(columns)),
           "qla_set_lane_columns")


def qla_get_lane_columns(ctx: int) -> int:
    v = ctypes.c_int()
    _check(load().qla_get_lane_columns(ctypes.c_void_p(ctx), ctypes.byref(v)),
           "qla_get_lane_columns")
    return v.value


def qla_batch_create(nx, ny, delta, precision: int = QLA_F32,
                     potential: int = QLA_V_SKEW_HALF, hip_stream: Optional[int] = None) -> int:
    count = len(nx)
    ia = (ctypes.c_int * count)(*[int(v) for v in nx])
    ib = (ctypes.c_int * count)(*[int(v) for v in ny])
    da = (ctypes.c_double * count)(*[float(v) for v in delta])
    out = ctypes.c_void_p()
    _check(load().qla_batch_create(count, ia, ib, da, int(precision), int(potential),
                                   ctypes.c_void_p(hip_stream) if hip_stream else None,
                                   ctypes.byref(out)), "qla_batch_create")
    return int(out.value)


def qla_batch_context(batch: int, i: int) -> int:
    out = ctypes.c_void_p()
    _check(load().qla_batch_context(ctypes.c_void_p(batch), int(i), ctypes.byref(out)),
           "qla_batch_context")
    return int(out.value)


def qla_batch_plan(batch: int, steps, mode: int = 0) -> None:
    arr = (ctypes.c_int64 * len(steps))(*[int(v) for v in steps])
    _check(load().qla_batch_plan(ctypes.c_void_p(batch), arr, int(mode)), "qla_batch_plan")


def qla_batch_plan_fixed(batch: int, steps, rows_per_segment: int, prefetch_rows: int,
                         steps_per_pass: int, fit: bool = False) -> None:
    arr = (ctypes.c_int64 * len(steps))(*[int(v) for v in steps])
    _check(load().qla_batch_plan_fixed(ctypes.c_void_p(batch), arr, int(rows_per_segment),
                                       int(prefetch_rows), int(steps_per_pass), int(bool(fit))),
           "qla_batch_plan_fixed")


def qla_batch_segment_rows(batch: int, i: int) -> int:
    v = ctypes.c_int()
    _check(load().qla_batch_segment_rows(ctypes.c_void_p(batch), int(i), ctypes.byref(v)),
           "qla_batch_segment_rows")
    return v.value


def qla_batch_run(batch: int) -> None:
    _check(load().qla_batch_run(ctypes.c_void_p(batch)), "qla_batch_run")


def qla_batch_plan_info(batch: int) -> dict:
    v = [ctypes.c_int() for _ in range(5)]
    u = ctypes.c_int64()
    _check(load().qla_batch_plan_info(ctypes.c_void_p(batch), *[ctypes.byref(x) for x in v],
                                      ctypes.byref(u)), "qla_batch_plan_info")
    return {"rows_per_segment": v[0].value, "prefetch_rows": v[1].value,
            "steps_per_pass": v[2].value, "mode": v[3].value, "passes": v[4].value,
            "site_updates": u.value}


def qla_batch_destroy(batch: int) -> None:
    _check(load().qla_batch_destroy(ctypes.c_void_p(batch)), "qla_batch_destroy")


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def qla_fno_create(height: int, width: int, in_channels: int, out_channels: int, channels: int,
                   modes: int, layers: int, proj_channels: int, max_batch: int, seed: int = 0,
                   hip_stream: Optional[int] = None) -> int:
    out = ctypes.c_void_p()
    _check(load().qla_fno_create(int(height), int(width), int(in_channels), int(out_channels),
                                 int(channels), int(modes), int(layers), int(proj_channels),
                                 int(max_batch), ctypes.c_uint64(int(seed)),
                                 ctypes.c_void_p(hip_stream) if hip_stream else None,
                                 ctypes.byref(out)), "qla_fno_create")
    return int(out.value)


def qla_fno_destroy(fno: int) -> None:
    _check(load().qla_fno_destroy(ctypes.c_void_p(fno)), "qla_fno_destroy")


def qla_fno_param_count(fno: int) -> int:
    v = ctypes.c_int64()
    _check(load().qla_fno_param_count(ctypes.c_void_p(fno), ctypes.byref(v)),
           "qla_fno_param_count")
    return int(v.value)


def qla_fno_get_params(fno: int) -> np.ndarray:
    out = np.empty(qla_fno_param_count(fno), dtype=np.float32)
    _check(load().qla_fno_get_params(ctypes.c_void_p(fno), _fptr(out)), "qla_fno_get_params")
    return out


def qla_fno_set_params(fno: int, params: np.ndarray) -> None:
    p = np.ascontiguousarray(params, dtype=np.float32)
    if p.size != qla_fno_param_count(fno):
        raise ValueError("parameter vector has the wrong length")
    _check(load().qla_fno_set_params(ctypes.c_void_p(fno), _fptr(p)), "qla_fno_set_params")


def qla_fno_get_grads(fno: int) -> np.ndarray:
    out = np.empty(qla_fno_param_count(fno), dtype=np.float32)
    _check(load().qla_fno_get_grads(ctypes.c_void_p(fno), _fptr(out)), "qla_fno_get_grads")
    return out


def qla_fno_forward(fno: int, input_device, batch: int, output_device) -> None:
    _check(load().qla_fno_forward(ctypes.c_void_p(fno), ctypes.c_void_p(_devptr(input_device)),
                                  int(batch), ctypes.c_void_p(_devptr(output_device))),
           "qla_fno_forward")


def qla_fno_loss_grad(fno: int, input_device, target_device, batch: int) -> float:
    loss = ctypes.c_float()
    _check(load().qla_fno_loss_grad(ctypes.c_void_p(fno), ctypes.c_void_p(_devptr(input_device)),
                                    ctypes.c_void_p(_devptr(target_device)), int(batch),
                                    ctypes.byref(loss)), "qla_fno_loss_grad")
    return float(loss.value)


def qla_fno_adam_step(fno: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                      eps: float = 1e-8) -> None:
    _check(load().qla_fno_adam_step(ctypes.c_void_p(fno), float(lr), float(beta1), float(beta2),
                                    float(eps)), "qla_fno_adam_step")


def qla_fno_train_step(fno: int, input_device, target_device, batch: int, lr: float,
                       loss_device=None) -> None:
    _check(load().qla_fno_train_step(ctypes.c_void_p(fno), ctypes.c_void_p(_devptr(input_device)),
                                     ctypes.c_void_p(_devptr(target_device)), int(batch),
                                     float(lr),
                                     ctypes.c_void_p(_devptr(loss_device))
                                     if loss_device is not None else None),
           "qla_fno_train_step")


def qla_fno_output_energy(fno: int, batch: int, energy_device) -> None:
    _check(load().qla_fno_output_energy(ctypes.c_void_p(fno), int(batch),
                                        ctypes.c_void_p(_devptr(energy_device))),
           "qla_fno_output_energy")


def qla_fno_band_fraction(fno: int, input_device, batch: int, first_channel: int,
                          channels: int, fraction_device) -> None:
    _check(load().qla_fno_band_fraction(ctypes.c_void_p(fno),
                                        ctypes.c_void_p(_devptr(input_device)), int(batch),
                                        int(first_channel), int(channels),
                                        ctypes.c_void_p(_devptr(fraction_device))),
           "qla_fno_band_fraction")


def qla_fno_pack(q_device, n_device, nx: int, ny: int, n_shift: float, input_device=None,
                 target_device=None, hip_stream: Optional[int] = None) -> None:
    def opt(x):
        return ctypes.c_void_p(_devptr(x)) if x is not None else None
    _check(load().qla_fno_pack(ctypes.c_void_p(_devptr(q_device)), opt(n_device), int(nx),
                               int(ny), float(n_shift), opt(input_device), opt(target_device),
                               ctypes.c_void_p(hip_stream) if hip_stream else None),
           "qla_fno_pack")


def qla_strerror(status: int) -> str:
    return load().qla_strerror(int(status)).decode()


def qla_last_error() -> str:
    return load().qla_last_error().decode(errors="replace")


class Lattice:
    """Owns one context; a convenience wrapper over the functions above."""

    def __init__(self, nx: int, ny: int, delta: float, precision: int = QLA_F64,
                 potential: int = QLA_V_SKEW_HALF, hip_stream: Optional[int] = None,
                 triple: int = QLA_TRIPLE_EZ):
        self.nx, self.ny = int(nx), int(ny)
        self.ctx = qla_create_triple(nx, ny, delta, precision, potential, triple, hip_stream)

    def close(self):
        if self.ctx:
            qla_destroy(self.ctx)
            self.ctx = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_index(self, n):
        qla_set_index(self.ctx, n)

    def init_packet(self, p):
        qla_init_packet(self.ctx, p.x0, p.y0, p.sigma, p.lam, p.phi, p.amp, p.planar)

    def advance(self, k: int):
        qla_advance(self.ctx, k)

    def fields(self, physical: bool = False) -> np.ndarray:
        return qla_get_fields(self.ctx, self.nx, self.ny, physical)

    def set_fields(self, q, step: int = 0):
        qla_set_fields(self.ctx, np.ascontiguousarray(q, dtype=np.float64), step)

    def energy(self) -> float:
        return qla_energy(self.ctx)

    def coefficients(self):
        return qla_get_coefficients(self.ctx, self.nx, self.ny)

    def divergence(self):
        return qla_divergence(self.ctx)

    @property
    def steps(self) -> int:
        return qla_step_count(self.ctx)
