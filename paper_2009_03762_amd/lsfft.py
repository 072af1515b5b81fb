"""Thin ctypes binding to liblsfft.so (C ABI: include/lsfft.h).

Argument marshalling only: every step of the solver runs in the HIP library.
The functions below carry the C names without the `lsfft_` prefix; `Solver`
is a small convenience wrapper owning one handle.  PyTorch is used only for
device memory and the current HIP stream.  If the library has not been
built, importing this module raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblsfft.so")

OK, ENOTCONV, EDIVERGED, EINVAL, ENOMEM, EDEVICE = 0, 1, 2, -1, -2, -3
TD, PCD = 0, 1
BASIC, FB, AFB, DGO, CD, ACD = 0, 1, 2, 3, 4, 5
F64, F32 = 0, 1
SCHEMES = {"basic": BASIC, "fb": FB, "afb": AFB, "dgo": DGO, "cd": CD, "acd": ACD}
PRECS = {"f64": F64, "f32": F32}
DISCS = {"td": TD, "pcd": PCD}
KERNELS = {"xpass": 0, "ypass_fwd": 1, "zpass": 2, "ypass_inv": 3, "uxpass": 4, "reduce": 5}


class Config(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3),
        ("h", C.c_double * 3),
        ("lam", C.POINTER(C.c_double)),
        ("mu", C.POINTER(C.c_double)),
        ("lambda0", C.c_double),
        ("mu0", C.c_double),
        ("disc", C.c_int32),
        ("scheme", C.c_int32),
        ("prec", C.c_int32),
        ("dgo_images", C.c_int32),
        ("dgo_weight_power", C.c_int32),
        ("stream", C.c_void_p),
        ("form", C.c_int32),
        ("f64_warmup", C.c_int32),
        ("eigenstrain", C.POINTER(C.c_double)),
        ("refine", C.c_int32),
        ("f64_until", C.c_double),
    ]


class Config1d(C.Structure):
    """lsfft_config_1d."""
    _fields_ = [
        ("n", C.c_int32),
        ("h", C.c_double),
        ("scheme", C.c_int32),
        ("disc", C.c_int32),
        ("prec", C.c_int32),
        ("dgo_images", C.c_int32),
        ("dgo_weight_power", C.c_int32),
        ("stream", C.c_void_p),
    ]


SCHEMES_1D = {"f": 0, "fd": 1, "cd": 2, "fd_hc": 3, "dgo": 4}


class Schedule(C.Structure):
    """lsfft_schedule: how one iteration's passes are cut into workgroups."""
    _fields_ = [
        ("stencil_planes", C.c_int32),
        ("y_cols", C.c_int32),
        ("z_cols", C.c_int32),
        ("xcd_order", C.c_int32),
    ]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def _load():
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                           "`python -m paper_2009_03762_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(_LIB_PATH)
    dp = C.POINTER(C.c_double)
    h = C.c_void_p
    sig = {
        "lsfft_create": (C.c_int, [C.POINTER(Config), C.POINTER(h)]),
        "lsfft_create_batch": (C.c_int, [C.POINTER(Config), C.c_int32, C.POINTER(h)]),
        "lsfft_solve_batch": (C.c_int, [h, dp, C.c_double, C.c_int32, C.c_void_p, C.c_void_p, dp,
                                        C.POINTER(C.c_int32), dp, C.POINTER(C.c_int32)]),
        "lsfft_batch_size": (C.c_int32, [h]),
        "lsfft_solve_group": (C.c_int, [C.POINTER(h), C.c_int32, dp, C.c_double, C.c_int32,
                                        C.POINTER(C.c_int32), C.POINTER(C.c_void_p), dp,
                                        C.POINTER(C.c_int32), dp, C.POINTER(C.c_int32)]),
        "lsfft_get_schedule": (C.c_int, [h, C.POINTER(Schedule)]),
        "lsfft_set_schedule": (C.c_int, [h, C.POINTER(Schedule)]),
        "lsfft_autotune": (C.c_int, [h, C.c_int32, C.POINTER(Schedule), dp, dp]),
        "lsfft_solve_1d": (C.c_int, [C.POINTER(Config1d), C.c_int32, dp, dp, dp, C.c_double, C.c_int32, dp, dp,
                                     C.POINTER(C.c_int32), dp, C.POINTER(C.c_int32)]),
        "lsfft_solve_1d_noalloc": (C.c_int, [C.POINTER(Config1d), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                             C.c_double, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                             C.c_void_p, C.c_void_p]),
        "lsfft_solve": (C.c_int, [h, dp, C.c_double, C.c_int32, dp, dp, dp, C.POINTER(C.c_int32), dp]),
        "lsfft_solve_device": (C.c_int, [h, dp, C.c_double, C.c_int32, C.c_void_p, C.c_void_p, dp,
                                         C.POINTER(C.c_int32), dp]),
        "lsfft_residual_history": (C.c_int, [h, dp, C.c_int32, C.POINTER(C.c_int32)]),
        "lsfft_stress_spectrum": (C.c_int, [h, C.c_void_p, C.c_void_p]),
        "lsfft_green_apply": (C.c_int, [h, C.c_void_p, C.c_void_p, dp]),
        "lsfft_stiffness_gradient": (C.c_int, [h, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
        "lsfft_set_timing": (C.c_int, [h, C.c_int32]),
        "lsfft_get_timing": (C.c_int, [h, dp, C.POINTER(C.c_int32)]),
        "lsfft_kernel_name": (C.c_char_p, [C.c_int32]),
        "lsfft_describe": (C.c_int, [h, C.c_char_p, C.c_int32]),
        "lsfft_destroy": (C.c_int, [h]),
        "lsfft_status_string": (C.c_char_p, [C.c_int]),
        "lsfft_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
EXPORTS = ("lsfft_create", "lsfft_create_batch", "lsfft_solve", "lsfft_solve_device", "lsfft_solve_batch",
           "lsfft_solve_group",
           "lsfft_batch_size", "lsfft_get_schedule", "lsfft_set_schedule", "lsfft_autotune", "lsfft_solve_1d",
           "lsfft_solve_1d_noalloc",
           "lsfft_residual_history",
           "lsfft_stress_spectrum", "lsfft_green_apply", "lsfft_stiffness_gradient", "lsfft_set_timing",
           "lsfft_get_timing",
           "lsfft_kernel_name", "lsfft_describe", "lsfft_destroy", "lsfft_status_string", "lsfft_version")


class LsfftError(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"{where}: {status_string(status)} ({status})")
        self.status = status


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def status_string(st):
    return _lib.lsfft_status_string(int(st)).decode()


def version():
    return _lib.lsfft_version().decode()


def kernel_name(i):
    return _lib.lsfft_kernel_name(int(i)).decode()


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


FORMS = {"auto": 0, "strain": 1, "displacement": 2}


def _eigenstrain(es, shape):
    """Host float64 copy (6, n3, n2, n1) of an eigenstrain, or None."""
    if es is None:
        return None
    es = np.ascontiguousarray(es, dtype=np.float64)
    if es.shape != (6,) + tuple(shape):
        raise ValueError(f"eigenstrain must have shape (6,) + {tuple(shape)}")
    return es


def _config(lam, mu, lambda0, mu0, scheme, disc, prec, h, dgo_images, dgo_weight_power, stream, form, f64_warmup,
            eigenstrain=None, refine=0, f64_until=0.0):
    if lam.ndim != 3 or lam.shape != mu.shape:
        raise ValueError("lam and mu must be 3D arrays of equal shape (n3, n2, n1)")
    n3, n2, n1 = lam.shape
    cfg = Config()
    cfg.n[:] = (n1, n2, n3)
    cfg.h[:] = tuple(float(v) for v in h)
    cfg.lam = _dptr(lam)
    cfg.mu = _dptr(mu)
    cfg.lambda0 = float(lambda0)
    cfg.mu0 = float(mu0)
    cfg.disc = DISCS[disc.lower()] if isinstance(disc, str) else int(disc)
    cfg.scheme = SCHEMES[scheme.lower()] if isinstance(scheme, str) else int(scheme)
    cfg.prec = PRECS[prec.lower()] if isinstance(prec, str) else int(prec)
    cfg.dgo_images = int(dgo_images)
    cfg.dgo_weight_power = int(dgo_weight_power)
    cfg.stream = _stream_handle(stream)
    cfg.form = FORMS[form] if isinstance(form, str) else int(form)
    cfg.f64_warmup = int(f64_warmup)
    cfg.eigenstrain = _dptr(eigenstrain)  # the caller keeps the array alive through the call
    cfg.refine = int(refine)
    cfg.f64_until = float(f64_until)
    return cfg


def create(lam, mu, lambda0, mu0, scheme="afb", disc="td", prec="f64", h=(1.0, 1.0, 1.0),
           dgo_images=4, dgo_weight_power=1, stream=None, form="auto", f64_warmup=0, eigenstrain=None, refine=0,
           f64_until=0.0):
    """lsfft_create.  lam, mu: float64 host arrays shaped (n3, n2, n1);
    eigenstrain: optional (6, n3, n2, n1) Voigt tensor components; refine:
    cycle length of the FP64 iterative refinement (F32 displacement form);
    f64_until: residual down to which an F32 solve runs in FP64 first."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    es = _eigenstrain(eigenstrain, lam.shape)
    cfg = _config(lam, mu, lambda0, mu0, scheme, disc, prec, h, dgo_images, dgo_weight_power, stream, form,
                  f64_warmup, es, refine, f64_until)
    handle = C.c_void_p()
    st = _lib.lsfft_create(C.byref(cfg), C.byref(handle))
    if st != OK:
        raise LsfftError(st, "lsfft_create")
    return handle


def create_batch(systems, scheme="afb", disc="td", prec="f64", h=(1.0, 1.0, 1.0), dgo_images=4,
                 dgo_weight_power=1, stream=None, form="auto", f64_warmup=0, refine=0, f64_until=0.0):
    """lsfft_create_batch.  systems: sequence of (lam, mu, lambda0, mu0) or
    (lam, mu, lambda0, mu0, eigenstrain) with float64 host arrays of one shape
    (n3, n2, n1) (eigenstrain: (6, n3, n2, n1) or None)."""
    arrays = []
    cfgs = (Config * len(systems))()
    for m, sysm in enumerate(systems):
        lam, mu, l0, m0 = sysm[:4]
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        es = _eigenstrain(sysm[4] if len(sysm) > 4 else None, lam.shape)
        arrays.append((lam, mu, es))   # keep the buffers alive through the call
        cfgs[m] = _config(lam, mu, l0, m0, scheme, disc, prec, h, dgo_images, dgo_weight_power, stream, form,
                          f64_warmup, es, refine, f64_until)
    handle = C.c_void_p()
    st = _lib.lsfft_create_batch(cfgs, len(systems), C.byref(handle))
    if st != OK:
        raise LsfftError(st, "lsfft_create_batch")
    return handle


def batch_size(handle):
    return int(_lib.lsfft_batch_size(handle))


def solve_1d(stiffness, CH, Ebar, scheme="f", disc="td", prec="f64", h=1.0, dgo_images=4, dgo_weight_power=1,
             tol=1e-12, maxit=10000, stream=None):
    """lsfft_solve_1d for bars of stiffness samples C, shaped (n,) or
    (count, n); CH and Ebar are scalars or (count,) arrays.  Returns a dict
    with status, E and T (shaped like C), iters, residual and the per-bar
    status."""
    Cin = np.asarray(stiffness, dtype=np.float64)
    Cb = np.ascontiguousarray(np.atleast_2d(Cin))
    count, n = Cb.shape
    CHb = np.ascontiguousarray(np.broadcast_to(np.asarray(CH, dtype=np.float64), (count,)))
    Ebb = np.ascontiguousarray(np.broadcast_to(np.asarray(Ebar, dtype=np.float64), (count,)))
    cfg = Config1d()
    cfg.n = n
    cfg.h = float(h)
    cfg.scheme = SCHEMES_1D[scheme.lower()] if isinstance(scheme, str) else int(scheme)
    cfg.disc = DISCS[disc.lower()] if isinstance(disc, str) else int(disc)
    cfg.prec = PRECS[prec.lower()] if isinstance(prec, str) else int(prec)
    cfg.dgo_images = int(dgo_images)
    cfg.dgo_weight_power = int(dgo_weight_power)
    cfg.stream = _stream_handle(stream)
    E = np.zeros((count, n))
    T = np.zeros((count, n))
    it = (C.c_int32 * count)()
    r = np.zeros(count)
    sts = (C.c_int32 * count)()
    st = _lib.lsfft_solve_1d(C.byref(cfg), count, _dptr(Cb), _dptr(CHb), _dptr(Ebb), float(tol), int(maxit),
                             _dptr(E), _dptr(T), it, _dptr(r), sts)
    if st < 0:
        raise LsfftError(st, "lsfft_solve_1d")
    shape = Cin.shape
    return {"status": st, "E": E.reshape(shape), "T": T.reshape(shape), "iters": np.array(list(it)),
            "residual": r, "bar_status": np.array(list(sts))}


def solve_1d_noalloc(C_dev, CH_dev, Ebar_dev, E_dev, T_dev, iters_dev, residual_dev, status_dev, scheme="f",
                     disc="td", prec="f64", h=1.0, dgo_images=4, dgo_weight_power=1, tol=1e-12, maxit=10000,
                     stream=None):
    """lsfft_solve_1d_noalloc on device tensors: C_dev (count, n) float64,
    CH_dev and Ebar_dev (count,) float64; outputs E_dev, T_dev (count, n)
    float64, iters_dev and status_dev (count,) int32, residual_dev (count,)
    float64 (any output but status_dev may be None).  Enqueues the work on
    `stream` (default: torch's current stream) and returns at once; raises
    LsfftError when nothing was enqueued."""
    import torch
    count, n = C_dev.shape
    for t, dt in ((C_dev, torch.float64), (CH_dev, torch.float64), (Ebar_dev, torch.float64),
                  (status_dev, torch.int32)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise ValueError("device tensors of the documented dtype, contiguous, are required")
    cfg = Config1d()
    cfg.n = n
    cfg.h = float(h)
    cfg.scheme = SCHEMES_1D[scheme.lower()] if isinstance(scheme, str) else int(scheme)
    cfg.disc = DISCS[disc.lower()] if isinstance(disc, str) else int(disc)
    cfg.prec = PRECS[prec.lower()] if isinstance(prec, str) else int(prec)
    cfg.dgo_images = int(dgo_images)
    cfg.dgo_weight_power = int(dgo_weight_power)
    cfg.stream = _stream_handle(stream if stream is not None else torch.cuda.current_stream())

    def ptr(t):
        return None if t is None else t.data_ptr()

    st = _lib.lsfft_solve_1d_noalloc(C.byref(cfg), count, ptr(C_dev), ptr(CH_dev), ptr(Ebar_dev), float(tol),
                                     int(maxit), ptr(E_dev), ptr(T_dev), ptr(iters_dev), ptr(residual_dev),
                                     ptr(status_dev))
    if st != OK:
        raise LsfftError(st, "lsfft_solve_1d_noalloc")


def get_schedule(handle):
    """lsfft_get_schedule, as a dict."""
    sch = Schedule()
    st = _lib.lsfft_get_schedule(handle, C.byref(sch))
    if st != OK:
        raise LsfftError(st, "lsfft_get_schedule")
    return sch.as_dict()


def set_schedule(handle, schedule):
    """lsfft_set_schedule from a dict with the four lsfft_schedule fields."""
    sch = Schedule(**{k: int(schedule[k]) for k, _ in Schedule._fields_})
    st = _lib.lsfft_set_schedule(handle, C.byref(sch))
    if st != OK:
        raise LsfftError(st, "lsfft_set_schedule")


def autotune(handle, iterations=16):
    """lsfft_autotune.  Returns (best schedule dict, ms per iteration of the
    schedule in force on entry, ms per iteration of the best)."""
    sch = Schedule()
    t0 = C.c_double(0.0)
    t1 = C.c_double(0.0)
    st = _lib.lsfft_autotune(handle, int(iterations), C.byref(sch), C.byref(t0), C.byref(t1))
    if st != OK:
        raise LsfftError(st, "lsfft_autotune")
    return sch.as_dict(), t0.value, t1.value


def solve_batch(handle, Ebars, tol, maxit, eps_dev=None, sig_dev=None):
    """lsfft_solve_batch.  Ebars: (count, 6) Voigt tensor components.  eps_dev /
    sig_dev: contiguous device tensors of the solver precision with count * 6 N
    elements, or None.  Returns (status, sig_mean (count, 6), iters, residual,
    per-system status)."""
    count = batch_size(handle)
    Eb = np.ascontiguousarray(Ebars, dtype=np.float64)
    if Eb.shape != (count, 6):
        raise ValueError(f"Ebars must have shape ({count}, 6)")
    sm = np.zeros((count, 6))
    it = (C.c_int32 * count)()
    r = np.zeros(count)
    sts = (C.c_int32 * count)()
    pe = eps_dev.data_ptr() if eps_dev is not None else None
    ps = sig_dev.data_ptr() if sig_dev is not None else None
    st = _lib.lsfft_solve_batch(handle, _dptr(Eb), float(tol), int(maxit), pe, ps, _dptr(sm), it, _dptr(r), sts)
    if st < 0:
        raise LsfftError(st, "lsfft_solve_batch")
    return st, sm, np.array(list(it)), r, np.array(list(sts))


def solve_group(handles, Ebars, tol, maxit, eps_devs=None):
    """lsfft_solve_group.  handles: sequence of solver handles; Ebars: one
    (B_i, 6) array per handle; maxit: an int, or one limit per handle;
    eps_devs: None or one device tensor (or None) per handle with
    B_i * 6 N_i elements of that solver's precision.
    Returns (status, [(sig_mean (B_i, 6), iters, residual, per-system status)
    per handle])."""
    count = len(handles)
    sizes = [batch_size(h) for h in handles]
    Eb = np.ascontiguousarray(np.concatenate([np.asarray(e, dtype=np.float64).reshape(-1, 6) for e in Ebars]))
    if Eb.shape != (sum(sizes), 6):
        raise ValueError("one (B, 6) load array per handle is required")
    total = sum(sizes)
    hs = (C.c_void_p * count)(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    pe = None
    if eps_devs is not None:
        pe = (C.c_void_p * count)(*[(t.data_ptr() if t is not None else None) for t in eps_devs])
    sm = np.zeros((total, 6))
    it = (C.c_int32 * total)()
    r = np.zeros(total)
    sts = (C.c_int32 * total)()
    each = None
    if np.ndim(maxit) > 0:
        each = (C.c_int32 * count)(*[int(m) for m in maxit])
        maxit = max(int(m) for m in maxit)
    st = _lib.lsfft_solve_group(hs, count, _dptr(Eb), float(tol), int(maxit), each, pe, _dptr(sm), it, _dptr(r),
                                sts)
    if st < 0:
        raise LsfftError(st, "lsfft_solve_group")
    its, stl = np.array(list(it)), np.array(list(sts))
    out, o = [], 0
    for b in sizes:
        out.append((sm[o:o + b], its[o:o + b], r[o:o + b], stl[o:o + b]))
        o += b
    return st, out


def destroy(handle):
    return _lib.lsfft_destroy(handle)


def _ebar(Ebar):
    Eb = np.ascontiguousarray(Ebar, dtype=np.float64)
    if Eb.shape != (6,):
        raise ValueError("Ebar must hold the 6 Voigt tensor components (11, 22, 33, 23, 13, 12)")
    return Eb


def solve(handle, Ebar, tol, maxit, eps=None, sig=None):
    """lsfft_solve with host outputs.  eps / sig: float64 arrays (6, n3, n2, n1) or None.
    Returns (status, sig_mean (6,), iters, residual)."""
    Eb = _ebar(Ebar)
    sm = np.zeros(6)
    it = C.c_int32(0)
    r = C.c_double(0.0)
    for a in (eps, sig):
        if a is not None and (a.dtype != np.float64 or not a.flags.c_contiguous):
            raise ValueError("host outputs must be C-contiguous float64")
    st = _lib.lsfft_solve(handle, _dptr(Eb), float(tol), int(maxit), _dptr(eps), _dptr(sig), _dptr(sm),
                          C.byref(it), C.byref(r))
    if st < 0:
        raise LsfftError(st, "lsfft_solve")
    return st, sm, it.value, r.value


def solve_device(handle, Ebar, tol, maxit, eps_dev=None, sig_dev=None):
    """lsfft_solve_device.  eps_dev / sig_dev: contiguous device tensors of the
    solver precision with 6 N elements, or None."""
    Eb = _ebar(Ebar)
    sm = np.zeros(6)
    it = C.c_int32(0)
    r = C.c_double(0.0)
    pe = eps_dev.data_ptr() if eps_dev is not None else None
    ps = sig_dev.data_ptr() if sig_dev is not None else None
    st = _lib.lsfft_solve_device(handle, _dptr(Eb), float(tol), int(maxit), pe, ps, _dptr(sm),
                                 C.byref(it), C.byref(r))
    if st < 0:
        raise LsfftError(st, "lsfft_solve_device")
    return st, sm, it.value, r.value


def residual_history(handle, cap=1 << 20):
    cnt = C.c_int32(0)
    probe = np.zeros(1)
    st = _lib.lsfft_residual_history(handle, _dptr(probe), 0, C.byref(cnt))
    if st != OK:
        raise LsfftError(st, "lsfft_residual_history")
    out = np.zeros(min(cnt.value, cap))
    st = _lib.lsfft_residual_history(handle, _dptr(out), len(out), C.byref(cnt))
    if st != OK:
        raise LsfftError(st, "lsfft_residual_history")
    return out


def stress_spectrum(handle, eps_dev, out_dev):
    st = _lib.lsfft_stress_spectrum(handle, eps_dev.data_ptr(), out_dev.data_ptr())
    if st != OK:
        raise LsfftError(st, "lsfft_stress_spectrum")


def green_apply(handle, in_dev, out_dev):
    r = C.c_double(0.0)
    st = _lib.lsfft_green_apply(handle, in_dev.data_ptr(), out_dev.data_ptr(), C.byref(r))
    if st != OK:
        raise LsfftError(st, "lsfft_green_apply")
    return r.value


def stiffness_gradient(handle, eps_a_dev, eps_b_dev, dj_dlambda=None, dj_dmu=None, dj_dyoung=None):
    """lsfft_stiffness_gradient: device tensors of the solver precision."""
    ptr = (lambda t: t.data_ptr() if t is not None else None)
    st = _lib.lsfft_stiffness_gradient(handle, eps_a_dev.data_ptr(), eps_b_dev.data_ptr(), ptr(dj_dlambda),
                                       ptr(dj_dmu), ptr(dj_dyoung))
    if st != OK:
        raise LsfftError(st, "lsfft_stiffness_gradient")


def describe(handle):
    """The kernel instantiations one iteration of this handle launches."""
    buf = C.create_string_buffer(1024)
    st = _lib.lsfft_describe(handle, buf, len(buf))
    if st != OK:
        raise LsfftError(st, "lsfft_describe")
    return buf.value.decode()


def set_timing(handle, kernel_id):
    st = _lib.lsfft_set_timing(handle, int(kernel_id))
    if st != OK:
        raise LsfftError(st, "lsfft_set_timing")


def get_timing(handle):
    ms = C.c_double(0.0)
    n = C.c_int32(0)
    st = _lib.lsfft_get_timing(handle, C.byref(ms), C.byref(n))
    if st != OK:
        raise LsfftError(st, "lsfft_get_timing")
    return ms.value, n.value


class Solver:
    """One solver handle; see `create` for the arguments."""

    def __init__(self, lam, mu, lambda0, mu0, **kw):
        self.shape = tuple(np.shape(lam))
        self.prec = kw.get("prec", "f64")
        self.handle = create(lam, mu, lambda0, mu0, **kw)

    def solve(self, Ebar, tol=1e-6, maxit=1000, fields=True):
        n3, n2, n1 = self.shape
        eps = np.zeros((6, n3, n2, n1)) if fields else None
        sig = np.zeros((6, n3, n2, n1)) if fields else None
        st, sm, it, r = solve(self.handle, Ebar, tol, maxit, eps, sig)
        return {"status": st, "eps": eps, "sig": sig, "sig_mean": sm, "iters": it, "residual": r}

    def solve_device(self, Ebar, tol=1e-6, maxit=1000, eps_dev=None, sig_dev=None):
        st, sm, it, r = solve_device(self.handle, Ebar, tol, maxit, eps_dev, sig_dev)
        return {"status": st, "sig_mean": sm, "iters": it, "residual": r}

    def residual_history(self):
        return residual_history(self.handle)

    def describe(self):
        return describe(self.handle)

    def close(self):
        if self.handle is not None:
            destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
