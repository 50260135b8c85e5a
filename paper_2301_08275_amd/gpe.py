"""Thin ctypes binding over libgpe.so (C ABI in include/gpe.h).

Functions named like the C ABI (gpe_create, gpe_evolve, ...) marshal
arguments only; every step of the solver runs in the HIP library.  `Context`
wraps them for numpy / torch callers.  There is no fallback: if the library
is missing or no HIP device is present the calls fail loudly.

PyTorch ships its own HIP runtime with the same soname as the system one.
When torch shares the process, import torch (and touch its device) before the
first call here, so that libgpe.so binds to the runtime torch already loaded.
"""
import contextlib
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpe.so")

GPE_OK = 0
GPE_EINVAL = -1
GPE_ENOMEM = -2
GPE_EDEVICE = -3
GPE_ENOTCONV = -4
GPE_ENONFINITE = -5
GPE_EBUSY = -6
GPE_EUNSUPPORTED = -7
GPE_ECANCELED = -8
STATUS_NAMES = {0: "GPE_OK", -1: "GPE_EINVAL", -2: "GPE_ENOMEM", -3: "GPE_EDEVICE",
                -4: "GPE_ENOTCONV", -5: "GPE_ENONFINITE", -6: "GPE_EBUSY",
                -7: "GPE_EUNSUPPORTED", -8: "GPE_ECANCELED"}

GPE_FP64 = 0
GPE_FP32 = 1
GPE_FP32_STATE = 2  # FP32 state in device memory, FP64 arithmetic
PRECISIONS = {"fp64": GPE_FP64, "fp32": GPE_FP32, "fp32s": GPE_FP32_STATE}


class gpe_desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("g", ctypes.c_double), ("precision", ctypes.c_int32),
                ("norm_target", ctypes.c_double)]


class gpe_harmonic(ctypes.Structure):
    _fields_ = [("w", ctypes.c_double * 3)]


class gpe_obs(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_double), ("energy", ctypes.c_double),
                ("mu", ctypes.c_double), ("e_kin", ctypes.c_double),
                ("e_pot", ctypes.c_double), ("e_int", ctypes.c_double),
                ("sigma", ctypes.c_double * 3), ("r_rms", ctypes.c_double)]


class gpe_spectra(ctypes.Structure):
    _fields_ = [("nbins", ctypes.c_int32), ("dk", ctypes.c_double),
                ("n_k", ctypes.POINTER(ctypes.c_double)),
                ("e_comp", ctypes.POINTER(ctypes.c_double)),
                ("e_incomp", ctypes.POINTER(ctypes.c_double)),
                ("e_qp", ctypes.POINTER(ctypes.c_double))]


GPE_TIMING_KINDS = 16


class gpe_timing(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("name", (ctypes.c_char * 32) * GPE_TIMING_KINDS),
                ("total_ms", ctypes.c_double * GPE_TIMING_KINDS),
                ("launches", ctypes.c_int64 * GPE_TIMING_KINDS),
                ("bytes", ctypes.c_double * GPE_TIMING_KINDS)]


SEPARABLE_FIELDS = ("w", "center", "quartic", "lattice", "q", "phase")


class gpe_separable(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double * 3) for f in SEPARABLE_FIELDS]


# void (*)(double t, gpe_separable *out, void *user)
POTENTIAL_FN = ctypes.CFUNCTYPE(None, ctypes.c_double, ctypes.POINTER(gpe_separable),
                                ctypes.c_void_p)


def fill_separable(out, params):
    """Write a dict of per-axis sequences (keys from SEPARABLE_FIELDS; missing
    keys are zero) into a gpe_separable."""
    unknown = set(params) - set(SEPARABLE_FIELDS)
    if unknown:
        raise ValueError("unknown potential parameters: %s" % sorted(unknown))
    for f in SEPARABLE_FIELDS:
        vals = params.get(f)
        arr = getattr(out, f)
        for j in range(3):
            arr[j] = float(vals[j]) if vals is not None and j < len(vals) else 0.0
    return out


class gpe_request(ctypes.Structure):
    _fields_ = [("desc", gpe_desc), ("trap", gpe_harmonic),
                ("psi0", ctypes.POINTER(ctypes.c_double)), ("mode", ctypes.c_int32),
                ("dt", ctypes.c_double), ("nsteps", ctypes.c_int64),
                ("keep_state", ctypes.c_int32)]


class gpe_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("obs", gpe_obs), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("steps_done", ctypes.c_int64)]


class gpe_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("running", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("busy_seconds", ctypes.c_double), ("site_steps", ctypes.c_double),
                ("bytes_in_use", ctypes.c_uint64)]


class gpe_tuning(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32 * 3), ("xcd_remap", ctypes.c_int32 * 3),
                ("pass_order", ctypes.c_int32 * 3), ("plan", ctypes.c_int32 * 3),
                ("stream", ctypes.c_int32 * 3), ("transpose", ctypes.c_int32),
                ("ms_per_step", ctypes.c_double)]


_P = ctypes.c_void_p
_D = ctypes.c_double
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_DP = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes); the C ABI declared in include/gpe.h
SIGNATURES = {
    "gpe_create": (_I32, [ctypes.POINTER(gpe_desc), _DP, ctypes.POINTER(gpe_harmonic), _P,
                          ctypes.POINTER(_P)]),
    "gpe_set_potential": (_I32, [_P, _DP, ctypes.POINTER(gpe_harmonic)]),
    "gpe_set_separable": (_I32, [_P, ctypes.POINTER(gpe_separable)]),
    "gpe_set_potential_fn": (_I32, [_P, POTENTIAL_FN, _P]),
    "gpe_set_time": (_I32, [_P, _D]),
    "gpe_set_imag_method": (_I32, [_P, _I32]),
    "gpe_get_time": (_I32, [_P, _DP]),
    "gpe_set_state": (_I32, [_P, _DP]),
    "gpe_set_state_device": (_I32, [_P, _P, _I32]),
    "gpe_get_state": (_I32, [_P, _DP]),
    "gpe_get_state_device": (_I32, [_P, _P, _I32]),
    "gpe_evolve": (_I32, [_P, _D, _I64]),
    "gpe_ground_state": (_I32, [_P, _D, _D, _I32, _I64, ctypes.POINTER(_I64), _DP]),
    "gpe_evolve_record": (_I32, [_P, _D, _I64, _I32, ctypes.POINTER(gpe_obs), _I64,
                                 ctypes.POINTER(_I64)]),
    "gpe_observables": (_I32, [_P, ctypes.POINTER(gpe_obs), ctypes.POINTER(gpe_spectra)]),
    "gpe_spectra_bins": (_I32, [_P]),
    "gpe_transform": (_I32, [_P, _I32, _I32]),
    "gpe_synchronize": (_I32, [_P]),
    "gpe_timing_enable": (_I32, [_P, _I32]),
    "gpe_timing_read": (_I32, [_P, ctypes.POINTER(gpe_timing)]),
    "gpe_device_bytes": (ctypes.c_uint64, [_P]),
    "gpe_device": (_I32, [_P]),
    "gpe_stream": (ctypes.c_void_p, [_P]),
    "gpe_steps_noalloc": (_I32, [ctypes.POINTER(gpe_desc), ctypes.POINTER(gpe_harmonic), _P,
                                 _I32, _D, _I64, _P]),
    "gpe_last_error": (ctypes.c_char_p, [_P]),
    "gpe_destroy": (None, [_P]),
    "gpe_server_create": (_I32, [ctypes.c_uint64, _I32, _I32, _I32, ctypes.POINTER(_P)]),
    "gpe_server_submit": (_I32, [_P, ctypes.POINTER(gpe_request), ctypes.POINTER(ctypes.c_uint64)]),
    "gpe_server_poll": (_I32, [_P, ctypes.c_uint64, ctypes.POINTER(gpe_result), _DP]),
    "gpe_server_cancel": (_I32, [_P, ctypes.c_uint64]),
    "gpe_server_wait_idle": (_I32, [_P]),
    "gpe_server_release": (_I32, [_P, ctypes.c_uint64]),
    "gpe_server_stats_read": (_I32, [_P, ctypes.POINTER(gpe_server_stats)]),
    "gpe_server_destroy": (None, [_P]),
    "gpe_request_bytes": (_I32, [ctypes.POINTER(gpe_desc), _I32, ctypes.POINTER(ctypes.c_uint64),
                                 ctypes.POINTER(ctypes.c_uint64)]),
    "gpe_autotune": (_I32, [ctypes.POINTER(gpe_desc), _I32, ctypes.POINTER(gpe_tuning)]),
    "gpe_tuning_set": (_I32, [ctypes.POINTER(gpe_desc), ctypes.POINTER(gpe_tuning)]),
    "gpe_tuning_get": (_I32, [ctypes.POINTER(gpe_desc), ctypes.POINTER(gpe_tuning),
                              ctypes.POINTER(_I32)]),
    "gpe_tuning_clear": (None, []),
    "gpe_tuning_save": (_I32, [ctypes.c_char_p]),
    "gpe_tuning_load": (_I32, [ctypes.c_char_p]),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load libgpe.so and declare the ABI.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libgpe.so is not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class GpeError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))


def _err(ctx):
    m = load_library().gpe_last_error(ctx)
    return m.decode() if m else ""


def _check(status, ctx=None):
    if status != GPE_OK:
        raise GpeError(status, _err(ctx))
    return status


def _dptr(a):
    return a.ctypes.data_as(_DP) if a is not None else None


# ----------------------------------------------------- ABI-named functions ---

def gpe_create(desc, V_host=None, V_an=None, hip_stream=None):
    lib = load_library()
    out = _P()
    st = lib.gpe_create(ctypes.byref(desc), _dptr(V_host),
                        ctypes.byref(V_an) if V_an is not None else None,
                        hip_stream, ctypes.byref(out))
    if st != GPE_OK:
        raise GpeError(st, _err(None))
    return out


def gpe_steps_noalloc(desc, trap, psi_dev, imaginary, dt, nsteps, hip_stream=None):
    """Allocation-free steps on a device state (a raw device pointer, int):
    see include/gpe.h.  trap: a gpe_harmonic or None."""
    st = load_library().gpe_steps_noalloc(ctypes.byref(desc),
                                          ctypes.byref(trap) if trap is not None else None,
                                          ctypes.c_void_p(psi_dev), int(imaginary), float(dt),
                                          int(nsteps), ctypes.c_void_p(hip_stream)
                                          if hip_stream else None)
    if st != GPE_OK:
        raise GpeError(st, _err(None))


def gpe_set_potential(ctx, V_host=None, V_an=None):
    return _check(load_library().gpe_set_potential(
        ctx, _dptr(V_host), ctypes.byref(V_an) if V_an is not None else None), ctx)


def gpe_set_separable(ctx, sep):
    return _check(load_library().gpe_set_separable(ctx, ctypes.byref(sep)), ctx)


def gpe_set_potential_fn(ctx, fn, user=None):
    """fn: a POTENTIAL_FN (or None); the caller keeps it alive while set."""
    return _check(load_library().gpe_set_potential_fn(
        ctx, fn if fn is not None else POTENTIAL_FN(), user), ctx)


GPE_IMAG_FROZEN, GPE_IMAG_EXACT = 0, 1
IMAG_METHODS = {"frozen": GPE_IMAG_FROZEN, "exact": GPE_IMAG_EXACT}


def gpe_set_imag_method(ctx, method):
    return _check(load_library().gpe_set_imag_method(ctx, int(method)), ctx)


def gpe_set_time(ctx, t):
    return _check(load_library().gpe_set_time(ctx, float(t)), ctx)


def gpe_get_time(ctx):
    t = _D(0)
    _check(load_library().gpe_get_time(ctx, ctypes.byref(t)), ctx)
    return t.value


def gpe_set_state(ctx, psi_host):
    return _check(load_library().gpe_set_state(ctx, _dptr(psi_host)), ctx)


def gpe_set_state_device(ctx, dptr, src):
    return _check(load_library().gpe_set_state_device(ctx, dptr, src), ctx)


def gpe_get_state(ctx, psi_host_out):
    return _check(load_library().gpe_get_state(ctx, _dptr(psi_host_out)), ctx)


def gpe_get_state_device(ctx, dptr, dst):
    return _check(load_library().gpe_get_state_device(ctx, dptr, dst), ctx)


def gpe_evolve(ctx, dt, nsteps):
    return _check(load_library().gpe_evolve(ctx, float(dt), int(nsteps)), ctx)


def gpe_ground_state(ctx, dt, tol, check_every, max_steps):
    """Returns (status, steps_done, energy); GPE_ENOTCONV is returned, not raised."""
    steps = _I64(0)
    energy = _D(0)
    st = load_library().gpe_ground_state(ctx, float(dt), float(tol), int(check_every),
                                         int(max_steps), ctypes.byref(steps),
                                         ctypes.byref(energy))
    if st not in (GPE_OK, GPE_ENOTCONV):
        raise GpeError(st, _err(ctx))
    return st, steps.value, energy.value


def gpe_observables(ctx, out, spec=None):
    return _check(load_library().gpe_observables(
        ctx, ctypes.byref(out), ctypes.byref(spec) if spec is not None else None), ctx)


def gpe_spectra_bins(ctx):
    return load_library().gpe_spectra_bins(ctx)


def gpe_transform(ctx, axis_mask, inverse):
    return _check(load_library().gpe_transform(ctx, int(axis_mask), int(inverse)), ctx)


def gpe_synchronize(ctx):
    return _check(load_library().gpe_synchronize(ctx), ctx)


def gpe_timing_enable(ctx, on):
    return _check(load_library().gpe_timing_enable(ctx, int(on)), ctx)


def gpe_timing_read(ctx):
    t = gpe_timing()
    _check(load_library().gpe_timing_read(ctx, ctypes.byref(t)), ctx)
    return {t.name[i].value.decode(): {"total_ms": t.total_ms[i], "launches": t.launches[i],
                                       "bytes": t.bytes[i]} for i in range(t.count)}


def gpe_device_bytes(ctx):
    return load_library().gpe_device_bytes(ctx)


def gpe_last_error(ctx):
    return _err(ctx)


def gpe_destroy(ctx):
    load_library().gpe_destroy(ctx)


def gpe_server_create(hbm_budget_bytes, max_slots, max_active, chunk_steps):
    out = _P()
    st = load_library().gpe_server_create(int(hbm_budget_bytes), int(max_slots),
                                          int(max_active), int(chunk_steps), ctypes.byref(out))
    if st != GPE_OK:
        raise GpeError(st, "gpe_server_create")
    return out


def gpe_server_submit(srv, req):
    rid = ctypes.c_uint64(0)
    st = load_library().gpe_server_submit(srv, ctypes.byref(req), ctypes.byref(rid))
    if st != GPE_OK:
        raise GpeError(st, "gpe_server_submit")
    return rid.value


def gpe_server_poll(srv, rid, out, psi_out=None):
    """Returns the status of the call (GPE_EBUSY while pending)."""
    return load_library().gpe_server_poll(srv, int(rid), ctypes.byref(out), _dptr(psi_out))


def gpe_server_cancel(srv, rid):
    return load_library().gpe_server_cancel(srv, int(rid))


def gpe_server_release(srv, rid):
    return load_library().gpe_server_release(srv, ctypes.c_uint64(rid))


def gpe_server_wait_idle(srv):
    return load_library().gpe_server_wait_idle(srv)


def gpe_server_stats_read(srv):
    st = gpe_server_stats()
    load_library().gpe_server_stats_read(srv, ctypes.byref(st))
    return {k: getattr(st, k) for k, _ in gpe_server_stats._fields_}


def gpe_server_destroy(srv):
    load_library().gpe_server_destroy(srv)


def gpe_request_bytes(desc, max_slots):
    """(bytes per shape class, bytes per running request) the server charges."""
    cb, sb = ctypes.c_uint64(0), ctypes.c_uint64(0)
    st = load_library().gpe_request_bytes(ctypes.byref(desc), int(max_slots), ctypes.byref(cb),
                                          ctypes.byref(sb))
    if st != GPE_OK:
        raise GpeError(st, "gpe_request_bytes")
    return cb.value, sb.value


def _tuning_dict(t, dim):
    return {"width": list(t.width[:dim]), "xcd_remap": list(t.xcd_remap[:dim]),
            "pass_order": list(t.pass_order[:dim]), "plan": list(t.plan[:dim]),
            "stream": list(t.stream[:dim]), "transpose": t.transpose,
            "ms_per_step": t.ms_per_step}


def gpe_autotune(desc, steps=10):
    """Time the launch shapes of this shape class; record and return the best."""
    t = gpe_tuning()
    st = load_library().gpe_autotune(ctypes.byref(desc), int(steps), ctypes.byref(t))
    if st != GPE_OK:
        raise GpeError(st, "gpe_autotune")
    return _tuning_dict(t, desc.dim)


def gpe_tuning_set(desc, width, xcd_remap, pass_order, plan=None, stream=None, transpose=0):
    t = gpe_tuning()
    t.transpose = int(transpose)
    for j in range(desc.dim):
        t.width[j] = int(width[j])
        t.xcd_remap[j] = int(xcd_remap[j])
        t.pass_order[j] = int(pass_order[j])
        t.plan[j] = int(plan[j]) if plan is not None else 0
        t.stream[j] = int(stream[j]) if stream is not None else 0
    st = load_library().gpe_tuning_set(ctypes.byref(desc), ctypes.byref(t))
    if st != GPE_OK:
        raise GpeError(st, "gpe_tuning_set")


def gpe_tuning_get(desc):
    """(entry as a dict, found) -- the defaults when there is no entry."""
    t, found = gpe_tuning(), _I32(0)
    st = load_library().gpe_tuning_get(ctypes.byref(desc), ctypes.byref(t), ctypes.byref(found))
    if st != GPE_OK:
        raise GpeError(st, "gpe_tuning_get")
    return _tuning_dict(t, desc.dim), bool(found.value)


def gpe_tuning_clear():
    load_library().gpe_tuning_clear()


def gpe_tuning_save(path):
    st = load_library().gpe_tuning_save(os.fsencode(path))
    if st != GPE_OK:
        raise GpeError(st, "gpe_tuning_save")


def gpe_tuning_load(path):
    st = load_library().gpe_tuning_load(os.fsencode(path))
    if st != GPE_OK:
        raise GpeError(st, "gpe_tuning_load")


# ------------------------------------------------------------- convenience ---

OBS_KEYS = ("norm", "energy", "mu", "e_kin", "e_pot", "e_int",
            "sigma_x", "sigma_y", "sigma_z", "r_rms")


class Context:
    """One solver instance on the current HIP device.

    shape: grid points per axis (2 or 3 entries); lo, hi: box; g: interaction;
    precision: "fp64", "fp32" (FP32 state and FFT) or "fp32s" (FP32 state,
    FP64 arithmetic); V: FP64 array of `shape` or None; harmonic:
    trap frequencies per axis (V = 1/2 sum w^2 x^2) or None; stream: a
    hipStream_t handle (int) such as torch.cuda.current_stream().cuda_stream.
    The null stream (handle 0, torch's default stream) cannot be handed to
    the library, whose NULL means "create a private stream": with stream None
    or 0 the context runs on a private stream, and the device-tensor calls
    (set_state_device, get_state_device) order themselves against the
    caller's current torch stream by waiting on the host.
    """

    def __init__(self, shape, lo, hi, g, precision="fp64", norm_target=1.0,
                 V=None, harmonic=None, stream=None):
        dim = len(shape)
        self.shape = tuple(int(s) for s in shape)
        self.dim = dim
        d = gpe_desc()
        d.dim = dim
        lo = np.broadcast_to(np.asarray(lo, np.float64), (dim,))
        hi = np.broadcast_to(np.asarray(hi, np.float64), (dim,))
        for j in range(dim):
            d.n[j] = self.shape[j]
            d.lo[j] = float(lo[j])
            d.hi[j] = float(hi[j])
        for j in range(dim, 3):
            d.n[j] = 1
        d.g = float(g)
        d.precision = PRECISIONS[precision]
        d.norm_target = float(norm_target)
        self.precision = precision
        self.desc = d
        Vh = None
        if V is not None:
            Vh = np.ascontiguousarray(V, dtype=np.float64)
            if Vh.shape != self.shape:
                raise ValueError("V shape %s != %s" % (Vh.shape, self.shape))
        an = None
        if harmonic is not None:
            an = gpe_harmonic()
            for j in range(dim):
                an.w[j] = float(harmonic[j])
        self._ctx = None
        self._vfn = None  # (callback object, exceptions it caught)
        self._ctx = gpe_create(d, Vh, an, ctypes.c_void_p(stream) if stream else None)
        self._own_stream = not stream

    @property
    def handle(self):
        return self._ctx

    def close(self):
        if self._ctx is not None:
            gpe_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_potential(self, V=None, harmonic=None):
        Vh = np.ascontiguousarray(V, dtype=np.float64) if V is not None else None
        an = None
        if harmonic is not None:
            an = gpe_harmonic()
            for j in range(self.dim):
                an.w[j] = float(harmonic[j])
        gpe_set_potential(self._ctx, Vh, an)
        self._vfn = None

    def set_separable(self, **params):
        """Static separable potential: keyword arrays w, center, quartic,
        lattice, q, phase (per axis; missing ones are zero)."""
        gpe_set_separable(self._ctx, fill_separable(gpe_separable(), params))
        self._vfn = None

    def set_potential_fn(self, fn):
        """Time-dependent separable potential: fn(t) returns a dict of the
        set_separable keywords at time t (None removes the potential).  An
        exception in fn stops the library call that ran it and is re-raised."""
        if fn is None:
            gpe_set_potential_fn(self._ctx, None)
            self._vfn = None
            return
        errors = []

        def trampoline(t, out, user):
            try:
                fill_separable(out.contents, fn(t))
            except BaseException as e:  # reported through a non-finite entry
                errors.append(e)
                out.contents.w[0] = float("nan")

        cb = POTENTIAL_FN(trampoline)
        gpe_set_potential_fn(self._ctx, cb)
        self._vfn = (cb, errors)

    @contextlib.contextmanager
    def _callbacks(self):
        """Re-raise an exception of the potential callback in place of the
        library error it caused."""
        try:
            yield
        except GpeError as err:
            if self._vfn and self._vfn[1]:
                e = self._vfn[1][-1]
                self._vfn[1].clear()
                raise e from err
            raise

    def set_imag_method(self, method):
        """Imaginary-time nonlinear substep: "frozen" (density held at the
        substep's start, the default) or "exact" (Bernoulli solution with a
        running chemical-potential shift; mu then has no first-order dt bias)."""
        if method not in IMAG_METHODS:
            raise ValueError("method must be one of %s" % sorted(IMAG_METHODS))
        gpe_set_imag_method(self._ctx, IMAG_METHODS[method])

    @property
    def time(self):
        return gpe_get_time(self._ctx)

    @time.setter
    def time(self, t):
        gpe_set_time(self._ctx, t)

    def set_state(self, psi):
        p = np.ascontiguousarray(psi, dtype=np.complex128)
        if p.shape != self.shape:
            raise ValueError("psi shape %s != %s" % (p.shape, self.shape))
        gpe_set_state(self._ctx, p.view(np.float64))

    def get_state(self):
        out = np.empty(self.shape, np.complex128)
        gpe_get_state(self._ctx, out.view(np.float64))
        return out

    def _device_tensor(self, tensor):
        """Check a torch tensor before its pointer reaches the library: a
        contiguous complex128/complex64 tensor of the context's shape on the
        context's HIP device.  Returns the library's precision code."""
        dtype = str(getattr(tensor, "dtype", None))
        if dtype not in ("torch.complex128", "torch.complex64"):
            raise ValueError("need a complex128 or complex64 tensor, got %s" % dtype)
        dev = getattr(tensor, "device", None)
        if getattr(dev, "type", None) != "cuda":
            raise ValueError("need a tensor on the context's HIP device, got %s" % (dev,))
        ordinal = load_library().gpe_device(self._ctx)
        if dev.index is not None and dev.index != ordinal:
            raise ValueError("tensor on device %d, context on device %d" % (dev.index, ordinal))
        if tuple(tensor.shape) != self.shape or not tensor.is_contiguous():
            raise ValueError("need a contiguous tensor of shape %s" % (self.shape,))
        return GPE_FP32 if dtype == "torch.complex64" else GPE_FP64

    def _caller_stream_sync(self, tensor):
        """A context on its private stream is not ordered with the caller's
        torch stream: wait for the caller's pending work on the tensor."""
        if self._own_stream:
            import torch

            torch.cuda.current_stream(tensor.device).synchronize()

    def set_state_device(self, tensor):
        """tensor: a contiguous torch complex128/complex64 CUDA tensor."""
        src = self._device_tensor(tensor)
        self._caller_stream_sync(tensor)
        gpe_set_state_device(self._ctx, ctypes.c_void_p(tensor.data_ptr()), src)
        if self._own_stream:
            gpe_synchronize(self._ctx)  # the caller may overwrite the tensor next

    def get_state_device(self, tensor):
        dst = self._device_tensor(tensor)
        self._caller_stream_sync(tensor)
        gpe_get_state_device(self._ctx, ctypes.c_void_p(tensor.data_ptr()), dst)
        if self._own_stream:
            gpe_synchronize(self._ctx)  # the caller's stream reads the tensor next

    def evolve(self, dt, nsteps):
        with self._callbacks():
            gpe_evolve(self._ctx, dt, nsteps)

    def evolve_record(self, dt, nsteps, every):
        """Evolve and return the observables after every `every` steps (list of dicts)."""
        cap = (int(nsteps) + int(every) - 1) // int(every)
        series = (gpe_obs * max(cap, 1))()
        count = _I64(0)
        with self._callbacks():
            st = load_library().gpe_evolve_record(self._ctx, float(dt), int(nsteps), int(every),
                                                  series, cap, ctypes.byref(count))
            _check(st, self._ctx)
        return [dict(zip(OBS_KEYS, [o.norm, o.energy, o.mu, o.e_kin, o.e_pot, o.e_int,
                                    o.sigma[0], o.sigma[1], o.sigma[2], o.r_rms]))
                for o in series[:count.value]]

    def ground_state(self, dt, tol=1e-10, check_every=10, max_steps=1000000):
        with self._callbacks():
            st, steps, energy = gpe_ground_state(self._ctx, dt, tol, check_every, max_steps)
        return steps, energy, st == GPE_OK

    def imag_steps(self, dt, nsteps):
        with self._callbacks():
            gpe_ground_state(self._ctx, dt, 0.0, 0, nsteps)

    def observables(self):
        o = gpe_obs()
        with self._callbacks():
            gpe_observables(self._ctx, o, None)
        vals = [o.norm, o.energy, o.mu, o.e_kin, o.e_pot, o.e_int,
                o.sigma[0], o.sigma[1], o.sigma[2], o.r_rms]
        return dict(zip(OBS_KEYS, vals))

    def spectra(self, with_obs=False):
        """Shell spectra (dict of arrays and dk); with_obs: also the observables
        computed by the same call, as (spectra, observables)."""
        nb = gpe_spectra_bins(self._ctx)
        arrs = {k: np.zeros(nb) for k in ("n_k", "e_comp", "e_incomp", "e_qp")}
        s = gpe_spectra()
        s.nbins = nb
        s.n_k = _dptr(arrs["n_k"])
        s.e_comp = _dptr(arrs["e_comp"])
        s.e_incomp = _dptr(arrs["e_incomp"])
        s.e_qp = _dptr(arrs["e_qp"])
        o = gpe_obs()
        with self._callbacks():
            gpe_observables(self._ctx, o, s)
        arrs["dk"] = s.dk
        if with_obs:
            return arrs, dict(zip(OBS_KEYS, [o.norm, o.energy, o.mu, o.e_kin, o.e_pot, o.e_int,
                                             o.sigma[0], o.sigma[1], o.sigma[2], o.r_rms]))
        return arrs

    def transform(self, axes=None, inverse=False):
        mask = 0
        for a in (range(self.dim) if axes is None else axes):
            mask |= 1 << a
        gpe_transform(self._ctx, mask, int(bool(inverse)))

    def synchronize(self):
        gpe_synchronize(self._ctx)

    def timing(self, on=None):
        if on is not None:
            gpe_timing_enable(self._ctx, on)
            return None
        return gpe_timing_read(self._ctx)

    def device_bytes(self):
        return gpe_device_bytes(self._ctx)


def make_desc(shape, lo, hi, g, precision="fp64", norm_target=1.0):
    dim = len(shape)
    d = gpe_desc()
    d.dim = dim
    lo = np.broadcast_to(np.asarray(lo, np.float64), (dim,))
    hi = np.broadcast_to(np.asarray(hi, np.float64), (dim,))
    for j in range(dim):
        d.n[j] = int(shape[j])
        d.lo[j] = float(lo[j])
        d.hi[j] = float(hi[j])
    for j in range(dim, 3):
        d.n[j] = 1
    d.g = float(g)
    d.precision = PRECISIONS[precision]
    d.norm_target = float(norm_target)
    return d


class Server:
    """Request scheduler on the current HIP device (gpe_server_* calls).

    budget: HBM bytes for admitted requests (0: the device's free memory);
    max_slots: slots per shape class; max_active: requests running at once
    (0: no cap, 1: one at a time); chunk_steps: steps per replayed graph of a
    small-grid class (each round runs whole replays).
    """

    def __init__(self, budget=0, max_slots=16, max_active=0, chunk_steps=16):
        self._srv = gpe_server_create(budget, max_slots, max_active, chunk_steps)
        self._keep = {}
        self._shapes = {}

    def submit(self, shape, lo, hi, g, psi0, mode="real", dt=1e-3, nsteps=100,
               precision="fp64", trap=None, norm_target=1.0, keep_state=False):
        r = gpe_request()
        r.desc = make_desc(shape, lo, hi, g, precision, norm_target)
        if trap is not None:
            for j, w in enumerate(trap):
                r.trap.w[j] = float(w)
        p = np.ascontiguousarray(psi0, dtype=np.complex128)
        if p.shape != tuple(shape):
            raise ValueError("psi0 shape %s != %s" % (p.shape, tuple(shape)))
        r.psi0 = p.view(np.float64).ctypes.data_as(_DP)
        r.mode = 1 if mode in ("imag", "ground", 1) else 0
        r.dt = float(dt)
        r.nsteps = int(nsteps)
        r.keep_state = 1 if keep_state else 0
        rid = gpe_server_submit(self._srv, r)
        self._keep[rid] = keep_state
        self._shapes[rid] = tuple(shape)
        return rid

    def poll(self, rid):
        """None while pending; else a dict with status, obs, times, state."""
        out = gpe_result()
        st = gpe_server_poll(self._srv, rid, out, None)
        if st == GPE_EBUSY:
            return None
        if st != GPE_OK:
            raise GpeError(st, "gpe_server_poll")
        res = {"status": out.status, "steps_done": out.steps_done,
               "t_submit": out.t_submit, "t_start": out.t_start, "t_done": out.t_done,
               "obs": dict(zip(OBS_KEYS, [out.obs.norm, out.obs.energy, out.obs.mu,
                                          out.obs.e_kin, out.obs.e_pot, out.obs.e_int,
                                          out.obs.sigma[0], out.obs.sigma[1],
                                          out.obs.sigma[2], out.obs.r_rms]))}
        if self._keep.get(rid):
            psi = np.empty(self._shapes[rid], np.complex128)
            st = gpe_server_poll(self._srv, rid, out, psi.view(np.float64))
            res["psi"] = psi if st == GPE_OK else None
        return res

    def cancel(self, rid):
        return gpe_server_cancel(self._srv, rid)

    def release(self, rid):
        """Drop a finished request's record and stored state."""
        st = gpe_server_release(self._srv, rid)
        if st == GPE_OK:
            self._keep.pop(rid, None)
            self._shapes.pop(rid, None)
        return st

    def wait_idle(self):
        gpe_server_wait_idle(self._srv)

    def stats(self):
        return gpe_server_stats_read(self._srv)

    def close(self):
        if self._srv is not None:
            gpe_server_destroy(self._srv)
            self._srv = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
