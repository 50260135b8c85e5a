"""Plain FP64 CPU oracle for the TSSP Gross-Pitaevskii solver (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module.  It shares no code
with the GPU library and never imports it.

All arrays are numpy complex128 (psi) or float64 (V), row-major, last axis
contiguous.  Functions return new arrays and never modify their inputs.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force=True):
    """Compile the oracle library with g++ (plain -O2, no fast-math)."""
    from .buildlib import build_oracle

    build_oracle(force=force)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lp = ctypes.POINTER(ctypes.c_long)
    c_int, c_long, c_double = ctypes.c_int, ctypes.c_long, ctypes.c_double
    lib.orc_set_threads.argtypes = [c_int]
    lib.orc_get_threads.restype = c_int
    lib.orc_fft.argtypes = [dp, c_int, ip, c_int]
    lib.orc_fft_axis.argtypes = [dp, c_int, ip, c_int, c_int]
    lib.orc_tssp_real.argtypes = [dp, c_int, ip, dp, dp, dp, c_double, c_double, c_long]
    lib.orc_tssp_imag.argtypes = [dp, c_int, ip, dp, dp, dp, c_double, c_double,
                                  c_long, c_double, c_int]
    lib.orc_nonlinear_imag.argtypes = [dp, c_int, ip, dp, dp, dp, c_double, c_double, c_int]
    lib.orc_ground_state.argtypes = [dp, c_int, ip, dp, dp, dp, c_double, c_double,
                                     c_double, c_int, c_long, c_double, c_int, lp, dp]
    lib.orc_observables.argtypes = [dp, c_int, ip, dp, dp, dp, c_double, dp]
    lib.orc_nonlinear_real.argtypes = [dp, c_int, ip, dp, dp, dp, c_double, c_double]
    lib.orc_kinetic_real.argtypes = [dp, c_int, ip, dp, dp, c_double]
    lib.orc_spectra_bins.argtypes = [c_int, ip, dp, dp, dp]
    lib.orc_spectra.argtypes = [dp, c_int, ip, dp, dp, c_int, dp, dp, dp, dp]
    for f in (lib.orc_fft, lib.orc_fft_axis, lib.orc_tssp_real, lib.orc_tssp_imag,
              lib.orc_ground_state, lib.orc_observables, lib.orc_spectra_bins,
              lib.orc_spectra, lib.orc_nonlinear_real, lib.orc_kinetic_real,
              lib.orc_nonlinear_imag):
        f.restype = c_int
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _shape(psi):
    n = (ctypes.c_int * 3)(*(list(psi.shape) + [1] * (3 - psi.ndim)))
    return psi.ndim, n


def _box(lo, hi, dim):
    lo = np.ascontiguousarray(np.broadcast_to(np.asarray(lo, np.float64), (dim,)))
    hi = np.ascontiguousarray(np.broadcast_to(np.asarray(hi, np.float64), (dim,)))
    return lo, hi


def _state(psi):
    return np.array(psi, dtype=np.complex128, order="C", copy=True)


def _pot(V, shape):
    if V is None:
        return None
    V = np.ascontiguousarray(V, dtype=np.float64)
    if V.shape != tuple(shape):
        raise ValueError("V shape %s does not match psi %s" % (V.shape, shape))
    return V


def _check(rc, name):
    if rc < 0:
        raise ValueError("oracle %s rejected its arguments (rc=%d)" % (name, rc))
    return rc


def set_threads(n):
    _load().orc_set_threads(int(n))


def get_threads():
    return _load().orc_get_threads()


def fft(psi, inverse=False):
    """Full n-d DFT (forward unnormalised; inverse carries 1/N_tot)."""
    lib = _load()
    out = _state(psi)
    dim, n = _shape(out)
    _check(lib.orc_fft(_dptr(out), dim, n, int(bool(inverse))), "fft")
    return out


def fft_axis(psi, axis, inverse=False):
    lib = _load()
    out = _state(psi)
    dim, n = _shape(out)
    _check(lib.orc_fft_axis(_dptr(out), dim, n, int(axis), int(bool(inverse))), "fft_axis")
    return out


def tssp_real(psi, lo, hi, V, g, dt, nsteps):
    lib = _load()
    out = _state(psi)
    dim, n = _shape(out)
    lo, hi = _box(lo, hi, dim)
    V = _pot(V, out.shape)
    _check(lib.orc_tssp_real(_dptr(out), dim, n, _dptr(lo), _dptr(hi),
                             _dptr(V) if V is not None else None,
                             float(g), float(dt), int(nsteps)), "tssp_real")
    return out


def separable_potential(shape, lo, hi, w=None, center=None, quartic=None, lattice=None,
                        q=None, phase=None):
    """V(r) = sum_j v_j(x_j) with v_j(x) = 1/2 w_j^2 (x - c_j)^2 + a_j (x - c_j)^4
    + s_j sin^2(q_j x + phi_j) on the grid x_j = lo_j + i h_j (the anharmonic
    traps and optical lattices of the feature list, in the form this
    implementation reads them; parameters not given are zero)."""
    dim = len(shape)
    lo, hi = _box(lo, hi, dim)

    def par(v, j):
        return 0.0 if v is None else float(v[j])

    V = np.zeros(shape)
    for j in range(dim):
        x = lo[j] + np.arange(shape[j]) * (hi[j] - lo[j]) / shape[j]
        d = x - par(center, j)
        v = (0.5 * par(w, j) ** 2 * d ** 2 + par(quartic, j) * d ** 4
             + par(lattice, j) * np.sin(par(q, j) * x + par(phase, j)) ** 2)
        V += v.reshape([shape[j] if k == j else 1 for k in range(dim)])
    return V


def tssp_real_tdep(psi, lo, hi, Vfun, g, dt, nsteps, t0=0.0):
    """Real-time Strang steps with a time-dependent potential Vfun(t) (an
    array of psi's shape).  Step s covers [t_s, t_s + dt], t_s = t0 + s dt:
    N(dt/2) with V at the midpoint t_s + dt/4 of its interval, K(dt), N(dt/2)
    with V at t_s + 3 dt/4 (an N substep holds |psi| fixed, so its exact
    solution integrates V over the interval; the midpoint rule keeps second
    order).  Unfused, in the order of the scheme."""
    lib = _load()
    out = _state(psi)
    dim, n = _shape(out)
    lo, hi = _box(lo, hi, dim)
    for s in range(int(nsteps)):
        ts = t0 + s * dt
        for t_mid in (ts + dt / 4, None, ts + 3 * dt / 4):
            if t_mid is None:
                _check(lib.orc_kinetic_real(_dptr(out), dim, n, _dptr(lo), _dptr(hi), float(dt)),
                       "kinetic_real")
                continue
            V = _pot(Vfun(t_mid), out.shape)
            _check(lib.orc_nonlinear_real(_dptr(out), dim, n, _dptr(lo), _dptr(hi),
                                          _dptr(V) if V is not None else None, float(g),
                                          float(dt) / 2), "nonlinear_real")
    return out


def tssp_imag(psi, lo, hi, V, g, dt, nsteps, norm_target=1.0, exact=False):
    """nsteps imaginary-time steps; exact: solve each N substep exactly
    instead of holding the density at its start value."""
    lib = _load()
    out = _state(psi)
    dim, n = _shape(out)
    lo, hi = _box(lo, hi, dim)
    V = _pot(V, out.shape)
    _check(lib.orc_tssp_imag(_dptr(out), dim, n, _dptr(lo), _dptr(hi),
                             _dptr(V) if V is not None else None,
                             float(g), float(dt), int(nsteps), float(norm_target),
                             int(bool(exact))),
           "tssp_imag")
    return out


def nonlinear_imag(psi, lo, hi, V, g, tau, exact=False):
    """One imaginary-time N(tau) substep."""
    lib = _load()
    out = _state(psi)
    dim, n = _shape(out)
    lo, hi = _box(lo, hi, dim)
    V = _pot(V, out.shape)
    _check(lib.orc_nonlinear_imag(_dptr(out), dim, n, _dptr(lo), _dptr(hi),
                                  _dptr(V) if V is not None else None, float(g), float(tau),
                                  int(bool(exact))), "nonlinear_imag")
    return out


def ground_state(psi, lo, hi, V, g, dt, tol=1e-10, check_every=10,
                 max_steps=1000000, norm_target=1.0, exact=False):
    """Returns (psi, steps_done, energy, converged)."""
    lib = _load()
    out = _state(psi)
    dim, n = _shape(out)
    lo, hi = _box(lo, hi, dim)
    V = _pot(V, out.shape)
    steps = ctypes.c_long(0)
    energy = ctypes.c_double(0)
    rc = _check(lib.orc_ground_state(_dptr(out), dim, n, _dptr(lo), _dptr(hi),
                                     _dptr(V) if V is not None else None,
                                     float(g), float(dt), float(tol), int(check_every),
                                     int(max_steps), float(norm_target), int(bool(exact)),
                                     ctypes.byref(steps), ctypes.byref(energy)),
                "ground_state")
    return out, steps.value, energy.value, rc == 0


OBS_KEYS = ("norm", "energy", "mu", "e_kin", "e_pot", "e_int",
            "sigma_x", "sigma_y", "sigma_z", "r_rms")


def observables(psi, lo, hi, V, g):
    lib = _load()
    p = np.ascontiguousarray(psi, dtype=np.complex128)
    dim, n = _shape(p)
    lo, hi = _box(lo, hi, dim)
    V = _pot(V, p.shape)
    out = np.zeros(10)
    _check(lib.orc_observables(_dptr(p), dim, n, _dptr(lo), _dptr(hi),
                               _dptr(V) if V is not None else None, float(g),
                               _dptr(out)), "observables")
    return dict(zip(OBS_KEYS, out.tolist()))


def spectra_bins(shape, lo, hi):
    lib = _load()
    dim = len(shape)
    n = (ctypes.c_int * 3)(*(list(shape) + [1] * (3 - dim)))
    lo, hi = _box(lo, hi, dim)
    dk = ctypes.c_double(0)
    nb = _check(lib.orc_spectra_bins(dim, n, _dptr(lo), _dptr(hi), ctypes.byref(dk)),
                "spectra_bins")
    return nb, dk.value


def spectra(psi, lo, hi):
    """Shell sums dict: n_k, e_comp, e_incomp, e_qp (float64 arrays) and dk."""
    lib = _load()
    p = np.ascontiguousarray(psi, dtype=np.complex128)
    dim, n = _shape(p)
    nb, dk = spectra_bins(p.shape, lo, hi)
    lo, hi = _box(lo, hi, dim)
    res = {k: np.zeros(nb) for k in ("n_k", "e_comp", "e_incomp", "e_qp")}
    _check(lib.orc_spectra(_dptr(p), dim, n, _dptr(lo), _dptr(hi), nb,
                           _dptr(res["n_k"]), _dptr(res["e_comp"]),
                           _dptr(res["e_incomp"]), _dptr(res["e_qp"])), "spectra")
    res["dk"] = dk
    return res
