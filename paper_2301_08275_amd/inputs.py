"""Seeded synthetic inputs: grids, potentials and initial wavefunctions.

This module holds no step of the solver's arithmetic (no FFT, no phase, no
reduction of the method).  It only draws random numbers and evaluates the
closed-form initial conditions and traps, so that the GPU library and the CPU
oracle are fed identical arrays.

Random numbers: SplitMix64 (Steele, Lea and Flood, 2014) in counter form,
draw i of a stream with seed s is mix(s + (i+1) * 0x9E3779B97F4A7C15);
uniforms are (x >> 11) * 2^-53 and normals come from Box-Muller with 1-u
inside the logarithm.
"""
import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, count, offset=0):
    """Raw 64-bit draws offset..offset+count-1 of the stream `seed`."""
    i = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed, count, offset=0):
    """Uniform doubles in [0, 1)."""
    return (splitmix64(seed, count, offset) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def normal_pairs(seed, npairs, offset=0):
    """Box-Muller: npairs pairs (z0, z1) of independent standard normals."""
    u = uniform(seed, 2 * npairs, offset)
    u1, u2 = u[0::2], u[1::2]
    r = np.sqrt(-2.0 * np.log(1.0 - u1))
    return r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)


def axes(shape, lo, hi):
    """Per-axis coordinates x_{j,i} = lo_j + i (hi_j - lo_j) / n_j."""
    dim = len(shape)
    lo = np.broadcast_to(np.asarray(lo, np.float64), (dim,))
    hi = np.broadcast_to(np.asarray(hi, np.float64), (dim,))
    return [lo[j] + np.arange(shape[j]) * ((hi[j] - lo[j]) / shape[j]) for j in range(dim)]


def cell_volume(shape, lo, hi):
    dim = len(shape)
    lo = np.broadcast_to(np.asarray(lo, np.float64), (dim,))
    hi = np.broadcast_to(np.asarray(hi, np.float64), (dim,))
    return float(np.prod((hi - lo) / np.asarray(shape, np.float64)))


def _mesh(shape, lo, hi):
    xs = axes(shape, lo, hi)
    return np.meshgrid(*xs, indexing="ij")


def harmonic(shape, lo, hi, omega):
    """V = 1/2 sum_j omega_j^2 x_j^2 on the grid (float64)."""
    X = _mesh(shape, lo, hi)
    V = np.zeros(shape)
    for j, x in enumerate(X):
        V += 0.5 * (omega[j] ** 2) * x * x
    return V


def normalise(psi, shape, lo, hi, target=1.0):
    dv = cell_volume(shape, lo, hi)
    return psi * math.sqrt(target / (dv * float(np.sum(np.abs(psi) ** 2))))


def gaussian(shape, lo, hi, widths=None, eps=1.0, norm=1.0):
    """psi ~ exp(-sum_j widths_j x_j^2 / (2 eps)), normalised to `norm`."""
    X = _mesh(shape, lo, hi)
    if widths is None:
        widths = [1.0] * len(shape)
    arg = np.zeros(shape)
    for j, x in enumerate(X):
        arg += widths[j] * x * x
    psi = np.exp(-arg / (2 * eps)).astype(np.complex128)
    return normalise(psi, shape, lo, hi, norm)


def noisy_gaussian(shape, lo, hi, seed, amp=0.01, widths=None):
    """Gaussian times (1 + amp (a + i b)), a, b = 2u - 1 drawn per site in
    row-major order (re then im), renormalised to 1."""
    psi = gaussian(shape, lo, hi, widths)
    u = uniform(seed, 2 * psi.size).reshape(psi.shape + (2,))
    noise = (2 * u[..., 0] - 1) + 1j * (2 * u[..., 1] - 1)
    return normalise(psi * (1 + amp * noise), shape, lo, hi)


def plane_wave(shape, lo, hi, m, amp=1.0):
    """A exp(i k.x) with k_j = 2 pi m_j / L_j."""
    X = _mesh(shape, lo, hi)
    dim = len(shape)
    lo = np.broadcast_to(np.asarray(lo, np.float64), (dim,))
    hi = np.broadcast_to(np.asarray(hi, np.float64), (dim,))
    ph = np.zeros(shape)
    for j, x in enumerate(X):
        ph += 2 * np.pi * m[j] / (hi[j] - lo[j]) * x
    return amp * np.exp(1j * ph)


def phase_field_modes(seed, kmax=8, dim=3):
    """Random phase spectrum: integer modes 1 <= |m| <= kmax, per-mode variance
    proportional to |m|^-2, Hermitian symmetric.  Returns (modes, coeff) for
    the independent half (first nonzero component positive), scaled so that
    the rms of |grad theta| on [0, 2 pi)^dim is 1.  Modes are enumerated in
    lexicographic order of m; each takes one Box-Muller pair (re, im)."""
    modes = []
    for m in np.ndindex(*([2 * kmax + 1] * dim)):
        mm = tuple(int(v) - kmax for v in m)
        r2 = sum(v * v for v in mm)
        if r2 < 1 or r2 > kmax * kmax:
            continue
        first = next(v for v in mm if v != 0)
        if first > 0:
            modes.append(mm)
    modes = np.array(modes, dtype=np.int64)
    z0, z1 = normal_pairs(seed, len(modes))
    k = np.sqrt((modes ** 2).sum(axis=1).astype(np.float64))
    coeff = (z0 + 1j * z1) / k
    # theta = sum over +m and -m: <|grad theta|^2> = 2 sum_half |m|^2 |c|^2
    grad2 = 2.0 * float(np.sum(k ** 2 * np.abs(coeff) ** 2))
    coeff = coeff / math.sqrt(grad2)
    return modes, coeff


def phase_field(n, seed, kmax=8, dtype=np.complex128):
    """psi = exp(i theta) on the periodic box [0, 2 pi)^3 at n^3 points, theta
    the band-limited random field of phase_field_modes.  theta is evaluated by
    direct summation of its Fourier series, one axis at a time (separable
    contraction over the 2 kmax + 1 modes per axis); no FFT."""
    modes, coeff = phase_field_modes(seed, kmax, 3)
    K = 2 * kmax + 1
    C = np.zeros((K, K, K), np.complex128)
    for (mx, my, mz), c in zip(modes, coeff):
        C[mx + kmax, my + kmax, mz + kmax] += c
        C[-mx + kmax, -my + kmax, -mz + kmax] += np.conj(c)
    x = 2 * np.pi * np.arange(n) / n
    m = np.arange(-kmax, kmax + 1)
    E = np.exp(1j * np.outer(m, x))  # (K, n)
    T1 = np.tensordot(C, E, axes=([2], [0]))          # (K, K, n): [mx, my, z]
    T2 = np.einsum("abz,by->ayz", T1, E)               # (K, n, n): [mx, y, z]
    out = np.empty((n, n, n), dtype=dtype)
    chunk = max(1, (1 << 22) // (n * n))
    T2f = T2.reshape(K, n * n)
    for x0 in range(0, n, chunk):
        x1 = min(n, x0 + chunk)
        th = (E[:, x0:x1].T @ T2f).real.reshape(x1 - x0, n, n)
        out[x0:x1] = np.exp(1j * th).astype(dtype)
    return out


def bao_initial(shape, lo, hi, gamma_y=2.0, gamma_z=4.0, eps1=0.25):
    """Dynamics-validation initial state: exp(-(x^2 + gy y^2 + gz z^2)/(2 eps1)),
    normalised numerically to 1."""
    return gaussian(shape, lo, hi, widths=[1.0, gamma_y, gamma_z][: len(shape)], eps=eps1)


def serving_trace(nreq, seed=4, rate=200.0, box=8.0):
    """The serving mix: a seeded Poisson stream of independent solves.

    Request i draws (in this order, from stream `seed`, 8 uniforms each):
    inter-arrival time (exponential, mean 1/rate), 2D (60 %) or 3D (40 %),
    grid size uniform over {64, 128, 256, 512}^2 or {64, 128, 256}^3, trap
    anisotropy a ~ U[1, 8] (V = (x^2 + a^2 y^2)/2 in 2D, (x^2 + y^2 + a^2 z^2)/2
    in 3D), g ~ U[0, 100], ground state or real time (half each; both a fixed
    step count), steps ~ U{200..2000}, FP32 or FP64 (half each).  The box is
    [-box, box)^d and dt = 1e-3.  The initial state (psi0_of) is a Gaussian with
    1 % noise seeded by the request index.
    """
    u = uniform(seed, 8 * nreq).reshape(nreq, 8)
    t = 0.0
    out = []
    for i in range(nreq):
        t += -math.log(1.0 - u[i, 0]) / rate
        dim = 2 if u[i, 1] < 0.6 else 3
        sizes = (64, 128, 256, 512) if dim == 2 else (64, 128, 256)
        n = sizes[min(len(sizes) - 1, int(u[i, 2] * len(sizes)))]
        a = 1.0 + 7.0 * u[i, 3]
        g = 100.0 * u[i, 4]
        mode = "imag" if u[i, 5] < 0.5 else "real"
        steps = 200 + min(1800, int(u[i, 6] * 1801))
        prec = "fp32" if u[i, 7] < 0.5 else "fp64"
        trap = [1.0, a] if dim == 2 else [1.0, 1.0, a]
        out.append(dict(index=i, arrival=t, shape=(n,) * dim, lo=(-box,) * dim, hi=(box,) * dim,
                        g=g, trap=trap, mode=mode, nsteps=steps, dt=1e-3, precision=prec))
    return out


def psi0_of(req, seed_base=40000):
    """Initial state of a serving request (see serving_trace)."""
    return noisy_gaussian(req["shape"], req["lo"], req["hi"], seed=seed_base + req["index"])
