"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances (FP64): transforms 1e-13 relative L2 (round-off of an O(log N)
deep FFT); states after many steps 1e-10 relative L2 and norm drift 1e-12
(the accuracy bar set for the FP64 path).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2301_08275_amd import gpe
from paper_2301_08275_amd import inputs as I

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def random_state(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


TRANSFORM_SHAPES = [(8, 8), (16, 32), (1024, 8), (8, 1024), (512, 64), (64, 256),
                    (128, 128), (8, 8, 8), (16, 32, 64), (1024, 8, 16), (8, 1024, 8),
                    (32, 16, 1024), (64, 64, 64), (256, 8, 32), (8, 512, 16)]


@pytest.mark.parametrize("shape", TRANSFORM_SHAPES)
def test_transform_parity(shape):
    say("transform", shape)
    lo, hi = (0.0,) * len(shape), (1.0,) * len(shape)
    x = random_state(shape, len(shape) * 100 + shape[0])
    with gpe.Context(shape, lo, hi, 0.0) as ctx:
        ctx.set_state(x)
        ctx.transform()
        got = ctx.get_state()
        assert rel(got, oracle.fft(x)) < 1e-13
        ctx.transform(inverse=True)
        back = ctx.get_state()
        assert rel(back, x) < 1e-13
        for ax in range(len(shape)):
            ctx.set_state(x)
            ctx.transform(axes=[ax])
            assert rel(ctx.get_state(), oracle.fft_axis(x, ax)) < 1e-13, ax
            ctx.set_state(x)
            ctx.transform(axes=[ax], inverse=True)
            assert rel(ctx.get_state(), oracle.fft_axis(x, ax, inverse=True)) < 1e-13, ax


def cfg0():
    shape, lo, hi = (128, 128), (-8.0, -8.0), (8.0, 8.0)
    return shape, lo, hi, I.harmonic(shape, lo, hi, [1.0, 1.0]), I.noisy_gaussian(shape, lo, hi, seed=1)


@pytest.mark.parametrize("potential", ["array", "analytic"])
def test_cfg0_real_time_1000_steps(potential):
    """2D 128^2, g = 10, harmonic trap, dt = 1e-3, 1000 steps."""
    say("cfg0 real time", potential)
    shape, lo, hi, V, psi0 = cfg0()
    ref = oracle.tssp_real(psi0, lo, hi, V, 10.0, 1e-3, 1000)
    kw = dict(V=V) if potential == "array" else dict(harmonic=[1.0, 1.0])
    with gpe.Context(shape, lo, hi, 10.0, **kw) as ctx:
        ctx.set_state(psi0)
        n0 = ctx.observables()["norm"]
        ctx.evolve(1e-3, 1000)
        got = ctx.get_state()
        n1 = ctx.observables()["norm"]
    assert rel(got, ref) < 1e-10
    assert abs(n1 - n0) < 1e-12


def test_evolve_split_calls_match_one_call():
    """Chunked calls close and reopen the half-steps; the result must agree."""
    shape, lo, hi, V, psi0 = cfg0()
    with gpe.Context(shape, lo, hi, 10.0, V=V) as ctx:
        ctx.set_state(psi0)
        ctx.evolve(1e-3, 100)
        one = ctx.get_state()
        ctx.set_state(psi0)
        for _ in range(4):
            ctx.evolve(1e-3, 25)
        four = ctx.get_state()
    assert rel(four, one) < 1e-13


@pytest.mark.parametrize("shape,steps", [((32, 32, 32), 1000), ((64, 64, 64), 100),
                                         ((16, 64, 128), 200), ((128, 16, 8), 200)])
def test_3d_real_time_parity(shape, steps):
    say("3d real time", shape, steps)
    lo, hi = (-6.0, -5.0, -4.0), (6.0, 5.0, 4.0)
    V = I.harmonic(shape, lo, hi, [1.0, 1.5, 2.0])
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=7, amp=0.05)
    ref = oracle.tssp_real(psi0, lo, hi, V, 25.0, 1e-3, steps)
    with gpe.Context(shape, lo, hi, 25.0, harmonic=[1.0, 1.5, 2.0]) as ctx:
        ctx.set_state(psi0)
        ctx.evolve(1e-3, steps)
        got = ctx.get_state()
    assert rel(got, ref) < 1e-10


def test_3d_plane_wave_exact_on_gpu():
    shape, lo, hi = (64, 32, 128), (0.0,) * 3, (2 * np.pi,) * 3
    m, A, g, dt, steps = (3, -2, 7), 0.7, 2.0, 1e-3, 1000
    psi0 = I.plane_wave(shape, lo, hi, m, A)
    k2 = sum(mm * mm for mm in m)
    expect = psi0 * np.exp(-1j * (k2 / 2 + g * A * A) * steps * dt)
    with gpe.Context(shape, lo, hi, g) as ctx:
        ctx.set_state(psi0)
        ctx.evolve(dt, steps)
        got = ctx.get_state()
    assert rel(got, expect) < 1e-12


def test_time_reversal_on_gpu():
    shape, lo, hi = (32, 64, 16), (-6.0,) * 3, (6.0,) * 3
    V = I.harmonic(shape, lo, hi, [1.0, 2.0, 3.0])
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=5)
    with gpe.Context(shape, lo, hi, 20.0, V=V) as ctx:
        ctx.set_state(psi0)
        ctx.evolve(1e-3, 300)
        mid = ctx.get_state()
        ctx.evolve(-1e-3, 300)
        back = ctx.get_state()
    assert rel(mid, psi0) > 1e-3
    assert rel(back, psi0) < 1e-12


def test_observables_parity():
    shape, lo, hi = (32, 64, 16), (-6.0, -7.0, -3.0), (6.0, 7.0, 3.0)
    V = I.harmonic(shape, lo, hi, [1.0, 2.0, 4.0])
    psi = I.noisy_gaussian(shape, lo, hi, seed=3, amp=0.2)
    ref = oracle.observables(psi, lo, hi, V, 7.5)
    for kw in (dict(V=V), dict(harmonic=[1.0, 2.0, 4.0])):
        with gpe.Context(shape, lo, hi, 7.5, **kw) as ctx:
            ctx.set_state(psi)
            got = ctx.observables()
        for k in gpe.OBS_KEYS:
            assert abs(got[k] - ref[k]) <= 1e-12 * max(1.0, abs(ref[k])), (k, got[k], ref[k])


def test_imag_time_fixed_steps_parity():
    shape, lo, hi = (32, 64, 16), (-8.0, -8.0, -4.0), (8.0, 8.0, 4.0)
    V = I.harmonic(shape, lo, hi, [1.0, 2.0, 4.0])
    psi0 = I.gaussian(shape, lo, hi)
    ref = oracle.tssp_imag(psi0, lo, hi, V, 50.0, 1e-3, 300)
    with gpe.Context(shape, lo, hi, 50.0, V=V) as ctx:
        ctx.set_state(psi0)
        ctx.imag_steps(1e-3, 300)
        got = ctx.get_state()
    assert rel(got, ref) < 1e-11


def test_ground_state_parity_2d_table_row():
    """2D Table 1 row g = 12.5484 on 64^2: same stopping step and energy as the
    oracle, and the printed mu and r_rms."""
    shape, lo, hi = (64, 64), (-12.0, -12.0), (12.0, 12.0)
    V = I.harmonic(shape, lo, hi, [1.0, 1.0])
    psi0 = I.gaussian(shape, lo, hi)
    ref, rsteps, rE, rconv = oracle.ground_state(psi0, lo, hi, V, 12.5484, 1e-3, tol=1e-10)
    with gpe.Context(shape, lo, hi, 12.5484, harmonic=[1.0, 1.0]) as ctx:
        ctx.set_state(psi0)
        steps, E, conv = ctx.ground_state(1e-3, tol=1e-10, check_every=10)
        got = ctx.get_state()
        o = ctx.observables()
    assert conv and rconv
    assert steps == rsteps
    assert abs(E - rE) < 1e-12
    assert rel(got, ref) < 1e-9
    assert abs(o["mu"] / 2.25609 - 1) < 1e-4
    assert abs(o["r_rms"] / 1.30656 - 1) < 1e-4


def test_errors_are_reported():
    with pytest.raises(gpe.GpeError) as e:
        gpe.Context((12, 16), (0, 0), (1, 1), 0.0)
    assert e.value.status == gpe.GPE_EINVAL
    with pytest.raises(gpe.GpeError) as e:
        gpe.Context((2048, 16), (0, 0), (1, 1), 0.0)
    assert e.value.status == gpe.GPE_EUNSUPPORTED
    with pytest.raises(gpe.GpeError) as e:
        gpe.Context((16, 16), (0, 0), (0, 1), 0.0)
    assert e.value.status == gpe.GPE_EINVAL
    with gpe.Context((16, 16), (0, 0), (1, 1), 0.0) as ctx:
        with pytest.raises(gpe.GpeError) as e:
            ctx.evolve(0.0, 3)
        assert e.value.status == gpe.GPE_EINVAL
