"""GPU parity of the separable analytic potentials (harmonic with a centre,
quartic, optical lattice) and of time-dependent potentials V(r, t) against the
oracle.  The GPU reads V from per-axis tables and fuses adjacent real-time N
half-steps (for V(r, t): the mean of the two midpoint potentials over dt); the
oracle steps unfused with the potential array at each midpoint."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2301_08275_amd import gpe
from paper_2301_08275_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


STATIC = dict(w=[1.0, 1.5, 2.0], center=[0.3, -0.2, 0.1], quartic=[0.05, 0.0, 0.02],
              lattice=[2.0, 1.0, 0.5], q=[1.5, 2.0, 1.0], phase=[0.0, 0.4, 1.0])


def params(dim, p):
    return {k: v[:dim] for k, v in p.items()}


def moving(t, dim):
    """Shaken lattice in a trap whose centre oscillates (a smooth V(r, t))."""
    p = dict(w=[1.0, 1.2, 1.5][:dim], center=[0.4 * math.sin(2.0 * t), 0.0, 0.0][:dim],
             quartic=[0.01] * dim, lattice=[1.0 + 0.5 * math.cos(3.0 * t), 0.8, 0.3][:dim],
             q=[2.0, 1.0, 1.5][:dim], phase=[0.3 * t, 0.0, 0.2][:dim])
    return p


CASES = [((64, 64), (-8.0, -8.0), (8.0, 8.0)),
         ((32, 32, 32), (-6.0, -6.0, -5.0), (6.0, 6.0, 5.0)),
         ((16, 64, 32), (-5.0, -8.0, -6.0), (5.0, 8.0, 6.0))]


@pytest.mark.parametrize("shape,lo,hi", CASES)
def test_static_separable_real_and_imag_time(shape, lo, hi):
    dim = len(shape)
    say("separable", shape)
    p = params(dim, STATIC)
    V = oracle.separable_potential(shape, lo, hi, **p)
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=11, amp=0.05)
    with gpe.Context(shape, lo, hi, 8.0) as ctx:
        ctx.set_separable(**p)
        ctx.set_state(psi0)
        o = ctx.observables()
        ref_o = oracle.observables(psi0, lo, hi, V, 8.0)
        assert abs(o["e_pot"] - ref_o["e_pot"]) < 1e-12 * abs(ref_o["e_pot"])
        ctx.evolve(1e-3, 150)
        assert rel(ctx.get_state(), oracle.tssp_real(psi0, lo, hi, V, 8.0, 1e-3, 150)) < 1e-10
        ctx.set_state(psi0)
        ctx.imag_steps(1e-3, 80)
        assert rel(ctx.get_state(), oracle.tssp_imag(psi0, lo, hi, V, 8.0, 1e-3, 80)) < 1e-10


@pytest.mark.parametrize("prec,tol", [("fp32s", 1e-5), ("fp32", 1e-4)])
def test_static_separable_fp32_forms(prec, tol):
    shape, lo, hi = CASES[1]
    p = params(3, STATIC)
    V = oracle.separable_potential(shape, lo, hi, **p)
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=12, amp=0.05)
    with gpe.Context(shape, lo, hi, 8.0, precision=prec) as ctx:
        ctx.set_separable(**p)
        ctx.set_state(psi0)
        ctx.evolve(1e-3, 100)
        assert rel(ctx.get_state(), oracle.tssp_real(psi0, lo, hi, V, 8.0, 1e-3, 100)) < tol


# the 1D grid has one pass per step, which carries both the opening and the
# closing phase (each with its own potential tables)
@pytest.mark.parametrize("shape,lo,hi", CASES[:2] + [((256,), (-10.0,), (10.0,))])
def test_time_dependent_potential_matches_the_unfused_oracle(shape, lo, hi):
    dim = len(shape)
    say("time-dependent", shape)
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=13, amp=0.05)
    g, dt = 6.0, 1e-3

    def Vfun(t):
        return oracle.separable_potential(shape, lo, hi, **moving(t, dim))

    calls = []
    with gpe.Context(shape, lo, hi, g) as ctx:
        ctx.set_potential_fn(lambda t: (calls.append(t), moving(t, dim))[1])
        ctx.set_state(psi0)
        ctx.time = 0.25
        ctx.evolve(dt, 70)           # split calls: the clock carries over
        ctx.evolve(dt, 1)
        ctx.evolve(dt, 59)
        assert abs(ctx.time - (0.25 + 130 * dt)) < 1e-12
        got = ctx.get_state()
        ref = oracle.tssp_real_tdep(psi0, lo, hi, Vfun, g, dt, 130, t0=0.25)
        assert rel(got, ref) < 1e-10
        # the observables take V at the clock
        o = ctx.observables()
        ref_o = oracle.observables(ref, lo, hi, Vfun(ctx.time), g)
        assert abs(o["e_pot"] - ref_o["e_pot"]) < 1e-10 * abs(ref_o["e_pot"])
        assert abs(o["energy"] - ref_o["energy"]) < 1e-10 * abs(ref_o["energy"])
        # the ground-state method holds V at the clock; imaginary time does not advance it
        t_now = ctx.time
        ctx.set_state(psi0)
        ctx.imag_steps(dt, 40)
        assert ctx.time == t_now
        ref_i = oracle.tssp_imag(psi0, lo, hi, Vfun(t_now), g, dt, 40)
        assert rel(ctx.get_state(), ref_i) < 1e-10
    assert min(calls) >= 0.25 and max(calls) <= t_now + 1e-12


def test_time_dependent_moving_trap_kohn_on_gpu():
    """Centre of mass against the closed form of Kohn's theorem (any g)."""
    shape, lo, hi = (64, 64), (-8.0, -8.0), (8.0, 8.0)
    A, W, w, dt = 0.5, 2.0, 1.0, 1e-3
    x = lo[0] + np.arange(shape[0]) * (hi[0] - lo[0]) / shape[0]
    with gpe.Context(shape, lo, hi, 5.0) as ctx:
        ctx.set_potential_fn(lambda t: dict(w=[w, 1.0], center=[A * math.sin(W * t), 0.0]))
        ctx.set_state(I.gaussian(shape, lo, hi))
        worst = 0.0
        for _ in range(4):
            ctx.evolve(dt, 500)
            t = ctx.time
            rho = np.abs(ctx.get_state()) ** 2
            X = float(np.sum(x[:, None] * rho) / np.sum(rho))
            Xk = A * w * w / (w * w - W * W) * (math.sin(W * t) - W / w * math.sin(w * t))
            worst = max(worst, abs(X - Xk))
    assert worst < 1e-6


def test_static_separable_graph_replay_is_bitwise_direct():
    shape, lo, hi = CASES[0]
    p = params(2, STATIC)
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=14, amp=0.05)
    out = []
    for timing in (False, True):
        with gpe.Context(shape, lo, hi, 8.0) as ctx:
            if timing:
                ctx.timing(True)
            ctx.set_separable(**p)
            ctx.set_state(psi0)
            ctx.evolve(1e-3, 100)
            ctx.ground_state(1e-3, tol=0.0, check_every=10, max_steps=70)
            out.append(ctx.get_state())
    assert np.array_equal(out[0], out[1])


def test_potential_errors():
    shape, lo, hi = CASES[0]
    with gpe.Context(shape, lo, hi, 1.0) as ctx:
        ctx.set_state(I.gaussian(shape, lo, hi))
        with pytest.raises(gpe.GpeError) as e:
            ctx.set_separable(w=[float("nan"), 1.0])
        assert e.value.status == gpe.GPE_EINVAL
        with pytest.raises(ValueError):
            ctx.set_separable(width=[1.0, 1.0])
        with pytest.raises(gpe.GpeError):
            ctx.time = float("inf")

        def bad(t):
            if t > 0.005:
                raise RuntimeError("callback failed at t=%g" % t)
            return dict(w=[1.0, 1.0])

        ctx.set_potential_fn(bad)
        with pytest.raises(RuntimeError):
            ctx.evolve(1e-3, 20)
        ctx.set_potential_fn(None)          # V = 0 again; the context still works
        ctx.set_state(I.gaussian(shape, lo, hi))
        ctx.evolve(1e-3, 5)
        assert abs(ctx.observables()["norm"] - 1.0) < 1e-12
