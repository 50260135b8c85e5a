"""GPU checks of the rotating step passes (tuning entry transpose = 1).

Each rotating pass reads whole lines of its axis from one state array and
writes them, as rows of W sites, to the other, in the layout the next pass
reads; the axes go in the order 2, 0, 1, so a step starts and ends in the
stored layout.  Per line the arithmetic is that of the in-place passes, so
real-time results are bitwise those of the in-place passes run in the same
axis order; imaginary time (its norm sums run over other tiles) agrees to
rounding, and both agree with the oracle."""
import sys

import numpy as np
import pytest

import oracle
from paper_2301_08275_amd import gpe
from paper_2301_08275_amd import inputs as I

pytestmark = pytest.mark.gpu

ORDER = [2, 0, 1]  # the axis order of the rotating passes


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(autouse=True)
def clean_table():
    gpe.gpe_tuning_clear()
    yield
    gpe.gpe_tuning_clear()


def set_rotating(d, width=(8, 8, 8), xcd=(1, 1, 1), stream=(0, 0, 0), plan=None):
    gpe.gpe_tuning_set(d, list(width), list(xcd), ORDER, stream=list(stream), transpose=1,
                       plan=plan)


def set_in_place(d):
    gpe.gpe_tuning_set(d, [16, 8, 0], [1, 1, 0], ORDER)


def real_run(shape, lo, hi, g, psi0, calls, prec="fp64", trap=None, V=None, sep=None):
    """Real-time steps in several calls (odd counts leave the state in the
    second array between calls); the state and the observables after each."""
    out = []
    with gpe.Context(shape, lo, hi, g, precision=prec, harmonic=trap, V=V) as ctx:
        if sep is not None:
            ctx.set_potential_fn(sep)
        ctx.set_state(psi0)
        for n in calls:
            ctx.evolve(1e-3, n)
            o = ctx.observables()
            out.append((ctx.get_state(), o["norm"], o["energy"]))
    return out


CASES = [((128, 128, 128), "fp64"), ((128, 128, 128), "fp32s"), ((128, 128, 128), "fp32"),
         ((64, 128, 256), "fp64"), ((256, 64, 128), "fp32s")]


@pytest.mark.parametrize("shape,prec", CASES)
def test_rotating_real_time_is_bitwise_the_in_place_passes(shape, prec):
    lo, hi = (-6.0, -7.0, -8.0), (6.0, 7.0, 8.0)
    trap = [1.0, 1.5, 2.0]
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=51)
    d = gpe.make_desc(shape, lo, hi, 25.0, prec)
    set_in_place(d)
    say("in place", shape, prec)
    ref = real_run(shape, lo, hi, 25.0, psi0, [3, 4, 1], prec, trap=trap)
    combos = [((8, 8, 8), (1, 1, 1), (0, 0, 0)), ((16, 16, 16), (0, 0, 0), (3, 1, 2)),
              ((8, 16, 8), (0, 1, 0), (1, 2, 3)), ((4, 4, 4), (1, 1, 1), (3, 3, 1)),
              ((4, 8, 16), (0, 1, 1), (0, 2, 0))]
    for width, xcd, stream in combos:
        set_rotating(d, width, xcd, stream)
        t, found = gpe.gpe_tuning_get(d)
        assert found and t["transpose"] == 1 and t["width"] == list(width)
        say("rotating", shape, prec, width, xcd, stream)
        got = real_run(shape, lo, hi, 25.0, psi0, [3, 4, 1], prec, trap=trap)
        for (a, na, ea), (b, nb, eb) in zip(got, ref):
            assert np.array_equal(a, b), (width, xcd, stream)
            # (the observables' sums follow the tile widths of the entry)
            assert abs(na - nb) <= 1e-14 * abs(nb) and abs(ea - eb) <= 1e-14 * abs(eb)


def test_rotating_passes_with_a_potential_array_and_a_moving_lattice():
    shape, lo, hi = (128, 128, 128), (-6.0,) * 3, (6.0,) * 3
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=52)
    V = I.harmonic(shape, lo, hi, [1.0, 2.0, 0.5]) + 0.1 * np.cos(
        np.add.outer(np.add.outer(np.arange(128), 2 * np.arange(128)), 3 * np.arange(128)) * 0.05)

    def lattice(t):
        return dict(w=[1.0, 1.0, 1.0], lattice=[0.5 + t, 0.0, 0.25], q=[2.0, 1.0, 3.0])

    d = gpe.make_desc(shape, lo, hi, 15.0)
    for kw in (dict(V=V), dict(sep=lattice)):
        set_in_place(d)
        ref = real_run(shape, lo, hi, 15.0, psi0, [5, 2], **kw)
        set_rotating(d)
        say("rotating with", list(kw))
        got = real_run(shape, lo, hi, 15.0, psi0, [5, 2], **kw)
        for (a, _, _), (b, _, _) in zip(got, ref):
            assert np.array_equal(a, b), list(kw)


def test_rotating_real_time_matches_the_oracle():
    shape, lo, hi = (128, 128, 128), (-6.0,) * 3, (6.0,) * 3
    trap = [1.0, 1.0, 1.5]
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=53)
    V = I.harmonic(shape, lo, hi, trap)
    d = gpe.make_desc(shape, lo, hi, 20.0)
    set_rotating(d)
    say("rotating vs oracle, 10 steps")
    got = real_run(shape, lo, hi, 20.0, psi0, [10], trap=trap)[0][0]
    ref = oracle.tssp_real(psi0, lo, hi, V, 20.0, 1e-3, 10)
    assert rel(got, ref) < 1e-12


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32s", 1e-6)])
def test_rotating_imaginary_time(prec, tol):
    shape, lo, hi = (128, 128, 128), (-6.0,) * 3, (6.0,) * 3
    trap = [1.0, 1.5, 2.0]
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=54)
    d = gpe.make_desc(shape, lo, hi, 10.0, prec)
    out = {}
    for form in ("in place", "rotating"):
        (set_in_place if form == "in place" else set_rotating)(d)
        say(form, "imaginary time", prec)
        with gpe.Context(shape, lo, hi, 10.0, precision=prec, harmonic=trap) as ctx:
            ctx.set_state(psi0)
            ctx.imag_steps(1e-3, 7)
            out[form] = (ctx.get_state(), ctx.observables()["energy"])
    a, b = out["rotating"], out["in place"]
    # (the renormalisation's sums differ in the last bits; with FP32 storage
    # that can move a stored value by one FP32 rounding)
    close = 1e-13 if prec == "fp64" else 1e-7
    assert rel(a[0], b[0]) < close and abs(a[1] - b[1]) < close * abs(b[1])
    if prec == "fp64":
        V = I.harmonic(shape, lo, hi, trap)
        ref = oracle.tssp_imag(psi0, lo, hi, V, 10.0, 1e-3, 7)
        assert rel(a[0], ref) < tol


def test_rotating_is_refused_where_it_does_not_apply():
    with pytest.raises(gpe.GpeError):
        gpe.gpe_tuning_set(gpe.make_desc((64, 64), (-1, -1), (1, 1), 1.0), [8, 8], [0, 0], [0, 1],
                           transpose=1)
    # small 3D grids run the in-place passes (and their step graphs) whatever the entry
    shape, lo, hi = (32, 32, 32), (-4.0,) * 3, (4.0,) * 3
    d = gpe.make_desc(shape, lo, hi, 5.0)
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=55)
    set_in_place(d)
    ref = real_run(shape, lo, hi, 5.0, psi0, [40], trap=[1.0, 1.0, 1.0])[0][0]
    set_rotating(d)
    got = real_run(shape, lo, hi, 5.0, psi0, [40], trap=[1.0, 1.0, 1.0])[0][0]
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("shape,prec", [((1024, 32, 64), "fp64"), ((32, 64, 1024), "fp32s"),
                                        ((64, 1024, 32), "fp32")])
def test_rotating_passes_on_1024_point_axes(shape, prec):
    """A 1024-point axis in the rotating form, with either radix plan (16
    points per thread, or 8 with one more exchange each way)."""
    lo, hi = (-6.0, -7.0, -8.0), (6.0, 7.0, 8.0)
    trap = [1.0, 1.5, 2.0]
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=56)
    d = gpe.make_desc(shape, lo, hi, 25.0, prec)
    big = [int(n == 1024) for n in shape]
    for plan in ([0, 0, 0], big):
        gpe.gpe_tuning_set(d, [16, 8, 0], [1, 1, 0], ORDER, plan=plan)
        say("in place", shape, prec, "plan", plan)
        ref = real_run(shape, lo, hi, 25.0, psi0, [3, 2], prec, trap=trap)
        for width in ((8, 8, 8), (4, 4, 4)):
            set_rotating(d, width=width, plan=plan)
            say("rotating", shape, prec, "plan", plan, "width", width)
            got = real_run(shape, lo, hi, 25.0, psi0, [3, 2], prec, trap=trap)
            for (a, _, _), (b, _, _) in zip(got, ref):
                assert np.array_equal(a, b), (plan, width)
