"""GPU checks of the launch-shape tuner: every candidate shape gives the same
arithmetic per line (bitwise-equal results for widths and tile orders; pass
orders agree with the oracle), and tuned contexts keep oracle parity."""
import itertools
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


@pytest.fixture(autouse=True)
def clean_table():
    gpe.gpe_tuning_clear()
    yield
    gpe.gpe_tuning_clear()


def run(shape, lo, hi, g, trap, psi0, steps, prec="fp64"):
    with gpe.Context(shape, lo, hi, g, precision=prec, harmonic=trap) as ctx:
        ctx.set_state(psi0)
        ctx.evolve(1e-3, steps)
        return ctx.get_state()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_widths_and_tile_orders_are_bitwise_neutral(prec):
    shape, lo, hi = (64, 32, 128), (-6.0,) * 3, (6.0,) * 3
    trap = [1.0, 2.0, 3.0]
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=7)
    d = gpe.make_desc(shape, lo, hi, 20.0, prec)
    ref = run(shape, lo, hi, 20.0, trap, psi0, 12, prec)
    for w0, w1, x0, x1 in itertools.product([8, 16], [8, 16], [0, 1], [0, 1]):
        gpe.gpe_tuning_set(d, [w0, w1, 0], [x0, x1, 0], [2, 1, 0])
        say(prec, "width", w0, w1, "xcd", x0, x1)
        got = run(shape, lo, hi, 20.0, trap, psi0, 12, prec)
        assert np.array_equal(got, ref), (w0, w1, x0, x1)
    # streaming loads and stores change the cache policy, not the values
    for stream in itertools.product(range(4), repeat=3):
        gpe.gpe_tuning_set(d, [16, 8, 0], [1, 1, 0], [2, 1, 0], stream=list(stream))
        say(prec, "stream", stream)
        got = run(shape, lo, hi, 20.0, trap, psi0, 12, prec)
        assert np.array_equal(got, ref), stream


def test_pass_orders_match_the_oracle():
    shape, lo, hi = (32, 64, 16), (-5.0,) * 3, (5.0,) * 3
    trap = [1.0, 1.5, 2.0]
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=8)
    V = I.harmonic(shape, lo, hi, trap)
    ref = oracle.tssp_real(psi0, lo, hi, V, 30.0, 1e-3, 20)
    d = gpe.make_desc(shape, lo, hi, 30.0)
    for order in itertools.permutations(range(3)):
        gpe.gpe_tuning_set(d, [8, 8, 0], [1, 1, 0], list(order))
        say("order", order)
        got = run(shape, lo, hi, 30.0, trap, psi0, 20)
        assert rel(got, ref) < 1e-12, order


@pytest.mark.parametrize("shape", [(128, 128), (64, 64, 64)])
def test_autotune_records_an_entry_and_keeps_parity(shape):
    dim = len(shape)
    lo, hi = (-8.0,) * dim, (8.0,) * dim
    trap = [1.0] * dim
    d = gpe.make_desc(shape, lo, hi, 10.0)
    say("autotune", shape)
    t = gpe.gpe_autotune(d, steps=5)
    assert t["ms_per_step"] > 0
    assert sorted(t["pass_order"]) == list(range(dim))
    got_t, found = gpe.gpe_tuning_get(d)
    assert found and got_t == t
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=9)
    V = I.harmonic(shape, lo, hi, trap)
    ref = oracle.tssp_real(psi0, lo, hi, V, 10.0, 1e-3, 30)
    got = run(shape, lo, hi, 10.0, trap, psi0, 30)
    assert rel(got, ref) < 1e-12


def test_server_uses_the_tuned_shapes():
    """A server class created after tuning (pass order changed) still gives
    the single-context result bitwise."""
    shape, lo, hi = (64, 64, 32), (-6.0,) * 3, (6.0,) * 3
    d = gpe.make_desc(shape, lo, hi, 5.0)
    gpe.gpe_tuning_set(d, [16, 16, 0], [0, 0, 0], [0, 2, 1])
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=10)
    ref = run(shape, lo, hi, 5.0, [1.0, 1.0, 2.0], psi0, 25)
    with gpe.Server(max_slots=4, chunk_steps=8) as srv:
        rid = srv.submit(shape, lo, hi, 5.0, psi0, mode="real", dt=1e-3, nsteps=25,
                         trap=[1.0, 1.0, 2.0], keep_state=True)
        srv.wait_idle()
        out = srv.poll(rid)
    assert out["status"] == gpe.GPE_OK
    assert rel(out["psi"], ref) < 1e-12


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32s", 3e-7), ("fp32", 3e-6)])
def test_alternative_radix_plan_matches_oracle(prec, tol):
    """1024-point axes with the alternative plan (8, 8, 8, 2; 8 points per
    thread), contiguous and strided: transforms and a few TSSP steps against
    the oracle."""
    shape, lo, hi = (8, 1024, 1024), (-4.0, -10.0, -10.0), (4.0, 10.0, 10.0)
    d = gpe.make_desc(shape, lo, hi, 2.0, prec)
    gpe.gpe_tuning_set(d, [16, 8, 0], [1, 1, 0], [2, 1, 0], plan=[0, 1, 1])
    x = I.noisy_gaussian(shape, lo, hi, seed=31)
    say("plan 1 transform", prec)
    with gpe.Context(shape, lo, hi, 2.0, precision=prec) as ctx:
        ctx.set_state(x)
        ctx.transform()
        got = ctx.get_state()
    assert rel(got, oracle.fft(x)) < tol
    say("plan 1 steps", prec)
    V = I.harmonic(shape, lo, hi, [1.0, 0.5, 0.5])
    ref = oracle.tssp_real(x, lo, hi, V, 2.0, 1e-3, 3)
    got = run(shape, lo, hi, 2.0, [1.0, 0.5, 0.5], x, 3, prec)
    assert rel(got, ref) < max(tol, 1e-12) * 10


@pytest.mark.parametrize("prec", ["fp32s", "fp32"])
@pytest.mark.parametrize("shape", [(256, 128, 64), (512, 32, 64)])
def test_two_half_tiles_are_bitwise_neutral(prec, shape):
    """Width 32 (FP32 storage): the plain step passes of the strided axes take
    32-column tiles that go through the LDS as two 16-column halves; the
    arithmetic of every line is that of the 16-column tiles."""
    lo, hi = (-6.0,) * 3, (6.0,) * 3
    trap = [1.0, 2.0, 3.0]
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=17)
    d = gpe.make_desc(shape, lo, hi, 20.0, prec)
    gpe.gpe_tuning_set(d, [16, 16, 0], [1, 1, 0], [2, 1, 0])
    ref = run(shape, lo, hi, 20.0, trap, psi0, 9, prec)
    for xcd, stream in [((1, 1, 0), (0, 0, 0)), ((0, 0, 0), (3, 1, 0)), ((1, 0, 0), (2, 3, 0))]:
        gpe.gpe_tuning_set(d, [32, 32, 0], list(xcd), [2, 1, 0], stream=list(stream))
        say(prec, shape, "two halves", xcd, stream)
        got = run(shape, lo, hi, 20.0, trap, psi0, 9, prec)
        assert np.array_equal(got, ref), (xcd, stream)
