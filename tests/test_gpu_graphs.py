"""Small single-context grids replay runs of identical steps (real time
between the opening and closing half-steps, imaginary time between two
checks) from HIP graphs.  The graph holds the same launches as the direct path (which runs
when per-pass timing is on), so both must give the same bits; the oracle
checks the step itself (the 128^2 runs of the parity tests use the graph)."""
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


def setup(shape, seed=3):
    d = len(shape)
    lo, hi = (-8.0,) * d, (8.0,) * d
    return lo, hi, I.noisy_gaussian(shape, lo, hi, seed=seed, amp=0.05)


def run(shape, calls, timing, prec="fp64", trap=None, with_log=False):
    lo, hi, psi0 = setup(shape)
    trap = trap or [1.0] * len(shape)
    with gpe.Context(shape, lo, hi, 20.0, precision=prec, harmonic=trap) as ctx:
        if timing:
            ctx.timing(True)
        ctx.set_state(psi0)
        out = []
        for call in calls:
            if call[0] == "evolve":
                ctx.evolve(call[1], call[2])
            elif call[0] == "imag":
                ctx.imag_steps(call[1], call[2])
            elif call[0] == "ground":
                out.append(ctx.ground_state(call[1], tol=call[2], check_every=call[3],
                                            max_steps=call[4]))
            else:
                ctx.set_potential(harmonic=call[1])
        return (ctx.get_state(), out) if with_log else ctx.get_state()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32s"])
@pytest.mark.parametrize("shape", [(64, 64), (128, 128), (32, 32, 32), (64, 64, 64)])
def test_graph_replay_is_bitwise_direct(shape, prec):
    calls = [("evolve", 1e-3, n) for n in (33, 34, 35, 66, 67, 100, 1, 2)]
    say("graph vs direct", shape, prec)
    a = run(shape, calls, timing=False, prec=prec)
    b = run(shape, calls, timing=True, prec=prec)
    assert np.array_equal(a, b)


def test_graph_dropped_when_the_potential_changes():
    shape = (64, 64)
    calls = [("evolve", 1e-3, 80), ("potential", [1.0, 3.0]), ("evolve", 1e-3, 80),
             ("potential", [2.0, 2.0]), ("evolve", 1e-3, 40)]
    a = run(shape, calls, timing=False)
    b = run(shape, calls, timing=True)
    assert np.array_equal(a, b)
    # and the physics of the second trap is the oracle's
    lo, hi, psi0 = setup(shape)
    ref = oracle.tssp_real(psi0, lo, hi, I.harmonic(shape, lo, hi, [1.0, 1.0]), 20.0, 1e-3, 80)
    ref = oracle.tssp_real(ref, lo, hi, I.harmonic(shape, lo, hi, [1.0, 3.0]), 20.0, 1e-3, 80)
    ref = oracle.tssp_real(ref, lo, hi, I.harmonic(shape, lo, hi, [2.0, 2.0]), 20.0, 1e-3, 40)
    assert rel(a, ref) < 1e-10


def test_many_time_steps_and_table_eviction():
    """More distinct dt values than the step-graph and table caches hold: the
    caches are trimmed and every call still matches the direct path."""
    shape = (32, 32, 32)
    dts = [1e-3 * (1 + 0.05 * k) for k in range(30)]
    calls = [("evolve", dt, 40) for dt in dts] + [("evolve", dts[0], 40)]
    a = run(shape, calls, timing=False)
    b = run(shape, calls, timing=True)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32s"])
@pytest.mark.parametrize("shape", [(64, 64), (32, 32, 32)])
def test_imaginary_time_graphs_are_bitwise_direct(shape, prec):
    calls = [("imag", 1e-3, n) for n in (31, 32, 33, 65, 100, 1)]
    calls += [("ground", 1e-3, 0.0, 10, 95), ("ground", 2e-3, 0.0, 100, 250),
              ("ground", 1e-3, 0.0, 7, 50), ("ground", 1e-3, 1e-5, 10, 20000)]
    say("imag graph vs direct", shape, prec)
    a, la = run(shape, calls, timing=False, prec=prec, with_log=True)
    b, lb = run(shape, calls, timing=True, prec=prec, with_log=True)
    assert np.array_equal(a, b)
    assert la == lb
    steps, energy, ok = la[-1]
    assert [x[0] for x in la[:3]] == [95, 250, 50] and not any(x[2] for x in la[:3])
    assert ok and 0 < steps < 20000 and steps % 10 == 0


def test_imaginary_time_graph_against_oracle():
    shape = (64, 64)
    lo, hi, psi0 = setup(shape)
    V = I.harmonic(shape, lo, hi, [1.0, 1.0])
    ref = oracle.tssp_imag(psi0, lo, hi, V, 20.0, 1e-3, 200)
    got = run(shape, [("imag", 1e-3, 200)], timing=False)
    assert rel(got, ref) < 1e-10
