"""Small single-context grids replay their steady-state real-time steps from a
HIP graph.  The graph holds the same launches as the direct path (which runs
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


def run(shape, calls, timing, prec="fp64", trap=None):
    lo, hi, psi0 = setup(shape)
    trap = trap or [1.0] * len(shape)
    with gpe.Context(shape, lo, hi, 20.0, precision=prec, harmonic=trap) as ctx:
        if timing:
            ctx.timing(True)
        ctx.set_state(psi0)
        for call in calls:
            if call[0] == "evolve":
                ctx.evolve(call[1], call[2])
            else:
                ctx.set_potential(harmonic=call[1])
        return ctx.get_state()


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
