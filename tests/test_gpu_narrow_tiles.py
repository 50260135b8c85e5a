"""Register-heavy passes on narrower tiles.  A 512-point strided axis tuned to
16-column tiles (1024 threads) runs its closing phase, imaginary-time passes,
spectral derivative and the server's batched slot passes on 8-column tiles,
with one row of partial sums per block of that shape.  States are bitwise
those of the run tuned to 8 columns throughout (tile width never changes the
arithmetic of a line) and match the oracle; the server's results match the
single-context ones."""
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


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32s", 2e-6), ("fp32", 3e-5)])
def test_heavy_passes_on_narrow_tiles(prec, tol):
    shape, lo, hi = (512, 8, 16), (-12.0, -3.0, -3.0), (12.0, 3.0, 3.0)
    trap = [0.5, 1.0, 1.0]
    g = 5.0
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=41, amp=0.05)
    V = I.harmonic(shape, lo, hi, trap)
    d = gpe.make_desc(shape, lo, hi, g, prec)
    out = {}
    for xw in (16, 8):
        # pass order z, y, x: the x pass closes real-time runs and opens
        # imaginary-time steps (which visit the axes in reverse)
        gpe.gpe_tuning_set(d, [xw, 8, 0], [0, 0, 0], [2, 1, 0])
        say(prec, "x tile width", xw)
        with gpe.Context(shape, lo, hi, g, precision=prec, harmonic=trap) as ctx:
            ctx.set_state(psi0)
            ctx.evolve(1e-3, 30)
            res = {"real": ctx.get_state(), "obs": ctx.observables(),
                   "spectra": ctx.spectra()}
            for meth in ("frozen", "exact"):
                ctx.set_imag_method(meth)
                ctx.set_state(psi0)
                ctx.imag_steps(1e-3, 40)
                res[meth] = ctx.get_state()
        out[xw] = res
    for key in ("real", "frozen", "exact"):
        assert np.array_equal(out[16][key], out[8][key]), key
    # observables and spectra: block partials differ with the tile shape, so
    # the sums agree to rounding
    for key in ("norm", "energy", "mu", "sigma_x"):
        a, b = out[16]["obs"][key], out[8]["obs"][key]
        assert abs(a - b) <= 1e-13 * max(1.0, abs(b)), key
    for key in ("n_k", "e_comp", "e_incomp", "e_qp"):
        a, b = out[16]["spectra"][key], out[8]["spectra"][key]
        assert float(np.max(np.abs(a - b))) <= 1e-12 * float(np.max(np.abs(b))), key
    ref = oracle.tssp_real(psi0, lo, hi, V, g, 1e-3, 30)
    assert rel(out[16]["real"], ref) < tol
    ref_o = oracle.observables(ref, lo, hi, V, g)
    assert abs(out[16]["obs"]["energy"] - ref_o["energy"]) < max(tol, 1e-12) * abs(ref_o["energy"])
    for meth in ("frozen", "exact"):
        ref_i = oracle.tssp_imag(psi0, lo, hi, V, g, 1e-3, 40, exact=(meth == "exact"))
        assert rel(out[16][meth], ref_i) < tol, meth


@pytest.mark.parametrize("prec", ["fp64", "fp32s"])
def test_server_slot_passes_on_narrow_tiles(prec):
    """2D 512 x 16 tuned to 16-column tiles with the strided axis last: the
    batched slot passes (and the norm partials of imaginary-time requests)
    run on 8-column tiles; each result matches its single-context run."""
    shape, lo, hi = (512, 16), (-12.0, -3.0), (12.0, 3.0)
    trap = [0.5, 1.0]
    d = gpe.make_desc(shape, lo, hi, 8.0, prec)
    gpe.gpe_tuning_set(d, [16, 0], [0, 0], [1, 0])
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=42, amp=0.05)
    refs = {}
    for mode in ("real", "imag"):
        with gpe.Context(shape, lo, hi, 8.0, precision=prec, harmonic=trap) as ctx:
            ctx.set_state(psi0)
            if mode == "real":
                ctx.evolve(1e-3, 50)
            else:
                ctx.imag_steps(1e-3, 50)
            refs[mode] = ctx.get_state()
    tol = 1e-12 if prec == "fp64" else 1e-6
    say("server", prec)
    with gpe.Server(max_slots=4, chunk_steps=16) as srv:
        ids = {mode: srv.submit(shape, lo, hi, 8.0, psi0, mode=mode, dt=1e-3, nsteps=50,
                                precision=prec, trap=trap, keep_state=True)
               for mode in ("real", "imag")}
        srv.wait_idle()
        for mode, rid in ids.items():
            out = srv.poll(rid)
            assert out["status"] == gpe.GPE_OK
            assert rel(out["psi"], refs[mode]) < tol, mode
