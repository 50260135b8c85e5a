"""GPU parity of the on-chip batched class (square 2D grids held in LDS, several
steps per launch) against the single-context path, the HBM-streaming batched
path and the oracle."""
import os
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2301_08275_amd import gpe
from paper_2301_08275_amd import inputs as I

pytestmark = pytest.mark.gpu

BOX = 8.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def request(i, n, mode, prec, nsteps):
    u = I.uniform(3000 + i, 2)
    lo, hi = (-BOX, -BOX), (BOX, BOX)
    return dict(shape=(n, n), lo=lo, hi=hi, g=100.0 * u[0], mode=mode, dt=1e-3, nsteps=nsteps,
                precision=prec, trap=[1.0, 1.0 + 7.0 * u[1]], keep_state=True,
                psi0=I.noisy_gaussian((n, n), lo, hi, seed=6000 + i, amp=0.05))


def single(req):
    with gpe.Context(req["shape"], req["lo"], req["hi"], req["g"], precision=req["precision"],
                     harmonic=req["trap"]) as ctx:
        ctx.set_state(req["psi0"])
        if req["mode"] == "real":
            ctx.evolve(req["dt"], req["nsteps"])
        else:
            ctx.imag_steps(req["dt"], req["nsteps"])
        return ctx.get_state(), ctx.observables()


def serve(reqs, onchip=True, chunk=8, timeout=120):
    os.environ["GPE_SERVER_ONCHIP"] = "1" if onchip else "0"
    # every edge the kernel holds (the server's default routes up to 64 there)
    os.environ["GPE_SERVER_ONCHIP_MAX_N"] = "128"
    try:
        with gpe.Server(max_slots=8, chunk_steps=chunk) as srv:
            ids = [srv.submit(**r) for r in reqs]
            t0 = time.time()
            srv.wait_idle()
            assert time.time() - t0 < timeout
            return [srv.poll(i) for i in ids]
    finally:
        os.environ.pop("GPE_SERVER_ONCHIP", None)
        os.environ.pop("GPE_SERVER_ONCHIP_MAX_N", None)


CASES = [(8, "fp64"), (16, "fp64"), (32, "fp64"), (64, "fp64"),
         (8, "fp32"), (32, "fp32"), (64, "fp32"), (128, "fp32")]


@pytest.mark.parametrize("n,prec", CASES)
def test_onchip_matches_single_context(n, prec):
    reqs = [request(k, n, mode, prec, steps)
            for k, (mode, steps) in enumerate([("real", 37), ("imag", 50), ("real", 1),
                                               ("imag", 3), ("real", 120)])]
    say("on-chip", n, prec)
    res = serve(reqs)
    tol = 1e-12 if prec == "fp64" else 1e-5
    for r, out in zip(reqs, res):
        assert out["status"] == gpe.GPE_OK, out
        assert out["steps_done"] == r["nsteps"]
        ref, obs = single(r)
        assert rel(out["psi"], ref) < tol, (n, prec, r["mode"], r["nsteps"])
        assert abs(out["obs"]["energy"] - obs["energy"]) <= 10 * tol * abs(obs["energy"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_onchip_matches_streaming_batched_path(prec):
    reqs = [request(10 + k, 64, "real" if k % 2 else "imag", prec, 60 + 13 * k)
            for k in range(6)]
    a = serve(reqs, onchip=True)
    b = serve(reqs, onchip=False)
    tol = 1e-13 if prec == "fp64" else 1e-6
    for x, y in zip(a, b):
        assert x["status"] == y["status"] == gpe.GPE_OK
        assert rel(x["psi"], y["psi"]) < tol


def test_onchip_against_oracle():
    for mode in ("real", "imag"):
        r = request(20, 64, mode, "fp64", 80)
        out = serve([r])[0]
        V = I.harmonic(r["shape"], r["lo"], r["hi"], r["trap"])
        f = oracle.tssp_real if mode == "real" else oracle.tssp_imag
        ref = f(r["psi0"], r["lo"], r["hi"], V, r["g"], r["dt"], r["nsteps"])
        assert rel(out["psi"], ref) < 1e-10, mode


def test_onchip_beside_large_classes():
    """On-chip requests run on the side stream while a large class runs on the
    main stream; every result still matches its single-context solve."""
    small = [request(30 + k, 64, "real", "fp64", 400) for k in range(4)]
    lo3, hi3 = (-BOX,) * 3, (BOX,) * 3
    big = dict(shape=(128, 128, 128), lo=lo3, hi=hi3, g=20.0, mode="imag", dt=1e-3, nsteps=60,
               precision="fp64", trap=[1.0, 1.0, 2.0], keep_state=True,
               psi0=I.noisy_gaussian((128,) * 3, lo3, hi3, seed=77, amp=0.05))
    res = serve([big] + small)
    for r, out in zip([big] + small, res):
        assert out["status"] == gpe.GPE_OK
        ref, _ = single(r)
        assert rel(out["psi"], ref) < 1e-12


def test_onchip_identical_alone_and_in_a_mix():
    reqs = [request(40 + k, 32, "imag" if k % 3 else "real", "fp64", 90 + 7 * k)
            for k in range(7)]
    mixed = serve(reqs)
    for k in (0, 4):
        alone = serve([reqs[k]])[0]
        assert np.array_equal(alone["psi"], mixed[k]["psi"])
