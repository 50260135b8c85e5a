"""Write the stored expected values of the full-size parity checks.

Only the CPU oracle (`oracle/`) and the seeded input generators
(`paper_2301_08275_amd/inputs.py`) run here; nothing from the GPU library.

    python tests/golden/make_oracle_goldens.py turbulence   # ~1.5 h on 8 cores
    python tests/golden/make_oracle_goldens.py ground       # ~1 h on 8 cores

turbulence_512_1000.npz -- the quantum-turbulence workload (512^3 periodic
  box [0, 2 pi)^3, V = 0, g = 1, psi = exp(i theta) with the seed-2 random
  phase, dt = 5e-4), 1000 real-time Strang steps: observables and the four
  shell spectra at steps 0, 100, ..., 1000, and psi after 1000 steps at 65536
  sites drawn with the seeded uniform generator (seed 512001).
ground_state_256.txt -- the anisotropic ground state (256^3 on [-12, 12)^3,
  trap frequencies (1, 2, 4), g = 50, Gaussian start exp(-(x^2 + 2y^2 + 4z^2)/2)
  normalised to 1, imaginary dt = 1e-3, energy every 10 steps, stop at the
  first check whose energy differs from the previous one by less than 1e-10):
  the stopping step, every check's energy and the final observables.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2301_08275_amd import inputs as I  # noqa: E402

SPEC_KEYS = ("n_k", "e_comp", "e_incomp", "e_qp")


def say(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


def sample_sites(total, count=65536, seed=512001):
    """Distinct flat site indices, sorted (seeded uniform draws)."""
    u = I.uniform(seed, 4 * count)
    idx = np.unique((u * total).astype(np.int64))
    rng_order = np.argsort(I.uniform(seed + 1, idx.size))
    return np.sort(idx[rng_order[:count]])


def turbulence(path, n=512, steps=1000, every=100):
    lo, hi = (0.0,) * 3, (2 * np.pi,) * 3
    say("phase field %d^3" % n)
    psi = I.phase_field(n, seed=2)
    obs, spec = [], {k: [] for k in SPEC_KEYS}
    t = 0
    while True:
        o = oracle.observables(psi, lo, hi, None, 1.0)
        s = oracle.spectra(psi, lo, hi)
        obs.append([o[k] for k in oracle.OBS_KEYS])
        for k in SPEC_KEYS:
            spec[k].append(s[k])
        say("step %d: norm %.17g energy %.17g" % (t, o["norm"], o["energy"]))
        if t == steps:
            break
        psi = oracle.tssp_real(psi, lo, hi, None, 1.0, 5e-4, every)
        t += every
    idx = sample_sites(psi.size)
    np.savez(path, steps=np.arange(0, steps + 1, every), obs=np.array(obs),
             obs_keys=np.array(oracle.OBS_KEYS), sites=idx.astype(np.int32),
             psi=psi.ravel()[idx], dk=s["dk"],
             **{k: np.array(v) for k, v in spec.items()})
    say("wrote", path)


def ground(path, n=256, g=50.0, dt=1e-3, tol=1e-10, check=10):
    shape, lo, hi = (n,) * 3, (-12.0,) * 3, (12.0,) * 3
    V = I.harmonic(shape, lo, hi, [1.0, 2.0, 4.0])
    psi = I.gaussian(shape, lo, hi, widths=[1.0, 2.0, 4.0])
    e_prev = oracle.observables(psi, lo, hi, V, g)["energy"]
    energies, t = [e_prev], 0
    while True:
        psi = oracle.tssp_imag(psi, lo, hi, V, g, dt, check)
        t += check
        e = oracle.observables(psi, lo, hi, V, g)["energy"]
        energies.append(e)
        if t % 500 == 0:
            say("step %d energy %.17g change %.3g" % (t, e, e - e_prev))
        if abs(e - e_prev) < tol:
            break
        e_prev = e
    o = oracle.observables(psi, lo, hi, V, g)
    with open(path, "w") as f:
        f.write("# Anisotropic ground state by the CPU oracle (written by make_oracle_goldens.py):\n"
                "# 256^3 on [-12,12)^3, trap (1, 2, 4), g = 50, Gaussian start, imaginary\n"
                "# dt = 1e-3 with renormalisation to 1 each step, energy every 10 steps, stop at\n"
                "# the first check whose energy differs from the previous one by < 1e-10.\n")
        f.write("steps_done %d\n" % t)
        for k in oracle.OBS_KEYS:
            f.write("%s %.17g\n" % (k, o[k]))
        f.write("# check energies (step 0, 10, 20, ...)\n")
        for e in energies:
            f.write("E %.17g\n" % e)
    say("wrote", path, "steps", t)


if __name__ == "__main__":
    oracle.set_threads(int(os.environ.get("ORACLE_THREADS", "0")))
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("turbulence", "all"):
        turbulence(os.path.join(HERE, "turbulence_512_1000.npz"))
    if what in ("ground", "all"):
        ground(os.path.join(HERE, "ground_state_256.txt"))
