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


@pytest.mark.parametrize("shape,lo,hi,prec", [
    ((32, 64, 16), (-6.0, -7.0, -3.0), (6.0, 7.0, 3.0), "fp64"),   # unequal lengths
    ((32, 32, 32), (-5.0,) * 3, (5.0,) * 3, "fp64"),                 # integer shells
    ((64, 128), (-6.0, -8.0), (6.0, 8.0), "fp64"),
    ((256,), (-10.0,), (10.0,), "fp64"),
    ((32, 32, 32), (-5.0,) * 3, (5.0,) * 3, "fp32s"),
])
def test_observables_with_spectra_parity(shape, lo, hi, prec):
    """Observables taken in the spectra sweep (real-space sums in the first
    forward pass, E_kin from the shell kernel by Parseval's identity on the
    whole grid) against the oracle and against a call without spectra."""
    w = [1.0, 2.0, 4.0][:len(shape)]
    V = I.harmonic(shape, lo, hi, w)
    psi = I.noisy_gaussian(shape, lo, hi, seed=4, amp=0.2)
    ref = oracle.observables(psi, lo, hi, V, 7.5)
    say("observables with spectra", shape, prec)
    with gpe.Context(shape, lo, hi, 7.5, harmonic=w, precision=prec) as ctx:
        ctx.set_state(psi)
        _, fused = ctx.spectra(with_obs=True)
        alone = ctx.observables()
    tol = 1e-12 if prec == "fp64" else 1e-6
    # (with FP32 storage the full transform behind E_kin is stored in FP32
    # after each axis, the per-axis passes of a call without spectra are not)
    same = 1e-13 if prec == "fp64" else 1e-8
    for k in gpe.OBS_KEYS:
        scale = max(1.0, abs(ref[k]))
        assert abs(fused[k] - ref[k]) <= tol * scale, (k, fused[k], ref[k])
        assert abs(fused[k] - alone[k]) <= same * scale, (k, fused[k], alone[k])


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


SPECTRA_CASES = [
    ((32, 32, 32), (0.0,) * 3, (2 * np.pi,) * 3),
    ((16, 8, 32), (0.0, -1.0, 0.0), (4.0, 1.0, 3.0)),
    ((64, 32), (-3.0, -2.0), (3.0, 2.0)),
    ((32, 32), (-3.0, -3.0), (3.0, 3.0)),     # 2D with integer shells
    ((8, 8, 8), (0.0,) * 3, (2 * np.pi,) * 3),
    # last axis of 128 or more: a wavefront's sites lie in one half-row
    ((8, 16, 128), (0.0,) * 3, (1.0, 1.5, 6.0)),
    ((16, 256), (-3.0, -4.0), (3.0, 4.0)),
]


@pytest.mark.parametrize("shape,lo,hi", SPECTRA_CASES)
def test_spectra_parity(shape, lo, hi):
    say("spectra", shape)
    rng = np.random.default_rng(5)
    psi = (1.2 + 0.3 * rng.standard_normal(shape)) * np.exp(1j * rng.standard_normal(shape))
    ref = oracle.spectra(psi, lo, hi)
    with gpe.Context(shape, lo, hi, 1.0) as ctx:
        ctx.set_state(psi)
        got = ctx.spectra()
    assert abs(got["dk"] - ref["dk"]) < 1e-15
    for key in ("n_k", "e_comp", "e_incomp", "e_qp"):
        scale = max(1e-300, float(np.sum(ref[key])))
        assert np.abs(got[key] - ref[key]).max() <= 1e-12 * scale, key


@pytest.mark.parametrize("shape,lo,hi,prec", [
    ((128, 128, 128), (0.0,) * 3, (2 * np.pi,) * 3, "fp64"),   # a wavefront in one half-row
    ((16, 32, 64), (0.0,) * 3, (1.0, 2.0, 3.0), "fp64"),       # wavefronts span rows
    ((64, 64), (-4.0, -4.0), (4.0, 4.0), "fp64"),
    ((128, 128, 128), (0.0,) * 3, (2 * np.pi,) * 3, "fp32s"),
])
def test_spectra_are_bitwise_reproducible(shape, lo, hi, prec):
    """Every shell sum is taken in a fixed order: the same state gives the same
    spectra bit for bit, call after call and context after context."""
    rng = np.random.default_rng(11)
    psi = (1.0 + 0.4 * rng.standard_normal(shape)) * np.exp(1j * rng.standard_normal(shape))
    runs = []
    for _ in range(2):
        with gpe.Context(shape, lo, hi, 1.0, precision=prec) as ctx:
            ctx.set_state(psi)
            runs.append(ctx.spectra())
            runs.append(ctx.spectra())
    for r in runs[1:]:
        for key in ("n_k", "e_comp", "e_incomp", "e_qp"):
            assert np.array_equal(r[key], runs[0][key]), key


def test_spectra_cfg2_initial_state():
    """exp(i theta) with a smooth random phase: irrotational and without
    quantum pressure, and the shell sums agree with the oracle."""
    n = 64
    lo, hi = (0.0,) * 3, (2 * np.pi,) * 3
    psi = I.phase_field(n, seed=2)
    ref = oracle.spectra(psi, lo, hi)
    with gpe.Context((n, n, n), lo, hi, 1.0, norm_target=(2 * np.pi) ** 3) as ctx:
        ctx.set_state(psi)
        got = ctx.spectra()
        obs = ctx.observables()
    ek = got["e_comp"].sum() + got["e_incomp"].sum() + got["e_qp"].sum()
    assert abs(ek / obs["e_kin"] - 1) < 1e-12
    assert got["e_incomp"].sum() < 1e-10 * ek
    for key in ("n_k", "e_comp", "e_incomp", "e_qp"):
        assert np.abs(got[key] - ref[key]).max() <= 1e-12 * float(np.sum(ref["e_comp"]) + np.sum(ref["n_k"]))


# ------------------------------------------------------------------ FP32 ---

def test_fp32_transform():
    shape = (64, 32, 128)
    x = random_state(shape, 3)
    with gpe.Context(shape, (0,) * 3, (1,) * 3, 0.0, precision="fp32") as ctx:
        ctx.set_state(x)
        ctx.transform()
        got = ctx.get_state()
    assert rel(got, oracle.fft(x)) < 2e-6


# The FP32 bars against the FP64 oracle: rel L2 <= 1e-4, norm drift <= 1e-6,
# energy rel error <= 1e-5.  "fp32s" (FP32 state in HBM, FP64 arithmetic in
# every pass) is the FP32 form the benchmark reports; "fp32" (FP32 state and
# FP32 FFT) is held to the same bars and marked where it misses them.
FP32_FFT_NORM = pytest.mark.xfail(
    reason="FP32 FFT arithmetic: the rounding of the FP32 butterflies drifts the norm "
           "~3.4e-6 per 1000 steps on the localised 2D trap state (bar 1e-6)", strict=False)
_ORACLE_TURB = {}


def oracle_turbulence(n, steps):
    """The oracle's turbulence run, computed once per size for every form."""
    if (n, steps) not in _ORACLE_TURB:
        lo, hi = (0.0,) * 3, (2 * np.pi,) * 3
        psi0 = I.phase_field(n, seed=2)
        ref = oracle.tssp_real(psi0, lo, hi, None, 1.0, 5e-4, steps)
        _ORACLE_TURB[(n, steps)] = (psi0, ref, oracle.observables(ref, lo, hi, None, 1.0))
    return _ORACLE_TURB[(n, steps)]


@pytest.mark.parametrize("prec", ["fp32s", "fp32"])
@pytest.mark.parametrize("n", [64, 128])
def test_fp32_turbulence_1000_steps(n, prec):
    """The turbulence workload at reduced size: each FP32 form against the
    FP64 oracle after 1000 steps at the FP32 bars."""
    say("fp32 turbulence", n, prec)
    lo, hi = (0.0,) * 3, (2 * np.pi,) * 3
    psi0, ref, o_ref = oracle_turbulence(n, 1000)
    with gpe.Context((n, n, n), lo, hi, 1.0, precision=prec,
                     norm_target=(2 * np.pi) ** 3) as ctx:
        ctx.set_state(psi0)
        n0 = ctx.observables()["norm"]
        ctx.evolve(5e-4, 1000)
        got = ctx.get_state()
        o = ctx.observables()
    err, dn = rel(got, ref), abs(o["norm"] - n0) / n0
    de = abs(o["energy"] - o_ref["energy"]) / abs(o_ref["energy"])
    say("  rel L2 %.3g, norm drift %.3g, energy %.3g" % (err, dn, de))
    assert err < 1e-4
    assert dn < 1e-6
    assert de < 1e-5


@pytest.mark.parametrize("prec", ["fp32s", pytest.param("fp32", marks=FP32_FFT_NORM)])
def test_fp32_cfg0_1000_steps(prec):
    """Each FP32 form on the 2D trap workload, 1000 steps, at the FP32 bars
    against the FP64 oracle."""
    shape, lo, hi, V, psi0 = cfg0()
    ref = oracle.tssp_real(psi0, lo, hi, V, 10.0, 1e-3, 1000)
    o_ref = oracle.observables(ref, lo, hi, V, 10.0)
    with gpe.Context(shape, lo, hi, 10.0, harmonic=[1.0, 1.0], precision=prec) as ctx:
        ctx.set_state(psi0)
        n0 = ctx.observables()["norm"]
        ctx.evolve(1e-3, 1000)
        got = ctx.get_state()
        o = ctx.observables()
    err, dn = rel(got, ref), abs(o["norm"] - n0) / n0
    de = abs(o["energy"] - o_ref["energy"]) / abs(o_ref["energy"])
    say("2D trap %s: rel L2 %.3g, norm drift %.3g, energy %.3g" % (prec, err, dn, de))
    assert err < 1e-4
    assert de < 1e-5
    assert dn < 1e-6


@pytest.mark.parametrize("prec", ["fp32s", "fp32"])
def test_fp32_ground_state_matches_table(prec):
    """A Table 1 row (2D, g = 62.742) in each FP32 form: the FP64 ground state
    (stop rule at 1e-10) sets the step count; the FP32 run takes the same
    number of imaginary-time steps (an energy stop rule at FP64 tolerances
    would fire on FP32 rounding noise).  mu and r_rms within 1e-5 of the FP64
    run; the FP64 run within 1e-3 of the printed values (the tolerance of the
    oracle's own Table 1 pin; this grid is coarser than the oracle's)."""
    shape, lo, hi = (64, 64), (-12.0, -12.0), (12.0, 12.0)
    with gpe.Context(shape, lo, hi, 62.742, harmonic=[1.0, 1.0]) as ctx:
        ctx.set_state(I.gaussian(shape, lo, hi))
        steps, E, conv = ctx.ground_state(1e-3, tol=1e-10, check_every=10)
        o64 = ctx.observables()
    assert conv
    assert abs(o64["mu"] / 4.61136 - 1) < 1e-3
    assert abs(o64["r_rms"] / 1.78722 - 1) < 1e-3
    with gpe.Context(shape, lo, hi, 62.742, harmonic=[1.0, 1.0], precision=prec) as ctx:
        ctx.set_state(I.gaussian(shape, lo, hi))
        ctx.imag_steps(1e-3, steps)
        o = ctx.observables()
    say("%s ground state after %d steps: mu %.9g (fp64 %.9g), r_rms %.9g (fp64 %.9g)"
        % (prec, steps, o["mu"], o64["mu"], o["r_rms"], o64["r_rms"]))
    assert abs(o["mu"] / o64["mu"] - 1) < 1e-5
    assert abs(o["r_rms"] / o64["r_rms"] - 1) < 1e-5


# ----------------------------------------- FP32 state, FP64 arithmetic ---
# One FP32 rounding per pass (the store), so the bars are far tighter than the
# FP32 form's: rounding noise grows like sqrt(passes) * 2^-25 ~ 1e-6 after
# 3000 passes, and round-to-nearest leaves no bias in the norm.

def test_fp32s_transform():
    shape = (64, 32, 128)
    x = random_state(shape, 3)
    with gpe.Context(shape, (0,) * 3, (1,) * 3, 0.0, precision="fp32s") as ctx:
        ctx.set_state(x)
        ctx.transform()
        got = ctx.get_state()
    assert rel(got, oracle.fft(x)) < 2e-7


@pytest.mark.parametrize("n", [64, 128])
def test_fp32s_turbulence(n):
    say("fp32s turbulence", n)
    lo, hi = (0.0,) * 3, (2 * np.pi,) * 3
    psi0 = I.phase_field(n, seed=2)
    steps = 1000 if n == 64 else 200
    ref = oracle.tssp_real(psi0, lo, hi, None, 1.0, 5e-4, steps)
    o_ref = oracle.observables(ref, lo, hi, None, 1.0)
    with gpe.Context((n, n, n), lo, hi, 1.0, precision="fp32s",
                     norm_target=(2 * np.pi) ** 3) as ctx:
        ctx.set_state(psi0)
        n0 = ctx.observables()["norm"]
        ctx.evolve(5e-4, steps)
        got = ctx.get_state()
        o = ctx.observables()
    assert rel(got, ref) < 1e-5
    assert abs(o["norm"] - n0) / n0 < 1e-8
    assert abs(o["energy"] - o_ref["energy"]) / abs(o_ref["energy"]) < 1e-7


def test_fp32s_cfg0_1000_steps():
    """The 2D trap workload: the state is localised (few sites carry the norm),
    so the random walk of the per-pass FP32 rounding in the norm is larger than
    on the turbulence state (measured 2.4e-8 after 1000 steps): bar 1e-7,
    ten times inside the FP32 form's 1e-6."""
    shape, lo, hi, V, psi0 = cfg0()
    ref = oracle.tssp_real(psi0, lo, hi, V, 10.0, 1e-3, 1000)
    with gpe.Context(shape, lo, hi, 10.0, harmonic=[1.0, 1.0], precision="fp32s") as ctx:
        ctx.set_state(psi0)
        ctx.evolve(1e-3, 1000)
        got = ctx.get_state()
        o = ctx.observables()
    assert rel(got, ref) < 1e-5
    assert abs(o["norm"] - 1) < 1e-7


def test_fp32s_ground_state_matches_fp64():
    """A Table 1 setup (2D, g = 62.742) for a fixed 4000 imaginary-time steps
    in FP32 state and in FP64 (a stop rule would compare convergence, not
    precision).  Slowly decaying modes keep the per-pass FP32 roundings for
    ~1/(gap dt) steps, a random walk of ~sqrt(8000) * 3e-8 (measured 4.1e-6):
    bars 2e-5 on the state and 1e-5 on mu and r_rms, inside the FP32 form's
    1e-4."""
    shape, lo, hi = (64, 64), (-12.0, -12.0), (12.0, 12.0)
    out = {}
    for prec in ("fp64", "fp32s"):
        with gpe.Context(shape, lo, hi, 62.742, harmonic=[1.0, 1.0], precision=prec) as ctx:
            ctx.set_state(I.gaussian(shape, lo, hi))
            ctx.imag_steps(1e-3, 4000)
            out[prec] = (ctx.get_state(), ctx.observables())
    (s64, o64), (s32, o32) = out["fp64"], out["fp32s"]
    say("fp32s ground state: rel %.3g, mu %.3g, r_rms %.3g" % (
        rel(s32, s64), o32["mu"] / o64["mu"] - 1, o32["r_rms"] / o64["r_rms"] - 1))
    assert rel(s32, s64) < 2e-5
    assert abs(o32["mu"] / o64["mu"] - 1) < 1e-5
    assert abs(o32["r_rms"] / o64["r_rms"] - 1) < 1e-5
    assert abs(o64["mu"] / 4.61136 - 1) < 2e-4


def test_fp32s_spectra_close_to_fp64():
    lo, hi = (0.0,) * 3, (2 * np.pi,) * 3
    psi0 = I.phase_field(64, seed=2)
    out = {}
    for prec in ("fp64", "fp32s"):
        with gpe.Context((64,) * 3, lo, hi, 1.0, precision=prec,
                         norm_target=(2 * np.pi) ** 3) as ctx:
            ctx.set_state(psi0)
            ctx.evolve(5e-4, 100)
            out[prec] = ctx.spectra()
    for key in ("n_k", "e_comp", "e_incomp", "e_qp"):
        a, b = out["fp32s"][key], out["fp64"][key]
        assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(b), key


# ------------------------------------------------ observable time series ---

@pytest.mark.parametrize("nsteps,every", [(100, 10), (95, 10), (7, 20)])
def test_evolve_record_matches_chunked_calls(nsteps, every):
    """gpe_evolve_record equals gpe_evolve in chunks of `every` followed by
    gpe_observables, record for record and in the final state (bitwise)."""
    shape, lo, hi, V, psi0 = cfg0()
    with gpe.Context(shape, lo, hi, 10.0, harmonic=[1.0, 1.0]) as ctx:
        ctx.set_state(psi0)
        series = ctx.evolve_record(1e-3, nsteps, every)
        end = ctx.get_state()
    ref, done = [], 0
    with gpe.Context(shape, lo, hi, 10.0, harmonic=[1.0, 1.0]) as ctx:
        ctx.set_state(psi0)
        while done < nsteps:
            n = min(every, nsteps - done)
            ctx.evolve(1e-3, n)
            ref.append(ctx.observables())
            done += n
        end_ref = ctx.get_state()
    assert len(series) == len(ref) == -(-nsteps // every)
    for a, b in zip(series, ref):
        assert a == b
    assert np.array_equal(end, end_ref)


def test_evolve_record_time_series_against_oracle():
    """The 3D anisotropic setup: sigma(t) and E(t) every 10 steps against the
    oracle's observables of its own chunked run."""
    shape, lo, hi = (32, 32, 32), (-6.0,) * 3, (6.0,) * 3
    trap = [1.0, 2.0, 4.0]
    V = I.harmonic(shape, lo, hi, trap)
    psi = I.noisy_gaussian(shape, lo, hi, seed=12)
    with gpe.Context(shape, lo, hi, 0.1, harmonic=trap) as ctx:
        ctx.set_state(psi)
        series = ctx.evolve_record(1e-3, 50, 10)
    for rec in series:
        psi = oracle.tssp_real(psi, lo, hi, V, 0.1, 1e-3, 10)
        o = oracle.observables(psi, lo, hi, V, 0.1)
        for key in ("norm", "energy", "sigma_x", "sigma_y", "sigma_z", "r_rms"):
            assert abs(rec[key] - o[key]) <= 1e-11 * abs(o[key]), key


def test_evolve_record_rejects_small_capacity():
    shape, lo, hi, V, psi0 = cfg0()
    with gpe.Context(shape, lo, hi, 10.0, harmonic=[1.0, 1.0]) as ctx:
        obs = (gpe.gpe_obs * 2)()
        count = gpe._I64(0)
        st = gpe.load_library().gpe_evolve_record(ctx._ctx, 1e-3, 30, 10, obs, 2,
                                                   gpe.ctypes.byref(count))
        assert st == gpe.GPE_EINVAL and count.value == 0


@pytest.mark.parametrize("shape", [(8, 16, 32), (16, 8, 64)])
def test_reductions_with_blocks_smaller_than_a_wavefront(shape):
    """Short strided axes run workgroups of 8-32 threads: observables and the
    imaginary-time renormalisation sums still match the oracle."""
    lo, hi = (-4.0,) * 3, (4.0,) * 3
    trap = [2.0, 1.0, 1.5]
    V = I.harmonic(shape, lo, hi, trap)
    psi = I.noisy_gaussian(shape, lo, hi, seed=21)
    o_ref = oracle.observables(psi, lo, hi, V, 3.0)
    ref = oracle.tssp_imag(psi, lo, hi, V, 3.0, 1e-3, 10)
    with gpe.Context(shape, lo, hi, 3.0, harmonic=trap) as ctx:
        ctx.set_state(psi)
        o = ctx.observables()
        ctx.imag_steps(1e-3, 10)
        got = ctx.get_state()
    for key in ("norm", "energy", "e_kin", "sigma_x", "sigma_y", "sigma_z"):
        assert abs(o[key] - o_ref[key]) <= 1e-12 * abs(o_ref[key]), key
    assert rel(got, ref) < 1e-12
