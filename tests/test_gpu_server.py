"""GPU tests of the serving scheduler (gpe_server_* calls).

Every request's result must match the single-context path and the oracle, be
bitwise identical whether it ran alone or in a mix, and the scheduler must
respect the HBM budget, cancellation and per-request failure isolation.
"""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2301_08275_amd import gpe
from paper_2301_08275_amd import inputs as I

pytestmark = pytest.mark.gpu

BOX = 8.0


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_req(i, shape, mode, prec="fp64", nsteps=None):
    """A request of the serving mix: trap anisotropy, g and noise seeded by i."""
    dim = len(shape)
    u = I.uniform(1000 + i, 3)
    a = 1.0 + 7.0 * u[0]
    g = 100.0 * u[1]
    trap = [1.0, a] if dim == 2 else [1.0, 1.0, a]
    lo, hi = (-BOX,) * dim, (BOX,) * dim
    psi0 = I.noisy_gaussian(shape, lo, hi, seed=5000 + i, amp=0.05)
    steps = nsteps if nsteps is not None else 20 + int(60 * u[2])
    return dict(shape=shape, lo=lo, hi=hi, g=g, psi0=psi0, mode=mode, dt=1e-3, nsteps=steps,
                precision=prec, trap=trap, keep_state=True)


def solve_alone_ctx(req):
    """The same request through the single-context API."""
    with gpe.Context(req["shape"], req["lo"], req["hi"], req["g"], precision=req["precision"],
                     harmonic=req["trap"]) as ctx:
        ctx.set_state(req["psi0"])
        if req["mode"] == "real":
            ctx.evolve(req["dt"], req["nsteps"])
        else:
            ctx.imag_steps(req["dt"], req["nsteps"])
        return ctx.get_state()


def run_all(srv, reqs, timeout=120):
    ids = [srv.submit(**r) for r in reqs]
    t0 = time.time()
    out = {}
    while len(out) < len(ids):
        for rid in ids:
            if rid not in out:
                res = srv.poll(rid)
                if res is not None:
                    out[rid] = res
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.002)
    return [out[i] for i in ids]


def mix():
    shapes2 = [(64, 64), (128, 128), (64, 128)]
    shapes3 = [(32, 32, 32), (64, 32, 16)]
    reqs = []
    for i in range(18):
        shape = shapes2[i % 3] if i % 5 != 4 else shapes3[(i // 5) % 2]
        mode = "real" if i % 2 == 0 else "imag"
        prec = "fp32" if i % 7 == 3 else ("fp32s" if i % 7 == 5 else "fp64")
        reqs.append(make_req(i, shape, mode, prec))
    return reqs


def test_server_results_match_single_context_and_oracle():
    reqs = mix()
    say("server mix of", len(reqs))
    with gpe.Server(max_slots=8, chunk_steps=8) as srv:
        res = run_all(srv, reqs)
        st = srv.stats()
    assert st["completed"] == len(reqs)
    for r, out in zip(reqs, res):
        assert out["status"] == gpe.GPE_OK, out
        assert out["steps_done"] == r["nsteps"]
        ref = solve_alone_ctx(r)
        tol = {"fp64": 1e-12, "fp32": 1e-5, "fp32s": 1e-6}[r["precision"]]
        assert rel(out["psi"], ref) < tol, (r["shape"], r["mode"], r["precision"])
    # every request against the oracle: 2D and 3D batched classes (on-chip,
    # graph replay), real and imaginary time, FP64 at 1e-10 and the FP32 forms
    # at the FP32 bar (rel L2 1e-4 against the FP64 oracle)
    for r, out in zip(reqs, res):
        ref, o = oracle_solve(r)
        bar = 1e-10 if r["precision"] == "fp64" else 1e-4
        err = rel(out["psi"], ref)
        assert err < bar, (r["shape"], r["mode"], r["precision"], err)
        ebar = 1e-9 if r["precision"] == "fp64" else 1e-5
        assert abs(out["obs"]["energy"] - o["energy"]) < ebar * abs(o["energy"])


def oracle_solve(r):
    V = I.harmonic(r["shape"], r["lo"], r["hi"], r["trap"])
    if r["mode"] == "real":
        ref = oracle.tssp_real(r["psi0"], r["lo"], r["hi"], V, r["g"], r["dt"], r["nsteps"])
    else:
        ref = oracle.tssp_imag(r["psi0"], r["lo"], r["hi"], V, r["g"], r["dt"], r["nsteps"])
    return ref, oracle.observables(ref, r["lo"], r["hi"], V, r["g"])


def test_large_requests_match_the_oracle():
    """256^3 requests (a class large enough for direct launches over its owned
    slots): FP64 real time and FP32-state imaginary time against the oracle,
    with a small request running beside them."""
    reqs = [make_req(40, (256, 256, 256), "real", "fp64", nsteps=12),
            make_req(41, (256, 256, 256), "imag", "fp32s", nsteps=12),
            make_req(42, (64, 64), "real", "fp64", nsteps=30)]
    say("server: two 256^3 requests and a small one")
    with gpe.Server(max_slots=4, chunk_steps=4) as srv:
        res = run_all(srv, reqs, timeout=300)
    for r, out in zip(reqs, res):
        assert out["status"] == gpe.GPE_OK and out["steps_done"] == r["nsteps"]
        ref, o = oracle_solve(r)
        err = rel(out["psi"], ref)
        say("  %s %s %s: rel L2 vs oracle %.3g" % (r["shape"], r["mode"], r["precision"], err))
        assert err < (1e-10 if r["precision"] == "fp64" else 1e-4)


def test_heavy_requests_are_first_come_first_served():
    """Requests of 2^23 points or more run one at a time in arrival order, and
    lighter requests queued behind a waiting heavy one start beside the
    running heavy one instead of waiting."""
    h1 = make_req(50, (256, 256, 128), "real", nsteps=300)
    h2 = make_req(51, (256, 256, 128), "real", nsteps=300)
    light = make_req(52, (64, 64), "real", nsteps=300)
    with gpe.Server(max_slots=4, chunk_steps=8) as srv:
        ids = [srv.submit(**h1), srv.submit(**h2), srv.submit(**light)]
        srv.wait_idle()
        r1, r2, rl = (srv.poll(i) for i in ids)
    assert all(r["status"] == gpe.GPE_OK for r in (r1, r2, rl))
    say("heavy 1 %.3f-%.3f, heavy 2 %.3f-%.3f, light %.3f-%.3f"
        % (r1["t_start"], r1["t_done"], r2["t_start"], r2["t_done"],
           rl["t_start"], rl["t_done"]))
    assert r2["t_start"] >= r1["t_done"] - 1e-3    # heavy 2 waited for heavy 1 alone
    assert rl["t_start"] < r1["t_done"]             # the light one passed heavy 2
    assert rl["t_done"] < r2["t_start"] + 1e-3


def test_heavy_stream_is_bitwise_neutral(monkeypatch):
    """A heavy request on the stream of its own (concurrent with the lighter
    classes) gives the same bits as when it takes its quanta on the main
    stream, and so do the lighter requests beside it."""
    reqs = [make_req(60, (256, 256, 128), "imag", nsteps=40),
            make_req(61, (128, 128), "real", nsteps=200),
            make_req(62, (64, 64, 64), "imag", "fp32s", nsteps=150),
            make_req(63, (64, 64), "real", "fp32", nsteps=300)]
    out = {}
    for beside in ("1", "0"):
        monkeypatch.setenv("GPE_SERVER_HEAVY_BESIDE", beside)
        say("heavy beside", beside)
        with gpe.Server(max_slots=4, chunk_steps=8) as srv:
            out[beside] = run_all(srv, reqs, timeout=300)
    for r, a, b in zip(reqs, out["1"], out["0"]):
        assert a["status"] == b["status"] == gpe.GPE_OK
        assert np.array_equal(a["psi"], b["psi"]), r["shape"]
        assert a["obs"]["energy"] == b["obs"]["energy"]


def test_result_is_identical_alone_and_in_the_mix():
    reqs = mix()
    probe = [reqs[1], reqs[4], reqs[3]]
    with gpe.Server(max_slots=8, chunk_steps=8) as srv:
        alone = [run_all(srv, [p])[0] for p in probe]
    with gpe.Server(max_slots=8, chunk_steps=8) as srv:
        mixed = run_all(srv, reqs)
    for p, a in zip(probe, alone):
        m = mixed[reqs.index(p)]
        assert np.array_equal(a["psi"], m["psi"])
        assert a["obs"]["energy"] == m["obs"]["energy"]


def max_overlap(res):
    """Largest number of requests running at the same instant."""
    ev = sorted([(r["t_start"], 1) for r in res] + [(r["t_done"], -1) for r in res],
                key=lambda e: (e[0], e[1]))
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return best


@pytest.mark.parametrize("fit", [1, 2])
def test_admission_respects_budget(fit):
    """A budget with room for the class and `fit` running requests: every
    request still finishes, never more than `fit` run at once, and the bytes
    held stay within the budget."""
    reqs = [make_req(i, (128, 128), "real", nsteps=40) for i in range(6)]
    cls_b, slot_b = gpe.gpe_request_bytes(gpe.make_desc((128, 128), -BOX, BOX, 1.0), 8)
    budget = cls_b + fit * slot_b + slot_b // 2
    with gpe.Server(budget=budget, max_slots=8, chunk_steps=4) as srv:
        res = run_all(srv, reqs)
        assert srv.stats()["bytes_in_use"] <= budget
    assert all(r["status"] == gpe.GPE_OK for r in res)
    assert max_overlap(res) <= fit


def test_max_active_one_is_one_at_a_time():
    reqs = [make_req(i, (64, 64), "real", nsteps=30) for i in range(5)]
    with gpe.Server(max_slots=8, max_active=1, chunk_steps=4) as srv:
        res = run_all(srv, reqs)
    assert max_overlap(res) == 1
    assert [r["t_start"] for r in res] == sorted(r["t_start"] for r in res)


def test_cancel_and_failure_isolation():
    good = make_req(1, (64, 64), "real", nsteps=50)
    bad = make_req(2, (64, 64), "real", nsteps=50)
    bad["psi0"] = bad["psi0"].copy()
    bad["psi0"][3, 5] = np.nan
    long = make_req(3, (128, 128), "real", nsteps=200000)
    with gpe.Server(max_slots=8, chunk_steps=8) as srv:
        lid = srv.submit(**long)
        ids = [srv.submit(**good), srv.submit(**bad)]
        time.sleep(0.05)
        srv.cancel(lid)
        srv.wait_idle()
        rl = srv.poll(lid)
        rg, rb = srv.poll(ids[0]), srv.poll(ids[1])
    assert rl["status"] == gpe.GPE_ECANCELED
    assert rb["status"] == gpe.GPE_ENONFINITE
    assert rg["status"] == gpe.GPE_OK
    assert rel(rg["psi"], solve_alone_ctx(good)) < 1e-12


def test_oversized_request_is_refused():
    with gpe.Server(budget=1 << 20, max_slots=2) as srv:
        with pytest.raises(gpe.GpeError) as e:
            srv.submit(**make_req(0, (256, 256), "real"))
        assert e.value.status == gpe.GPE_ENOMEM


def test_release_drops_finished_records():
    long = make_req(4, (128, 128), "real", nsteps=200000)
    short = make_req(5, (64, 64), "real", nsteps=20)
    with gpe.Server(max_slots=4, chunk_steps=4) as srv:
        lid = srv.submit(**long)
        sid = srv.submit(**short)
        while srv.poll(sid) is None:
            time.sleep(0.002)
        assert srv.release(lid) == gpe.GPE_EBUSY      # still running
        assert srv.release(sid) == gpe.GPE_OK
        with pytest.raises(gpe.GpeError):
            srv.poll(sid)                              # the record is gone
        assert srv.release(sid) == gpe.GPE_EINVAL
        srv.cancel(lid)
        srv.wait_idle()
        assert srv.poll(lid)["status"] == gpe.GPE_ECANCELED
        assert srv.release(lid) == gpe.GPE_OK


def test_stress_mixed_requests_with_cancellations():
    """120 small requests of every kind (2D/3D, real/imaginary, three
    precisions, on-chip and streaming classes), a tight budget and random
    cancellations: every request ends with a definite status, the budget
    holds, and the uncancelled results match the single-context path."""
    rng = np.random.default_rng(7)
    shapes = [(32, 32), (64, 64), (128, 128), (64, 32), (16, 16, 16), (32, 32, 16)]
    precs = ["fp64", "fp32", "fp32s"]
    reqs = []
    for i in range(120):
        shape = shapes[i % len(shapes)]
        mode = "imag" if i % 3 == 0 else "real"
        r = make_req(100 + i, shape, mode, precs[i % 3], nsteps=int(rng.integers(1, 60)))
        reqs.append(r)
    cls = {}
    for r in reqs:
        key = (r["shape"], r["precision"], r["mode"])
        if key not in cls:
            cls[key] = gpe.gpe_request_bytes(gpe.make_desc(r["shape"], -BOX, BOX, 1.0,
                                                           r["precision"]), 4)
    budget = sum(c for c, s in cls.values()) // 2 + 6 * max(s for c, s in cls.values())
    say("stress: budget %d bytes" % budget)
    with gpe.Server(budget=budget, max_slots=4, chunk_steps=4) as srv:
        ids = [srv.submit(**r) for r in reqs]
        cancel = set(int(k) for k in rng.choice(len(ids), size=15, replace=False))
        for k in sorted(cancel):
            time.sleep(0.001)
            srv.cancel(ids[k])
        srv.wait_idle()
        st = srv.stats()
        res = [srv.poll(i) for i in ids]
        assert st["bytes_in_use"] <= budget
    assert st["completed"] == len(reqs)
    for k, (r, out) in enumerate(zip(reqs, res)):
        if k in cancel:
            assert out["status"] in (gpe.GPE_OK, gpe.GPE_ECANCELED)
        else:
            assert out["status"] == gpe.GPE_OK, (k, out)
    # a sample of the uncancelled results against the single-context path
    for k in range(0, len(reqs), 17):
        if k in cancel or res[k]["status"] != gpe.GPE_OK:
            continue
        tol = {"fp64": 1e-12, "fp32": 1e-5, "fp32s": 1e-6}[reqs[k]["precision"]]
        assert rel(res[k]["psi"], solve_alone_ctx(reqs[k])) < tol, k
