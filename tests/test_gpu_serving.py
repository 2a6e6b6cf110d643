"""GPU serving: the continuous-batching VQE server through the C ABI.

A job's result must be the same alone and in any mix (bitwise: each batch entry is computed
by the same kernels in the same order whatever else runs, and the host update is plain IEEE
arithmetic); one job's trajectory is checked against the CPU oracle's steepest descent
(|dE| <= 1e-10 Ha per step, theta within 1e-9).
"""
import json
import os
import time

import numpy as np
import pytest

from oracle import ansatz, hamiltonian
from paper_2402_17993_amd.inputs import make_integrals, make_thetas, uccsd_excitations

pytestmark = pytest.mark.gpu

LR = 0.1


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ucc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2402_17993_amd import ucc as u
    u.lib()
    return u


def make_ctx(ucc, n, ne, seed):
    h1, h2 = make_integrals(n // 2, seed)
    return ucc.Context(n, ne, h1, h2, uccsd_excitations(n, ne), max_batch=0)


def solo_sd(ctx, th0, iters, lr=LR):
    """The same steepest descent through plain ucc_energy_grad calls, one vector at a time."""
    th = np.array(th0, dtype=np.float64)
    es = []
    for i in range(iters + 1):
        e, g = ctx.energy_grad(th)
        es.append(e[0])
        if i < iters:
            th = th - lr * g[0]
    return np.array(es), th


def test_results_identical_alone_and_in_the_mix(ucc):
    say("case: serving mix of 8q, 12q (three Hamiltonians), 16q (two Hamiltonians, three starts)")
    ctxs = {"m1": make_ctx(ucc, 12, 8, 101), "m2": make_ctx(ucc, 12, 8, 102),
            "m3": make_ctx(ucc, 12, 8, 103), "d": make_ctx(ucc, 16, 8, 104),
            "s": make_ctx(ucc, 8, 4, 105), "d2": make_ctx(ucc, 16, 8, 106)}
    assert ctxs["m1"].batch_compatible(ctxs["m2"]) and ctxs["m1"].batch_compatible(ctxs["m3"])
    # two 16-qubit Hamiltonians share a launch through per-entry value tables in the mix (the
    # single-table pair walk runs them alone): the results must not differ by one bit
    assert ctxs["d"].batch_compatible(ctxs["d2"])
    jobs = [("m1", 1), ("m2", 2), ("m3", 3), ("d", 4), ("d", 5), ("s", 6), ("d2", 7)]
    iters = 5
    th0 = {j: make_thetas(ctxs[c].n_exc, seed, 0.05) for j, (c, seed) in enumerate(jobs)}
    alone = {j: solo_sd(ctxs[c], th0[j], iters) for j, (c, _) in enumerate(jobs)}
    with ucc.Server(slots=16) as srv:
        tickets = {j: srv.submit(ctxs[c], th0[j], iters, LR) for j, (c, _) in enumerate(jobs)}
        res = {j: srv.wait(t) for j, t in tickets.items()}
    for j in res:
        assert res[j]["status"] == 0 and res[j]["rounds"] == iters + 1
        assert np.array_equal(res[j]["energies"], alone[j][0]), j
        assert np.array_equal(res[j]["theta"], alone[j][1]), j
    # the 8-qubit job against the oracle's steepest descent
    h1, h2 = make_integrals(4, 105)
    h, g = hamiltonian.spin_orbital_integrals(h1, h2)
    es_ref, th_ref = ansatz.steepest_descent(h, g, 8, 15, uccsd_excitations(8, 4), th0[5], iters, LR)
    assert np.max(np.abs(res[5]["energies"] - es_ref)) <= 1e-10
    assert np.max(np.abs(res[5]["theta"] - th_ref)) <= 1e-9


def test_jobs_of_the_mix_sizes_against_oracle_and_alone(ucc):
    """Monomer 12q/8e, dimer 18q/10e and trimer 24q/14e jobs (the serving mix's sizes) served
    together: each trajectory equals its solo run bitwise and the oracle's steepest descent
    (tests/golden/serving_jobs.json) to 1e-10 Ha per step, amplitudes to 1e-9."""
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "serving_jobs.json")))
    iters, lr = gold["iters"], gold["lr"]
    jobs = []
    for jb in gold["jobs"]:
        say(f"case: served {jb['n']}q/{jb['ne']}e job, integrals seed {jb['integral_seed']}")
        ctx = make_ctx(ucc, jb["n"], jb["ne"], jb["integral_seed"])
        jobs.append((ctx, make_thetas(ctx.n_exc, jb["theta_seed"], gold["theta_scale"]), jb))
    alone = [solo_sd(ctx, th, iters, lr) for ctx, th, _ in jobs]
    with ucc.Server(slots=8) as srv:
        tickets = [srv.submit(ctx, th, iters, lr) for ctx, th, _ in jobs]
        res = [srv.wait(t) for t in tickets]
    for r, a, (_, _, jb) in zip(res, alone, jobs):
        assert r["status"] == 0 and r["rounds"] == iters + 1
        assert np.array_equal(r["energies"], a[0]) and np.array_equal(r["theta"], a[1]), jb["n"]
        de = float(np.max(np.abs(r["energies"] - np.array(jb["energies"]))))
        dt = float(np.max(np.abs(r["theta"] - np.array(jb["theta"]))))
        say(f"{jb['n']}q: max |dE| {de:.2e}, max |dtheta| {dt:.2e}")
        assert de <= 1e-10 and dt <= 1e-9, jb["n"]
    for ctx, _, _ in jobs:
        ctx.close()


def test_jobs_join_while_others_run(ucc):
    say("case: short 12q jobs submitted while a long 16q job runs")
    long_ctx, short_ctx = make_ctx(ucc, 16, 8, 111), make_ctx(ucc, 12, 8, 112)
    th_long = make_thetas(long_ctx.n_exc, 7, 0.05)
    th_short = [make_thetas(short_ctx.n_exc, 8 + i, 0.05) for i in range(3)]
    ref_long = solo_sd(long_ctx, th_long, 150, 0.05)
    ref_short = [solo_sd(short_ctx, t, 2) for t in th_short]
    with ucc.Server(slots=8) as srv:
        tl = srv.submit(long_ctx, th_long, 150, 0.05)
        time.sleep(0.02)
        ts = [srv.submit(short_ctx, t, 2, LR) for t in th_short]
        rs = [srv.wait(t) for t in ts]
        still_running = srv.poll(tl) is None
        rl = srv.wait(tl)
    assert still_running, "the short jobs should finish while the long one runs"
    for r, ref in zip(rs, ref_short):
        assert np.array_equal(r["energies"], ref[0]) and np.array_equal(r["theta"], ref[1])
    assert np.array_equal(rl["energies"], ref_long[0]) and np.array_equal(rl["theta"], ref_long[1])


def test_admission_by_device_footprint(ucc):
    say("case: budget for two 12q jobs, three submitted")
    ctx = make_ctx(ucc, 12, 8, 121)
    fp = ctx.plan_info()["job_footprint"]
    ths = [make_thetas(ctx.n_exc, 20 + i, 0.05) for i in range(3)]
    refs = [solo_sd(ctx, t, 8) for t in ths]
    with ucc.Server(hbm_budget=2 * fp + fp // 2, slots=8) as srv:
        ts = [srv.submit(ctx, t, 8, LR) for t in ths]
        rs = [srv.wait(t) for t in ts]
    for r, ref in zip(rs, refs):
        assert np.array_equal(r["energies"], ref[0]) and np.array_equal(r["theta"], ref[1])
    # the third job is admitted only after one of the first two left
    first_done = min(rs[0]["done_s"], rs[1]["done_s"])
    assert rs[2]["admit_s"] >= first_done - 1e-3
    assert rs[2]["rounds"] == 9


def test_queue_limit_cancel_and_errors(ucc):
    say("case: queue limit, cancellation, busy context, budget and ticket errors")
    ctx = make_ctx(ucc, 16, 8, 131)
    other = make_ctx(ucc, 12, 8, 132)
    th = make_thetas(ctx.n_exc, 30, 0.05)
    with ucc.Server(slots=1, max_queue=1) as srv:
        ta = srv.submit(ctx, th, 100000, 0.01)
        busy = 0
        ok = []
        for i in range(3):
            try:
                ok.append(srv.submit(other, make_thetas(other.n_exc, 40 + i, 0.05), 1, LR))
            except ucc.UCCError as e:
                assert e.status == ucc.STATUS_CODES["UCC_EBUSY"]
                busy += 1
        assert busy >= 1
        # a context with a job in flight refuses direct evaluation
        with pytest.raises(ucc.UCCError) as ei:
            ctx.energy(th)
        assert ei.value.status == ucc.STATUS_CODES["UCC_EBUSY"]
        srv.cancel(ta)
        ra = srv.wait(ta)
        assert ra["status"] == ucc.STATUS_CODES["UCC_ECANCELED"]
        assert 0 <= ra["rounds"] < 100001
        for t in ok:
            assert srv.wait(t)["status"] == 0
        with pytest.raises(ucc.UCCError) as ei:
            srv.wait(987654321)
        assert ei.value.status == ucc.STATUS_CODES["UCC_ENOTFOUND"]
    # the context is free again
    assert np.isfinite(ctx.energy(th)[0])
    with ucc.Server(hbm_budget=1024, slots=4) as srv:
        with pytest.raises(ucc.UCCError) as ei:
            srv.submit(ctx, th, 1, LR)
        assert ei.value.status == ucc.STATUS_CODES["UCC_ENOMEM"]
