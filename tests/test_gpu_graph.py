"""GPU tests of the evaluation graph (launch_mode 3, ucc_energy_grad_jobs): every pass of an
energy + gradient call in one persistent launch, items gated by per-entry counters.

  * the graph's energies and gradients equal those of the per-pass launches of a context with
    the same tiles and workgroups, bit for bit (the same pass bodies run every item), and the
    oracle's to |dE| <= 1e-10 Ha, max_k |dg_k| <= 1e-9;
  * jobs of different sizes (12, 18 and 24 qubits) in ONE launch give each job's result alone,
    bit for bit, and the 24-qubit job matches the stored oracle values;
  * a launch whose waits are bounded by 1 us gives up: every workgroup exits, the outputs are
    NaN, and the call (or ucc_graph_status) reports UCC_EDEVICE; the bound is the kernel's own,
    forced from the host, so every kernel still ends normally.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import hamiltonian, sector
from paper_2402_17993_amd.inputs import make_integrals, make_thetas, uccsd_excitations

pytestmark = pytest.mark.gpu

E_TOL = 1e-10
G_TOL = 1e-9
HERE = os.path.dirname(os.path.abspath(__file__))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ucc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2402_17993_amd import ucc as u
    u.lib()
    return u


def load(name):
    return json.load(open(os.path.join(HERE, "golden", f"{name}.json")))


def per_pass_twin(ucc, n, ne, h1, h2, exc, B, **kw):
    """A launch_mode 1 context with the tiles and workgroups launch_mode 3 chooses."""
    k = min(n, 13)
    return ucc.Context(n, ne, h1, h2, exc, max_batch=B, launch_mode=1, block_threads=512,
                       tile_qubits=k, tile_qubits_exp=k, tile_qubits_rev=k, **kw)


@pytest.mark.parametrize("n,ne,seed,B,kw", [
    (8, 4, 0, 3, {}),                        # one tile: the loop form of the bodies
    (12, 8, 1, 5, {}),                       # one 12-qubit tile, stored states
    (16, 8, 3, 4, {}),                       # 8 tiles, stored states
    (16, 8, 3, 4, dict(store_states=2)),     # recomputing reverse sweep
    (18, 10, 0, 64, {}),                     # the benchmark batch
])
def test_graph_equals_per_pass_and_oracle(ucc, n, ne, seed, B, kw):
    say(f"case: graph {n}q/{ne}e seed {seed} B {B} {kw}")
    h1, h2 = make_integrals(n // 2, seed)
    exc = uccsd_excitations(n, ne)
    th = make_thetas(len(exc), seed + 1, 0.05, batch=B)
    g = ucc.Context(n, ne, h1, h2, exc, max_batch=B, launch_mode=3, **kw)
    e3, g3 = g.energy_grad(th)
    info = g.plan_info()
    say(f"graph grid {info['graph_grid']}, LDS {info['graph_lds']} B, passes "
        f"{info['n_fwd_passes']}/{info['n_exp_passes']}/{info['n_rev_passes']}")
    assert info["launch_mode"] == 3 and info["graph_grid"] > 0
    pp = per_pass_twin(ucc, n, ne, h1, h2, exc, B, **kw)
    e1, g1 = pp.energy_grad(th)
    assert np.array_equal(e3, e1) and np.array_equal(g3, g1)
    # energy-only calls of a launch_mode 3 context run the per-pass launches: same energies
    assert np.array_equal(g.energy(th), pp.energy(th))
    if n <= 16:
        hh, gg = hamiltonian.spin_orbital_integrals(h1, h2)
        for b in (0, B - 1):
            e_ref, g_ref = sector.energy_and_gradient(hh, gg, n, (1 << ne) - 1, exc, th[b])
            assert abs(e3[b] - e_ref) <= E_TOL
            assert np.max(np.abs(g3[b] - g_ref)) <= G_TOL
    g.close()
    pp.close()


def test_graph_batch64_against_stored_oracle_values(ucc):
    say("case: graph 18q/10e batch 64 against all 64 stored oracle energies and gradients")
    gold = load("dimer_18q")
    n, ne = gold["n"], gold["ne"]
    h1, h2 = make_integrals(n // 2, gold["integral_seed"])
    exc = uccsd_excitations(n, ne)
    th = make_thetas(len(exc), gold["theta_seed"], gold["theta_scale"], batch=gold["batch"])
    g = ucc.Context(n, ne, h1, h2, exc, max_batch=64, launch_mode=3)
    g.profile(True)
    e, gr = g.energy_grad(th)
    st = g.profile_read()
    g.profile(False)
    assert st["graph"]["launches"] == 1 and st["fwd"]["launches"] == 0
    for b, ent in gold["entries"].items():
        b = int(b)
        assert abs(e[b] - ent["energy"]) <= E_TOL, b
        assert np.max(np.abs(gr[b] - np.array(ent["grad"]))) <= G_TOL, b
    g.close()


def test_jobs_of_three_sizes_in_one_launch(ucc):
    say("case: one graph launch over a 12q (B 2), an 18q (B 3) and a 24q (B 1) job")
    gold18, gold24 = load("dimer_18q"), load("large_24q")
    specs = [(12, 8, 31, None), (18, 10, gold18["integral_seed"], gold18), (24, 14, gold24["integral_seed"], gold24)]
    ctxs, thetas, twins = [], [], []
    for n, ne, seed, gold in specs:
        h1, h2 = make_integrals(n // 2, seed)
        exc = uccsd_excitations(n, ne)
        if n == 12:
            th = make_thetas(len(exc), 40, 0.05, batch=2)
        elif n == 18:
            th = make_thetas(len(exc), gold["theta_seed"], gold["theta_scale"], batch=gold["batch"])[:3]
        else:
            th = make_thetas(len(exc), gold["theta_seed"], gold["theta_scale"])[None, :]
        ctxs.append(ucc.Context(n, ne, h1, h2, exc, max_batch=th.shape[0], launch_mode=3))
        twins.append(per_pass_twin(ucc, n, ne, h1, h2, exc, th.shape[0]))
        thetas.append(th)
    mix = ucc.energy_grad_jobs(ctxs, thetas)
    grids = {c.plan_info()["graph_grid"] for c in ctxs}
    assert len(grids) == 1 and grids.pop() > 0
    for c, t, th, (e, g), (n, _, _, gold) in zip(ctxs, twins, thetas, mix, specs):
        alone = c.energy_grad(th)
        pp = t.energy_grad(th)
        say(f"{n}q: mix == alone {np.array_equal(e, alone[0]) and np.array_equal(g, alone[1])}, "
            f"== per-pass {np.array_equal(e, pp[0]) and np.array_equal(g, pp[1])}")
        assert np.array_equal(e, alone[0]) and np.array_equal(g, alone[1])
        assert np.array_equal(e, pp[0]) and np.array_equal(g, pp[1])
        if n == 18:
            for b in range(3):
                ent = gold["entries"][str(b)]
                assert abs(e[b] - ent["energy"]) <= E_TOL
                assert np.max(np.abs(g[b] - np.array(ent["grad"]))) <= G_TOL
        if n == 24:
            assert abs(e[0] - gold["energy"]) <= E_TOL
            assert np.max(np.abs(g[0] - np.array(gold["grad"]))) <= G_TOL
    # the same through torch tensors (device pointers, stream-ordered)
    import torch
    dev = [torch.tensor(th, device="cuda:0") for th in thetas]
    mix_t = ucc.energy_grad_jobs(ctxs, dev)
    torch.cuda.synchronize()
    for (e, g), (et, gt) in zip(mix, mix_t):
        assert np.array_equal(e, et.cpu().numpy()) and np.array_equal(g, gt.cpu().numpy())
    for c in ctxs + twins:
        c.close()


def test_graph_rejects_bad_job_lists(ucc):
    h1, h2 = make_integrals(4, 0)
    exc = uccsd_excitations(8, 4)
    g = ucc.Context(8, 4, h1, h2, exc, launch_mode=3)
    pp = ucc.Context(8, 4, h1, h2, exc, launch_mode=1)
    th = make_thetas(len(exc), 1, 0.05)
    with pytest.raises(ucc.UCCError) as e1:
        ucc.energy_grad_jobs([g, pp], [th, th])
    assert e1.value.status == ucc.STATUS_CODES["UCC_EINVAL"]
    with pytest.raises(ucc.UCCError) as e2:
        ucc.energy_grad_jobs([g, g], [th, th])
    assert e2.value.status == ucc.STATUS_CODES["UCC_EINVAL"]
    g.close()
    pp.close()


def test_graph_gives_up_when_waits_are_bounded_by_1us(ucc):
    say("case: 24q/14e B 1 graph with graph_wait_us = 1 (the launch must give up)")
    gold = load("large_24q")
    n, ne = gold["n"], gold["ne"]
    h1, h2 = make_integrals(n // 2, gold["integral_seed"])
    exc = uccsd_excitations(n, ne)
    th = make_thetas(len(exc), gold["theta_seed"], gold["theta_scale"])
    g = ucc.Context(n, ne, h1, h2, exc, launch_mode=3, graph_wait_us=1)
    with pytest.raises(ucc.UCCError) as ei:
        g.energy_grad(th)  # host outputs: the call checks the launch itself
    assert ei.value.status == ucc.STATUS_CODES["UCC_EDEVICE"]
    import torch
    E, G = g.energy_grad(torch.tensor(th, device="cuda:0"))
    torch.cuda.synchronize()
    assert torch.isnan(E).all() and torch.isnan(G).all()
    with pytest.raises(ucc.UCCError):
        g.graph_status()
    g.graph_status()  # the mark was cleared by the check
    g.close()
    # the default bound: the same job completes and matches the stored oracle values
    ok = ucc.Context(n, ne, h1, h2, exc, launch_mode=3)
    e, gr = ok.energy_grad(th)
    ok.graph_status()
    assert abs(e[0] - gold["energy"]) <= E_TOL
    assert np.max(np.abs(gr[0] - np.array(gold["grad"]))) <= G_TOL
    ok.close()


def test_server_rounds_of_three_sizes_share_graph_launches(ucc):
    say("case: server, launch_mode 3 jobs of 12q (x2), 18q (x2) and 24q (x1), 3 steps each")
    from paper_2402_17993_amd.ucc import Server
    gold24 = load("large_24q")
    specs = [(12, 8, 31), (18, 10, 0), (24, 14, gold24["integral_seed"])]
    ctxs, twins, jobs = [], [], []
    for i, (n, ne, seed) in enumerate(specs):
        h1, h2 = make_integrals(n // 2, seed)
        exc = uccsd_excitations(n, ne)
        ctxs.append(ucc.Context(n, ne, h1, h2, exc, max_batch=0, launch_mode=3))
        k = min(n, 13)
        twins.append(ucc.Context(n, ne, h1, h2, exc, max_batch=0, launch_mode=1, block_threads=512,
                                 tile_qubits=k, tile_qubits_exp=k, tile_qubits_rev=k))
        if n == 24:
            jobs.append((i, make_thetas(len(exc), gold24["theta_seed"], gold24["theta_scale"])))
        else:
            jobs += [(i, make_thetas(len(exc), 50 + 2 * i, 0.05)), (i, make_thetas(len(exc), 51 + 2 * i, 0.05))]
    with Server(slots=8) as srv:
        mix = [srv.wait(t) for t in [srv.submit(ctxs[i], th, 3, 0.1) for i, th in jobs]]
    for (i, th), r in zip(jobs, mix):
        with Server(slots=8) as srv:
            alone = srv.wait(srv.submit(ctxs[i], th, 3, 0.1))
        with Server(slots=8) as srv:
            twin = srv.wait(srv.submit(twins[i], th, 3, 0.1))
        say(f"{specs[i][0]}q job: mix == alone {np.array_equal(alone['energies'], r['energies'])}, "
            f"== per-pass {np.array_equal(twin['energies'], r['energies'])}")
        assert np.array_equal(alone["energies"], r["energies"]) and np.array_equal(alone["theta"], r["theta"])
        assert np.array_equal(twin["energies"], r["energies"]) and np.array_equal(twin["theta"], r["theta"])
    # the 24-qubit job's first energy is the stored oracle value
    assert abs(mix[-1]["energies"][0] - gold24["energy"]) <= E_TOL
    for c in ctxs + twins:
        c.close()
