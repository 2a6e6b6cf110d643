"""GPU parity above 20 qubits: the HIP path through the C ABI against stored oracle values
computed on the N / S_z sector (tests/golden/make_golden.py, oracle/sector.py).

24 qubits / 14 electrons (the serving mix's trimer size, 256 MiB per state, K = 1,715) and
26 qubits / 14 electrons (1 GiB per state, K = 2,478): the energy and every gradient
component at theta ~ U(-0.05, 0.05), |dE| <= 1e-10 Ha and max_k |dg_k| <= 1e-9.  These
exercise many global bits, long window lists and large offsets, which the smaller parity
cases do not reach.
"""
import json
import os
import sys

import numpy as np
import pytest

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


def inputs_of(gold):
    n, ne = gold["n"], gold["ne"]
    h1, h2 = make_integrals(n // 2, gold["integral_seed"])
    exc = uccsd_excitations(n, ne)
    th = make_thetas(len(exc), gold["theta_seed"], gold["theta_scale"])
    return n, ne, h1, h2, exc, th


def check(e, gr, gold):
    de = abs(float(e) - gold["energy"])
    dg = float(np.max(np.abs(np.asarray(gr) - np.array(gold["grad"]))))
    say(f"|dE| = {de:.2e}, max |dg| = {dg:.2e}")
    assert de <= E_TOL and dg <= G_TOL


@pytest.mark.parametrize("kw", [dict(), dict(store_states=1), dict(autotune=True),
                                dict(tile_qubits=14, tile_qubits_rev=14)],
                         ids=["default", "stored-states", "autotuned", "rev-tile-14"])
def test_24q_energy_gradient_against_oracle(ucc, kw):
    gold = load("large_24q")
    n, ne, h1, h2, exc, th = inputs_of(gold)
    say(f"case: 24q/14e seed 0 energy+grad, {kw}")
    ctx = ucc.Context(n, ne, h1, h2, exc, **kw)
    e, gr = ctx.energy_grad(th)
    check(e[0], gr[0], gold)
    e_only = ctx.energy(th)
    assert abs(e_only[0] - gold["energy"]) <= E_TOL
    ctx.close()


def test_24q_batch_entries_equal_solo(ucc):
    gold = load("large_24q")
    n, ne, h1, h2, exc, th = inputs_of(gold)
    say("case: 24q/14e batch of 3 (the golden vector in the middle) against solo, bitwise")
    rows = np.stack([make_thetas(len(exc), 5, 0.05), th, make_thetas(len(exc), 6, 0.05)])
    ctx = ucc.Context(n, ne, h1, h2, exc, max_batch=3)
    e, gr = ctx.energy_grad(rows)
    check(e[1], gr[1], gold)
    solo = ucc.Context(n, ne, h1, h2, exc)
    e1, g1 = solo.energy_grad(th)
    assert e1[0] == e[1] and np.array_equal(g1[0], gr[1])
    ctx.close()
    solo.close()


@pytest.mark.parametrize("kw", [dict(), dict(tile_qubits_rev=14)], ids=["default", "rev-tile-14"])
def test_26q_energy_gradient_against_oracle(ucc, kw):
    gold = load("large_26q")
    n, ne, h1, h2, exc, th = inputs_of(gold)
    say(f"case: 26q/14e seed 0 energy+grad (all 2,478 components), {kw}")
    ctx = ucc.Context(n, ne, h1, h2, exc, **kw)
    e, gr = ctx.energy_grad(th)
    check(e[0], gr[0], gold)
    ctx.close()
