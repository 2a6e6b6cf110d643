"""Pins of the sector-restricted oracle (oracle/sector.py) against the full-space oracle and
against closed forms it does not share.

The full-space oracle is pinned elsewhere (dense Kronecker matrices, expm, shift rule, closed
forms); here the sector version must reproduce it entry by entry wherever both fit, and must
reproduce the closed-form theta = 0 values on a system too large for the full-space one.
"""
import math

import numpy as np
import pytest

from oracle import ansatz, closed_forms, hamiltonian, sector, trotter_free
from paper_2402_17993_amd.inputs import make_integrals, make_thetas, uccsd_excitations


def system(n, ne, seed=0, order="interleaved"):
    h1, h2 = make_integrals(n // 2, seed)
    h, g = hamiltonian.spin_orbital_integrals(h1, h2, order)
    return h1, h2, h, g


def test_sector_basis_matches_brute_force():
    for n, na, nb, order in ((10, 3, 3, "interleaved"), (10, 2, 4, "interleaved"), (8, 2, 1, "blocked")):
        basis = sector.sector_basis(n, na, nb, order)
        sg = sector.spin_of_orbitals(n, order)
        am = sum(1 << q for q in range(n) if sg[q] == 0)
        bm = sum(1 << q for q in range(n) if sg[q] == 1)
        x = np.arange(1 << n, dtype=np.int64)
        want = x[(np.bitwise_count(x & am) == na) & (np.bitwise_count(x & bm) == nb)]
        assert np.array_equal(basis, want)
        assert basis.size == math.comb(n // 2, na) * math.comb(n // 2, nb)


def test_apply_h_equals_full_space():
    rng = np.random.default_rng(5)
    for n, ne, order in ((8, 4, "interleaved"), (10, 6, "interleaved"), (10, 4, "blocked")):
        _, _, h, g = system(n, ne, 3, order)
        hf = sum(1 << q for q in range(ne)) if order == "interleaved" else \
            sum(1 << q for q in range(ne // 2)) | sum(1 << (n // 2 + q) for q in range(ne // 2))
        basis = sector.hf_sector(n, hf, order)[0]
        v = rng.normal(size=basis.size) + 1j * rng.normal(size=basis.size)
        full = hamiltonian.apply_h(h, g, sector.to_full(n, basis, v))
        # H keeps the sector: nothing outside it
        outside = np.ones(1 << n, dtype=bool)
        outside[basis] = False
        assert np.max(np.abs(full[outside])) == 0.0
        for block in (1 << 18, 7):
            mine = sector.apply_h(h, g, n, basis, v, order, block=block)
            assert np.max(np.abs(mine - full[basis])) <= 1e-12 * max(1.0, np.max(np.abs(full)))


@pytest.mark.parametrize("n,ne,slices,order", [(8, 4, 1, 1), (10, 6, 1, 1), (12, 8, 1, 1),
                                                (8, 4, 2, 1), (8, 4, 1, 2)])
def test_energy_and_gradient_equal_full_space(n, ne, slices, order):
    _, _, h, g = system(n, ne)
    exc = uccsd_excitations(n, ne)
    th = make_thetas(len(exc), 1, 0.1)
    hf = (1 << ne) - 1
    e_full, g_full = ansatz.energy_and_gradient(h, g, n, hf, exc, th, slices=slices, order=order)
    e, gr, st = sector.energy_and_gradient(h, g, n, hf, exc, th, slices=slices, order=order,
                                           return_states=True)
    assert abs(e - e_full) <= 1e-12
    assert np.max(np.abs(gr - g_full)) <= 1e-12
    assert abs(np.linalg.norm(st["psi"]) - 1.0) <= 1e-13
    back = st["psi_back"]
    assert abs(back[sector.positions(st["basis"], np.array([hf]))[0]] - 1.0) <= 1e-13
    # cached pairs give the same numbers bitwise
    pairs = sector.all_pairs(n, st["basis"], exc)
    e2, g2 = sector.energy_and_gradient(h, g, n, hf, exc, th, pairs=pairs, slices=slices, order=order)
    assert e2 == e and np.array_equal(g2, gr)


def test_state_equals_full_space_trotter_state():
    n, ne = 10, 4
    _, _, h, g = system(n, ne, 2)
    exc = uccsd_excitations(n, ne)
    th = make_thetas(len(exc), 4, 0.3)
    basis, psi = sector.trotter_state(n, (1 << ne) - 1, exc, th)
    full = ansatz.trotter_state(n, (1 << ne) - 1, exc, th)
    assert np.max(np.abs(sector.to_full(n, basis, psi) - full)) <= 1e-14


def test_blocked_order_energy_equals_interleaved():
    """The same fermionic ansatz in the blocked spin-orbital order (P6 on the sector path)."""
    n, ne = 10, 6
    h1, h2 = make_integrals(n // 2, 0)
    h, g = hamiltonian.spin_orbital_integrals(h1, h2)
    hb, gb = hamiltonian.spin_orbital_integrals(h1, h2, "blocked")
    exc = uccsd_excitations(n, ne)
    th = make_thetas(len(exc), 1, 0.1)
    ns = n // 2
    remap = lambda q: -1 if q < 0 else (q // 2) + ns * (q % 2)  # noqa: E731
    excb = np.array([[remap(int(q)) for q in row] for row in exc])
    hfb = sum(1 << remap(q) for q in range(ne))
    e = sector.energy(h, g, n, (1 << ne) - 1, exc, th)
    eb = sector.energy(hb, gb, n, hfb, excb, th, orbital_order="blocked")
    assert abs(e - eb) <= 1e-12


def test_theta_zero_closed_forms_beyond_the_full_space_oracle():
    """20 qubits, 10 electrons: E(0) = closed-form HF energy, dE/dtheta(0) = Slater-Condon."""
    n, ne = 20, 10
    h1, h2, h, g = system(n, ne, 7)
    exc = uccsd_excitations(n, ne)
    e, gr = sector.energy_and_gradient(h, g, n, (1 << ne) - 1, exc, np.zeros(len(exc)))
    assert abs(e - closed_forms.hf_energy_spatial(h1, h2, ne)) <= 1e-11
    assert np.max(np.abs(gr - closed_forms.gradient_at_zero(h, g, range(ne), exc))) <= 1e-11


def test_trotter_free_equals_full_space():
    n, ne = 8, 4
    _, _, h, g = system(n, ne, 1)
    exc = uccsd_excitations(n, ne)
    th = make_thetas(len(exc), 2, 0.2)
    hf = (1 << ne) - 1
    ks = [0, 3, len(exc) - 1]
    e_full, g_full = trotter_free.trotter_free_energy_and_gradient(h, g, n, hf, exc, th, ks=ks)
    e, gr = sector.trotter_free_energy_and_gradient(h, g, n, hf, exc, th, ks=ks)
    assert abs(e - e_full) <= 1e-12
    assert np.max(np.abs(gr[ks] - g_full[ks])) <= 1e-12
    assert np.all(np.isnan(np.delete(gr, ks)))


def test_planted_mistakes_fail():
    """A dropped term, a flipped sign or a swapped operand in the sector path would be caught:
    perturbed variants of its inputs move E away from the full-space value by far more than the
    tolerance used above."""
    n, ne = 8, 4
    _, _, h, g = system(n, ne)
    exc = uccsd_excitations(n, ne)
    th = make_thetas(len(exc), 1, 0.1)
    hf = (1 << ne) - 1
    e_full = ansatz.energy(h, g, n, hf, exc, th)
    g_drop = g.copy()
    g_drop[0, 1, 0, 1] = g_drop[1, 0, 1, 0] = 0.0
    assert abs(sector.energy(h, g_drop, n, hf, exc, th) - e_full) > 1e-6
    exc_swapped = exc.copy()
    exc_swapped[[len(exc) - 1, len(exc) - 2]] = exc_swapped[[len(exc) - 2, len(exc) - 1]]
    th_neg = th.copy()
    th_neg[0] = -th_neg[0]
    assert abs(sector.energy(h, g, n, hf, exc, th_neg) - e_full) > 1e-6
