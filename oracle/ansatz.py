"""Trotterized UCCSD state, energy and adjoint gradient.

Test infrastructure only (see oracle/__init__.py).

Ansatz (Eqs. 3-4): |Psi> = exp(T - T^dag)|HF>, T built from
    singles  T_k = a_a^dag a_i                (i occupied, a virtual)
    doubles  T_k = a_a^dag a_b^dag a_j a_i    (i < j occupied, a < b virtual)
First-order Trotter product with one slice (Eq. 5, M = 1): the factors
U_k = exp(theta_k G_k), G_k = T_k - T_k^dag, are applied to |HF> in the
order of the excitation list.  The paper writes each factor as a product of
commuting Pauli exponentials; one factor per excitation is the same operator
(pinned in the tests).  Reading: one amplitude theta_k per listed excitation,
no extra factor 1/2 (the 1/2 of Eq. 4 counts each double twice when i, j
and a, b run unrestricted).

Each factor acts as a rotation on pairs of basis states: wherever
T_k|u> = s|v> (s = +-1),
    psi'[u] = cos(theta) psi[u] - s sin(theta) psi[v]
    psi'[v] = cos(theta) psi[v] + s sin(theta) psi[u]
and leaves every other amplitude alone.  This is exp(theta G) because G
maps u -> s v, v -> -s u, and kills everything else, so G^3 = -G and
exp(theta G) = 1 + sin(theta) G + (1 - cos(theta)) G^2.

Gradient: dE/dtheta_k = 2 Re <lambda_k| G_k |psi_k>, with psi_k the state
after factor k and lambda_k = U_{k+1}^dag ... U_K^dag H psi_K, swept from
k = K down to 1 (the adjoint method).

Trotter variants (Eqs. 5 and 6): M slices of the first-order product apply
the list M times with angles theta/M; the second-order (symmetric) product
applies, per slice, the list in order and then in reverse order, with
angles theta/(2M).  Reading: factors act in the order they are listed (the
first row first), as for M = 1.  A parameter that occurs several times gets
the sum of its occurrences' adjoint terms, each times the angle scale.

Pinned by: dense expm of G_k, the four-term parameter-shift rule and
central finite differences, the Slater-Condon gradient at theta = 0.
"""
from __future__ import annotations

import numpy as np

from .fermion import ladder_action
from .hamiltonian import apply_h, energy as _energy


def excitation_ops(row):
    """Operator product T_k for one row (i, j, a, b) of the excitation list."""
    i, j, a, b = (int(x) for x in row)
    if j < 0:
        return [(a, True), (i, False)]
    return [(a, True), (b, True), (j, False), (i, False)]


def excitation_pairs(n, row):
    """(u, v, s) with T_k|u> = s|v>, over all basis states."""
    return ladder_action(n, excitation_ops(row))


def hf_state(n, hf_occ):
    """|HF> for an occupation bitmask (default convention: 2^n_elec - 1)."""
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[int(hf_occ)] = 1.0
    return psi


def apply_factor(psi, pairs, theta):
    """exp(theta G_k) psi."""
    u, v, s = pairs
    c, sn = np.cos(theta), np.sin(theta)
    out = psi.copy()
    out[u] = c * psi[u] - s * sn * psi[v]
    out[v] = c * psi[v] + s * sn * psi[u]
    return out


def apply_generator(psi, pairs):
    """G_k psi."""
    u, v, s = pairs
    out = np.zeros_like(psi)
    out[v] = s * psi[u]
    out[u] = -s * psi[v]
    return out


def all_pairs(n, exc):
    return [excitation_pairs(n, row) for row in np.asarray(exc).reshape(-1, 4)]


def trotter_sequence(n_exc, slices=1, order=1):
    """Factors of Eq. 5 (order 1) or Eq. 6 (order 2) in the order they act: the parameter
    index of each factor, and the scale of its angle (1/M, or 1/(2M))."""
    if slices < 1 or order not in (1, 2):
        raise ValueError("slices >= 1 and order 1 or 2")
    one = list(range(n_exc)) if order == 1 else list(range(n_exc)) + list(range(n_exc - 1, -1, -1))
    return one * slices, 1.0 / (slices * order)


def apply_sequence(psi, pairs, theta, slices=1, order=1):
    """The Trotter product for amplitudes theta applied to psi."""
    seq, scale = trotter_sequence(len(pairs), slices, order)
    theta = np.asarray(theta, dtype=np.float64)
    for k in seq:
        psi = apply_factor(psi, pairs[k], scale * theta[k])
    return psi


def trotter_state(n, hf_occ, exc, theta, pairs=None, slices=1, order=1):
    """The Trotter product applied to |HF> (U_K ... U_1 |HF> for Eq. 5 with M = 1)."""
    if pairs is None:
        pairs = all_pairs(n, exc)
    return apply_sequence(hf_state(n, hf_occ), pairs, theta, slices, order)


def energy(h, g, n, hf_occ, exc, theta, pairs=None, slices=1, order=1):
    """Trotterized UCCSD energy <Psi|H|Psi> (the VQE cost)."""
    psi = trotter_state(n, hf_occ, exc, theta, pairs, slices, order)
    return _energy(h, g, psi)[0]


def energy_and_gradient(h, g, n, hf_occ, exc, theta, pairs=None, return_states=False,
                        slices=1, order=1):
    """(E, dE/dtheta) by a forward pass and an adjoint reverse sweep over the factors."""
    if pairs is None:
        pairs = all_pairs(n, exc)
    theta = np.asarray(theta, dtype=np.float64)
    seq, scale = trotter_sequence(theta.size, slices, order)
    psi = trotter_state(n, hf_occ, exc, theta, pairs, slices, order)
    lam = apply_h(h, g, psi)
    e = np.vdot(psi, lam)
    psi_final = psi.copy()
    grad = np.zeros(theta.size)
    for k in reversed(seq):
        grad[k] += scale * 2.0 * np.vdot(lam, apply_generator(psi, pairs[k])).real
        psi = apply_factor(psi, pairs[k], -scale * theta[k])
        lam = apply_factor(lam, pairs[k], -scale * theta[k])
    if return_states:
        return float(e.real), grad, dict(psi=psi_final, psi_back=psi, im_e=float(e.imag))
    return float(e.real), grad


def steepest_descent(h, g, n, hf_occ, exc, theta0, steps, lr):
    """VQE by steepest descent: theta <- theta - lr * grad, fixed steps.

    Returns (energies[steps + 1], theta_final); energies[s] is E before
    update s (the last one after the final update).
    """
    pairs = all_pairs(n, exc)
    theta = np.array(theta0, dtype=np.float64)
    es = []
    for _ in range(steps):
        e, gr = energy_and_gradient(h, g, n, hf_occ, exc, theta, pairs)
        es.append(e)
        theta = theta - lr * gr
    es.append(energy(h, g, n, hf_occ, exc, theta, pairs))
    return np.array(es), theta
