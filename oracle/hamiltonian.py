"""The electronic Hamiltonian of Eq. 2 and its action on a state vector.

Test infrastructure only (see oracle/__init__.py).

    H = sum_{PQ} h_{PQ} a_P^dag a_Q + 1/2 sum_{PQRS} g_{PQRS} a_P^dag a_Q^dag a_S a_R

over spin orbitals.  Reading of the paper's notation (it does not spell the
index convention out): g_{PQRS} = <PQ|RS> (physicist) = (PR|QS) (chemist);
the input h2 is the chemist-order spatial array (pr|qs).  Spin-orbital
integrals vanish unless spins match: h_{PQ} needs sigma_P = sigma_Q, and
<PQ|RS> needs sigma_P = sigma_R and sigma_Q = sigma_S.  No constant
(nuclear repulsion, frozen core) is included.

apply_h_literal  every term of Eq. 2 applied one by one (small n).
apply_h          the same sum with the four orderings of each two-body
                 operator merged by anticommutation, and the inner sum over
                 annihilation pairs done as one matrix product.  Pinned to
                 apply_h_literal and to the dense Kronecker H in the tests.
"""
from __future__ import annotations

import numpy as np

from .fermion import apply_product


def orbital_maps(n_spatial: int, order: str = "interleaved"):
    """spatial(q), spin(q) index arrays for the spin-orbital ordering."""
    n = 2 * n_spatial
    q = np.arange(n)
    if order == "interleaved":
        return q // 2, q % 2
    if order == "blocked":
        return q % n_spatial, q // n_spatial
    raise ValueError(order)


def spin_orbital_integrals(h1, h2, order: str = "interleaved"):
    """h[P,Q] and g[P,Q,R,S] = <PQ|RS> from spatial h1 and chemist h2."""
    h1 = np.asarray(h1, dtype=np.float64)
    h2 = np.asarray(h2, dtype=np.float64)
    ns = h1.shape[0]
    sp, sg = orbital_maps(ns, order)
    same = (sg[:, None] == sg[None, :]).astype(np.float64)
    h = h1[np.ix_(sp, sp)] * same
    # g[P,Q,R,S] = (P R | Q S) * d(sP,sR) d(sQ,sS)
    g = h2[sp[:, None, None, None], sp[None, None, :, None],
           sp[None, :, None, None], sp[None, None, None, :]]
    g = g * same[:, None, :, None] * same[None, :, None, :]
    return h, g


def apply_h_literal(h, g, psi):
    """sigma = H psi, one term of Eq. 2 at a time."""
    n = h.shape[0]
    out = np.zeros_like(psi)
    for p in range(n):
        for q in range(n):
            if h[p, q] != 0.0:
                apply_product(n, [(p, True), (q, False)], psi, h[p, q], out)
    for p in range(n):
        for q in range(n):
            for r in range(n):
                for s in range(n):
                    c = g[p, q, r, s]
                    if c != 0.0:
                        apply_product(n, [(p, True), (q, True), (s, False), (r, False)],
                                      psi, 0.5 * c, out)
    return out


def _pairs(n):
    return [(r, s) for r in range(n) for s in range(r + 1, n)]


def apply_h(h, g, psi):
    """sigma = H psi (Eq. 2).

    Two-body part: terms with P = Q or R = S vanish; for P < Q, R < S the four
    orderings combine to W[PQ,RS] a_P^dag a_Q^dag a_S a_R with
    W = (g_PQRS - g_QPRS - g_PQSR + g_QPSR) / 2.  The vectors a_S a_R psi are
    formed once per pair, mixed by W (one matrix product), and raised by
    a_P^dag a_Q^dag.
    """
    n = h.shape[0]
    psi = np.asarray(psi, dtype=np.complex128)
    out = np.zeros_like(psi)
    for p in range(n):
        for q in range(n):
            if h[p, q] != 0.0:
                apply_product(n, [(p, True), (q, False)], psi, h[p, q], out)
    pairs = _pairs(n)
    pi = np.array([p for p, _ in pairs])
    qi = np.array([q for _, q in pairs])
    w = 0.5 * (g[pi[:, None], qi[:, None], pi[None, :], qi[None, :]]
               - g[qi[:, None], pi[:, None], pi[None, :], qi[None, :]]
               - g[pi[:, None], qi[:, None], qi[None, :], pi[None, :]]
               + g[qi[:, None], pi[:, None], qi[None, :], pi[None, :]])
    rows = np.flatnonzero(np.any(w != 0.0, axis=1))
    cols = np.flatnonzero(np.any(w != 0.0, axis=0))
    if rows.size == 0:
        return out
    phi = np.zeros((cols.size, psi.size), dtype=np.complex128)
    for k, c in enumerate(cols):
        r, s = pairs[c]
        apply_product(n, [(s, False), (r, False)], psi, 1.0, phi[k])
    xi = w[np.ix_(rows, cols)] @ phi
    del phi
    for k, rrow in enumerate(rows):
        p, q = pairs[rrow]
        apply_product(n, [(p, True), (q, True)], xi[k], 1.0, out)
    return out


def energy(h, g, psi):
    """E = <psi|H|psi>; returns (Re E, Im E)."""
    sigma = apply_h(h, g, psi)
    e = np.vdot(psi, sigma)
    return float(e.real), float(e.imag)
