"""The oracle's Hamiltonian action, energy and adjoint gradient, stored on one N / S_z sector.

Test infrastructure only (see oracle/__init__.py).

Every term of the Hamiltonian of Eq. 2 and every factor exp(theta_k (T_k - T_k^dag)) of
Eqs. 3-5 moves electrons between spin orbitals of the same spin: creation and annihilation
operators come in spin-matched pairs.  A state that starts as |HF> therefore has exactly
zero amplitude on every basis state whose numbers of alpha and beta electrons differ from
those of |HF>.  This module does the arithmetic of ansatz.py, hamiltonian.py and
trotter_free.py (the same ladder-operator products on integer bitstrings, the same sums and
the same per-pair rotations) but keeps a vector only on the basis states of that sector:
a sorted array `basis` of their indices, an amplitude per entry, positions of operator
images found by binary search.  Nothing is approximated: the dropped amplitudes are the
exact zeros the full-space oracle carries.  At 26 qubits and 14 electrons the sector holds
C(13, 7)^2 = 2,944,656 states instead of 2^26 (47 MB per vector instead of 1 GiB), which is
what lets the oracle reach the large systems at all.

Two-body part of H psi: as in hamiltonian.apply_h, the four orderings of a two-body term
with P < Q, R < S are merged into W[PQ, RS] a_P^dag a_Q^dag a_S a_R.  W only connects pairs
of the same spin content (both alpha, both beta, one of each), because the integrals
vanish otherwise; the intermediate vectors a_S a_R psi of one spin content live on the
sector with those two electrons removed.  They are formed a block of intermediate states at
a time (entry x of a_S a_R psi is the sum over y of <x|a_S a_R|y> psi[y], and the only y is
the image of x under the adjoint a_R^dag a_S^dag, with the same real sign), mixed by W in
one matrix product, and raised by a_P^dag a_Q^dag into the output.  The block size bounds
memory and changes nothing else.

Pinned by (tests/test_oracle_sector.py): equality with the full-space oracle (itself pinned
to dense Kronecker matrices, expm, closed forms and the shift rule) for H psi, energies,
gradients, the Trotter variants and the Trotter-free ansatz at 8 to 12 qubits, in both
orbital orders and with tiny blocks; the closed-form Hartree-Fock energy and Slater-Condon
gradient at theta = 0 on a system the full-space oracle cannot hold; the sector size and
membership against a brute-force filter; norm 1 and the reverse sweep returning |HF>.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse
import scipy.sparse.linalg

from .ansatz import apply_factor, apply_generator, excitation_ops, trotter_sequence
from .fermion import ladder_action, popcount
from .hamiltonian import _pairs, orbital_maps
from .trotter_free import generator_matrix


def spin_of_orbitals(n: int, order: str = "interleaved") -> np.ndarray:
    """sigma(q) for every spin orbital q (0 alpha, 1 beta)."""
    return orbital_maps(n // 2, order)[1]


def sector_basis(n: int, n_alpha: int, n_beta: int, order: str = "interleaved") -> np.ndarray:
    """Sorted indices of the basis states with n_alpha alpha and n_beta beta electrons."""
    sg = spin_of_orbitals(n, order)
    if n_alpha < 0 or n_beta < 0:
        return np.zeros(0, dtype=np.int64)

    def strings(bits, k):
        return np.array([sum(1 << int(bits[c]) for c in comb)
                         for comb in itertools.combinations(range(len(bits)), k)], dtype=np.int64)

    a = strings(np.flatnonzero(sg == 0), n_alpha)
    b = strings(np.flatnonzero(sg == 1), n_beta)
    if a.size == 0 or b.size == 0:
        return np.zeros(0, dtype=np.int64)
    return np.sort((a[:, None] | b[None, :]).ravel())


def hf_sector(n: int, hf_occ: int, order: str = "interleaved"):
    """(basis, n_alpha, n_beta) of the sector that holds |HF>."""
    sg = spin_of_orbitals(n, order)
    occ = [q for q in range(n) if (int(hf_occ) >> q) & 1]
    na = sum(1 for q in occ if sg[q] == 0)
    nb = len(occ) - na
    return sector_basis(n, na, nb, order), na, nb


def positions(basis: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Position of each basis index of idx in the sorted array basis; raises if one is absent."""
    idx = np.asarray(idx, dtype=np.int64)
    p = np.searchsorted(basis, idx)
    if idx.size and (np.any(p >= basis.size) or np.any(basis[np.minimum(p, basis.size - 1)] != idx)):
        raise ValueError("operator image outside the sector")
    return p


def hf_state(basis: np.ndarray, hf_occ: int) -> np.ndarray:
    psi = np.zeros(basis.size, dtype=np.complex128)
    psi[positions(basis, np.array([hf_occ]))[0]] = 1.0
    return psi


def to_full(n: int, basis: np.ndarray, v: np.ndarray) -> np.ndarray:
    """The 2^n vector with v on the sector and zeros elsewhere (small n only)."""
    out = np.zeros(1 << n, dtype=np.complex128)
    out[basis] = v
    return out


def excitation_pairs(n: int, basis: np.ndarray, row):
    """(pos u, pos v, s) with T_k|u> = s|v>, for every u of the sector.  Only states with the
    annihilated orbitals occupied and the created ones empty can give a non-zero image, so
    the ladder operators are applied to those alone."""
    ops = excitation_ops(row)
    ann = sum(1 << q for q, dagger in ops if not dagger)
    cre = sum(1 << q for q, dagger in ops if dagger)
    cand = basis[((basis & ann) == ann) & ((basis & cre) == 0)]
    src, dst, s = ladder_action(n, ops, src=cand)
    return positions(basis, src), positions(basis, dst), s


def all_pairs(n: int, basis: np.ndarray, exc):
    return [excitation_pairs(n, basis, row) for row in np.asarray(exc).reshape(-1, 4)]


def apply_h(h, g, n: int, basis: np.ndarray, psi, order: str = "interleaved", block: int = 1 << 18):
    """sigma = H psi (Eq. 2) for psi stored on `basis` (one N / S_z sector)."""
    psi = np.asarray(psi, dtype=np.complex128)
    out = np.zeros_like(psi)
    for p in range(n):
        for q in range(n):
            if h[p, q] != 0.0:
                src, dst, sign = ladder_action(n, [(p, True), (q, False)], src=basis)
                if src.size:
                    out[positions(basis, dst)] += h[p, q] * sign * psi[positions(basis, src)]
    pairs = _pairs(n)
    pi = np.array([p for p, _ in pairs])
    qi = np.array([q for _, q in pairs])
    w = 0.5 * (g[pi[:, None], qi[:, None], pi[None, :], qi[None, :]]
               - g[qi[:, None], pi[:, None], pi[None, :], qi[None, :]]
               - g[pi[:, None], qi[:, None], qi[None, :], pi[None, :]]
               + g[qi[:, None], pi[:, None], qi[None, :], pi[None, :]])
    sg = spin_of_orbitals(n, order)
    kind = np.array([sg[p] + sg[q] for p, q in pairs])  # number of beta electrons in the pair
    n_alpha = int(popcount(basis[:1] & sum(1 << q for q in range(n) if sg[q] == 0))[0]) if basis.size else 0
    n_beta = int(popcount(basis[:1] & sum(1 << q for q in range(n) if sg[q] == 1))[0]) if basis.size else 0
    for t in (0, 1, 2):
        mine = kind == t
        if np.any(w[np.ix_(mine, ~mine)] != 0.0) or np.any(w[np.ix_(~mine, mine)] != 0.0):
            raise ValueError("two-body integrals connect pairs of different spin content")
        rows = np.flatnonzero(mine & np.any(w != 0.0, axis=1))
        cols = np.flatnonzero(mine & np.any(w != 0.0, axis=0))
        if rows.size == 0 or cols.size == 0:
            continue
        wt = w[np.ix_(rows, cols)]
        inter = sector_basis(n, n_alpha - (2 - t), n_beta - t, order)
        for lo in range(0, inter.size, block):
            x = inter[lo:lo + block]
            phi = np.zeros((cols.size, x.size), dtype=np.complex128)
            for k, c in enumerate(cols):
                r, s = pairs[c]
                # <x| a_s a_r |y> = <y| a_r^dag a_s^dag |x>
                xs, ys, sign = ladder_action(n, [(r, True), (s, True)], src=x)
                if xs.size:
                    phi[k, np.searchsorted(x, xs)] = sign * psi[positions(basis, ys)]
            xi = wt @ phi
            del phi
            for k, rrow in enumerate(rows):
                p, q = pairs[rrow]
                xs, ys, sign = ladder_action(n, [(p, True), (q, True)], src=x)
                if xs.size:
                    out[positions(basis, ys)] += 1.0 * sign * xi[k, np.searchsorted(x, xs)]
    return out


def energy_of_state(h, g, n, basis, psi, order="interleaved"):
    """<psi|H|psi>: (Re, Im)."""
    e = np.vdot(psi, apply_h(h, g, n, basis, psi, order))
    return float(e.real), float(e.imag)


def trotter_state(n, hf_occ, exc, theta, basis=None, pairs=None, slices=1, order=1,
                  orbital_order="interleaved"):
    """(basis, Trotter product applied to |HF>) on the HF sector."""
    if basis is None:
        basis = hf_sector(n, hf_occ, orbital_order)[0]
    theta = np.asarray(theta, dtype=np.float64)
    seq, scale = trotter_sequence(theta.size, slices, order)
    psi = hf_state(basis, hf_occ)
    for k in seq:
        pk = pairs[k] if pairs is not None else excitation_pairs(n, basis, exc[k])
        psi = apply_factor(psi, pk, scale * theta[k])
    return basis, psi


def energy(h, g, n, hf_occ, exc, theta, basis=None, pairs=None, slices=1, order=1,
           orbital_order="interleaved"):
    """Trotterized UCCSD energy (Eqs. 2-5) computed on the HF sector."""
    basis, psi = trotter_state(n, hf_occ, exc, theta, basis, pairs, slices, order, orbital_order)
    return energy_of_state(h, g, n, basis, psi, orbital_order)[0]


def energy_and_gradient(h, g, n, hf_occ, exc, theta, basis=None, pairs=None, slices=1, order=1,
                        orbital_order="interleaved", return_states=False):
    """(E, dE/dtheta): forward product, lambda = H psi, adjoint sweep over the factors in
    reverse, as ansatz.energy_and_gradient, with every vector on the HF sector.  Without
    `pairs`, each factor's pairs are recomputed when needed (memory stays at a few vectors)."""
    if basis is None:
        basis = hf_sector(n, hf_occ, orbital_order)[0]
    theta = np.asarray(theta, dtype=np.float64)
    exc = np.asarray(exc).reshape(-1, 4)

    def pk(k):
        return pairs[k] if pairs is not None else excitation_pairs(n, basis, exc[k])

    seq, scale = trotter_sequence(theta.size, slices, order)
    _, psi = trotter_state(n, hf_occ, exc, theta, basis, pairs, slices, order, orbital_order)
    lam = apply_h(h, g, n, basis, psi, orbital_order)
    e = np.vdot(psi, lam)
    psi_final = psi.copy()
    grad = np.zeros(theta.size)
    for k in reversed(seq):
        p = pk(k)
        grad[k] += scale * 2.0 * np.vdot(lam, apply_generator(psi, p)).real
        psi = apply_factor(psi, p, -scale * theta[k])
        lam = apply_factor(lam, p, -scale * theta[k])
    if return_states:
        return float(e.real), grad, dict(basis=basis, psi=psi_final, psi_back=psi, im_e=float(e.imag))
    return float(e.real), grad


def trotter_free_energy_and_gradient(h, g, n, hf_occ, exc, theta, ks=(), basis=None, pairs=None,
                                     orbital_order="interleaved"):
    """Trotter-free energy exp(A)|HF>, A = sum_k theta_k G_k (Sec. 3.2), by expm_multiply on
    the sector-restricted generator, and the gradient components listed in ks from the
    Frechet derivative (block-triangular expm_multiply), as trotter_free.py does over 2^n
    states.  Components not listed are NaN."""
    if basis is None:
        basis = hf_sector(n, hf_occ, orbital_order)[0]
    exc = np.asarray(exc).reshape(-1, 4)
    if pairs is None:
        pairs = all_pairs(n, basis, exc)
    theta = np.asarray(theta, dtype=np.float64)
    D = basis.size
    A = generator_matrix(n, exc, theta, pairs, dim=D)
    v = hf_state(basis, hf_occ).real
    psi = scipy.sparse.linalg.expm_multiply(A, v)
    lam = apply_h(h, g, n, basis, psi.astype(np.complex128), orbital_order)
    e = float(np.vdot(psi, lam).real)
    grad = np.full(theta.size, np.nan)
    rhs = np.concatenate([np.zeros(D), v])
    for k in ks:
        Gk = generator_matrix(n, exc[k:k + 1], [1.0], pairs[k:k + 1], dim=D)
        big = scipy.sparse.bmat([[A, Gk], [None, A]], format="csr")
        dpsi = scipy.sparse.linalg.expm_multiply(big, rhs)[:D]
        grad[k] = 2.0 * float(np.vdot(lam, dpsi).real)
    return e, grad
