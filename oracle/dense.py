"""Dense-matrix constructions for small systems (n <= ~10 qubits).

Test infrastructure only (see oracle/__init__.py).

These build the same objects as fermion/hamiltonian/ansatz by a different
route (Kronecker products of 2x2 matrices, scipy.linalg.expm,
numpy.linalg.eigh), so that each can pin the other.

    a_q = Z x ... x Z x sigma^- x I x ... x I   (Z on qubits 0..q-1)

with qubit q = bit q of the index; numpy.kron puts its first factor on the
most significant bit, so the factors are listed from qubit n-1 down to 0.
"""
from __future__ import annotations

import itertools
from functools import reduce

import numpy as np
import scipy.linalg

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
LOWER = np.array([[0, 1], [0, 0]], dtype=np.complex128)  # |0><1|: empties an occupied orbital
PAULI = {"I": I2, "X": X, "Y": Y, "Z": Z}


def annihilator(n, q):
    factors = []
    for k in range(n - 1, -1, -1):
        if k > q:
            factors.append(I2)
        elif k == q:
            factors.append(LOWER)
        else:
            factors.append(Z)
    return reduce(np.kron, factors)


def ladder_ops(n):
    a = [annihilator(n, q) for q in range(n)]
    ad = [m.conj().T for m in a]
    return a, ad


def hamiltonian_dense(h, g):
    """Eq. 2 as a dense 2^n x 2^n matrix."""
    n = h.shape[0]
    a, ad = ladder_ops(n)
    H = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for p in range(n):
        for q in range(n):
            if h[p, q] != 0.0:
                H += h[p, q] * (ad[p] @ a[q])
    for p in range(n):
        for q in range(n):
            pq = ad[p] @ ad[q]
            for r in range(n):
                for s in range(n):
                    if g[p, q, r, s] != 0.0:
                        H += 0.5 * g[p, q, r, s] * (pq @ a[s] @ a[r])
    return H


def generator_dense(n, row):
    """G_k = T_k - T_k^dag for one excitation row (i, j, a, b)."""
    a, ad = ladder_ops(n)
    i, j, aa, bb = (int(x) for x in row)
    if j < 0:
        T = ad[aa] @ a[i]
    else:
        T = ad[aa] @ ad[bb] @ a[j] @ a[i]
    return T - T.conj().T


def trotter_state_dense(n, hf_occ, exc, theta):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[int(hf_occ)] = 1.0
    for row, t in zip(np.asarray(exc).reshape(-1, 4), theta):
        psi = scipy.linalg.expm(t * generator_dense(n, row)) @ psi
    return psi


def number_and_sz(n, order="interleaved"):
    idx = np.arange(1 << n)
    bits = (idx[:, None] >> np.arange(n)[None, :]) & 1
    if order == "interleaved":
        beta = np.arange(n) % 2
    else:
        beta = (np.arange(n) >= n // 2).astype(int)
    n_b = (bits * beta[None, :]).sum(1)
    n_tot = bits.sum(1)
    return n_tot, n_tot - 2 * n_b  # (N, 2 Sz)


def fci_energy(H, n, n_elec, order="interleaved"):
    """Lowest eigenvalue of H in the N = n_elec, S_z = 0 sector (CAS-CI analog)."""
    n_tot, two_sz = number_and_sz(n, order)
    sel = np.flatnonzero((n_tot == n_elec) & (two_sz == 0))
    sub = H[np.ix_(sel, sel)]
    return float(np.linalg.eigvalsh(sub)[0])


def pauli_matrix(label):
    """label[q] is the Pauli on qubit q."""
    return reduce(np.kron, [PAULI[c] for c in reversed(label)])


def pauli_decompose(M, tol=1e-12):
    """{label: coeff} with M = sum coeff * P_label (brute force over 4^n)."""
    n = int(np.log2(M.shape[0]))
    out = {}
    for labels in itertools.product("IXYZ", repeat=n):
        lab = "".join(labels)
        c = np.trace(pauli_matrix(lab).conj().T @ M) / (1 << n)
        if abs(c) > tol:
            out[lab] = c
    return out
