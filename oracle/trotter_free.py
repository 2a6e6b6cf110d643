"""Trotter-free UCCSD: |Psi> = exp(sum_k theta_k (T_k - T_k^dag)) |HF>.

Test infrastructure only (see oracle/__init__.py).

Sec. 3.2 (with Table 6 and Table S3) contrasts the Trotterized ansatz with
the exponential of the whole anti-Hermitian cluster operator acting on |HF>,
computed without any product formula by SciPy's expm_multiply (the action of
a matrix exponential on a vector).  This module computes the same thing the
same way: the generator

    A = sum_k theta_k G_k,   G_k = T_k - T_k^dag

is assembled as a sparse matrix over all 2^n basis states from the
ladder-operator pairs of each excitation (wherever T_k|u> = s|v>, G_k maps
u -> s v and v -> -s u, so A[v, u] += theta_k s and A[u, v] -= theta_k s),
and exp(A) |HF> comes from scipy.sparse.linalg.expm_multiply.  The energy is
<Psi|H|Psi> with the ladder-operator Hamiltonian of Eq. 2.

Pinned by: scipy.linalg.expm of the dense Kronecker-built generator, the
closed-form rotation of a single excitation, the product of pairwise
commuting factors, the limit of Trotter products (error ~ 1/M), unitarity,
time reversal, and additivity over non-interacting fragments.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse
import scipy.sparse.linalg

from .ansatz import all_pairs, hf_state
from .hamiltonian import energy as _energy


def generator_matrix(n, exc, theta, pairs=None):
    """Sparse A = sum_k theta_k (T_k - T_k^dag) over the 2^n basis states (CSR, float64)."""
    if pairs is None:
        pairs = all_pairs(n, exc)
    theta = np.asarray(theta, dtype=np.float64)
    rows, cols, vals = [], [], []
    for (u, v, s), t in zip(pairs, theta):
        s = np.asarray(s, dtype=np.float64)
        rows += [v, u]
        cols += [u, v]
        vals += [t * s, -t * s]
    if not rows:
        return scipy.sparse.csr_matrix((1 << n, 1 << n))
    A = scipy.sparse.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                shape=(1 << n, 1 << n))
    return A.tocsr()


def trotter_free_state(n, hf_occ, exc, theta, pairs=None, psi0=None):
    """exp(A) psi0 (psi0 = |HF> by default) by expm_multiply."""
    A = generator_matrix(n, exc, theta, pairs)
    v = hf_state(n, hf_occ) if psi0 is None else np.asarray(psi0, dtype=np.complex128)
    # A is real: apply it to the real and imaginary parts separately
    re = scipy.sparse.linalg.expm_multiply(A, v.real.copy())
    im = scipy.sparse.linalg.expm_multiply(A, v.imag.copy()) if np.any(v.imag) else np.zeros_like(re)
    return re + 1j * im


def trotter_free_energy(h, g, n, hf_occ, exc, theta, pairs=None):
    """<Psi|H|Psi> for the Trotter-free state."""
    return _energy(h, g, trotter_free_state(n, hf_occ, exc, theta, pairs))[0]
