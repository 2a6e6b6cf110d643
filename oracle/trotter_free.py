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

The gradient dE/dtheta_k = 2 Re <H Psi| (d/dtheta_k exp(A)) |HF> uses the
Frechet derivative of the matrix exponential in direction G_k, read from the
block-triangular identity exp([[A, G], [0, A]]) = [[exp(A), L(A, G)], [0, exp(A)]]
(Van Loan): expm_multiply of the doubled sparse matrix applied to [0; |HF>]
returns [L(A, G_k)|HF>; exp(A)|HF>].

Pinned by: scipy.linalg.expm of the dense Kronecker-built generator, the
closed-form rotation of a single excitation, the product of pairwise
commuting factors, the limit of Trotter products (error ~ 1/M), unitarity,
time reversal, and additivity over non-interacting fragments; the gradient
by central differences, the Slater-Condon gradient at theta = 0 and the
Trotterized gradient of commuting excitations.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse
import scipy.sparse.linalg

from .ansatz import all_pairs, hf_state
from .hamiltonian import apply_h, energy as _energy


def generator_matrix(n, exc, theta, pairs=None, dim=None):
    """Sparse A = sum_k theta_k (T_k - T_k^dag) over the 2^n basis states (CSR, float64).
    With dim, pairs index a basis of dim states (a sector) instead of all 2^n."""
    if pairs is None:
        pairs = all_pairs(n, exc)
    N = (1 << n) if dim is None else int(dim)
    theta = np.asarray(theta, dtype=np.float64)
    rows, cols, vals = [], [], []
    for (u, v, s), t in zip(pairs, theta):
        s = np.asarray(s, dtype=np.float64)
        rows += [v, u]
        cols += [u, v]
        vals += [t * s, -t * s]
    if not rows:
        return scipy.sparse.csr_matrix((N, N))
    A = scipy.sparse.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                shape=(N, N))
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


def trotter_free_energy_and_gradient(h, g, n, hf_occ, exc, theta, pairs=None, ks=None):
    """(E, dE/dtheta) of the Trotter-free ansatz; each component from the Frechet derivative
    of exp(A) in direction G_k (block-triangular expm_multiply, see the module header).  With
    ks, only those components are computed (the others are NaN)."""
    if pairs is None:
        pairs = all_pairs(n, exc)
    theta = np.asarray(theta, dtype=np.float64)
    A = generator_matrix(n, exc, theta, pairs)
    v = hf_state(n, hf_occ).real
    psi = scipy.sparse.linalg.expm_multiply(A, v)
    lam = apply_h(h, g, psi.astype(np.complex128))
    e = float(np.vdot(psi, lam).real)
    N = 1 << n
    grad = np.full(theta.size, np.nan)
    rhs = np.concatenate([np.zeros(N), v])
    for k in (range(theta.size) if ks is None else ks):
        Gk = generator_matrix(n, exc[k:k + 1], [1.0], pairs[k:k + 1])
        big = scipy.sparse.bmat([[A, Gk], [None, A]], format="csr")
        dpsi = scipy.sparse.linalg.expm_multiply(big, rhs)[:N]
        grad[k] = 2.0 * float(np.vdot(lam, dpsi).real)
    return e, grad
