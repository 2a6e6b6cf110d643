"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module only draws numbers and lists indices; it holds none of the
method's arithmetic (no Hamiltonian, no ansatz, no energy).  Both the
HIP path and the CPU oracle consume what it returns.

Conventions (the paper leaves them open, Sec. 2.3):
  * spin orbital q = 2*p + sigma (sigma = 0 alpha, 1 beta), p spatial;
  * qubit q is bit q of a basis-state index (little-endian);
  * the Hartree-Fock reference occupies spin orbitals 0 .. n_elec-1.

Integrals stand in for the paper's FMO fragment integrals (Eq. 2), which
were produced from ABINIT-MP dumps that are not available.
"""
from __future__ import annotations

import itertools

import numpy as np

__all__ = [
    "make_integrals",
    "uccsd_excitations",
    "make_thetas",
    "WORKLOADS",
]


def make_integrals(n_spatial: int, seed: int):
    """Random real active-space integrals with the symmetries of Eq. 2.

    h1: symmetric, off-diagonal N(0, 0.5) averaged with its transpose, then
        -1.5 added to the diagonal.
    h2: chemist-order (pq|rs), drawn N(0, 0.1), averaged over the 8 index
        permutations of real orbitals, then every element in the orbit of
        (pq|pq) is replaced by its absolute value (positive pair-diagonal).
    h1 is drawn before h2 from numpy.random.default_rng(seed).
    """
    ns = int(n_spatial)
    rng = np.random.default_rng(seed)
    a = rng.normal(0.0, 0.5, size=(ns, ns))
    h1 = 0.5 * (a + a.T) - 1.5 * np.eye(ns)
    b = rng.normal(0.0, 0.1, size=(ns, ns, ns, ns))
    perms = (
        b,
        b.transpose(1, 0, 2, 3),
        b.transpose(0, 1, 3, 2),
        b.transpose(1, 0, 3, 2),
        b.transpose(2, 3, 0, 1),
        b.transpose(3, 2, 0, 1),
        b.transpose(2, 3, 1, 0),
        b.transpose(3, 2, 1, 0),
    )
    h2 = sum(perms) / 8.0
    for p in range(ns):
        for q in range(ns):
            v = abs(h2[p, q, p, q])
            h2[p, q, p, q] = v
            h2[q, p, p, q] = v
            h2[p, q, q, p] = v
            h2[q, p, q, p] = v
    return np.ascontiguousarray(h1), np.ascontiguousarray(h2)


def uccsd_excitations(n_qubits: int, n_elec: int) -> np.ndarray:
    """All spin-conserving singles and doubles out of the HF reference.

    Returns an int32 array [K, 4] of spin-orbital indices (i, j, a, b):
    a single i -> a is stored as (i, -1, a, -1); a double is (i, j, a, b)
    with i < j occupied and a < b virtual.  Order (the Trotter order of
    Eq. 5 used by default): singles lexicographic in (i, a), then doubles
    lexicographic in (i, j, a, b), keeping those whose beta count in
    {i, j} equals the beta count in {a, b}.
    """
    occ = list(range(n_elec))
    vir = list(range(n_elec, n_qubits))
    rows = []
    for i in occ:
        for a in vir:
            if (i & 1) == (a & 1):
                rows.append((i, -1, a, -1))
    for i, j in itertools.combinations(occ, 2):
        for a, b in itertools.combinations(vir, 2):
            if (i & 1) + (j & 1) == (a & 1) + (b & 1):
                rows.append((i, j, a, b))
    return np.asarray(rows, dtype=np.int32).reshape(-1, 4)


def make_thetas(n_exc: int, seed: int, scale: float, batch: int | None = None):
    """Amplitudes theta ~ U(-scale, scale).

    With batch=None: one vector from default_rng(seed).
    With batch=B: B vectors, vector b drawn from default_rng(seed + b).
    """
    if batch is None:
        return np.random.default_rng(seed).uniform(-scale, scale, size=n_exc)
    out = np.empty((batch, n_exc))
    for b in range(batch):
        out[b] = np.random.default_rng(seed + b).uniform(-scale, scale, size=n_exc)
    return out


# Workload sizes (qubits, electrons, theta scale).  The 18-qubit batch is the
# throughput workload; the others are parity and serving cases.
WORKLOADS = {
    "h4_8q": dict(n_qubits=8, n_elec=4, seed=0, theta_scale=0.1),
    "h8_16q": dict(n_qubits=16, n_elec=8, seed=0, theta_scale=0.05),
    "dimer_18q_b64": dict(n_qubits=18, n_elec=10, seed=0, theta_scale=0.05, batch=64),
    "monomer_12q": dict(n_qubits=12, n_elec=8, theta_scale=0.05),
    "dimer_18q": dict(n_qubits=18, n_elec=10, theta_scale=0.05),
    "trimer_24q": dict(n_qubits=24, n_elec=14, theta_scale=0.05),
    "large_26q": dict(n_qubits=26, n_elec=14, seed=0, theta_scale=0.05),
}
