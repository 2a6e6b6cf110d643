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
    "magnitude_order",
    "fragment_orbitals",
    "fragment_integrals",
    "delocalizing_rotation",
    "rotate_integrals",
    "embed_amplitudes",
    "rotate_amplitudes",
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


def magnitude_order(h1, h2, n_elec: int, exc) -> np.ndarray:
    """Permutation of the excitation list into decreasing magnitude of a first-order estimate
    of each amplitude (the magnitude ordering the paper's circuits use, Sec. 2.3): singles
    f_ai / (f_ii - f_aa), doubles <ij||ab> / (f_ii + f_jj - f_aa - f_bb), with the Fock
    matrix of the reference f_pq = h_pq + sum_{k occupied} (<pk|qk> - <pk|kq>) in spin
    orbitals (<pq|rs> = (pr|qs) for matching spins).  Equal magnitudes keep the list order.
    Apply as exc[perm] (and theta[perm])."""
    exc = np.asarray(exc)
    ns = h1.shape[0]
    n = 2 * ns
    sp = np.arange(n) // 2
    sg = np.arange(n) % 2

    def g(p, q, r, s_):  # <pq|rs> in spin orbitals
        if sg[p] != sg[r] or sg[q] != sg[s_]:
            return 0.0
        return h2[sp[p], sp[r], sp[q], sp[s_]]

    f = np.zeros((n, n))
    for p in range(n):
        for q in range(n):
            v = h1[sp[p], sp[q]] if sg[p] == sg[q] else 0.0
            for k in range(n_elec):
                v += g(p, k, q, k) - g(p, k, k, q)
            f[p, q] = v
    est = np.empty(len(exc))
    for m, (i, j, a, b) in enumerate(exc):
        if j < 0:
            num, den = f[a, i], f[i, i] - f[a, a]
        else:
            num = g(i, j, a, b) - g(i, j, b, a)
            den = f[i, i] + f[j, j] - f[a, a] - f[b, b]
        est[m] = abs(num) / max(abs(den), 1e-8)
    return np.argsort(-est, kind="stable")


# ---------------------------------------------------------------- fragment systems
# Inputs of the size-consistency experiment of Sec. 3.2 (Table 6): identical fragments far
# apart (no integral couples two of them), described either by orbitals localized on the
# fragments (LMO) or by orbitals delocalized over a pair (CMO).  These functions only lay out
# and rotate the inputs (integrals and the amplitudes of one cluster operator written in
# another orbital basis); the energies come from the oracle or the GPU path.


def fragment_orbitals(n_frag: int, ns_frag: int, nocc_frag: int) -> np.ndarray:
    """Spatial index, in the combined system, of orbital p of fragment f ([n_frag, ns_frag]):
    all fragments' occupied orbitals first (fragment by fragment), then all virtual ones, so
    the combined Hartree-Fock reference is the lowest orbitals."""
    out = np.empty((n_frag, ns_frag), dtype=np.int64)
    nv = ns_frag - nocc_frag
    for f in range(n_frag):
        for p in range(ns_frag):
            out[f, p] = f * nocc_frag + p if p < nocc_frag else n_frag * nocc_frag + f * nv + (p - nocc_frag)
    return out


def fragment_integrals(frags, nocc_frag: int):
    """Block-diagonal (h1, h2) of non-interacting fragments [(h1_f, h2_f), ...] of equal size,
    in the orbital layout of fragment_orbitals."""
    nf, ns = len(frags), frags[0][0].shape[0]
    m = fragment_orbitals(nf, ns, nocc_frag)
    N = nf * ns
    h1 = np.zeros((N, N))
    h2 = np.zeros((N, N, N, N))
    for f, (a1, a2) in enumerate(frags):
        ix = m[f]
        h1[np.ix_(ix, ix)] = a1
        h2[np.ix_(ix, ix, ix, ix)] = a2
    return h1, h2


def delocalizing_rotation(ns_frag: int, nocc_frag: int) -> np.ndarray:
    """Orthogonal U of two fragments (spatial, old orbital x new orbital): orbital p of A and
    of B become (A_p + B_p) / sqrt(2) and (A_p - B_p) / sqrt(2).  Occupied orbitals mix only
    with occupied ones and virtual with virtual, so the Hartree-Fock determinant is unchanged
    (up to sign); the new order is occupied pairs, then virtual pairs."""
    m = fragment_orbitals(2, ns_frag, nocc_frag)
    U = np.zeros((2 * ns_frag, 2 * ns_frag))
    r = 1.0 / np.sqrt(2.0)
    for p in range(ns_frag):
        base = 2 * p if p < nocc_frag else 2 * nocc_frag + 2 * (p - nocc_frag)
        a, b = m[0, p], m[1, p]
        U[a, base], U[b, base] = r, r
        U[a, base + 1], U[b, base + 1] = r, -r
    return U


def rotate_integrals(h1, h2, U):
    """Integrals over the orbitals phi'_q = sum_p U[p, q] phi_p (real, chemist order)."""
    h1r = U.T @ h1 @ U
    h2r = np.einsum("pqrs,pa,qb,rc,sd->abcd", h2, U, U, U, U, optimize=True)
    return np.ascontiguousarray(h1r), np.ascontiguousarray(h2r)


def embed_amplitudes(exc_frag, thetas_frag, n_frag: int, ns_frag: int, nocc_frag: int, exc_all):
    """Amplitudes over the combined excitation list exc_all: each fragment's excitation
    (rows of exc_frag, fragment spin-orbital indices) carries that fragment's amplitude, every
    other excitation (those across fragments) 0."""
    m = fragment_orbitals(n_frag, ns_frag, nocc_frag)
    index = {tuple(int(x) for x in r): k for k, r in enumerate(np.asarray(exc_all))}
    out = np.zeros(len(exc_all))
    for f in range(n_frag):
        so = lambda q: -1 if q < 0 else 2 * int(m[f, q // 2]) + (q & 1)  # noqa: E731
        for r, t in zip(np.asarray(exc_frag), thetas_frag[f]):
            out[index[tuple(so(int(q)) for q in r)]] = t
    return out


def rotate_amplitudes(exc, theta, U):
    """The same cluster operator written in the rotated orbitals (U as in rotate_integrals,
    spin-free, occupied and virtual spaces each mapped to themselves).  T1 = sum t_ai a_a^+ a_i
    and T2 = (1/4) sum tau_abij a_a^+ a_b^+ a_j a_i (tau antisymmetric, tau_abij = theta of
    row (i, j, a, b) for i < j, a < b) transform as tensors; the result is read back on the
    same list of excitations, which holds every non-zero element."""
    exc = np.asarray(exc)
    n = 2 * U.shape[0]
    Us = np.zeros((n, n))
    Us[0::2, 0::2] = U
    Us[1::2, 1::2] = U
    t1 = np.zeros((n, n))
    tau = np.zeros((n, n, n, n))
    for (i, j, a, b), t in zip(exc, theta):
        if j < 0:
            t1[a, i] = t
        else:
            tau[a, b, i, j], tau[b, a, i, j], tau[a, b, j, i], tau[b, a, j, i] = t, -t, -t, t
    t1r = Us.T @ t1 @ Us
    taur = np.einsum("abij,aA,bB,iI,jJ->ABIJ", tau, Us, Us, Us, Us, optimize=True)
    out = np.empty(len(exc))
    for k, (i, j, a, b) in enumerate(exc):
        out[k] = t1r[a, i] if j < 0 else taur[a, b, i, j]
    # nothing outside the list
    rest1 = t1r.copy()
    rest2 = taur.copy()
    for i, j, a, b in exc:
        if j < 0:
            rest1[a, i] = 0.0
        else:
            rest2[a, b, i, j] = rest2[b, a, i, j] = rest2[a, b, j, i] = rest2[b, a, j, i] = 0.0
    if max(np.max(np.abs(rest1)), np.max(np.abs(rest2))) > 1e-12:
        raise ValueError("rotated cluster operator has terms outside the excitation list")
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
