"""Closed-form values at theta = 0 (textbook Slater-Condon rules).

Test infrastructure only (see oracle/__init__.py).

At theta = 0 the ansatz state is |HF> (Eq. 3), so
    E(0) = E_HF = 2 sum_i h_ii + sum_ij [2 (ii|jj) - (ij|ji)]
over the n_elec/2 doubly occupied spatial orbitals (closed shell), and,
since G_k|HF> = T_k|HF> and <HF|T_k = 0,
    dE/dtheta_k (0) = 2 <HF| H T_k |HF>
which the Slater-Condon rules give without any qubit mapping:
    single i->a:      2 (h_ia + sum_{m occ} <im||am>)
    double ij->ab:    2 <ij||ab>,  <pq||rs> = <pq|rs> - <pq|sr>
for T = a_a^dag a_i and T = a_a^dag a_b^dag a_j a_i (Eq. 4).
"""
from __future__ import annotations

import numpy as np


def hf_energy_spatial(h1, h2, n_elec):
    occ = range(n_elec // 2)
    e = 0.0
    for i in occ:
        e += 2.0 * h1[i, i]
        for j in occ:
            e += 2.0 * h2[i, i, j, j] - h2[i, j, j, i]
    return e


def gradient_at_zero(h, g, occ, exc):
    """Spin-orbital Slater-Condon values of 2 <HF|H T_k|HF>."""
    occ = list(occ)
    out = []
    for row in np.asarray(exc).reshape(-1, 4):
        i, j, a, b = (int(x) for x in row)
        if j < 0:
            f = h[i, a] + sum(g[i, m, a, m] - g[i, m, m, a] for m in occ)
            out.append(2.0 * f)
        else:
            out.append(2.0 * (g[i, j, a, b] - g[i, j, b, a]))
    return np.array(out)
