"""Fermionic ladder operators on computational-basis states.

Test infrastructure only (see oracle/__init__.py).

Convention (Jordan-Wigner, the mapping this path uses in place of the
paper's SCBKT, Sec. 2.3): spin orbital q is bit q of the basis index, bit
value 1 = occupied, and

    a_q |x> = (-1)^{#occupied orbitals below q in x} |x with bit q cleared>
              if bit q of x is set, else 0,
    a_q^dagger |x> = same sign, bit q set, if bit q of x is clear, else 0.

Pinned by: tests/test_oracle_pins.py (dense Kronecker construction of the
same operators, anticommutation relations, Slater-Condon closed forms).
"""
from __future__ import annotations

import numpy as np


def popcount(x: np.ndarray) -> np.ndarray:
    return np.bitwise_count(x)


def ladder_action(n: int, ops, src=None):
    """Action of an operator product on basis states.

    ops: sequence of (q, dagger) written left to right as in the product
         o_1 o_2 ... o_m; the rightmost factor acts first.
    src: optional array of basis indices to act on (default: all 2^n).

    Returns (src, dst, sign): for every basis index src on which the product
    is non-zero, product |src> = sign |dst>.  sign is an int64 array of +-1.
    """
    if src is None:
        src = np.arange(1 << n, dtype=np.int64)
    else:
        src = np.asarray(src, dtype=np.int64)
    y = src.copy()
    sign = np.ones(src.shape, dtype=np.int64)
    alive = np.ones(src.shape, dtype=bool)
    for q, dagger in reversed(list(ops)):
        bit = (y >> q) & 1
        if dagger:
            alive &= bit == 0
        else:
            alive &= bit == 1
        below = popcount(y & ((1 << q) - 1)) & 1
        sign = np.where(below == 1, -sign, sign)
        y = y ^ (1 << q)
    return src[alive], y[alive], sign[alive]


def apply_product(n: int, ops, psi: np.ndarray, coeff=1.0, out=None):
    """out += coeff * (o_1 ... o_m) psi.  The map src -> dst is injective."""
    if out is None:
        out = np.zeros_like(psi)
    src, dst, sign = ladder_action(n, ops)
    if src.size:
        out[dst] += coeff * sign * psi[src]
    return out
