"""Batch encoding of N slot values into one plaintext polynomial (client side).

Test infrastructure only (see the package docstring).

NSHEDB packs S = N values into one ciphertext (Sec. 4.1, data storage and
encoding).  With t prime and t = 1 (mod 2N), X^N + 1 splits into N distinct
linear factors (X - zeta) over Z_t, so Z_t[X]/(X^N+1) is isomorphic to Z_t^N
by evaluation at the N primitive 2N-th roots of unity zeta = psi^e, e odd.

Slot order (the paper is silent; slot-wise operations such as EQ do not
depend on it): the 2 x N/2 layout in which slot s < N/2 is the value at
psi^(3^s) and slot N/2 + s the value at psi^(-3^s), exponents mod 2N, so that
the automorphism X -> X^3 rotates each half by one slot and X -> X^(-1) swaps
the halves.  psi is nt.root_of_unity(t, 2N).
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from . import nt


@lru_cache(maxsize=None)
def slot_exponents(n: int) -> tuple[int, ...]:
    """Odd exponent e (mod 2n) whose root psi^e carries slot s."""
    two_n = 2 * n
    half = n // 2
    out = []
    g = 1
    for _ in range(half):
        out.append(g)
        g = g * 3 % two_n
    return tuple(out + [(two_n - e) % two_n for e in out])


def evaluate(poly, t: int) -> list[int]:
    """Slot values of a plaintext polynomial: m(psi^(e_s)) mod t, by Horner,
    straight from the definition (O(N^2); the pin of the fast path)."""
    n = len(poly)
    psi = nt.root_of_unity(t, 2 * n)
    out = []
    for e in slot_exponents(n):
        z = pow(psi, e, t)
        acc = 0
        for c in reversed(list(poly)):
            acc = (acc * z + int(c)) % t
        out.append(acc)
    return out


def _dft_matrix_apply(vec: np.ndarray, t: int, root: int) -> np.ndarray:
    """Cyclic transform X_j = sum_i v_i root^(ij) mod t (radix-2, numpy)."""
    n = len(vec)
    bits = n.bit_length() - 1
    idx = np.arange(n)
    rev = np.zeros(n, dtype=np.int64)
    for b in range(bits):
        rev |= ((idx >> b) & 1) << (bits - 1 - b)
    x = vec.astype(np.int64)[rev]
    pw = np.empty(n, dtype=np.int64)
    pw[0] = 1
    for e in range(1, n):
        pw[e] = pw[e - 1] * root % t
    m = 1
    while m < n:
        tw = pw[(n // (2 * m)) * np.arange(m)]
        y = x.reshape(n // (2 * m), 2, m)
        u = y[:, 0, :]
        v = y[:, 1, :] * tw[None, :] % t
        x = np.stack(((u + v) % t, (u - v) % t), axis=1).reshape(n)
        m *= 2
    return x


def decode(poly, t: int) -> np.ndarray:
    """Slot values m(psi^(e_s)) mod t for every slot s (fast path).

    m(psi^(2k+1)) = sum_i (m_i psi^i) (psi^2)^(ik): a cyclic transform of the
    psi-twisted coefficients; slot s reads index k = (e_s - 1) / 2."""
    n = len(poly)
    psi = nt.root_of_unity(t, 2 * n)
    coeffs = np.array([int(c) % t for c in poly], dtype=np.int64)
    tw = np.array([pow(psi, i, t) for i in range(n)], dtype=np.int64)
    vals = _dft_matrix_apply(coeffs * tw % t, t, psi * psi % t)
    ks = (np.array(slot_exponents(n), dtype=np.int64) - 1) // 2
    return vals[ks]


def encode(slots, t: int) -> np.ndarray:
    """The unique plaintext polynomial (coefficients in [0, t)) whose slot
    values are `slots` mod t: the inverse of `decode`."""
    n = len(slots)
    psi = nt.root_of_unity(t, 2 * n)
    vals = np.zeros(n, dtype=np.int64)
    ks = (np.array(slot_exponents(n), dtype=np.int64) - 1) // 2
    vals[ks] = np.array([int(v) % t for v in slots], dtype=np.int64)
    psi_inv = pow(psi, -1, t)
    n_inv = pow(n, -1, t)
    c = _dft_matrix_apply(vals, t, psi_inv * psi_inv % t)
    untw = np.array([pow(psi_inv, i, t) * n_inv % t for i in range(n)],
                    dtype=np.int64)
    return c * untw % t
