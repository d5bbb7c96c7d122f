"""Slot rotations and the rotate-and-add aggregation (COUNT / SUM), exact.

Test infrastructure only (see the package docstring).

NSHEDB aggregates a batch-encoded ciphertext by repeated rotation and
addition with a doubling pattern, so that after log2 of the slot count steps
every slot holds the total (Sec. 4.2.2, aggregation: COUNT, SUM).  A rotation
of BFV slots is the ring automorphism sigma_g : a(X) -> a(X^g) (g odd mod
2N) applied to both ciphertext components, followed by key switching from
sigma_g(s) back to s (the library-level method, which the paper leaves to
SEAL).  With the 2 x N/2 slot layout of oracle.encoding, g = 3^r rotates
each half left by r slots and g = 2N - 1 swaps the halves, so rotations by
N/4, N/8, ..., 1 within the halves followed by one swap sum all N slots.
"""
from __future__ import annotations

import numpy as np

from . import bfv
from . import query
from . import ring


def automorphism(poly, g: int) -> np.ndarray:
    """sigma_g(a) for a in Z[X]/(X^N + 1): the term a_i X^i goes to
    a_i X^(i g mod 2N), and X^(N + k) = -X^k."""
    a = ring.as_object(poly)
    n = len(a)
    if g % 2 == 0:
        raise ValueError("g must be odd")
    out = np.zeros(n, dtype=object)
    for i in range(n):
        k = (i * g) % (2 * n)
        if k < n:
            out[k] += a[i]
        else:
            out[k - n] -= a[i]
    return out


def rotation_element(n: int, r: int) -> int:
    """Galois element rotating each half of the slots left by r."""
    return pow(3, r % (n // 2), 2 * n)


def swap_element(n: int) -> int:
    """Galois element exchanging the two halves of the slots."""
    return 2 * n - 1


def sum_elements(n: int) -> list[int]:
    """Galois elements used by sum_slots, in order of use."""
    out = []
    r = n // 4
    while r >= 1:
        out.append(rotation_element(n, r))
        r //= 2
    return out + [swap_element(n)]


def galois_key(params: bfv.Params, sk: bfv.SecretKey, g: int, rnd) -> bfv.RelinKey:
    """Switching key from sigma_g(s) to s (randomness from
    `synth.switch_randomness`)."""
    return bfv.switching_key(params, sk.s, automorphism(sk.s, g), rnd.a, rnd.e)


def apply_galois(params: bfv.Params, key: bfv.RelinKey, ct, g: int) -> tuple:
    """(sigma_g(c0), sigma_g(c1)) decrypts under sigma_g(s); switching the
    second component back to s gives (sigma_g(c0) + k0, k1)."""
    Q = params.Q
    c0 = automorphism(ct[0], g) % Q
    c1 = automorphism(ct[1], g) % Q
    k0, k1 = bfv.key_switch(params, key, c1)
    return ((c0 + k0) % Q, k1 % Q)


def sum_slots(params: bfv.Params, keys: dict, ct) -> tuple:
    """COUNT / SUM: ct <- ct + rot(ct) over sum_elements; every slot of the
    result holds the sum of all slots of ct (mod t)."""
    for g in sum_elements(params.n):
        ct = query.add(params, ct, apply_galois(params, keys[g], ct, g))
    return ct
