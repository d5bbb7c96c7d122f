"""Range comparisons (LT, LE, BETWEEN) over the equality machinery, exact.

Test infrastructure only (see the package docstring).

The paper defines x < y as the membership of z = x - y in the negative half
A = {-(p-1)/2, ..., -1} of Z_p, written as a sum of Fermat equalities
(Eq. eq:inequality): LT = sum over a in A of 1 - (z - a)^(p-1).  It is valid
when |x - y| <= (p-1)/2 (larger differences wrap around; a limit the paper
leaves implicit).  Expanding each term with C(p-1, k) = (-1)^k (mod p) makes
that sum one polynomial f(z) = sum_k c_k z^k of degree p - 1 with
c_k = -sum_{a in A} a^(p-1-k) (mod p) for k >= 1 and c_0 = 0; the
coefficients of even k < p - 1 vanish (the half-range power sums of even
exponent are half of a full-range sum, which is 0), and c_(p-1) = -(p-1)/2.
So f(z) = c_(p-1) z^(p-1) + z g(z^2) with g of degree (p-3)/2.  The paper
evaluates comparisons with the optimization it cites (a polynomial
evaluation); the reading taken here is baby-step giant-step evaluation of
g, with every power of z^2 that is a power of two taken from the equality
chain's squarings:

  levels[a] = z^(2^a), a = 0..K (p = 2^K + 1: the EQ chain);
  w = levels[1]; babies B_i = w^i, i < k (B_0 the trivial encryption of 1,
  powers of two from the chain, others B_h * B_(i-h), h the largest power
  of two below i); giants W_j = w^(k j), j < m (powers of two from the
  chain, others W_h * W_(j-h)); k = 2^ceil((K-1)/2), m = 2^(K-1) / k;
  G_j = sum_i c_(2(jk+i)+1) B_i (scalar products, centred coefficients);
  g = G_0 + sum_{j>=1} G_j * W_j, the m - 1 products' exact tensors added
  before one scale-and-round and one relinearization (bfv.mul_sum_relin);
  LT = c_(p-1) levels[K] + z * g.

LE(x, y) = 1 - LT(y, x); BETWEEN(x, lo, hi) = LE(lo, x) * LE(x, hi), the
product of two comparisons (Sec. 4.2.2, BETWEEN).

This program is fixed: the device evaluates exactly these products in this
order (same k, m, factorizations and summed giant-step tensors), so that its
ciphertexts equal the oracle's bit for bit at every size, and its
multiplicative depth (18 at p = 65537, before the scalar combination; one
more for BETWEEN) is what the library's depth budget charges.  A change to
the program is a change to both sides and to their stored digests.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from . import bfv
from . import nt
from . import query
from . import ring


# ----------------------------------------------------- plaintext algebra ---

def negative_half(p: int) -> list[int]:
    """A = {-(p-1)/2, ..., -1} as residues mod p."""
    return [(-a) % p for a in range(1, (p - 1) // 2 + 1)]


def lt_coefficients_direct(p: int) -> list[int]:
    """c_0..c_(p-1) of f(z) = sum_{a in A} (1 - (z - a)^(p-1)) mod p, from the
    binomial expansion: c_k = -sum_a a^(p-1-k) for k >= 1, c_0 = |A| - sum_a
    a^(p-1) = 0.  O(p^2): small p only."""
    A = negative_half(p)
    c = [0] * p
    c[0] = (len(A) - sum(pow(a, p - 1, p) for a in A)) % p
    for k in range(1, p):
        c[k] = (-sum(pow(a, p - 1 - k, p) for a in A)) % p
    return c


def _cyclic_dft(x: np.ndarray, root: int, p: int) -> np.ndarray:
    """y_k = sum_e x_e root^(e k) mod p for a power-of-two length (radix-2
    decimation in time, numpy int64; p < 2^31)."""
    n = len(x)
    if n == 1:
        return x % p
    even = _cyclic_dft(x[0::2], root * root % p, p)
    odd = _cyclic_dft(x[1::2], root * root % p, p)
    tw = np.ones(n // 2, dtype=np.int64)
    for e in range(1, n // 2):
        tw[e] = tw[e - 1] * root % p
    t = odd * tw % p
    return np.concatenate([(even + t) % p, (even - t) % p])


@lru_cache(maxsize=None)
def lt_coefficients(p: int) -> tuple[int, ...]:
    """The same coefficients for any Fermat prime p, via the multiplicative
    group: with gamma a primitive root and F = [z in A], c_k = -sum_{e}
    F(gamma^e) gamma^(-e k) for 1 <= k <= p-2 (the sum over z != 0 of F(z)
    z^(-k)), c_(p-1) = -|A|, c_0 = F(0) = 0; the sum over e is a cyclic
    transform of length p - 1 = 2^K."""
    g = nt.primitive_root(p)
    A = set(negative_half(p))
    F = np.zeros(p - 1, dtype=np.int64)
    z = 1
    for e in range(p - 1):
        F[e] = 1 if z in A else 0
        z = z * g % p
    Y = _cyclic_dft(F, pow(g, p - 2, p), p)
    c = [0] * p
    for k in range(1, p - 1):
        c[k] = int(-Y[k]) % p
    c[p - 1] = (-len(A)) % p
    return tuple(c)


def eval_poly(c: list[int], z: int, p: int) -> int:
    acc = 0
    for ck in reversed(c):
        acc = (acc * z + ck) % p
    return acc


def centred(v: int, p: int) -> int:
    v %= p
    return v - p if v > p // 2 else v


def shape(p: int) -> tuple[int, int, int]:
    """(K, k, m): p = 2^K + 1, k babies and m giants with k m = 2^(K-1)."""
    K = (p - 1).bit_length() - 1
    if (1 << K) + 1 != p or K < 2:
        raise ValueError("p must be a Fermat prime 2^K + 1 with K >= 2")
    kb = (K - 1 + 1) // 2
    return K, 1 << kb, 1 << (K - 1 - kb)


def _split(i: int) -> tuple[int, int]:
    h = 1 << (i.bit_length() - 1)
    return h, i - h


def lt_program_plain(p: int, z: int) -> int:
    """The evaluation program of the module docstring run on one residue z
    mod p (no encryption): must equal f(z)."""
    K, k, m = shape(p)
    c = lt_coefficients(p)
    levels = [z % p]
    for _ in range(K):
        levels.append(levels[-1] * levels[-1] % p)
    babies = [1, levels[1]]
    for i in range(2, k):
        h, r = _split(i)
        babies.append(levels[h.bit_length()] if r == 0 else babies[h] * babies[r] % p)
    giants = [1, levels[(k).bit_length()]]
    for j in range(2, m):
        h, r = _split(j)
        giants.append(levels[k.bit_length() + h.bit_length() - 1] if r == 0
                      else giants[h] * giants[r] % p)
    g = 0
    for j in range(m):
        Gj = sum(centred(c[2 * (j * k + i) + 1], p) * babies[i] for i in range(k)) % p
        g = (g + Gj * giants[j]) % p
    return (centred(c[p - 1], p) * levels[K] + levels[0] * g) % p


# ------------------------------------------------------------ ciphertexts ---

def trivial_one(params: bfv.Params) -> tuple:
    """The trivial encryption (Delta, 0) of the constant 1."""
    c0 = np.zeros(params.n, dtype=object)
    c0[0] = params.delta
    return (c0, np.zeros(params.n, dtype=object))


def scalar_mul(params: bfv.Params, ct, c: int) -> tuple:
    """c * ct for an integer c: [c c0]_Q, [c c1]_Q (encrypts c m)."""
    Q = params.Q
    return tuple((ring.as_object(a) * c) % Q for a in ct)


def lincomb(params: bfv.Params, cts, coeffs) -> tuple:
    """[sum_i coeffs_i * cts_i]_Q, component-wise (exact)."""
    Q = params.Q
    out = None
    for ct, c in zip(cts, coeffs):
        term = tuple(ring.as_object(a) * c for a in ct)
        out = term if out is None else tuple(u + v for u, v in zip(out, term))
    return tuple(u % Q for u in out)


def lt(params: bfv.Params, rk: bfv.RelinKey, x, y) -> tuple:
    """Encrypted [x < y] for |x - y| <= (p-1)/2 (Eq. eq:inequality), by the
    program of the module docstring."""
    p = params.t
    K, k, m = shape(p)
    c = lt_coefficients(p)
    z = bfv.sub(params, x, y)
    levels = [z]
    for _ in range(K):
        levels.append(bfv.square_relin(params, rk, levels[-1]))
    babies = [trivial_one(params), levels[1]]
    for i in range(2, k):
        h, r = _split(i)
        babies.append(levels[h.bit_length()] if r == 0
                      else bfv.mul_relin(params, rk, babies[h], babies[r]))
    giants = [None, levels[k.bit_length()]]
    for j in range(2, m):
        h, r = _split(j)
        giants.append(levels[k.bit_length() + h.bit_length() - 1] if r == 0
                      else bfv.mul_relin(params, rk, giants[h], giants[r]))
    # g = G_0 + sum_{j >= 1} G_j W_j, the products' tensors summed before one
    # scale-and-round and one relinearization (bfv.mul_sum_relin)
    G = [lincomb(params, babies, [centred(c[2 * (j * k + i) + 1], p) for i in range(k)])
         for j in range(m)]
    g = G[0]
    if m > 1:
        g = query.add(params, g, bfv.mul_sum_relin(params, rk,
                                                   [(G[j], giants[j]) for j in range(1, m)]))
    return query.add(params, scalar_mul(params, levels[K], centred(c[p - 1], p)),
                     bfv.mul_relin(params, rk, z, g))


def le(params: bfv.Params, rk: bfv.RelinKey, x, y) -> tuple:
    """Encrypted [x <= y] = 1 - LT(y, x)."""
    return bfv.sub(params, trivial_one(params), lt(params, rk, y, x))


def between(params: bfv.Params, rk: bfv.RelinKey, x, lo, hi) -> tuple:
    """Encrypted [lo <= x <= hi] = LE(lo, x) * LE(x, hi) (Sec. 4.2.2)."""
    return bfv.mul_relin(params, rk, le(params, rk, lo, x), le(params, rk, x, hi))
