"""Exact arithmetic in Z[X]/(X^N + 1) for the oracle.

Test infrastructure only (see the package docstring).

Polynomials are numpy object arrays (or sequences) of Python ints, lowest
degree first.  Two product routines:

* `negacyclic_schoolbook` - the definition: c_k = sum_{i+j=k} a_i b_j
  - sum_{i+j=k+N} a_i b_j.  O(N^2), for small N and as the pin of the other.
* `negacyclic_product` / `negacyclic_dot` - the same exact integer result via
  the oracle's own residue basis (31-bit NTT primes, unrelated to any device
  basis): reduce, multiply with a negacyclic NTT in numpy int64, and return
  to integers by the Chinese remainder theorem.  Products of two residues are
  below 2^62, so int64 numpy arithmetic is exact.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from . import nt

# The oracle's own basis: primes below 2^31 that are 1 mod 2^16 (so every
# power-of-two N <= 2^15 has a negacyclic NTT).  Several hundred exist; a
# product bounded by 2^B needs about B/31 of them.
_OWN_STEP = 1 << 16
_OWN_MAX = 120


@lru_cache(maxsize=None)
def own_primes() -> tuple[int, ...]:
    return tuple(nt.primes_congruent_one_below(1 << 31, _OWN_STEP, _OWN_MAX))


def as_object(a) -> np.ndarray:
    """Coerce a polynomial to a 1-D object array of Python ints."""
    if isinstance(a, np.ndarray) and a.dtype == object:
        return a
    return np.array([int(x) for x in a], dtype=object)


def negacyclic_schoolbook(a, b) -> np.ndarray:
    """c = a * b mod (X^N + 1), straight from the definition (pure Python)."""
    n = len(a)
    if len(b) != n:
        raise ValueError("length mismatch")
    c = [0] * n
    for i in range(n):
        ai = int(a[i])
        if ai == 0:
            continue
        for j in range(n):
            k = i + j
            if k < n:
                c[k] += ai * int(b[j])
            else:
                c[k - n] -= ai * int(b[j])
    return np.array(c, dtype=object)


def _bitrev_perm(n: int) -> np.ndarray:
    bits = n.bit_length() - 1
    idx = np.arange(n)
    rev = np.zeros(n, dtype=np.int64)
    for b in range(bits):
        rev |= ((idx >> b) & 1) << (bits - 1 - b)
    return rev


def _powers(base: np.ndarray, p: np.ndarray, n: int) -> np.ndarray:
    """[k, n] table of base^e mod p for e < n (row-wise base and p)."""
    out = np.empty((len(p), n), dtype=np.int64)
    out[:, 0] = 1
    for e in range(1, n):
        out[:, e] = out[:, e - 1] * base % p
    return out


@lru_cache(maxsize=None)
def _tables(primes: tuple[int, ...], n: int):
    """Twist and twiddle tables for a negacyclic NTT of length n per prime.

    psi is a primitive 2n-th root of unity mod p; the negacyclic transform is
    the cyclic transform (omega = psi^2) of the psi-twisted input."""
    p = np.array(primes, dtype=np.int64)
    psi = np.array([nt.root_of_unity(q, 2 * n) for q in primes], dtype=np.int64)
    psi_inv = np.array([pow(int(x), -1, q) for x, q in zip(psi, primes)],
                       dtype=np.int64)
    n_inv = np.array([pow(n, -1, q) for q in primes], dtype=np.int64)
    twist = _powers(psi, p, n)
    untwist = _powers(psi_inv, p, n) * n_inv[:, None] % p[:, None]
    omega = _powers(psi * psi % p, p, n)
    omega_inv = _powers(psi_inv * psi_inv % p, p, n)
    return p, twist, untwist, omega, omega_inv, _bitrev_perm(n)


def _cyclic_ntt(x: np.ndarray, p: np.ndarray, wpow: np.ndarray,
                rev: np.ndarray) -> np.ndarray:
    """Iterative radix-2 decimation-in-time transform, X_j = sum_i x_i w^(ij),
    on each row (bit-reversed input order, natural output order)."""
    k, n = x.shape
    x = x[:, rev]
    pc = p[:, None, None]
    m = 1
    while m < n:
        tw = wpow[:, (n // (2 * m)) * np.arange(m)]          # w_{2m}^j
        y = x.reshape(k, n // (2 * m), 2, m)
        u = y[:, :, 0, :]
        v = y[:, :, 1, :] * tw[:, None, :] % pc
        x = np.stack(((u + v) % pc, (u - v) % pc), axis=2).reshape(k, n)
        m *= 2
    return x


def _residues(a: np.ndarray, primes: tuple[int, ...]) -> np.ndarray:
    """[k, N] int64 residues in [0, p) of a signed integer polynomial."""
    return np.stack([(a % q).astype(np.int64) for q in primes])


def _crt_signed(r: np.ndarray, primes: tuple[int, ...]) -> np.ndarray:
    """Integers in (-M/2, M/2] from residues [k, N] (M = product of primes)."""
    M = 1
    for q in primes:
        M *= q
    acc = np.zeros(r.shape[1], dtype=object)
    for i, q in enumerate(primes):
        Mi = M // q
        acc = acc + r[i].astype(object) * (Mi * pow(Mi, -1, q))
    acc = acc % M
    half = M // 2
    return np.where(acc > half, acc - M, acc)


def _basis_for(bound: int) -> tuple[int, ...]:
    """Smallest prefix of the own basis whose product exceeds 2*bound."""
    prs = own_primes()
    M, k = 1, 0
    while M <= 2 * bound:
        if k == len(prs):
            raise ValueError("product bound too large for the own basis")
        M *= prs[k]
        k += 1
    return prs[:k]


def _max_abs(a: np.ndarray) -> int:
    return max((abs(int(x)) for x in a), default=0)


class OwnBasis:
    """Residue basis of the oracle's own primes, large enough that every
    integer of absolute value <= `bound` is determined by its residues."""

    def __init__(self, bound: int, n: int):
        self.primes = _basis_for(max(int(bound), 1))
        self.n = n
        (self.p, self.twist, self.untwist, self.omega, self.omega_inv,
         self.rev) = _tables(self.primes, n)
        self.pc = self.p[:, None]

    def residues(self, a) -> np.ndarray:
        """[k, N] residues of a signed integer polynomial."""
        a = np.asarray(a)
        if a.dtype != object and np.abs(a).max(initial=0) < (1 << 62):
            return np.stack([a.astype(np.int64) % q for q in self.primes])
        return _residues(as_object(a), self.primes)

    def forward(self, r: np.ndarray) -> np.ndarray:
        """Negacyclic transform per row: evaluations at odd powers of psi."""
        return _cyclic_ntt(r * self.twist % self.pc, self.p, self.omega, self.rev)

    def inverse(self, f: np.ndarray) -> np.ndarray:
        return _cyclic_ntt(f, self.p, self.omega_inv, self.rev) * self.untwist % self.pc

    def mul(self, fa: np.ndarray, fb: np.ndarray) -> np.ndarray:
        return fa * fb % self.pc

    def add(self, fa: np.ndarray, fb: np.ndarray) -> np.ndarray:
        return (fa + fb) % self.pc

    def to_int(self, r: np.ndarray) -> np.ndarray:
        """Signed integers from residues (CRT)."""
        return _crt_signed(r, self.primes)


def negacyclic_dot(pairs) -> np.ndarray:
    """sum_j a_j * b_j in Z[X]/(X^N+1), exactly, for a list of (a_j, b_j)."""
    pairs = [(as_object(a), as_object(b)) for a, b in pairs]
    n = len(pairs[0][0])
    bound = sum(_max_abs(a) * _max_abs(b) for a, b in pairs) * n
    B = OwnBasis(bound, n)
    acc = np.zeros((len(B.primes), n), dtype=np.int64)
    for a, b in pairs:
        acc = B.add(acc, B.mul(B.forward(B.residues(a)), B.forward(B.residues(b))))
    return B.to_int(B.inverse(acc))


def negacyclic_product(a, b) -> np.ndarray:
    """a * b in Z[X]/(X^N+1), exactly."""
    return negacyclic_dot([(a, b)])
