"""Number theory for the oracle: primality, NTT-friendly primes, roots.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

# Deterministic Miller-Rabin: the first twelve primes as bases are a proven
# witness set for every n < 3.3e24 (Sorenson and Webster, 2015), which covers
# every modulus this project uses (all below 2^64).
_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Deterministic primality for n < 3.3e24 (strong-pseudoprime test)."""
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    if n >= 3_317_044_064_679_887_385_961_981:
        raise ValueError("is_prime: outside the deterministic range")
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x == 1 or x == n - 1:
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def primes_congruent_one_below(bound: int, step: int, count: int,
                               exclude: tuple[int, ...] = ()) -> list[int]:
    """The `count` largest primes p < bound with p = 1 (mod step), descending."""
    out: list[int] = []
    k = (bound - 2) // step
    while len(out) < count:
        if k <= 0:
            raise ValueError("not enough primes below the bound")
        c = k * step + 1
        if c < bound and c not in exclude and is_prime(c):
            out.append(c)
        k -= 1
    return out


def factorize_small(n: int) -> list[int]:
    """Distinct prime factors by trial division (n is q - 1 for q < 2^64 with
    a large power of two, so the odd cofactor is small enough)."""
    fs = []
    d = 2
    while d * d <= n:
        if n % d == 0:
            fs.append(d)
            while n % d == 0:
                n //= d
        d += 1 if d == 2 else 2
    if n > 1:
        fs.append(n)
    return fs


def primitive_root(q: int) -> int:
    """Smallest generator of the multiplicative group mod prime q."""
    fs = factorize_small(q - 1)
    g = 2
    while True:
        if all(pow(g, (q - 1) // f, q) != 1 for f in fs):
            return g
        g += 1


def root_of_unity(q: int, order: int) -> int:
    """g^((q-1)/order) for the smallest primitive root g: a primitive
    `order`-th root of unity mod q (requires order | q - 1)."""
    if (q - 1) % order:
        raise ValueError("order does not divide q - 1")
    return pow(primitive_root(q), (q - 1) // order, q)


def integer_root(x: int, k: int) -> int:
    """floor(x^(1/k)) for integers x >= 0, k >= 1, by bisection."""
    lo, hi = 0, 1 << (x.bit_length() // k + 1)
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if mid ** k <= x:
            lo = mid
        else:
            hi = mid - 1
    return lo


def default_modulus_chain(log_qp_bits: int = 881, n_primes: int = 18,
                          step: int = 1 << 16, n_special: int = 1):
    """Default data primes q_0..q_{L-1} and special prime(s).

    Reading of the paper's parameters (Sec. 5.1: n = 32768, log Q = 881,
    t = 65537): the 881 bits bound the largest modulus used, Q*P.  Split it
    into `n_primes` primes, each at most floor(2^(881/18)) so that
    log2(Q*P) <= 881, each = 1 (mod 2^16) so that a negacyclic NTT of every
    length N <= 2^15 exists.  The largest `n_special` are the special primes
    (returned as one int when there is one, else as a tuple, descending);
    the other n_primes - n_special, in descending order, are the data
    primes.
    """
    bound = integer_root(1 << log_qp_bits, n_primes)
    ps = primes_congruent_one_below(bound + 1, step, n_primes)
    sp = ps[0] if n_special == 1 else tuple(ps[:n_special])
    return ps[n_special:], sp
