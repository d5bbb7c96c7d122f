"""Default BFV parameters (host logic).

NSHEDB runs at n = 32768, log Q = 881, p = t = 65537 (Sec. 5.1).  The
library needs the modulus split into primes: here log2(Q * P) <= 881 is
split into 18 primes, each the largest available = 1 (mod 2^16) at or below
floor(2^(881/18)) (all in [2^48, 2^49), the device word); the largest is the
special prime P and the other 17 (descending) are the data primes.
"""
from __future__ import annotations

PAPER_T = 65537
PAPER_LOG2_N = 15
PAPER_LOG_QP = 881
N_PRIMES = 18
STEP = 1 << 16


def _is_prime(n: int) -> bool:
    # deterministic Miller-Rabin below 3.3e24 with the first twelve primes
    bases = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    if n < 2:
        return False
    for b in bases:
        if n % b == 0:
            return n == b
    d, s = n - 1, 0
    while not d & 1:
        d >>= 1
        s += 1
    for a in bases:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _root(x: int, k: int) -> int:
    lo, hi = 0, 1 << (x.bit_length() // k + 1)
    while lo < hi:
        mid = (lo + hi + 1) >> 1
        if mid ** k <= x:
            lo = mid
        else:
            hi = mid - 1
    return lo


def modulus_chain(log_qp: int = PAPER_LOG_QP, n_primes: int = N_PRIMES, n_special: int = 1):
    """(data primes q_0..q_{L-1} descending, special prime P or, for
    n_special = 2, the tuple of the two largest primes)."""
    bound = _root(1 << log_qp, n_primes)
    out = []
    k = (bound - 1) // STEP
    while len(out) < n_primes:
        c = k * STEP + 1
        if c <= bound and _is_prime(c):
            out.append(c)
        k -= 1
    return out[n_special:], (out[0] if n_special == 1 else tuple(out[:n_special]))


def paper_params(log2_n: int = PAPER_LOG2_N, t: int = PAPER_T, alpha: int = 1) -> dict:
    """The paper's parameters; alpha special primes (one key-switching digit
    per alpha data primes)."""
    q, P = modulus_chain(n_special=alpha)
    return {"log2_n": log2_n, "t": t, "q": q, "P": P}
