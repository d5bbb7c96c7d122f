"""Pins for oracle.nt: primality, prime search, roots of unity, parameters."""
import math

import pytest

from oracle import nt


def _trial_prime(n):
    if n < 2:
        return False
    d = 2
    while d * d <= n:
        if n % d == 0:
            return False
        d += 1
    return True


def test_is_prime_matches_trial_division_exhaustively():
    assert [n for n in range(20000) if nt.is_prime(n)] == \
        [n for n in range(20000) if _trial_prime(n)]


@pytest.mark.parametrize("n", [561, 41041, 2047, 1373653, 25326001,
                               3215031751, 2152302898747, 3474749660383,
                               341550071728321])
def test_is_prime_rejects_carmichael_and_strong_pseudoprimes(n):
    # Carmichael numbers and the smallest strong pseudoprimes to the first
    # 1..7 prime bases (published tables); all composite.
    assert not nt.is_prime(n)


@pytest.mark.parametrize("p", [65537, 2**31 - 1, 2**61 - 1, 998244353,
                               (1 << 64) - 59])
def test_is_prime_accepts_known_primes(p):
    assert nt.is_prime(p)


def test_prime_search_is_complete_and_descending():
    got = nt.primes_congruent_one_below(200000, 64, 12)
    brute = [p for p in range(199999, 0, -1) if p % 64 == 1 and _trial_prime(p)][:12]
    assert got == brute


def test_primitive_root_of_fermat_prime():
    # 3 generates Z_65537^* (Pepin's test base); 2 has order 32 there.
    assert nt.primitive_root(65537) == 3
    assert pow(2, 32, 65537) == 1


@pytest.mark.parametrize("q,order", [(65537, 65536), (65537, 2048), (17, 16),
                                     (257, 256), (998244353, 1 << 23)])
def test_root_of_unity_has_exact_order(q, order):
    w = nt.root_of_unity(q, order)
    assert pow(w, order, q) == 1
    assert pow(w, order // 2, q) == q - 1


def test_integer_root_exact():
    for x in [0, 1, 2, 7, 8, 9, 10**40, (1 << 881) - 1, 1 << 881]:
        for k in [1, 2, 3, 18]:
            r = nt.integer_root(x, k)
            assert r ** k <= x < (r + 1) ** k


def test_default_modulus_chain_matches_paper_sizes():
    # Sec. 5.1: n = 32768, log Q = 881 (read as log2(Q*P) <= 881).
    q, P = nt.default_modulus_chain()
    allp = q + [P]
    assert len(q) == 17 and len(set(allp)) == 18
    assert all(nt.is_prime(x) and x % 65536 == 1 for x in allp)
    assert all(P > x for x in q) and q == sorted(q, reverse=True)
    bits = sum(math.log2(x) for x in allp)
    assert 880.9 < bits <= 881
    prod = 1
    for x in allp:
        prod *= x
    assert prod < 1 << 881
    # every prime fits the device word: below 2^49
    assert all(x < 1 << 49 for x in allp)
