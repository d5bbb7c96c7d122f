"""Pins for oracle.ring (exact negacyclic products) and oracle.ntt_def."""
import random

import numpy as np
import pytest

from oracle import ring, ntt_def, nt


def _rand_poly(rng, n, bits):
    return [rng.randrange(-(1 << bits), 1 << bits) for _ in range(n)]


def test_schoolbook_small_known_values():
    # (1 + X)^2 = 1 + 2X + X^2 and X^2 = -1 mod X^2 + 1
    assert list(ring.negacyclic_schoolbook([1, 1], [1, 1])) == [0, 2]
    # X^(N-1) * X = X^N = -1
    n = 8
    a = [0] * n
    a[n - 1] = 1
    b = [0] * n
    b[1] = 1
    assert list(ring.negacyclic_schoolbook(a, b)) == [-1] + [0] * (n - 1)


@pytest.mark.parametrize("n,bits", [(1, 5), (2, 40), (8, 300), (64, 900), (16, 1700)])
def test_product_matches_schoolbook(n, bits):
    rng = random.Random(n * 1000 + bits)
    a, b = _rand_poly(rng, n, bits), _rand_poly(rng, n, bits // 2 + 3)
    assert list(ring.negacyclic_product(a, b)) == list(ring.negacyclic_schoolbook(a, b))


def test_dot_matches_sum_of_schoolbooks():
    rng = random.Random(7)
    n = 32
    pairs = [(_rand_poly(rng, n, 49), _rand_poly(rng, n, 881)) for _ in range(5)]
    want = np.zeros(n, dtype=object)
    for a, b in pairs:
        want = want + ring.negacyclic_schoolbook(a, b)
    assert list(ring.negacyclic_dot(pairs)) == list(want)


def test_product_extreme_coefficients():
    # all coefficients at the bound: the result sits at the edge of the basis
    n = 16
    big = (1 << 1000) - 1
    a = [big] * n
    b = [-big] * n
    assert list(ring.negacyclic_product(a, b)) == list(ring.negacyclic_schoolbook(a, b))


def test_own_basis_forward_is_evaluation_at_odd_roots():
    n = 16
    rng = random.Random(3)
    a = [rng.randrange(0, 1 << 30) for _ in range(n)]
    B = ring.OwnBasis(1 << 40, n)
    f = B.forward(B.residues(a))
    for k, q in enumerate(B.primes):
        assert list(f[k]) == ntt_def.evaluations(a, q)


def test_ntt_definition_turns_products_into_slotwise_products():
    q = 257
    n = 8
    rng = random.Random(5)
    a = [rng.randrange(q) for _ in range(n)]
    b = [rng.randrange(q) for _ in range(n)]
    c = [int(x) % q for x in ring.negacyclic_schoolbook(a, b)]
    ea, eb, ec = (ntt_def.evaluations(v, q) for v in (a, b, c))
    assert ec == [x * y % q for x, y in zip(ea, eb)]
    # and the roots used are exactly the N roots of X^N + 1
    psi = nt.root_of_unity(q, 2 * n)
    assert all(pow(psi, (2 * j + 1) * n, q) == q - 1 for j in range(n))
