"""Pins for oracle.encoding (batch encoding, client side)."""
import random

import numpy as np
import pytest

from oracle import encoding, ring


@pytest.mark.parametrize("t,n", [(17, 8), (257, 128), (65537, 64), (65537, 1024)])
def test_decode_inverts_encode(t, n):
    rng = random.Random(t + n)
    s = [rng.randrange(t) for _ in range(n)]
    assert list(encoding.decode(encoding.encode(s, t), t)) == s


@pytest.mark.parametrize("t,n", [(17, 8), (257, 16), (65537, 32)])
def test_fast_decode_equals_horner_definition(t, n):
    rng = random.Random(n)
    m = [rng.randrange(t) for _ in range(n)]
    assert list(encoding.decode(m, t)) == encoding.evaluate(m, t)


def test_slot_exponents_are_the_roots_of_x_n_plus_1():
    n = 64
    ex = encoding.slot_exponents(n)
    assert sorted(ex) == list(range(1, 2 * n, 2))


@pytest.mark.parametrize("t,n", [(257, 128), (65537, 256)])
def test_ring_product_is_slotwise_product(t, n):
    rng = random.Random(11)
    a = [rng.randrange(t) for _ in range(n)]
    b = [rng.randrange(t) for _ in range(n)]
    c = ring.negacyclic_product(encoding.encode(a, t), encoding.encode(b, t)) % t
    assert list(encoding.decode(c, t)) == [x * y % t for x, y in zip(a, b)]


def test_constant_one_fills_every_slot():
    t, n = 65537, 128
    one = [1] + [0] * (n - 1)
    assert list(encoding.decode(one, t)) == [1] * n


def test_automorphism_x3_rotates_rows_by_one():
    # m(X) -> m(X^3): the value at psi^(3^s) moves to slot s - 1.
    t, n = 257, 32
    rng = random.Random(2)
    s = [rng.randrange(t) for _ in range(n)]
    m = encoding.encode(s, t)
    r = [0] * n
    for i, c in enumerate(m):
        k = (3 * i) % (2 * n)
        if k < n:
            r[k] = (r[k] + int(c)) % t
        else:
            r[k - n] = (r[k - n] - int(c)) % t
    got = list(encoding.decode(r, t))
    h = n // 2
    assert got[:h] == s[1:h] + s[:1]
    assert got[h:] == s[h + 1:] + s[h:h + 1]
