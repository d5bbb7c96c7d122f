"""Pins for oracle.compare: the comparison polynomial against the literal
sum of Fermat equalities (Eq. eq:inequality), its structure, the
evaluation program on plaintexts, and encrypted LT / LE / BETWEEN by
decryption over every pair in range (t = 17) and edge cases (t = 257)."""
import numpy as np
import pytest

import synth
from oracle import bfv, compare, encoding


@pytest.mark.parametrize("p", [5, 17, 257])
def test_fast_coefficients_equal_the_definition(p):
    assert list(compare.lt_coefficients(p)) == compare.lt_coefficients_direct(p)


@pytest.mark.parametrize("p", [17, 257])
def test_polynomial_is_the_literal_sum(p):
    """f(z) equals sum_{a in A} (1 - (z - a)^(p-1)) mod p (Eq. eq:inequality,
    computed term by term with pow) and the indicator of A, for every z."""
    c = list(compare.lt_coefficients(p))
    A = compare.negative_half(p)
    for z in range(p):
        literal = sum(1 - pow((z - a) % p, p - 1, p) for a in A) % p
        assert compare.eval_poly(c, z, p) == literal == int(z in set(A))


def test_polynomial_structure_at_the_paper_prime():
    p = 65537
    c = compare.lt_coefficients(p)
    assert all(c[k] == 0 for k in range(0, p - 1, 2))
    assert c[p - 1] == (p + 1) // 2
    A = set(compare.negative_half(p))
    rng = np.random.default_rng(0)
    for z in [0, 1, 2, 32767, 32768, 32769, 65535, 65536] + list(rng.integers(0, p, 8)):
        assert compare.eval_poly(list(c), int(z), p) == int(int(z) in A)


@pytest.mark.parametrize("p", [5, 17, 257])
def test_program_equals_polynomial_every_residue(p):
    c = list(compare.lt_coefficients(p))
    for z in range(p):
        assert compare.lt_program_plain(p, z) == compare.eval_poly(c, z, p)


def test_program_at_the_paper_prime_sampled():
    p = 65537
    A = set(compare.negative_half(p))
    rng = np.random.default_rng(1)
    for z in [0, 1, 65536, 32768, 32769] + list(rng.integers(0, p, 6)):
        assert compare.lt_program_plain(p, int(z)) == int(int(z) in A)


def test_shapes():
    assert compare.shape(65537) == (16, 256, 128)
    assert compare.shape(257) == (8, 16, 8)
    assert compare.shape(17) == (4, 4, 2)
    with pytest.raises(ValueError):
        compare.shape(97)


def _setup(n, t, seed=12):
    pr = bfv.paper_params(n, t)
    sk, rk = bfv.keygen(pr, synth.key_randomness(seed, n, pr.moduli_pq, pr.L))
    return pr, sk, rk


def _enc(pr, sk, v, seed):
    return bfv.encrypt_slots(pr, sk, v, synth.enc_randomness(seed, pr.n, pr.q))


@pytest.fixture(scope="module")
def t17():
    return _setup(8, 17)


def test_lt_every_pair_in_range_t17(t17):
    """Every (x, y) in [0, 16]^2 with |x - y| <= 8 (the valid range)."""
    pr, sk, rk = t17
    pairs = [(a, b) for a in range(17) for b in range(17) if abs(a - b) <= 8]
    pairs += [(0, 0)] * (-len(pairs) % 8)
    for c in range(len(pairs) // 8):
        chunk = pairs[8 * c: 8 * c + 8]
        x = [a for a, _ in chunk]
        y = [b for _, b in chunk]
        out = compare.lt(pr, rk, _enc(pr, sk, x, 300 + c), _enc(pr, sk, y, 400 + c))
        assert list(bfv.decrypt_slots(pr, sk, out)) == [int(a < b) for a, b in chunk]


def test_mul_sum_relin_decrypts_to_the_sum_of_products(t17):
    """One scale-and-round and relinearization of summed tensors decrypts to
    the slot-wise sum of the products (mod t), within the noise budget, and
    for a single pair it is the textbook product exactly."""
    pr, sk, rk = t17
    rng = np.random.default_rng(12)
    xs = [rng.integers(0, 17, 8) for _ in range(5)]
    ys = [rng.integers(0, 17, 8) for _ in range(5)]
    pairs = [(_enc(pr, sk, x, 500 + i), _enc(pr, sk, y, 600 + i))
             for i, (x, y) in enumerate(zip(xs, ys))]
    out = bfv.mul_sum_relin(pr, rk, pairs)
    want = sum(x * y for x, y in zip(xs, ys)) % 17
    assert list(bfv.decrypt_slots(pr, sk, out)) == list(want)
    assert bfv.noise_bits(pr, sk, out, encoding.encode(want, pr.t)) > 0
    one = bfv.mul_sum_relin(pr, rk, pairs[:1])
    ref = bfv.mul_relin(pr, rk, *pairs[0])
    for u, v in zip(one, ref):
        assert np.array_equal(u, v)


def test_lt_wraps_outside_the_range(t17):
    """|x - y| > (p-1)/2 wraps: the result is membership of (x - y) mod p in
    the negative half, not x < y (the domain limit of the method)."""
    pr, sk, rk = t17
    x = [0, 0, 16, 12, 3, 9, 1, 15]
    y = [9, 16, 0, 2, 14, 0, 12, 5]
    out = compare.lt(pr, rk, _enc(pr, sk, x, 500), _enc(pr, sk, y, 501))
    A = set(compare.negative_half(17))
    assert list(bfv.decrypt_slots(pr, sk, out)) == [int((a - b) % 17 in A) for a, b in zip(x, y)]
    assert [int((a - b) % 17 in A) for a, b in zip(x, y)] != [int(a < b) for a, b in zip(x, y)]


def test_le_and_between_t17(t17):
    pr, sk, rk = t17
    rng = np.random.default_rng(2)
    for c in range(3):
        x = rng.integers(4, 13, 8)
        y = rng.integers(4, 13, 8)
        cx, cy = _enc(pr, sk, x, 600 + c), _enc(pr, sk, y, 610 + c)
        le = compare.le(pr, rk, cx, cy)
        assert list(bfv.decrypt_slots(pr, sk, le)) == list((x <= y).astype(int))
    x = np.array([4, 5, 6, 7, 8, 9, 10, 11])
    lo, hi = np.full(8, 6), np.full(8, 9)
    out = compare.between(pr, rk, _enc(pr, sk, x, 620), _enc(pr, sk, lo, 621),
                          _enc(pr, sk, hi, 622))
    assert list(bfv.decrypt_slots(pr, sk, out)) == list(((x >= 6) & (x <= 9)).astype(int))


def test_lt_t257_edges_and_budget():
    """t = 257, N = 128 (k = 16 babies, m = 8 giants): differences 0, +-1,
    +-127, +-128 and random ones; the budget stays positive."""
    pr, sk, rk = _setup(128, 257)
    rng = np.random.default_rng(3)
    y = rng.integers(0, 257, pr.n)
    lo, hi = np.maximum(-128, -y), np.minimum(128, 256 - y)
    d = lo + (rng.random(pr.n) * (hi - lo + 1)).astype(np.int64)
    d[:7] = [0, 1, -1, 127, -127, 128, -128]
    y[:7] = 128
    x = y + d
    assert x.min() >= 0 and x.max() < 257
    out = compare.lt(pr, rk, _enc(pr, sk, x, 700), _enc(pr, sk, y, 701))
    want = (x < y).astype(int)
    assert list(bfv.decrypt_slots(pr, sk, out)) == list(want)
    assert bfv.noise_bits(pr, sk, out, encoding.encode(want, pr.t)) > 0
