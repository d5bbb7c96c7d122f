"""Pins for oracle.bfv: the textbook BFV ciphertext arithmetic and the
Fermat equality chain, checked against closed forms, brute force, exact
rational arithmetic and the scheme's algebraic identities."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import bfv, encoding, ring, nt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _setup(n, t=65537, q=None, P=None, seed=0, alpha=1):
    if q is None:
        pr = bfv.paper_params(n, t, alpha)
    else:
        pr = bfv.Params(n, t, tuple(q), P)
    sk, rk = bfv.keygen(pr, synth.key_randomness(seed, n, pr.moduli_pq, pr.dnum))
    return pr, sk, rk


def _enc(pr, sk, slots, seed):
    return bfv.encrypt_slots(pr, sk, slots, synth.enc_randomness(seed, pr.n, pr.q))


@pytest.fixture(scope="module")
def small():
    return _setup(64)


@pytest.fixture(scope="module")
def cfg0():
    return _setup(1024)


# ------------------------------------------------------------ primitives ---

def test_round_div_is_nearest_integer():
    for x in range(-50, 51):
        for d in (1, 3, 7, 65537):
            assert bfv.round_div([x], d)[0] == round(Fraction(x, d))


def test_centred_range():
    M = 1001
    c = bfv.centred(list(range(-3 * M, 3 * M)), M)
    assert max(c) == 500 and min(c) == -500
    assert all((int(a) - b) % M == 0 for a, b in zip(c, range(-3 * M, 3 * M)))


def test_limbs_round_trip():
    pr = bfv.paper_params(16)
    rng = np.random.default_rng(1)
    vals = [int.from_bytes(rng.bytes(110), "little") % pr.Q for _ in range(16)]
    vals[0], vals[1] = 0, pr.Q - 1
    back = bfv.from_limbs(bfv.to_limbs(vals, pr.q), pr.q)
    assert list(back) == vals


def test_gadget_is_crt_basis():
    pr = bfv.paper_params(16)
    for j in range(pr.L):
        g = pr.gadget(j)
        assert all(g % pr.q[i] == (1 if i == j else 0) for i in range(pr.L))


def test_hybrid_parameters():
    """Two special primes: the same 18 primes, the two largest special, so
    Q*P keeps its 881 bits; digits are consecutive pairs of data primes."""
    one, two = bfv.paper_params(16), bfv.paper_params(16, alpha=2)
    assert two.alpha == 2 and two.L == 16 and two.dnum == 8
    assert sorted(one.moduli_pq) == sorted(two.moduli_pq)
    assert two.special == (one.P, one.q[0])
    assert two.P * two.Q == one.P * one.Q and (two.P * two.Q).bit_length() <= 881
    for j in range(two.dnum):
        assert two.digit_modulus(j) == two.q[2 * j] * two.q[2 * j + 1]


def test_hybrid_gadget_is_crt_basis_of_digit_groups():
    pr = bfv.paper_params(16, alpha=2)
    for j in range(pr.dnum):
        g = pr.gadget(j)
        assert 0 <= g < pr.Q
        assert all(g % pr.q[i] == (1 if i // 2 == j else 0) for i in range(pr.L))


def test_hybrid_digits_recompose():
    """sum_j [c]_{Q_j} g_j = c (mod Q) for any c (the Chinese remainder
    theorem over the digit moduli), with each digit in [0, Q_j)."""
    pr = bfv.paper_params(16, alpha=2)
    rng = np.random.default_rng(3)
    for _ in range(20):
        c = int.from_bytes(rng.bytes(110), "little") % pr.Q
        Qs = [pr.q[2 * j] * pr.q[2 * j + 1] for j in range(pr.dnum)]
        d = [c % Qj for Qj in Qs]
        assert all(0 <= dj < Qj for dj, Qj in zip(d, Qs))
        assert sum(dj * pr.gadget(j) for j, dj in enumerate(d)) % pr.Q == c


def test_ragged_last_digit():
    """L not a multiple of alpha: the last digit holds the remaining prime."""
    q, P = nt.default_modulus_chain(n_special=2)
    pr = bfv.Params(16, 257, tuple(q[:5]), P)
    assert pr.dnum == 3 and pr.digit_primes(2) == (q[4],)
    for j in range(3):
        g = pr.gadget(j)
        assert all(g % q[i] == (1 if i // 2 == j else 0) for i in range(5))


def test_depth_matches_paper_table():
    gold = json.load(open(os.path.join(GOLDEN, "eq_depth.json")))
    pr = bfv.paper_params(64, gold["p"])
    assert pr.squarings() == gold["equality_depth"]
    assert math.ceil(math.log2(gold["p"] - 1)) == gold["equality_depth"]


# ------------------------------------------------------ encrypt / decrypt ---

@pytest.mark.parametrize("seed", [1, 2])
def test_decrypt_inverts_encrypt(small, seed):
    pr, sk, _ = small
    x = np.random.default_rng(seed).integers(0, pr.t, pr.n)
    ct = _enc(pr, sk, x, seed)
    assert list(bfv.decrypt_slots(pr, sk, ct)) == list(x)
    assert all(0 <= int(c) < pr.Q for c in ct[0])


def test_fresh_noise_is_the_encryption_error(small):
    # t*phase - Q*m = t*e - (Q mod t)*m exactly, for ct = (Delta m + e - a s, a)
    pr, sk, _ = small
    x = np.arange(pr.n) % pr.t
    rnd = synth.enc_randomness(9, pr.n, pr.q)
    m = encoding.encode(x, pr.t)
    ct = bfv.encrypt(pr, sk, m, rnd)
    w = bfv.centred(pr.t * bfv.phase(pr, sk, ct) - pr.Q * ring.as_object(m), pr.t * pr.Q)
    want = pr.t * ring.as_object(rnd.e) - (pr.Q % pr.t) * ring.as_object(m)
    assert list(w) == list(want)


# --------------------------------------------------------------- multiply ---

def _schoolbook_multiply(pr, x, y):
    """Textbook product through an independent route: schoolbook products
    and Fraction rounding."""
    Q = pr.Q
    a0, a1 = bfv.centred(x[0], Q), bfv.centred(x[1], Q)
    b0, b1 = bfv.centred(y[0], Q), bfv.centred(y[1], Q)
    sb = ring.negacyclic_schoolbook
    d0 = sb(a0, b0)
    d1 = sb(a0, b1) + sb(a1, b0)
    d2 = sb(a1, b1)
    return tuple(np.array([round(Fraction(pr.t * int(v), Q)) % Q for v in d], dtype=object)
                 for d in (d0, d1, d2))


def test_multiply_matches_schoolbook_and_exact_rounding():
    pr, sk, _ = _setup(8)
    rng = np.random.default_rng(4)
    x = _enc(pr, sk, rng.integers(0, pr.t, 8), 5)
    y = _enc(pr, sk, rng.integers(0, pr.t, 8), 6)
    got = bfv.multiply(pr, x, y)
    want = _schoolbook_multiply(pr, x, y)
    for g, w in zip(got, want):
        assert list(g) == list(w)


def test_square_equals_multiply_self(small):
    pr, sk, _ = small
    x = _enc(pr, sk, np.arange(pr.n), 3)
    for a, b in zip(bfv.square(pr, x), bfv.multiply(pr, x, x)):
        assert list(a) == list(b)


def test_three_component_product_decrypts_to_slotwise_product(small):
    pr, sk, _ = small
    rng = np.random.default_rng(8)
    a, b = rng.integers(0, pr.t, pr.n), rng.integers(0, pr.t, pr.n)
    ct3 = bfv.multiply(pr, _enc(pr, sk, a, 1), _enc(pr, sk, b, 2))
    assert list(bfv.decrypt_slots(pr, sk, ct3)) == list(a * b % pr.t)


# ----------------------------------------------------------- relinearize ---

def test_relinearize_matches_schoolbook_route():
    pr, sk, rk = _setup(8)
    rng = np.random.default_rng(12)
    ct3 = bfv.multiply(pr, _enc(pr, sk, rng.integers(0, pr.t, 8), 1),
                       _enc(pr, sk, rng.integers(0, pr.t, 8), 2))
    got = bfv.relinearize(pr, rk, ct3)
    # independent route: schoolbook products, Fraction rounding
    u = [np.zeros(8, dtype=object), np.zeros(8, dtype=object)]
    for j, qj in enumerate(pr.q):
        dj = ring.as_object(ct3[2]) % qj
        u[0] = u[0] + ring.negacyclic_schoolbook(dj, rk.b[j])
        u[1] = u[1] + ring.negacyclic_schoolbook(dj, rk.a[j])
    for b in range(2):
        want = [(int(c) + round(Fraction(int(v), pr.P))) % pr.Q for c, v in zip(ct3[b], u[b])]
        assert list(got[b]) == want


def test_relinearize_identity_and_error_bound(small):
    """c0' + c1' s = c0 + c1 s + c2 s^2 + sum_j D_j e_j / P - r0 - r1 s
    (mod Q) with |r_b| <= 1/2: the key-switch error stays below its bound."""
    pr, sk, rk = small
    rng = np.random.default_rng(5)
    ct3 = bfv.multiply(pr, _enc(pr, sk, rng.integers(0, pr.t, pr.n), 1),
                       _enc(pr, sk, rng.integers(0, pr.t, pr.n), 2))
    ct2 = bfv.relinearize(pr, rk, ct3)
    diff = bfv.centred(bfv.phase(pr, sk, ct2) - bfv.phase(pr, sk, ct3), pr.Q)
    bound = pr.L * pr.n * max(pr.q) * 19 / pr.P + 0.5 + pr.n / 2
    assert max(abs(int(v)) for v in diff) <= bound
    # and the relinearization key is what it claims: b_j + a_j s = e_j + P g_j s^2 (mod PQ)
    s2 = ring.negacyclic_product(sk.s, sk.s)
    kr = synth.key_randomness(0, pr.n, pr.moduli_pq, pr.L)
    for j in (0, pr.L - 1):
        lhs = (rk.b[j] + ring.negacyclic_product(rk.a[j], sk.s)) % pr.PQ
        rhs = (ring.as_object(kr.e[j]) + pr.P * pr.gadget(j) * s2) % pr.PQ
        assert list(lhs) == list(rhs)


def test_hybrid_relinearize_matches_schoolbook_route():
    """Two-prime digits: D_j = [c2]_{q_2j q_2j+1}, products by schoolbook,
    rounding by exact fractions of P = P_0 P_1."""
    pr, sk, rk = _setup(8, alpha=2)
    rng = np.random.default_rng(13)
    ct3 = bfv.multiply(pr, _enc(pr, sk, rng.integers(0, pr.t, 8), 1),
                       _enc(pr, sk, rng.integers(0, pr.t, 8), 2))
    got = bfv.relinearize(pr, rk, ct3)
    P = pr.special[0] * pr.special[1]
    u = [np.zeros(8, dtype=object), np.zeros(8, dtype=object)]
    for j in range(pr.L // 2):
        dj = ring.as_object(ct3[2]) % (pr.q[2 * j] * pr.q[2 * j + 1])
        u[0] = u[0] + ring.negacyclic_schoolbook(dj, rk.b[j])
        u[1] = u[1] + ring.negacyclic_schoolbook(dj, rk.a[j])
    for b in range(2):
        want = [(int(c) + round(Fraction(int(v), P))) % pr.Q for c, v in zip(ct3[b], u[b])]
        assert list(got[b]) == want


def test_hybrid_relinearize_identity_and_error_bound():
    """As with one-prime digits: the phase changes by sum_j D_j e_j / P plus
    rounding, now with D_j < Q_j ~ 2^98 and P ~ 2^98."""
    pr, sk, rk = _setup(64, alpha=2)
    rng = np.random.default_rng(5)
    ct3 = bfv.multiply(pr, _enc(pr, sk, rng.integers(0, pr.t, pr.n), 1),
                       _enc(pr, sk, rng.integers(0, pr.t, pr.n), 2))
    ct2 = bfv.relinearize(pr, rk, ct3)
    diff = bfv.centred(bfv.phase(pr, sk, ct2) - bfv.phase(pr, sk, ct3), pr.Q)
    Qj = max(pr.q[2 * j] * pr.q[2 * j + 1] for j in range(pr.dnum))
    bound = pr.dnum * pr.n * Qj * 19 / pr.P + 0.5 + pr.n / 2
    assert max(abs(int(v)) for v in diff) <= bound
    s2 = ring.negacyclic_product(sk.s, sk.s)
    kr = synth.key_randomness(0, pr.n, pr.moduli_pq, pr.dnum)
    for j in (0, pr.dnum - 1):
        lhs = (rk.b[j] + ring.negacyclic_product(rk.a[j], sk.s)) % pr.PQ
        rhs = (ring.as_object(kr.e[j]) + pr.P * pr.gadget(j) * s2) % pr.PQ
        assert list(lhs) == list(rhs)


def test_hybrid_eq_chain_decrypts():
    pr, sk, rk = _setup(64, alpha=2)
    x, y = synth.column_pair_half_match(4, 64)
    _check_chain(pr, sk, rk, x, y, 21)


def test_mul_relin_decrypts_to_product(small):
    pr, sk, rk = small
    rng = np.random.default_rng(6)
    a, b = rng.integers(0, pr.t, pr.n), rng.integers(0, pr.t, pr.n)
    ct = bfv.mul_relin(pr, rk, _enc(pr, sk, a, 1), _enc(pr, sk, b, 2))
    assert len(ct) == 2
    assert list(bfv.decrypt_slots(pr, sk, ct)) == list(a * b % pr.t)


# ------------------------------------------------------------- EQ chain ---

def _check_chain(pr, sk, rk, x, y, seed):
    cx, cy = _enc(pr, sk, x, seed), _enc(pr, sk, y, seed + 1)
    levels, out = bfv.eq_chain(pr, rk, cx, cy)
    z = (np.asarray(x) - np.asarray(y)) % pr.t
    budgets = []
    for k, lv in enumerate(levels):
        want = [pow(int(v), 1 << k, pr.t) for v in z]
        assert list(bfv.decrypt_slots(pr, sk, lv)) == want, f"level {k}"
        budgets.append(bfv.noise_bits(pr, sk, lv, encoding.encode(want, pr.t)))
    mask = bfv.decrypt_slots(pr, sk, out)
    assert list(mask) == [int(a == b) for a, b in zip(np.asarray(x) % pr.t, np.asarray(y) % pr.t)]
    return levels, budgets


def test_eq_chain_small_workload_all_levels(cfg0):
    """The small workload: N = 1024, p = 65537, half-matching 16-bit columns
    plus edge differences; every level decrypts to z^(2^k) (Fermat), the
    mask is [x == y], the budget is positive and falls at every level."""
    pr, sk, rk = cfg0
    x, y = synth.column_pair_half_match(0, pr.n)
    x, y = synth.edge_differences(x, y, pr.t)
    levels, budgets = _check_chain(pr, sk, rk, x, y, 1)
    gold = json.load(open(os.path.join(GOLDEN, "eq_depth.json")))
    assert len(levels) == gold["equality_depth"] + 1
    assert all(b > 0 for b in budgets)
    assert all(b1 < b0 for b0, b1 in zip(budgets, budgets[1:]))


def test_eq_chain_pepin_and_special_values(cfg0):
    pr, sk, rk = cfg0
    gold = json.load(open(os.path.join(GOLDEN, "fermat_pepin.json")))
    zs = [c["z"] for c in gold["cases"]]
    y = np.full(pr.n, 7, dtype=np.int64)
    x = (y + np.resize(np.array(zs), pr.n)) % pr.t
    cx, cy = _enc(pr, sk, x, 3), _enc(pr, sk, y, 4)
    levels, out = bfv.eq_chain(pr, rk, cx, cy)
    for i, c in enumerate(gold["cases"]):
        for k, v in c["after_squarings"].items():
            assert bfv.decrypt_slots(pr, sk, levels[int(k)])[i] == v
    assert bfv.decrypt_slots(pr, sk, out)[0] == gold["eq_mask"]["equal"]
    assert bfv.decrypt_slots(pr, sk, out)[3] == gold["eq_mask"]["unequal"]


def test_eq_brute_force_all_pairs_t17():
    """Every (x, y) in Z_17^2 (289 pairs) over 37 ciphertexts of 8 slots."""
    pr, sk, rk = _setup(8, t=17)
    assert pr.squarings() == 4
    pairs = [(a, b) for a in range(17) for b in range(17)]
    pairs += [(0, 0)] * (37 * 8 - len(pairs))
    for c in range(37):
        chunk = pairs[8 * c: 8 * c + 8]
        x = [a for a, _ in chunk]
        y = [b for _, b in chunk]
        cx, cy = _enc(pr, sk, x, 100 + c), _enc(pr, sk, y, 200 + c)
        _, out = bfv.eq_chain(pr, rk, cx, cy)
        assert list(bfv.decrypt_slots(pr, sk, out)) == [int(a == b) for a, b in chunk]


def test_eq_all_differences_t257():
    """t = 257, N = 128 (8 squarings): every difference x - y in Z_257."""
    pr, sk, rk = _setup(128, t=257)
    assert pr.squarings() == 8
    rng = np.random.default_rng(257)
    d = np.concatenate([np.arange(257), rng.integers(0, 257, 3 * 128 - 257)])
    y = rng.integers(0, 257, 3 * 128)
    x = (y + d) % 257
    for c in range(3):
        sl = slice(128 * c, 128 * c + 128)
        cx, cy = _enc(pr, sk, x[sl], 10 + c), _enc(pr, sk, y[sl], 20 + c)
        _, out = bfv.eq_chain(pr, rk, cx, cy)
        assert list(bfv.decrypt_slots(pr, sk, out)) == list((d[sl] == 0).astype(int))


def test_eq_general_exponent_square_and_multiply():
    """A non-Fermat prime (t = 97, t - 1 = 96 = 0b1100000): square-and-
    multiply still yields 1 - z^(t-1) = [x == y]."""
    pr, sk, rk = _setup(16, t=97)
    rng = np.random.default_rng(97)
    y = rng.integers(0, 97, 16)
    x = np.where(rng.random(16) < 0.5, y, rng.integers(0, 97, 16))
    cx, cy = _enc(pr, sk, x, 1), _enc(pr, sk, y, 2)
    _, out = bfv.eq_chain(pr, rk, cx, cy)
    assert list(bfv.decrypt_slots(pr, sk, out)) == list((x == y).astype(int))


def test_noise_meter_flags_budget_exhaustion():
    """Too few data primes: the budget goes negative before the last level,
    and the meter's verdict (budget > 0) agrees with whether each level
    decrypts correctly."""
    q_all, P = nt.default_modulus_chain()
    pr, sk, rk = _setup(256, q=q_all[:7], P=P)
    x, y = synth.column_pair_half_match(5, pr.n)
    cx, cy = _enc(pr, sk, x, 1), _enc(pr, sk, y, 2)
    levels, out = bfv.eq_chain(pr, rk, cx, cy)
    z = (x - y) % pr.t
    verdicts = []
    for k, lv in enumerate(levels):
        want = [pow(int(v), 1 << k, pr.t) for v in z]
        ok = list(bfv.decrypt_slots(pr, sk, lv)) == want
        b = bfv.noise_bits(pr, sk, lv, encoding.encode(want, pr.t))
        assert ok == (b > 0), f"level {k}: budget {b}"
        verdicts.append(ok)
    assert verdicts[0] and not verdicts[-1]


# --------------------------------------------------- three-prime digits ---

def test_three_prime_digits_parameters_and_gadget():
    """alpha = 3: the three largest of the 18 primes special, 15 data primes
    in 5 digits of three; the gadget is the CRT basis of the digit groups."""
    one, three = bfv.paper_params(16), bfv.paper_params(16, alpha=3)
    assert (three.L, three.alpha, three.dnum) == (15, 3, 5)
    assert sorted(one.moduli_pq) == sorted(three.moduli_pq)
    assert three.P * three.Q == one.P * one.Q
    for j in range(three.dnum):
        g = three.gadget(j)
        assert all(g % three.q[i] == (1 if i // 3 == j else 0) for i in range(three.L))
        assert three.digit_modulus(j) == three.q[3 * j] * three.q[3 * j + 1] * three.q[3 * j + 2]


def test_three_prime_relinearize_matches_schoolbook_route():
    pr, sk, rk = _setup(8, alpha=3)
    rng = np.random.default_rng(14)
    ct3 = bfv.multiply(pr, _enc(pr, sk, rng.integers(0, pr.t, 8), 1),
                       _enc(pr, sk, rng.integers(0, pr.t, 8), 2))
    got = bfv.relinearize(pr, rk, ct3)
    P = pr.special[0] * pr.special[1] * pr.special[2]
    u = [np.zeros(8, dtype=object), np.zeros(8, dtype=object)]
    for j in range(5):
        dj = ring.as_object(ct3[2]) % (pr.q[3 * j] * pr.q[3 * j + 1] * pr.q[3 * j + 2])
        u[0] = u[0] + ring.negacyclic_schoolbook(dj, rk.b[j])
        u[1] = u[1] + ring.negacyclic_schoolbook(dj, rk.a[j])
    for b in range(2):
        want = [(int(c) + round(Fraction(int(v), P))) % pr.Q for c, v in zip(ct3[b], u[b])]
        assert list(got[b]) == want


def test_three_prime_eq_chain_decrypts():
    pr, sk, rk = _setup(64, alpha=3)
    x, y = synth.column_pair_half_match(5, 64)
    _check_chain(pr, sk, rk, x, y, 31)
