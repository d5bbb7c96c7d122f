"""Pins for oracle.galois: the automorphism against schoolbook products and
composition, its action on slots against the definition of the slot
layout, Galois keys against their defining identity, and rotations /
rotate-and-add sums by decryption."""
import numpy as np
import pytest

import synth
from oracle import bfv, encoding, galois, query, ring


def test_automorphism_is_a_ring_homomorphism():
    rng = np.random.default_rng(0)
    n, M = 16, 1000003
    a = [int(v) for v in rng.integers(0, M, n)]
    b = [int(v) for v in rng.integers(0, M, n)]
    for g in (3, 5, 9, 31, 2 * n - 1):
        lhs = galois.automorphism(ring.negacyclic_schoolbook(a, b), g) % M
        rhs = ring.negacyclic_schoolbook(list(galois.automorphism(a, g) % M),
                                         list(galois.automorphism(b, g) % M))
        assert [int(v) % M for v in lhs] == [int(v) % M for v in rhs]


def test_automorphism_composes_and_inverts():
    rng = np.random.default_rng(1)
    n = 32
    a = [int(v) for v in rng.integers(-50, 50, n)]
    for g, h in [(3, 5), (9, 2 * n - 1), (27, 7)]:
        gh = galois.automorphism(galois.automorphism(a, g), h)
        assert list(gh) == list(galois.automorphism(a, g * h % (2 * n)))
        ginv = pow(g, -1, 2 * n)
        assert list(galois.automorphism(galois.automorphism(a, g), ginv)) == a
    # X -> X^g sends X to X^g, with X^N = -1
    x = [0] * n
    x[1] = 1
    img = galois.automorphism(x, 2 * n - 1)
    assert img[n - 1] == -1 and sum(abs(int(v)) for v in img) == 1


@pytest.mark.parametrize("n,t", [(8, 17), (64, 257)])
def test_rotation_elements_act_on_slots(n, t):
    """On plaintexts (no encryption): decode(sigma_g(encode(v))) is v with
    each half rotated left by r for g = 3^r, and the halves swapped for
    g = 2N - 1; both follow from the slot layout's definition."""
    rng = np.random.default_rng(n)
    v = rng.integers(0, t, n)
    m = encoding.encode(v, t)
    h = n // 2
    for r in (1, 2, h - 1):
        got = encoding.evaluate(galois.automorphism(m, galois.rotation_element(n, r)) % t, t)
        want = list(np.roll(v[:h], -r)) + list(np.roll(v[h:], -r))
        assert got == want
    got = encoding.evaluate(galois.automorphism(m, galois.swap_element(n)) % t, t)
    assert got == list(v[h:]) + list(v[:h])


def _setup(n, t, seed=3, alpha=1):
    pr = bfv.paper_params(n, t, alpha)
    sk, rk = bfv.keygen(pr, synth.key_randomness(seed, n, pr.moduli_pq, pr.dnum))
    keys = {g: galois.galois_key(pr, sk, g,
                                 synth.switch_randomness(100 + i, n, pr.moduli_pq, pr.dnum))
            for i, g in enumerate(galois.sum_elements(n))}
    return pr, sk, rk, keys


@pytest.fixture(scope="module", params=[1, 2], ids=["alpha1", "alpha2"])
def n64(request):
    return _setup(64, 65537, alpha=request.param)


def test_galois_key_identity(n64):
    pr, sk, _, keys = n64
    for g, key in keys.items():
        sg = galois.automorphism(sk.s, g)
        for j in range(pr.dnum):
            lhs = (key.b[j] + bfv.poly_mul(key.a[j], sk.s)) % pr.PQ
            rhs = (pr.P * pr.gadget(j) * sg) % pr.PQ
            err = bfv.centred((lhs - rhs) % pr.PQ, pr.PQ)
            assert max(abs(int(e)) for e in err) <= 6 * 3.2 + 1


def test_rotations_decrypt_to_rotated_slots(n64):
    pr, sk, _, keys = n64
    rng = np.random.default_rng(4)
    v = rng.integers(0, pr.t, pr.n)
    ct = bfv.encrypt_slots(pr, sk, v, synth.enc_randomness(5, pr.n, pr.q))
    h = pr.n // 2
    for g in galois.sum_elements(pr.n):
        out = galois.apply_galois(pr, keys[g], ct, g)
        got = list(bfv.decrypt_slots(pr, sk, out))
        if g == galois.swap_element(pr.n):
            want = list(v[h:]) + list(v[:h])
        else:
            r = next(r for r in range(h) if galois.rotation_element(pr.n, r) == g)
            want = list(np.roll(v[:h], -r)) + list(np.roll(v[h:], -r))
        assert got == want
        assert bfv.noise_bits(pr, sk, out, encoding.encode(want, pr.t)) > 0


def test_sum_slots_counts_and_sums(n64):
    """COUNT of a 0/1 mask and SUM of a masked column: every slot holds the
    total mod t (Sec. 4.2.2 aggregation)."""
    pr, sk, rk, keys = n64
    rng = np.random.default_rng(6)
    mask = (rng.random(pr.n) < 0.3).astype(np.int64)
    price = rng.integers(0, 1000, pr.n)
    cm = bfv.encrypt_slots(pr, sk, mask, synth.enc_randomness(7, pr.n, pr.q))
    cp = bfv.encrypt_slots(pr, sk, price, synth.enc_randomness(8, pr.n, pr.q))
    count = galois.sum_slots(pr, keys, cm)
    assert list(bfv.decrypt_slots(pr, sk, count)) == [int(mask.sum()) % pr.t] * pr.n
    total = galois.sum_slots(pr, keys, query.select(pr, rk, cp, cm))
    assert list(bfv.decrypt_slots(pr, sk, total)) == [int((mask * price).sum()) % pr.t] * pr.n


def test_sum_slots_all_values_t17():
    """Brute force at t = 17, N = 8: the sum of every slot, for slots holding
    every residue."""
    pr, sk, _, keys = _setup(8, 17, seed=9)
    assert galois.sum_elements(8) == [9, 3, 15]   # rotate by 2, by 1, swap halves
    for c in range(4):
        v = (np.arange(8) + 8 * c) % 17
        ct = bfv.encrypt_slots(pr, sk, v, synth.enc_randomness(20 + c, 8, pr.q))
        out = galois.sum_slots(pr, keys, ct)
        assert list(bfv.decrypt_slots(pr, sk, out)) == [int(v.sum()) % 17] * 8
