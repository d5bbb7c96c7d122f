"""Pins for oracle.query (IN, GROUP BY, SELECT and BFV addition): decrypted
results against plain set membership, partitions and products, by brute
force over small plaintext spaces."""
import numpy as np
import pytest

import synth
from oracle import bfv, encoding, query


def _setup(n, t):
    pr = bfv.paper_params(n, t)
    sk, rk = bfv.keygen(pr, synth.key_randomness(11, n, pr.moduli_pq, pr.L))
    return pr, sk, rk


def _enc(pr, sk, slots, seed):
    return bfv.encrypt_slots(pr, sk, slots, synth.enc_randomness(seed, pr.n, pr.q))


@pytest.fixture(scope="module")
def t17():
    return _setup(8, 17)


def test_add_decrypts_to_slot_sum(t17):
    pr, sk, _ = t17
    rng = np.random.default_rng(1)
    a, b = rng.integers(0, 17, 8), rng.integers(0, 17, 8)
    s = query.add(pr, _enc(pr, sk, a, 1), _enc(pr, sk, b, 2))
    assert list(bfv.decrypt_slots(pr, sk, s)) == list((a + b) % 17)
    # add(x, y) - y = x exactly, coefficient for coefficient
    cx, cy = _enc(pr, sk, a, 3), _enc(pr, sk, b, 4)
    back = bfv.sub(pr, query.add(pr, cx, cy), cy)
    assert all(list(u) == list(v) for u, v in zip(back, cx))


def test_in_closed_form_is_the_indicator():
    """sum over y in S of 1 - (x - y)^(p-1) mod p is [x in S] for distinct
    members: the identity the IN operator rests on (Eq. eq:in)."""
    p = 17
    rng = np.random.default_rng(2)
    for _ in range(20):
        S = rng.choice(p, size=int(rng.integers(1, 6)), replace=False)
        for x in range(p):
            v = sum(1 - pow((x - int(y)) % p, p - 1, p) for y in S) % p
            assert v == int(x in set(int(s) for s in S))


@pytest.mark.parametrize("members", [[3], [0, 16], [1, 5, 9, 13], [2, 4, 6, 8, 10]])
def test_in_mask_all_values_t17(t17, members):
    """Every x in Z_17 (three 8-slot ciphertexts) against an encrypted set."""
    pr, sk, rk = t17
    xs = list(range(17)) + [members[0]] * 7
    S = [_enc(pr, sk, np.full(8, m), 50 + i) for i, m in enumerate(members)]
    for c in range(3):
        x = xs[8 * c: 8 * c + 8]
        out = query.in_mask(pr, rk, _enc(pr, sk, x, 10 + c), S)
        assert list(bfv.decrypt_slots(pr, sk, out)) == [int(v in members) for v in x]


def test_in_mask_counts_repeated_members(t17):
    """A repeated member counts once per occurrence (the sum of Eq. eq:in
    taken literally): the reading for multisets."""
    pr, sk, rk = t17
    x = np.array([4, 4, 5, 6, 7, 4, 0, 1])
    S = [_enc(pr, sk, np.full(8, 4), 60), _enc(pr, sk, np.full(8, 4), 61),
         _enc(pr, sk, np.full(8, 6), 62)]
    out = query.in_mask(pr, rk, _enc(pr, sk, x, 63), S)
    assert list(bfv.decrypt_slots(pr, sk, out)) == [2 * int(v == 4) + int(v == 6) for v in x]


def test_group_masks_partition_the_column(t17):
    """GROUP BY over the distinct values present: each mask is its group's
    indicator and the masks sum to the all-ones vector."""
    pr, sk, rk = t17
    x = np.array([1, 2, 3, 1, 2, 3, 3, 1])
    groups = [_enc(pr, sk, np.full(8, g), 70 + g) for g in (1, 2, 3)]
    cx = _enc(pr, sk, x, 74)
    masks = query.group_masks(pr, rk, cx, groups)
    for g, m in zip((1, 2, 3), masks):
        assert list(bfv.decrypt_slots(pr, sk, m)) == list((x == g).astype(int))
    total = query.add_many(pr, masks)
    assert list(bfv.decrypt_slots(pr, sk, total)) == [1] * 8


def test_select_keeps_matching_values():
    """SELECT price WHERE id == key (Eq. eq:select) at t = 257, N = 128:
    price * EQ(id, key) keeps the price where the ids match, 0 elsewhere,
    with budget to spare after the extra level."""
    pr, sk, rk = _setup(128, 257)
    rng = np.random.default_rng(5)
    ids = rng.integers(0, 8, 128)
    price = rng.integers(0, 257, 128)
    key = 3
    cid, ckey = _enc(pr, sk, ids, 80), _enc(pr, sk, np.full(128, key), 81)
    cprice = _enc(pr, sk, price, 82)
    _, mask = bfv.eq_chain(pr, rk, cid, ckey)
    sel = query.select(pr, rk, cprice, mask)
    want = np.where(ids == key, price, 0)
    assert list(bfv.decrypt_slots(pr, sk, sel)) == list(want)
    assert bfv.noise_bits(pr, sk, sel, encoding.encode(want, pr.t)) > 0
