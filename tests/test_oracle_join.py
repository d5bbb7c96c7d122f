"""Pins for oracle.join: the basis plaintext against its closed form, the
plaintext product against schoolbook multiplication and slot-wise
products, Extract/Broadcast by decryption, and the fused join-aggregation
against a plain equi-join."""
import numpy as np
import pytest

import synth
from oracle import bfv, encoding, galois, join, nt, ring


@pytest.mark.parametrize("n,t", [(8, 17), (64, 257)])
def test_basis_plain_closed_form(n, t):
    """Slot j's basis plaintext is N^-1 zeta_j^(-i) mod t, zeta_j = psi^(e_j)
    the slot's root (inverse transform of a one-hot slot vector)."""
    pr = bfv.Params(n, t, (1,), 1)
    psi = nt.root_of_unity(t, 2 * n)
    exps = encoding.slot_exponents(n)
    ninv = pow(n, -1, t)
    for j in (0, 1, n // 2 - 1, n // 2, n - 1):
        zinv = pow(pow(psi, exps[j], t), -1, t)
        want = [ninv * pow(zinv, i, t) % t for i in range(n)]
        got = join.basis_plain(pr, j)
        assert [int(v) for v in got] == want
        assert encoding.evaluate(got, t) == [int(s == j) for s in range(n)]


def _setup(n, t, seed=21):
    pr = bfv.paper_params(n, t)
    sk, rk = bfv.keygen(pr, synth.key_randomness(seed, n, pr.moduli_pq, pr.L))
    keys = {g: galois.galois_key(pr, sk, g, synth.switch_randomness(900 + i, n, pr.moduli_pq, pr.L))
            for i, g in enumerate(galois.sum_elements(n))}
    return pr, sk, rk, keys


@pytest.fixture(scope="module")
def n64():
    return _setup(64, 65537)


def test_mul_plain_matches_schoolbook_and_slots(n64):
    pr, sk, _, _ = n64
    rng = np.random.default_rng(1)
    v, w = rng.integers(0, pr.t, pr.n), rng.integers(0, pr.t, pr.n)
    ct = bfv.encrypt_slots(pr, sk, v, synth.enc_randomness(2, pr.n, pr.q))
    m = encoding.encode(w, pr.t)
    out = join.mul_plain(pr, ct, m)
    mc = [int(x) - pr.t if int(x) > pr.t // 2 else int(x) for x in m]
    for c_in, c_out in zip(ct, out):
        ref = ring.negacyclic_schoolbook([int(x) for x in c_in], mc)
        assert [int(x) % pr.Q for x in ref] == [int(x) for x in c_out]
    assert list(bfv.decrypt_slots(pr, sk, out)) == list(v * w % pr.t)


def test_extract_and_broadcast(n64):
    pr, sk, _, keys = n64
    v = np.random.default_rng(3).integers(0, 1000, pr.n)
    ct = bfv.encrypt_slots(pr, sk, v, synth.enc_randomness(4, pr.n, pr.q))
    for j in (0, 5, pr.n // 2, pr.n - 1):
        e = join.extract(pr, ct, j)
        assert list(bfv.decrypt_slots(pr, sk, e)) == [int(v[j]) if s == j else 0 for s in range(pr.n)]
        b = join.broadcast(pr, keys, ct, j)
        assert list(bfv.decrypt_slots(pr, sk, b)) == [int(v[j])] * pr.n


def test_join_sum_is_the_equi_join(n64):
    """Fact table A (64 rows, keys from B's and some unmatched), reference
    table B (unique keys, one attribute): the fused join-aggregation over
    three reference rows gives each A row the attribute of its matching B
    row among them, 0 otherwise."""
    pr, sk, rk, keys = n64
    rng = np.random.default_rng(5)
    b_key = rng.permutation(np.arange(100, 100 + pr.n))
    b_attr = rng.integers(1, 5000, pr.n)
    a_key = rng.choice(np.concatenate([b_key[:6], np.array([7, 8, 9])]), pr.n)
    enc = lambda v, s: bfv.encrypt_slots(pr, sk, v, synth.enc_randomness(s, pr.n, pr.q))
    rows = [0, 2, 4]
    out = join.join_sum(pr, rk, keys, enc(a_key, 6), enc(b_key, 7), enc(b_attr, 8), rows)
    lookup = {int(b_key[j]): int(b_attr[j]) for j in rows}
    assert list(bfv.decrypt_slots(pr, sk, out)) == [lookup.get(int(k), 0) for k in a_key]
