"""The library's noise budget and depth accounting (host arithmetic, no GPU),
pinned against the oracle: its model of the noise (fresh budget, bits per
multiplication) must stay below the exact noise the oracle measures at
every level of an EQ chain, and a chain as deep as the reported budget must
still decrypt.  The comparison program's depth must equal the depth of the
oracle's own program (Sec. 2.1.2: depth(A x B) = max(depth A, depth B) + 1;
Table table:noise_levels)."""
import ctypes
import math
from unittest import mock

import numpy as np
import pytest

import synth
from oracle import bfv, compare, encoding, nt
from paper_2602_24271_amd import _lib, params


def budget(log2_n, t=65537, q=None, P=None):
    lib = _lib.load()
    if q is None:
        q, P = params.modulus_chain()
    qa = (ctypes.c_uint64 * len(q))(*q)
    pr = _lib.NsheParams(log2_n, t, len(q), ctypes.cast(qa, ctypes.POINTER(ctypes.c_uint64)), P)
    b = _lib.NsheBudget()
    _lib.check(lib.nshe_budget_of(ctypes.byref(pr), ctypes.byref(b)))
    return b


def test_paper_parameters_budget():
    """Sec. 5.1 parameters: EQ (16), LT (18 + 1) and BETWEEN fit; the
    figures the header states."""
    b = budget(15)
    assert b.depth_budget == 23
    assert abs(b.fresh_bits - 799.06) < 0.01 and abs(b.level_bits - 33.0) < 1e-3
    assert b.lt_depth == 18


def test_bad_parameters_rejected_without_a_device():
    lib = _lib.load()
    assert lib.nshe_budget_of(None, None) == -1
    q, P = params.modulus_chain()
    qa = (ctypes.c_uint64 * 3)(97, 193, 257)
    pr = _lib.NsheParams(10, 65537, 3, ctypes.cast(qa, ctypes.POINTER(ctypes.c_uint64)), P)
    b = _lib.NsheBudget()
    assert lib.nshe_budget_of(ctypes.byref(pr), ctypes.byref(b)) == -1


def _chain_noise(log2_n, L, levels, seed=0):
    """Exact budgets (bits) of the oracle's ciphertexts after 0..levels
    squarings of a fresh difference, with the true plaintexts."""
    n = 1 << log2_n
    primes = nt.primes_congruent_one_below(1 << 49, 1 << 16, L + 1)
    pr = bfv.Params(n, 65537, tuple(primes[1:]), primes[0])
    sk, rk = bfv.keygen(pr, synth.key_randomness(seed, n, pr.moduli_pq, pr.L))
    x, y = synth.column_pair_half_match(seed, n)
    z = (x - y) % pr.t
    ct = bfv.sub(pr, bfv.encrypt_slots(pr, sk, x, synth.enc_randomness(1, n, pr.q)),
                 bfv.encrypt_slots(pr, sk, y, synth.enc_randomness(2, n, pr.q)))
    out = []
    for k in range(levels + 1):
        m = encoding.encode([pow(int(v), 2 ** k, pr.t) for v in z], pr.t)
        out.append(bfv.noise_bits(pr, sk, ct, m))
        if k < levels:
            ct = bfv.square_relin(pr, rk, ct)
    return pr, primes, out


@pytest.mark.parametrize("log2_n,L", [(6, 4), (8, 4), (10, 8)])
def test_model_below_measured_noise_through_the_budget(log2_n, L):
    """Small moduli so that the budget is a few levels: the oracle's exact
    budget at every level up to the reported depth budget is at least the
    model's, and positive (the ciphertext still decrypts)."""
    primes = nt.primes_congruent_one_below(1 << 49, 1 << 16, L + 1)
    b = budget(log2_n, q=primes[1:], P=primes[0])
    assert 1 <= b.depth_budget <= 12
    pr, _, meas = _chain_noise(log2_n, L, b.depth_budget)
    assert abs(b.fresh_bits - (math.log2(pr.Q) - math.log2(2 * pr.t * (19 + pr.t)))) < 1e-6
    for k, got in enumerate(meas):
        assert got >= b.fresh_bits - k * b.level_bits, (k, got)
    assert meas[-1] > 0


def test_model_below_measured_noise_paper_chain():
    """The paper's 17 primes at N = 1024: every one of the 16 EQ levels
    keeps at least the model's budget."""
    b = budget(10)
    _, _, meas = _chain_noise(10, 17, 16)
    for k, got in enumerate(meas):
        assert got >= b.fresh_bits - k * b.level_bits, (k, got)


def _program_depths(p):
    """Depth of the oracle's comparison program, by running it on depths
    (every product max + 1, every sum or scalar product the max)."""
    pr = bfv.Params(8, p, (3,), 5)
    patches = [
        mock.patch.object(compare.bfv, "sub", lambda pr, a, b: max(a, b)),
        mock.patch.object(compare.bfv, "square_relin", lambda pr, rk, a: a + 1),
        mock.patch.object(compare.bfv, "mul_relin", lambda pr, rk, a, b: max(a, b) + 1),
        mock.patch.object(compare.bfv, "mul_sum_relin",
                          lambda pr, rk, pairs: max(max(a, b) for a, b in pairs) + 1),
        mock.patch.object(compare, "lincomb", lambda pr, cts, co: max(cts)),
        mock.patch.object(compare.query, "add", lambda pr, a, b: max(a, b)),
        mock.patch.object(compare, "scalar_mul", lambda pr, a, c: a),
        mock.patch.object(compare, "trivial_one", lambda pr: 0),
        mock.patch.object(compare, "lt_coefficients", lambda p: [0] * p),
    ]
    for m in patches:
        m.start()
    try:
        return compare.lt(pr, None, 0, 0)
    finally:
        for m in patches:
            m.stop()


@pytest.mark.parametrize("p", [5, 17, 257, 65537])
def test_comparison_depth_matches_the_oracle_program(p):
    q, P = params.modulus_chain()
    b = budget(3, t=p, q=q, P=P)
    assert b.lt_depth == _program_depths(p)


def test_no_comparison_depth_without_a_fermat_prime():
    q, P = params.modulus_chain()
    assert budget(3, t=97, q=q, P=P).lt_depth == -1
    assert budget(3, t=9, q=q, P=P).lt_depth == -1


def test_two_special_primes_budget():
    """16 data primes (two special primes): one prime less of noise budget,
    still room for BETWEEN (LT's 18 + 1, plus 1)."""
    lib = _lib.load()
    q, (P0, P1) = params.modulus_chain(n_special=2)
    qa = (ctypes.c_uint64 * len(q))(*q)
    pr = _lib.NsheParams(15, 65537, len(q), ctypes.cast(qa, ctypes.POINTER(ctypes.c_uint64)),
                         P0, 2, P1)
    b = _lib.NsheBudget()
    _lib.check(lib.nshe_budget_of(ctypes.byref(pr), ctypes.byref(b)))
    log2q = sum(math.log2(x) for x in q)
    assert abs(b.fresh_bits - (log2q - math.log2(2 * 65537 * (19 + 65537)))) < 1e-9
    assert b.depth_budget == 22 and b.depth_budget >= b.lt_depth + 2
