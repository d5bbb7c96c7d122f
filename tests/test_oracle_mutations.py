"""Planted mistakes: each plausible slip in the oracle must make at least
one of its pins fail.  The mistakes are planted in the oracle only, on the
CPU, through monkeypatching; nothing here touches a device."""
import numpy as np
import pytest

import synth
from oracle import bfv, ring
from tests import test_oracle_bfv as pins


def _dropped_cross_term(pr, x, y):
    Q = pr.Q
    a0, a1 = bfv.centred(x[0], Q), bfv.centred(x[1], Q)
    b0, b1 = bfv.centred(y[0], Q), bfv.centred(y[1], Q)
    d0 = ring.negacyclic_product(a0, b0)
    d1 = ring.negacyclic_product(a0, b1)            # a1*b0 missing
    d2 = ring.negacyclic_product(a1, b1)
    return tuple(bfv._scale_round(pr, d) for d in (d0, d1, d2))


def _floor_instead_of_round(pr, d):
    return (pr.t * ring.as_object(d)) // pr.Q % pr.Q


def _uncentred_lift(pr, x, y):
    Q = pr.Q
    a0, a1 = ring.as_object(x[0]) % Q, ring.as_object(x[1]) % Q
    b0, b1 = ring.as_object(y[0]) % Q, ring.as_object(y[1]) % Q
    d0 = ring.negacyclic_product(a0, b0)
    d1 = ring.negacyclic_dot([(a0, b1), (a1, b0)])
    d2 = ring.negacyclic_product(a1, b1)
    return tuple(bfv._scale_round(pr, d) for d in (d0, d1, d2))


def _wrong_sign_finish(pr, z):
    Q = pr.Q
    c0 = (-ring.as_object(z[0])) % Q
    c0[0] = (c0[0] + pr.delta) % Q
    return (c0, ring.as_object(z[1]) % Q)              # c1 not negated


class _ShiftedGadget(bfv.Params):
    def gadget(self, j):                                 # index off by one
        return super().gadget((j + 1) % self.L)


class _FirstPrimeDigits(bfv.Params):
    def digit_modulus(self, j):                          # a digit's second prime dropped
        return self.q[j * self.alpha]


def _run_expect_failure(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_dropped_cross_term_is_caught(monkeypatch):
    monkeypatch.setattr(bfv, "multiply", _dropped_cross_term)
    pr, sk, _ = pins._setup(64)
    _run_expect_failure(pins.test_three_component_product_decrypts_to_slotwise_product,
                        (pr, sk, None))


def test_floor_rounding_is_caught(monkeypatch):
    monkeypatch.setattr(bfv, "_scale_round", _floor_instead_of_round)
    _run_expect_failure(pins.test_multiply_matches_schoolbook_and_exact_rounding)


def test_uncentred_lift_is_caught(monkeypatch):
    monkeypatch.setattr(bfv, "multiply", _uncentred_lift)
    _run_expect_failure(pins.test_multiply_matches_schoolbook_and_exact_rounding)


def test_wrong_sign_in_finish_is_caught(monkeypatch):
    monkeypatch.setattr(bfv, "finish", _wrong_sign_finish)
    pr, sk, rk = pins._setup(64)
    x, y = synth.column_pair_half_match(0, 64)
    _run_expect_failure(pins._check_chain, pr, sk, rk, x, y, 1)


def test_transposed_gadget_is_caught():
    base = bfv.paper_params(64)
    pr = _ShiftedGadget(base.n, base.t, base.q, base.P)
    sk, rk = bfv.keygen(pr, synth.key_randomness(0, 64, pr.moduli_pq, pr.L))
    _run_expect_failure(pins.test_mul_relin_decrypts_to_product, (pr, sk, rk))


def test_dropped_digit_prime_is_caught():
    base = bfv.paper_params(64, alpha=2)
    pr = _FirstPrimeDigits(base.n, base.t, base.q, base.special)
    sk, rk = bfv.keygen(pr, synth.key_randomness(0, 64, pr.moduli_pq, pr.dnum))
    _run_expect_failure(pins.test_mul_relin_decrypts_to_product, (pr, sk, rk))


def test_one_special_prime_division_is_caught(monkeypatch):
    """Dividing by one special prime instead of their product P."""
    real = bfv.round_div

    def half_p(x, d):
        base = bfv.paper_params(8, alpha=2)
        return real(x, base.special[0] if d == base.P else d)
    monkeypatch.setattr(bfv, "round_div", half_p)
    _run_expect_failure(pins.test_hybrid_relinearize_matches_schoolbook_route)
