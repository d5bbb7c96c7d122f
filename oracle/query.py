"""Query operators built on the equality mask, in exact integers.

Test infrastructure only (see the package docstring).

NSHEDB turns SQL operators into ciphertext arithmetic around EQ
(Sec. 4.2.2, query operators):

* IN (set membership, Eq. eq:in): the sum over the set S of EQ(x, y); with
  distinct members at most one term is 1 per slot, so the sum decrypts to
  the indicator [x in S];
* GROUP BY: one equality mask per distinct group value;
* SELECT (Eq. eq:select): the selected column times the mask (one more
  multiplication followed by relinearization);
* the sums above are BFV additions (Sec. 2.1.6), exact per coefficient
  modulo Q, so their order does not change the result.
"""
from __future__ import annotations

from . import bfv
from . import ring


def add(params: bfv.Params, x, y) -> tuple:
    """Component-wise [x + y]_Q (BFV addition, Sec. 2.1.6)."""
    Q = params.Q
    return tuple((ring.as_object(a) + ring.as_object(b)) % Q for a, b in zip(x, y))


def add_many(params: bfv.Params, cts) -> tuple:
    """[sum of the ciphertexts]_Q, component-wise."""
    cts = list(cts)
    if not cts:
        raise ValueError("empty sum")
    acc = cts[0]
    for c in cts[1:]:
        acc = add(params, acc, c)
    return acc


def group_masks(params: bfv.Params, rk: bfv.RelinKey, x, values) -> list:
    """GROUP BY: EQ(x, v) for every encrypted group value v."""
    return [bfv.eq_chain(params, rk, x, v)[1] for v in values]


def in_mask(params: bfv.Params, rk: bfv.RelinKey, x, members) -> tuple:
    """IN(x, S) = sum over y in S of EQ(x, y) (Eq. eq:in)."""
    return add_many(params, group_masks(params, rk, x, members))


def select(params: bfv.Params, rk: bfv.RelinKey, column, mask) -> tuple:
    """SELECT column WHERE mask (Eq. eq:select): column * mask, relinearized."""
    return bfv.mul_relin(params, rk, column, mask)
