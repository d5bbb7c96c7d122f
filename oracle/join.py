"""Extract, Broadcast and the fused equi-join aggregation, exact.

Test infrastructure only (see the package docstring).

The paper derives two operations from BFV's primitives (Sec. 2.1.6): Extract
multiplies a ciphertext by the plaintext basis vector of one slot, and
Broadcast replicates that slot's value everywhere by extraction followed by
rotations and additions.  Its JOIN (Sec. 4.2.2, JOIN) extracts and broadcasts
each reference-table key, masks the fact table with the equality of the
keys, multiplies the mask with the reference table's projected attribute
(also extracted and broadcast) and adds over the reference rows.  Readings:

* a plaintext-ciphertext product is ([c0 m]_Q, [c1 m]_Q) with m the
  plaintext polynomial's centred representative, computed exactly in
  Z[X]/(X^N + 1);
* Broadcast = sum_slots(Extract) (the rotate-and-add of oracle.galois),
  exact because every other slot of the extracted ciphertext is 0;
* the fused join-aggregation over reference rows R:
  out = sum_{j in R} EQ(A.key, bcast(B.key, j)) * bcast(B.attr, j), which
  for unique reference keys decrypts, in each fact row, to the attribute of
  its matching reference row (0 if none).
"""
from __future__ import annotations

import numpy as np

from . import bfv
from . import encoding
from . import galois
from . import query
from . import ring


def mul_plain(params: bfv.Params, ct, m_poly) -> tuple:
    """ct * m for a plaintext polynomial m (coefficients in [0, t), taken as
    centred representatives)."""
    Q, t = params.Q, params.t
    m = [int(v) % t for v in m_poly]
    m = np.array([v - t if v > t // 2 else v for v in m], dtype=object)
    return tuple(bfv.poly_mul(ring.as_object(c), m) % Q for c in ct)


def basis_plain(params: bfv.Params, j: int) -> np.ndarray:
    """The plaintext polynomial whose slot j is 1 and every other slot 0."""
    v = np.zeros(params.n, dtype=np.int64)
    v[j] = 1
    return encoding.encode(v, params.t)


def extract(params: bfv.Params, ct, j: int) -> tuple:
    return mul_plain(params, ct, basis_plain(params, j))


def broadcast(params: bfv.Params, keys: dict, ct, j: int) -> tuple:
    return galois.sum_slots(params, keys, extract(params, ct, j))


def join_sum(params: bfv.Params, rk: bfv.RelinKey, keys: dict, a_key, b_key, b_attr,
             rows) -> tuple:
    """sum over reference rows j of EQ(A.key, bcast(B.key, j)) *
    bcast(B.attr, j), one fact-table ciphertext a_key."""
    out = None
    for j in rows:
        mask = bfv.eq_chain(params, rk, a_key, broadcast(params, keys, b_key, j))[1]
        term = bfv.mul_relin(params, rk, mask, broadcast(params, keys, b_attr, j))
        out = term if out is None else query.add(params, out, term)
    return out
