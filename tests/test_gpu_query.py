"""Device parity of the operators built on EQ: BFV addition and sums, IN
(Eq. eq:in), GROUP BY masks and SELECT (Eq. eq:select), bit-exact against
the oracle and decrypting to the plain query results."""
import numpy as np
import pytest
import torch

import synth
from oracle import bfv, query
from tests.gpu_common import Setup

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def s256():
    return Setup(8, seed=4)


def _column(S, seed, values):
    rng = np.random.default_rng(seed)
    return rng.choice(values, S.pr.n)


def test_add_and_sum(s256):
    S = s256
    rng = np.random.default_rng(1)
    slots = [rng.integers(0, S.pr.t, S.pr.n) for _ in range(3)]
    cts = [S.enc(v, 10 + i) for i, v in enumerate(slots)]
    a, b = S.to_dev(cts[:1]), S.to_dev(cts[1:2])
    np.testing.assert_array_equal(S.ctx.add(a, b)[0].cpu().numpy(),
                                  S.limbs(query.add(S.pr, cts[0], cts[1])))
    stack = torch.stack([S.to_dev([c]) for c in cts])          # [3][1][2][L][N]
    got = S.ctx.sum(stack)
    want = query.add_many(S.pr, cts)
    np.testing.assert_array_equal(got[0].cpu().numpy(), S.limbs(want))
    assert list(bfv.decrypt_slots(S.pr, S.sk, want)) == list(sum(slots) % S.pr.t)
    zero = S.ctx.sum(stack[:0])
    assert int(zero.abs().sum()) == 0


@pytest.mark.parametrize("members,wave_ct", [([7], 0), ([3, 11, 40000], 2), ([0, 1, 2, 3, 4], 3)])
def test_in_mask_matches_oracle(s256, members, wave_ct):
    S = s256
    vals = np.array(sorted(set(members + [5, 6, 65536])))
    xs = [_column(S, 20 + c, vals) for c in range(2)]
    cxs = [S.enc(x, 30 + c) for c, x in enumerate(xs)]
    cm = [S.enc(np.full(S.pr.n, m), 40 + i) for i, m in enumerate(members)]
    got = S.ctx.in_mask(S.to_dev(cxs), S.to_dev(cm), wave_ct=wave_ct)
    torch.cuda.synchronize()
    for c, (x, cx) in enumerate(zip(xs, cxs)):
        want = query.in_mask(S.pr, S.rk, cx, cm)
        np.testing.assert_array_equal(got[c].cpu().numpy(), S.limbs(want))
        mask = bfv.decrypt_slots(S.pr, S.sk, S.from_dev(got[c:c + 1])[0])
        assert list(mask) == [int(v in members) for v in x]


def test_in_mask_empty_set_is_zero(s256):
    S = s256
    x = S.to_dev([S.enc(np.arange(S.pr.n), 50)])
    empty = torch.empty((0, 2, S.pr.L, S.pr.n), dtype=torch.int64, device=S.ctx.device)
    got = S.ctx.in_mask(x, empty)
    assert int(got.abs().sum()) == 0


def test_group_masks_and_select(s256):
    """GROUP BY over dictionary ids, then SELECT a price column with one
    group's mask: each mask equals the oracle's, the masks partition the
    column, and the selection keeps that group's prices."""
    S = s256
    ids = _column(S, 60, np.array([1, 2, 3]))
    price = np.random.default_rng(61).integers(0, 1000, S.pr.n)
    cid = S.enc(ids, 62)
    groups = [S.enc(np.full(S.pr.n, g), 63 + g) for g in (1, 2, 3)]
    masks = S.ctx.group_masks(S.to_dev([cid]), S.to_dev(groups), wave_ct=2)
    torch.cuda.synchronize()
    want = query.group_masks(S.pr, S.rk, cid, groups)
    for m, w, g in zip(masks, want, (1, 2, 3)):
        np.testing.assert_array_equal(m[0].cpu().numpy(), S.limbs(w))
        assert list(bfv.decrypt_slots(S.pr, S.sk, w)) == list((ids == g).astype(int))
    cprice = S.enc(price, 70)
    sel = S.ctx.select(S.to_dev([cprice]), masks[1])
    want_sel = query.select(S.pr, S.rk, cprice, want[1])
    np.testing.assert_array_equal(sel[0].cpu().numpy(), S.limbs(want_sel))
    assert list(bfv.decrypt_slots(S.pr, S.sk, want_sel)) == list(np.where(ids == 2, price, 0))
