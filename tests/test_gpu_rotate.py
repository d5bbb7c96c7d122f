"""Device parity of slot rotations and the rotate-and-add aggregation
(COUNT, SUM; Sec. 4.2.2): bit-exact against the oracle, decrypting to rotated
slots and to totals."""
import numpy as np
import pytest
import torch

from oracle import bfv, galois, query
from tests.gpu_common import Setup, galois_keys

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def s256():
    S = Setup(8, seed=6)
    S.keys = galois_keys(S)
    return S


def test_galois_elements_match_oracle(s256):
    assert s256.ctx.galois_elements() == galois.sum_elements(s256.pr.n)


def test_rotations_match_oracle(s256):
    S = s256
    v = np.random.default_rng(1).integers(0, S.pr.t, S.pr.n)
    cts = [S.enc(v, 2), S.enc(v[::-1].copy(), 3)]
    dev = S.to_dev(cts)
    for g in galois.sum_elements(S.pr.n):
        got = S.ctx.rotate(dev, g)
        for k, ct in enumerate(cts):
            want = galois.apply_galois(S.pr, S.keys[g], ct, g)
            np.testing.assert_array_equal(got[k].cpu().numpy(), S.limbs(want))


def test_missing_key_is_reported(s256):
    from paper_2602_24271_amd._lib import NsheError
    S = s256
    dev = S.to_dev([S.enc(np.zeros(S.pr.n, dtype=np.int64), 4)])
    with pytest.raises(NsheError) as e:
        S.ctx.rotate(dev, 5)
    assert e.value.code == -6
    with pytest.raises(NsheError):
        S.ctx.set_galois_key(4, torch.zeros((S.pr.L, 2, S.pr.L + 1, S.pr.n), dtype=torch.int64,
                                            device=S.ctx.device))


def test_count_and_sum_of_a_selection(s256):
    """COUNT(*) WHERE id = key and SUM(price) WHERE id = key, on the device
    from the mask on: each step bit-exact, totals decrypt in every slot."""
    S = s256
    rng = np.random.default_rng(7)
    ids = rng.integers(0, 4, S.pr.n)
    price = rng.integers(0, 200, S.pr.n)
    cid, ckey, cprice = S.enc(ids, 8), S.enc(np.full(S.pr.n, 2), 9), S.enc(price, 10)
    mask = S.ctx.eq_mask(S.to_dev([cid]), S.to_dev([ckey]))
    _, want_mask = bfv.eq_chain(S.pr, S.rk, cid, ckey)
    np.testing.assert_array_equal(mask[0].cpu().numpy(), S.limbs(want_mask))
    count = S.ctx.sum_slots(mask)
    want_count = galois.sum_slots(S.pr, S.keys, want_mask)
    np.testing.assert_array_equal(count[0].cpu().numpy(), S.limbs(want_count))
    assert list(bfv.decrypt_slots(S.pr, S.sk, want_count)) == [int((ids == 2).sum())] * S.pr.n
    sel = S.ctx.select(S.to_dev([cprice]), mask)
    total = S.ctx.sum_slots(sel)
    want_total = galois.sum_slots(S.pr, S.keys, query.select(S.pr, S.rk, cprice, want_mask))
    np.testing.assert_array_equal(total[0].cpu().numpy(), S.limbs(want_total))
    assert list(bfv.decrypt_slots(S.pr, S.sk, want_total)) == \
        [int(price[ids == 2].sum()) % S.pr.t] * S.pr.n
