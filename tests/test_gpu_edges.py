"""Edge cases on the device: the largest and smallest prime counts the
library is built for (bit-exact against the oracle), and degenerate
operator inputs (repeated IN members, LT outside its range, an empty
join, a join row out of range)."""
import numpy as np
import pytest
import torch

import synth
from oracle import bfv, compare, join, nt, query
from paper_2602_24271_amd import Context
from tests.gpu_common import Setup, galois_keys, require_gpu

pytestmark = pytest.mark.gpu


class CustomSetup(Setup):
    """Setup with an explicit prime chain (q descending, then P)."""

    def __init__(self, log2_n, q, P, t=65537, seed=0):
        require_gpu()
        n = 1 << log2_n
        self.pr = bfv.Params(n, t, tuple(q), P)
        self.sk, self.rk = bfv.keygen(self.pr, synth.key_randomness(seed, n, self.pr.moduli_pq,
                                                                     self.pr.L))
        self.ctx = Context(log2_n, t, list(q), P)
        self.ctx.set_relin_key(torch.from_numpy(self.rk.limbs(self.pr)).to(self.ctx.device))


def test_prime_count_extremes_bit_exact():
    """L = 24 (the most primes): one squaring and the whole mask."""
    L = 24
    primes = nt.primes_congruent_one_below(1 << 49, 1 << 16, L + 1)
    S = CustomSetup(8, primes[1:], primes[0], seed=L)
    x, y = synth.column_pair_half_match(L, S.pr.n)
    cx, cy = S.enc(x, 1), S.enc(y, 2)
    dz = S.ctx.sub(S.to_dev([cx]), S.to_dev([cy]))
    sq = S.ctx.square_relin(dz)
    np.testing.assert_array_equal(sq[0].cpu().numpy(),
                                  S.limbs(bfv.square_relin(S.pr, S.rk, bfv.sub(S.pr, cx, cy))))
    levels, want = bfv.eq_chain(S.pr, S.rk, cx, cy)
    got = S.ctx.eq_mask(S.to_dev([cx]), S.to_dev([cy]))
    np.testing.assert_array_equal(got[0].cpu().numpy(), S.limbs(want))
    assert list(bfv.decrypt_slots(S.pr, S.sk, want)) == list((x == y).astype(int))


def test_two_primes_depth_budget():
    """L = 2 (Q of 98 bits): the budget allows two multiplications, so the
    16-level mask is refused with NSHE_EDEPTH before any work (it would not
    decrypt), while the squarings the budget allows are bit-exact and still
    decrypt; the binding's per-ciphertext depth counter refuses the third."""
    from paper_2602_24271_amd._lib import NsheError, NSHE_EDEPTH
    L = 2
    primes = nt.primes_congruent_one_below(1 << 49, 1 << 16, L + 1)
    S = CustomSetup(8, primes[1:], primes[0], seed=L)
    assert S.ctx.depth_budget == 2
    x, y = synth.column_pair_half_match(L, S.pr.n)
    cx, cy = S.enc(x, 1), S.enc(y, 2)
    dx, dy = S.to_dev([cx]), S.to_dev([cy])
    with pytest.raises(NsheError) as e:
        S.ctx.eq_mask(dx, dy)
    assert e.value.code == NSHE_EDEPTH
    ws = S.ctx.workspace(1)
    out = torch.empty_like(dx)
    rc = S.ctx._lib.nshe_eq_mask(S.ctx._h, dx.data_ptr(), dy.data_ptr(), out.data_ptr(), 1, 0,
                                 ws.data_ptr(), ws.numel(), None)
    assert rc == NSHE_EDEPTH
    z = S.ctx.sub(dx, dy)
    want = bfv.sub(S.pr, cx, cy)
    zz = (x - y) % S.pr.t
    for k in (1, 2):
        z = S.ctx.square_relin(z)
        want = bfv.square_relin(S.pr, S.rk, want)
        np.testing.assert_array_equal(z[0].cpu().numpy(), S.limbs(want))
        assert S.ctx.depth(z) == k
        assert list(bfv.decrypt_slots(S.pr, S.sk, want)) == \
            [pow(int(v), 2 ** k, S.pr.t) for v in zz]
    with pytest.raises(NsheError) as e:
        S.ctx.square_relin(z)
    assert e.value.code == NSHE_EDEPTH


@pytest.fixture(scope="module")
def s256():
    S = Setup(8, seed=15)
    S.keys = galois_keys(S, seed=800)
    return S


def test_in_mask_repeated_members(s256):
    S = s256
    x = np.random.default_rng(2).choice(np.array([4, 5, 6]), S.pr.n)
    cx = S.enc(x, 3)
    members = [S.enc(np.full(S.pr.n, v), 10 + i) for i, v in enumerate([4, 4, 6])]
    got = S.ctx.in_mask(S.to_dev([cx]), S.to_dev(members))
    want = query.in_mask(S.pr, S.rk, cx, members)
    np.testing.assert_array_equal(got[0].cpu().numpy(), S.limbs(want))
    assert list(bfv.decrypt_slots(S.pr, S.sk, want)) == [2 * int(v == 4) + int(v == 6) for v in x]


def test_join_degenerate_inputs(s256):
    from paper_2602_24271_amd._lib import NsheError
    S = s256
    a = S.to_dev([S.enc(np.arange(S.pr.n), 20)])
    b = S.to_dev([S.enc(np.arange(S.pr.n), 21)])
    empty = S.ctx.join_sum(a, b, b, [])
    assert int(empty.abs().sum()) == 0
    for bad in ([-1], [S.pr.n]):
        with pytest.raises(NsheError) as e:
            S.ctx.join_sum(a, b, b, bad)
        assert e.value.code == -1


def test_lt_outside_range_matches_oracle():
    """|x - y| > (t-1)/2 wraps; the device computes the same integers."""
    S = Setup(3, t=17, seed=16)
    x = [0, 0, 16, 12, 3, 9, 1, 15]
    y = [9, 16, 0, 2, 14, 0, 12, 5]
    cx, cy = S.enc(x, 30), S.enc(y, 31)
    got = S.ctx.compare(S.to_dev([cx]), S.to_dev([cy]), "lt")
    want = compare.lt(S.pr, S.rk, cx, cy)
    np.testing.assert_array_equal(got[0].cpu().numpy(), S.limbs(want))
    A = set(compare.negative_half(17))
    assert list(bfv.decrypt_slots(S.pr, S.sk, want)) == [int((a - b) % 17 in A) for a, b in zip(x, y)]


def test_launch_sequence_is_data_oblivious(s256):
    """The same kernels, launch counts and work for a structured encrypted
    column and for uniform residues: nothing in the path depends on values."""
    S = s256
    x, y = synth.column_structured(1, S.pr.n)
    enc = S.to_dev([S.enc(x, 40)]), S.to_dev([S.enc(y, 41)])
    uni = tuple(synth.uniform_device_residues((1, 2), list(S.pr.q), S.pr.n, 42 + i, S.ctx.device)
                for i in range(2))
    seen = []
    for a, b in (enc, uni):
        S.ctx.profile(True)
        S.ctx.eq_mask(a, b)
        torch.cuda.synchronize()
        rec = S.ctx.profile_read()
        S.ctx.profile(False)
        seen.append({k: (v["launches"], v["work"]) for k, v in rec.items()})
    assert seen[0] == seen[1] and seen[0]
