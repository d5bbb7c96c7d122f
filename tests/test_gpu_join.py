"""Device parity of plaintext products, Extract / Broadcast (Sec. 2.1.6)
and the fused equi-join aggregation (Sec. 4.2.2, JOIN): bit-exact against the
oracle, decrypting to the plain join."""
import numpy as np
import pytest
import torch

from oracle import bfv, encoding, join
from tests.gpu_common import Setup, galois_keys

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def s256():
    S = Setup(8, seed=14)
    S.keys = galois_keys(S, seed=700)
    return S


def test_mul_plain_matches_oracle(s256):
    S = s256
    rng = np.random.default_rng(1)
    cts = [S.enc(rng.integers(0, S.pr.t, S.pr.n), 2), S.enc(rng.integers(0, S.pr.t, S.pr.n), 3)]
    m = encoding.encode(rng.integers(0, S.pr.t, S.pr.n), S.pr.t)
    got = S.ctx.mul_plain(S.to_dev(cts), torch.from_numpy(np.asarray(m, dtype=np.int64)).to(S.ctx.device))
    for k, ct in enumerate(cts):
        np.testing.assert_array_equal(got[k].cpu().numpy(), S.limbs(join.mul_plain(S.pr, ct, m)))


def test_extract_and_broadcast_match_oracle(s256):
    S = s256
    v = np.random.default_rng(4).integers(0, 5000, S.pr.n)
    ct = S.enc(v, 5)
    dev = S.to_dev([ct])
    for j in (0, 5, S.pr.n // 2, S.pr.n - 1):
        e = S.ctx.extract(dev, j)
        np.testing.assert_array_equal(e[0].cpu().numpy(), S.limbs(join.extract(S.pr, ct, j)))
        b = S.ctx.extract(dev, j, broadcast=True)
        want = join.broadcast(S.pr, S.keys, ct, j)
        np.testing.assert_array_equal(b[0].cpu().numpy(), S.limbs(want))
        assert list(bfv.decrypt_slots(S.pr, S.sk, want)) == [int(v[j])] * S.pr.n


def test_join_sum_matches_oracle(s256):
    S = s256
    rng = np.random.default_rng(6)
    b_key = rng.permutation(np.arange(1000, 1000 + S.pr.n))
    b_attr = rng.integers(1, 40000, S.pr.n)
    a_keys = [rng.choice(np.concatenate([b_key[:8], np.array([1, 2, 3])]), S.pr.n) for _ in range(2)]
    ca = [S.enc(a, 10 + i) for i, a in enumerate(a_keys)]
    cbk, cba = S.enc(b_key, 20), S.enc(b_attr, 21)
    rows = [1, 3]
    got = S.ctx.join_sum(S.to_dev(ca), S.to_dev([cbk]), S.to_dev([cba]), rows)
    torch.cuda.synchronize()
    lookup = {int(b_key[j]): int(b_attr[j]) for j in rows}
    for i in range(2):
        want = join.join_sum(S.pr, S.rk, S.keys, ca[i], cbk, cba, rows)
        np.testing.assert_array_equal(got[i].cpu().numpy(), S.limbs(want))
        assert list(bfv.decrypt_slots(S.pr, S.sk, want)) == [lookup.get(int(k), 0) for k in a_keys[i]]
