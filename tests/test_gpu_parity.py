"""Device parity: every library call against the exact-integer oracle,
residue for residue (bit-exact), on seeded inputs."""
import numpy as np
import pytest
import torch

import synth
from oracle import bfv, encoding, ntt_def
from tests.gpu_common import Setup, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def s1k():
    return Setup(10)


@pytest.fixture(scope="module")
def s64():
    return Setup(6)


def _rand_ct(S, seed, n_ct=1):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_ct):
        x = rng.integers(0, S.pr.t, S.pr.n)
        out.append(S.enc(x, seed * 100 + k))
    return out


def _assert_same(S, dev, want_cts):
    got = dev.cpu().numpy()
    for i, ct in enumerate(want_cts):
        np.testing.assert_array_equal(got[i], S.limbs(ct))


# ------------------------------------------------------------------- NTT ---

def test_ntt_matches_definition(s64):
    S = s64
    rng = np.random.default_rng(1)
    polys = np.stack([np.stack([rng.integers(0, q, S.pr.n) for q in S.pr.q]) for _ in range(2)])
    got = S.ctx.ntt(torch.from_numpy(polys).to(S.ctx.device)).cpu().numpy()
    for p in range(2):
        for i, q in enumerate(S.pr.q):
            assert list(got[p, i]) == ntt_def.evaluations(list(polys[p, i]), q), (p, i)


def test_ntt_small_workload_sampled(s1k):
    S = s1k
    rng = np.random.default_rng(2)
    polys = np.stack([rng.integers(0, q, S.pr.n) for q in S.pr.q])[None]
    got = S.ctx.ntt(torch.from_numpy(polys).to(S.ctx.device)).cpu().numpy()
    for i in (0, 7, S.pr.L - 1):
        for j in (0, 1, 511, 1023, int(rng.integers(0, 1024))):
            assert got[0, i, j] == ntt_def.evaluation_at(list(polys[0, i]), S.pr.q[i], j)


@pytest.mark.parametrize("log2_n,split", [(3, 1), (5, 1), (7, 1), (8, 1), (9, 1), (11, 1),
                                           (12, 1), (13, 1), (14, 1), (15, 1), (15, 0)])
def test_ntt_every_size_sampled(log2_n, split):
    """Every transform size (one, two and three register rounds, exchanges
    within a wavefront and across the workgroup; at 2^15 both the split
    half-limb and the full-limb forward), sampled against the definition."""
    require_gpu()
    from paper_2602_24271_amd import Context
    pr = bfv.paper_params(1 << log2_n)
    ctx = Context(log2_n, pr.t, list(pr.q), pr.P)
    ctx.set_tuning(split_forward=split)
    rng = np.random.default_rng(100 + log2_n)
    polys = np.stack([np.stack([rng.integers(0, q, pr.n) for q in pr.q]) for _ in range(2)])
    got = ctx.ntt(torch.from_numpy(polys).to(ctx.device)).cpu().numpy()
    js = sorted({0, 1, pr.n // 2 - 1, pr.n // 2, pr.n - 1, int(rng.integers(0, pr.n))})
    for p in range(2):
        for i in (0, pr.L // 2, pr.L - 1):
            for j in js:
                want = ntt_def.evaluation_at(list(polys[p, i]), pr.q[i], j)
                assert got[p, i, j] == want, (log2_n, split, p, i, j)


# ----------------------------------------------------- ciphertext calls ---

def test_sub_matches_oracle(s1k):
    S = s1k
    a, b = _rand_ct(S, 3, 2), _rand_ct(S, 4, 2)
    out = S.ctx.sub(S.to_dev(a), S.to_dev(b))
    _assert_same(S, out, [bfv.sub(S.pr, x, y) for x, y in zip(a, b)])


def test_multiply_matches_oracle(s1k):
    S = s1k
    a, b = _rand_ct(S, 5, 2), _rand_ct(S, 6, 2)
    out = S.ctx.multiply(S.to_dev(a), S.to_dev(b))
    _assert_same(S, out, [bfv.multiply(S.pr, x, y) for x, y in zip(a, b)])


def test_relinearize_matches_oracle(s1k):
    S = s1k
    a, b = _rand_ct(S, 7, 1), _rand_ct(S, 8, 1)
    c3 = bfv.multiply(S.pr, a[0], b[0])
    out = S.ctx.relinearize(S.to_dev([c3]))
    _assert_same(S, out, [bfv.relinearize(S.pr, S.rk, c3)])


def test_square_relin_matches_oracle(s1k):
    S = s1k
    a = _rand_ct(S, 9, 3)
    out = S.ctx.square_relin(S.to_dev(a))
    _assert_same(S, out, [bfv.square_relin(S.pr, S.rk, x) for x in a])


def test_mul_relin_matches_oracle_and_decrypts(s1k):
    S = s1k
    rng = np.random.default_rng(10)
    xa, xb = rng.integers(0, S.pr.t, S.pr.n), rng.integers(0, S.pr.t, S.pr.n)
    a, b = S.enc(xa, 11), S.enc(xb, 12)
    out = S.ctx.mul_relin(S.to_dev([a]), S.to_dev([b]))
    want = bfv.mul_relin(S.pr, S.rk, a, b)
    _assert_same(S, out, [want])
    assert list(bfv.decrypt_slots(S.pr, S.sk, S.from_dev(out)[0])) == list(xa * xb % S.pr.t)


def test_eq_chain_every_level_small_workload(s1k):
    """N = 1024, p = 65537: every one of the 16 squarings bit-exact, the
    final mask ciphertext bit-exact, and the mask decrypts to [x == y]."""
    S = s1k
    x, y = synth.column_pair_half_match(0, S.pr.n)
    x, y = synth.edge_differences(x, y, S.pr.t)
    cx, cy = S.enc(x, 1), S.enc(y, 2)
    levels, out = bfv.eq_chain(S.pr, S.rk, cx, cy)
    z = S.ctx.sub(S.to_dev([cx]), S.to_dev([cy]))
    _assert_same(S, z, [levels[0]])
    for k in range(1, len(levels)):
        z = S.ctx.square_relin(z)
        _assert_same(S, z, [levels[k]])
    got = S.ctx.eq_mask(S.to_dev([cx]), S.to_dev([cy]))
    _assert_same(S, got, [out])
    mask = bfv.decrypt_slots(S.pr, S.sk, S.from_dev(got)[0])
    assert list(mask) == list((x == y).astype(int))


def test_eq_mask_broadcast_constant(s1k):
    """Structured column (sorted dictionary ids) against one encrypted
    constant broadcast over several ciphertexts."""
    S = s1k
    x, y = synth.column_structured(1, 3 * S.pr.n)
    cxs = [S.enc(x[k * S.pr.n:(k + 1) * S.pr.n], 20 + k) for k in range(3)]
    cy = S.enc(y[:S.pr.n], 30)
    got = S.ctx.eq_mask(S.to_dev(cxs), S.to_dev([cy]))
    for k in range(3):
        _, want = bfv.eq_chain(S.pr, S.rk, cxs[k], cy)
        np.testing.assert_array_equal(got[k].cpu().numpy(), S.limbs(want))


def test_crafted_coefficients_take_the_exact_path(s1k):
    """Coefficients (Q-1)/2, (Q+1)/2, 0, 1, Q-1 and residues q_i - 1 sit on
    the centred-lift decision boundary; results stay bit-exact and the
    exact fallback is counted."""
    S = s1k
    Q = S.pr.Q
    rng = np.random.default_rng(13)
    special = [(Q - 1) // 2, (Q + 1) // 2, 0, 1, Q - 1, (Q - 3) // 2, (Q + 3) // 2]
    c0 = [special[i % len(special)] if i % 5 == 0 else int(rng.integers(0, 1 << 62)) * int(rng.integers(1, 1 << 62)) % Q
          for i in range(S.pr.n)]
    c1 = [special[(i + 3) % len(special)] if i % 7 == 0 else int(rng.integers(0, 1 << 62)) ** 13 % Q
          for i in range(S.pr.n)]
    ct = (np.array(c0, dtype=object), np.array(c1, dtype=object))
    S.ctx.reset_margin_events()
    out = S.ctx.multiply(S.to_dev([ct]), S.to_dev([ct]))
    _assert_same(S, out, [bfv.multiply(S.pr, ct, ct)])
    assert S.ctx.margin_events() > 0
    out = S.ctx.square_relin(S.to_dev([ct]))
    _assert_same(S, out, [bfv.square_relin(S.pr, S.rk, ct)])


def test_empty_and_shape_errors(s1k):
    S = s1k
    e = torch.empty((0, 2, S.pr.L, S.pr.n), dtype=torch.int64, device=S.ctx.device)
    assert S.ctx.eq_mask(e, e).shape[0] == 0
    assert S.ctx.square_relin(e).shape[0] == 0
    bad = torch.zeros((1, 2, S.pr.L, S.pr.n // 2), dtype=torch.int64, device=S.ctx.device)
    with pytest.raises(ValueError):
        S.ctx.square_relin(bad)


def test_margin_counter_quiet_on_encryptions(s1k):
    S = s1k
    S.ctx.reset_margin_events()
    a = _rand_ct(S, 40, 2)
    S.ctx.square_relin(S.to_dev(a))
    assert S.ctx.margin_events() == 0
