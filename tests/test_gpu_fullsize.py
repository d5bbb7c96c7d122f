"""Full paper size (N = 32768, 17 + 1 primes of ~49 bits, p = 65537):
sampled NTT outputs, one squaring bit-exact against the oracle (also under
a second launch shape), the whole 16-squaring mask decrypting to [x == y]
with budget to spare, the benchmark's 32-ciphertext configuration, and LT
decrypting to [x < y]."""
import numpy as np
import pytest
import torch

import synth
from oracle import bfv, encoding, ntt_def, ring
from tests.gpu_common import Setup

pytestmark = pytest.mark.gpu


def test_full_size_ntt_sampled(s32k):
    S = s32k
    rng = np.random.default_rng(3)
    polys = np.stack([rng.integers(0, q, S.pr.n) for q in S.pr.q])[None]
    got = S.ctx.ntt(torch.from_numpy(polys).to(S.ctx.device)).cpu().numpy()
    for i in (0, S.pr.L - 1):
        for j in (0, 32767, int(rng.integers(0, 32768))):
            assert got[0, i, j] == ntt_def.evaluation_at(list(polys[0, i]), S.pr.q[i], j)


def test_full_size_square_and_mask(s32k):
    S = s32k
    x, y = synth.column_pair_half_match(0, S.pr.n)
    x, y = synth.edge_differences(x, y, S.pr.t)
    cx, cy = S.enc(x, 1), S.enc(y, 2)
    z0 = bfv.sub(S.pr, cx, cy)
    want1 = bfv.square_relin(S.pr, S.rk, z0)
    dz = S.ctx.sub(S.to_dev([cx]), S.to_dev([cy]))
    got1 = S.ctx.square_relin(dz)
    np.testing.assert_array_equal(got1[0].cpu().numpy(), S.limbs(want1))
    # the other launch shapes (one workgroup per forward limb, other key
    # chunks and block sizes) give the same integers
    start = S.ctx.tuning()
    try:
        S.ctx.set_tuning(split_forward=0, ks_chunk=4, ew_block=64)
        got2 = S.ctx.square_relin(dz)
        np.testing.assert_array_equal(got2[0].cpu().numpy(), S.limbs(want1))
    finally:
        S.ctx.set_tuning(**start)
    out = S.ctx.eq_mask(S.to_dev([cx]), S.to_dev([cy]))
    got = S.from_dev(out)[0]
    mask = bfv.decrypt_slots(S.pr, S.sk, got)
    assert list(mask) == list((x == y).astype(int))
    m_true = encoding.encode((x == y).astype(int), S.pr.t)
    assert bfv.noise_bits(S.pr, S.sk, got, m_true) > 100


def test_full_size_lt_decrypts(s32k):
    """LT at the paper's parameters (p = 65537: 16 squarings, 256 babies,
    128 giants) on one ciphertext of 15-bit values against a broadcast
    constant: decrypts to [x < y] with budget left."""
    S = s32k
    rng = np.random.default_rng(11)
    x = rng.integers(0, 1 << 15, S.pr.n)
    x[:5] = [20000, 19999, 20001, 0, 32767]
    cx, cy = S.enc(x, 21), S.enc(np.full(S.pr.n, 20000), 22)
    out = S.ctx.compare(S.to_dev([cx]), S.to_dev([cy]), "lt")
    got = S.from_dev(out)[0]
    want = (x < 20000).astype(int)
    assert list(bfv.decrypt_slots(S.pr, S.sk, got)) == list(want)
    budget = bfv.noise_bits(S.pr, S.sk, got, encoding.encode(want, S.pr.t))
    print(f"LT budget left at N=32768: {budget:.1f} bits")
    assert budget > 0


def test_full_size_bench_configuration(s32k):
    """The benchmark's launch configuration: 32 ciphertexts (2^20 rows) in
    one call.  Distinct ciphertexts x_k = Enc(x) + (Delta m_k, 0) with known
    plaintexts; one squaring level bit-exact for the first and last, and the
    whole mask decrypting to [x_k == y] on a spread of them."""
    S = s32k
    n_ct = 32
    rng = np.random.default_rng(12)
    x, y = synth.column_pair_half_match(3, S.pr.n)
    cx, cy = S.enc(x, 31), S.enc(y, 32)
    shifts = [np.where(rng.random(S.pr.n) < 0.25, rng.integers(1, S.pr.t, S.pr.n), 0)
              for _ in range(n_ct)]
    shifts[0][:] = 0
    cts = []
    for d in shifts:
        m = encoding.encode(d, S.pr.t)
        c0 = (ring.as_object(cx[0]) + S.pr.delta * ring.as_object(m)) % S.pr.Q
        cts.append((c0, cx[1]))
    dx = S.to_dev(cts)
    dy = S.to_dev([cy])
    dz = S.ctx.sub(dx, S.to_dev([cy] * n_ct))
    sq = S.ctx.square_relin(dz)
    for k in (0, n_ct - 1):
        want = bfv.square_relin(S.pr, S.rk, bfv.sub(S.pr, cts[k], cy))
        np.testing.assert_array_equal(sq[k].cpu().numpy(), S.limbs(want))
    out = S.ctx.eq_mask(dx, dy)
    got = S.from_dev(out)
    for k in (0, 1, 7, 13, 20, 26, n_ct - 1):
        xk = (x + shifts[k]) % S.pr.t
        assert list(bfv.decrypt_slots(S.pr, S.sk, got[k])) == list((xk == y % S.pr.t).astype(int))


def test_full_size_batched_waves(s32k):
    """Batched EQ at full size: three instances of 3, 1 and 2 ciphertexts,
    each against its own broadcast constant, in graph waves of 2 (replayed
    twice): every mask equals the single-instance call's and decrypts."""
    S = s32k
    rng = np.random.default_rng(13)
    x = rng.integers(0, 1 << 16, S.pr.n)
    cx = S.enc(x, 41)
    items, plain = [], []
    for k, m in enumerate((3, 1, 2)):
        c = int(x[k])
        cts, xs = [], []
        for i in range(m):
            d = np.where(rng.random(S.pr.n) < 0.5, 0, rng.integers(1, S.pr.t, S.pr.n))
            mm = encoding.encode(d, S.pr.t)
            cts.append(((ring.as_object(cx[0]) + S.pr.delta * ring.as_object(mm)) % S.pr.Q, cx[1]))
            xs.append((x + d) % S.pr.t)
        items.append((S.to_dev(cts), S.to_dev([S.enc(np.full(S.pr.n, c), 50 + k)])))
        plain.append((xs, c))
    for rep in range(2):
        outs = S.ctx.eq_mask_batched(items, wave_ct=2, use_graph=True)
        torch.cuda.synchronize()
    for (dx, dy), o, (xs, c) in zip(items, outs, plain):
        ref = S.ctx.eq_mask(dx, dy)
        np.testing.assert_array_equal(o.cpu().numpy(), ref.cpu().numpy())
        got = S.from_dev(o)
        for i in range(len(xs)):
            assert list(bfv.decrypt_slots(S.pr, S.sk, got[i])) == list((xs[i] == c).astype(int))


def test_full_size_chain_matches_levels(s32k):
    """The EQ chain (each level's mod-down fused with the next level's lift,
    the split inverse's last stage applied by the consumers) gives the
    integers of the separate squarings, each bit-exact against the oracle
    above, followed by the oracle's finish."""
    S = s32k
    x, y = synth.column_pair_half_match(3, 2 * S.pr.n)
    cts = [S.enc(x[k * S.pr.n:(k + 1) * S.pr.n], 7 + k) for k in range(2)]
    cys = [S.enc(y[k * S.pr.n:(k + 1) * S.pr.n], 9 + k) for k in range(2)]
    z = S.ctx.sub(S.to_dev(cts), S.to_dev(cys))
    for _ in range(S.ctx.squarings):
        z = S.ctx.square_relin(z)
    levels = S.from_dev(z)
    got = S.ctx.eq_mask(S.to_dev(cts), S.to_dev(cys))
    for k in range(2):
        np.testing.assert_array_equal(got[k].cpu().numpy(), S.limbs(bfv.finish(S.pr, levels[k])))
