"""Device parity with key switching by digits of several data primes
(hybrid: alpha = 2, the paper's 18 primes as 16 data primes and two special
primes, digits D_j = [c2]_{q_2j q_2j+1}, P = P_0 P_1; alpha = 3, 15 data
primes and three special primes, digits of three primes), bit-exact against
the oracle, for each alpha:

* N = 1024 against the oracle computed here: relinearization, squarings,
  products, every level of the EQ chain (Eq. eq:equality) and its mask, a
  broadcast constant, the exact-lift fallback, rotations and the
  rotate-and-add with real Galois keys, both key-switch ciphertext chunks;
* N = 64 at p = 65537: LT, LE and BETWEEN (Eq. eq:inequality), the paper's
  comparison program shape;
* N = 32768 against the stored oracle digests (tests/golden/fullsize_a2_*,
  fullsize_a3_*): the split digit transforms, the fused chain (k_sub_lift,
  k_moddown_lift, k_moddown_finish with the several-prime mod-down), 8 (4)
  ciphertexts of each 2^20-row column, rotations, SELECT, Extract,
  Broadcast, JOIN and the comparisons at t = 17.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import bfv, galois
from paper_2602_24271_amd import Context
from tests import fullsize_cases as fc
from tests.gpu_common import Setup, galois_keys

pytestmark = pytest.mark.gpu


ALPHAS = [2, 3]


@pytest.fixture(scope="module", params=ALPHAS, ids=[f"alpha{a}" for a in ALPHAS])
def a1k(request):
    return Setup(10, alpha=request.param)


def _full(request, alpha):
    return request.getfixturevalue(f"s32k_a{alpha}")


COLUMN_CTS = {2: fc.A2_COLUMN_CTS, 3: fc.A3_COLUMN_CTS}


def _rand_ct(S, seed, n_ct=1):
    rng = np.random.default_rng(seed)
    return [S.enc(rng.integers(0, S.pr.t, S.pr.n), seed * 100 + k) for k in range(n_ct)]


def _same(S, dev, want_cts):
    got = dev.cpu().numpy()
    for i, ct in enumerate(want_cts):
        np.testing.assert_array_equal(got[i], S.limbs(ct))


# ------------------------------------------------------------ N = 1024 ---

def test_context_describes_its_digits(a1k):
    S = a1k
    a = S.pr.alpha
    assert (S.ctx.alpha, S.ctx.dnum, S.ctx.L) == (a, 18 // a - 1, 18 - a)
    assert S.ctx.key_shape == (S.ctx.dnum, 2, 18, S.pr.n)
    assert S.ctx.special == list(S.pr.special)
    with pytest.raises(ValueError):
        S.ctx.set_relin_key(torch.zeros((S.ctx.L, 2, S.ctx.L + 1, S.pr.n), dtype=torch.int64,
                                        device=S.ctx.device))


def test_multiply_keeps_residues(a1k):
    """A three-component product is returned as canonical residues (the
    digit pairs are only the relinearization's internal format)."""
    S = a1k
    a, b = _rand_ct(S, 5, 2), _rand_ct(S, 6, 2)
    out = S.ctx.multiply(S.to_dev(a), S.to_dev(b))
    _same(S, out, [bfv.multiply(S.pr, x, y) for x, y in zip(a, b)])


def test_relinearize_and_square(a1k):
    S = a1k
    a, b = _rand_ct(S, 7), _rand_ct(S, 8)
    c3 = bfv.multiply(S.pr, a[0], b[0])
    _same(S, S.ctx.relinearize(S.to_dev([c3])), [bfv.relinearize(S.pr, S.rk, c3)])
    sq = _rand_ct(S, 9, 3)
    _same(S, S.ctx.square_relin(S.to_dev(sq)), [bfv.square_relin(S.pr, S.rk, x) for x in sq])


@pytest.mark.parametrize("chunk", [4, 32])
def test_mul_relin_chunks(a1k, chunk):
    S = a1k
    rng = np.random.default_rng(10)
    xa, xb = rng.integers(0, S.pr.t, S.pr.n), rng.integers(0, S.pr.t, S.pr.n)
    a, b = S.enc(xa, 11), S.enc(xb, 12)
    start = S.ctx.tuning()
    try:
        S.ctx.set_tuning(ks_chunk=chunk)
        out = S.ctx.mul_relin(S.to_dev([a]), S.to_dev([b]))
    finally:
        S.ctx.set_tuning(**start)
    _same(S, out, [bfv.mul_relin(S.pr, S.rk, a, b)])
    assert list(bfv.decrypt_slots(S.pr, S.sk, S.from_dev(out)[0])) == list(xa * xb % S.pr.t)


def test_eq_chain_every_level(a1k):
    S = a1k
    x, y = synth.column_pair_half_match(0, S.pr.n)
    x, y = synth.edge_differences(x, y, S.pr.t)
    cx, cy = S.enc(x, 1), S.enc(y, 2)
    levels, out = bfv.eq_chain(S.pr, S.rk, cx, cy)
    z = S.ctx.sub(S.to_dev([cx]), S.to_dev([cy]))
    _same(S, z, [levels[0]])
    for k in range(1, len(levels)):
        z = S.ctx.square_relin(z)
        _same(S, z, [levels[k]])
    got = S.ctx.eq_mask(S.to_dev([cx]), S.to_dev([cy]))
    _same(S, got, [out])
    assert list(bfv.decrypt_slots(S.pr, S.sk, S.from_dev(got)[0])) == list((x == y).astype(int))


def test_eq_mask_broadcast_and_batched(a1k):
    S = a1k
    x, y = synth.column_structured(1, 3 * S.pr.n)
    cxs = [S.enc(x[k * S.pr.n:(k + 1) * S.pr.n], 20 + k) for k in range(3)]
    cy = S.enc(y[:S.pr.n], 30)
    want = [bfv.eq_chain(S.pr, S.rk, c, cy)[1] for c in cxs]
    _same(S, S.ctx.eq_mask(S.to_dev(cxs), S.to_dev([cy])), want)
    outs = S.ctx.eq_mask_batched([(S.to_dev(cxs[:2]), S.to_dev([cy])),
                                  (S.to_dev(cxs[2:]), S.to_dev([cy]))], wave_ct=2, use_graph=True)
    _same(S, outs[0], want[:2])
    _same(S, outs[1], want[2:])


def _eq_both_schedules(S, dx, dy):
    """EQ of dx against dy with one stream and with the call's two halves on
    two streams (tuning streams); also out aliasing x.  Returns the one-stream
    mask after checking that the others equal it."""
    start = S.ctx.tuning()
    try:
        S.ctx.set_tuning(streams=1)
        one = S.ctx.eq_mask(dx, dy)
        S.ctx.set_tuning(streams=2)
        two = S.ctx.eq_mask(dx, dy)
        xa = dx.clone()
        S.ctx.eq_mask(xa, dy, out=xa)
    finally:
        S.ctx.set_tuning(**start)
    assert torch.equal(two, one)
    assert torch.equal(xa, one)
    return one


def test_eq_mask_two_streams(a1k):
    """33 ciphertexts (halves of 16 and 17 on two streams): the same masks as
    on one stream, the first and last (the same pair) the oracle's, with y per
    ciphertext and broadcast."""
    S = a1k
    x, y = synth.column_pair_half_match(5, S.pr.n)
    cx, cy = S.enc(x, 51), S.enc(y, 52)
    want = bfv.eq_chain(S.pr, S.rk, cx, cy)[1]
    dx, dy = S.to_dev([cx]), S.to_dev([cy])
    ox = synth.uniform_device_residues((31, 2), S.ctx.q, S.ctx.n, 53, S.ctx.device)
    oy = synth.uniform_device_residues((31, 2), S.ctx.q, S.ctx.n, 54, S.ctx.device)
    X = torch.cat([dx, ox, dx]).contiguous()
    for Y in (torch.cat([dy, oy, dy]).contiguous(), dy):
        got = _eq_both_schedules(S, X, Y)
        _same(S, got[[0, 32]], [want, want])


def test_wide_lift_window(a1k):
    S = a1k
    x, y = synth.column_pair_half_match(3, S.pr.n)
    cx, cy = S.enc(x, 5), S.enc(y, 6)
    S.ctx.set_debug(wide_lift_window=True)
    try:
        out = S.ctx.eq_mask(S.to_dev([cx]), S.to_dev([cy]))
    finally:
        S.ctx.set_debug()
    _same(S, out, [bfv.eq_chain(S.pr, S.rk, cx, cy)[1]])


def test_rotations_and_sum_slots(a1k):
    """Rotations: the automorphism's canonical digit source is turned into
    digit pairs by k_digit_mrc before the key switch."""
    S = a1k
    keys = galois_keys(S)
    v = np.random.default_rng(41).integers(0, S.pr.t, S.pr.n)
    ct = S.enc(v, 41)
    g = galois.rotation_element(S.pr.n, 1)
    rot = S.ctx.rotate(S.to_dev([ct]), g)
    _same(S, rot, [galois.apply_galois(S.pr, keys[g], ct, g)])
    tot = S.ctx.sum_slots(S.to_dev([ct]))
    _same(S, tot, [galois.sum_slots(S.pr, keys, ct)])
    assert list(bfv.decrypt_slots(S.pr, S.sk, S.from_dev(tot)[0])) == [int(v.sum()) % S.pr.t] * S.pr.n


# -------------------------------------------------------------- N = 64 ---

@pytest.mark.parametrize("alpha", ALPHAS)
def test_lt_le_between_paper_prime_n64(alpha):
    S = Setup(6, alpha=alpha)
    E = fc.Env.from_keys(S.pr, S.sk, S.rk)
    g = fc.load_golden(f"a{alpha}_lt_n64")
    (x, y, lo, hi), cts = fc.lt_n64_inputs(E)
    dev = [S.to_dev([c]) for c in cts]
    lt = S.ctx.compare(dev[0], dev[1], "lt")
    fc.check(g, "lt", lt[0].cpu().numpy())
    assert list(bfv.decrypt_slots(S.pr, S.sk, S.from_dev(lt)[0])) == list((x < y).astype(int))
    fc.check(g, "le", S.ctx.compare(dev[0], dev[1], "le")[0].cpu().numpy())
    bt = S.ctx.between(dev[0], dev[2], dev[3])
    fc.check(g, "between", bt[0].cpu().numpy())


# ----------------------------------------------------------- N = 32768 ---

def _env(S):
    return fc.Env.from_keys(S.pr, S.sk, S.rk)


@pytest.mark.parametrize("alpha", ALPHAS)
def test_full_size_chain_every_level_and_paths(request, alpha):
    S = _full(request, alpha)
    E = _env(S)
    g = fc.load_golden(f"a{alpha}_eq_edges")
    x, y, cx, cy = fc.eq_edges_inputs(E)
    dx, dy = S.to_dev([cx]), S.to_dev([cy])
    z = S.ctx.sub(dx, dy)
    fc.check(g, "level_00", z[0].cpu().numpy())
    for k in range(1, 17):
        z = S.ctx.square_relin(z)
        fc.check(g, f"level_{k:02d}", z[0].cpu().numpy())
    mask = S.ctx.eq_mask(dx, dy)
    fc.check(g, "mask", mask[0].cpu().numpy())
    assert list(bfv.decrypt_slots(S.pr, S.sk, S.from_dev(mask)[0])) == list((x == y).astype(int))
    outs = S.ctx.eq_mask_batched([(dx, dy)], wave_ct=1, use_graph=True)
    fc.check(g, "mask", outs[0][0].cpu().numpy())
    # a product's three components (canonical residues) relinearized on
    # their own: the same first level
    z0 = S.ctx.sub(dx, dy)
    fc.check(g, "level_01", S.ctx.relinearize(S.ctx.multiply(z0, z0))[0].cpu().numpy())
    start = S.ctx.tuning()
    try:
        # the full-limb transforms and unsplit consumers at 2^15
        S.ctx.set_tuning(split_forward=0)
        fc.check(g, "level_01", S.ctx.square_relin(S.ctx.sub(dx, dy))[0].cpu().numpy())
        fc.check(g, "mask", S.ctx.eq_mask(dx, dy)[0].cpu().numpy())
    finally:
        S.ctx.set_tuning(**start)


@pytest.mark.parametrize("alpha", ALPHAS)
def test_full_size_key_switch_chunks(request, alpha):
    """The benchmark's shape of the key-switch product: 33 ciphertexts (16
    per pass with the digit transforms by parity, a ragged last chunk of
    one), squared once at every chunk width (4, 8, 16, 32): all equal, and
    the first and last ciphertexts (the golden input) bit-exact against the
    oracle's level."""
    S = _full(request, alpha)
    E = _env(S)
    g = fc.load_golden(f"a{alpha}_eq_edges")
    x, y, cx, cy = fc.eq_edges_inputs(E)
    z1 = S.ctx.sub(S.to_dev([cx]), S.to_dev([cy]))
    others = synth.uniform_device_residues((31, 2), S.ctx.q, S.ctx.n, 77, S.ctx.device)
    z = torch.cat([z1, others, z1]).contiguous()
    start = S.ctx.tuning()
    outs = []
    try:
        for ch in (4, 8, 16, 32):
            S.ctx.set_tuning(ks_chunk=ch)
            outs.append(S.ctx.square_relin(z))
    finally:
        S.ctx.set_tuning(**start)
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    fc.check(g, "level_01", outs[0][0].cpu().numpy())
    fc.check(g, "level_01", outs[0][32].cpu().numpy())


@pytest.mark.parametrize("alpha", ALPHAS)
def test_full_size_eq_mask_two_streams(request, alpha):
    """The benchmark's schedule at the paper's size: 33 ciphertexts, the
    call's halves on two streams, equal to one stream; the first and last
    ciphertexts (the golden pair) bit-exact against the oracle's mask."""
    S = _full(request, alpha)
    E = _env(S)
    g = fc.load_golden(f"a{alpha}_eq_edges")
    x, y, cx, cy = fc.eq_edges_inputs(E)
    dx, dy = S.to_dev([cx]), S.to_dev([cy])
    ox = synth.uniform_device_residues((31, 2), S.ctx.q, S.ctx.n, 78, S.ctx.device)
    oy = synth.uniform_device_residues((31, 2), S.ctx.q, S.ctx.n, 79, S.ctx.device)
    X = torch.cat([dx, ox, dx]).contiguous()
    for Y in (torch.cat([dy, oy, dy]).contiguous(), dy):
        got = _eq_both_schedules(S, X, Y)
        fc.check(g, "mask", got[0].cpu().numpy())
        fc.check(g, "mask", got[32].cpu().numpy())


@pytest.mark.parametrize("alpha", ALPHAS)
def test_full_size_batched_two_streams(request, alpha):
    """Batched EQ at the paper's size with waves of 32: 40 ciphertexts (the
    golden pair first) in instances of 25 and 15, half-waves of 16, 16 and 8
    on two streams: equal to the plain call on one stream, the golden pair's
    mask the oracle's."""
    S = _full(request, alpha)
    E = _env(S)
    g = fc.load_golden(f"a{alpha}_eq_edges")
    x, y, cx, cy = fc.eq_edges_inputs(E)
    dx, dy = S.to_dev([cx]), S.to_dev([cy])
    ox = synth.uniform_device_residues((39, 2), S.ctx.q, S.ctx.n, 80, S.ctx.device)
    oy = synth.uniform_device_residues((39, 2), S.ctx.q, S.ctx.n, 81, S.ctx.device)
    X = torch.cat([dx, ox]).contiguous()
    Y = torch.cat([dy, oy]).contiguous()
    items = [(X[:25], Y[:25]), (X[25:], Y[25:])]
    start = S.ctx.tuning()
    try:
        S.ctx.set_tuning(streams=1)
        ref = [S.ctx.eq_mask(a, b) for a, b in items]
        S.ctx.set_tuning(streams=2)
        for rep in range(2):
            outs = S.ctx.eq_mask_batched(items, wave_ct=32, use_graph=True)
            torch.cuda.synchronize()
            for o, r in zip(outs, ref):
                assert torch.equal(o, r)
    finally:
        S.ctx.set_tuning(**start)
    fc.check(g, "mask", ref[0][0].cpu().numpy())


@pytest.mark.parametrize("alpha", ALPHAS)
def test_full_size_columns(request, alpha):
    S = _full(request, alpha)
    E = _env(S)
    n_ct = COLUMN_CTS[alpha]
    gu = fc.load_golden(f"a{alpha}_eq_column_uniform")
    pairs = [fc.column_uniform_cts(E, k) for k in range(n_ct)]
    out = S.ctx.eq_mask(S.to_dev([p[0] for p in pairs]), S.to_dev([p[1] for p in pairs]))
    got = out.cpu().numpy()
    for k in range(n_ct):
        fc.check(gu, f"mask_{k:02d}", got[k])
    gs = fc.load_golden(f"a{alpha}_eq_column_structured")
    xs = S.to_dev([fc.column_structured_ct(E, k) for k in range(n_ct)])
    out = S.ctx.eq_mask(xs, S.to_dev([fc.column_structured_constant(E)]))
    got = out.cpu().numpy()
    for k in range(n_ct):
        fc.check(gs, f"mask_{k:02d}", got[k])


def _uniform_keys(S):
    """Stand-in (uniform) Galois keys for every element of the sum, loaded
    once per context."""
    if not getattr(S, "uniform_keys_loaded", False):
        for gel, limbs in fc.uniform_galois_limbs(S.pr).items():
            S.ctx.set_galois_key(gel, torch.from_numpy(limbs).to(S.ctx.device))
        S.uniform_keys_loaded = True


@pytest.mark.parametrize("alpha", ALPHAS)
def test_full_size_rotations(request, alpha):
    S = _full(request, alpha)
    _uniform_keys(S)
    E = _env(S)
    g = fc.load_golden(f"a{alpha}_rotations")
    v, ct = fc.rotate_inputs(E)
    gel, key = fc.real_rotation(E)
    S.ctx.set_galois_key(gel, torch.from_numpy(key.limbs(S.pr)).to(S.ctx.device))
    out = S.ctx.rotate(S.to_dev([ct]), gel)
    fc.check(g, "rotate", out[0].cpu().numpy())
    h = S.pr.n // 2
    want = np.concatenate([np.roll(v[:h], -1), np.roll(v[h:], -1)])
    assert list(bfv.decrypt_slots(S.pr, S.sk, S.from_dev(out)[0])) == list(want)
    # the real key of rotation by one replaced the stand-in: reload it
    S.ctx.set_galois_key(gel, torch.from_numpy(fc.uniform_galois_limbs(S.pr)[gel]).to(S.ctx.device))
    fc.check(g, "sum_slots", S.ctx.sum_slots(S.to_dev([ct]))[0].cpu().numpy())


@pytest.mark.parametrize("alpha", ALPHAS)
def test_full_size_sum_slots_two_streams(request, alpha):
    """The rotate-and-add over 33 ciphertexts (the golden one first and last)
    on one stream and with its halves on two: equal, and the golden
    ciphertexts' sums the oracle's."""
    S = _full(request, alpha)
    _uniform_keys(S)
    E = _env(S)
    g = fc.load_golden(f"a{alpha}_rotations")
    v, ct = fc.rotate_inputs(E)
    d = S.to_dev([ct])
    others = synth.uniform_device_residues((31, 2), S.ctx.q, S.ctx.n, 82, S.ctx.device)
    X = torch.cat([d, others, d]).contiguous()
    start = S.ctx.tuning()
    try:
        S.ctx.set_tuning(streams=1)
        one = S.ctx.sum_slots(X)
        S.ctx.set_tuning(streams=2)
        two = S.ctx.sum_slots(X)
    finally:
        S.ctx.set_tuning(**start)
    assert torch.equal(two, one)
    fc.check(g, "sum_slots", one[0].cpu().numpy())
    fc.check(g, "sum_slots", one[32].cpu().numpy())


@pytest.mark.parametrize("alpha", ALPHAS)
def test_full_size_products_and_join(request, alpha):
    S = _full(request, alpha)
    _uniform_keys(S)
    E = _env(S)
    g = fc.load_golden(f"a{alpha}_products")
    price, mask, cp, cm = fc.select_inputs(E)
    sel = S.ctx.select(S.to_dev([cp]), S.to_dev([cm]))
    fc.check(g, "select", sel[0].cpu().numpy())
    _, ct = fc.extract_inputs(E)
    fc.check(g, "extract", S.ctx.extract(S.to_dev([ct]), fc.EXTRACT_SLOT)[0].cpu().numpy())
    fc.check(g, "broadcast",
             S.ctx.extract(S.to_dev([ct]), fc.EXTRACT_SLOT, broadcast=True)[0].cpu().numpy())
    gj = fc.load_golden(f"a{alpha}_join")
    *_, ca, cbk, cba = fc.join_inputs(E)
    out = S.ctx.join_sum(S.to_dev([ca]), S.to_dev([cbk]), S.to_dev([cba]), [fc.JOIN_SLOT])
    fc.check(gj, "join", out[0].cpu().numpy())


@pytest.mark.parametrize("alpha", ALPHAS)
def test_full_size_lt_between_t17(request, alpha):
    S = _full(request, alpha)
    E17 = _env(S).with_t(17)
    g = fc.load_golden(f"a{alpha}_lt_t17")
    ctx = Context(15, 17, list(S.pr.q), list(S.pr.special))
    ctx.set_relin_key(torch.from_numpy(S.rk.limbs(S.pr)).to(ctx.device))
    _, cts = fc.lt17_inputs(E17)
    dev = [S.to_dev([c]) for c in cts]
    fc.check(g, "lt", ctx.compare(dev[0], dev[1], "lt")[0].cpu().numpy())
    fc.check(g, "between", ctx.between(dev[0], dev[2], dev[3])[0].cpu().numpy())
    ctx.close()


@pytest.mark.parametrize("alpha", ALPHAS)
def test_full_size_autotune_keeps_the_two_kernel_key_switch(request, alpha):
    """The fused key switch exists for one-prime digits only: the autotuner
    must not report it (it would time a path the context never takes)."""
    S = _full(request, alpha)
    x = synth.uniform_device_residues((2, 2), S.ctx.q, S.ctx.n, 5, S.ctx.device)
    start = S.ctx.tuning()
    try:
        tuned = S.ctx.autotune(x, max_wave_ct=2)
        assert tuned["ks_fused"] == 0 and tuned["ms_per_ct"] > 0
    finally:
        S.ctx.set_tuning(**start)
