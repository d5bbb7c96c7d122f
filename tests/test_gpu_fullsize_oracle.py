"""Bit-exact parity at the paper's size (N = 32768, 17 + 1 primes, p = 65537;
Sec. 5.1) against the oracle's stored digests (tests/golden/fullsize_*.json,
written by tests/golden/make_fullsize.py from the oracle alone):

* the EQ chain (Eq. eq:equality): all 16 squaring levels through
  nshe_square_relin and the production nshe_eq_mask (fused chain) mask;
* a whole 2^20-row column (32 ciphertexts, the benchmark's launch shape):
  seed 0 column against column, seed 1 sorted dictionary ids against a
  broadcast constant;
* a rotation with a real Galois key, and the rotate-and-add COUNT/SUM
  (Sec. 4.2.2, aggregation; the mod-down that adds into the running sum)
  and Broadcast with stand-in (uniform) Galois keys;
* SELECT (Eq. eq:select), Extract (Sec. 2.1.6) and the fused JOIN
  (Sec. 4.2.2);
* LT and BETWEEN (Eq. eq:inequality) at t = 17 on directly encrypted
  plaintext polynomials (the summed giant-step tensor and the split
  inverse at 2^15), and at the paper's p = 65537 at N = 64 (256 babies,
  128 giants);
* the exact-lift fallback at every call site under the widened window.
"""
import numpy as np
import pytest
import torch

from oracle import bfv, encoding, galois
from paper_2602_24271_amd import Context
from tests import fullsize_cases as fc
from tests.gpu_common import Setup

pytestmark = pytest.mark.gpu


def _env(S):
    return fc.Env.from_keys(S.pr, S.sk, S.rk)


def _dev(S, cts):
    return S.to_dev(cts)


def test_eq_chain_every_level_and_mask(s32k):
    S = s32k
    E = _env(S)
    g = fc.load_golden("eq_edges")
    x, y, cx, cy = fc.eq_edges_inputs(E)
    dx, dy = _dev(S, [cx]), _dev(S, [cy])
    z = S.ctx.sub(dx, dy)
    fc.check(g, "level_00", z[0].cpu().numpy())
    for k in range(1, 17):
        z = S.ctx.square_relin(z)
        fc.check(g, f"level_{k:02d}", z[0].cpu().numpy())
    mask = S.ctx.eq_mask(dx, dy)
    fc.check(g, "mask", mask[0].cpu().numpy())
    got = S.from_dev(mask)[0]
    assert list(bfv.decrypt_slots(S.pr, S.sk, got)) == list((x == y).astype(int))


@pytest.mark.parametrize("fused", [0, 1])
def test_key_switch_paths_full_size(s32k, fused):
    """Both key-switch products at N = 32768 (digit transforms written and
    then multiplied by the key, or the two fused in one kernel), through a
    squaring level, the whole mask, a batched wave and a rotate-and-add:
    bit-exact against the oracle."""
    S = s32k
    E = _env(S)
    g = fc.load_golden("eq_edges")
    x, y, cx, cy = fc.eq_edges_inputs(E)
    dx, dy = _dev(S, [cx]), _dev(S, [cy])
    start = S.ctx.tuning()
    try:
        S.ctx.set_tuning(ks_fused=fused, split_forward=1)
        fc.check(g, "level_01", S.ctx.square_relin(S.ctx.sub(dx, dy))[0].cpu().numpy())
        fc.check(g, "mask", S.ctx.eq_mask(dx, dy)[0].cpu().numpy())
        outs = S.ctx.eq_mask_batched([(dx, dy)], wave_ct=1, use_graph=True)
        fc.check(g, "mask", outs[0][0].cpu().numpy())
    finally:
        S.ctx.set_tuning(**start)


def test_eq_column_uniform_2p20_rows(s32k):
    """configs[1] seed 0 in the benchmark's launch shape: 32 ciphertexts in
    one nshe_eq_mask call, every mask bit-exact."""
    S = s32k
    E = _env(S)
    g = fc.load_golden("eq_column_uniform")
    pairs = [fc.column_uniform_cts(E, k) for k in range(fc.COLUMN_CTS)]
    out = S.ctx.eq_mask(_dev(S, [p[0] for p in pairs]), _dev(S, [p[1] for p in pairs]))
    got = out.cpu().numpy()
    for k in range(fc.COLUMN_CTS):
        fc.check(g, f"mask_{k:02d}", got[k])
    x, y = fc.column_uniform_slots(E, 5)
    assert list(bfv.decrypt_slots(S.pr, S.sk, S.from_dev(out[5:6])[0])) == \
        list((x == y).astype(int))


def test_eq_column_structured_2p20_rows(s32k):
    """configs[1] seed 1: the sorted, skewed dictionary column against one
    encrypted id broadcast over 32 ciphertexts."""
    S = s32k
    E = _env(S)
    g = fc.load_golden("eq_column_structured")
    xs = _dev(S, [fc.column_structured_ct(E, k) for k in range(fc.COLUMN_CTS)])
    out = S.ctx.eq_mask(xs, _dev(S, [fc.column_structured_constant(E)]))
    got = out.cpu().numpy()
    for k in range(fc.COLUMN_CTS):
        fc.check(g, f"mask_{k:02d}", got[k])
    x, c = fc.column_structured_slots(E)
    hit = int(np.argmax(x == c)) // S.pr.n
    m = bfv.decrypt_slots(S.pr, S.sk, S.from_dev(out[hit:hit + 1])[0])
    assert list(m) == list((x[hit * S.pr.n:(hit + 1) * S.pr.n] == c).astype(int))


@pytest.fixture(scope="module")
def uniform_keys(s32k):
    """Stand-in Galois keys (uniform residues) for every element of the
    rotate-and-add sum, loaded into the device context."""
    S = s32k
    for gel, limbs in fc.uniform_galois_limbs(S.pr).items():
        S.ctx.set_galois_key(gel, torch.from_numpy(limbs).to(S.ctx.device))
    return True


def test_rotation_with_a_real_key(s32k):
    S = s32k
    E = _env(S)
    g = fc.load_golden("rotations")
    v, ct = fc.rotate_inputs(E)
    gel, key = fc.real_rotation(E)
    S.ctx.set_galois_key(gel, torch.from_numpy(key.limbs(S.pr)).to(S.ctx.device))
    out = S.ctx.rotate(_dev(S, [ct]), gel)
    fc.check(g, "rotate", out[0].cpu().numpy())
    got = bfv.decrypt_slots(S.pr, S.sk, S.from_dev(out)[0])
    h = S.pr.n // 2
    want = np.concatenate([np.roll(v[:h], -1), np.roll(v[h:], -1)])
    assert list(got) == list(want)


def test_sum_slots_full_size(s32k, uniform_keys):
    S = s32k
    E = _env(S)
    g = fc.load_golden("rotations")
    _, ct = fc.rotate_inputs(E)
    assert S.ctx.galois_elements() == galois.sum_elements(S.pr.n)
    start = S.ctx.tuning()
    try:
        for fused in (0, 1):
            S.ctx.set_tuning(ks_fused=fused)
            out = S.ctx.sum_slots(_dev(S, [ct]))
            fc.check(g, "sum_slots", out[0].cpu().numpy())
    finally:
        S.ctx.set_tuning(**start)


def test_select_extract_broadcast_full_size(s32k, uniform_keys):
    S = s32k
    E = _env(S)
    g = fc.load_golden("products")
    price, mask, cp, cm = fc.select_inputs(E)
    sel = S.ctx.select(_dev(S, [cp]), _dev(S, [cm]))
    fc.check(g, "select", sel[0].cpu().numpy())
    assert list(bfv.decrypt_slots(S.pr, S.sk, S.from_dev(sel)[0])) == \
        list((price * mask) % S.pr.t)
    v, ct = fc.extract_inputs(E)
    ex = S.ctx.extract(_dev(S, [ct]), fc.EXTRACT_SLOT)
    fc.check(g, "extract", ex[0].cpu().numpy())
    want = np.zeros(S.pr.n, dtype=np.int64)
    want[fc.EXTRACT_SLOT] = v[fc.EXTRACT_SLOT]
    assert list(bfv.decrypt_slots(S.pr, S.sk, S.from_dev(ex)[0])) == list(want)
    bc = S.ctx.extract(_dev(S, [ct]), fc.EXTRACT_SLOT, broadcast=True)
    fc.check(g, "broadcast", bc[0].cpu().numpy())


def test_join_full_size(s32k, uniform_keys):
    S = s32k
    E = _env(S)
    g = fc.load_golden("join")
    *_, ca, cbk, cba = fc.join_inputs(E)
    out = S.ctx.join_sum(_dev(S, [ca]), _dev(S, [cbk]), _dev(S, [cba]), [fc.JOIN_SLOT])
    fc.check(g, "join", out[0].cpu().numpy())


def test_lt_between_t17_full_size(s32k):
    """t = 17 (4 squarings, 4 babies, 2 giants) at N = 32768: the giant-step
    tensor sum and the split inverse of the comparison program."""
    S = s32k
    E17 = _env(S).with_t(17)
    g = fc.load_golden("lt_t17")
    ctx = Context(15, 17, list(S.pr.q), S.pr.P)
    ctx.set_relin_key(torch.from_numpy(S.rk.limbs(S.pr)).to(ctx.device))
    _, cts = fc.lt17_inputs(E17)
    dev = [S.to_dev([c]) for c in cts]
    lt = ctx.compare(dev[0], dev[1], "lt")
    fc.check(g, "lt", lt[0].cpu().numpy())
    bt = ctx.between(dev[0], dev[2], dev[3])
    fc.check(g, "between", bt[0].cpu().numpy())
    ctx.close()


def test_lt_le_between_paper_prime_n64():
    """p = 65537 at N = 64: the paper's comparison program shape (16
    squarings, 256 babies, 128 giants, 127 summed giant-step tensors)."""
    S = Setup(6)
    E = fc.Env.from_keys(S.pr, S.sk, S.rk)
    g = fc.load_golden("lt_n64")
    (x, y, lo, hi), cts = fc.lt_n64_inputs(E)
    dev = [S.to_dev([c]) for c in cts]
    lt = S.ctx.compare(dev[0], dev[1], "lt")
    fc.check(g, "lt", lt[0].cpu().numpy())
    assert list(bfv.decrypt_slots(S.pr, S.sk, S.from_dev(lt)[0])) == list((x < y).astype(int))
    le = S.ctx.compare(dev[0], dev[1], "le")
    fc.check(g, "le", le[0].cpu().numpy())
    bt = S.ctx.between(dev[0], dev[2], dev[3])
    fc.check(g, "between", bt[0].cpu().numpy())
    assert list(bfv.decrypt_slots(S.pr, S.sk, S.from_dev(bt)[0])) == \
        list(((lo <= x) & (x <= hi)).astype(int))


def _frac(count, coefficients):
    return count / coefficients


def test_wide_lift_window_every_site():
    """Under NSHE_DEBUG_WIDE_LIFT_WINDOW about half of all lifts take the
    exact mixed-radix path: results stay bit-exact and every call site
    counts its fallbacks.  N = 1024 (one workgroup per limb: k_lift,
    k_scale, k_i64_lift) against the oracle computed here."""
    S = Setup(10)
    x, y = fc.synth.column_pair_half_match(0, S.pr.n)
    cx, cy = S.enc(x, 1), S.enc(y, 2)
    S.ctx.set_debug(wide_lift_window=True)
    S.ctx.reset_margin_events()
    try:
        out = S.ctx.eq_mask(S.to_dev([cx]), S.to_dev([cy]))
        _, want = bfv.eq_chain(S.pr, S.rk, cx, cy)
        np.testing.assert_array_equal(out[0].cpu().numpy(), S.limbs(want))
        prod = S.ctx.mul_relin(S.to_dev([cx]), S.to_dev([cy]))
        np.testing.assert_array_equal(prod[0].cpu().numpy(),
                                      S.limbs(bfv.mul_relin(S.pr, S.rk, cx, cy)))
        sites = S.ctx.margin_sites()
    finally:
        S.ctx.set_debug()
    n = S.pr.n
    print("margin sites at N=1024:", sites)
    # 16 levels x 2 polys x N lifts; 16 x 3 polys x N scale lifts; 2 x 2 x N operand lifts
    assert _frac(sites[0], 16 * 2 * n) > 0.3
    assert _frac(sites[1], 16 * 3 * n) > 0.3
    assert _frac(sites[5], 4 * n) > 0.3


def test_wide_lift_window_every_site_full_size(s32k):
    """N = 32768 (split transforms: the fused chain's k_sub_lift,
    k_moddown_lift and the split k_scale, in the plain call and in a batched
    wave; k_i64_lift; without the split transforms, k_lift and k_scale in a
    batched wave): bit-exact against the stored oracle digests."""
    S = s32k
    E = _env(S)
    g = fc.load_golden("eq_edges")
    x, y, cx, cy = fc.eq_edges_inputs(E)
    dx, dy = _dev(S, [cx]), _dev(S, [cy])
    S.ctx.set_debug(wide_lift_window=True)
    S.ctx.reset_margin_events()
    try:
        mask = S.ctx.eq_mask(dx, dy)
        fc.check(g, "mask", mask[0].cpu().numpy())
        lvl1 = S.ctx.square_relin(S.ctx.sub(dx, dy))
        fc.check(g, "level_01", lvl1[0].cpu().numpy())
        outs = S.ctx.eq_mask_batched([(dx, dy)], wave_ct=1, use_graph=False)
        fc.check(g, "mask", outs[0][0].cpu().numpy())
        start = S.ctx.tuning()
        try:
            # unsplit transforms: every level lifts with k_lift, scales with
            # the unsplit k_scale
            S.ctx.set_tuning(split_forward=0)
            outs = S.ctx.eq_mask_batched([(dx, dy)], wave_ct=1, use_graph=False)
            fc.check(g, "mask", outs[0][0].cpu().numpy())
        finally:
            S.ctx.set_tuning(**start)
        sites = S.ctx.margin_sites()
    finally:
        S.ctx.set_debug()
    n = S.pr.n
    print("margin sites at N=32768:", sites)
    assert all(sites[i] > 0 for i in range(6)), sites
    assert _frac(sites[0], 2 * 16 * n) > 0.3          # the unsplit wave's lifts
    assert _frac(sites[1], 16 * 3 * n) > 0.3          # the unsplit wave's scale
    assert _frac(sites[2], 2 * 16 * 3 * n) > 0.3      # two chains' split scale
    assert _frac(sites[3], 2 * 15 * 2 * n) > 0.3      # two chains' fused mod-down + lift
    assert _frac(sites[4], 2 * 2 * n) > 0.3           # two fused chains' first lift
    assert _frac(sites[5], 2 * n) > 0.3               # square_relin's operand lift


def test_check_inputs_switch(s32k):
    """NSHE_DEBUG_CHECK_INPUTS: a residue outside [0, q_i) is refused before
    any work; valid inputs pass unchanged."""
    from paper_2602_24271_amd._lib import NsheError, NSHE_EINVAL
    S = s32k
    E = _env(S)
    _, _, cx, cy = fc.eq_edges_inputs(E)
    dx, dy = _dev(S, [cx]), _dev(S, [cy])
    S.ctx.set_debug(check_inputs=True)
    try:
        z = S.ctx.sub(dx, dy)
        fc.check(fc.load_golden("eq_edges"), "level_00", z[0].cpu().numpy())
        bad = dx.clone()
        bad[0, 1, 3, 77] = S.pr.q[3]
        with pytest.raises(NsheError) as e:
            S.ctx.square_relin(bad)
        assert e.value.code == NSHE_EINVAL
        bad[0, 1, 3, 77] = -1
        with pytest.raises(NsheError):
            S.ctx.eq_mask(bad, dy)
    finally:
        S.ctx.set_debug()
