"""Device parity of the batched EQ (uneven instances, waves, graph replay)."""
import numpy as np
import pytest
import torch

import synth
from oracle import bfv
from tests.gpu_common import Setup

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def s256():
    return Setup(8)


def _instances(S, sizes, seed):
    items, want = [], []
    for k, m in enumerate(sizes):
        x, _ = synth.column_pair_half_match(seed + k, m * S.pr.n)
        c = int(x[0])
        x[::3] = c                       # a third of the rows match the constant
        cxs = [S.enc(x[i * S.pr.n:(i + 1) * S.pr.n], seed * 1000 + k * 10 + i) for i in range(m)]
        cy = S.enc(np.full(S.pr.n, c), seed * 1000 + k * 10 + 9)
        items.append((S.to_dev(cxs), S.to_dev([cy])))
        want.append([bfv.eq_chain(S.pr, S.rk, cx, cy)[1] for cx in cxs])
    return items, want


@pytest.mark.parametrize("wave_ct,use_graph", [(0, False), (2, True), (4, True)])
def test_batched_matches_oracle(s256, wave_ct, use_graph):
    S = s256
    items, want = _instances(S, [1, 3, 2], 50)
    for rep in range(2):                 # second pass replays a cached graph
        outs = S.ctx.eq_mask_batched(items, wave_ct=wave_ct, use_graph=use_graph)
        torch.cuda.synchronize()
        for o, w in zip(outs, want):
            for i, ct in enumerate(w):
                np.testing.assert_array_equal(o[i].cpu().numpy(), S.limbs(ct))


def test_batched_two_streams(s256):
    """75 ciphertexts in uneven instances, waves of 32: with two streams the
    half-waves of 16 (the last of 11) alternate between the caller's stream
    and the context's second one.  Every mask equals the plain call's on one
    stream (graphs or not, the graphs replayed), and an encrypted pair's
    equals the oracle's."""
    S = s256
    rng = np.random.default_rng(31)
    x, y = rng.integers(0, S.pr.t, S.pr.n), rng.integers(0, S.pr.t, S.pr.n)
    x[::2] = y[::2]
    cx, cy = S.enc(x, 310), S.enc(y, 311)
    want = bfv.eq_chain(S.pr, S.rk, cx, cy)[1]
    items = []
    for k, m in enumerate([20, 1, 33, 21]):
        xs = synth.uniform_device_residues((m, 2), S.ctx.q, S.ctx.n, 200 + k, S.ctx.device)
        ys = synth.uniform_device_residues((1 if k % 2 else m, 2), S.ctx.q, S.ctx.n, 300 + k,
                                           S.ctx.device)
        if k == 2:
            xs[5] = S.to_dev([cx])[0]
            ys[5] = S.to_dev([cy])[0]
        items.append((xs, ys))
    start = S.ctx.tuning()
    try:
        S.ctx.set_tuning(streams=1)
        ref = [S.ctx.eq_mask(xs, ys) for xs, ys in items]
        S.ctx.set_tuning(streams=2)
        for use_graph in (True, False):
            for rep in range(2):
                outs = S.ctx.eq_mask_batched(items, wave_ct=32, use_graph=use_graph)
                torch.cuda.synchronize()
                for o, r in zip(outs, ref):
                    assert torch.equal(o, r)
    finally:
        S.ctx.set_tuning(**start)
    np.testing.assert_array_equal(ref[2][5].cpu().numpy(), S.limbs(want))


def test_tunings_do_not_change_results(s256):
    """Every launch shape gives the same integers (and the oracle's)."""
    S = s256
    items, want = _instances(S, [2, 1], 70)
    start = S.ctx.tuning()
    try:
        for ks, blk in [(4, 64), (8, 128), (32, 256)]:
            S.ctx.set_tuning(ks_chunk=ks, ew_block=blk)
            outs = S.ctx.eq_mask_batched(items, wave_ct=3, use_graph=True)
            torch.cuda.synchronize()
            for o, w in zip(outs, want):
                for i, ct in enumerate(w):
                    np.testing.assert_array_equal(o[i].cpu().numpy(), S.limbs(ct))
    finally:
        S.ctx.set_tuning(**start)


def test_set_tuning_rejects_bad_values(s256):
    from paper_2602_24271_amd._lib import NsheError
    for bad in [dict(ks_chunk=5), dict(ew_block=32), dict(split_forward=2), dict(wave_ct=-1),
                dict(ks_fused=2), dict(streams=0), dict(streams=3)]:
        with pytest.raises(NsheError):
            s256.ctx.set_tuning(**bad)


def test_autotune_then_batched(s256):
    """The autotuner picks valid shapes and a wave; the batched call that
    uses them (wave_ct = 0) still matches the oracle."""
    S = s256
    items, want = _instances(S, [3, 2, 1], 90)
    start = S.ctx.tuning()
    try:
        tuned = S.ctx.autotune(items[0][0], max_wave_ct=4)
        assert tuned["ks_chunk"] in (4, 8, 16, 32)
        assert tuned["ew_block"] in (64, 128, 256)
        assert 1 <= tuned["wave_ct"] <= 4
        assert tuned["ms_per_ct"] > 0
        assert {k: tuned[k] for k in start} == S.ctx.tuning()
        outs = S.ctx.eq_mask_batched(items, wave_ct=0, use_graph=True)
        torch.cuda.synchronize()
        for o, w in zip(outs, want):
            for i, ct in enumerate(w):
                np.testing.assert_array_equal(o[i].cpu().numpy(), S.limbs(ct))
    finally:
        S.ctx.set_tuning(**start)
