"""nshe_eq_mask_noalloc, the EQ entry point for callers that cannot allocate,
against nshe_eq_mask (the same computation with a caller workspace), both
through the C ABI: bit-exact on two calls in a row on one device, the
second with a smaller input; at N = 32768 the scratch's one ciphertext, and
the refusal of two before any work."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import bfv
from paper_2602_24271_amd import Context, _lib
from tests.gpu_common import Setup

pytestmark = pytest.mark.gpu


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _noalloc(ctx, x, y, n_ct, bcast):
    out = torch.full_like(x[:n_ct], -1)
    rc = ctx._lib.nshe_eq_mask_noalloc(ctx._h, x.data_ptr(), y.data_ptr(), out.data_ptr(), n_ct,
                                       bcast, _stream())
    _lib.check(rc)
    return out


def _with_workspace(ctx, x, y, n_ct, bcast):
    out = torch.full_like(x[:n_ct], -2)
    ws = torch.empty(ctx.workspace_bytes(n_ct), dtype=torch.uint8, device=ctx.device)
    rc = ctx._lib.nshe_eq_mask(ctx._h, x.data_ptr(), y.data_ptr(), out.data_ptr(), n_ct, bcast,
                               ws.data_ptr(), ws.numel(), _stream())
    _lib.check(rc)
    return out


def test_noalloc_two_calls_match_the_workspace_entry():
    """N = 4096 (eight ciphertexts fit the scratch): five ciphertexts column
    against column, then two against a broadcast one."""
    S = Setup(12, seed=21)
    n = S.pr.n
    x, y = synth.column_pair_half_match(21, 5 * n)
    dx = S.to_dev([S.enc(x[k * n:(k + 1) * n], 100 + k) for k in range(5)])
    dy = S.to_dev([S.enc(y[k * n:(k + 1) * n], 200 + k) for k in range(5)])
    a = _noalloc(S.ctx, dx, dy, 5, 0)
    b = _with_workspace(S.ctx, dx, dy, 5, 0)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    x2, y2 = dx[3:5].contiguous(), dy[:1].contiguous()
    c = _noalloc(S.ctx, x2, y2, 2, 1)
    d = _with_workspace(S.ctx, x2, y2, 2, 1)
    torch.cuda.synchronize()
    assert torch.equal(c, d)
    got = S.from_dev(c)
    for i, k in enumerate((3, 4)):
        assert list(bfv.decrypt_slots(S.pr, S.sk, got[i])) == \
            list((x[k * n:(k + 1) * n] == y[:n]).astype(int))
    with pytest.raises(_lib.NsheError) as e:
        _noalloc(S.ctx, torch.zeros((9, 2, S.pr.L, n), dtype=torch.int64, device=S.ctx.device),
                 dy, 9, 1)
    assert e.value.code == _lib.NSHE_ENOMEM


@pytest.mark.parametrize("alpha", [1, 3])
def test_noalloc_full_size_one_ciphertext(alpha):
    """N = 32768 with a stand-in (uniform) key and uniform residues (the
    arithmetic is the same for any key), one- and three-prime key-switching
    digits: one ciphertext, then an empty call; two ciphertexts are
    refused."""
    ctx = Context.paper(15, alpha=alpha)
    key = synth.uniform_device_residues((ctx.dnum, 2), ctx.moduli_pq, ctx.n, 31, ctx.device)
    ctx.set_relin_key(key)
    x = synth.uniform_device_residues((1, 2), ctx.q, ctx.n, 32, ctx.device)
    y = synth.uniform_device_residues((1, 2), ctx.q, ctx.n, 33, ctx.device)
    a = _noalloc(ctx, x, y, 1, 0)
    b = _with_workspace(ctx, x, y, 1, 0)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert int(a.min()) >= 0
    _noalloc(ctx, x, y, 0, 0)
    x2 = torch.cat([x, y]).contiguous()
    with pytest.raises(_lib.NsheError) as e:
        _noalloc(ctx, x2, x2, 2, 0)
    assert e.value.code == _lib.NSHE_ENOMEM and "scratch" in str(e.value)
    ctx.close()
