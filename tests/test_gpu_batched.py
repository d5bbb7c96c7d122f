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
