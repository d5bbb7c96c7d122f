"""Device parity of the range comparisons (Eq. eq:inequality; BETWEEN,
Sec. 4.2.2): LT, LE and BETWEEN bit-exact against the oracle's program at
t = 17 (every in-range pair) and t = 257 (edge differences), decrypting to
the plain comparisons."""
import numpy as np
import pytest
import torch

from oracle import bfv, compare
from tests.gpu_common import Setup

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def s17():
    return Setup(3, t=17, seed=8)


@pytest.fixture(scope="module")
def s257():
    return Setup(7, t=257, seed=9)


def test_lt_every_pair_in_range_t17(s17):
    S = s17
    pairs = [(a, b) for a in range(17) for b in range(17) if abs(a - b) <= 8]
    pairs += [(0, 0)] * (-len(pairs) % 8)
    xs = [[a for a, _ in pairs[8 * c: 8 * c + 8]] for c in range(len(pairs) // 8)]
    ys = [[b for _, b in pairs[8 * c: 8 * c + 8]] for c in range(len(pairs) // 8)]
    cx = [S.enc(x, 100 + i) for i, x in enumerate(xs)]
    cy = [S.enc(y, 200 + i) for i, y in enumerate(ys)]
    got = S.ctx.compare(S.to_dev(cx), S.to_dev(cy), "lt")
    torch.cuda.synchronize()
    for i in range(len(xs)):
        want = compare.lt(S.pr, S.rk, cx[i], cy[i])
        np.testing.assert_array_equal(got[i].cpu().numpy(), S.limbs(want))
        assert list(bfv.decrypt_slots(S.pr, S.sk, want)) == \
            [int(a < b) for a, b in zip(xs[i], ys[i])]


def test_le_and_between_t17(s17):
    S = s17
    rng = np.random.default_rng(5)
    x = [rng.integers(4, 13, 8) for _ in range(2)]
    y = [rng.integers(4, 13, 8) for _ in range(2)]
    cx = [S.enc(v, 300 + i) for i, v in enumerate(x)]
    cy = [S.enc(v, 310 + i) for i, v in enumerate(y)]
    got = S.ctx.compare(S.to_dev(cx), S.to_dev(cy), "le")
    for i in range(2):
        want = compare.le(S.pr, S.rk, cx[i], cy[i])
        np.testing.assert_array_equal(got[i].cpu().numpy(), S.limbs(want))
        assert list(bfv.decrypt_slots(S.pr, S.sk, want)) == list((x[i] <= y[i]).astype(int))
    xb = np.array([4, 5, 6, 7, 8, 9, 10, 11])
    clo, chi, cxb = S.enc(np.full(8, 6), 320), S.enc(np.full(8, 9), 321), S.enc(xb, 322)
    got = S.ctx.between(S.to_dev([cxb, cxb]), S.to_dev([clo]), S.to_dev([chi]))
    want = compare.between(S.pr, S.rk, cxb, clo, chi)
    for i in range(2):
        np.testing.assert_array_equal(got[i].cpu().numpy(), S.limbs(want))
    assert list(bfv.decrypt_slots(S.pr, S.sk, want)) == list(((xb >= 6) & (xb <= 9)).astype(int))


def test_lt_t257_edges_broadcast(s257):
    """t = 257, N = 128: a column against one encrypted constant (broadcast)
    with differences 0, +-1, +-127, +-128 present."""
    S = s257
    rng = np.random.default_rng(6)
    xs = [rng.integers(0, 257, S.pr.n) for _ in range(2)]
    xs[0][:7] = [128, 129, 127, 255, 1, 256, 0]
    cx = [S.enc(v, 400 + i) for i, v in enumerate(xs)]
    cy = S.enc(np.full(S.pr.n, 128), 410)
    got = S.ctx.compare(S.to_dev(cx), S.to_dev([cy]), "lt")
    torch.cuda.synchronize()
    for i in range(2):
        want = compare.lt(S.pr, S.rk, cx[i], cy)
        np.testing.assert_array_equal(got[i].cpu().numpy(), S.limbs(want))
        assert list(bfv.decrypt_slots(S.pr, S.sk, want)) == list((xs[i] < 128).astype(int))


def test_compare_rejects_non_fermat_t():
    """t = 97 (t - 1 not a power of two): no comparison polynomial; the
    workspace query returns 0 and the call NSHE_EUNSUPPORTED before touching
    any buffer."""
    S = Setup(4, t=97, seed=1)
    x = S.to_dev([S.enc(np.zeros(S.pr.n, dtype=np.int64), 1)])
    assert S.ctx._lib.nshe_compare_workspace_bytes(S.ctx._h, 1) == 0
    from paper_2602_24271_amd._lib import NsheError, NSHE_EUNSUPPORTED
    with pytest.raises(NsheError) as e:
        S.ctx.compare(x, x)
    assert e.value.code == NSHE_EUNSUPPORTED
    rc = S.ctx._lib.nshe_compare(S.ctx._h, x.data_ptr(), x.data_ptr(), 0, 0, x.data_ptr(), 1,
                                 None, 0, None)
    assert rc == -7
