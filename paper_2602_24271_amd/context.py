"""Python face of the library: torch tensors in, torch tensors out.

Every call marshals pointers, sizes and the current HIP stream into the C
ABI (libnshe.so); all arithmetic runs in the library's kernels.  Device
memory (ciphertexts, keys, workspace) comes from PyTorch's allocator.
"""
from __future__ import annotations

import ctypes
import weakref

import torch

from . import _lib


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class Context:
    """BFV context on one HIP device (NSHEDB Sec. 5.1 parameters by default)."""

    def __init__(self, log2_n: int, t: int, q, P, device: int = 0):
        """P: the special prime, or a sequence of alpha special primes (key
        switching with digits of alpha data primes, alpha = 1, 2 or 3)."""
        lib = _lib.load()
        self.device = torch.device("cuda", device)
        special = [int(P)] if isinstance(P, int) else [int(x) for x in P]
        if len(special) not in (1, 2, 3):
            raise ValueError("one, two or three special primes")
        sp = special + [0] * (3 - len(special))
        qa = (ctypes.c_uint64 * len(q))(*q)
        pr = _lib.NsheParams(log2_n, t, len(q), ctypes.cast(qa, ctypes.POINTER(ctypes.c_uint64)),
                             sp[0], len(special), sp[1], sp[2])
        h = ctypes.c_void_p()
        _lib.check(lib.nshe_ctx_create(ctypes.byref(pr), device, ctypes.byref(h)))
        self._h = h
        self._lib = lib
        info = _lib.NsheInfo()
        _lib.check(lib.nshe_ctx_info(h, ctypes.byref(info)))
        self.n = info.n
        self.L = info.L
        self.L_ext = info.L_ext
        self.squarings = info.squarings
        self.ext_primes = [info.ext_primes[i] for i in range(info.L_ext)]
        self.depth_budget = info.depth_budget
        self.lt_depth = info.lt_depth
        self.fresh_bits = info.fresh_bits
        self.level_bits = info.level_bits
        self.alpha = info.alpha
        self.dnum = info.dnum
        # per-ciphertext-array level counter (Sec. 2.1.2): the depth of every
        # output this context produced, by tensor identity (an entry leaves
        # with its tensor); arrays it did not produce count as fresh
        # (depth 0) unless set_depth says otherwise
        self._depths = {}
        self.q = list(q)
        self.special = special
        self.P = special[0]
        self.moduli_pq = self.q + special
        self.t = t
        self._ws = None
        self._key = None

    @classmethod
    def paper(cls, log2_n: int = 15, device: int = 0, alpha: int = 1) -> "Context":
        """The paper's parameters (Sec. 5.1); alpha = 2 or 3 takes the two or
        three largest of the 18 primes as special primes (16 or 15 data
        primes)."""
        from .params import paper_params
        p = paper_params(log2_n, alpha=alpha)
        return cls(p["log2_n"], p["t"], p["q"], p["P"], device)

    @property
    def key_shape(self):
        """Shape of a relinearization or Galois key: [dnum, 2, L + alpha, N]."""
        return (self.dnum, 2, self.L + self.alpha, self.n)

    def close(self):
        if self._h:
            self._lib.nshe_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ helpers
    def ct_shape(self, n_ct: int):
        return (n_ct, 2, self.L, self.n)

    def workspace_bytes(self, n_ct: int) -> int:
        return int(self._lib.nshe_workspace_bytes(self._h, n_ct))

    def workspace(self, n_ct: int) -> torch.Tensor:
        return self._workspace_bytes(self.workspace_bytes(n_ct))

    def _workspace_bytes(self, need: int) -> torch.Tensor:
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def _check_ct(self, x: torch.Tensor, comps: int = 2) -> int:
        if x.dtype != torch.int64 or x.device != self.device or not x.is_contiguous():
            raise ValueError("ciphertexts must be contiguous int64 tensors on the context device")
        if x.dim() != 4 or x.shape[1] != comps or x.shape[2] != self.L or x.shape[3] != self.n:
            raise ValueError(f"expected shape [n_ct, {comps}, {self.L}, {self.n}], got {tuple(x.shape)}")
        return x.shape[0]

    # ------------------------------------------------------------ depth
    def depth(self, x: torch.Tensor) -> int:
        """Multiplicative depth of a ciphertext array (0 if unknown)."""
        return self._depths.get(id(x), 0)

    def set_depth(self, x: torch.Tensor, depth: int) -> None:
        k = id(x)
        if k not in self._depths:
            weakref.finalize(x, self._depths.pop, k, None)
        self._depths[k] = int(depth)

    def op_depth(self, op: str, arg: int = 0) -> int:
        d = ctypes.c_int()
        _lib.check(self._lib.nshe_op_depth(self._h, _lib.OPS[op], arg, ctypes.byref(d)))
        return d.value

    def _depth_after(self, op: str, *inputs, arg: int = 0) -> int:
        """Depth of an operation's result from its inputs' (raises NsheError
        NSHE_EDEPTH beyond the budget, before anything is enqueued)."""
        d = ctypes.c_int()
        din = max([self.depth(x) for x in inputs] + [0])
        _lib.check(self._lib.nshe_depth_after(self._h, _lib.OPS[op], arg, din, ctypes.byref(d)))
        return d.value

    def _tag(self, out: torch.Tensor, depth: int) -> torch.Tensor:
        self.set_depth(out, depth)
        return out

    # ------------------------------------------------------------ debug
    def set_debug(self, wide_lift_window: bool = False, check_inputs: bool = False) -> None:
        flags = (_lib.NSHE_DEBUG_WIDE_LIFT_WINDOW if wide_lift_window else 0) | \
                (_lib.NSHE_DEBUG_CHECK_INPUTS if check_inputs else 0)
        _lib.check(self._lib.nshe_set_debug(self._h, flags))

    def margin_sites(self) -> list:
        """Exact-lift fallbacks taken per call site (see nshe_margin_sites)."""
        buf = (ctypes.c_uint64 * _lib.NSHE_MARGIN_SITES)()
        n = ctypes.c_int()
        _lib.check(self._lib.nshe_margin_sites(self._h, buf, _lib.NSHE_MARGIN_SITES,
                                               ctypes.byref(n), _stream()))
        return [int(buf[i]) for i in range(n.value)]

    # ---------------------------------------------------------------- API
    def set_relin_key(self, evk: torch.Tensor) -> None:
        want = self.key_shape
        if evk.dtype != torch.int64 or tuple(evk.shape) != want or evk.device != self.device:
            raise ValueError(f"relin key must be int64 {want} on the context device")
        evk = evk.contiguous()
        _lib.check(self._lib.nshe_set_relin_key(self._h, _ptr(evk), evk.numel(), _stream()))
        self._key = evk  # keep alive until the stream has consumed it
        torch.cuda.current_stream().synchronize()
        self._key = None

    def sub(self, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
        n = self._check_ct(x)
        if self._check_ct(y) != n:
            raise ValueError("x and y must hold the same number of ciphertexts")
        d = self._depth_after("add", x, y)
        out = torch.empty_like(x)
        _lib.check(self._lib.nshe_sub(self._h, _ptr(x), _ptr(y), _ptr(out), n, _stream()))
        return self._tag(out, d)

    def add(self, a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
        n = self._check_ct(a)
        if self._check_ct(b) != n:
            raise ValueError("a and b must hold the same number of ciphertexts")
        d = self._depth_after("add", a, b)
        out = torch.empty_like(a)
        _lib.check(self._lib.nshe_add(self._h, _ptr(a), _ptr(b), _ptr(out), n, _stream()))
        return self._tag(out, d)

    def sum(self, cts: torch.Tensor) -> torch.Tensor:
        """cts: int64 [k][n_ct][2][L][N] -> their sum [n_ct][2][L][N]."""
        if cts.dim() != 5 or not cts.is_contiguous() or cts.dtype != torch.int64:
            raise ValueError("expected a contiguous int64 [k][n_ct][2][L][N] tensor")
        k = int(cts.shape[0])
        n = int(cts.shape[1])
        d = self._depth_after("add", cts)
        out = torch.empty(self.ct_shape(n), dtype=torch.int64, device=cts.device)
        _lib.check(self._lib.nshe_sum(self._h, _ptr(cts), k, _ptr(out), n, _stream()))
        return self._tag(out, d)

    def in_mask(self, x: torch.Tensor, members: torch.Tensor, wave_ct: int = 0,
                use_graph: bool = True) -> torch.Tensor:
        """IN(x, S) (Eq. eq:in); members: k single ciphertexts [k][2][L][N]."""
        n = self._check_ct(x)
        k = self._check_ct(members)
        d = self._depth_after("in", x, members, arg=k)
        out = torch.empty_like(x)
        need = int(self._lib.nshe_in_workspace_bytes(self._h, n, k, wave_ct))
        ws = self._workspace_bytes(need)
        _lib.check(self._lib.nshe_in_mask(self._h, _ptr(x), _ptr(members), k, _ptr(out), n,
                                          wave_ct, 1 if use_graph else 0, _ptr(ws), ws.numel(),
                                          _stream()))
        return self._tag(out, d)

    def group_masks(self, x: torch.Tensor, values: torch.Tensor, wave_ct: int = 0,
                    use_graph: bool = True) -> list:
        """GROUP BY: EQ(x, v) for each of the k encrypted group values
        (values: [k][2][L][N]), as one batched call."""
        self._check_ct(values)
        items = [(x, values[j:j + 1]) for j in range(values.shape[0])]
        return self.eq_mask_batched(items, wave_ct=wave_ct, use_graph=use_graph)

    def select(self, column: torch.Tensor, mask: torch.Tensor) -> torch.Tensor:
        """SELECT column WHERE mask (Eq. eq:select): column * mask, relinearized."""
        return self.mul_relin(column, mask)

    def _cmp_ws(self, n: int) -> torch.Tensor:
        need = int(self._lib.nshe_compare_workspace_bytes(self._h, n))
        if need == 0:
            raise ValueError("comparisons need t = 2^K + 1 prime")
        return self._workspace_bytes(need)

    def compare(self, x: torch.Tensor, y: torch.Tensor, op: str = "lt") -> torch.Tensor:
        """[x < y] (op "lt") or [x <= y] (op "le") for |x - y| <= (t-1)/2
        (Eq. eq:inequality); y: as many ciphertexts as x, or one (broadcast)."""
        n = self._check_ct(x)
        ny = self._check_ct(y)
        if ny not in (n, 1):
            raise ValueError("y must hold n_ct ciphertexts or one")
        code = {"lt": 0, "le": 1}[op]
        d = self._depth_after("lt", x, y)
        out = torch.empty_like(x)
        ws = self._cmp_ws(n)
        _lib.check(self._lib.nshe_compare(self._h, _ptr(x), _ptr(y), int(ny == 1 and n != 1),
                                          code, _ptr(out), n, _ptr(ws), ws.numel(), _stream()))
        return self._tag(out, d)

    def between(self, x: torch.Tensor, lo: torch.Tensor, hi: torch.Tensor) -> torch.Tensor:
        """[lo <= x <= hi] = LE(lo, x) * LE(x, hi); lo, hi: as many ciphertexts
        as x, or one each (broadcast)."""
        n = self._check_ct(x)
        nl, nh = self._check_ct(lo), self._check_ct(hi)
        if nl != nh or nl not in (n, 1):
            raise ValueError("lo and hi must both hold n_ct ciphertexts or one")
        d = self._depth_after("between", x, lo, hi)
        out = torch.empty_like(x)
        ws = self._cmp_ws(n)
        _lib.check(self._lib.nshe_between(self._h, _ptr(x), _ptr(lo), _ptr(hi),
                                          int(nl == 1 and n != 1), _ptr(out), n, _ptr(ws),
                                          ws.numel(), _stream()))
        return self._tag(out, d)

    def mul_plain(self, x: torch.Tensor, pt: torch.Tensor) -> torch.Tensor:
        """x times the plaintext polynomial pt (int64 [N], values in [0, t))."""
        n = self._check_ct(x)
        if pt.dtype != torch.int64 or pt.device != self.device or tuple(pt.shape) != (self.n,):
            raise ValueError("pt must be an int64 [N] tensor on the context device")
        d = self._depth_after("mul_plain", x)
        out = torch.empty_like(x)
        ws = self.workspace(n)
        _lib.check(self._lib.nshe_mul_plain(self._h, _ptr(x), _ptr(pt.contiguous()), _ptr(out), n,
                                            _ptr(ws), ws.numel(), _stream()))
        return self._tag(out, d)

    def extract(self, x: torch.Tensor, slot: int, broadcast: bool = False) -> torch.Tensor:
        """Extract one slot (others zero), or Broadcast it to every slot."""
        n = self._check_ct(x)
        d = self._depth_after("mul_plain", x)
        out = torch.empty_like(x)
        ws = self.workspace(n)
        _lib.check(self._lib.nshe_extract(self._h, _ptr(x), slot, int(bool(broadcast)), _ptr(out),
                                          n, _ptr(ws), ws.numel(), _stream()))
        return self._tag(out, d)

    def join_sum(self, a_key: torch.Tensor, b_key: torch.Tensor, b_attr: torch.Tensor,
                 rows) -> torch.Tensor:
        """Fused equi-join aggregation over the reference rows `rows`."""
        n = self._check_ct(a_key)
        if self._check_ct(b_key) != 1 or self._check_ct(b_attr) != 1:
            raise ValueError("b_key and b_attr must be one ciphertext each")
        rows = list(rows)
        d = self._depth_after("join", a_key, b_key, b_attr)
        arr = (ctypes.c_int32 * max(1, len(rows)))(*rows)
        out = torch.empty_like(a_key)
        ws = self._workspace_bytes(int(self._lib.nshe_join_workspace_bytes(self._h, n)))
        _lib.check(self._lib.nshe_join_sum(self._h, _ptr(a_key), _ptr(b_key), _ptr(b_attr), arr,
                                           len(rows), _ptr(out), n, _ptr(ws), ws.numel(),
                                           _stream()))
        return self._tag(out, d)

    def galois_elements(self) -> list:
        """Galois elements whose keys nshe_sum_slots needs, in order of use."""
        n = ctypes.c_int(0)
        buf = (ctypes.c_uint32 * 64)()
        _lib.check(self._lib.nshe_galois_elements(self._h, buf, 64, ctypes.byref(n)))
        return [int(buf[i]) for i in range(n.value)]

    def set_galois_key(self, g: int, key: torch.Tensor) -> None:
        if key.dtype != torch.int64 or not key.is_contiguous() or key.device != self.device:
            raise ValueError("key must be a contiguous int64 tensor on the context device")
        if tuple(key.shape) != self.key_shape:
            raise ValueError("key must have shape [dnum, 2, L+alpha, N]")
        _lib.check(self._lib.nshe_set_galois_key(self._h, g, _ptr(key), key.numel(), _stream()))

    def rotate(self, x: torch.Tensor, g: int) -> torch.Tensor:
        n = self._check_ct(x)
        d = self._depth_after("add", x)
        out = torch.empty_like(x)
        ws = self.workspace(n)
        _lib.check(self._lib.nshe_rotate(self._h, _ptr(x), g, _ptr(out), n, _ptr(ws), ws.numel(),
                                         _stream()))
        return self._tag(out, d)

    def sum_slots(self, x: torch.Tensor) -> torch.Tensor:
        """COUNT / SUM aggregation: every slot of the result holds the sum of
        all slots of its ciphertext."""
        n = self._check_ct(x)
        d = self._depth_after("add", x)
        out = torch.empty_like(x)
        ws = self.workspace(n)
        _lib.check(self._lib.nshe_sum_slots(self._h, _ptr(x), _ptr(out), n, _ptr(ws), ws.numel(),
                                            _stream()))
        return self._tag(out, d)

    def square_relin(self, x: torch.Tensor) -> torch.Tensor:
        n = self._check_ct(x)
        d = self._depth_after("mul", x)
        out = torch.empty_like(x)
        ws = self.workspace(n)
        _lib.check(self._lib.nshe_square_relin(self._h, _ptr(x), _ptr(out), n, _ptr(ws),
                                               ws.numel(), _stream()))
        return self._tag(out, d)

    def mul_relin(self, a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
        n = self._check_ct(a)
        if self._check_ct(b) != n:
            raise ValueError("a and b must hold the same number of ciphertexts")
        d = self._depth_after("mul", a, b)
        out = torch.empty_like(a)
        ws = self.workspace(n)
        _lib.check(self._lib.nshe_mul_relin(self._h, _ptr(a), _ptr(b), _ptr(out), n, _ptr(ws),
                                            ws.numel(), _stream()))
        return self._tag(out, d)

    def multiply(self, a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
        n = self._check_ct(a)
        if self._check_ct(b) != n:
            raise ValueError("a and b must hold the same number of ciphertexts")
        d = self._depth_after("mul", a, b)
        out = torch.empty((n, 3, self.L, self.n), dtype=torch.int64, device=self.device)
        ws = self.workspace(n)
        _lib.check(self._lib.nshe_multiply(self._h, _ptr(a), _ptr(b), _ptr(out), n, _ptr(ws),
                                           ws.numel(), _stream()))
        return self._tag(out, d)

    def relinearize(self, c3: torch.Tensor) -> torch.Tensor:
        n = self._check_ct(c3, comps=3)
        d = self._depth_after("add", c3)
        out = torch.empty((n, 2, self.L, self.n), dtype=torch.int64, device=self.device)
        ws = self.workspace(n)
        _lib.check(self._lib.nshe_relinearize(self._h, _ptr(c3), _ptr(out), n, _ptr(ws),
                                              ws.numel(), _stream()))
        return self._tag(out, d)

    def eq_mask(self, x: torch.Tensor, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """EQ(x, y) = 1 - (x - y)^(t-1) (Eq. eq:equality).  y holds as many
        ciphertexts as x, or one ciphertext broadcast to all of them."""
        n = self._check_ct(x)
        ny = self._check_ct(y)
        if ny not in (n, 1):
            raise ValueError("y must hold n_ct ciphertexts or one")
        bcast = 1 if (ny == 1 and n != 1) else 0
        d = self._depth_after("eq", x, y)
        if out is None:
            out = torch.empty_like(x)
        ws = self.workspace(n)
        _lib.check(self._lib.nshe_eq_mask(self._h, _ptr(x), _ptr(y), _ptr(out), n, bcast, _ptr(ws),
                                          ws.numel(), _stream()))
        return self._tag(out, d)

    def eq_mask_batched(self, items, wave_ct: int = 0, use_graph: bool = True, outs=None):
        """items: list of (x, y) with y one ciphertext (broadcast) or as many
        as x.  Returns the list of outputs."""
        arr = (_lib.NsheItem * len(items))()
        res = []
        depths = [self._depth_after("eq", x, y) for x, y in items]
        for i, (x, y) in enumerate(items):
            n = self._check_ct(x)
            ny = self._check_ct(y)
            if ny not in (n, 1):
                raise ValueError("y must hold n_ct ciphertexts or one")
            out = outs[i] if outs is not None else torch.empty_like(x)
            self._tag(out, depths[i])
            res.append(out)
            arr[i] = _lib.NsheItem(_ptr(x), _ptr(y), _ptr(out), n, 1 if (ny == 1 and n != 1) else 0)
        total = sum(int(x.shape[0]) for x, _ in items)
        wave = wave_ct if wave_ct > 0 else (self.tuning()["wave_ct"] or self.DEFAULT_WAVE)
        wave = min(wave, total)
        need = int(self._lib.nshe_batched_workspace_bytes(self._h, wave, total))
        ws = self._workspace_bytes(need)
        _lib.check(self._lib.nshe_eq_mask_batched(self._h, arr, len(items), wave,
                                                  1 if use_graph else 0, _ptr(ws), ws.numel(),
                                                  _stream()))
        return res

    TUNING_FIELDS = tuple(f for f, _ in _lib.NsheTuning._fields_)
    DEFAULT_WAVE = 32  # batched wave when neither the call nor the tuning sets one

    def tuning(self) -> dict:
        t = _lib.NsheTuning()
        _lib.check(self._lib.nshe_get_tuning(self._h, ctypes.byref(t)))
        return {f: int(getattr(t, f)) for f in self.TUNING_FIELDS}

    def set_tuning(self, **kw) -> None:
        cur = self.tuning()
        unknown = set(kw) - set(cur)
        if unknown:
            raise ValueError(f"unknown tuning fields {sorted(unknown)}")
        cur.update(kw)
        t = _lib.NsheTuning(**cur)
        _lib.check(self._lib.nshe_set_tuning(self._h, ctypes.byref(t)))

    def autotune(self, sample: torch.Tensor, max_wave_ct: int) -> dict:
        """Measure and set the launch shapes and batched wave size (see
        nshe_autotune) on `sample` ciphertexts, with a workspace for
        max_wave_ct ciphertexts.  Returns the tuning plus the best
        per-ciphertext level time ("ms_per_ct")."""
        n = self._check_ct(sample)
        if max_wave_ct < 1:
            raise ValueError("max_wave_ct must be >= 1")
        ws = self.workspace(max_wave_ct)
        t = _lib.NsheTuning()
        ms = ctypes.c_double(0.0)
        _lib.check(self._lib.nshe_autotune(self._h, _ptr(sample), n, max_wave_ct, _ptr(ws),
                                           ws.numel(), _stream(), ctypes.byref(t),
                                           ctypes.byref(ms)))
        out = {f: int(getattr(t, f)) for f in self.TUNING_FIELDS}
        out["ms_per_ct"] = ms.value
        return out

    def ntt(self, polys: torch.Tensor) -> torch.Tensor:
        """Forward negacyclic NTT of [n_poly, L, N] int64 limbs: evaluations
        at psi_i^(2j+1) in natural j order."""
        if polys.dim() != 3 or polys.shape[1] != self.L or polys.shape[2] != self.n:
            raise ValueError("polys must be [n_poly, L, N]")
        polys = polys.contiguous()
        n = polys.shape[0]
        out = torch.empty_like(polys)
        ws = torch.empty(2 * n * self.L * self.n * 8, dtype=torch.uint8, device=self.device)
        _lib.check(self._lib.nshe_ntt(self._h, _ptr(polys), _ptr(out), n, 0, _ptr(ws), ws.numel(),
                                      _stream()))
        return out

    def profile(self, enable: bool) -> None:
        _lib.check(self._lib.nshe_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        arr = (_lib.NsheKernelStat * 16)()
        n = ctypes.c_int()
        _lib.check(self._lib.nshe_profile_read(self._h, arr, 16, ctypes.byref(n)))
        return {arr[i].name.decode(): {"launches": arr[i].launches, "ms": arr[i].total_ms,
                                        "work": arr[i].work} for i in range(n.value)}

    def margin_events(self) -> int:
        v = ctypes.c_uint64()
        _lib.check(self._lib.nshe_margin_events(self._h, ctypes.byref(v), _stream()))
        return v.value

    def reset_margin_events(self) -> None:
        _lib.check(self._lib.nshe_reset_margin_events(self._h, _stream()))
