"""Seeded inputs and oracle evaluations of the parity cases at the paper's
size (N = 32768 slots, the 17 + 1 primes of about 49 bits, p = 65537;
Sec. 5.1), plus two cases at other (N, t) that reach the same kernels, and
the same cases with key switching by digits of two data primes (16 data
primes, two special primes: the a2_ cases) and of three (15 data primes,
three special primes: the a3_ cases).

The oracle needs minutes per case at this size, so its results are kept as
SHA-256 digests of the exchange-format arrays (int64 residues, C order,
little-endian) in tests/golden/fullsize_<case>.json, written by
tests/golden/make_fullsize.py, which runs only the oracle on the inputs
built here.  The GPU tests build the same inputs here, run the library and
compare digests of its outputs (with sampled coefficients to show where a
mismatch lies).  Every input comes from the seeded generators of synth.py.

A case is a list of units; a unit is (name, function of an Env returning
{label: int64 array}), so the writer can spread units over processes.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

import synth
from oracle import bfv, compare, encoding, galois, join, query

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
KEY_SEED = 0                 # the relinearization key of every case (as Setup)
COLUMN_CTS = 32              # 2^20 rows of 32768 slots: the benchmark's column
UNIFORM_KEY_SEED = 900       # stand-in Galois keys: seeds 900 + i, i-th sum element
JOIN_SLOT = 12345
EXTRACT_SLOT = 20000


# ------------------------------------------------------------ digests ---

def digest(arr) -> str:
    a = np.ascontiguousarray(np.asarray(arr), dtype="<i8")
    return hashlib.sha256(a.tobytes()).hexdigest()


def sample_positions(shape, k: int = 24, seed: int = 1) -> list:
    rng = np.random.default_rng(seed)
    idx = [tuple(int(rng.integers(0, d)) for d in shape) for _ in range(k)]
    return [tuple(0 for _ in shape)] + idx


def record(arr) -> dict:
    a = np.asarray(arr)
    pos = sample_positions(a.shape)
    return {"sha256": digest(a), "shape": list(a.shape),
            "sample": [[list(p), int(a[p])] for p in pos]}


def load_golden(case: str) -> dict:
    with open(os.path.join(GOLDEN_DIR, f"fullsize_{case}.json")) as f:
        return json.load(f)


def check(golden: dict, label: str, arr) -> None:
    """Assert that arr (int64, exchange format) is the oracle's output
    `label` of the golden record, naming differing sampled coefficients."""
    want = golden["outputs"][label]
    a = np.asarray(arr)
    assert list(a.shape) == want["shape"], f"{label}: shape {a.shape} != {want['shape']}"
    if digest(a) == want["sha256"]:
        return
    bad = [(p, int(a[tuple(p)]), v) for p, v in want["sample"] if int(a[tuple(p)]) != v]
    raise AssertionError(f"{golden['case']}/{label}: output differs from the oracle's; "
                         f"{len(bad)} of {len(want['sample'])} sampled coefficients differ "
                         f"(position, got, want): {bad[:6]}")


# -------------------------------------------------------------- setup ---

class Env:
    """Oracle parameters, secret key and relinearization key (keys from
    KEY_SEED, as the GPU tests' Setup draws them); alpha special primes."""

    def __init__(self, log2_n: int = 15, t: int = 65537, alpha: int = 1):
        n = 1 << log2_n
        self.pr = bfv.paper_params(n, t, alpha)
        self.sk, self.rk = bfv.keygen(self.pr, synth.key_randomness(
            KEY_SEED, n, self.pr.moduli_pq, self.pr.dnum))

    def enc(self, slots, seed):
        return bfv.encrypt_slots(self.pr, self.sk, slots,
                                 synth.enc_randomness(seed, self.pr.n, self.pr.q))

    def enc_poly(self, m, seed):
        return bfv.encrypt(self.pr, self.sk, m, synth.enc_randomness(seed, self.pr.n, self.pr.q))

    def limbs(self, ct) -> np.ndarray:
        return np.stack([bfv.to_limbs(c, self.pr.q) for c in ct])

    @classmethod
    def from_keys(cls, pr, sk, rk) -> "Env":
        """An Env over keys already drawn (the GPU tests' Setup)."""
        e = object.__new__(cls)
        e.pr, e.sk, e.rk = pr, sk, rk
        return e

    def with_t(self, t: int) -> "Env":
        """The same keys under another plaintext modulus (the keys do not
        depend on t)."""
        e = object.__new__(Env)
        e.pr = bfv.Params(self.pr.n, t, self.pr.q, self.pr.special)
        e.sk, e.rk = self.sk, self.rk
        return e


def uniform_galois_limbs(pr) -> dict:
    """Stand-in switching keys (uniform residues) for every element of the
    rotate-and-add sum, in the exchange format."""
    return {g: synth.uniform_switch_key(UNIFORM_KEY_SEED + i, pr.n, pr.moduli_pq, pr.dnum)
            for i, g in enumerate(galois.sum_elements(pr.n))}


def oracle_key(pr, limbs) -> bfv.RelinKey:
    m = pr.moduli_pq
    return bfv.RelinKey([bfv.from_limbs(limbs[j, 0], m) for j in range(pr.dnum)],
                        [bfv.from_limbs(limbs[j, 1], m) for j in range(pr.dnum)])


_UNIFORM_KEYS = {}


def uniform_galois_keys(pr) -> dict:
    k = (pr.n, pr.alpha)
    if k not in _UNIFORM_KEYS:
        _UNIFORM_KEYS[k] = {g: oracle_key(pr, x) for g, x in uniform_galois_limbs(pr).items()}
    return _UNIFORM_KEYS[k]


# ------------------------------------------------------------- inputs ---

def eq_edges_inputs(E: Env):
    """One ciphertext pair: seed-0 half-matching 16-bit values with the
    edge differences 0, +-1, 3, (p-1)/2 in the first slots."""
    x, y = synth.column_pair_half_match(0, E.pr.n)
    x, y = synth.edge_differences(x, y, E.pr.t)
    return x, y, E.enc(x, 1), E.enc(y, 2)


def column_uniform_slots(E: Env, k: int):
    """Ciphertext k of a 2^20-row column pair: seed 0, x uniform 16-bit and
    y = x on a seeded half of the rows (column against column)."""
    x, y = synth.column_pair_half_match(0, COLUMN_CTS * E.pr.n)
    s = slice(k * E.pr.n, (k + 1) * E.pr.n)
    return x[s], y[s]


def column_uniform_cts(E: Env, k: int):
    x, y = column_uniform_slots(E, k)
    return E.enc(x, 1000 + k), E.enc(y, 2000 + k)


def column_structured_slots(E: Env):
    """The 2^20-row structured column of seed 1: sorted dictionary ids with
    skewed frequencies, against one id of the dictionary."""
    x, y = synth.column_structured(1, COLUMN_CTS * E.pr.n)
    return x, int(y[0])


def column_structured_ct(E: Env, k: int):
    x, _ = column_structured_slots(E)
    return E.enc(x[k * E.pr.n:(k + 1) * E.pr.n], 3000 + k)


def column_structured_constant(E: Env):
    _, c = column_structured_slots(E)
    return E.enc(np.full(E.pr.n, c), 3999)


def rotate_inputs(E: Env):
    v = np.random.default_rng(40).integers(0, E.pr.t, E.pr.n)
    return v, E.enc(v, 40)


def real_rotation(E: Env):
    """Galois element of a rotation by one slot and its (real) key."""
    g = galois.rotation_element(E.pr.n, 1)
    key = galois.galois_key(E.pr, E.sk, g, synth.switch_randomness(500, E.pr.n,
                                                                     E.pr.moduli_pq, E.pr.dnum))
    return g, key


def select_inputs(E: Env):
    rng = np.random.default_rng(50)
    price = rng.integers(0, 40000, E.pr.n)
    mask = (rng.random(E.pr.n) < 0.3).astype(np.int64)
    return price, mask, E.enc(price, 50), E.enc(mask, 51)


def extract_inputs(E: Env):
    v = np.random.default_rng(52).integers(0, E.pr.t, E.pr.n)
    return v, E.enc(v, 52)


def join_inputs(E: Env):
    rng = np.random.default_rng(53)
    b_key = rng.permutation(np.arange(1, E.pr.n + 1))
    b_attr = rng.integers(1, 40000, E.pr.n)
    a_key = rng.choice(np.concatenate([b_key[JOIN_SLOT - 2:JOIN_SLOT + 2], [0]]), E.pr.n)
    return a_key, b_key, b_attr, E.enc(a_key, 54), E.enc(b_key, 55), E.enc(b_attr, 56)


def lt17_inputs(E17: Env):
    """Plaintext polynomials mod 17 encrypted directly (t = 17 has no slots
    at N = 32768; the arithmetic is the same)."""
    n = E17.pr.n
    ms = [synth.plain_poly(60 + i, n, 17) for i in range(4)]
    return ms, [E17.enc_poly(m, 60 + i) for i, m in enumerate(ms)]


def lt_n64_inputs(E: Env):
    """Slots of 15-bit values (so |x - y| <= (p-1)/2), edge differences in
    the first slots."""
    rng = np.random.default_rng(70)
    x = rng.integers(0, 1 << 15, E.pr.n)
    y = rng.integers(0, 1 << 15, E.pr.n)
    x[:6] = [5, 4, 6, 0, 32767, 100]
    y[:6] = [5, 5, 5, 32767, 0, 100]
    lo = np.minimum(x, y)
    hi = lo + rng.integers(0, 2000, E.pr.n)
    return (x, y, lo, hi), [E.enc(v, 70 + i) for i, v in enumerate((x, y, lo, hi))]


# --------------------------------------------------------------- cases ---

def _eq_edges(E: Env) -> dict:
    _, _, cx, cy = eq_edges_inputs(E)
    levels, mask = bfv.eq_chain(E.pr, E.rk, cx, cy)
    out = {f"level_{i:02d}": E.limbs(z) for i, z in enumerate(levels)}
    out["mask"] = E.limbs(mask)
    return out


def _column_uniform(k: int):
    def run(E: Env) -> dict:
        cx, cy = column_uniform_cts(E, k)
        return {f"mask_{k:02d}": E.limbs(bfv.eq_chain(E.pr, E.rk, cx, cy)[1])}
    return run


def _column_structured(k: int):
    def run(E: Env) -> dict:
        cx, cy = column_structured_ct(E, k), column_structured_constant(E)
        return {f"mask_{k:02d}": E.limbs(bfv.eq_chain(E.pr, E.rk, cx, cy)[1])}
    return run


def _rotate_real(E: Env) -> dict:
    _, ct = rotate_inputs(E)
    g, key = real_rotation(E)
    return {"rotate": E.limbs(galois.apply_galois(E.pr, key, ct, g))}


def _sum_slots(E: Env) -> dict:
    _, ct = rotate_inputs(E)
    return {"sum_slots": E.limbs(galois.sum_slots(E.pr, uniform_galois_keys(E.pr), ct))}


def _select(E: Env) -> dict:
    _, _, cp, cm = select_inputs(E)
    return {"select": E.limbs(query.select(E.pr, E.rk, cp, cm))}


def _extract(E: Env) -> dict:
    _, ct = extract_inputs(E)
    return {"extract": E.limbs(join.extract(E.pr, ct, EXTRACT_SLOT))}


def _broadcast(E: Env) -> dict:
    _, ct = extract_inputs(E)
    return {"broadcast": E.limbs(join.broadcast(E.pr, uniform_galois_keys(E.pr), ct,
                                                EXTRACT_SLOT))}


def _join(E: Env) -> dict:
    *_, ca, cbk, cba = join_inputs(E)
    return {"join": E.limbs(join.join_sum(E.pr, E.rk, uniform_galois_keys(E.pr), ca, cbk, cba,
                                          [JOIN_SLOT]))}


def _lt17(E: Env) -> dict:
    E17 = E.with_t(17)
    _, cts = lt17_inputs(E17)
    return {"lt": E17.limbs(compare.lt(E17.pr, E17.rk, cts[0], cts[1]))}


def _between17(E: Env) -> dict:
    E17 = E.with_t(17)
    _, cts = lt17_inputs(E17)
    return {"between": E17.limbs(compare.between(E17.pr, E17.rk, cts[0], cts[2], cts[3]))}


def _lt_n64(E: Env) -> dict:
    _, cts = lt_n64_inputs(E)
    return {"lt": E.limbs(compare.lt(E.pr, E.rk, cts[0], cts[1])),
            "le": E.limbs(compare.le(E.pr, E.rk, cts[0], cts[1])),
            "between": E.limbs(compare.between(E.pr, E.rk, cts[0], cts[2], cts[3]))}


A2_COLUMN_CTS = 8             # ciphertexts of each column checked with two-prime digits
A3_COLUMN_CTS = 4             # ... and with three-prime digits

# case -> (log2 N of its Env, [(unit name, function)]); CASE_ALPHA gives the
# special primes of a case's Env (1 if absent)
CASES = {
    "eq_edges": (15, [("chain", _eq_edges)]),
    "eq_column_uniform": (15, [(f"ct{k:02d}", _column_uniform(k)) for k in range(COLUMN_CTS)]),
    "eq_column_structured": (15, [(f"ct{k:02d}", _column_structured(k))
                                  for k in range(COLUMN_CTS)]),
    "rotations": (15, [("rotate", _rotate_real), ("sum_slots", _sum_slots)]),
    "products": (15, [("select", _select), ("extract", _extract), ("broadcast", _broadcast)]),
    "join": (15, [("join", _join)]),
    "lt_t17": (15, [("lt", _lt17), ("between", _between17)]),
    "lt_n64": (6, [("lt", _lt_n64)]),
    "a2_eq_edges": (15, [("chain", _eq_edges)]),
    "a2_eq_column_uniform": (15, [(f"ct{k:02d}", _column_uniform(k))
                                  for k in range(A2_COLUMN_CTS)]),
    "a2_eq_column_structured": (15, [(f"ct{k:02d}", _column_structured(k))
                                     for k in range(A2_COLUMN_CTS)]),
    "a2_rotations": (15, [("rotate", _rotate_real), ("sum_slots", _sum_slots)]),
    "a2_products": (15, [("select", _select), ("extract", _extract), ("broadcast", _broadcast)]),
    "a2_join": (15, [("join", _join)]),
    "a2_lt_t17": (15, [("lt", _lt17), ("between", _between17)]),
    "a2_lt_n64": (6, [("lt", _lt_n64)]),
    "a3_eq_edges": (15, [("chain", _eq_edges)]),
    "a3_eq_column_uniform": (15, [(f"ct{k:02d}", _column_uniform(k))
                                  for k in range(A3_COLUMN_CTS)]),
    "a3_eq_column_structured": (15, [(f"ct{k:02d}", _column_structured(k))
                                     for k in range(A3_COLUMN_CTS)]),
    "a3_rotations": (15, [("rotate", _rotate_real), ("sum_slots", _sum_slots)]),
    "a3_products": (15, [("select", _select), ("extract", _extract), ("broadcast", _broadcast)]),
    "a3_join": (15, [("join", _join)]),
    "a3_lt_t17": (15, [("lt", _lt17), ("between", _between17)]),
    "a3_lt_n64": (6, [("lt", _lt_n64)]),
}
CASE_ALPHA = {c: int(c[1]) for c in CASES if c[:3] in ("a2_", "a3_")}
