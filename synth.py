"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds random-number generation and workload shapes only: none of
the method's arithmetic.  Everything the encryption scheme draws at random
(secret key, uniform masks, error samples) is drawn here and handed to the
client-side code as plain arrays; plaintext columns are drawn here too.

Streams: numpy.random.SeedSequence(seed).spawn(k) in a fixed order per
function, so a given (function, seed) always yields the same arrays.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

PAPER_BITS = 16          # column values are 16-bit integers (Sec. 5.4 storage)
ERROR_SIGMA = 3.2        # rounded-Gaussian width (HE-standard practice)


def _gens(seed: int, k: int) -> list[np.random.Generator]:
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


def ternary(rng: np.random.Generator, n: int) -> np.ndarray:
    """n i.i.d. values uniform in {-1, 0, 1} (int64)."""
    return rng.integers(-1, 2, size=n, dtype=np.int64)


def gaussian(rng: np.random.Generator, n: int, sigma: float = ERROR_SIGMA) -> np.ndarray:
    """n i.i.d. rounded normal(0, sigma) samples, clipped at 6 sigma (int64)."""
    v = np.rint(rng.normal(0.0, sigma, size=n))
    lim = np.floor(6 * sigma)
    return np.clip(v, -lim, lim).astype(np.int64)


def uniform_residues(rng: np.random.Generator, moduli, n: int) -> np.ndarray:
    """[len(moduli), n] int64, row i i.i.d. uniform in [0, moduli[i])."""
    return np.stack([rng.integers(0, int(m), size=n, dtype=np.int64) for m in moduli])


@dataclass
class KeyRandomness:
    s: np.ndarray              # [N] ternary secret
    a: list                    # L arrays [len(moduli_pq), N] uniform residues
    e: list                    # L arrays [N] errors


def key_randomness(seed: int, n: int, moduli_pq, n_digits: int) -> KeyRandomness:
    g = _gens(seed, 1 + 2 * n_digits)
    s = ternary(g[0], n)
    a = [uniform_residues(g[1 + 2 * j], moduli_pq, n) for j in range(n_digits)]
    e = [gaussian(g[2 + 2 * j], n) for j in range(n_digits)]
    return KeyRandomness(s, a, e)


@dataclass
class SwitchRandomness:
    a: list                    # L arrays [len(moduli_pq), N] uniform residues
    e: list                    # L arrays [N] errors


def switch_randomness(seed: int, n: int, moduli_pq, n_digits: int) -> SwitchRandomness:
    """Randomness of one key switching key (e.g. a Galois key)."""
    g = _gens(seed, 2 * n_digits)
    a = [uniform_residues(g[2 * j], moduli_pq, n) for j in range(n_digits)]
    e = [gaussian(g[2 * j + 1], n) for j in range(n_digits)]
    return SwitchRandomness(a, e)


@dataclass
class EncRandomness:
    a: np.ndarray              # [L, N] uniform residues mod the data primes
    e: np.ndarray              # [N] errors


def enc_randomness(seed: int, n: int, moduli_q) -> EncRandomness:
    g = _gens(seed, 2)
    return EncRandomness(uniform_residues(g[0], moduli_q, n), gaussian(g[1], n))


def uniform_switch_key(seed: int, n: int, moduli_pq, n_digits: int) -> np.ndarray:
    """int64 [n_digits][2][len(moduli_pq)][n] i.i.d. uniform residues: the
    exchange format of a key switching key, as a stand-in key whose rows are
    not derived from any secret (key switching is defined for any key; such
    a key exercises the arithmetic, not decryption)."""
    g = _gens(seed, 2 * n_digits)
    return np.stack([np.stack([uniform_residues(g[2 * j + b], moduli_pq, n) for b in range(2)])
                     for j in range(n_digits)])


def plain_poly(seed: int, n: int, t: int) -> np.ndarray:
    """A plaintext polynomial with n i.i.d. coefficients uniform in [0, t)
    (int64), for encrypting coefficient vectors directly when t has no
    slots at this ring degree."""
    return _gens(seed, 1)[0].integers(0, t, size=n, dtype=np.int64)


# ---------------------------------------------------------------- columns ---

def column_pair_half_match(seed: int, n_rows: int, bits: int = PAPER_BITS):
    """x uniform in [0, 2^bits); y = x on a seeded half of the rows, else
    uniform (i.i.d. uniform pairs would almost never match)."""
    g = _gens(seed, 3)
    x = g[0].integers(0, 1 << bits, size=n_rows, dtype=np.int64)
    other = g[1].integers(0, 1 << bits, size=n_rows, dtype=np.int64)
    same = g[2].random(n_rows) < 0.5
    return x, np.where(same, x, other)


def column_structured(seed: int, n_rows: int, n_dict: int = 64, zipf_a: float = 1.3):
    """Sorted dictionary ids 1..n_dict with skewed frequencies (clustered
    runs, the shape of a sorted foreign-key column), and one constant id
    from the dictionary broadcast to every row."""
    g = _gens(seed, 2)
    w = 1.0 / np.arange(1, n_dict + 1) ** zipf_a
    ids = g[0].choice(np.arange(1, n_dict + 1), size=n_rows, p=w / w.sum())
    x = np.sort(ids).astype(np.int64)
    y = np.full(n_rows, int(g[1].integers(1, n_dict + 1)), dtype=np.int64)
    return x, y


def edge_differences(x: np.ndarray, y: np.ndarray, t: int) -> tuple[np.ndarray, np.ndarray]:
    """Overwrite the first slots so that x - y takes the edge values
    0, 1, -1 (= t - 1), 3 and (t - 1) / 2 (mod t)."""
    x = x.copy()
    y = y.copy()
    for i, d in enumerate((0, 1, t - 1, 3, (t - 1) // 2)):
        if i < len(x):
            y[i] = 5 if len(x) > 0 else 0
            x[i] = (5 + d) % t
    return x, y


def log_uniform_sizes(seed: int, count: int, lo: int, hi: int) -> np.ndarray:
    """`count` integers log-uniform in [lo, hi] (instance row counts)."""
    g = _gens(seed, 1)[0]
    v = np.exp(g.uniform(np.log(lo), np.log(hi), size=count))
    return np.clip(np.rint(v), lo, hi).astype(np.int64)


# ------------------------------------------- device-resident bench inputs ---

def uniform_device_residues(shape_prefix, moduli, n: int, seed: int, device):
    """torch int64 tensor [*shape_prefix, len(moduli), n] with limb i uniform
    in [0, moduli[i]), generated on `device` from a seeded torch generator.
    A uniform pair of polynomials has the distribution of a fresh RLWE
    ciphertext, which is all a data-oblivious kernel can see."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    out = torch.empty((*shape_prefix, len(moduli), n), dtype=torch.int64, device=device)
    for i, m in enumerate(moduli):
        out[..., i, :] = torch.randint(0, int(m), (*shape_prefix, n), generator=gen,
                                       device=device, dtype=torch.int64)
    return out
