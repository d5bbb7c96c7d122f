"""Textbook word-level BFV and the Fermat equality mask, in exact integers.

Test infrastructure only (see the package docstring).

Every ciphertext here is a tuple of polynomials with integer coefficients in
[0, Q); every operation is written from its integer definition, with
rounding done on exact Python integers.  The paper fixes the scheme (BFV,
Sec. 1 and 2.1.5), the parameters (n = 32768, log Q = 881, p = t = 65537,
Sec. 5.1) and the mask (Eq. eq:equality, evaluated by exponentiation by
squaring, Sec. 4.3.1); it leaves the RNS split, distributions, relinearization
method and rounding conventions to the library (SEAL).  The readings taken
here are:

* Q*P spans at most 881 bits; P is the special modulus of key switching,
  one prime (the default) or the product of alpha primes;
* secret key uniform ternary, errors rounded Gaussian (sigma 3.2), drawn by
  the caller and passed in;
* secret-key encryption ct = ([Delta*m + e - a*s]_Q, a), Delta = floor(Q/t);
* multiply: centred lifts to (-Q/2, Q/2), exact products in Z[X]/(X^N+1),
  then c_k = [round(t * d_k / Q)]_Q (no ties: Q odd, gcd(t, Q) = 1);
* relinearize after every multiply with digits of alpha data primes each
  (alpha = the number of special primes; one digit per data prime when
  alpha = 1): the data primes are taken in order in groups of alpha, group j
  with product Q_j, D_j = [c_2]_{Q_j} in [0, Q_j), key
  evk_j = ([-a_j s + e_j + P g_j s^2]_{PQ}, a_j) with
  g_j = (Q/Q_j) * [(Q/Q_j)^-1]_{Q_j}, and
  c_b' = [c_b + round(sum_j D_j evk_j[b] / P)]_Q (no ties: P odd).  Several
  primes per digit is the hybrid key switching of Han and Ki ("Better
  bootstrapping for approximate homomorphic encryption", CT-RSA 2020): fewer,
  larger digits, with P at least as large as a digit;
* the constant 1 of "1 - z^(p-1)" is the trivial encryption (Delta, 0).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import nt
from . import ring
from . import encoding


# ------------------------------------------------------------ parameters ---

@dataclass(frozen=True)
class Params:
    n: int                      # ring degree = number of slots
    t: int                      # plaintext modulus p (prime, = 1 mod 2n)
    q: tuple                    # data primes q_0 .. q_{L-1}
    special: object             # special prime(s) of key switching: an int
                                # (one prime) or a tuple of alpha primes

    def __post_init__(self):
        sp = self.special
        object.__setattr__(self, "special", (int(sp),) if isinstance(sp, (int, np.integer))
                           else tuple(int(x) for x in sp))

    @property
    def L(self) -> int:
        return len(self.q)

    @property
    def alpha(self) -> int:
        """Data primes per key-switching digit = number of special primes."""
        return len(self.special)

    @property
    def dnum(self) -> int:
        """Number of key-switching digits, ceil(L / alpha)."""
        return -(-self.L // self.alpha)

    def digit_primes(self, j: int) -> tuple:
        """The data primes of digit j: q_{j alpha} .. q_{min(L, (j+1) alpha) - 1}."""
        return tuple(self.q[j * self.alpha:(j + 1) * self.alpha])

    def digit_modulus(self, j: int) -> int:
        """Q_j, the product of digit j's primes."""
        out = 1
        for x in self.digit_primes(j):
            out *= x
        return out

    @property
    def P(self) -> int:
        """The special modulus: the product of the special primes."""
        out = 1
        for x in self.special:
            out *= x
        return out

    @property
    def Q(self) -> int:
        out = 1
        for x in self.q:
            out *= x
        return out

    @property
    def PQ(self) -> int:
        return self.Q * self.P

    @property
    def delta(self) -> int:
        return self.Q // self.t

    @property
    def moduli_pq(self) -> tuple:
        """Limb order of a relinearization-key polynomial: q_0..q_{L-1}, then
        the special primes."""
        return tuple(self.q) + self.special

    def gadget(self, j: int) -> int:
        """g_j = (Q/Q_j) [(Q/Q_j)^-1]_{Q_j}: g_j = 1 mod Q_j, 0 mod Q_i (i != j)."""
        Qj = self.digit_modulus(j)
        qh = self.Q // Qj
        return qh * pow(qh, -1, Qj)

    def squarings(self) -> int:
        """Multiplicative depth of EQ: ceil(log2(t - 1)) (Table
        table:noise_levels, equality row)."""
        return (self.t - 2).bit_length()


def paper_params(n: int = 32768, t: int = 65537, alpha: int = 1) -> Params:
    """The paper's parameters (Sec. 5.1) with alpha special primes (and
    18 - alpha data primes)."""
    q, P = nt.default_modulus_chain(n_special=alpha)
    return Params(n, t, tuple(q), P)


# --------------------------------------------------------- integer helpers ---

def reduce(a, M: int) -> np.ndarray:
    return ring.as_object(a) % M


def centred(a, M: int) -> np.ndarray:
    """Representatives in (-M/2, M/2] (for odd M: |x| <= (M-1)/2)."""
    a = ring.as_object(a) % M
    return np.where(a > M // 2, a - M, a)


def round_div(x, d: int) -> np.ndarray:
    """Nearest integer to x / d for integer x and d > 0 (halves round up;
    no call below can meet a half)."""
    return (2 * ring.as_object(x) + d) // (2 * d)


def to_limbs(poly, moduli) -> np.ndarray:
    """Exchange format: [len(moduli), N] int64 residues in [0, m_i)."""
    a = ring.as_object(poly)
    return np.stack([(a % m).astype(np.int64) for m in moduli])


def from_limbs(limbs, moduli) -> np.ndarray:
    """Integers in [0, prod(moduli)) from residues (Chinese remainder)."""
    limbs = np.asarray(limbs)
    M = 1
    for m in moduli:
        M *= m
    acc = np.zeros(limbs.shape[-1], dtype=object)
    for i, m in enumerate(moduli):
        Mi = M // m
        acc = acc + limbs[i].astype(object) * (Mi * pow(Mi, -1, m))
    return acc % M


def poly_mul(a, b) -> np.ndarray:
    return ring.negacyclic_product(a, b)


# ------------------------------------------------------------------- keys ---

@dataclass
class SecretKey:
    s: np.ndarray                     # ternary coefficients (object ints)


@dataclass
class RelinKey:
    b: list                           # dnum polys mod PQ
    a: list                           # dnum polys mod PQ
    _own_cache: dict = field(default_factory=dict, repr=False)

    def limbs(self, params: Params) -> np.ndarray:
        """Exchange format [dnum][2][L+alpha][N] int64, limbs in moduli_pq
        order, coefficient domain."""
        m = params.moduli_pq
        return np.stack([np.stack([to_limbs(self.b[j], m), to_limbs(self.a[j], m)])
                         for j in range(params.dnum)])


def switching_key(params: Params, s, s_from, a_limbs, errors) -> RelinKey:
    """Key switching key from s_from to s: per digit j,
    (b_j, a_j) = ([-a_j s + e_j + P g_j s_from]_{PQ}, a_j)."""
    PQ = params.PQ
    s = ring.as_object(s)
    s_from = ring.as_object(s_from)
    bs, as_ = [], []
    for j in range(params.dnum):
        a = from_limbs(a_limbs[j], params.moduli_pq)
        e = ring.as_object(errors[j])
        b = (-poly_mul(a, s) + e + params.P * params.gadget(j) * s_from) % PQ
        bs.append(b)
        as_.append(a)
    return RelinKey(bs, as_)


def keygen(params: Params, rnd) -> tuple[SecretKey, RelinKey]:
    """Secret key and relinearization key (switching from s^2 to s) from
    caller-drawn randomness (`synth.key_randomness`)."""
    s = ring.as_object(rnd.s)
    s2 = poly_mul(s, s)
    return SecretKey(s), switching_key(params, s, s2, rnd.a, rnd.e)


# ------------------------------------------------------ encrypt / decrypt ---

def encrypt(params: Params, sk: SecretKey, m_poly, rnd) -> tuple:
    """Secret-key BFV encryption of plaintext polynomial m (coefficients in
    [0, t)) with caller-drawn randomness (`synth.enc_randomness`)."""
    Q = params.Q
    a = from_limbs(rnd.a, params.q)
    e = ring.as_object(rnd.e)
    c0 = (params.delta * ring.as_object(m_poly) + e - poly_mul(a, sk.s)) % Q
    return (c0, a)


def phase(params: Params, sk: SecretKey, ct) -> np.ndarray:
    """[c_0 + c_1 s + c_2 s^2 + ...]_Q in [0, Q)."""
    Q = params.Q
    acc = ring.as_object(ct[0]) % Q
    spow = None
    for k in range(1, len(ct)):
        spow = sk.s if spow is None else poly_mul(spow, sk.s)
        acc = (acc + poly_mul(ct[k], spow)) % Q
    return acc


def decrypt(params: Params, sk: SecretKey, ct) -> np.ndarray:
    """Plaintext polynomial [round(t * phase / Q)]_t."""
    return round_div(params.t * phase(params, sk, ct), params.Q) % params.t


def noise_bits(params: Params, sk: SecretKey, ct, m_true) -> float:
    """Remaining budget log2(Q / (2 |w|_inf)) with w = t*phase - Q*m_true
    reduced to (-tQ/2, tQ/2]; decryption returns m_true iff the result is
    positive.  `m_true` is the true plaintext polynomial."""
    Q, t = params.Q, params.t
    w = centred(t * phase(params, sk, ct) - Q * ring.as_object(m_true), t * Q)
    wmax = max(abs(int(x)) for x in w)
    if wmax == 0:
        return math.log2(Q)
    return math.log2(Q) - math.log2(2 * wmax)


# --------------------------------------------------------------- evaluate ---

def sub(params: Params, x, y) -> tuple:
    """Component-wise [x - y]_Q (BFV subtraction, Sec. 2.1.6)."""
    Q = params.Q
    return tuple((ring.as_object(a) - ring.as_object(b)) % Q for a, b in zip(x, y))


def _scale_round(params: Params, d) -> np.ndarray:
    return round_div(params.t * d, params.Q) % params.Q


def tensor(params: Params, x, y) -> tuple:
    """The exact tensor components d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1
    of two ciphertexts' centred lifts, as integer polynomials."""
    Q = params.Q
    a0, a1 = centred(x[0], Q), centred(x[1], Q)
    b0, b1 = centred(y[0], Q), centred(y[1], Q)
    n = params.n
    B = ring.OwnBasis(n * (Q // 2) ** 2 * 2, n)
    fa0, fa1 = B.forward(B.residues(a0)), B.forward(B.residues(a1))
    fb0, fb1 = B.forward(B.residues(b0)), B.forward(B.residues(b1))
    d0 = B.to_int(B.inverse(B.mul(fa0, fb0)))
    d1 = B.to_int(B.inverse(B.add(B.mul(fa0, fb1), B.mul(fa1, fb0))))
    d2 = B.to_int(B.inverse(B.mul(fa1, fb1)))
    return (d0, d1, d2)


def multiply(params: Params, x, y) -> tuple:
    """Textbook BFV product (before relinearization), three components."""
    return tuple(_scale_round(params, d) for d in tensor(params, x, y))


def square(params: Params, x) -> tuple:
    """multiply(x, x), computing the shared transforms once."""
    Q = params.Q
    a0, a1 = centred(x[0], Q), centred(x[1], Q)
    n = params.n
    B = ring.OwnBasis(n * (Q // 2) ** 2 * 2, n)
    fa0, fa1 = B.forward(B.residues(a0)), B.forward(B.residues(a1))
    d0 = B.to_int(B.inverse(B.mul(fa0, fa0)))
    f01 = B.mul(fa0, fa1)
    d1 = B.to_int(B.inverse(B.add(f01, f01)))
    d2 = B.to_int(B.inverse(B.mul(fa1, fa1)))
    return tuple(_scale_round(params, d) for d in (d0, d1, d2))


def _evk_transformed(params: Params, rk: RelinKey, B: ring.OwnBasis):
    key = B.primes
    if key not in rk._own_cache:
        rk._own_cache.clear()
        rk._own_cache[key] = [(B.forward(B.residues(rk.b[j])), B.forward(B.residues(rk.a[j])))
                              for j in range(params.dnum)]
    return rk._own_cache[key]


def _switch_basis(params: Params) -> ring.OwnBasis:
    """The own basis of a key switch's exact sums: |sum_j D_j k_j| is below
    dnum max(Q_j) PQ N."""
    mods = [params.digit_modulus(j) for j in range(params.dnum)]
    return ring.OwnBasis(params.dnum * max(mods) * params.PQ * params.n, params.n)


def prepare_key(params: Params, key: RelinKey) -> None:
    """Transform a switching key into the basis key_switch uses (cached on
    the key; a speed-up only, key_switch does it on first use anyway)."""
    _evk_transformed(params, key, _switch_basis(params))


def key_switch(params: Params, key: RelinKey, c) -> tuple:
    """Key switching of one polynomial c (coefficients mod Q) with a
    switching key for some s' (b_j + a_j s = e_j + P g_j s' mod PQ): digits
    D_j = [c]_{Q_j} in [0, Q_j) (one data prime each when alpha = 1), and
    (round(sum_j D_j b_j / P), round(sum_j D_j a_j / P)) mod Q, whose phase
    is c * s' plus a small error."""
    Q, P, n = params.Q, params.P, params.n
    c = ring.as_object(c)
    mods = [params.digit_modulus(j) for j in range(params.dnum)]
    digits = [(c % Qj).astype(np.int64) if Qj < (1 << 62) else c % Qj for Qj in mods]
    B = _switch_basis(params)
    evk = _evk_transformed(params, key, B)
    acc0 = np.zeros((len(B.primes), n), dtype=np.int64)
    acc1 = np.zeros_like(acc0)
    for j, dj in enumerate(digits):
        fd = B.forward(B.residues(dj))
        acc0 = B.add(acc0, B.mul(fd, evk[j][0]))
        acc1 = B.add(acc1, B.mul(fd, evk[j][1]))
    u0 = B.to_int(B.inverse(acc0))
    u1 = B.to_int(B.inverse(acc1))
    return (round_div(u0, P) % Q, round_div(u1, P) % Q)


def relinearize(params: Params, rk: RelinKey, ct3) -> tuple:
    """Key switching of the s^2 component (digits of alpha data primes)."""
    Q = params.Q
    c0, c1, c2 = (ring.as_object(c) for c in ct3)
    k0, k1 = key_switch(params, rk, c2)
    return ((c0 + k0) % Q, (c1 + k1) % Q)


def square_relin(params: Params, rk: RelinKey, x) -> tuple:
    return relinearize(params, rk, square(params, x))


def mul_relin(params: Params, rk: RelinKey, x, y) -> tuple:
    return relinearize(params, rk, multiply(params, x, y))


def mul_sum_relin(params: Params, rk: RelinKey, pairs) -> tuple:
    """A sum of products with one scale-and-round and one relinearization:
    the pairs' exact tensors are added as integers, then [round(t D / Q)]_Q
    and relinearized (it decrypts to the sum of the products)."""
    D = None
    for x, y in pairs:
        d = tensor(params, x, y)
        D = d if D is None else tuple(u + v for u, v in zip(D, d))
    return relinearize(params, rk, tuple(_scale_round(params, d) for d in D))


def finish(params: Params, z) -> tuple:
    """(Delta, 0) - z: the encryption of 1 - z (slot-wise)."""
    Q = params.Q
    c0 = (-ring.as_object(z[0])) % Q
    c0[0] = (c0[0] + params.delta) % Q
    return (c0, (-ring.as_object(z[1])) % Q)


def eq_chain(params: Params, rk: RelinKey, x, y) -> tuple[list, tuple]:
    """EQ(x, y) = 1 - (x - y)^(t-1) by left-to-right square-and-multiply on
    the exponent t - 1, relinearizing after every product.  Returns the list
    of intermediate ciphertexts (index 0 = x - y, then one per squaring) and
    the output.  For a Fermat prime t (t - 1 = 2^k) the list holds exactly k
    squarings."""
    z = sub(params, x, y)
    levels = [z]
    e = params.t - 1
    acc = z
    for bit in bin(e)[3:]:
        acc = square_relin(params, rk, acc)
        if bit == "1":
            acc = mul_relin(params, rk, acc, z)
        levels.append(acc)
    return levels, finish(params, acc)


# ----------------------------------------------------------- slot helpers ---

def encrypt_slots(params: Params, sk: SecretKey, slots, rnd) -> tuple:
    return encrypt(params, sk, encoding.encode(slots, params.t), rnd)


def decrypt_slots(params: Params, sk: SecretKey, ct) -> np.ndarray:
    return encoding.decode(decrypt(params, sk, ct), params.t)
