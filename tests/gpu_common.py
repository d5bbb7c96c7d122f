"""Shared fixtures for the device parity tests: oracle keys and ciphertexts
moved to the device in the exchange format, and back."""
import numpy as np
import torch

import synth
from oracle import bfv
from paper_2602_24271_amd import Context


def require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("device tests need a HIP device")


class Setup:
    """Oracle parameters/keys plus a device context holding the same
    relinearization key."""

    def __init__(self, log2_n: int, t: int = 65537, seed: int = 0, alpha: int = 1):
        require_gpu()
        n = 1 << log2_n
        self.pr = bfv.paper_params(n, t, alpha)
        self.sk, self.rk = bfv.keygen(self.pr, synth.key_randomness(seed, n, self.pr.moduli_pq,
                                                                     self.pr.dnum))
        self.ctx = Context(log2_n, t, list(self.pr.q), list(self.pr.special))
        evk = torch.from_numpy(self.rk.limbs(self.pr)).to(self.ctx.device)
        self.ctx.set_relin_key(evk)

    def enc(self, slots, seed):
        return bfv.encrypt_slots(self.pr, self.sk, slots, synth.enc_randomness(seed, self.pr.n,
                                                                               self.pr.q))

    def enc_poly(self, m, seed):
        return bfv.encrypt(self.pr, self.sk, m, synth.enc_randomness(seed, self.pr.n, self.pr.q))

    def to_dev(self, cts):
        """list of oracle ciphertexts -> int64 [n, comps, L, N] on the device."""
        arr = np.stack([np.stack([bfv.to_limbs(c, self.pr.q) for c in ct]) for ct in cts])
        return torch.from_numpy(arr).to(self.ctx.device)

    def limbs(self, ct):
        return np.stack([bfv.to_limbs(c, self.pr.q) for c in ct])

    def from_dev(self, t):
        a = t.cpu().numpy()
        return [tuple(bfv.from_limbs(a[i, k], self.pr.q) for k in range(a.shape[1]))
                for i in range(a.shape[0])]


def galois_keys(S: Setup, seed: int = 500):
    """Oracle Galois keys for every element of the rotate-and-add sum, also
    loaded into the device context."""
    from oracle import galois
    keys = {}
    for i, g in enumerate(galois.sum_elements(S.pr.n)):
        rnd = synth.switch_randomness(seed + i, S.pr.n, S.pr.moduli_pq, S.pr.dnum)
        keys[g] = galois.galois_key(S.pr, S.sk, g, rnd)
        S.ctx.set_galois_key(g, torch.from_numpy(keys[g].limbs(S.pr)).to(S.ctx.device))
    return keys
