"""The negacyclic number-theoretic transform written from its definition.

Test infrastructure only (see the package docstring).

For a prime q = 1 (mod 2N) and psi = nt.root_of_unity(q, 2N) (a primitive
2N-th root of unity), the negacyclic transform of a(X) in Z_q[X]/(X^N+1) is
the vector of evaluations A_j = a(psi^(2j+1)) mod q, j = 0..N-1: the N roots
of X^N + 1.  Products in the ring become slot-wise products of these values.
O(N^2) and pure Python: for small N only.
"""
from __future__ import annotations

from . import nt


def evaluations(a, q: int) -> list[int]:
    """[a(psi^(2j+1)) mod q for j in range(N)]."""
    n = len(a)
    psi = nt.root_of_unity(q, 2 * n)
    out = []
    for j in range(n):
        z = pow(psi, 2 * j + 1, q)
        acc = 0
        for c in reversed(list(a)):
            acc = (acc * z + int(c)) % q
        out.append(acc)
    return out


def evaluation_at(a, q: int, j: int) -> int:
    """a(psi^(2j+1)) mod q for one index j (Horner, O(N))."""
    n = len(a)
    psi = nt.root_of_unity(q, 2 * n)
    z = pow(psi, 2 * j + 1, q)
    acc = 0
    for c in reversed(list(a)):
        acc = (acc * z + int(c)) % q
    return acc
