"""Exact-integer CPU oracle for the NSHEDB equality-mask hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or
links this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code, tables or constants with the HIP
library: it derives its own primes, its own NTT basis and its own CRT
constants, and reaches every ciphertext through plain big-integer
definitions.

What it computes (NSHEDB, Sec. 2.1.6-2.1.7, Sec. 4.2.2 and Sec. 4.3.1):

* word-level BFV over R_Q = Z_Q[X]/(X^N + 1) with batch encoding of N slots
  in Z_t (Sec. 4.1 data storage; BFV operations, Sec. 2.1.6);
* the equality mask EQ(x, y) = 1 - (x - y)^(p-1) (Eq. eq:equality), which for
  a Fermat prime p = t (p - 1 = 2^k) is exactly k chained squarings, each
  followed by relinearization (Sec. 4.3.1, equality checks: exponentiation by
  squaring with ceil(log2(p-1)) multiplications; Sec. 2.1.2, relinearization
  after every multiplication);
* an exact noise meter (Sec. 2.1.2 multiplicative depth / noise budget).

Modules
  nt        primality, NTT-friendly prime search, roots of unity
  ring      exact products in Z[X]/(X^N+1): schoolbook and own-basis NTT + CRT
  encoding  batch encoding of slot vectors (client side)
  bfv       parameters, keys, encryption, textbook multiply/relinearize, EQ,
            decryption and noise
  query     operators built on EQ: IN (Eq. eq:in), GROUP BY masks, SELECT
            (Eq. eq:select), BFV addition
  galois    slot rotations (automorphisms + key switching) and the
            rotate-and-add aggregation of COUNT / SUM
  compare   LT / LE / BETWEEN: the comparison polynomial of the Fermat sum
            and its baby-step giant-step evaluation
  join      plaintext products, Extract, Broadcast and the fused equi-join
            aggregation
  ntt_def   the negacyclic number-theoretic transform written from its
            definition (O(N^2)), for checking a device transform's output

Every function is pinned by a `-m "not gpu"` test against something other
than itself (brute force, closed forms, Fermat/Pepin identities,
homomorphism properties); see tests/test_oracle_*.py.
"""
