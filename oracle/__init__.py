"""Plain CPU oracle for the rotation-free HE Conv/FC layers (test infrastructure).

This package is the slow, obviously-correct reference that the GPU path is
checked against.  Only the test suite, the smoke check and the CPU-baseline leg
of the benchmark may import it; the product path never does.  It shares no code
with the HIP library: it has its own primes, roots, NTT, packing and scheme
algebra, written from the paper (Sec. II-A, II-C, III-A, III-B) in the exact
BFV-style reading documented per function.

Modules
  params   primes, roots of unity, Delta, CRT
  ring     negacyclic products: schoolbook definition and a textbook NTT
  packing  conv packing (Eq. i_batch / k_batch_new, generalised) and FC packing
           (Eq. i(x) formula / w(x) formula, Theorem 1)
  bfv      key generation, c0 encryption, server evaluation (Alg. 1 / Alg. 2),
           client evaluation and decryption
  network  integer conv / FC reference, plain-20 harness between layers
  counts   Table I / Table III operation counts (and the generalised packing's
           per-layer counts that reduce to them) and Table II byte formulas
  cserver  ctypes binding of c/he_oracle.c, a plain C build of the server
           evaluation (same steps as bfv.server_conv / server_fc, timed as the
           CPU baseline; checked against bfv and the stored digests)

Parity notes: every function is pinned by a CPU test against a closed form,
a brute-force definition, an invariant or a value printed in the paper, except
the harness requantisation between layers, which the paper does not define
(parity unpinned; the same harness feeds both sides).
"""
