"""Reference oracle for HERS encrypted search (test infrastructure only).

This package is a plain, slow, exact CPU implementation of what the HERS
encrypted-search path computes: textbook FV (Fan-Vercauteren) over
Z_q[x]/(x^n+1) with Python big integers, the per-dimension SIMD slot encoding
of the HERS paper (Sec. 3.2, Eq. 2-4, Alg. "HERS Enrollment" and Alg. "HERS
Search"), and the counter-based random generator both sides draw from.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import it.  It shares no code with the GPU library and never imports it;
the library never imports this package.

Modules
  philox  -- Philox4x64-10 (Salmon et al., SC'11), and the samplers built on it
  primes  -- prime-selection rule for q, t and 2n-th roots of unity
  ring    -- exact negacyclic polynomial products over Z
  fv      -- KeyGen / Encrypt / Decrypt / Add / Multiply / Relinearize (App. A)
  hers    -- slot encoding and the enrollment/search protocols (Sec. 3.2, App. B)

Every function states the passage of the paper it follows.  Points where the
paper is silent or ambiguous follow the readings listed with each function.
"""
