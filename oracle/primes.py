"""Parameter rules: ciphertext primes q_i, plaintext modulus t, roots of unity.

Test infrastructure (oracle).  The paper fixes n = 4096, t = 1,032,193 and a q
made of three 36-bit primes (Sec. 4.1, "Implementation Details"), and defines
the rings R_t = Z_t[x]/(x^n+1), R_q = Z_q[x]/(x^n+1) (App. A, "Mathematical
Notation").  It does not state how the primes are chosen.  Reading used here
(it reproduces the paper's t for n = 4096 and 20 bits):

  * an NTT-friendly prime p satisfies p = 1 (mod 2n), so that Z_p holds a
    primitive 2n-th root of unity and x^n + 1 splits into linear factors;
  * for each requested bit width b (in the order given) take the largest such
    prime below 2^b that has not been taken yet;
  * t is the largest such prime below 2^t_bits.
"""

from sympy import isprime, primitive_root as _sympy_primitive_root


def ntt_primes(bit_widths, two_n, exclude=()):
    """Largest unused primes p < 2^b with p = 1 (mod two_n), one per width."""
    taken = set(exclude)
    out = []
    for b in bit_widths:
        p = ((1 << b) - 1) // two_n * two_n + 1
        while p >= (1 << b):
            p -= two_n
        while p > 2:
            if p not in taken and isprime(p):
                break
            p -= two_n
        if p <= 2:
            raise ValueError("no NTT-friendly prime of %d bits" % b)
        taken.add(p)
        out.append(p)
    return out


def plain_modulus(t_bits, two_n):
    """t: the largest prime below 2^t_bits with t = 1 (mod 2n)."""
    return ntt_primes([t_bits], two_n)[0]


def smallest_generator(p):
    """Smallest primitive root modulo the prime p."""
    return int(_sympy_primitive_root(p))


def psi(p, two_n):
    """Primitive 2n-th root of unity mod p: g^((p-1)/2n), g the smallest generator."""
    assert (p - 1) % two_n == 0
    return pow(smallest_generator(p), (p - 1) // two_n, p)
