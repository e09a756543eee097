"""Exact arithmetic in Z[x]/(x^n + 1) with Python integers.

Test infrastructure (oracle).  The FV rings are R_q = Z_q[x]/(x^n+1) and
R_t = Z_t[x]/(x^n+1) (App. A, "Mathematical Notation"; the paper's Phi_n is
read as x^n + 1 with n a power of two).  Ciphertext multiplication (App. A,
Alg. "Ciphertext Multiplication") needs the product of integer
representatives over Z before the t/q scaling, so products here are exact
over Z and reduction mod x^n + 1 is the negacyclic fold c_k - c_{k+n}.

`negacyclic_mul` evaluates both operands at x = 2^W (Kronecker substitution),
multiplies the two Python integers and reads the coefficients back; with W
large enough that every coefficient of the product fits in W-1 bits plus sign
this is the polynomial product exactly.  `negacyclic_mul_schoolbook` is the
O(n^2) definition used to pin it.
"""


def center(x, q):
    """Representative of x mod q in (-q/2, q/2] (q odd: in (-q/2, q/2))."""
    x %= q
    return x - q if 2 * x > q else x


def negacyclic_mul_schoolbook(a, b):
    """Product in Z[x]/(x^n+1) by the definition: x^n = -1."""
    n = len(a)
    assert len(b) == n
    c = [0] * n
    for i, ai in enumerate(a):
        if ai == 0:
            continue
        for j, bj in enumerate(b):
            k = i + j
            if k < n:
                c[k] += ai * bj
            else:
                c[k - n] -= ai * bj
    return c


def _slot_bits(bound):
    # every packed coefficient must satisfy |c| < 2^(W-1)
    return max(8, ((bound.bit_length() + 2 + 7) // 8) * 8)


def _pack_nonneg(a, nbytes):
    return int.from_bytes(b"".join(x.to_bytes(nbytes, "little") for x in a), "little")


def _pack(a, w):
    """Evaluate sum_i a_i 2^(w i) for signed integer coefficients, |a_i| < 2^(w-1)."""
    nbytes = w // 8
    pos = _pack_nonneg([x if x > 0 else 0 for x in a], nbytes)
    neg = _pack_nonneg([-x if x < 0 else 0 for x in a], nbytes)
    return pos - neg


def _unpack(v, w, count):
    """Signed base-2^w digits of v, lowest first; digits lie in [-2^(w-1), 2^(w-1))."""
    half = 1 << (w - 1)
    # shift every digit into [0, 2^w) so the bytes can be sliced directly
    bias = _pack([half] * count, w)
    u = v + bias
    assert u >= 0
    nbytes = w // 8
    raw = u.to_bytes(nbytes * count + 1, "little")
    assert raw[-1] == 0, "value out of range for the packing width"
    return [int.from_bytes(raw[i * nbytes:(i + 1) * nbytes], "little") - half for i in range(count)]


def negacyclic_sum_of_products(pairs, n, coeff_bound):
    """sum_k a_k * b_k in Z[x]/(x^n+1), exactly, for integer polynomials.

    `coeff_bound` must bound every |a_i|, |b_j| of every pair.  Evaluation at
    2^W is a ring homomorphism Z[x] -> Z, so the sum of the evaluated products
    is the evaluated sum; it is unpacked once.
    """
    pairs = list(pairs)
    bound = coeff_bound * coeff_bound * n * max(1, len(pairs))
    w = _slot_bits(bound)
    acc = 0
    for a, b in pairs:
        assert len(a) == n and len(b) == n
        acc += _pack(a, w) * _pack(b, w)
    full = _unpack(acc, w, 2 * n)
    return [full[k] - full[k + n] for k in range(n)]


def negacyclic_mul(a, b, coeff_bound=None):
    """a * b in Z[x]/(x^n+1), exactly."""
    n = len(a)
    if coeff_bound is None:
        coeff_bound = max(1, max(abs(x) for x in a), max(abs(x) for x in b))
    return negacyclic_sum_of_products([(a, b)], n, coeff_bound)
