"""Textbook FV (Fan-Vercauteren) with exact integers.

Test infrastructure (oracle).  Follows App. A of the HERS paper: Alg. "Key
Generation", "Encryption", "Decryption", "Ciphertext Addition" and
"Ciphertext Multiplication".  Polynomials are Python lists of n integers;
elements of R_q are kept as canonical representatives in [0, q).

Readings of points the paper leaves open (each also listed in the design notes):
  * x^n + 1 for Phi_n; n a power of two.
  * theta_sk and u are drawn from R_2 = {0,1}^n (the algorithms' literal R_2).
  * chi is a centred binomial with eta = 20 (sigma = sqrt 10).
  * the representative of m in Delta*m is canonical, m_i in [0, t).
  * integer representatives entering the tensor product are centred, in
    (-q/2, q/2); q is odd so this is unambiguous.
  * rounding to nearest needs no tie rule: t*X/q has denominator q (odd),
    so it is never a half-integer.
  * evaluation keys use an RNS gadget refined by a power-of-two base w = 2^w_bits
    (the paper's base-w decomposition with l digits when q has one prime):
    digit (rho, l) of c2 is bits [l*w_bits, (l+1)*w_bits) of
    y_rho = [c2 * (q/q_rho)^-1]_{q_rho}, and its gadget value is
    g_{rho,l} = (q/q_rho) * 2^(l*w_bits) mod q, so that sum y_{rho,l} g_{rho,l} = c2 mod q.
    w_bits = 0 means one digit per prime (l = 0 only).
"""

from dataclasses import dataclass, field

from . import philox
from .primes import ntt_primes, plain_modulus
from .ring import center, negacyclic_mul, negacyclic_sum_of_products


@dataclass
class Params:
    n: int
    qbits: tuple
    t_bits: int
    w_bits: int = 0
    eta: int = 20
    q_primes: list = field(init=False)
    q: int = field(init=False)
    t: int = field(init=False)
    delta: int = field(init=False)

    def __post_init__(self):
        two_n = 2 * self.n
        self.t = plain_modulus(self.t_bits, two_n)
        self.q_primes = ntt_primes(list(self.qbits), two_n, exclude=(self.t,))
        q = 1
        for p in self.q_primes:
            q *= p
        self.q = q
        # Alg. "Encryption": Delta = floor(q / t)
        self.delta = q // self.t

    @property
    def k(self):
        return len(self.q_primes)

    def digit_count(self, rho):
        if self.w_bits == 0:
            return 1
        return (self.q_primes[rho].bit_length() + self.w_bits - 1) // self.w_bits

    def gadget(self):
        """List of (rho, l, g_{rho,l}) in key order."""
        out = []
        for rho, p in enumerate(self.q_primes):
            qhat = self.q // p
            for l in range(self.digit_count(rho)):
                shift = l * self.w_bits
                out.append((rho, l, (qhat << shift) % self.q))
        return out


# ----------------------------------------------------------------------------- helpers

def crt(residues, primes):
    """The integer in [0, prod p) with the given residues."""
    q = 1
    for p in primes:
        q *= p
    x = 0
    for r, p in zip(residues, primes):
        qh = q // p
        x += r * qh * pow(qh, -1, p)
    return x % q


def to_residues(poly, primes):
    """res[rho][j] = poly[j] mod p_rho."""
    return [[c % p for c in poly] for p in primes]


def from_residues(res, primes):
    n = len(res[0])
    return [crt([res[r][j] for r in range(len(primes))], primes) for j in range(n)]


def poly_mod(a, q):
    return [x % q for x in a]


def poly_add(a, b, q):
    return [(x + y) % q for x, y in zip(a, b)]


def poly_neg(a, q):
    return [(-x) % q for x in a]


def poly_mul_q(a, b, q):
    """Product in R_q of canonical representatives (exact over Z, then mod q)."""
    return poly_mod(negacyclic_mul([center(x, q) for x in a], [center(x, q) for x in b]), q)


def sample_uniform_q(params, key, obj):
    """Uniform element of R_q (residues drawn independently; CRT-combined)."""
    res = philox.sample_uniform_residues(key, obj, params.n, params.q_primes)
    return from_residues(res, params.q_primes)


# ----------------------------------------------------------------------------- KeyGen

KEY_OBJ_S = (0, 0, 0)
KEY_OBJ_A = (1, 0, 0)
KEY_OBJ_E = (2, 0, 0)


def key_obj_rlk_a(g):
    return (3, g, 0)


def key_obj_rlk_e(g):
    return (4, g, 0)


def keygen(params, seed):
    """Alg. "Key Generation": theta_sk from R_2; pk = ([-(a s + e)]_q, a);
    one evaluation key ([-(a_g s + e_g) + g s^2]_q, a_g) per gadget element g."""
    n, q = params.n, params.q
    key = (seed, philox.DOMAIN_KEYGEN)
    s = philox.sample_binary(key, KEY_OBJ_S, n)
    a = sample_uniform_q(params, key, KEY_OBJ_A)
    e = philox.sample_cbd(key, KEY_OBJ_E, n, params.eta)
    as_ = poly_mul_q(a, s, q)
    pk0 = poly_neg(poly_add(as_, poly_mod(e, q), q), q)
    pk = (pk0, a)
    s2 = poly_mul_q(s, s, q)
    rlk = []
    for g_idx, (_rho, _l, g) in enumerate(params.gadget()):
        ag = sample_uniform_q(params, key, key_obj_rlk_a(g_idx))
        eg = philox.sample_cbd(key, key_obj_rlk_e(g_idx), n, params.eta)
        b = poly_neg(poly_add(poly_mul_q(ag, s, q), poly_mod(eg, q), q), q)
        b = poly_add(b, [(g * x) % q for x in s2], q)
        rlk.append((b, ag))
    return s, pk, rlk


# ----------------------------------------------------------------------------- Encrypt / Decrypt

def encrypt(params, pk, m, key, obj3):
    """Alg. "Encryption": ct = ([Delta m + pk0 u + e1]_q, [pk1 u + e2]_q).

    `m` has coefficients in [0, t).  u, e1, e2 are the Philox objects
    (obj3[0], obj3[1], 0/1/2) under `key`."""
    n, q = params.n, params.q
    u = philox.sample_binary(key, (obj3[0], obj3[1], 0), n)
    e1 = philox.sample_cbd(key, (obj3[0], obj3[1], 1), n, params.eta)
    e2 = philox.sample_cbd(key, (obj3[0], obj3[1], 2), n, params.eta)
    ct0 = [(params.delta * mi + x + e) % q for mi, x, e in zip(m, poly_mul_q(pk[0], u, q), e1)]
    ct1 = [(x + e) % q for x, e in zip(poly_mul_q(pk[1], u, q), e2)]
    return (ct0, ct1)


def encrypt_sk(params, sk, m, key, obj3):
    """Encryption under the secret key (reading of Sec. 3.2, "Search Protocol",
    where the client encrypts its query with its private key; App. A defines
    only the public-key form): ct = ([Delta m - a s + e]_q, a), a uniform in R_q,
    e from chi, so that ct0 + ct1 s = Delta m + e.

    `m` has coefficients in [0, t).  a, e are the Philox objects
    (obj3[0], obj3[1], 0/1) under `key`."""
    n, q = params.n, params.q
    a = sample_uniform_q(params, key, (obj3[0], obj3[1], 0))
    e = philox.sample_cbd(key, (obj3[0], obj3[1], 1), n, params.eta)
    a_s = poly_mul_q(a, sk, q)
    ct0 = [(params.delta * mi - x + ei) % q for mi, x, ei in zip(m, a_s, e)]
    return (ct0, a)


def decrypt(params, sk, ct):
    """Alg. "Decryption": pt = [round(t/q [ct0 + ct1 s]_q)]_t, returned in [0, t).

    A ciphertext of degree 2 (c0, c1, c2) decrypts with c2 s^2 added."""
    q, t = params.q, params.t
    x = poly_add(ct[0], poly_mul_q(ct[1], sk, q), q)
    if len(ct) == 3:
        x = poly_add(x, poly_mul_q(ct[2], poly_mul_q(sk, sk, q), q), q)
    return [round_div(t * center(v, q), q) % t for v in x]


def noise(params, sk, ct, m):
    """Infinity norm of v = [ct0 + ct1 s - Delta m]_q (centred): the decryption noise."""
    q = params.q
    x = poly_add(ct[0], poly_mul_q(ct[1], sk, q), q)
    if len(ct) == 3:
        x = poly_add(x, poly_mul_q(ct[2], poly_mul_q(sk, sk, q), q), q)
    return max(abs(center(v - params.delta * (mi % params.t), q)) for v, mi in zip(x, m))


def round_div(num, den):
    """Nearest integer to num/den for den > 0 (floor(num/den + 1/2))."""
    return (2 * num + den) // (2 * den)


# ----------------------------------------------------------------------------- Add / Multiply

def add(params, a, b):
    """Alg. "Ciphertext Addition": component-wise sum mod q."""
    return tuple(poly_add(x, y, params.q) for x, y in zip(a, b))


def tensor(params, pairs):
    """Exact tensor of centred lifts, summed over pairs of ciphertexts:
    X0 = sum a0 b0, X1 = sum (a0 b1 + a1 b0), X2 = sum a1 b1, over Z[x]/(x^n+1)."""
    n, q = params.n, params.q
    lifted = [([center(x, q) for x in a[0]], [center(x, q) for x in a[1]],
               [center(x, q) for x in b[0]], [center(x, q) for x in b[1]]) for a, b in pairs]
    bound = q // 2 + 1
    x0 = negacyclic_sum_of_products([(a0, b0) for a0, a1, b0, b1 in lifted], n, bound)
    x1 = negacyclic_sum_of_products([(a0, b1) for a0, a1, b0, b1 in lifted]
                                    + [(a1, b0) for a0, a1, b0, b1 in lifted], n, bound)
    x2 = negacyclic_sum_of_products([(a1, b1) for a0, a1, b0, b1 in lifted], n, bound)
    return x0, x1, x2


def scale_round(params, X):
    """c = [round(t X / q)]_q coefficient-wise (Alg. "Ciphertext Multiplication")."""
    q, t = params.q, params.t
    return [round_div(t * x, q) % q for x in X]


def relin_digits(params, c2):
    """Gadget digits y_{rho,l} of c2 (see module docstring), in key order."""
    q = params.q
    out = []
    for rho, p in enumerate(params.q_primes):
        qhat_inv = pow(q // p, -1, p)
        y = [(c * qhat_inv) % p for c in c2]
        for l in range(params.digit_count(rho)):
            if params.w_bits == 0:
                out.append(y)
            else:
                sh, mask = l * params.w_bits, (1 << params.w_bits) - 1
                out.append([(v >> sh) & mask for v in y])
    return out


def relinearize(params, rlk, c):
    """(c0, c1, c2) -> (c0 + sum_g y_g rlk_g[0], c1 + sum_g y_g rlk_g[1]) mod q."""
    q, n = params.q, params.n
    c0, c1, c2 = c
    digits = relin_digits(params, c2)
    bound = q
    s0 = negacyclic_sum_of_products([(y, r[0]) for y, r in zip(digits, rlk)], n, bound)
    s1 = negacyclic_sum_of_products([(y, r[1]) for y, r in zip(digits, rlk)], n, bound)
    return (poly_add(c0, poly_mod(s0, q), q), poly_add(c1, poly_mod(s1, q), q))


def multiply(params, rlk, a, b):
    """Alg. "Ciphertext Multiplication": tensor, scale by t/q and round, relinearize."""
    X = tensor(params, [(a, b)])
    c = tuple(scale_round(params, x) for x in X)
    return relinearize(params, rlk, c)
