"""HERS encoding and protocols (enrollment and search) on top of the FV oracle.

Test infrastructure (oracle).  Follows Sec. 3.2 of the HERS paper (Eq. 2-4,
"Enrollment Protocol", "Search Protocol") and App. B (Alg. "HERS Enrollment",
Alg. "HERS Search").

Readings of the paper (also listed in the design notes):
  * Encoding (Eq. 2-4 with the SIMD/CRT batching the paper states it uses):
    a slot vector z in Z_t^n is the polynomial m in R_t with
    m(psi^(2j+1)) = z_j for j = 0..n-1, psi the primitive 2n-th root of unity
    of `primes.psi`; the ring product is then the slot-wise product.  The
    query's dimension i fills every slot, which is the constant polynomial
    [q_i]_t.  Gallery block b, dimension i holds item b*n + j in slot j,
    zero-padded past m (footnote to Eq. 4: blocks of n items).
  * Gallery encryption is the batch form: one fresh Encrypt per (block, dim),
    randomness object (b, i, {0: u, 1: e1, 2: e2}) under key (seed, GALLERY).
    The probe's dimension i uses object (0, i, .) under key (seed, PROBE).
  * The query is encrypted with the public key (the algorithm's Encrypt, the
    only one App. A defines); the protocol text's "using the private key" is
    kept as a second form, encrypt_probe_sk (key (seed, PROBE_SK)).
  * Search, fused form F: per block the exact tensor of the centred lifts is
    summed over the d dimensions, scaled by t/q and rounded once per
    component, then relinearized once; the score accumulator starts at the
    trivial zero ciphertext.  The paper-literal form L (multiply, which
    rescales and relinearizes, then add, per dimension) is kept as a
    cross-check: both decrypt to the same scores.
  * Scores are read back centred in [-t/2, t/2) (the paper's [.]_t).
"""

import numpy as np

from . import fv, philox
from .primes import psi as _psi


# ----------------------------------------------------------------------------- slot encoding

_VAND = {}


def _vandermonde(n, t):
    """V[j, k] = psi^((2j+1) k) mod t and its inverse n^-1 psi^(-(2j+1) k) (transposed)."""
    key = (n, t)
    if key not in _VAND:
        root = _psi(t, 2 * n)
        pw = np.array([pow(root, e, t) for e in range(2 * n)], dtype=np.int64)
        ipw = np.array([pow(root, (2 * n - e) % (2 * n), t) for e in range(2 * n)], dtype=np.int64)
        j = np.arange(n, dtype=np.int64)
        expo = ((2 * j[:, None] + 1) * j[None, :]) % (2 * n)      # [slot j, coeff k]
        V = pw[expo]
        n_inv = pow(n, -1, t)
        Vinv = (ipw[expo].T * n_inv) % t                           # [coeff k, slot j]
        _VAND[key] = (V, Vinv)
    return _VAND[key]


def encode_slots(params, z):
    """z: (..., n) slot values (any integers) -> coefficients in [0, t) (..., n)."""
    n, t = params.n, params.t
    z = np.asarray(z, dtype=np.int64) % t
    _, Vinv = _vandermonde(n, t)
    return (z @ Vinv.T) % t


def decode_slots(params, m):
    """Coefficients (..., n) -> slot values in [0, t)."""
    n, t = params.n, params.t
    m = np.asarray(m, dtype=np.int64) % t
    V, _ = _vandermonde(n, t)
    return (m @ V.T) % t


def encode_slots_direct(params, z):
    """Definition, pure Python, O(n^2): m_k = n^-1 sum_j z_j psi^(-(2j+1) k) mod t."""
    n, t = params.n, params.t
    root = _psi(t, 2 * n)
    rinv = pow(root, -1, t)
    n_inv = pow(n, -1, t)
    return [n_inv * sum(int(z[j]) * pow(rinv, (2 * j + 1) * k, t) for j in range(n)) % t
            for k in range(n)]


def evaluate_at_slot(params, m, j):
    """m(psi^(2j+1)) mod t, by Horner; the definition of slot j."""
    t = params.t
    x = pow(_psi(t, 2 * params.n), 2 * j + 1, t)
    acc = 0
    for c in reversed(list(m)):
        acc = (acc * x + int(c)) % t
    return acc


# ----------------------------------------------------------------------------- protocols

def blocks(m, n):
    return (m + n - 1) // n


def gallery_plaintexts(params, P, b):
    """Plaintexts of gallery block b: list over dims i of coefficient lists (Eq. 3)."""
    n = params.n
    P = np.asarray(P, dtype=np.int64)
    d, m = P.shape
    z = np.zeros((d, n), dtype=np.int64)
    lo, hi = b * n, min(m, (b + 1) * n)
    z[:, : hi - lo] = P[:, lo:hi]
    return [[int(c) for c in row] for row in encode_slots(params, z)]


def probe_plaintext(params, qi):
    """Eq. 2: dimension value in every slot = the constant polynomial [q_i]_t."""
    m = [0] * params.n
    m[0] = int(qi) % params.t
    return m


def encrypt_gallery_block(params, pk, P, b, seed):
    """Alg. "HERS Enrollment" (batch form): the d ciphertexts of block b."""
    key = (seed, philox.DOMAIN_GALLERY)
    return [fv.encrypt(params, pk, m, key, (b, i)) for i, m in enumerate(gallery_plaintexts(params, P, b))]


def encrypt_gallery(params, pk, P, seed, block_ids=None):
    M = blocks(np.asarray(P).shape[1], params.n)
    ids = range(M) if block_ids is None else block_ids
    return {b: encrypt_gallery_block(params, pk, P, b, seed) for b in ids}


def enroll_append(params, pk, running, P_new, k0, seed):
    """Alg. "HERS Enrollment", online form.  `running` maps block b to its d
    ciphertexts and holds items 0 .. k0-1; P_new [d][c] are items k0 .. k0+c-1.
    The client encodes the batch at its slot offset (v = k0 mod n), split at
    block boundaries, and encrypts one ciphertext per (block, dimension) with
    randomness object (b, i) under key (seed, ENROLL); the server adds each
    into the block's running ciphertext, which for a block that held no item
    is the trivial zero ciphertext.  Returns the updated dict."""
    n = params.n
    P_new = np.asarray(P_new, dtype=np.int64)
    d, c = P_new.shape
    key = (seed, philox.DOMAIN_ENROLL)
    out = dict(running)
    for b in range(k0 // n, (k0 + c - 1) // n + 1):
        lo, hi = max(k0, b * n), min(k0 + c, (b + 1) * n)
        z = np.zeros((d, n), dtype=np.int64)
        z[:, lo - b * n: hi - b * n] = P_new[:, lo - k0: hi - k0]
        fresh = [fv.encrypt(params, pk, [int(v) for v in row], key, (b, i))
                 for i, row in enumerate(encode_slots(params, z))]
        if k0 <= b * n:
            out[b] = fresh
        else:
            out[b] = [fv.add(params, r, f) for r, f in zip(out[b], fresh)]
    return out


def encrypt_probe(params, pk, qvec, seed):
    """Alg. "HERS Search", client side: one ciphertext per dimension."""
    key = (seed, philox.DOMAIN_PROBE)
    return [fv.encrypt(params, pk, probe_plaintext(params, qi), key, (0, i)) for i, qi in enumerate(qvec)]


def encrypt_probe_sk(params, sk, qvec, seed):
    """The query encrypted with the client's secret key (Sec. 3.2, "Search
    Protocol"): dimension i is fv.encrypt_sk of [q_i]_t with randomness object
    (0, i, .) under key (seed, PROBE_SK)."""
    key = (seed, philox.DOMAIN_PROBE_SK)
    return [fv.encrypt_sk(params, sk, probe_plaintext(params, qi), key, (0, i)) for i, qi in enumerate(qvec)]


def search_block(params, rlk, probe_cts, gallery_cts):
    """Form F for one block: sum_i tensor(probe_i, gallery_i), t/q round, one relin."""
    X = fv.tensor(params, list(zip(probe_cts, gallery_cts)))
    c = tuple(fv.scale_round(params, x) for x in X)
    return fv.relinearize(params, rlk, c)


def search_block_unrelinearized(params, probe_cts, gallery_cts):
    """Form F before relinearization: the degree-2 ciphertext (c0, c1, c2)."""
    X = fv.tensor(params, list(zip(probe_cts, gallery_cts)))
    return tuple(fv.scale_round(params, x) for x in X)


def search_block_literal(params, rlk, probe_cts, gallery_cts):
    """Form L: per dimension CipherMultiply (rescale + relin), then CipherAdd,
    starting from the trivial zero ciphertext."""
    q, n = params.q, params.n
    s = ([0] * n, [0] * n)
    for a, b in zip(probe_cts, gallery_cts):
        s = fv.add(params, s, fv.multiply(params, rlk, a, b))
    return s


def decrypt_scores(params, sk, score_cts, m):
    """Alg. "HERS Search", client side: decrypt each block, decode its slots,
    centre mod t; scores for items 0..m-1 in order."""
    n, t = params.n, params.t
    out = []
    for b in sorted(score_cts):
        pt = fv.decrypt(params, sk, score_cts[b])
        z = decode_slots(params, pt)
        z = np.where(z >= (t + 1) // 2, z - t, z)
        take = min(n, m - b * n)
        out.extend(int(v) for v in z[:take])
    return np.array(out, dtype=np.int64)


def top_k(scores, k):
    """Alg. "HERS Search", client side, last step: the nearest neighbours are
    the items of highest decrypted score (the argmax for k = 1); among equal
    scores the lower item index comes first.  Returns (indices, scores) of the
    k best, best first: the definition, a sort by (-score, index)."""
    s = [int(v) for v in scores]
    order = sorted(range(len(s)), key=lambda i: (-s[i], i))[:k]
    return np.array(order, dtype=np.int64), np.array([s[i] for i in order], dtype=np.int64)


def plaintext_scores(P, qvec):
    """Eq. 1: r(P, q) = P^T q, the exact result encrypted search must reproduce."""
    return np.asarray(P, dtype=np.int64).T @ np.asarray(qvec, dtype=np.int64)
