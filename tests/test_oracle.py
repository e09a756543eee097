"""Pins of the oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: an independent library
implementation, a value the paper prints, a closed form, an algebraic identity
or brute force on tiny inputs.
"""

import json
import os
import random

import numpy as np
import pytest
from sympy import isprime

from oracle import fv, hers, philox, primes, rerank
from oracle.primes import ntt_primes, plain_modulus, psi
from oracle.ring import center, negacyclic_mul, negacyclic_mul_schoolbook, negacyclic_sum_of_products

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _paper():
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        return json.load(f)


# ----------------------------------------------------------------------------- Philox

def _numpy_block(ctr, key):
    """Philox4x64-10 block from numpy's independent implementation.  numpy
    increments its 256-bit counter before producing a block."""
    c = sum(int(x) << (64 * i) for i, x in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    cw = np.array([(c >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=cw)
    return [int(x) for x in g.random_raw(4)]


@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (0, 0, 0, 0)),
    ((1, 2), (0, 0, 0, 0)),
    ((201, 1), (3, 7, 0, 0)),
    ((2**64 - 1, 2**63), (2**64 - 1, 2**64 - 1, 5, 9)),
    ((123456789, 3), (17, 0, 127, 2)),
])
def test_philox_matches_numpy(key, ctr):
    assert list(philox.philox4x64_10(ctr, key)) == _numpy_block(ctr, key)


def test_philox_stream_addressing():
    key, obj = (5, 2), (3, 4, 1)
    w = philox.words(key, obj, 10)
    assert w[4:8] == list(philox.philox4x64_10((1, 3, 4, 1), key))
    assert w[9] == philox.philox4x64_10((2, 3, 4, 1), key)[1]


def test_samplers_ranges_and_moments():
    n = 4096
    key = (11, 1)
    s = philox.sample_binary(key, (0, 0, 0), n)
    assert set(s) <= {0, 1} and abs(sum(s) - n / 2) < 5 * (n / 4) ** 0.5
    e = np.array(philox.sample_cbd(key, (1, 0, 0), 4 * n))
    assert e.min() >= -20 and e.max() <= 20
    assert abs(e.mean()) < 0.2 and abs(e.var() - 10.0) < 0.8       # CBD(20): variance eta/2
    primes = [1032193, 0xffffee001]
    r = philox.sample_uniform_residues(key, (2, 0, 0), n, primes)
    for row, p in zip(r, primes):
        row = np.array(row, dtype=np.float64)
        assert row.min() >= 0 and row.max() < p
        assert abs(row.mean() / p - 0.5) < 0.03


def test_binary_sampler_bit_layout():
    key, obj = (9, 9), (1, 2, 3)
    w = philox.words(key, obj, 2)
    s = philox.sample_binary(key, obj, 128)
    assert s[0] == w[0] & 1 and s[63] == w[0] >> 63 and s[64] == w[1] & 1


# ----------------------------------------------------------------------------- primes

def test_paper_plain_modulus():
    """Sec. 4.1 prints t = 1,032,193 for n = 4096; the selection rule reproduces it."""
    pv = _paper()["encryption_parameters"]
    assert plain_modulus(20, 2 * pv["n"]) == pv["t"]


def test_prime_rule_is_largest():
    """Brute force: every larger candidate p = 1 mod 2n below 2^b is composite."""
    for bits, two_n in [(36, 8192), (20, 4096), (54, 4096), (44, 16384), (21, 16384)]:
        p = ntt_primes([bits], two_n)[0]
        assert isprime(p) and p % two_n == 1 and p < 2**bits
        c = p + two_n
        while c < 2**bits:
            assert not isprime(c)
            c += two_n


def test_q_primes_distinct_and_sized():
    qs = ntt_primes([36, 36, 36], 8192)
    assert len(set(qs)) == 3 and all(p.bit_length() == 36 for p in qs)
    assert qs == sorted(qs, reverse=True)
    pv = _paper()["encryption_parameters"]
    assert len(qs) == pv["q_prime_count"] and all(p.bit_length() == pv["q_prime_bits"] for p in qs)


@pytest.mark.parametrize("p,n", [(1032193, 4096), (1032193, 2048), (1785857, 8192), (0xffffee001, 4096)])
def test_psi_is_primitive_2n_root(p, n):
    r = psi(p, 2 * n)
    assert pow(r, n, p) == p - 1          # psi^n = -1: root of x^n + 1
    assert pow(r, 2 * n, p) == 1


# ----------------------------------------------------------------------------- ring

@pytest.mark.parametrize("n", [1, 2, 4, 8, 32, 64])
def test_negacyclic_mul_vs_schoolbook(n):
    rng = random.Random(n)
    for bound in [1, 63, 2**36, 2**107]:
        a = [rng.randint(-bound, bound) for _ in range(n)]
        b = [rng.randint(-bound, bound) for _ in range(n)]
        assert negacyclic_mul(a, b) == negacyclic_mul_schoolbook(a, b)


def test_negacyclic_extremes_and_x_shift():
    n, B = 16, 2**107
    a = [B] * n
    b = [-B] * n
    assert negacyclic_mul(a, b) == negacyclic_mul_schoolbook(a, b)
    # multiplying by x rotates and negates the wrapped coefficient (x^n = -1)
    x = [0, 1] + [0] * (n - 2)
    c = list(range(1, n + 1))
    assert negacyclic_mul(c, x) == [-n] + c[:-1]


def test_sum_of_products_matches_sum():
    rng = random.Random(7)
    n, B = 32, 2**60
    pairs = [([rng.randint(-B, B) for _ in range(n)], [rng.randint(-B, B) for _ in range(n)]) for _ in range(5)]
    want = [0] * n
    for a, b in pairs:
        want = [x + y for x, y in zip(want, negacyclic_mul_schoolbook(a, b))]
    assert negacyclic_sum_of_products(pairs, n, B) == want


# ----------------------------------------------------------------------------- slot encoding

def _small_params(n=64, qbits=(36, 36), t_bits=20, w_bits=0):
    return fv.Params(n=n, qbits=qbits, t_bits=t_bits, w_bits=w_bits)


def test_encode_matches_interpolation_definition():
    p = _small_params(n=128)
    rng = np.random.default_rng(3)
    z = rng.integers(-63, 64, size=p.n)
    m = hers.encode_slots(p, z[None, :])[0]
    assert [int(x) for x in m] == hers.encode_slots_direct(p, z)
    for j in [0, 1, 77, 127]:
        assert hers.evaluate_at_slot(p, m, j) == z[j] % p.t


def test_encode_decode_roundtrip_large_n():
    p = fv.Params(n=4096, qbits=(36,), t_bits=20)
    rng = np.random.default_rng(4)
    z = rng.integers(0, p.t, size=(2, p.n))
    m = hers.encode_slots(p, z)
    assert np.array_equal(hers.decode_slots(p, m), z)
    for j in [0, 2047, 4095]:
        assert hers.evaluate_at_slot(p, m[1], j) == z[1, j]


def test_constant_polynomial_fills_every_slot():
    """Eq. 2: the query's value replicated in all slots is the constant polynomial."""
    p = _small_params(n=64)
    m = hers.probe_plaintext(p, -17)
    assert np.all(hers.decode_slots(p, m) == (-17) % p.t)


def test_ring_product_is_slotwise_product():
    """CRT batching: multiplication in R_t acts slot-wise (convolution theorem)."""
    p = _small_params(n=32)
    rng = np.random.default_rng(5)
    z1, z2 = rng.integers(0, p.t, size=(2, p.n))
    m1 = [int(x) for x in hers.encode_slots(p, z1[None])[0]]
    m2 = [int(x) for x in hers.encode_slots(p, z2[None])[0]]
    prod = [c % p.t for c in negacyclic_mul_schoolbook(m1, m2)]
    assert np.array_equal(hers.decode_slots(p, prod), (z1 * z2) % p.t)


# ----------------------------------------------------------------------------- FV identities

@pytest.fixture(scope="module")
def toy():
    p = fv.Params(n=256, qbits=(36, 36, 36), t_bits=20, w_bits=0)
    sk, pk, rlk = fv.keygen(p, 77)
    return p, sk, pk, rlk


def test_public_key_relation(toy):
    """pk0 + pk1 s = -e with |e| <= eta (Alg. "Key Generation")."""
    p, sk, pk, _ = toy
    v = fv.poly_add(pk[0], fv.poly_mul_q(pk[1], sk, p.q), p.q)
    assert max(abs(center(x, p.q)) for x in v) <= p.eta


def test_relin_key_relation(toy):
    """rlk_g0 + rlk_g1 s = g s^2 - e_g with |e_g| <= eta."""
    p, sk, _, rlk = toy
    s2 = fv.poly_mul_q(sk, sk, p.q)
    for (rho, l, g), (b, a) in zip(p.gadget(), rlk):
        v = fv.poly_add(b, fv.poly_mul_q(a, sk, p.q), p.q)
        v = [(x - g * y) % p.q for x, y in zip(v, s2)]
        assert max(abs(center(x, p.q)) for x in v) <= p.eta


@pytest.mark.parametrize("w_bits", [0, 12])
def test_gadget_identity(w_bits):
    """sum_g y_g * g = c2 (mod q) for the digits of any c2."""
    p = fv.Params(n=8, qbits=(36, 30), t_bits=12, w_bits=w_bits)
    rng = random.Random(w_bits)
    c2 = [rng.randrange(p.q) for _ in range(p.n)] + []
    c2[0], c2[1] = 0, p.q - 1
    digits = fv.relin_digits(p, c2)
    gad = p.gadget()
    assert len(digits) == len(gad)
    for j in range(p.n):
        assert sum(d[j] * g for d, (_, _, g) in zip(digits, gad)) % p.q == c2[j]
        if w_bits:
            assert all(d[j] < 2**w_bits for d in digits)


def test_encrypt_decrypt_and_add(toy):
    p, sk, pk, _ = toy
    rng = np.random.default_rng(6)
    z1, z2 = rng.integers(-500, 500, size=(2, p.n))
    m1 = [int(x) for x in hers.encode_slots(p, z1[None])[0]]
    m2 = [int(x) for x in hers.encode_slots(p, z2[None])[0]]
    c1 = fv.encrypt(p, pk, m1, (1, 2), (0, 0))
    c2 = fv.encrypt(p, pk, m2, (1, 2), (0, 1))
    assert fv.decrypt(p, sk, c1) == m1
    s = fv.add(p, c1, c2)
    assert np.array_equal(hers.decode_slots(p, fv.decrypt(p, sk, s)), (z1 + z2) % p.t)
    # fresh noise: |e1 + pk0 u ... | bounded by eta (1 + n) for binary u, s
    assert fv.noise(p, sk, c1, m1) <= p.eta * (2 * p.n + 1)


def test_secret_key_encryption(toy):
    """ct = (Delta m - a s + e, a): ct0 + ct1 s - Delta m is exactly the error e
    (|e| <= eta, where a dropped or mis-signed a s term would leave a value
    of the size of q), it decrypts to m and adds like a public-key ciphertext."""
    p, sk, pk, _ = toy
    rng = np.random.default_rng(9)
    z = rng.integers(-500, 500, size=p.n)
    m = [int(x) for x in hers.encode_slots(p, z[None])[0]]
    key = (5, philox.DOMAIN_PROBE_SK)
    c = fv.encrypt_sk(p, sk, m, key, (0, 3))
    assert c[1] == fv.sample_uniform_q(p, key, (0, 3, 0))
    e = philox.sample_cbd(key, (0, 3, 1), p.n, p.eta)
    x = fv.poly_add(c[0], fv.poly_mul_q(c[1], sk, p.q), p.q)
    assert [fv.center(v - p.delta * mi, p.q) for v, mi in zip(x, m)] == e
    assert fv.noise(p, sk, c, m) <= p.eta
    assert fv.decrypt(p, sk, c) == m
    c2 = fv.encrypt(p, pk, m, (1, 2), (0, 0))
    assert np.array_equal(hers.decode_slots(p, fv.decrypt(p, sk, fv.add(p, c, c2))), (2 * z) % p.t)


def test_search_with_secret_key_probe_decrypts_to_inner_products(toy):
    """The query encrypted under the secret key (Sec. 3.2, "Search
    Protocol"), searched against public-key gallery ciphertexts: the decrypted
    scores are P^T q (Eq. 1)."""
    p, sk, pk, rlk = toy
    rng = np.random.default_rng(10)
    d, m = 3, p.n + 5
    P = rng.integers(-63, 64, size=(d, m))
    qv = rng.integers(-63, 64, size=d)
    probe = hers.encrypt_probe_sk(p, sk, qv, 11)
    S = {b: hers.search_block(p, rlk, probe, hers.encrypt_gallery_block(p, pk, P, b, 12)) for b in range(2)}
    assert np.array_equal(hers.decrypt_scores(p, sk, S, m), hers.plaintext_scores(P, qv))


def test_multiply_relin_is_slotwise_product(toy):
    p, sk, pk, rlk = toy
    rng = np.random.default_rng(8)
    z1, z2 = rng.integers(-63, 64, size=(2, p.n))
    m1 = [int(x) for x in hers.encode_slots(p, z1[None])[0]]
    m2 = [int(x) for x in hers.encode_slots(p, z2[None])[0]]
    c1 = fv.encrypt(p, pk, m1, (3, 2), (0, 0))
    c2 = fv.encrypt(p, pk, m2, (3, 2), (0, 1))
    X = fv.tensor(p, [(c1, c2)])
    deg2 = tuple(fv.scale_round(p, x) for x in X)
    assert np.array_equal(hers.decode_slots(p, fv.decrypt(p, sk, deg2)), (z1 * z2) % p.t)
    prod = fv.multiply(p, rlk, c1, c2)
    assert np.array_equal(hers.decode_slots(p, fv.decrypt(p, sk, prod)), (z1 * z2) % p.t)


def test_scale_round_brute_force():
    """round(t X / q) against exact rational rounding, on values next to the
    rounding boundaries (t X = (q +- 1)/2 mod q) and at the range ends."""
    from fractions import Fraction
    p = fv.Params(n=8, qbits=(36, 36), t_bits=20)
    q, t = p.q, p.t
    tinv = pow(t, -1, q)
    xs = [0, 1, -1, q // 2, -(q // 2), 3 * q, -5 * q + 7]
    for r in [(q - 1) // 2, (q + 1) // 2, 1, q - 1]:
        base = (r * tinv) % q               # t * base = r (mod q)
        xs += [base, base - q, base + 11 * q, base - 1000 * q]
    got = fv.scale_round(p, xs)
    for x, g in zip(xs, got):
        f = Fraction(t * x, q)
        fl = f.numerator // f.denominator
        want = fl + (1 if f - fl > Fraction(1, 2) else 0)
        assert f - fl != Fraction(1, 2)     # q odd: no ties
        assert g == want % q


# ----------------------------------------------------------------------------- HERS search

def _features(rng, d, m):
    return rng.integers(-63, 64, size=(d, m)), rng.integers(-63, 64, size=d)


def test_search_scores_equal_plaintext_inner_products():
    """Eq. 1 and Eq. 4: decrypted encrypted scores are exactly P^T q; ragged last block."""
    p = fv.Params(n=256, qbits=(36, 36, 36), t_bits=20)
    sk, pk, rlk = fv.keygen(p, 5)
    rng = np.random.default_rng(9)
    d, m = 6, 2 * 256 + 37
    P, qv = _features(rng, d, m)
    G = hers.encrypt_gallery(p, pk, P, 31)
    Q = hers.encrypt_probe(p, pk, qv, 41)
    S = {b: hers.search_block(p, rlk, Q, G[b]) for b in G}
    assert np.array_equal(hers.decrypt_scores(p, sk, S, m), hers.plaintext_scores(P, qv))


def test_fused_and_literal_forms_decrypt_alike():
    """Form F (sum, one rescale, one relin) and form L (Alg. "HERS Search" per
    dimension) differ in ciphertext bits but not in decrypted scores."""
    p = fv.Params(n=128, qbits=(36, 36, 36), t_bits=20)
    sk, pk, rlk = fv.keygen(p, 6)
    rng = np.random.default_rng(10)
    d, m = 4, 100
    P, qv = _features(rng, d, m)
    G = hers.encrypt_gallery(p, pk, P, 32)
    Q = hers.encrypt_probe(p, pk, qv, 42)
    F = {0: hers.search_block(p, rlk, Q, G[0])}
    L = {0: hers.search_block_literal(p, rlk, Q, G[0])}
    assert F[0] != L[0]
    want = hers.plaintext_scores(P, qv)
    assert np.array_equal(hers.decrypt_scores(p, sk, F, m), want)
    assert np.array_equal(hers.decrypt_scores(p, sk, L, m), want)


def test_online_enrollment_fills_slots_at_offsets():
    """Alg. "HERS Enrollment", online form: after batches that start mid-block
    and straddle block boundaries, every block decrypts to the enrolled items
    in their slots (item b*n + j in slot j) and zero in empty slots, and the
    search over the appended gallery decrypts to P^T q."""
    p = fv.Params(n=64, qbits=(36, 36, 36), t_bits=20)
    sk, pk, rlk = fv.keygen(p, 8)
    rng = np.random.default_rng(12)
    d, n = 3, 64
    sizes = [5, 1, 70, 52, 64, 3]        # mid-block start, straddles, exact fill, new block
    P, qv = _features(rng, d, sum(sizes))
    run, k0 = {}, 0
    for j, c in enumerate(sizes):
        run = hers.enroll_append(p, pk, run, P[:, k0:k0 + c], k0, 700 + j)
        k0 += c
        for b, cts in run.items():
            for i, ct in enumerate(cts):
                z = hers.decode_slots(p, fv.decrypt(p, sk, ct))
                z = np.where(z >= (p.t + 1) // 2, z - p.t, z)
                lo, hi = b * n, min(k0, (b + 1) * n)
                want = np.zeros(n, dtype=np.int64)
                want[: hi - lo] = P[i, lo:hi]
                assert np.array_equal(z, want), (j, b, i)
    assert sorted(run) == list(range(hers.blocks(k0, n)))
    Q = hers.encrypt_probe(p, pk, qv, 43)
    S = {b: hers.search_block(p, rlk, Q, run[b]) for b in run}
    assert np.array_equal(hers.decrypt_scores(p, sk, S, k0), hers.plaintext_scores(P, qv))


def test_online_enrollment_adds_fresh_encryptions():
    """The server half is CipherAdd: a block filled by two batches holds the
    sum of the two fresh encryptions, which differ from the batch-form
    gallery encryption (another randomness domain)."""
    p = fv.Params(n=32, qbits=(36, 36), t_bits=20)
    sk, pk, rlk = fv.keygen(p, 9)
    rng = np.random.default_rng(13)
    P, _ = _features(rng, 2, 32)
    one = hers.enroll_append(p, pk, {}, P[:, :10], 0, 1)
    two = hers.enroll_append(p, pk, one, P[:, 10:], 10, 2)
    alone = hers.enroll_append(p, pk, {}, np.concatenate([np.zeros((2, 10), np.int64), P[:, 10:]], 1), 0, 2)
    for i in range(2):
        assert two[0][i] == fv.add(p, one[0][i], alone[0][i])
    assert two[0][0] != hers.encrypt_gallery_block(p, pk, P, 0, 2)[0]


def _horner_at(poly, x, t):
    acc = 0
    for c in reversed(list(poly)):
        acc = (acc * x + int(c)) % t
    return acc


def test_automorphism_moves_slot_positions():
    """m(x) -> m(x^g) evaluated at psi^(2j+1) is m at psi^(g(2j+1)) (checked by
    Horner on both sides), so g = 5^s moves position p + s to position p in
    both rows of the slot layout."""
    p = fv.Params(n=64, qbits=(36,), t_bits=20)
    n, t = p.n, p.t
    rng = np.random.default_rng(21)
    z = rng.integers(0, t, size=n)
    m = [int(v) for v in hers.encode_slots(p, z)]
    root = primes.psi(t, 2 * n)
    for s in (1, 2, 5, 31):
        g = rerank.galois_element(n, s)
        mg = rerank.automorphism(m, g, t)
        for j in range(n):
            assert _horner_at(mg, pow(root, 2 * j + 1, t), t) == _horner_at(m, pow(root, g * (2 * j + 1), t), t)
        zg = hers.decode_slots(p, mg)
        for r in (0, 1):
            for pos in range(n // 2):
                src = rerank.slot_of_position(n, r, (pos + s) % (n // 2))
                assert zg[rerank.slot_of_position(n, r, pos)] == z[src]
    # the positions of both rows cover every slot once
    slots = {rerank.slot_of_position(n, r, pos) for r in (0, 1) for pos in range(n // 2)}
    assert slots == set(range(n))


def test_rotation_decrypts_to_automorphism():
    """Key switching with a rotation key: Dec(rotate(Enc(m))) = m(x^g) mod t."""
    p = fv.Params(n=64, qbits=(36, 36, 36), t_bits=20)
    sk, pk, rlk = fv.keygen(p, 22)
    keys = rerank.rotation_keygen(p, 22, 8)
    rng = np.random.default_rng(23)
    m = [int(v) for v in rng.integers(0, p.t, size=p.n)]
    ct = fv.encrypt(p, pk, m, (5, philox.DOMAIN_PROBE), (0, 0))
    for key, s in zip(keys, rerank.steps(8)):
        g = rerank.galois_element(p.n, s)
        assert fv.decrypt(p, sk, rerank.rotate(p, key, ct, g)) == rerank.automorphism(m, g, p.t)


def test_rerank_scores_equal_inner_products():
    """Packed 1:1 re-ranking: every item's score is its inner product with the
    probe (Eq. 1 restricted to the item); segments past the last item are 0."""
    p = fv.Params(n=128, qbits=(36, 36, 36), t_bits=20)
    sk, pk, rlk = fv.keygen(p, 24)
    W, D = 16, 12
    keys = rerank.rotation_keygen(p, 24, W)
    rng = np.random.default_rng(25)
    S = rerank.segments_per_ct(p.n, W)
    count = 2 * S + 3
    F, qv = rng.integers(-63, 64, size=(D, count)), rng.integers(-63, 64, size=D)
    items = rerank.encrypt_items(p, pk, F, W, 26)
    probe = rerank.encrypt_probe(p, pk, qv, W, 27)
    want = F.T.astype(np.int64) @ qv.astype(np.int64)
    for c, item in enumerate(items):
        got = rerank.decrypt_scores(p, sk, rerank.rerank_ct(p, rlk, keys, probe, item, W), W)
        lo, hi = c * S, min(count, (c + 1) * S)
        assert np.array_equal(got[: hi - lo], want[lo:hi]) and not got[hi - lo:].any(), c


def test_search_with_digit_split_gadget():
    p = fv.Params(n=128, qbits=(54, 54), t_bits=20, w_bits=18)
    sk, pk, rlk = fv.keygen(p, 7)
    assert len(rlk) == 6
    rng = np.random.default_rng(11)
    d, m = 5, 128
    P, qv = _features(rng, d, m)
    G = hers.encrypt_gallery(p, pk, P, 33)
    Q = hers.encrypt_probe(p, pk, qv, 43)
    S = {0: hers.search_block(p, rlk, Q, G[0])}
    assert np.array_equal(hers.decrypt_scores(p, sk, S, m), hers.plaintext_scores(P, qv))


def test_single_prime_toy_config_exceeds_noise_budget():
    """With q one 54-bit prime (n = 2048, t ~ 2^20) the product noise exceeds
    Delta/2 = 2^33: ciphertexts are still defined, decryption of the scores is not."""
    p = fv.Params(n=2048, qbits=(54,), t_bits=20, w_bits=18)
    assert (p.delta // 2).bit_length() == 34
    sk, pk, rlk = fv.keygen(p, 201)
    rng = np.random.default_rng(101)
    P, qv = _features(rng, 4, 2048)
    G = hers.encrypt_gallery(p, pk, P, 301)
    Q = hers.encrypt_probe(p, pk, qv, 401)
    c = hers.search_block_unrelinearized(p, Q, G[0])
    want = [int(x) for x in hers.encode_slots(p, hers.plaintext_scores(P, qv)[None, :])[0]]
    assert fv.noise(p, sk, c, want) > p.delta // 2


def test_top_k_definition():
    """The client's last step (Alg. "HERS Search"): argmax, and the k best with
    ties broken by lower index, on a hand-checked example and against a
    brute-force maximum removal."""
    idx, val = hers.top_k([3, 5, -2, 5, 1, 5], 4)
    assert idx.tolist() == [1, 3, 5, 0] and val.tolist() == [5, 5, 5, 3]
    rng = np.random.default_rng(13)
    s = rng.integers(-4, 5, size=200)
    left, want = list(range(200)), []
    for _ in range(50):                             # repeatedly take the first maximal item
        best = max(left, key=lambda i: (s[i], -i))
        want.append(best)
        left.remove(best)
    assert hers.top_k(s, 50)[0].tolist() == want
    assert hers.top_k(s, 1)[0][0] == int(np.argmax(s))


def test_table2_operation_counts(toy, monkeypatch):
    """Table 2, HERS row: ceil(m/n) d ciphertext multiplications, ceil(m/n)(d-1)
    additions and no rotations.  Counted on the oracle's paper-literal search
    (Alg. "HERS Search" as printed: per block, multiply each dimension's
    ciphertexts and add the product into the running score; the first product
    lands on the zero accumulator, so a block takes d - 1 additions)."""
    case = _paper()["table2_hers_counts"]
    assert case["rotations"] == 0
    p, sk, pk, rlk = toy
    d, m = 3, 2 * p.n + 3
    rng = np.random.default_rng(12)
    P = rng.integers(-63, 64, size=(d, m))
    qv = rng.integers(-63, 64, size=d)
    probe = hers.encrypt_probe(p, pk, qv, 13)
    gallery = hers.encrypt_gallery(p, pk, P, 14)
    counts = {"mul": 0, "add": 0}
    mul, add = fv.multiply, fv.add

    def counting_mul(*a):
        counts["mul"] += 1
        return mul(*a)

    def counting_add(params, x, y):
        if any(any(c) for c in x):                  # not the zero accumulator
            counts["add"] += 1
        return add(params, x, y)

    monkeypatch.setattr(fv, "multiply", counting_mul)
    monkeypatch.setattr(fv, "add", counting_add)
    S = {b: hers.search_block_literal(p, rlk, probe, gallery[b]) for b in gallery}
    M = -(-m // p.n)
    assert len(gallery) == M and counts["mul"] == M * d and counts["add"] == M * (d - 1)
    monkeypatch.undo()
    assert np.array_equal(hers.decrypt_scores(p, sk, S, m), hers.plaintext_scores(P, qv))