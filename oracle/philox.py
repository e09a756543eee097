"""Philox4x64-10 counter-based generator and the samplers drawn from it.

Test infrastructure (oracle).  The HERS paper samples keys, encryption
randomness and errors (App. A, Alg. "Key Generation" and Alg. "Encryption":
uniform elements of R_q, elements of R_2 and draws from the error
distribution chi) but does not fix a generator.  To make ciphertexts
reproducible, both this oracle and the GPU library draw every random word from
Philox4x64-10 as published by Salmon, Moraes, Dror and Shaw ("Parallel random
numbers: as easy as 1, 2, 3", SC'11): a 4x64-bit counter block, a 2x64-bit
key, ten rounds of two 64x64->128 multiplies with the round key bumped by the
Weyl constants between rounds.

Word addressing (shared convention, written independently on both sides):
    word(key, obj, w) = Philox(key, counter=(w // 4, obj[0], obj[1], obj[2]))[w % 4]
where key = (seed, domain) and obj is a 3-word object id.

Samplers (readings of the paper's R_2, chi and "uniform in R_q"):
  binary      coefficient j = bit (j mod 64) of word j // 64              (R_2 = {0,1})
  cbd         coefficient j = popcount(w_j & M20) - popcount((w_j >> 20) & M20),
              M20 = 2^20 - 1: centred binomial with eta = 20, sigma = sqrt(10)
  uniform     residue rho of coefficient j = (w_{2(rho n + j)} + 2^64 w_{2(rho n + j)+1}) mod q_rho;
              independent uniform residues are a uniform element of Z_q by the CRT.
"""

MASK64 = (1 << 64) - 1
# Round multipliers and Weyl key increments of Philox4x64 (Salmon et al. 2011).
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B

# Domains separate the independent uses of one seed.
DOMAIN_KEYGEN = 1
DOMAIN_GALLERY = 2
DOMAIN_PROBE = 3
DOMAIN_ENROLL = 4
DOMAIN_RERANK_ITEMS = 5
DOMAIN_RERANK_PROBE = 6
DOMAIN_PROBE_SK = 7


def philox4x64_10(ctr, key):
    """One Philox4x64-10 block: 4 output words for counter `ctr` under `key`."""
    c0, c1, c2, c3 = (int(x) & MASK64 for x in ctr)
    k0, k1 = (int(x) & MASK64 for x in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return (c0, c1, c2, c3)


def words(key, obj, count):
    """The first `count` 64-bit words of the stream of object `obj` under `key`."""
    out = []
    nblk = (count + 3) // 4
    for blk in range(nblk):
        out.extend(philox4x64_10((blk, obj[0], obj[1], obj[2]), key))
    return out[:count]


def sample_binary(key, obj, n):
    """Element of R_2: n coefficients in {0, 1}."""
    w = words(key, obj, (n + 63) // 64)
    return [(w[j // 64] >> (j % 64)) & 1 for j in range(n)]


def sample_cbd(key, obj, n, eta=20):
    """Error polynomial: centred binomial, coefficients in [-eta, eta]."""
    m = (1 << eta) - 1
    w = words(key, obj, n)
    return [bin(x & m).count("1") - bin((x >> eta) & m).count("1") for x in w]


def sample_uniform_residues(key, obj, n, q_primes):
    """Uniform element of R_q as residues: res[rho][j] in [0, q_rho)."""
    k = len(q_primes)
    w = words(key, obj, 2 * k * n)
    res = []
    for rho, p in enumerate(q_primes):
        row = []
        for j in range(n):
            lo = w[2 * (rho * n + j)]
            hi = w[2 * (rho * n + j) + 1]
            row.append((lo + (hi << 64)) % p)
        res.append(row)
    return res
