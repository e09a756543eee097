"""Host-side checks of libhers: it loads, exports the C ABI, and resolves
parameters exactly as the oracle's prime rule does (no GPU needed)."""

import ctypes
import json
import math
import os
import re

import pytest

from oracle import fv
from oracle.primes import ntt_primes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hers.h")


def _lib():
    from paper_2003_12197_amd import hers_gpu
    return hers_gpu


def _declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(hers_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    hg = _lib()
    lib = ctypes.CDLL(hg.LIB_PATH)
    syms = _declared_symbols()
    assert len(syms) >= 19
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(hg.EXPORTS), "binding and header disagree"


@pytest.mark.parametrize("n,qbits,t_bits,w_bits,d_max", [
    (2048, (54,), 20, 18, 16),
    (2048, (54, 54), 20, 0, 16),
    (4096, (36, 36, 36), 20, 0, 64),
    (4096, (36, 36, 36), 20, 0, 128),
    (8192, (44, 44, 44, 43, 43), 21, 0, 128),
])
def test_resolve_matches_oracle_prime_rule(n, qbits, t_bits, w_bits, d_max):
    info = _lib().resolve(n, qbits, t_bits, w_bits, d_max)
    op = fv.Params(n=n, qbits=qbits, t_bits=t_bits, w_bits=w_bits)
    assert [info.q[i] for i in range(info.k)] == op.q_primes
    assert info.t == op.t
    assert info.num_digits == len(op.gadget())
    # exact-product base: distinct primes < 2^30, 1 mod 2n, product > 4 * 2 d n ((q-1)/2)^2
    aux = [info.aux[i] for i in range(info.num_aux)]
    assert len(set(aux)) == len(aux) and not set(aux) & set(op.q_primes + [op.t])
    assert all(p < 2**30 and p % (2 * n) == 1 for p in aux)
    assert aux == ntt_primes([30] * len(aux), 2 * n, exclude=op.q_primes + [op.t])
    P = math.prod(aux)
    xmax = 2 * d_max * n * ((op.q - 1) // 2) ** 2
    assert P > 4 * xmax
    # minimal: one prime fewer would not do (with the one bit of slack the rule keeps)
    assert math.prod(aux[:-1]) < 8 * xmax


def test_resolve_rejects_bad_parameters():
    hg = _lib()
    with pytest.raises(hg.HersError):
        hg.resolve(3000, (36,), 20)                # not a power of two
    with pytest.raises(hg.HersError):
        hg.resolve(4096, (36,), 20, d_max=200)     # 200 * 63^2 >= t/2: scores would wrap mod t


def test_table3_memory_matches_canonical_layout():
    """Table 3: 100M-item gallery memory.  One canonical ciphertext per (block,
    dimension) of 2 polynomials x 3 residues x n coefficients in 8-byte words
    gives 143/286/572/2289 GiB against the paper's 140/280/550/2200 GB."""
    pv = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))["table3_memory_gb"]
    info = _lib().resolve(4096, (36, 36, 36), 20, 0, 32)
    M = (pv["m"] + info.n - 1) // info.n
    for d, gb in zip(pv["dims"], pv["memory_gb"]):
        gib = M * d * 2 * info.k * info.n * 8 / 2**30
        assert abs(gib - gb) / gb < 0.05
