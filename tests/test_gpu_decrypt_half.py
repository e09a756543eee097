"""GPU: score decoding on ciphertexts whose t x / q lies next to a half-integer.

Decryption (Alg. "Decryption": [round(t/q [c0 + c1 s]_q)]_t, then the slot
decode) first rounds a 64-bit fixed-point sum of the fractions t / q_i and
takes the exact CRT form only when that sum is within sum_i q_i 2^-64 of a
carry.  A valid ciphertext never gets there (t x / q sits near an integer), so
these score ciphertexts are built to: c1 = 0 and c0 = x with t x / q just
below and just above a half-integer, beside integers, and at random, one value
per coefficient.  The decoded slots equal the oracle's decryption of the same
ciphertexts, from the one-kernel decryption (n = 4096, three primes) and the
two-kernel one.  Integer work: tolerance 0.
"""

import random

import numpy as np
import pytest
import torch

from oracle import fv, hers

pytestmark = pytest.mark.gpu

CONFIGS = {
    "c5": dict(n=4096, qbits=(36, 36, 36), t_bits=20, w_bits=0),
    "c3s": dict(n=256, qbits=(44, 44, 44, 43, 43), t_bits=21, w_bits=0),
}


def coefficients(q, t, n, seed):
    """n values x in [0, q): next to the half-integer points of t x / q (both
    sides), next to integer points, the middle of [0, q), and random."""
    rng = random.Random(seed)
    xs = [q // 2, (q + 1) // 2, 0, q - 1]
    while len(xs) < n:
        j = rng.randrange(t)
        c = (2 * j + 1) * q // (2 * t)                 # t c / q just below j + 1/2
        kind = rng.randrange(4)
        if kind == 0:
            xs += [c, c + 1]
        elif kind == 1:
            xs += [(j * q // t + rng.randrange(-3, 4)) % q]
        else:
            xs += [rng.randrange(q)]
    return xs[:n]


@pytest.mark.parametrize("cfg", sorted(CONFIGS))
def test_decoding_next_to_half_integer(gpu_lib, cfg):
    c = CONFIGS[cfg]
    op = fv.Params(**c)
    ctx = gpu_lib.Context(d_max=16, **c)
    assert ctx.q == op.q_primes and ctx.t == op.t
    sk, _, _ = ctx.keygen(301)
    osk, _, _ = fv.keygen(op, 301)
    n, k = ctx.n, ctx.k
    print("case %s: n=%d k=%d, two blocks" % (cfg, n, k), flush=True)
    blocks = {b: (coefficients(op.q, op.t, n, 40 + b), [0] * n) for b in range(2)}
    sc = np.zeros((2, 2, k, n), dtype=np.int64)
    for b, (c0, _) in blocks.items():
        sc[b, 0] = np.array(fv.to_residues(c0, op.q_primes), dtype=np.int64)
    try:
        for m in (2 * n - 7, 1):                       # a ragged second block; a single item
            want = hers.decrypt_scores(op, osk, {b: blocks[b] for b in range(ctx.blocks(m))}, m)
            for fused in (1, 0):                       # one kernel per block (where it fits), then two
                ctx.set_option("dec_fused", fused)
                got = ctx.decrypt_scores(sk, torch.from_numpy(sc).to(ctx.device), m).cpu().numpy()
                assert np.array_equal(got, want), (m, fused)
                # the loaded-key form too
                ctx.load_secret_key(sk)
                got = ctx.decrypt_scores(None, torch.from_numpy(sc).to(ctx.device), m).cpu().numpy()
                assert np.array_equal(got, want), (m, fused)
    finally:
        ctx.set_option("dec_fused", 1)
