"""GPU: the exact rescale on accumulators next to a half-integer.

The rescale (Alg. "Ciphertext Multiplication": c = [round(t X / q)]_q) first
rounds from the top two 64-bit words of the fixed-point fraction and takes all
words only when that fraction is within 2^-64 of one half.  Random inputs
essentially never get there, so these accumulators are built to: with
t X = (q +- 1)/2 (mod q), t X / q lies 1/(2q) from a half-integer, and 1/(2q)
is below the two-word sum's own error bound, so the two words alone cannot
decide.  Expected values come from the oracle's scale_round on the same X.
Integer work: tolerance 0.
"""

import numpy as np
import pytest
import torch

from oracle import fv

pytestmark = pytest.mark.gpu

CONFIGS = {
    # three 36-bit primes (three fraction words) and five 44/43-bit primes (four)
    "r36": dict(n=2048, qbits=(36, 36, 36), t_bits=20, w_bits=0),
    "c3s": dict(n=256, qbits=(44, 44, 44, 43, 43), t_bits=21, w_bits=0),
}


def half_way_accumulators(q, t):
    """Integers X with t X / q within 1/(2q) of a half-integer, of both signs
    and magnitudes up to a few q, plus two plain ones."""
    tinv = pow(t, -1, q)
    lo = ((q - 1) // 2 * tinv) % q         # t X = (q - 1)/2 (mod q): just below m + 1/2
    hi = ((q + 1) // 2 * tinv) % q         # t X = (q + 1)/2 (mod q): just above m + 1/2
    return [lo, hi, lo - q, hi - q, lo + 3 * q, hi - 5 * q, -lo, -hi, 0, tinv]


@pytest.mark.parametrize("cfg", sorted(CONFIGS))
def test_rescale_next_to_half_integer(gpu_lib, cfg):
    c = CONFIGS[cfg]
    op = fv.Params(**c)
    ctx = gpu_lib.Context(d_max=16, **c)
    assert ctx.q == op.q_primes and ctx.t == op.t
    ctx.keygen(201)
    n, K, k = ctx.n, ctx.K, ctx.k
    aux = [ctx.info.aux[r] for r in range(K)]
    P = 1
    for p in aux:
        P *= p
    Xs = half_way_accumulators(op.q, op.t)
    assert all(4 * abs(X) < P for X in Xs)
    M = len(Xs)
    m = M * n
    print("case %s: n=%d k=%d K=%d blocks=%d" % (cfg, n, k, K, M), flush=True)
    # d = 1.  Gallery block b: first polynomial the constant X_b, second 0; probe (1, 0).
    # A constant polynomial's transform is that constant in every slot, so the
    # search-form rows are X_b mod p_r throughout, and the tensor is (X_b, 0, 0).
    gal = np.zeros((M, K, 1, 2, n), dtype=np.uint32)
    for b, X in enumerate(Xs):
        for r, p in enumerate(aux):
            gal[b, r, 0, 0, :] = X % p
    prb = np.zeros((K, 1, 2, n), dtype=np.uint32)
    prb[:, 0, 0, :] = 1
    dev = ctx.device
    gallery = torch.from_numpy(gal.reshape(-1).view(np.int32)).to(dev)
    probe = torch.from_numpy(prb.reshape(-1).view(np.int32)).to(dev)
    assert gallery.numel() == ctx.lib.hers_gallery_words(ctx.handle, m, 1)
    assert probe.numel() == ctx.lib.hers_probe_words(ctx.handle, 1)
    for call in range(2):
        scores = ctx.search(gallery, m, 1, probe)
        torch.cuda.synchronize()
        got = scores.cpu().numpy()                          # [M][2][k][n]
        assert got.shape == (M, 2, k, n)
        for b, X in enumerate(Xs):
            c0 = fv.scale_round(op, [X])[0]
            want = np.zeros((2, k, n), dtype=np.int64)
            want[0, :, 0] = [c0 % qi for qi in op.q_primes]
            assert np.array_equal(got[b], want), (cfg, call, b, X)
