"""GPU parity at the largest single-GPU configuration, at full size and in
the launch configuration the benchmark times: 10^8 items x d = 32, n = 4096,
q = 3 x 36-bit primes, t = 1,032,193 (24,415 blocks, the last holding 256
items).

App. B Alg. "HERS Enrollment" and "HERS Search" with App. A Alg.
"Ciphertext Multiplication" and "Decryption": the gallery is enrolled on the
GPU in chunks, searched as 64 overlapped chunks with one multiply-accumulate
workgroup per CU (schedule 8, the autotuner's choice at this size), with the
two-kernel and the fused relinearization (the same score ciphertexts), and
decrypted in one kernel per block.  Every decrypted score equals P^T q; the
ragged last block's score ciphertexts equal the oracle's residue by residue.
Integer work: tolerance 0."""

import numpy as np
import pytest
import torch

from oracle import fv, hers, philox
from paper_2003_12197_amd import synth

pytestmark = pytest.mark.gpu

CFG = dict(n=4096, qbits=(36, 36, 36), t_bits=20, w_bits=0)
D, M_ITEMS = 32, 100_000_000
FEATURE_SEED, QUERY_SEED, KEY_SEED, GAL_SEED, PROBE_SEED = 1000, 2000, 201, 301, 401


def res(poly, primes):
    return np.array(fv.to_residues(poly, primes), dtype=np.int64)


@pytest.mark.timeout(900)
def test_largest_configuration_full_size(gpu_lib):
    n = CFG["n"]
    print("case c5 full: n=4096 q=3x36 d=32 m=10^8", flush=True)
    ctx = gpu_lib.Context(d_max=D, **CFG)
    dev = ctx.device
    sk, _, _ = ctx.keygen(KEY_SEED)
    M = ctx.blocks(M_ITEMS)
    qv, mate = synth.probe_for(QUERY_SEED, FEATURE_SEED, n, D, M_ITEMS)
    gal = ctx.new_gallery(M_ITEMS, D)
    want = np.empty(M_ITEMS, dtype=np.int64)
    chunk = 2048
    ws = ctx.workspace(gpu_lib.OP_ENCRYPT_GALLERY, chunk * n, D)
    for b0 in range(0, M, chunk):
        nb = min(chunk, M - b0)
        P = synth.gallery_features(FEATURE_SEED, n, D, M_ITEMS, block0=b0, nblocks=nb)
        hi = min(M_ITEMS, (b0 + nb) * n)
        want[b0 * n:hi] = P.T[:hi - b0 * n].astype(np.int64) @ qv.astype(np.int64)
        ctx.encrypt_gallery(torch.from_numpy(P).to(dev), M_ITEMS, GAL_SEED, block0=b0, nblocks=nb, gallery=gal,
                            workspace=ws)
        if b0 // chunk % 4 == 3:
            print("  enrolled %d / %d blocks" % (b0 + nb, M), flush=True)
    del ws
    pr = ctx.encrypt_probe(qv, PROBE_SEED)
    scores = []
    try:
        ctx.set_option("mac_variant", 8)
        ctx.set_option("overlap_chunks", 64)
        ctx.set_option("mac_wgs_per_cu", 1)
        wss = ctx.workspace(gpu_lib.OP_SEARCH, 8192 * n, D)
        for fuse in (1 << 30, 1):                       # two-kernel, then fused relinearization
            ctx.set_option("relin_fuse_min_wgs", fuse)
            scores.append(ctx.search(gal, M_ITEMS, D, pr, workspace=wss))
            torch.cuda.synchronize()
        print("case c5 full: searched", flush=True)
    finally:
        ctx.set_option("relin_fuse_min_wgs", 0)
        ctx.set_option("overlap_chunks", 0)
        ctx.set_option("mac_wgs_per_cu", 0)
    assert torch.equal(scores[0], scores[1])
    del scores[1]
    del gal
    out = ctx.decrypt_scores(sk, scores[0], M_ITEMS).cpu().numpy()
    assert np.array_equal(out, want)
    assert out[mate] == out.max()
    # the ragged last block against the oracle
    op = fv.Params(**CFG)
    b = M - 1
    osk, opk, orlk = fv.keygen(op, KEY_SEED)
    assert sk.cpu().numpy().tolist() == osk
    # hers.encrypt_gallery_block(op, opk, P, b, GAL_SEED) for block b, from that block's features alone
    # (the whole P would not fit in host memory as the oracle's int64 copy)
    pts = hers.gallery_plaintexts(op, synth.gallery_block(FEATURE_SEED, b, n, D, M_ITEMS), 0)
    key = (GAL_SEED, philox.DOMAIN_GALLERY)
    og = [fv.encrypt(op, opk, pt, key, (b, i)) for i, pt in enumerate(pts)]
    S = hers.search_block(op, orlk, hers.encrypt_probe(op, opk, qv, PROBE_SEED), og)
    got = scores[0][b].cpu().numpy()
    assert np.array_equal(got[0], res(S[0], op.q_primes))
    assert np.array_equal(got[1], res(S[1], op.q_primes))
