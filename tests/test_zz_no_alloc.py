"""hers_search_noalloc (the search with its workspace in the library's static
scratch array, for callers that cannot allocate) against hers_search, called
through the C ABI: bit-identical score ciphertexts on two calls in a row, the
second with a smaller gallery, and on a gallery larger than one chunk of the
array.  Integer work: tolerance 0."""

import numpy as np
import pytest
import torch

from paper_2003_12197_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(300)
def test_noalloc_search_equals_search(gpu_lib):
    print("case noalloc: n=4096 q=3x36 d=16, 200 blocks then 5 blocks + 7 items", flush=True)
    ctx = gpu_lib.Context(n=4096, qbits=(36, 36, 36), t_bits=20, w_bits=0, d_max=16)
    sk, _, _ = ctx.keygen(41)
    per_block = int(ctx.lib.hers_workspace_bytes(ctx.handle, 2, ctx.n, 1))
    scratch = 64 << 20
    d = 16
    m1 = 200 * ctx.n                         # more blocks than one chunk of the scratch array
    assert ctx.blocks(m1) * per_block > scratch
    P = synth.gallery_features(42, ctx.n, d, m1)
    gal = ctx.encrypt_gallery(torch.from_numpy(P).to(ctx.device), m1, 43)
    qv, _ = synth.probe_for(44, 42, ctx.n, d, m1)
    pr = ctx.encrypt_probe(torch.from_numpy(qv).to(ctx.device), 45)
    m2 = 5 * ctx.n + 7
    P2, q2 = synth.uniform_features(46, d, m2)
    gal2 = ctx.encrypt_gallery(torch.from_numpy(P2).to(ctx.device), m2, 47)
    pr2 = ctx.encrypt_probe(torch.from_numpy(q2).to(ctx.device), 48)
    want1 = ctx.search(gal, m1, d, pr)
    want2 = ctx.search(gal2, m2, d, pr2)
    got1 = ctx.search_noalloc(gal, m1, d, pr, ctx.new_scores(m1).fill_(-1))
    got2 = ctx.search_noalloc(gal2, m2, d, pr2, ctx.new_scores(m2).fill_(-1))
    torch.cuda.synchronize()
    assert torch.equal(got1, want1)
    assert torch.equal(got2, want2)
    out = ctx.decrypt_scores(sk, got2, m2).cpu().numpy()
    assert np.array_equal(out, P2.T.astype(np.int64) @ q2.astype(np.int64))
