"""Serving loop on the GPU: continuous batching with memory admission.

Each request's score ciphertexts must be bit-identical whether it is served
alone (hers_encrypt_probe + hers_search + hers_decrypt_scores with the same
seed) or in a mix with other requests on other galleries; decrypted scores
equal P^T q.  Tolerance: bit-exact."""

import numpy as np
import pytest
import torch

from oracle import hers
from paper_2003_12197_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serving(gpu_lib):
    print("case serving: n=2048 q=3x36, three galleries of uneven m and d", flush=True)
    ctx = gpu_lib.Context(n=2048, qbits=(36, 36, 36), t_bits=20, w_bits=0, d_max=16)
    sk, pk, rlk = ctx.keygen(31)
    gals = []
    for gi, (m, d) in enumerate([(3 * 2048 + 5, 5), (1000, 16), (5 * 2048, 8)]):
        P, _ = synth.uniform_features(700 + gi, d, m)
        g = ctx.encrypt_gallery(torch.from_numpy(P).to(ctx.device), m, 800 + gi)
        gals.append((g, m, d, P))
    rng = np.random.default_rng(123)
    reqs = []
    for j in range(14):
        gi = j % 3
        qv = rng.integers(-63, 64, size=gals[gi][2]).astype(np.int32)
        reqs.append((gi, qv, 9000 + j))
    # each request served alone through the direct calls
    alone = []
    for gi, qv, seed in reqs:
        g, m, d, P = gals[gi]
        pr = ctx.encrypt_probe(torch.from_numpy(qv).to(ctx.device), seed)
        sc = ctx.search(g, m, d, pr)
        out = ctx.decrypt_scores(sk, sc, m)
        torch.cuda.synchronize()
        alone.append((sc.cpu().numpy().reshape(-1).view(np.uint64).copy(), out.cpu().numpy()))
    return gpu_lib, ctx, sk, gals, reqs, alone


def _serve(gpu_lib, ctx, sk, gals, reqs, arena_bytes, max_batch):
    srv = gpu_lib.Server(ctx, sk, arena_bytes, max_batch=max_batch)
    try:
        gids = [srv.add_gallery(g, m, d) for g, m, d, _ in gals]
        tickets = [srv.submit(gids[gi], qv, seed) for gi, qv, seed in reqs]
        results = [srv.wait(t, scores=True, ciphertexts=True) for t in tickets]
        stats = srv.stats()
    finally:
        srv.close()
    return results, stats


def test_mixed_requests_equal_alone(serving):
    gpu_lib, ctx, sk, gals, reqs, alone = serving
    results, stats = _serve(gpu_lib, ctx, sk, gals, reqs, 256 << 20, 8)
    assert stats["completed"] == len(reqs) and stats["waves"] >= 2
    for j, ((lat, out, ct), (ct1, out1)) in enumerate(zip(results, alone)):
        gi, qv, _ = reqs[j]
        assert np.array_equal(ct, ct1), j
        assert np.array_equal(out, out1), j
        assert np.array_equal(out, hers.plaintext_scores(gals[gi][3], qv)), j
        assert lat > 0


def test_memory_admission_defers_and_completes(serving):
    """An arena with room for about two requests plus one wave's workspace:
    later requests wait for memory, every result is still exact."""
    gpu_lib, ctx, sk, gals, reqs, alone = serving
    per_req = 6 << 20
    results, stats = _serve(gpu_lib, ctx, sk, gals, reqs[:8], 2 * per_req + (8 << 20), 4)
    assert stats["completed"] == 8
    assert stats["deferrals"] > 0
    for j, (lat, out, ct) in enumerate(results):
        assert np.array_equal(ct, alone[j][0]), j


def test_request_larger_than_arena_is_rejected(serving):
    gpu_lib, ctx, sk, gals, reqs, alone = serving
    srv = gpu_lib.Server(ctx, sk, 1 << 20, max_batch=4)
    try:
        gid = srv.add_gallery(*gals[2][:3])
        with pytest.raises(gpu_lib.HersError):
            srv.submit(gid, reqs[2][1], 1)
    finally:
        srv.close()
