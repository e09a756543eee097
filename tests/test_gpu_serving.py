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


def _align(x):
    return (x + 255) // 256 * 256


def _request_bytes(ctx, m, d):
    """Arena bytes of one request: probe search form, score ciphertexts, scores."""
    lib, h = ctx.lib, ctx.handle
    return (_align(int(lib.hers_probe_words(h, d)) * 4)
            + _align(ctx.blocks(m) * int(lib.hers_ct_words(h)) * 8) + _align(m * 4))


def _wave_bytes(ctx, m, d, nreq, blocks):
    """Arena bytes of one wave's workspace: probe encryption, decryption and
    `blocks` blocks of search per request."""
    lib, h = ctx.lib, ctx.handle
    enc = int(lib.hers_workspace_bytes(h, 1, 0, d))
    dec = int(lib.hers_workspace_bytes(h, 3, min(m, 256 * ctx.n), 1))
    per = int(lib.hers_workspace_bytes(h, 2, ctx.n, 1))
    return _align(enc) + _align(dec) + _align(per * blocks * nreq)


@pytest.mark.timeout(120)
def test_memory_admission_defers_and_completes(serving):
    """An arena with room for two requests and one wave's workspace, eight
    requests on one gallery: every later request needs the memory of an
    earlier, completed one, which is returned only when its result is
    collected.  The results are collected from a second thread that starts
    late, so the loop waits with nothing in flight and the queue full until
    memory comes back; every result is still bit-identical."""
    import threading
    import time
    gpu_lib, ctx, sk, gals, reqs, alone = serving
    g, m, d, _ = gals[2]
    sub = [(j, r) for j, r in enumerate(reqs) if r[0] == 2]
    sub = (sub * 3)[:8]
    req_b = _request_bytes(ctx, m, d)
    arena = 2 * req_b + _wave_bytes(ctx, m, d, 1, ctx.blocks(m)) + req_b // 2
    srv = gpu_lib.Server(ctx, sk, arena, max_batch=4)
    results = {}
    try:
        gid = srv.add_gallery(g, m, d)
        tickets = [srv.submit(gid, qv, seed) for _, (_, qv, seed) in sub]

        def collect():
            time.sleep(0.5)                  # the first two complete, the rest wait for memory
            for t in tickets:
                results[t] = srv.wait(t, scores=True, ciphertexts=True)

        th = threading.Thread(target=collect)
        th.start()
        th.join(90)
        assert not th.is_alive(), "results were not all delivered"
        stats = srv.stats()
    finally:
        srv.close()
    assert stats["completed"] == 8 and stats["deferrals"] > 0
    assert stats["arena_peak"] <= arena
    for t, (j, _) in zip(tickets, sub):
        lat, out, ct = results[t]
        assert np.array_equal(ct, alone[j][0]), j
        assert np.array_equal(out, alone[j][1]), j


def test_close_with_queued_requests_returns(serving):
    """Closing a server whose queue holds requests that cannot be admitted
    (no result collected, arena full) returns instead of waiting forever."""
    gpu_lib, ctx, sk, gals, reqs, alone = serving
    g, m, d, _ = gals[2]
    req_b = _request_bytes(ctx, m, d)
    srv = gpu_lib.Server(ctx, sk, req_b + _wave_bytes(ctx, m, d, 1, ctx.blocks(m)) + 4096, max_batch=1)
    gid = srv.add_gallery(g, m, d)
    for j in range(3):
        srv.submit(gid, reqs[2][1], 70 + j)
    srv.close()


def test_request_larger_than_arena_is_rejected(serving):
    gpu_lib, ctx, sk, gals, reqs, alone = serving
    srv = gpu_lib.Server(ctx, sk, 1 << 20, max_batch=4)
    try:
        gid = srv.add_gallery(*gals[2][:3])
        with pytest.raises(gpu_lib.HersError):
            srv.submit(gid, reqs[2][1], 1)
    finally:
        srv.close()
