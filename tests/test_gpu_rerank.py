"""GPU parity of the two-stage search's second stage (packed 1:1 re-ranking)
against the oracle, bit for bit, and of the whole two-stage pipeline against
plain inner products.  Integer work: tolerance 0."""

import numpy as np
import pytest
import torch

from oracle import fv, rerank
from paper_2003_12197_amd import synth

pytestmark = pytest.mark.gpu


def res(poly, primes):
    return np.array(fv.to_residues(poly, primes), dtype=np.int64)


@pytest.fixture(scope="module")
def rr(gpu_lib):
    # 22-bit t: 100 features at the +-63 bound sum below t/2
    print("case rerank: n=2048 q=3x36 t=22 bits W=128 D=100", flush=True)
    cfg = dict(n=2048, qbits=(36, 36, 36), t_bits=22, w_bits=0)
    ctx = gpu_lib.Context(d_max=128, **cfg)
    op = fv.Params(**cfg)
    sk, pk, rlk = ctx.keygen(41)
    osk, opk, orlk = fv.keygen(op, 41)
    W, D = 128, 100
    rk = ctx.rotation_keygen(41, W)
    S = ctx.n // W
    count = 3 * S + 5
    F, qv = synth.uniform_features(42, D, count)
    icanon = torch.empty((4, 2, ctx.k, ctx.n), dtype=torch.int64, device=ctx.device)
    items = ctx.rerank_encrypt(torch.from_numpy(F).to(ctx.device), W, 43, canon=icanon)
    pcanon = torch.empty((1, 2, ctx.k, ctx.n), dtype=torch.int64, device=ctx.device)
    probe = ctx.rerank_encrypt(torch.from_numpy(qv.reshape(D, 1).copy()).to(ctx.device), W, 44, replicate=True,
                               canon=pcanon)
    torch.cuda.synchronize()
    return dict(ctx=ctx, op=op, sk=sk, osk=osk, opk=opk, orlk=orlk, W=W, D=D, S=S, count=count, F=F, qv=qv, rk=rk,
                items=items, icanon=icanon.cpu().numpy(), pcanon=pcanon.cpu().numpy())


def test_rotation_keys_bit_exact(rr):
    ork = rerank.rotation_keygen(rr["op"], 41, rr["W"])
    ctx = rr["ctx"]
    got = rr["rk"].view(len(ork), ctx.L, 2, ctx.k, ctx.n).cpu().numpy()
    for st, key in enumerate(ork):
        for gi, (b, a) in enumerate(key):
            assert np.array_equal(got[st, gi, 0], res(b, rr["op"].q_primes)), (st, gi)
            assert np.array_equal(got[st, gi, 1], res(a, rr["op"].q_primes)), (st, gi)


def test_packed_items_and_probe_bit_exact(rr):
    op = rr["op"]
    oitems = rerank.encrypt_items(op, rr["opk"], rr["F"], rr["W"], 43)
    assert len(oitems) == 4
    for c, ct in enumerate(oitems):
        assert np.array_equal(rr["icanon"][c, 0], res(ct[0], op.q_primes)), c
        assert np.array_equal(rr["icanon"][c, 1], res(ct[1], op.q_primes)), c
    oprobe = rerank.encrypt_probe(op, rr["opk"], rr["qv"], rr["W"], 44)
    assert np.array_equal(rr["pcanon"][0, 0], res(oprobe[0], op.q_primes))
    assert np.array_equal(rr["pcanon"][0, 1], res(oprobe[1], op.q_primes))


def test_rerank_bit_exact_and_scores(rr):
    """Selected ciphertexts (an out-of-range id among them) give the oracle's
    rotate-and-add ciphertexts, with the full and a one-ciphertext workspace;
    decrypted segment scores are the items' inner products, 0 past the last
    item and for the out-of-range id."""
    ctx, op, W, S = rr["ctx"], rr["op"], rr["W"], rr["S"]
    ids = torch.tensor([3, 0, 9, 2], dtype=torch.int64)
    probe = ctx.rerank_encrypt(torch.from_numpy(rr["qv"].reshape(rr["D"], 1).copy()).to(ctx.device), W, 44,
                               replicate=True)
    oprobe = rerank.encrypt_probe(op, rr["opk"], rr["qv"], W, 44)
    oitems = rerank.encrypt_items(op, rr["opk"], rr["F"], W, 43)
    ork = rerank.rotation_keygen(op, 41, W)
    one = torch.empty(int(ctx.lib.hers_workspace_bytes(ctx.handle, 7, 1, 0)), dtype=torch.uint8, device=ctx.device)
    want = {3: rerank.rerank_ct(op, rr["orlk"], ork, oprobe, oitems[3], W)}
    for ws, fuse in ((None, 1), (one, 0)):                  # fused key switching, then the default choice
        ctx.set_option("relin_fuse_min_wgs", fuse)
        out = ctx.rerank(rr["items"], ids, probe, W, workspace=ws)
        got = out.cpu().numpy()
        assert np.array_equal(got[0, 0], res(want[3][0], op.q_primes))
        assert np.array_equal(got[0, 1], res(want[3][1], op.q_primes))
        assert not got[2].any()
        sc = ctx.rerank_decrypt(rr["sk"], out, W).cpu().numpy()
        plain = rr["F"].T.astype(np.int64) @ rr["qv"].astype(np.int64)
        for j, c in enumerate(ids.tolist()):
            exp = np.zeros(S, dtype=np.int64)
            lo, hi = c * S, min(rr["count"], (c + 1) * S)
            if c < 4:
                exp[: hi - lo] = plain[lo:hi]
            assert np.array_equal(sc[j], exp), (j, c)
    ctx.set_option("relin_fuse_min_wgs", 0)


def test_two_stage_pipeline_full_size(gpu_lib):
    """The two-stage search at n = 4096: HERS on 16 dimensions over 2^17
    items, top-1000 on the GPU, then re-ranking of the candidates' packed
    ciphertexts with 192 features (W = 256): every re-ranked score equals the
    plain 192-dimensional inner product, and the best re-ranked item is the
    probe's mate."""
    print("case two-stage: n=4096 m=2^17 d1=16 D=192 K=1000", flush=True)
    n, m, d1, D, W, K = 4096, 1 << 17, 16, 192, 256, 1000
    ctx1 = gpu_lib.Context(n=n, qbits=(36, 36, 36), t_bits=20, w_bits=0, d_max=16)
    ctx2 = gpu_lib.Context(n=n, qbits=(36, 36, 36), t_bits=22, w_bits=0, d_max=192)
    sk1, _, _ = ctx1.keygen(51)
    sk2, _, _ = ctx2.keygen(52)
    ctx2.rotation_keygen(52, W)
    full = synth.gallery_features(61, n, D, m)                  # 192-D templates, quantised unit vectors
    coarse = np.ascontiguousarray(full[:d1])                    # first-stage representation
    q_full, mate = synth.probe_for(62, 61, n, D, m, noise=0.03)   # the mate ranks 49th on the 16 coordinates
    q_coarse = np.ascontiguousarray(q_full[:d1])
    g1 = ctx1.encrypt_gallery(torch.from_numpy(coarse).to(ctx1.device), m, 71)
    items = ctx2.rerank_encrypt(torch.from_numpy(full).to(ctx2.device), W, 72)
    p1 = ctx1.encrypt_probe(torch.from_numpy(q_coarse).to(ctx1.device), 73)
    s1 = ctx1.decrypt_scores(sk1, ctx1.search(g1, m, d1, p1), m)
    idx, _ = ctx1.topk(s1, m, K)
    S = n // W
    cts = torch.unique(idx // S)
    p2 = ctx2.rerank_encrypt(torch.from_numpy(q_full.reshape(D, 1).copy()).to(ctx2.device), W, 74, replicate=True)
    sc = ctx2.rerank_decrypt(sk2, ctx2.rerank(items, cts, p2, W), W).cpu().numpy()
    plain = full.T.astype(np.int64) @ q_full.astype(np.int64)
    c = cts.cpu().numpy()
    for j in range(len(c)):
        assert np.array_equal(sc[j], plain[c[j] * S:(c[j] + 1) * S]), j
    cand = idx.cpu().numpy()
    assert mate in set(cand.tolist())
    best = cand[np.argmax(plain[cand])]
    assert int(best) == mate or plain[best] == plain[mate]
