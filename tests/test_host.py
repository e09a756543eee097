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


def test_double_precision_modular_arithmetic(tmp_path):
    """The double-precision modular arithmetic of the transforms (ModQF,
    ModQB in ntt.h), compiled for the host, against exact integers: ModQF
    products are the residue in [0, q); ModQB products are congruent and of
    magnitude < 0.7 q for |a| <= 16 q; ModQB reductions are congruent and of
    magnitude <= q/2 + 1; the u64 <-> double conversions are exact below 2^52.
    Primes just below 2^36, 2^44 and 2^45 (the largest the balanced path
    accepts), operands random and at the extremes."""
    import random
    import shutil
    import subprocess

    from oracle import primes

    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    src = os.path.join(os.path.dirname(__file__), "native", "f64_modarith.cpp")
    exe = str(tmp_path / "f64_modarith")
    subprocess.run([gxx, "-O2", "-std=c++17", "-Wno-unknown-pragmas", "-o", exe, src], check=True)
    rng = random.Random(2003)
    cases = []
    for bits in (36, 44, 45):
        for q in primes.ntt_primes([bits, bits], 8192):
            for _ in range(400):
                w = rng.randrange(q)
                cases.append(("F", q, rng.randrange(4 * q), w))
                cases.append(("B", q, rng.randrange(-16 * q, 16 * q + 1), w))
                cases.append(("R", q, rng.randrange(-16 * q, 16 * q + 1), 0))
            for a in (0, 1, q - 1, 4 * q - 1):
                cases.append(("F", q, a, q - 1))
            for a in (-16 * q, 16 * q, -16 * q + 1, 16 * q - 1, 8 * q + q // 2):
                cases.append(("B", q, a, q - 1))
                cases.append(("R", q, a, 0))
    for v in (0, 1, 2**36 - 5, 2**51 + 12345, 2**52 - 1):
        cases.append(("C", 0, v, 0))
    inp = "".join("%s %d %d %d\n" % c for c in cases)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split()
    assert len(out) == len(cases)
    for (op, q, a, w), r in zip(cases, out):
        r = int(r)
        if op == "F":
            assert r == a * w % q, (op, q, a, w, r)
        elif op == "B":
            assert (r - a * w) % q == 0 and 10 * abs(r) < 7 * q, (op, q, a, w, r)
        elif op == "R":
            assert (r - a) % q == 0 and 2 * abs(r) <= q + 2, (op, q, a, r)
        else:
            assert r == a, (op, a, r)


def test_rescale_two_word_rounding_matches_all_words(tmp_path):
    """The exact rescale's round(F) (Alg. "Ciphertext Multiplication": scale by
    t/q and round) is first formed from the top two 64-bit fraction words and
    recomputed from all W words only when that fraction is within 2^-64 of
    one half.  Checked with exact integers: the W-word sum's rounding, the
    two-word sum's rounding and near-half flag, and that an unflagged
    two-word result always equals the W-word one, on random words and on
    carry and borrow chains built so that the two-word sum lands on the other
    side of one half (and is flagged)."""
    import random
    import shutil
    import subprocess

    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    src = os.path.join(os.path.dirname(__file__), "native", "rescale_round.cpp")
    exe = str(tmp_path / "rescale_round")
    subprocess.run([gxx, "-O2", "-std=c++17", "-Wno-unknown-pragmas", "-o", exe, src], check=True)
    M = (1 << 64) - 1
    H = 1 << 63
    rng = random.Random(2003)
    cases = []      # (W, y, gamma, phi[r][w], psi[w])
    for _ in range(3000):
        W, K = rng.randint(1, 6), rng.choice((1, 2, 3, 8, 16, 32))
        y = [rng.randrange(1 << rng.choice((30, 32))) for _ in range(K)]
        phi = [[rng.randrange(1 << 64) for _ in range(W)] for _ in range(K)]
        psi = [rng.randrange(1 << 64) for _ in range(W)]
        cases.append((W, y, rng.randrange(40), phi, psi))
    for W in (3, 4, 5):
        # one polynomial term, top fraction word around 1/2, random lower words
        for top in (H - 2, H - 1, H, H + 1):
            for _ in range(20):
                cases.append((W, [1], 0, [[rng.randrange(1 << 64) for _ in range(W - 1)] + [top]], [0] * W))
        # a carry from the dropped lowest word lifts the sum from just below 1/2 to exactly 1/2
        cases.append((W, [1, 1], 0, [[M] * (W - 1) + [H - 1], [1] + [0] * (W - 1)], [0] * W))
        # a borrow from the dropped lowest word takes 1/2 to just below it
        cases.append((W, [1], 1, [[0] * (W - 1) + [H]], [1] + [0] * (W - 1)))
        # the same around -1/2 and 3/2 (negative and integer parts)
        cases.append((W, [1], 1, [[0] * W], [M] * (W - 1) + [H - 1]))
        cases.append((W, [3, 1], 0, [[M] * (W - 1) + [H - 1], [1] + [0] * (W - 1)], [0] * W))
        # largest operands: every word and y at their maximum
        cases.append((W, [(1 << 32) - 1] * 32, (1 << 32) - 1, [[M] * W for _ in range(32)], [M] * W))
    inp = "".join("%d %d %d %s %s %s\n" % (W, len(y), g, " ".join(map(str, y)),
                                           " ".join(str(v) for row in phi for v in row), " ".join(map(str, psi)))
                  for W, y, g, phi, psi in cases)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.splitlines()
    assert len(out) == len(cases)

    def rounded(W, y, g, phi, psi, w0):
        num = sum(yr * sum(row[w] << (64 * w) for w in range(w0, W)) for yr, row in zip(y, phi))
        num -= g * sum(psi[w] << (64 * w) for w in range(w0, W))
        num %= 1 << (64 * (W + 1))                     # the kernel's W + 1 words wrap
        r = ((num + (1 << (64 * W - 1))) >> (64 * W)) & M
        top = (num >> (64 * (W - 1))) & M
        return r - (1 << 64) if r >> 63 else r, top in (H - 1, H)

    flips = 0
    for (W, y, g, phi, psi), line in zip(cases, out):
        rs, nh, rw = (int(v) for v in line.split())
        full, _ = rounded(W, y, g, phi, psi, 0)
        short, near = rounded(W, y, g, phi, psi, W - 2 if W > 2 else 0)
        assert rw == full, (W, y, g)
        assert (rs, bool(nh)) == (short, near), (W, y, g)
        assert nh or rs == rw, (W, y, g)             # the fallback is taken whenever it is needed
        flips += W > 2 and short != full
    assert flips >= 6      # the built chains do reach the W-word fallback


@pytest.mark.parametrize("n,t_bits,qbits", [
    (4096, 20, (36, 36, 36)),            # the 10^8 x 32 ring
    (8192, 21, (44, 44, 44, 43, 43)),    # the batched ring
    (1024, 20, (44, 44, 32)),            # primes of unequal size
    (256, 20, (60, 60, 60, 60)),         # wide primes, fraction form still on
    (256, 20, (61,) * 6),                # the widest primes: a window of 3/4 beside each carry
])
def test_decryption_scale_fraction_form(tmp_path, n, t_bits, qbits):
    """Alg. "Decryption" scales [c0 + c1 s]_q by t/q and rounds.  The kernel
    first forms round(t x / q) mod t from 64-bit fixed-point fractions
    t / q_i and falls back to the exact CRT form when the rounded sum's low
    word is within sum_i q_i of a carry.  Checked on the host with the
    resolved constants against round(t x / q) mod t computed with exact
    integers: random x, x just beside the half-integer points of t x / q
    (where the fraction form must step aside), x near the integer points (a
    valid ciphertext's small noise) and the ends of [0, q)."""
    import random
    import shutil
    import subprocess

    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    csrc = os.path.join(ROOT, "paper_2003_12197_amd", "csrc")
    exe = str(tmp_path / "decrypt_scale")
    subprocess.run([gxx, "-O2", "-std=c++17", "-Wno-unknown-pragmas", "-o", exe,
                    os.path.join(os.path.dirname(__file__), "native", "decrypt_scale.cpp"),
                    os.path.join(csrc, "params.cpp")], check=True)
    k = len(qbits)
    # the harness prints the resolved t and q_i first; read them with an empty input
    head = subprocess.run([exe], input="%d %d %d %s\n" % (n, t_bits, k, " ".join(map(str, qbits))),
                          capture_output=True, text=True, check=True).stdout.split()
    t, qs = int(head[1]), [int(v) for v in head[2:2 + k]]
    q = 1
    for qi in qs:
        q *= qi
    rng = random.Random(12197 + n + k)
    xs = [rng.randrange(q) for _ in range(1500)] + [0, 1, q - 1]
    near_half, near_int = [q // 2, (q + 1) // 2], []            # t x / q within t / 2q of t / 2 (t odd)
    for _ in range(300):
        j = rng.randrange(t)
        c = (2 * j + 1) * q // (2 * t)                 # t c / q just below j + 1/2
        near_half += [(c + dlt) % q for dlt in range(-2, 4)]
        c = j * q // t
        near_int += [(c + dlt) % q for dlt in (-(1 << 20), -5, 0, 5, 1 << 20)]
    xs += near_half + near_int
    lines = "".join(" ".join(str(x % qi) for qi in qs) + "\n" for x in xs)
    out = subprocess.run([exe], input="%d %d %d %s\n" % (n, t_bits, k, " ".join(map(str, qbits))) + lines,
                         capture_output=True, text=True, check=True).stdout.splitlines()[1:]
    assert len(out) == len(xs)
    fast_n = 0
    for x, line in zip(xs, out):
        fast, v, exact = (int(w) for w in line.split())
        want = (2 * t * x + q) // (2 * q) % t          # round(t x / q) mod t (no ties: q is odd, x < q)
        assert exact == want, (x, exact, want)
        if fast:
            assert v == want, (x, v, want)
        fast_n += fast
    if sum(qs) < (1 << 54):
        # a window of sum_i q_i / 2^64 < 2^-10 beside each carry: the fraction form decides all but
        # the near-half points, and steps aside beside some of them
        assert fast_n >= len(xs) - len(near_half)
        hs = set(near_half)
        assert any(x in hs and line.startswith("0 ") for x, line in zip(xs, out))
    elif sum(qs) < (1 << 64):
        assert fast_n > 0                               # wide primes: a wide window, some decided
    else:
        assert fast_n == 0                              # (no parameter set reaches a sum of 2^64)
