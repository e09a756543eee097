"""Seeded synthetic inputs for tests and benchmarks (no HERS arithmetic here).

The paper's galleries (MegaFace 1M faces, 100M synthetic fingerprints with the
NIST SD4 probe/mate pairs, ImageNet; Sec. 4.2) and its DeepMDS++ compressed
representations are not available.  Stand-ins with the same shapes:

  * features are integers in [-63, 63]; a compressed representation x in R^d
    is drawn N(0, I_d), L2-normalised, scaled and rounded, then clipped to the
    feature bound.  The scale is the paper's quantisation step 0.004 (Sec. 3.2,
    "Encoding Scheme"; x 250) where the bound allows it, else the scale that
    puts the bound at four standard deviations of a coordinate (63 sqrt(d) / 4),
    so that almost no coordinate clips (x 89 at d = 32, x 126 at d = 64);
  * gallery block b (items b*n .. b*n + n - 1) is generated from its own
    generator PCG64(seed + b), so any block can be regenerated on its own;
  * a probe is a gallery item (its mate) plus N(0, (0.4 / sqrt(d))^2) noise per
    coordinate (a noise vector of norm about 0.4), re-normalised and quantised
    the same way (the probe/mate structure of NIST SD4);
  * the toy workload draws features uniformly in [-63, 63].
"""

import math

import numpy as np

QUANT_STEP = 0.004
FEATURE_BOUND = 63


def quant_scale(d):
    """Integers per unit of a coordinate: 1 / 0.004, or less where 4 standard
    deviations of a unit vector's coordinate (4 / sqrt(d)) would pass the bound."""
    return min(1.0 / QUANT_STEP, FEATURE_BOUND * math.sqrt(d) / 4.0)


def quantize(x):
    """Real unit-vector features [..., d] -> integers at the scale of
    quant_scale(d), clipped to the bound."""
    x = np.asarray(x)
    s = quant_scale(x.shape[-1])
    return np.clip(np.rint(x * s), -FEATURE_BOUND, FEATURE_BOUND).astype(np.int32)


def uniform_features(seed, d, m):
    """Toy workload: [d][m] integers uniform in [-63, 63], and a probe [d]."""
    rng = np.random.default_rng(seed)
    P = rng.integers(-FEATURE_BOUND, FEATURE_BOUND + 1, size=(d, m)).astype(np.int32)
    q = rng.integers(-FEATURE_BOUND, FEATURE_BOUND + 1, size=d).astype(np.int32)
    return P, q


def _unit_rows(rng, count, d):
    x = rng.standard_normal((count, d))
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def gallery_block(seed, b, n, d, m_total):
    """Features of gallery block b as int32 [d][n] (columns past m_total are 0)."""
    rng = np.random.Generator(np.random.PCG64(seed + b))
    x = _unit_rows(rng, n, d)
    out = quantize(x).T.copy()
    valid = max(0, min(n, m_total - b * n))
    out[:, valid:] = 0
    return out


def gallery_features(seed, n, d, m_total, block0=0, nblocks=None):
    """int32 [d][nblocks * n] for blocks block0 .. block0 + nblocks - 1 (whole
    blocks: columns past m_total are zero)."""
    M = (m_total + n - 1) // n
    if nblocks is None:
        nblocks = M - block0
    return np.concatenate([gallery_block(seed, b, n, d, m_total) for b in range(block0, block0 + nblocks)], axis=1)


def probe_for(seed, gallery_seed, n, d, m_total, noise=None):
    """A probe whose mate is a seeded gallery item; returns (probe int32 [d], mate index).
    `noise` is the standard deviation per coordinate (default 0.4 / sqrt(d))."""
    if noise is None:
        noise = 0.4 / math.sqrt(d)
    rng = np.random.default_rng(seed)
    mate = int(rng.integers(0, m_total))
    b, j = divmod(mate, n)
    brng = np.random.Generator(np.random.PCG64(gallery_seed + b))
    x = _unit_rows(brng, n, d)[j]
    y = x + noise * rng.standard_normal(d)
    y /= np.linalg.norm(y)
    return quantize(y), mate


def clip_fraction(seed, n, d):
    """Fraction of quantised coordinates that hit the clip bound (one block)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = _unit_rows(rng, n, d) * quant_scale(d)
    return float(np.mean(np.abs(np.rint(x)) > FEATURE_BOUND))


def serving_galleries(seed, count=8, lo=1e3, hi=5e6, dims=(16, 32, 64)):
    """Sizes log-uniform in [lo, hi] and d uniform over `dims`."""
    rng = np.random.default_rng(seed)
    sizes = [int(round(10 ** rng.uniform(math.log10(lo), math.log10(hi)))) for _ in range(count)]
    ds = [int(rng.choice(dims)) for _ in range(count)]
    return sizes, ds


def poisson_arrivals(seed, rate, count, ngalleries):
    """Arrival times (s) of a Poisson stream and the gallery each request targets."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    return np.cumsum(gaps), rng.integers(0, ngalleries, size=count)
