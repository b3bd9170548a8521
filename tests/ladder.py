"""The first rung of the error-control ladder, computed from the definitions.

Used by the tests to say which outcome the compressor must take for a block:
kept bits K0 from eq. (4) (read as sign + exponent + m0 mantissa bits), the
truncation of v = x - mu to those bits done on values (rationals) rather than
on bit patterns, and the exact check |x - x'| <= e of eq. (1). Nothing here is
shared with, or imported from, either implementation.
"""
import math
from fractions import Fraction

import numpy as np

# element type -> (W bits, E exponent bits, smallest normal exponent)
TYPES = {np.float32: (32, 8, -126), np.float64: (64, 11, -1022)}


def spec(dtype):
    return TYPES[np.dtype(dtype).type]


def p_of(y, emin):
    """Unbiased exponent of |y|; zero and subnormals take emin (eq. (4))."""
    y = abs(float(y))
    if y == 0.0:
        return emin
    _, ex = math.frexp(y)  # y = f * 2^ex, 0.5 <= f < 1
    return max(ex - 1, emin)


def total_order_extrema(blk):
    """(min, max) under IEEE totalOrder (-0 below +0)."""
    T = blk.dtype.type
    u = blk.view(np.uint32 if T == np.float32 else np.uint64)
    sign = u.dtype.type(1) << u.dtype.type(8 * u.itemsize - 1)
    key = np.where(u & sign, ~u, u | sign)
    return blk[int(np.argmin(key))], blk[int(np.argmax(key))]


def truncate(v, m, emin):
    """v truncated toward zero to m fraction bits below its leading bit (the
    IEEE prefix of sign, exponent and m mantissa bits), as a rational."""
    V = Fraction(float(v))
    if V == 0:
        return V
    q = Fraction(2) ** (p_of(v, emin) - m)
    t = (abs(V) // q) * q
    return t if V > 0 else -t


def passes(blk, mu, e, m, emin):
    """Every value of the block reconstructs within e with m mantissa bits."""
    T = blk.dtype.type
    E = Fraction(float(e))
    for x in blk:
        v = T(x - mu)
        vt = truncate(v, m, emin)
        vtT = T(float(vt))
        assert Fraction(float(vtT)) == vt  # few bits: representable
        xr = T(mu + vtT)
        if abs(Fraction(float(x)) - Fraction(float(xr))) > E:
            return False
    return True


def first_rung(blk, e):
    """(mu, m0, K0) of a finite, non-constant block for bound e."""
    T = blk.dtype.type
    W, E, emin = spec(T)
    mn, mx = total_order_extrema(blk)
    mu = T(T(0.5) * mn + T(0.5) * mx)
    r = max(abs(T(mx - mu)), abs(T(mn - mu)))
    m0 = max(0, p_of(r, emin) - p_of(e, emin))
    return mu, m0, min(W, 1 + E + m0)


def expected_outcome(blk, e):
    """'K0', 'K0+1' or 'raw' for a finite, non-constant block, by brute force
    with rationals; plus K0."""
    T = blk.dtype.type
    W, E, emin = spec(T)
    mu, m0, K0 = first_rung(blk, e)
    mant = W - 1 - E
    if passes(blk, mu, e, min(m0, mant), emin):
        return "K0", K0
    if K0 < W and passes(blk, mu, e, min(m0 + 1, mant), emin):
        return "K0+1", K0
    return "raw", K0


def outcomes_of_stream(x, info):
    """For every non-constant finite block of a stream (parsed with streamfmt):
    the stored outcome relative to its first rung: 'K0', 'K0+1', 'raw' (raw
    although finite), with K0. Non-finite blocks are skipped."""
    b = info["b"]
    e = info["e"]
    ranks = np.cumsum(info["state"]) - 1
    out = []
    for k in np.nonzero(info["state"])[0]:
        blk = np.ascontiguousarray(x[k * b:(k + 1) * b])
        if not np.all(np.isfinite(blk)):
            continue
        _, _, K0 = first_rung(blk, e)
        K = int(info["K"][ranks[k]])
        if K == 0xFF:
            out.append(("raw", K0))
        elif K == K0:
            out.append(("K0", K0))
        elif K == K0 + 1:
            out.append(("K0+1", K0))
        else:
            out.append((f"K={K}", K0))
    return out


def subnormal_blocks(dtype, count, seed, b=8):
    """Seeded blocks of b values near the subnormal range with a subnormal
    bound each: (blocks, bounds). Such bounds lie below 2^p(e) (p clamps at
    the smallest normal exponent), so the first rung can fail and the second
    one, or raw storage, must take over."""
    T = np.dtype(dtype).type
    W, E, emin = spec(T)
    mant = W - 1 - E
    sub = 2.0 ** (emin - mant)
    r = np.random.default_rng(seed)
    blocks, bounds = [], []
    for _ in range(count):
        k = int(r.integers(mant - 3, mant + 3))
        blk = (r.integers(-2 ** k, 2 ** k, b).astype(np.float64) * sub).astype(T)
        e = T(float(r.integers(1, 2 ** (k - int(r.integers(1, 6))))) * sub)
        blocks.append(blk)
        bounds.append(e)
    return blocks, bounds


def constructed_blocks(dtype):
    """Two hand-made blocks of 8 values: {0, 2^emin} x 4 with a subnormal
    bound e < 2^(emin - 1), which the first rung (no mantissa bit: v' = 0)
    fails and the second (one mantissa bit: v' = v exactly) passes; and
    {0, 2^emin, 3 ulp, 0...} at the smallest subnormal bound, which both fail
    (stored raw although K0 < W). Returns [(block, eb, outcome)]."""
    T = np.dtype(dtype).type
    W, E, emin = spec(T)
    sub = 2.0 ** (emin - (W - 1 - E))
    a = np.array([0.0, 2.0 ** emin] * 4, dtype=T)
    c = np.array([0.0, 2.0 ** emin, 3 * sub, 0.0, 0.0, 0.0, 0.0, 0.0], dtype=T)
    e_mid = 1e-40 if T == np.float32 else 1e-310
    return [(a, e_mid, "K0+1"), (c, sub, "raw")]


def subnormal_field(dtype, nblk, b, seed):
    """(x, eb): a field of nblk blocks of b values for one subnormal absolute
    bound (1e-40 for float32, 1e-310 for float64) that mixes blocks kept at
    K0 bits, at K0 + 1 bits, raw ones and constant ones: the hand-made
    {0, 2^emin} block first, then blocks of small integers times a power of
    two near the smallest normal number (a coarse grid makes a short
    truncation exact or not, depending on the grid and the block's range)."""
    T = np.dtype(dtype).type
    W, E, emin = spec(T)
    mant = W - 1 - E
    sub = 2.0 ** (emin - mant)
    eb = 1e-40 if T == np.float32 else 1e-310
    r = np.random.default_rng(seed)
    parts = [np.resize(blk, b).astype(T) for blk, _, want in constructed_blocks(T) if want == "K0+1"]
    while len(parts) < nblk:
        g = int(r.integers(mant - 3, mant + 2))
        M = int(2 ** r.integers(0, 7)) if len(parts) % 16 else 0
        parts.append((r.integers(-M, M + 1, b).astype(np.float64) * 2.0 ** g * sub).astype(T))
    return np.concatenate(parts[:nblk]), eb
