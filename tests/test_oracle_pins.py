"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here re-types the oracle's code: exactness is checked with rational
arithmetic (fractions.Fraction), truncation is done on values rather than bit
patterns, and fixtures under tests/golden/ come from the paper's worked example
or are derived by hand from the definitions.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import szref
import streamfmt as sf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers ---

def exact_max_err(x, y):
    """max |x - y| computed exactly (Fraction on the largest candidates)."""
    x = np.asarray(x).ravel()
    y = np.asarray(y).ravel()
    d = np.abs(x.astype(np.float64) - y.astype(np.float64))
    if d.size == 0:
        return Fraction(0)
    # double differences of the candidates are re-done exactly
    cand = np.argsort(d)[-8:]
    return max(abs(Fraction(float(x[i])) - Fraction(float(y[i]))) for i in cand)


def within(x, y, e):
    """Every |x_i - y_i| <= e exactly (eq. (1))."""
    x = np.asarray(x).ravel()
    y = np.asarray(y).ravel()
    d = np.abs(x.astype(np.float64) - y.astype(np.float64))
    E = Fraction(float(e))
    # anything the double difference puts clearly below e is below e; the rest
    # (within a relative 1e-6 of e, or above) is decided with rationals
    sus = np.nonzero(d >= float(e) * (1 - 1e-6))[0]
    for i in sus:
        if abs(Fraction(float(x[i])) - Fraction(float(y[i]))) > E:
            return False
    return True


def f32(v):
    return np.float32(v)


def rng(seed):
    return np.random.default_rng(seed)


def smooth_field(n, seed, dtype=np.float32, noise=1e-3):
    r = rng(seed)
    t = np.arange(n) / n
    x = np.zeros(n)
    for _ in range(6):
        x += np.sin(2 * np.pi * r.uniform(1, 200) * t + r.uniform(0, 6.28))
    x += noise * r.standard_normal(n)
    x[(t > 0.3) & (t < 0.4)] = 0.0
    return x.astype(dtype)


# --------------------------------------------------- P1: the error bound ---

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("eb", [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-7])
@pytest.mark.parametrize("block", [8, 64, 128, 1024])
def test_p1_error_bound_rel(dtype, eb, block):
    x = smooth_field(30011, 7, dtype)
    s = szref.compress(x, eb, "rel", block)
    y = szref.decompress(s)
    e = szref.error_bound(x, eb, "rel", block)
    assert y.dtype == x.dtype and y.shape == x.shape
    assert within(x, y, e)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_p1_error_bound_abs_wide_exponents(dtype):
    r = rng(11)
    # values spread over many binades, both signs, some exact zeros
    x = (r.standard_normal(20000) * 10.0 ** r.integers(-30, 30, 20000)).astype(dtype)
    x[::97] = 0.0
    for eb in [1e-20, 1e-3, 1.0, 1e10]:
        s = szref.compress(x, eb, "abs", 128)
        y = szref.decompress(s)
        e = szref.error_bound(x, eb, "abs", 128)
        assert within(x, y, e)


def test_p1_subnormals_and_signed_zeros():
    tiny = np.float32(1.4e-45)
    x = np.array([0.0, -0.0, tiny, -tiny, 3 * tiny, 1e-39, -1e-39, 1e-38] * 16, dtype=np.float32)
    for eb in [0.0, 1e-45, 1e-40, 1e-38]:
        s = szref.compress(x, eb, "abs", 8)
        y = szref.decompress(s)
        e = szref.error_bound(x, eb, "abs", 8)
        assert within(x, y, e)


def test_p1_extreme_range_float32():
    big = np.finfo(np.float32).max
    x = np.array([big, -big, big / 3, -big / 7, 1.0, -1.0, 0.0, 5e37] * 4, dtype=np.float32)
    for eb in [0.0, 1e-3, 0.5]:
        s = szref.compress(x, eb, "rel", 8)
        y = szref.decompress(s)
        e = szref.error_bound(x, eb, "rel", 8)
        assert within(x, y, e)


# --------------------------------------------------- e from REL and ABS ---

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_error_bound_is_largest_T_below_range_times_eb(dtype):
    r = rng(3)
    for trial in range(50):
        x = (r.standard_normal(257) * 10.0 ** r.integers(-5, 5)).astype(dtype)
        eb = float(10.0 ** r.uniform(-7, -1))
        e = dtype(szref.error_bound(x, eb, "rel", 8))
        ed = eb * (float(x.max()) - float(x.min()))  # double arithmetic
        assert float(e) <= ed
        assert float(np.nextafter(e, dtype(np.inf))) > ed
    # non-finite values are left out of the range; none finite -> e = 0
    x = np.array([np.nan, 1.0, np.inf, 3.0, -np.inf, 2.0, 2.0, 2.0], dtype=dtype)
    assert szref.error_bound(x, 0.5, "rel", 8) == 1.0
    x = np.array([np.nan] * 8, dtype=dtype)
    assert szref.error_bound(x, 0.5, "rel", 8) == 0.0
    # ABS: eb itself, rounded down into T
    e = szref.error_bound(np.zeros(8, np.float32), 0.1, "abs", 8)
    assert float(np.float32(e)) <= 0.1 < float(np.nextafter(np.float32(e), np.float32(1)))


# --------------------------------------------- P2: constant-block rule ---

def _blocks(x, b):
    n = x.size
    return [x[k * b:min(n, (k + 1) * b)] for k in range((n + b - 1) // b)]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_p2_constant_rule(dtype):
    x = smooth_field(64 * 500, 5, dtype, noise=1e-4)
    for eb in [1e-1, 1e-2, 1e-3]:
        s = szref.compress(x, eb, "rel", 64)
        info = sf.parse(s)
        e = Fraction(float(info["e"]))
        for k, blk in enumerate(_blocks(x, 64)):
            mn, mx = Fraction(float(blk.min())), Fraction(float(blk.max()))
            const = not info["state"][k]
            if const:
                # every value within e of the stored mid value (Alg. 1 constant test)
                mu = Fraction(float(info["mu"][k]))
                assert mx - mu <= e and mu - mn <= e
                assert mx - mn <= 2 * e
            if mx == mn:
                assert const
            if mx - mn > 2 * e:
                assert not const
            mid = (mn + mx) / 2
            if Fraction(float(dtype(float(mid)))) == mid and mx - mn <= 2 * e:
                assert const


def test_p2_exact_decision_at_ties():
    """The constant test is exact even where fl(mx - mu) rounds onto e."""
    r = rng(17)
    decided = {True: 0, False: 0}
    for trial in range(3000):
        mn = np.float32(r.standard_normal() * 10.0 ** r.integers(-3, 3))
        mx = np.float32(mn + abs(r.standard_normal()) * 10.0 ** r.integers(-8, 3))
        if not (mx > mn):
            continue
        mu = np.float32(np.float32(0.5) * mn + np.float32(0.5) * mx)
        # pick e on the rounding tie of the larger side, or one step off it
        e = max(np.float32(mx - mu), np.float32(mu - mn))
        e = [e, np.nextafter(e, np.float32(0)), np.nextafter(e, np.float32(np.inf))][trial % 3]
        x = np.array([mn, mx] * 4, dtype=np.float32)
        s = szref.compress(x, float(e), "abs", 8)
        info = sf.parse(s)
        assert float(info["e"]) == float(e)
        M = Fraction(float(info["mu"][0])) if not info["state"][0] else Fraction(float(mu))
        exact = (Fraction(float(mx)) - M <= Fraction(float(e))) and \
                (M - Fraction(float(mn)) <= Fraction(float(e)))
        assert (not info["state"][0]) == exact
        decided[exact] += 1
    assert decided[True] > 100 and decided[False] > 100


# ------------------------------------------------- P3: section costs ---

def test_p3_all_constant_float32_cr_124():
    n = 1 << 20
    x = np.full(n, 3.25, dtype=np.float32)
    s = szref.compress(x, 1e-2, "abs", 128)
    info = sf.parse(s)
    assert info["n_nc"] == 0 and info["mid_total"] == 0
    nblk = n // 128
    # one state bit and one 4-byte mu per block, plus header and alignment
    assert len(s) == 96 + nblk // 8 + 4 * nblk
    cr = x.nbytes / len(s)
    assert 123.5 < cr < 512 / 4.125 + 1e-9
    # the paper's per-field maximum CR at REL 1E-2 is 124 (Table of CRs)
    assert round(512 / 4.125) == 124


def test_p3_all_constant_float64():
    n = 1 << 18
    x = np.full(n, -7.0, dtype=np.float64)
    s = szref.compress(x, 0.0, "rel", 128)
    nblk = n // 128
    assert len(s) == 96 + nblk // 8 + 8 * nblk
    assert 125.0 < x.nbytes / len(s) < 1024 / 8.125 + 1e-9


# ----------------------------------- P4: eq. (4) bit budget, brute force ---

def _p(y):
    """Unbiased exponent of |y| as eq. (4) uses it (zero/subnormal: emin)."""
    y = abs(float(y))
    if y == 0.0:
        return -126
    m, ex = math.frexp(y)  # y = m * 2^ex, 0.5 <= m < 1
    return max(ex - 1, -126)


def _truncate_value(v, m):
    """|v| truncated to m fraction bits below its leading bit, as a Fraction."""
    V = Fraction(float(v))
    if V == 0:
        return V
    q = Fraction(2) ** (_p(v) - m)
    t = (abs(V) // q) * q
    return t if V > 0 else -t


def _passes(blk, mu, e, m):
    """Truncation-only reconstruction with m mantissa bits meets e exactly."""
    E = Fraction(float(e))
    for x in blk:
        v = np.float32(x - mu)
        vt = _truncate_value(v, m)
        vt32 = np.float32(float(vt))
        assert Fraction(float(vt32)) == vt  # representable: it has few bits
        xr = np.float32(mu + vt32)
        if abs(Fraction(float(x)) - Fraction(float(xr))) > E:
            return False
    return True


def test_p4_bit_budget_brute_force():
    r = rng(23)
    adversarial_checked = 0
    for trial in range(400):
        scale = 10.0 ** r.integers(-6, 6)
        blk = (r.standard_normal(8) * scale + r.standard_normal() * scale * 3).astype(np.float32)
        if trial % 2 == 0:
            # adversarial: a block symmetric about 0 (so mu = 0 and v = x) whose
            # extreme |v| has an all-ones mantissa, the worst case for truncation
            a = np.array([abs(blk[0]) + scale], dtype=np.float32)
            a = (a.view(np.uint32) | np.uint32(0x007FFFFF)).view(np.float32)[0]
            inner = np.clip(blk[2:], -a * 0.99, a * 0.99).astype(np.float32)
            blk = np.concatenate([[a, -a], inner]).astype(np.float32)
        eb = float(10.0 ** r.uniform(-6, -1)) * scale
        s = szref.compress(blk, eb, "abs", 8)
        info = sf.parse(s)
        if not info["state"][0]:
            continue
        e = info["e"]
        mn, mx = blk.min(), blk.max()
        mu = np.float32(np.float32(0.5) * mn + np.float32(0.5) * mx)
        rr = max(abs(np.float32(mx - mu)), abs(np.float32(mn - mu)))
        m0 = max(0, _p(rr) - _p(e))
        passes = [_passes(blk, mu, e, m) for m in range(24)]
        m_bf = passes.index(True) if True in passes else None
        K = int(info["K"][0])
        # the oracle takes the first of m0, m0 + 1 that passes, else raw
        if K == 0xFF:
            assert not passes[min(m0, 23)] and not passes[min(m0 + 1, 23)]
        else:
            m_used = K - 9
            want = m0 if passes[min(m0, 23)] else m0 + 1
            assert m_used == min(want, 23)
            assert m_bf is not None and m_bf <= m_used
        if trial % 2 == 0 and m_bf is not None:
            # eq. (4) is not wasteful: at most one bit beyond the brute-force minimum
            assert m0 <= m_bf + 1
            adversarial_checked += 1
        # with a normal e the truncation alone errs by < 2^(p(r) - m0) <= 2^p(e) <= e
        if e >= np.finfo(np.float32).tiny and m0 <= 23:
            bound = Fraction(2) ** (_p(rr) - m0)
            assert bound <= Fraction(float(e))
    assert adversarial_checked > 50


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_p4_ladder_second_rung_and_raw(dtype):
    """The error-control ladder (error control of Sec. I; Alg. 1's bit
    budget): with a subnormal bound e, 2^p(e) exceeds e, so the first rung
    (K0 kept bits, eq. (4)) can fail; the oracle must then store the block at
    K0 + 1 when that passes, else raw. Outcomes decided by brute force with
    rationals (ladder.py), on hand-made and seeded blocks."""
    import ladder
    W = ladder.spec(dtype)[0]
    for blk, eb, want in ladder.constructed_blocks(dtype):
        s = szref.compress(blk, eb, "abs", 8)
        info = sf.parse(s)
        assert info["state"][0]
        got, K0 = ladder.expected_outcome(blk, info["e"])
        assert got == want and K0 < W
        assert ladder.outcomes_of_stream(blk, info) == [(want, K0)]
        assert within(blk, szref.decompress(s), info["e"])
    seen = {"K0": 0, "K0+1": 0, "raw": 0}
    blocks, bounds = ladder.subnormal_blocks(dtype, 240, 31)
    for blk, e in zip(blocks, bounds):
        s = szref.compress(blk, float(e), "abs", 8)
        info = sf.parse(s)
        assert info["e"] == e
        if not info["state"][0]:
            continue
        want, K0 = ladder.expected_outcome(blk, e)
        assert ladder.outcomes_of_stream(blk, info) == [(want, K0)], (blk, e)
        seen[want] += 1
        assert within(blk, szref.decompress(s), e)
    assert min(seen.values()) >= 5, seen


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("block", [8, 128])
def test_p4_ladder_field_outcomes(dtype, block):
    """The field the GPU ladder test uses: every non-constant block's stored
    outcome (K0, K0 + 1 or raw) equals the brute-force outcome, and each
    outcome occurs many times."""
    import ladder
    x, eb = ladder.subnormal_field(dtype, 400, block, 7)
    s = szref.compress(x, eb, "abs", block)
    info = sf.parse(s)
    got = ladder.outcomes_of_stream(x, info)
    ks = np.nonzero(info["state"])[0]
    assert len(got) == len(ks)
    for k, (o, K0) in zip(ks, got):
        want, K0w = ladder.expected_outcome(np.ascontiguousarray(x[k * block:(k + 1) * block]), info["e"])
        assert (o, K0) == (want, K0w), k
    counts = {o: sum(1 for g, _ in got if g == o) for o in ("K0", "K0+1", "raw")}
    assert min(counts.values()) >= 40, counts
    assert within(x, szref.decompress(s), info["e"])


def test_p4_truncation_bound_exhaustive_window():
    """For every float32 |v| <= r in a window of binades, keeping m0 mantissa
    bits errs by < 2^(p(r) - m0) (the bound eq. (4) relies on)."""
    for p_r, m0 in [(-3, 5), (0, 11), (4, 2)]:
        lo = np.float32(2.0 ** (p_r - 3))
        hi = np.float32(2.0 ** (p_r + 1))  # r < 2^(p_r+1)
        u = np.arange(lo.view(np.uint32), hi.view(np.uint32), dtype=np.uint32)
        v = u.view(np.float32).astype(np.float64)
        ex = np.floor(np.log2(v))
        q = np.exp2(ex - m0)
        t = np.floor(v / q) * q  # exact in double: few bits
        assert np.all(v - t < 2.0 ** (p_r - m0))
        assert np.all(v - t >= 0)


# ---------------------------------------- P5: the paper's worked example ---

def test_p5_worked_example_codes_and_bytes():
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    vals = np.array(g["values"], dtype=np.float32)
    assert [hex(int(u)) for u in vals.view(np.uint32)] == g["float32_bits"]
    # a block whose mid value is exactly 0, so the normalized values are the
    # printed ones; a tiny bound keeps all 32 bits (s = 0)
    blk = np.array(list(vals) + [-vals.max(), 0.0, 0.0, 0.0, 0.0], dtype=np.float32)
    s = szref.compress(blk, 1e-30, "abs", 8)
    info = sf.parse(s)
    assert info["mu"][0] == 0.0 and info["K"][0] == 32
    codes = sf.unpack_codes(info["codes"][0], 8)
    assert codes[:3] == g["identical_leading_bytes"]
    # kept bytes of the first three values, most significant first
    want = bytes.fromhex("3dfcb924" + "ed91" + "f80347")
    assert bytes(info["mid"][:9]) == want


# ------------------------------------ P6: decode of leading-byte sources ---

def _build_stream(dtype_code, b, n, blocks):
    """Assemble a stream by hand from per-block records (test fixture)."""
    import struct
    w = 4 if dtype_code == 0 else 8
    nblk = (n + b - 1) // b
    nc = [blk for blk in blocks if blk["state"]]
    mid = b"".join(blk.get("mid", b"") for blk in nc)
    hdr = struct.pack("<IBBBBII", 0x4D585A53, 1, dtype_code, 0, 1, b, 0)
    hdr += struct.pack("<4Q", n, 0, 0, 0) + struct.pack("<Q", n) + struct.pack("<d", 0.0)
    hdr += struct.pack("<4Q", 0, nblk, len(nc), len(mid))
    a16 = lambda x: (x + 15) & ~15
    out = bytearray(hdr)
    st = bytearray((nblk + 7) // 8)
    for k, blk in enumerate(blocks):
        if blk["state"]:
            st[k // 8] |= 1 << (k % 8)
    out += st
    out += bytes(a16(len(out)) - len(out))
    for blk in blocks:
        out += struct.pack("<I" if w == 4 else "<Q", blk["mu_bits"])
    out += bytes(a16(len(out)) - len(out))
    out += bytes(blk["K"] for blk in nc)
    out += bytes(a16(len(out)) - len(out))
    for blk in nc:
        cb = bytearray(b // 4)
        for i, c in enumerate(blk["codes"]):
            cb[i // 4] |= c << (6 - 2 * (i % 4))
        out += cb
    out += bytes(a16(len(out)) - len(out))
    out += mid
    return np.frombuffer(bytes(out), dtype=np.uint8)


def golden_index_propagation_stream():
    g = json.load(open(os.path.join(GOLDEN, "decode_index_propagation.json")))
    blk = dict(state=1, mu_bits=int(g["mu_bits"], 16), K=g["K"], codes=g["codes"],
               mid=bytes.fromhex(g["mid_hex"]))
    stream = _build_stream(0, g["block_size"], 8, [blk])
    want = np.array([int(h, 16) for h in g["expected_bits"]], dtype=np.uint32)
    return stream, want


def test_p6_index_propagation_golden():
    stream, want = golden_index_propagation_stream()
    y = szref.decompress(stream)
    assert np.array_equal(y.view(np.uint32), want)


# ----------------------------------------------- P7: sizes and eq. (5) ---

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("block", [8, 32, 128, 512])
def test_p7_sizes_and_shift(dtype, block):
    x = smooth_field(20000 + 37, 13, dtype)
    x[block * 3 + 1] = np.nan  # one raw block
    for eb in [1e-2, 1e-4]:
        s = szref.compress(x, eb, "rel", block)
        info = sf.parse(s)
        assert info["offsets"]["total"] == len(s)
        W = 32 if dtype == np.float32 else 64
        mid = 0
        for r in range(info["n_nc"]):
            K = int(info["K"][r])
            k = int(np.nonzero(info["state"])[0][r])
            nk = sf.block_len(info, k)
            if K == 0xFF:
                mid += nk * info["w"]
                continue
            nb, sh = sf.nb_of(K)
            assert (K + sh) % 8 == 0 and 0 <= sh <= 7  # eq. (5)
            assert 1 + (8 if W == 32 else 11) <= K <= W
            codes = sf.unpack_codes(info["codes"][r], nk)
            assert max(codes) <= min(3, nb)
            mid += sum(nb - c for c in codes)
        assert mid == info["mid_total"]
        assert int(info["n_nc"]) == int(info["state"].sum())


# ------------------------------------------------------- P8: PSNR bound ---

@pytest.mark.parametrize("eb", [1e-2, 4e-3, 1e-3, 1e-4])
def test_p8_psnr_lower_bound(eb):
    x = smooth_field(1 << 16, 19, np.float32)
    y = szref.decompress(szref.compress(x, eb, "rel", 128))
    d = x.astype(np.float64) - y.astype(np.float64)
    mse = float(np.mean(d * d))
    rng_ = float(x.max()) - float(x.min())
    psnr = 20 * math.log10(rng_ / math.sqrt(mse)) if mse > 0 else math.inf
    assert psnr >= -20 * math.log10(eb)  # eq. (7) with RMSE <= e
    # consistent with the paper's Hurricane figures: 74.4, 62, 54.6 dB
    for p_, e_ in [(74.4, 1e-3), (62.0, 4e-3), (54.6, 1e-2)]:
        assert p_ >= -20 * math.log10(e_)


# -------------------------------------------------- P9: closed forms ---

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_p9_ramp_constant_iff_slope_fits(dtype):
    b = 128
    i = np.arange(b * 64)
    for a, e in [(2.0 ** -10, 2.0 ** -10 * 127 / 2), (2.0 ** -10, 2.0 ** -10 * 126 / 2)]:
        x = (a * i).astype(dtype)
        s = szref.compress(x, e, "abs", b)
        info = sf.parse(s)
        const = a * (b - 1) <= 2 * e
        assert bool((~info["state"]).all()) == const
        assert bool(info["state"].all()) == (not const)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_p9_zero_bound_is_value_exact(dtype):
    x = smooth_field(5000, 29, dtype)
    y = szref.decompress(szref.compress(x, 0.0, "abs", 64))
    assert np.array_equal(x, y)  # -0 and +0 compare equal


def test_p9_constant_field():
    x = np.full((10, 30, 7), -2.5, np.float32)
    s = szref.compress(x, 1e-3, "rel", 16)
    info = sf.parse(s)
    assert info["n_nc"] == 0
    assert np.array_equal(szref.decompress(s), x)


# ------------------------------------------ raw blocks and edge cases ---

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_raw_blocks_bit_identical(dtype):
    x = smooth_field(1000, 31, dtype)
    x[5] = np.nan
    x[300] = np.inf
    x[301] = -np.inf
    s = szref.compress(x, 1e-3, "rel", 128)
    y = szref.decompress(s)
    info = sf.parse(s)
    for k in (0, 2):
        sl = slice(k * 128, (k + 1) * 128)
        assert np.array_equal(x[sl].view(info["udtype"]), y[sl].view(info["udtype"]))
    ok = np.isfinite(x)
    assert within(x[ok], y[ok], szref.error_bound(x, 1e-3, "rel", 128))


def test_empty_and_ragged():
    x = np.zeros(0, np.float32)
    s = szref.compress(x, 1e-3, "rel", 128)
    assert len(s) == 96
    assert szref.decompress(s).size == 0
    for n in [1, 7, 127, 129, 1000, 1023]:
        x = smooth_field(n, n, np.float32)
        s = szref.compress(x, 1e-3, "rel", 128)
        y = szref.decompress(s)
        assert within(x, y, szref.error_bound(x, 1e-3, "rel", 128))


def test_invalid_params():
    x = np.zeros(16, np.float32)
    for kw in [dict(block=7), dict(block=2048), dict(block=4), dict(eb=-1.0), dict(eb=float("nan"))]:
        args = dict(eb=1e-3, mode="rel", block=128)
        args.update(kw)
        with pytest.raises(szref.OracleError):
            szref.compress(x, args["eb"], args["mode"], args["block"])


# ---------------------------------------- P10: determinism, corruption ---

def test_p10_deterministic():
    x = smooth_field(50000, 37, np.float32)
    a = szref.compress(x, 1e-3, "rel", 128)
    b = szref.compress(x.copy(), 1e-3, "rel", 128)
    assert np.array_equal(a, b)


def test_decoder_rejects_corruption_without_crashing():
    x = smooth_field(4096, 41, np.float32)
    s = szref.compress(x, 1e-3, "rel", 64)
    info = sf.parse(s)
    r = rng(43)
    statuses = set()
    for trial in range(300):
        c = s.copy()
        pos = int(r.integers(0, len(c)))
        c[pos] ^= np.uint8(1 << int(r.integers(0, 8)))
        statuses.add(szref.decompress_status(c))
    for cut in [0, 50, 96, info["offsets"]["K"], len(s) - 1]:
        statuses.add(szref.decompress_status(s[:cut]))
    assert statuses <= {szref.OK, szref.ECORRUPT}
    assert szref.ECORRUPT in statuses
    # a bad K byte is caught
    c = s.copy()
    c[info["offsets"]["K"]] = 3
    assert szref.decompress_status(c) == szref.ECORRUPT
