"""Seeded, bounded fuzzing of the GPU decoder with corrupted streams.

The decoder's contract: every read of the stream stays below in_bytes, every
write stays inside the output, and a malformed stream reports SZ_ECORRUPT
(3) through the device status word; nothing else. Each case corrupts a clean
stream written by the oracle -- header fields, state bits, mu, K bytes, code
bytes, mid bytes, truncations, bursts of random bytes -- and decodes it into
an output with guard regions on both sides. Every status must be 0 or 3;
corruptions whose outcome the format fixes must give exactly that outcome
(a header size field or a state bit changed, a K byte outside [1 + E, W], a
truncation: 3; a mu or mid byte changed: 0, and only the values of the block
that owns the byte may change). A stream that the oracle's decoder accepts
must decode to the oracle's values. A decode of the clean stream with the
same workspace after corrupted ones must still equal the oracle's values.
"""
import numpy as np
import pytest

from oracle import szref
import streamfmt as sf
from gpu_util import same_bits

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GUARD = 1024  # elements of sentinel before and after the output
CASES = 160


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_13020_amd import szx
    szx.lib()


def field(n, dtype, seed):
    """Smooth waves with a zero run (constant blocks) and scattered NaN/inf
    (raw blocks)."""
    r = np.random.default_rng(seed)
    t = np.arange(n) / n
    x = np.zeros(n)
    for _ in range(4):
        x += r.uniform(0.2, 2) * np.sin(2 * np.pi * r.uniform(1, 200) * t + r.uniform(0, 6.28))
    x += 1e-3 * r.standard_normal(n)
    x[(t > 0.3) & (t < 0.36)] = 0.0
    x[r.choice(n, 12, replace=False)] = np.nan
    x[r.choice(n, 6, replace=False)] = np.inf
    return x.astype(dtype)


def mid_owner(info):
    """First mid byte of every block (nblk + 1 entries): the stored bytes of
    a coded value are its kept bytes less its leading-byte code; a raw block
    stores its words whole; a constant block stores none."""
    b, w, nblk, n = info["b"], info["w"], info["nblk"], info["n"]
    nc = np.nonzero(info["state"])[0]
    nk = np.minimum(b, n - nc * b)
    K = info["K"].astype(np.int64)
    codes = ((info["codes"][:, :, None] >> np.array([6, 4, 2, 0], np.uint8)) & 3).reshape(len(nc), b)
    live = np.arange(b)[None, :] < nk[:, None]
    nb = (K + 7) // 8
    coded = nb * nk - (codes * live).sum(1)
    per = np.where(K == 0xFF, nk * w, coded)
    size = np.zeros(nblk, np.int64)
    size[nc] = per
    return np.concatenate([[0], np.cumsum(size)])


class Decoder:
    """Decodes host streams with one device workspace and a guarded output."""

    def __init__(self, exp, n, dtype):
        from paper_2201_13020_amd import szx
        self.szx = szx
        self.exp = exp
        self.n = n
        self.tdt = torch.float32 if dtype == np.float32 else torch.float64
        self.udt = np.uint32 if dtype == np.float32 else np.uint64
        wsz = szx.workspace_size(exp["dtype"], exp["dims"], exp["eb"], exp["mode"], exp["block"])
        self.ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")
        self.big = torch.empty(n + 2 * GUARD, dtype=self.tdt, device="cuda")
        self.sentinel = torch.full((GUARD,), -7.25, dtype=self.tdt, device="cuda")
        self.status = torch.empty(1, dtype=torch.uint32, device="cuda")

    def __call__(self, stream, in_bytes=None):
        s = np.ascontiguousarray(stream, dtype=np.uint8)
        d = torch.from_numpy(s.copy() if s.size else np.zeros(16, np.uint8)).cuda()
        self.big[:GUARD] = self.sentinel
        self.big[GUARD + self.n:] = self.sentinel
        out = self.big[GUARD:GUARD + self.n]
        self.szx.decompress(d, s.size if in_bytes is None else in_bytes, self.exp, out=out, status=self.status,
                            ws=self.ws)
        torch.cuda.synchronize()
        assert torch.equal(self.big[:GUARD], self.sentinel), "write before the output"
        assert torch.equal(self.big[GUARD + self.n:], self.sentinel), "write after the output"
        return out.cpu().numpy().view(self.udt), int(self.status.cpu().view(torch.int32).item())


def same_or_nan(a_bits, b_bits):
    """Equal words, or NaN on both sides (a corrupted mu can make mu + d a
    NaN, whose payload the IEEE standard leaves open)."""
    ft = np.float32 if a_bits.dtype == np.uint32 else np.float64
    both_nan = np.isnan(a_bits.view(ft)) & np.isnan(b_bits.view(ft))
    return bool(np.all((a_bits == b_bits) | both_nan))


CONFIGS = [(np.float32, 8, 70_037), (np.float32, 128, 70_037), (np.float32, 1024, 70_037),
           (np.float64, 16, 40_011), (np.float64, 128, 40_011), (np.float64, 512, 40_011)]


@pytest.mark.parametrize("dtype,block,n", CONFIGS, ids=[f"{np.dtype(c[0]).name}-b{c[1]}" for c in CONFIGS])
def test_corrupted_streams(dtype, block, n):
    seed = 1000 * block + np.dtype(dtype).itemsize
    print(f"[fuzz] dtype={np.dtype(dtype).name} b={block} n={n} seed={seed}", flush=True)
    x = field(n, dtype, seed)
    ref = szref.compress(x, 1e-3, "rel", block)
    info = sf.parse(ref)
    off = info["offsets"]
    total = off["total"]
    assert info["n_nc"] > 10 and not info["state"].all()
    assert (info["K"] == 0xFF).any() and ((info["K"] != 0xFF).sum() > 10)
    want = szref.decompress(ref).ravel().view(np.uint32 if dtype == np.float32 else np.uint64)
    from paper_2201_13020_amd import szx
    exp = szx.inspect(ref[:96].tobytes())
    dec = Decoder(exp, n, dtype)
    y, st = dec(ref)
    assert st == 0 and np.array_equal(y, want)

    w = info["w"]
    kmin, W = (9, 32) if dtype == np.float32 else (12, 64)
    starts = mid_owner(info)
    assert starts[-1] == info["mid_total"]
    r = np.random.default_rng(seed)
    stats = {}

    def blocks_outside(yc, k_lo, k_hi):
        lo, hi = k_lo * block, min(n, k_hi * block)
        return np.array_equal(yc[:lo], want[:lo]) and np.array_equal(yc[hi:], want[hi:])

    for case in range(CASES):
        kind = ["header_field", "header_byte", "state", "mu", "K_bad", "K_any", "codes", "mid",
                "truncate", "burst", "multi", "body"][case % 12]
        c = ref.copy()
        in_bytes = None
        fixed = None  # the status the format fixes, if it does
        k_own = None
        if kind == "header_field":
            # a checked field: magic, version, element type, ndims, b, dims, n, nblk, n_nc, mid_total
            f = int(r.integers(0, 10))
            at = [0, 4, 5, 7, 8, 16, 48, 72, 80, 88][f]
            c[at] ^= np.uint8(r.integers(1, 256))
            fixed = 3
        elif kind == "header_byte":
            c[int(r.integers(0, 96))] ^= np.uint8(r.integers(1, 256))
        elif kind == "state":
            k = int(r.integers(0, info["nblk"]))
            c[off["state"] + k // 8] ^= np.uint8(1 << (k % 8))
            fixed = 3
        elif kind == "mu":
            k = int(r.integers(0, info["nblk"]))
            c[off["mu"] + k * w + int(r.integers(0, w))] ^= np.uint8(r.integers(1, 256))
            fixed, k_own = 0, k
        elif kind == "K_bad":
            rank = int(r.integers(0, info["n_nc"]))
            bad = [v for v in range(256) if v != 0xFF and not kmin <= v <= W]
            c[off["K"] + rank] = bad[int(r.integers(0, len(bad)))]
            fixed = 3
        elif kind == "K_any":
            c[off["K"] + int(r.integers(0, info["n_nc"]))] = np.uint8(r.integers(0, 256))
        elif kind == "codes":
            for _ in range(int(r.integers(1, 4))):
                c[off["codes"] + int(r.integers(0, info["n_nc"] * (block // 4)))] = np.uint8(r.integers(0, 256))
        elif kind == "mid":
            if info["mid_total"] == 0:
                continue
            m = int(r.integers(0, info["mid_total"]))
            c[off["mid"] + m] ^= np.uint8(r.integers(1, 256))
            fixed, k_own = 0, int(np.searchsorted(starts, m, side="right") - 1)
        elif kind == "truncate":
            in_bytes = int(r.integers(0, total))
            c = c[:max(in_bytes, 1)].copy()
            fixed = 3
        elif kind == "burst":
            at = int(r.integers(96, total))
            ln = int(min(r.integers(1, 65), total - at))
            c[at:at + ln] = r.integers(0, 256, ln, dtype=np.uint8)
        elif kind == "multi":
            for _ in range(int(r.integers(2, 6))):
                at = int(r.integers(0, total))
                c[at] ^= np.uint8(r.integers(1, 256))
        else:  # the header kept, every other byte random
            c[96:] = r.integers(0, 256, total - 96, dtype=np.uint8)
        yc, st = dec(c, in_bytes)
        stats[(kind, st)] = stats.get((kind, st), 0) + 1
        assert st in (0, 3), (case, kind, st)
        if fixed is not None:
            assert st == fixed, (case, kind, st)
        # a stream that the oracle's decoder accepts decodes to its values
        cref = c[:in_bytes] if in_bytes is not None else c
        if szref.decompress_status(cref) == 0:
            assert st == 0, (case, kind)
            assert same_or_nan(yc, szref.decompress(cref).ravel().view(yc.dtype)), (case, kind)
        if k_own is not None:
            assert blocks_outside(yc, k_own, k_own + 1), (case, kind, k_own)
        if case % 16 == 15:
            y, st = dec(ref)
            assert st == 0 and np.array_equal(y, want), case
    print(f"[fuzz] outcomes {sorted(stats.items())}", flush=True)
    # the random kinds reach both outcomes somewhere in the run
    assert any(k == "body" and s == 3 for k, s in stats)


def test_corrupted_fields_in_a_batch():
    """A decompression batch of clean and corrupted streams: each field's
    status is its own, and the clean fields decode exactly."""
    from paper_2201_13020_amd import szx
    print("[fuzz] batch of 16 fields", flush=True)
    r = np.random.default_rng(77)
    streams, nbytes, exps, wants, corrupt = [], [], [], [], []
    for i in range(16):
        dtype = np.float32 if i % 2 == 0 else np.float64
        n = int(r.integers(5_000, 30_000))
        x = field(n, dtype, 500 + i)
        ref = szref.compress(x, 1e-3, "rel", 64)
        c = ref.copy()
        bad = i % 4 in (1, 2)
        if bad:
            info = sf.parse(ref)
            if i % 4 == 1:  # a state bit: the rank count no longer matches n_nc
                k = int(r.integers(0, info["nblk"]))
                c[info["offsets"]["state"] + k // 8] ^= np.uint8(1 << (k % 8))
            else:  # random body
                c[96:] = r.integers(0, 256, c.size - 96, dtype=np.uint8)
        streams.append(torch.from_numpy(c).cuda())
        nbytes.append(c.size)
        exps.append(szx.inspect(ref[:96].tobytes()))
        wants.append(szref.decompress(ref).ravel())
        corrupt.append(bad)
    b = szx.decompress_batch(streams, nbytes, exps)
    for t in b.statuses:
        t.fill_(99)  # the batch resets every field's status
    b.run()
    torch.cuda.synchronize()
    for i in range(16):
        st = int(b.statuses[i].cpu().view(torch.int32).item())
        if corrupt[i]:
            assert st == 3 if i % 4 == 1 else st in (0, 3), (i, st)
        else:
            assert st == 0, i
            assert same_bits(b.outs[i].cpu().numpy(), wants[i]), i
    b.close()
