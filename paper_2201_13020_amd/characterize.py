"""Characterisations of the method on synthetic fields (analysis, not part of
the compression path; it runs the HIP path through the C ABI and inspects
its streams with torch on the device).

* block_range_cdf: the CDF of a block's relative value range, the block's
  max - min over the field's global finite range (Sec. III, the CDF figure
  of block value ranges), at several block sizes.
* block_size_sweep: compression ratio and PSNR against the block size
  (Sec. IV-C, the exploration of block sizes), with the maximum error over
  the bound.
* space_overhead: eq. (6). The extra bytes that the right shift of eq. (5)
  stores, over the compressed size. With the shift, a value of a non-constant
  block stores nb - c_i whole bytes (nb = (K + s) / 8, c_i its leading-byte
  code). Without it, the K kept bits less the identical leading bytes of the
  unshifted K-bit words, 8 c0_i bits, c0_i = min(3, floor(K / 8),
  identical leading bytes of q0_i and q0_(i-1)), q0 the top K bits of
  v = fl(x - mu), zero before each block's first value. Raw blocks store the
  same in both and are left out.

Run: python -m paper_2201_13020_amd.characterize --out result.json [--markdown result.md]
"""
import argparse
import json
import math
import struct

import numpy as np
import torch

from . import szx, synth


def _finite_range(x):
    f = x[torch.isfinite(x)]
    if f.numel() == 0:
        return 0.0
    return float(f.max().double() - f.min().double())


def block_range_cdf(x, blocks=(8, 16, 32, 64, 128), thresholds=(1e-4, 1e-3, 1e-2, 1e-1)):
    """{block: {threshold: fraction of blocks whose relative range <= it}}."""
    x = x.reshape(-1)
    g = _finite_range(x)
    out = {}
    for b in blocks:
        n = x.numel() // b * b
        xb = x[:n].reshape(-1, b).double()
        rr = (xb.amax(1) - xb.amin(1))
        if n < x.numel():
            t = x[n:].double()
            rr = torch.cat([rr, (t.max() - t.min()).reshape(1)])
        rr = rr / g if g > 0 else torch.zeros_like(rr)
        out[b] = {thr: round(float((rr <= thr).double().mean()), 5) for thr in thresholds}
    return out


def _roundtrip(x, eb, block, dims):
    out, size = szx.compress(x, eb, "rel", block, dims=dims)
    torch.cuda.synchronize()
    n = int(size.cpu().view(torch.int64).item())
    y, st = szx.decompress(out, n, dict(dtype=x.dtype, dims=dims, block=block))
    torch.cuda.synchronize()
    assert int(st.cpu().view(torch.int32).item()) == 0
    return out[:n], y


def block_size_sweep(x, ebs=(1e-3, 1e-4), blocks=(8, 16, 32, 64, 128, 256, 512, 1024)):
    """[{eb, block, ratio, psnr_db, max_err_over_e}] for a device field."""
    dims = tuple(x.shape)
    g = _finite_range(x)
    xd = x.reshape(-1).double()
    rows = []
    for eb in ebs:
        for b in blocks:
            s, y = _roundtrip(x, eb, b, dims)
            hdr = s[:96].cpu().numpy().tobytes()
            e_bits = struct.unpack_from("<Q", hdr, 64)[0]
            e = struct.unpack("<d", struct.pack("<Q", e_bits))[0] if x.dtype == torch.float64 else \
                struct.unpack("<f", struct.pack("<I", e_bits & 0xFFFFFFFF))[0]
            err = (xd - y.double()).abs()
            mse = float((err * err).mean())
            psnr = 20 * math.log10(g) - 10 * math.log10(mse) if mse > 0 else float("inf")
            rows.append(dict(eb=eb, block=b, ratio=round(x.numel() * x.element_size() / s.numel(), 4),
                             psnr_db=round(psnr, 3), max_err_over_e=round(float(err.max()) / e, 5) if e > 0 else 0.0))
    return rows


def _sections(nblk, n_nc, w, b, mid_total):
    a16 = lambda v: (v + 15) // 16 * 16
    st = 96
    mu = a16(st + (nblk + 7) // 8)
    kb = a16(mu + nblk * w)
    codes = a16(kb + n_nc)
    mid = a16(codes + n_nc * (b // 4))
    return dict(state=st, mu=mu, K=kb, codes=codes, mid=mid, total=a16(mid + mid_total))


def space_overhead(x, stream, block):
    """Eq. (6) for one compressed field. Returns the stored bits with the
    shift (as the stream holds them), without it, and the overhead."""
    x = x.reshape(-1)
    w = x.element_size()
    W = 8 * w
    hdr = stream[:96].cpu().numpy().tobytes()
    n = struct.unpack_from("<Q", hdr, 48)[0]
    nblk, n_nc, mid_total = struct.unpack_from("<3Q", hdr, 72)
    sec = _sections(nblk, n_nc, w, block, mid_total)
    dev = x.device
    st = stream[sec["state"]:sec["state"] + (nblk + 7) // 8]
    bitpos = torch.arange(8, device=dev, dtype=torch.uint8)
    state = ((st.unsqueeze(1) >> bitpos) & 1).reshape(-1)[:nblk].bool()
    nc_blocks = torch.nonzero(state).reshape(-1)
    K = stream[sec["K"]:sec["K"] + n_nc].long()
    keep = K != 0xFF  # raw blocks are the same either way
    blocks = nc_blocks[keep]
    K = K[keep]
    if blocks.numel() == 0:
        return dict(bits_shifted=0, bits_unshifted=0, overhead=0.0, stream_bytes=int(stream.numel()))
    codes_all = stream[sec["codes"]:sec["codes"] + n_nc * (block // 4)].reshape(n_nc, block // 4)[keep]
    shifts = torch.tensor([6, 4, 2, 0], device=dev, dtype=torch.uint8)
    c = ((codes_all.unsqueeze(2) >> shifts) & 3).reshape(-1, block).long()
    mu = stream[sec["mu"]:sec["mu"] + nblk * w].view(x.dtype)
    idx = blocks.unsqueeze(1) * block + torch.arange(block, device=dev).unsqueeze(0)
    valid = idx < n
    xv = x[idx.clamp(max=n - 1)]
    v = xv - mu[blocks].unsqueeze(1)  # fl(x - mu) in the element type
    # the IEEE words as int64 (float64: two's complement of the 64-bit word)
    bits = v.view(torch.int32).long() & 0xFFFFFFFF if w == 4 else v.view(torch.int64)
    s = (8 - K % 8) % 8
    nb = (K + s) // 8
    # with the shift: nb - c stored bytes per valid value
    shifted = ((nb.unsqueeze(1) - c) * 8 * valid).sum()
    # without: the top K bits, leading identical bytes of consecutive words
    low = (torch.ones_like(K) << (W - K)) - 1
    topmask = ~low if w == 8 else (~low) & 0xFFFFFFFF
    q0 = bits & topmask.unsqueeze(1)
    prev = torch.cat([torch.zeros_like(q0[:, :1]), q0[:, :-1]], 1)
    diff = q0 ^ prev
    lead = torch.zeros_like(diff)
    for j in range(3):  # identical leading bytes, at most 3
        byte_j = (diff >> (W - 8 * (j + 1))) & 0xFF
        lead = torch.where((lead == j) & (byte_j == 0), lead + 1, lead)
    c0 = torch.minimum(lead, (K // 8).unsqueeze(1).expand_as(lead))
    unshifted = ((K.unsqueeze(1) - 8 * c0) * valid).sum()
    shifted, unshifted = int(shifted), int(unshifted)
    return dict(bits_shifted=shifted, bits_unshifted=unshifted, stream_bytes=int(stream.numel()),
                overhead=round((shifted - unshifted) / (8.0 * stream.numel()), 6))


def _fields(small):
    if small:
        return {"turbulence 40x100x100": synth.turbulence_3d((40, 100, 100)),
                "sphere 180x360": synth.sphere_2d(180, 360),
                "sines 2^18": synth.sines_1d(1 << 18)}
    return {"turbulence 100x500x500": synth.make("turbulence"),
            "sphere 1800x3600": synth.make("sphere"),
            "sines 2^20": synth.make("sines")}


def run(small=False):
    out = {"cdf": {}, "sweep": {}, "overhead": {}}
    for name, xh in _fields(small).items():
        x = torch.from_numpy(np.ascontiguousarray(xh)).cuda()
        out["cdf"][name] = block_range_cdf(x)
        out["sweep"][name] = block_size_sweep(x)
        rows = []
        for eb in (1e-2, 1e-3, 1e-4):
            for b in (8, 16, 32, 64, 128):
                s, _ = _roundtrip(x, eb, b, tuple(x.shape))
                r = space_overhead(x, s, b)
                r.update(eb=eb, block=b)
                rows.append(r)
        out["overhead"][name] = rows
    return out


def markdown(res):
    """The results as markdown tables: eq. (6) overhead per field, bound and
    block size; compression ratio and PSNR per block size; the block-range
    CDF."""
    lines = ["## Eq. (6) space overhead of the right shift (raw blocks left out)", "",
             "| field | REL | " + " | ".join(f"b = {b}" for b in (8, 16, 32, 64, 128)) + " |",
             "|---|---|" + "---|" * 5]
    for name, rows in res["overhead"].items():
        for eb in (1e-2, 1e-3, 1e-4):
            cells = []
            for b in (8, 16, 32, 64, 128):
                r = [x for x in rows if float(x["eb"]) == eb and int(x["block"]) == b]
                cells.append(f"{100 * r[0]['overhead']:.1f} %" if r else "-")
            lines.append(f"| {name} | {eb:g} | " + " | ".join(cells) + " |")
    blocks = (8, 16, 32, 64, 128, 256, 512, 1024)
    lines += ["", "## Compression ratio / PSNR (dB) against block size (max error / e in brackets)", "",
              "| field | REL | " + " | ".join(f"b = {b}" for b in blocks) + " |", "|---|---|" + "---|" * len(blocks)]
    for name, rows in res["sweep"].items():
        for eb in sorted({float(r["eb"]) for r in rows}, reverse=True):
            cells = []
            for b in blocks:
                r = [x for x in rows if float(x["eb"]) == eb and int(x["block"]) == b]
                cells.append(f"{r[0]['ratio']:.2f} / {r[0]['psnr_db']:.1f} ({r[0]['max_err_over_e']:.3f})"
                             if r else "-")
            lines.append(f"| {name} | {eb:g} | " + " | ".join(cells) + " |")
    lines += ["", "## Fraction of blocks whose relative value range is at most a threshold", ""]
    for name, cdf in res["cdf"].items():
        thr = sorted({float(t) for col in cdf.values() for t in col})
        lines += [f"{name}:", "", "| block | " + " | ".join(f"<= {t:g}" for t in thr) + " |",
                  "|---|" + "---|" * len(thr)]
        for b, col in cdf.items():
            vals = {float(t): v for t, v in col.items()}
            lines.append(f"| {b} | " + " | ".join(f"{vals[t]:.4f}" for t in thr) + " |")
        lines.append("")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="write the results as JSON")
    ap.add_argument("--small", action="store_true")
    ap.add_argument("--from-json", default=None, help="format results written earlier instead of running")
    ap.add_argument("--markdown", default=None, help="write the results as markdown tables")
    a = ap.parse_args()
    res = json.load(open(a.from_json)) if a.from_json else run(a.small)
    text = json.dumps(res, indent=1, default=str)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    if a.markdown:
        with open(a.markdown, "w") as f:
            f.write(markdown(res))
    print(text)


if __name__ == "__main__":
    main()
