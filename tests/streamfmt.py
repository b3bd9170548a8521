"""Reader of the compressed stream layout, for tests only.

Splits a stream into its header fields and sections and expands the per-block
records (state, mu, K, codes, mid-byte slices) so that tests can check them
against what the paper fixes. It decodes nothing numerically.
"""
import struct

import numpy as np

HDR = 96


def _a16(x):
    return (x + 15) & ~15


def parse(stream):
    s = bytes(np.asarray(stream, dtype=np.uint8))
    (magic, ver, dtype, ebm, ndims, b, _res) = struct.unpack_from("<IBBBBII", s, 0)
    dims = struct.unpack_from("<4Q", s, 16)
    n, = struct.unpack_from("<Q", s, 48)
    eb, = struct.unpack_from("<d", s, 56)
    e_bits, nblk, n_nc, mid_total = struct.unpack_from("<4Q", s, 64)
    w = 4 if dtype == 0 else 8
    state_off = HDR
    mu_off = _a16(state_off + (nblk + 7) // 8)
    k_off = _a16(mu_off + nblk * w)
    codes_off = _a16(k_off + n_nc)
    mid_off = _a16(codes_off + n_nc * (b // 4))
    total = mid_off + mid_total
    tdt = np.float32 if dtype == 0 else np.float64
    udt = np.uint32 if dtype == 0 else np.uint64
    e = np.frombuffer(struct.pack("<Q", e_bits)[:w], dtype=tdt)[0]
    state = np.unpackbits(np.frombuffer(s, np.uint8, (nblk + 7) // 8, state_off),
                          bitorder="little")[:nblk].astype(bool)
    mu = np.frombuffer(s, tdt, nblk, mu_off)
    K = np.frombuffer(s, np.uint8, n_nc, k_off)
    codes = np.frombuffer(s, np.uint8, n_nc * (b // 4), codes_off).reshape(n_nc, b // 4)
    return dict(magic=magic, version=ver, dtype=tdt, udtype=udt, w=w, eb_mode=ebm,
                ndims=ndims, b=b, dims=dims[:ndims], n=n, eb=eb, e=e, nblk=nblk,
                n_nc=n_nc, mid_total=mid_total, state=state, mu=mu, K=K,
                codes=codes, mid=np.frombuffer(s, np.uint8, mid_total, mid_off),
                offsets=dict(state=state_off, mu=mu_off, K=k_off, codes=codes_off,
                             mid=mid_off, total=total), raw=s)


def unpack_codes(row, count):
    """The 2-bit codes of one block, first element in the top bits of byte 0."""
    out = []
    for i in range(count):
        out.append((int(row[i // 4]) >> (6 - 2 * (i % 4))) & 3)
    return out


def block_len(info, k):
    return min(info["b"], info["n"] - k * info["b"])


def nb_of(K):
    s = (8 - K % 8) % 8
    return (K + s) // 8, s
