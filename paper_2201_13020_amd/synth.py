"""Seeded synthetic fields standing in for the paper's datasets.

The paper evaluates on SDRBench fields (CESM-ATM, Hurricane, Miranda, Nyx,
QMCPack, SCALE-LetKF; Sec. VI, table of applications), all single precision.
Those files are not available here, so these generators produce fields with
the same shapes and the properties the method depends on: local smoothness
(Sec. IV: most blocks have a small value range) and exact zero regions. They
contain none of the compressor's arithmetic; both the GPU path and the CPU
oracle consume the same arrays.

Seeds: numpy default_rng(13020 + 1000 * stream + field), one stream per workload. Values are generated in
float64 and rounded once to the element type. Zeros are assigned (+0.0), never
produced by multiplying with a mask.
"""
import numpy as np


def _rng(stream, field=0):
    return np.random.default_rng(13020 + 1000 * stream + field)


def sines_1d(n=1 << 20, field=0, noise=1e-3, dtype=np.float32):
    """1-D field: sum of 8 sines with log-uniform frequencies in [1, 4096]
    cycles over the field and uniform phases, plus N(0, noise^2) noise."""
    r = _rng(1, field)
    f = np.exp(r.uniform(np.log(1.0), np.log(4096.0), 8))
    ph = r.uniform(0.0, 2 * np.pi, 8)
    t = np.arange(n, dtype=np.float64) / n
    x = np.zeros(n, dtype=np.float64)
    for j in range(8):
        x += np.sin(2 * np.pi * f[j] * t + ph[j])
    x += noise * r.standard_normal(n)
    return x.astype(dtype)


def _spectral_field(shape, r, slope):
    """Real Gaussian random field with amplitude |k|^slope (k = 0 removed),
    normalised to zero mean and unit standard deviation."""
    white = r.standard_normal(shape)
    F = np.fft.rfftn(white)
    ks = [np.fft.fftfreq(s) for s in shape[:-1]] + [np.fft.rfftfreq(shape[-1])]
    grids = np.meshgrid(*ks, indexing="ij", sparse=True)
    k2 = sum(g * g for g in grids)
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (slope / 2.0), 0.0)
    F *= amp
    del amp, k2
    x = np.fft.irfftn(F, s=shape, axes=tuple(range(len(shape))))
    x -= x.mean()
    sd = x.std()
    if sd > 0:
        x /= sd
    return x


def turbulence_3d(shape=(100, 500, 500), field=0, zero_frac=0.2, dtype=np.float32):
    """3-D field in the shape of a Hurricane field: a Gaussian random field
    whose energy spectrum falls as k^(-5/3) (amplitude |k|^(-11/6) in 3-D),
    with exact-zero regions where a second, smoother field (|k|^-3) lies
    below its zero_frac quantile."""
    r = _rng(2, field)
    x = _spectral_field(shape, r, -11.0 / 6.0)
    if zero_frac > 0:
        m = _spectral_field(shape, r, -3.0)
        thr = np.quantile(m, zero_frac)
        x[m < thr] = 0.0
    return x.astype(dtype)


def _legendre_rows(lmax, x):
    """Fully normalised associated Legendre values P[l][m] at the points x
    (standard recurrences in m then l)."""
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    P = np.zeros((lmax + 1, lmax + 1, x.size))
    P[0, 0] = 1.0
    for m in range(1, lmax + 1):
        P[m, m] = np.sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * P[m - 1, m - 1]
    for m in range(0, lmax):
        P[m + 1, m] = np.sqrt(2.0 * m + 3.0) * x * P[m, m]
    for m in range(0, lmax + 1):
        for l in range(m + 2, lmax + 1):
            a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = np.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
            P[l, m] = a * (x * P[l - 1, m] - b * P[l - 2, m])
    return P


def sphere_2d(nlat=1800, nlon=3600, lmax=64, field=0, dtype=np.float32):
    """2-D latitude-longitude field in the shape of a CESM-ATM field: a sum of
    spherical harmonics up to degree lmax with N(0, (l+1)^-2) coefficients."""
    r = _rng(3, field)
    a = r.standard_normal((lmax + 1, lmax + 1)) / (np.arange(lmax + 1)[:, None] + 1.0)
    b = r.standard_normal((lmax + 1, lmax + 1)) / (np.arange(lmax + 1)[:, None] + 1.0)
    b[:, 0] = 0.0
    l_idx, m_idx = np.meshgrid(np.arange(lmax + 1), np.arange(lmax + 1), indexing="ij")
    a[m_idx > l_idx] = 0.0
    b[m_idx > l_idx] = 0.0
    theta = (np.arange(nlat) + 0.5) * np.pi / nlat
    P = _legendre_rows(lmax, np.cos(theta))  # [l, m, lat]
    A = np.einsum("lm,lmt->tm", a, P)  # cos coefficients per latitude
    Bc = np.einsum("lm,lmt->tm", b, P)
    spec = np.zeros((nlat, nlon // 2 + 1), dtype=np.complex128)
    spec[:, 0] = A[:, 0] * nlon
    spec[:, 1:lmax + 1] = (A[:, 1:] - 1j * Bc[:, 1:]) * (nlon / 2.0)
    x = np.fft.irfft(spec, n=nlon, axis=1)
    return x.astype(dtype)


def qc_state_1d(n=1 << 28, field=0, decay=20.0, chunk=1 << 24):
    """1-D float64 field in the shape of a quantum-circuit state vector:
    n/2 complex amplitudes with |a_k| = exp(-decay * k / (n/2)) and uniform
    phases, stored as interleaved real and imaginary parts, normalised so
    that the squared magnitudes sum to 1."""
    assert n % 2 == 0
    r = _rng(4, field)
    half = n // 2
    # sum of |a_k|^2 in closed form for the normalisation
    q = np.exp(-2.0 * decay / half)
    norm = np.sqrt((1.0 - q ** half) / (1.0 - q))
    out = np.empty(n, dtype=np.float64)
    for s in range(0, half, chunk):
        e = min(half, s + chunk)
        k = np.arange(s, e, dtype=np.float64)
        mag = np.exp(-decay * k / half) / norm
        ph = r.uniform(0.0, 2 * np.pi, e - s)
        out[2 * s:2 * e:2] = mag * np.cos(ph)
        out[2 * s + 1:2 * e:2] = mag * np.sin(ph)
    return out


# The workload configurations. Shapes at full size; tests scale them down.
CONFIGS = {
    "sines": dict(gen="sines_1d", shape=(1 << 20,), dtype="float32", rel=(1e-3,)),
    "turbulence": dict(gen="turbulence_3d", shape=(100, 500, 500), dtype="float32", rel=(1e-2, 1e-3, 1e-4)),
    "sphere": dict(gen="sphere_2d", shape=(1800, 3600), dtype="float32", rel=(1e-3, 1e-5)),
    "state": dict(gen="qc_state_1d", shape=(1 << 28,), dtype="float64", rel=(1e-3, 1e-5)),
}


def make(name, shape=None, field=0):
    """Field of configuration `name`, optionally at a smaller shape."""
    c = CONFIGS[name]
    shape = tuple(c["shape"] if shape is None else shape)
    if c["gen"] == "sines_1d":
        return sines_1d(shape[0], field)
    if c["gen"] == "turbulence_3d":
        return turbulence_3d(shape, field)
    if c["gen"] == "sphere_2d":
        return sphere_2d(shape[0], shape[1], field=field)
    if c["gen"] == "qc_state_1d":
        return qc_state_1d(shape[0], field)
    raise KeyError(name)


# ------------------------------------------------------- many-field batches --
#
# A batch of fields of uneven sizes and both element types (the workload of
# the batched path). The specs come from numpy default_rng(13020 + 1000 * 6);
# each field's values come from torch's generator seeded with 13020 + 6000 +
# index, on whatever device the caller names (the full batch is several GiB,
# so it is generated where it is used). The content follows the generators
# above: 1-D fields are sums of sines with noise, 2-D and 3-D fields are cut
# from periodic Gaussian random fields with a k^(-5/3) energy spectrum, half
# of them with exact-zero regions.

_BATCH_STREAM = 6


def batch_specs(count=4096, median=1 << 20, sigma=1.25, lo=4 << 10, hi=64 << 20, f64_frac=0.2,
                ebs=(1e-2, 1e-3, 1e-4), seed_stream=_BATCH_STREAM):
    """Field specs: byte size ~ LogNormal(ln median, sigma) redrawn until it
    lies in [lo, hi]; float64 with probability f64_frac; 1 to 3 dims with
    log-uniform aspect ratios in [1/8, 8] (the element count is the product of
    the dims); a relative bound drawn from ebs."""
    r = _rng(seed_stream, 0)
    specs = []
    for i in range(count):
        while True:
            s = float(np.exp(r.normal(np.log(median), sigma)))
            if lo <= s <= hi:
                break
        f64 = r.random() < f64_frac
        w = 8 if f64 else 4
        n0 = max(1, int(s) // w)
        nd = int(r.integers(1, 4))
        if nd == 1:
            dims = (n0,)
        else:
            a = r.uniform(np.log(1 / 8), np.log(8), nd)
            a -= a.mean()
            base = np.log(n0) / nd
            dims = tuple(max(1, int(round(float(np.exp(base + ai))))) for ai in a)
        eb = float(ebs[int(r.integers(0, len(ebs)))])
        zero = nd > 1 and r.random() < 0.5
        specs.append(dict(index=i, dims=dims, dtype="float64" if f64 else "float32", eb=eb,
                          zero_regions=bool(zero), seed=13020 + 1000 * seed_stream + i))
    return specs


def spec_elems(spec):
    n = 1
    for d in spec["dims"]:
        n *= int(d)
    return n


def _torch_spectral(shape, g, slope, device):
    import torch
    white = torch.randn(shape, generator=g, device=device, dtype=torch.float64)
    F = torch.fft.rfftn(white)
    del white
    ks = [torch.fft.fftfreq(s, device=device, dtype=torch.float64) for s in shape[:-1]]
    ks.append(torch.fft.rfftfreq(shape[-1], device=device, dtype=torch.float64))
    k2 = torch.zeros((), device=device, dtype=torch.float64)
    for ax, k in enumerate(ks):
        view = [1] * len(shape)
        view[ax] = k.numel()
        k2 = k2 + (k * k).view(view)
    amp = torch.where(k2 > 0, k2.clamp_min(1e-300) ** (slope / 2.0), torch.zeros_like(k2))
    x = torch.fft.irfftn(F * amp, s=shape)
    x -= x.mean()
    sd = x.std()
    if sd > 0:
        x /= sd
    return x


_MOTHERS = {}


def _mothers(device):
    """Periodic Gaussian random fields (k^(-5/3) energy spectrum) in 2-D and
    3-D, with smoother fields (|k|^-3) whose global 20 % quantile marks the
    zero regions; generated once per device. Batch fields of 2 and 3 dims are
    cut from them at seeded offsets, indices wrapping around (the fields are
    periodic), so no field needs an FFT of its own."""
    import torch
    key = str(device)
    if key not in _MOTHERS:
        big = torch.device(device).type == "cuda"
        g = torch.Generator(device=device)
        g.manual_seed(13020 + 1000 * _BATCH_STREAM + 999_999)
        out = {}
        for nd, shape in ((2, (4096, 4096) if big else (512, 512)), (3, (384, 384, 384) if big else (64, 64, 64))):
            x = _torch_spectral(shape, g, -11.0 / 6.0, device)
            m = _torch_spectral(shape, g, -3.0, device)
            flat = m.reshape(-1)
            step = max(1, flat.numel() // (1 << 20))
            thr = torch.quantile(flat[::step], 0.2)
            out[nd] = (x, m < thr)
        _MOTHERS[key] = out
    return _MOTHERS[key]


def batch_field(spec, device="cpu"):
    """Values of one batch field as a contiguous torch tensor of the spec's
    dims and element type on `device`."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(spec["seed"])
    dims = tuple(int(d) for d in spec["dims"])
    dt = torch.float64 if spec["dtype"] == "float64" else torch.float32
    if len(dims) == 1:
        n = dims[0]
        u = torch.rand(16, generator=g, device=device, dtype=torch.float64)
        f = torch.exp(u[:8] * np.log(4096.0))
        ph = u[8:] * (2 * np.pi)
        t = torch.arange(n, device=device, dtype=torch.float64) / n
        x = torch.zeros(n, device=device, dtype=torch.float64)
        for j in range(8):
            x += torch.sin(2 * np.pi * f[j] * t + ph[j])
        x += 1e-3 * torch.randn(n, generator=g, device=device, dtype=torch.float64)
        return x.to(dt).contiguous()
    mother, zmask = _mothers(device)[len(dims)]
    u = torch.rand(len(dims), generator=g, device=device, dtype=torch.float64).cpu()
    idx = []
    for ax, d in enumerate(dims):
        M = mother.shape[ax]
        o = int(u[ax] * M)
        view = [1] * len(dims)
        view[ax] = d
        idx.append(((torch.arange(d, device=device) + o) % M).view(view))
    x = mother[tuple(idx)].to(dt)
    if spec["zero_regions"]:
        x[zmask[tuple(idx)]] = 0.0
    return x.contiguous()


# ----------------------------------------------------------- serving traces --
#
# Requests of the serving workload: Poisson arrivals at a given rate, 60 %
# compressions and 40 % decompressions, byte sizes ~ LogNormal(ln 4 MiB, 1.5)
# redrawn until in [64 KiB, 256 MiB], float64 with probability 0.2. A
# compression reads a slice of a pre-generated device field of its element
# type (offset given as a fraction of the free room); a decompression reads a
# resident item picked by a uniform draw. numpy default_rng(13020 + 7000 +
# seed).

_SERVE_STREAM = 7


def serve_trace(count, rate, seed=0, median=4 << 20, sigma=1.5, lo=64 << 10, hi=256 << 20, f64_frac=0.2,
                compress_frac=0.6):
    """Arrays of one trace: t (seconds from the start), kind (0 compress,
    1 decompress), nbytes, f64 (bool), pos (uniform [0, 1): slice offset or
    item pick)."""
    r = _rng(_SERVE_STREAM, seed)
    gaps = r.exponential(1.0 / rate, count) if rate > 0 else np.zeros(count)
    t = np.cumsum(gaps) - gaps[0]
    kind = (r.random(count) >= compress_frac).astype(np.int32)
    nbytes = np.empty(count, dtype=np.int64)
    for i in range(count):
        while True:
            s = float(np.exp(r.normal(np.log(median), sigma)))
            if lo <= s <= hi:
                break
        nbytes[i] = int(s)
    f64 = r.random(count) < f64_frac
    pos = r.random(count)
    return dict(t=t, kind=kind, nbytes=nbytes, f64=f64, pos=pos)
