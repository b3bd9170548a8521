"""Seeded synthetic fields standing in for the paper's datasets.

The paper evaluates on SDRBench fields (CESM-ATM, Hurricane, Miranda, Nyx,
QMCPack, SCALE-LetKF; Sec. VI, table of applications), all single precision.
Those files are not available here, so these generators produce fields with
the same shapes and the properties the method depends on: local smoothness
(Sec. IV: most blocks have a small value range) and exact zero regions. They
contain none of the compressor's arithmetic; both the GPU path and the CPU
oracle consume the same arrays.

Seeds: numpy default_rng(13020 + 1000 * cfg + field). Values are generated in
float64 and rounded once to the element type. Zeros are assigned (+0.0), never
produced by multiplying with a mask.
"""
import numpy as np


def _rng(cfg, field=0):
    return np.random.default_rng(13020 + 1000 * cfg + field)


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
    x = np.fft.irfftn(F, s=shape)
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
    "cfg1": dict(gen="sines_1d", shape=(1 << 20,), dtype="float32", rel=(1e-3,)),
    "cfg2": dict(gen="turbulence_3d", shape=(100, 500, 500), dtype="float32", rel=(1e-2, 1e-3, 1e-4)),
    "cfg3a": dict(gen="sphere_2d", shape=(1800, 3600), dtype="float32", rel=(1e-3, 1e-5)),
    "cfg3b": dict(gen="qc_state_1d", shape=(1 << 28,), dtype="float64", rel=(1e-3, 1e-5)),
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
