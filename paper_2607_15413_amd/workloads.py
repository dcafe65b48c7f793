"""Seeded synthetic fields shaped like the paper's workloads.

This module only draws inputs: it contains none of the compressor's
arithmetic and is shared, unchanged, by the tests (HIP path and oracle alike)
and the benchmark.  Every field is drawn with ``numpy.random.default_rng``
in float64 in the documented order and cast to float32 at the end.

The paper evaluates on SDRBench / Open-SciVis fields (Sec. V-A, Table II)
that are not available here; these generators stand in for them:

* ``sinusoid_field``        1-D sum of 8 sinusoids + Gaussian noise
* ``grf_field``             3-D Gaussian random field, power spectrum k^-3
                            (NYX-like per-field size at 512^3)
* ``piecewise_quadratic``   3-D piecewise quadratic with jumps and zero
                            regions (Hurricane-like per-field size at
                            100 x 500 x 500)
* ``batch_fields``          64 uneven fields for the batched form
* ``request_stream``        Poisson request stream for the served form
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

try:  # multi-threaded FFTs when scipy is present (identical results)
    import scipy.fft as _fft

    def _rfftn(a):
        return _fft.rfftn(a, workers=-1)

    def _irfftn(a, shape):
        return _fft.irfftn(a, s=shape, workers=-1)
except Exception:  # pragma: no cover
    def _rfftn(a):
        return np.fft.rfftn(a)

    def _irfftn(a, shape):
        return np.fft.irfftn(a, s=shape)


def sinusoid_field(n: int = 1 << 20, seed: int = 0, noise_sigma: float = 1e-3) -> np.ndarray:
    """x_i = sum_k A_k sin(2 pi i / P_k + phi_k) + eps_i.

    Draw order: A ~ U[0.1, 1]^8, P ~ U[64, 65536]^8, phi ~ U[0, 2 pi]^8,
    then eps ~ N(0, noise_sigma) (noise_sigma read as a standard deviation).
    """
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.1, 1.0, 8)
    period = rng.uniform(64.0, 65536.0, 8)
    phase = rng.uniform(0.0, 2.0 * math.pi, 8)
    eps = rng.normal(0.0, noise_sigma, n)
    i = np.arange(n, dtype=np.float64)
    x = eps
    for k in range(8):
        x = x + amp[k] * np.sin(2.0 * math.pi * i / period[k] + phase[k])
    return x.astype(np.float32)


def grf_field(shape=(512, 512, 512), seed: int = 1, slope: float = -3.0) -> np.ndarray:
    """Isotropic Gaussian random field with P(k) ~ k^slope, scaled to [-1, 1].

    White N(0, 1) noise (seed) -> rfftn -> multiply by |k|^(slope/2) with
    k from fftfreq * size per axis (the k = 0 mode set to 0) -> irfftn ->
    affine map of [min, max] onto [-1, 1].  Returned flattened row-major.
    """
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(shape)
    spec = _rfftn(white)
    del white
    kx = np.fft.fftfreq(shape[0]) * shape[0]
    ky = np.fft.fftfreq(shape[1]) * shape[1]
    kz = np.fft.rfftfreq(shape[2]) * shape[2]
    # scale slab by slab to bound memory
    kyz2 = ky[:, None] ** 2 + kz[None, :] ** 2
    for a in range(shape[0]):
        k2 = kx[a] ** 2 + kyz2
        with np.errstate(divide="ignore"):
            amp = np.where(k2 > 0, k2 ** (slope / 4.0), 0.0)
        spec[a] *= amp
    field = _irfftn(spec, shape)
    del spec
    lo = field.min()
    hi = field.max()
    field -= lo
    field *= 2.0 / (hi - lo)
    field -= 1.0
    return field.astype(np.float32).reshape(-1)


def piecewise_quadratic(shape=(100, 500, 500), seed: int = 2, boxes_per_axis: int = 4,
                        zero_fraction: float = 0.1) -> np.ndarray:
    """Piecewise-smooth 3-D field of boxes_per_axis^3 axis-aligned regions.

    Draw order: for each axis, boxes_per_axis - 1 distinct sorted cut
    positions in [1, size - 1]; then for each region in C order, 10
    coefficients ~ N(0, 1) of a full quadratic in the global integer indices
    (1, i, j, k, i^2, j^2, k^2, ij, ik, jk), an offset magnitude ~ U[1, 100]
    and its sign (+/- with probability 1/2); finally round(zero_fraction *
    regions) distinct regions are set exactly to 0.0.
    """
    rng = np.random.default_rng(seed)
    nreg = boxes_per_axis ** 3
    cuts = []
    for size in shape:
        c = np.sort(rng.choice(np.arange(1, size), boxes_per_axis - 1, replace=False))
        cuts.append(c)
    coef = np.empty((nreg, 10))
    offset = np.empty(nreg)
    for r in range(nreg):
        coef[r] = rng.standard_normal(10)
        mag = rng.uniform(1.0, 100.0)
        sign = 1.0 if rng.random() < 0.5 else -1.0
        offset[r] = sign * mag
    nzero = int(round(zero_fraction * nreg))
    zero = np.zeros(nreg, dtype=bool)
    zero[rng.choice(nreg, nzero, replace=False)] = True

    ni, nj, nk = shape
    bi = np.searchsorted(cuts[0], np.arange(ni), side="right")
    bj = np.searchsorted(cuts[1], np.arange(nj), side="right")
    bk = np.searchsorted(cuts[2], np.arange(nk), side="right")
    j = np.arange(nj, dtype=np.float64)[:, None]
    k = np.arange(nk, dtype=np.float64)[None, :]
    out = np.empty(shape, dtype=np.float32)
    for i in range(ni):
        reg = (bi[i] * boxes_per_axis + bj[:, None]) * boxes_per_axis + bk[None, :]
        c = coef[reg]
        fi = float(i)
        v = (c[..., 0] + c[..., 1] * fi + c[..., 2] * j + c[..., 3] * k
             + c[..., 4] * fi * fi + c[..., 5] * j * j + c[..., 6] * k * k
             + c[..., 7] * fi * j + c[..., 8] * fi * k + c[..., 9] * j * k
             + offset[reg])
        v[zero[reg]] = 0.0
        out[i] = v.astype(np.float32)
    return out.reshape(-1)


@dataclass
class BatchField:
    data: np.ndarray       # float32, flattened
    rel: float             # REL error bound
    kind: str              # "sinusoid" or "grf"


def batch_sizes(count: int = 64, seed: int = 3, lo: int = 1 << 14, hi: int = 1 << 24):
    """Log-uniform sizes in [lo, hi); a multiple of 256 is bumped by one."""
    rng = np.random.default_rng(seed)
    sizes = []
    for _ in range(count):
        n = int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        if n % 256 == 0:
            n += 1
        sizes.append(n)
    return sizes


def batch_fields(count: int = 64, seed: int = 3, lo: int = 1 << 14, hi: int = 1 << 24,
                 grf_shape=(256, 256, 256)) -> list:
    """Uneven fields for the batched form.

    Sizes from ``batch_sizes``; then per field, in order: a coin (< 0.5 ->
    sinusoid field with a drawn sub-seed, else a contiguous slice at a drawn
    offset of one k^-3 master field of grf_shape drawn with a drawn seed) and
    a REL bound drawn from {1e-2, 1e-3, 1e-4}.
    """
    sizes = batch_sizes(count, seed, lo, hi)
    rng = np.random.default_rng(seed + 1000)
    master_seed = int(rng.integers(0, 2 ** 31))
    master = None
    fields = []
    for n in sizes:
        if rng.random() < 0.5:
            sub = int(rng.integers(0, 2 ** 31))
            data = sinusoid_field(n, sub)
            kind = "sinusoid"
        else:
            if master is None:
                master = grf_field(grf_shape, master_seed)
            if n > master.size:
                raise ValueError("field larger than the master field")
            off = int(rng.integers(0, master.size - n + 1))
            data = master[off:off + n].copy()
            kind = "grf"
        rel = float(rng.choice([1e-2, 1e-3, 1e-4]))
        fields.append(BatchField(data, rel, kind))
    return fields


@dataclass
class Request:
    arrival_s: float       # arrival time from the start of the stream
    op: str                # "compress" or "decompress"
    offset: int            # slice start in the master field
    n: int                 # elements
    rel: float             # REL error bound


def sparse_field(n: int = 1 << 27, seed: int = 5, spacing: int = 20000) -> np.ndarray:
    """Zeros with one spike per `spacing` elements on average: n // spacing
    positions drawn uniformly (with repetition), values U[-50, 50].  At REL
    1e-3 most tiles are all zero, so the stream is mostly its rate header
    (CR near the format's cap of 128; about 122 for the 512^3 size)."""
    rng = np.random.default_rng(seed)
    x = np.zeros(n, dtype=np.float32)
    k = max(1, n // spacing)
    x[rng.integers(0, n, k)] = rng.uniform(-50, 50, k).astype(np.float32)
    return x


def request_stream(rate_per_s: float, count: int = 10000, seed: int = 4, lo: int = 1 << 10,
                   hi: int = 1 << 26, master_n: int = 269 * 500 * 500,
                   compress_fraction: float = 0.7) -> list:
    """Open-loop Poisson arrivals of compress / decompress requests.

    Per request, in order: exponential inter-arrival (rate_per_s), a coin for
    the operation (< compress_fraction -> compress), a log-uniform size in
    [lo, hi), a slice offset in the master field and a REL from {1e-3, 1e-4}.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += float(rng.exponential(1.0 / rate_per_s))
        op = "compress" if rng.random() < compress_fraction else "decompress"
        n = int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        n = min(n, master_n)
        off = int(rng.integers(0, master_n - n + 1))
        rel = float(rng.choice([1e-3, 1e-4]))
        out.append(Request(t, op, off, n, rel))
    return out
