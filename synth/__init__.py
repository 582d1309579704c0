"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only draws numbers and lays them out in arrays.  It holds none
of the arithmetic of the stencils, the interval DP or the cost model, so
either side can use it without depending on the other.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used in its counter-based form

    x_k = mix64(seed + (k + 1) * 0x9E3779B97F4A7C15)      (mod 2^64)

so any element can be produced independently and vectorised in numpy.
    uniform f64 in [0,1):  (x >> 11) * 2^-53
    uniform f32 in [0,1):  (x >> 40) * 2^-24
    integer in [a,b]:      a + x mod (b - a + 1)

Each workload draws from its own stream: stream s uses seed mix64(BASE_SEED + s).
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 1802
GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# One stream per workload.
STREAM_JACOBI1D = 1
STREAM_JACOBI2D = 2
STREAM_HEAT3D = 3
STREAM_BATCHED = 4
STREAM_CHAIN = 5
STREAM_MLP = 6
STREAM_TESTS = 7


def _mix64(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=False)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def stream_seed(stream: int, base: int = BASE_SEED) -> int:
    """Seed of stream `stream`: one SplitMix64 output of the base seed."""
    return int(_mix64(np.array([(base + stream) % (1 << 64)], dtype=np.uint64))[0])


def raw64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """n consecutive 64-bit outputs of the counter-based SplitMix64 stream."""
    k = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed % (1 << 64)) + k * GAMMA
    return _mix64(z)


def uniform_f64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    x = raw64(seed, n, offset)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_f32(seed: int, n: int, offset: int = 0) -> np.ndarray:
    x = raw64(seed, n, offset)
    return ((x >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)).astype(np.float32)


def randint(seed: int, n: int, lo: int, hi: int, offset: int = 0) -> np.ndarray:
    """Integers in [lo, hi] (inclusive); bias <= (hi-lo+1)/2^64."""
    x = raw64(seed, n, offset)
    return (np.int64(lo) + (x % np.uint64(hi - lo + 1)).astype(np.int64)).astype(np.int64)


# ---------------------------------------------------------------- fields ----

def _interior_mask(shape) -> np.ndarray:
    m = np.zeros(shape, dtype=bool)
    m[tuple(slice(1, s - 1) for s in shape)] = True
    return m


def uniform_field(shape, stream: int, dtype=np.float64, zero_boundary: bool = True) -> np.ndarray:
    """Every cell uniform[0,1) from `stream`; the outer face set to 0 when asked."""
    n = int(np.prod(shape))
    seed = stream_seed(stream)
    if dtype == np.float32:
        a = uniform_f32(seed, n).reshape(shape)
    else:
        a = uniform_f64(seed, n).reshape(shape).astype(dtype, copy=False)
    if zero_boundary:
        a = np.where(_interior_mask(shape), a, dtype(0) if callable(dtype) else 0).astype(dtype)
    return np.ascontiguousarray(a)


def jacobi1d_input(n: int = 4096) -> np.ndarray:
    """N f64 points, interior uniform[0,1) from stream 1, u[0] = u[N-1] = 0."""
    return uniform_field((n,), STREAM_JACOBI1D, np.float64, zero_boundary=True)


def jacobi2d_input(ny: int = 4096, nx: int = 4096, noise: float = 1e-3, modes=(1, 1)) -> np.ndarray:
    """sin(m_y pi y) sin(m_x pi x) on the unit square plus noise*(2U-1) on the interior.

    y_i = i/(ny-1), x_j = j/(nx-1); the boundary is set to exactly 0.  The
    noise draws come from stream 2.  `noise=0` gives the pure Fourier mode.
    """
    my, mx = modes
    yi = np.arange(ny, dtype=np.float64) / (ny - 1)
    xj = np.arange(nx, dtype=np.float64) / (nx - 1)
    a = np.outer(np.sin(my * math.pi * yi), np.sin(mx * math.pi * xj))
    if noise != 0.0:
        u = uniform_f64(stream_seed(STREAM_JACOBI2D), ny * nx).reshape(ny, nx)
        a = a + noise * (2.0 * u - 1.0)
    a[0, :] = 0.0
    a[-1, :] = 0.0
    a[:, 0] = 0.0
    a[:, -1] = 0.0
    return np.ascontiguousarray(a)


def heat3d_input(n: int = 512, nz: int | None = None, ny: int | None = None, nx: int | None = None) -> np.ndarray:
    """Interior uniform[0,1) f64 from stream 3, zero boundary."""
    shape = (nz or n, ny or n, nx or n)
    return uniform_field(shape, STREAM_HEAT3D, np.float64, zero_boundary=True)


def to_bf16_bits(a32: np.ndarray) -> np.ndarray:
    """Round f32 to bf16 (nearest, ties to even; NaN kept quiet); returns uint16 bit patterns."""
    b = np.ascontiguousarray(a32, dtype=np.float32).view(np.uint32)
    nan = (b & np.uint32(0x7FFFFFFF)) > np.uint32(0x7F800000)
    lsb = (b >> np.uint32(16)) & np.uint32(1)
    r = ((b + np.uint32(0x7FFF) + lsb) >> np.uint32(16)).astype(np.uint16)
    r = np.where(nan, ((b >> np.uint32(16)) | np.uint32(0x40)).astype(np.uint16), r)
    return r.astype(np.uint16)


def from_bf16_bits(h: np.ndarray) -> np.ndarray:
    return (np.ascontiguousarray(h, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def batched_instances(count: int = 256, lo: int = 128, hi: int = 2048, tlo: int = 32, thi: int = 512):
    """Shapes and step counts of the uneven batch, from stream 4.

    Returns a list of (ny, nx, T).  ny, nx uniform in [lo, hi] independently,
    T uniform in [tlo, thi].
    """
    seed = stream_seed(STREAM_BATCHED)
    ny = randint(seed, count, lo, hi, offset=0)
    nx = randint(seed, count, lo, hi, offset=count)
    T = randint(seed, count, tlo, thi, offset=2 * count)
    return [(int(a), int(b), int(c)) for a, b, c in zip(ny, nx, T)]


def batched_field(index: int, ny: int, nx: int) -> np.ndarray:
    """Instance `index` of the batch: every cell uniform[0,1) as f32 (outer ring kept fixed)."""
    seed = stream_seed(STREAM_BATCHED + 1000 * (index + 1))
    return np.ascontiguousarray(uniform_f32(seed, ny * nx).reshape(ny, nx))


def chain_dims(n: int = 4096, lo: int = 1, hi: int = 100, stream: int = STREAM_CHAIN) -> np.ndarray:
    """p_0..p_N int64 uniform in [lo, hi] from stream 5."""
    return randint(stream_seed(stream), n + 1, lo, hi)


def test_rng(tag: int) -> int:
    """Seed for ad-hoc test data (stream 7, sub-stream `tag`)."""
    return stream_seed(STREAM_TESTS * 1000003 + tag)
