"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws input data; it contains no step of the selection method.
Every generator takes an explicit seed and returns numpy arrays on the host.

Workload shapes follow the paper's experiments (§10, "Unsorted Selection":
2^28 keys per processor, Zipf-distributed integers, k in {2^10, 2^20, 2^26})
and the single-GPU workloads built on them:

* uniform u32 keys on [0, 2^32)
* uniform f32 keys on [0, 1) on the 2^-24 grid (the law of an fp32 uniform
  draw; about 16 copies of every value at 2^28 keys)
* Zipf(s) over V distinct values by an inverse-CDF table, key = rank - 1
* all keys equal except a Bernoulli(frac) subset of uniform u32 keys
* ragged rows: lengths lognormal around a median, clipped; N(0,1) f32 keys;
  per-row k uniform in [1, min(len, k_max)]
* dense N(0,1) f32 score matrices and upstream gradients
* objects for the most-frequent-objects problem: Zipf(s = 1) over 2^20
  values and a negative binomial (r = 1000, p = 0.05), the two input
  distributions of §10.2; (key, value) pairs for the sum aggregation
* f32 keys rich in special values (signed zeros, infinities, NaN payloads,
  subnormals, heavy repeats)
"""
import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform_u32(n, seed):
    return _rng(seed).integers(0, 2**32, size=n, dtype=np.uint32)


def uniform_f32_grid(n, seed):
    """Uniform on [0,1) with 24-bit resolution: m * 2^-24, m uniform in [0, 2^24)."""
    m = _rng(seed).integers(0, 2**24, size=n, dtype=np.uint32)
    out = m.astype(np.float32)
    out *= np.float32(2.0**-24)
    return out


def normal_f32(shape, seed):
    return _rng(seed).standard_normal(size=shape, dtype=np.float32)


def zipf_u32(n, s, V, seed, chunk=1 << 24):
    """Zipf(s) over ranks 1..V by inverse CDF; returns key = rank - 1."""
    r = np.arange(1, V + 1, dtype=np.float64)
    w = r ** (-float(s))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    cdf[-1] = 1.0
    rng = _rng(seed)
    out = np.empty(n, np.uint32)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        u = rng.random(b - a)
        out[a:b] = np.minimum(np.searchsorted(cdf, u, side="right"), V - 1)
    return out


def all_equal_except(n, frac, value, seed):
    """All keys = value except a Bernoulli(frac) subset of uniform u32 keys."""
    rng = _rng(seed)
    out = np.full(n, value, np.uint32)
    mask = rng.random(n) < frac
    out[mask] = rng.integers(0, 2**32, size=int(mask.sum()), dtype=np.uint32)
    return out


def lognormal_rows(rows, median, sigma, lo, hi, k_max, seed):
    """Ragged rows: returns (keys f32[sum len], row_off u64[R+1], k u32[R])."""
    rng = _rng(seed)
    lens = np.rint(np.exp(rng.normal(np.log(median), sigma, size=rows)))
    lens = np.clip(lens, lo, hi).astype(np.int64)
    kk = np.array([rng.integers(1, min(int(L), k_max) + 1) for L in lens], np.uint32)
    off = np.zeros(rows + 1, np.uint64)
    off[1:] = np.cumsum(lens)
    keys = rng.standard_normal(size=int(off[-1]), dtype=np.float32)
    return keys, off, kk


def specials_f32(n, seed):
    """f32 keys mixing ordinary values with every special case of the order."""
    rng = _rng(seed)
    pool = np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -1.0, 1e-45, -1e-45,
                     1.17549435e-38, -1.17549435e-38, 3.4028235e38, -3.4028235e38,
                     0.5, 2.0], np.float32)
    nan_bits = np.array([0x7FC00000, 0xFFC00000, 0x7F800001, 0xFFFFFFFF, 0x7FBFFFFF],
                        np.uint32)
    out = rng.standard_normal(size=n).astype(np.float32)
    pick = rng.random(n)
    sel = pick < 0.35
    out[sel] = pool[rng.integers(0, pool.size, size=int(sel.sum()))]
    nsel = (pick >= 0.35) & (pick < 0.45)
    bits = out.view(np.uint32)
    bits[nsel] = nan_bits[rng.integers(0, nan_bits.size, size=int(nsel.sum()))]
    return out


def small_alphabet_u32(n, alphabet, seed):
    """u32 keys drawn from {0, ..., alphabet-1} (forces many ties)."""
    return _rng(seed).integers(0, alphabet, size=n, dtype=np.uint32)


def negbin_u32(n, r, p, U, seed, chunk=1 << 24):
    """Negative binomial(r, p) objects, clipped to [0, U)."""
    rng = _rng(seed)
    out = np.empty(n, np.uint32)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        out[a:b] = np.minimum(rng.negative_binomial(r, p, size=b - a), U - 1)
    return out


def keyed_values(n, U, s, vmax, seed):
    """(key, value) pairs: keys Zipf(s) over U, values uniform in [0, vmax]."""
    keys = zipf_u32(n, s, U, seed)
    values = _rng(seed + 1).integers(0, vmax + 1, size=n, dtype=np.uint32)
    return keys, values
