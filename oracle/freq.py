"""CPU oracle for the top-k most frequent objects (§7) and the top-k sum
aggregation (§8) — TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's algorithms, step by step in its order, on one address space:

  PAC (§7.1, Algorithm of Figure "sample"): Bernoulli sample at rate rho,
      count the sampled objects, select the k most frequently sampled.
  EC (§7.2): the same sample and counts, select the k* most frequently
      sampled, count those k* exactly in the whole input, return the k most
      frequent of them by exact count.
  Sum aggregation (§8): aggregate the (key, value) input by key, take the
      weighted sample of the sums, then proceed as PAC (or EC with exact sums).

"The k most frequent" follows the unique order of §2 with the count as the
value: larger counts first, ties by ascending object (a reading: the paper
leaves ties open).  Counts and sums are integers, so every result is exact.
"""
import math

import numpy as np

from . import _p, lib

_U32 = np.uint32


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def top_by_count(counts, k, candidates=None):
    """The k first objects in the order (count descending, object ascending),
    among `candidates` (all objects if None).  Returns (objects, counts)."""
    counts = np.asarray(counts)
    objs = np.arange(counts.size, dtype=np.int64) if candidates is None else \
        np.asarray(candidates, dtype=np.int64)
    c = counts[objs].astype(np.int64)
    order = np.lexsort((objs, -c))[:k]
    return objs[order].astype(np.uint32), counts[objs[order]]


# ----------------------------------------------------------- sampling ----

def take_mask(n, T, seed, tag):
    """The Bernoulli sample of positions 0..n-1 at rate T / 2^32 (per-element
    decisions, word i % 4 of Philox4x32-10 at counter (i/4, 0, tag, 2))."""
    L = lib()
    return np.array([bool(L.orc_take(seed, tag, i, T)) for i in range(n)], bool)


def sample_counts(keys, U, T, seed, tag):
    """Counts by object of the Bernoulli sample (§7.1); returns (counts[U], sample size)."""
    keys = _u32(keys)
    counts = np.empty(U, np.uint32)
    ns = np.zeros(1, np.uint64)
    rc = lib().orc_sample_counts(_p(keys), keys.size, U, seed, tag, T, _p(counts), _p(ns))
    if rc != 0:
        raise ValueError("key outside [0, U)")
    return counts, int(ns[0])


def exact_counts(keys, U):
    keys = _u32(keys)
    counts = np.empty(U, np.uint32)
    if lib().orc_exact_counts(_p(keys), keys.size, U, _p(counts)) != 0:
        raise ValueError("key outside [0, U)")
    return counts


# ------------------------------------------------------ PAC and EC (§7) --

def pac_from_counts(scounts, k):
    """PAC's selection step: the k most frequently sampled objects."""
    return top_by_count(scounts, k)


def ec_from_counts(scounts, exact, k, kstar):
    """EC's steps after sampling: the k* most frequently sampled objects,
    their exact counts, the k most frequent of them by exact count."""
    cand, _ = top_by_count(scounts, kstar)
    return top_by_count(exact, k, candidates=cand)


def pac(keys, U, k, T, seed, tag=0):
    """PAC on the input: returns (objects[k], sample counts[k], sample size)."""
    sc, ns = sample_counts(keys, U, T, seed, tag)
    ids, cnt = pac_from_counts(sc, k)
    return ids, cnt, ns


def ec(keys, U, k, kstar, T, seed, tag=0):
    """EC on the input: returns (objects[k], exact counts[k], sample size)."""
    sc, ns = sample_counts(keys, U, T, seed, tag)
    ids, cnt = ec_from_counts(sc, exact_counts(keys, U), k, kstar)
    return ids, cnt, ns


def error(exact, returned):
    """The error of §7 in absolute terms: the count of the most frequent
    object not returned minus that of the least frequent returned (0 if that
    is not positive, i.e. the result is exact)."""
    exact = np.asarray(exact, np.int64)
    mask = np.zeros(exact.size, bool)
    mask[np.asarray(returned, np.int64)] = True
    if mask.all():
        return 0
    return max(0, int(exact[~mask].max()) - int(exact[mask].min()))


# ------------------------------------------------------ sample sizes ------

def sample_size_pac(n, k, eps, delta):
    """Expected sample size rho n of PAC for an (eps, delta)-approximation
    (§7.1, equation "sampleSize")."""
    return 4.0 / eps ** 2 * max(3.0 / k * math.log(4.0 * n / delta),
                                2.0 * math.log(2.0 * k / delta))


def sample_size_ec(n, kstar, eps, delta):
    """Expected sample size of EC counting k* objects exactly (§7.2, Lemma "topkec")."""
    return 2.0 / (eps ** 2 * kstar) * math.log(n / delta)


def kstar_paper(k, eps, n, delta, p):
    """The k* that §7.2 derives for p PEs: max(k, (1/eps) sqrt(2 log p / p ln(n / delta)))."""
    if p <= 1:
        return k
    return max(k, int(math.ceil(1.0 / eps * math.sqrt(2.0 * math.log2(p) / p *
                                                       math.log(n / delta)))))


def threshold(n, sample_size):
    """Sampling threshold T = rho 2^32 for an expected sample size (rho <= 1):
    T = min(2^32, ceil(sample_size 2^32 / n))."""
    if n == 0:
        return 1 << 32
    t = math.ceil(sample_size * 4294967296.0 / n)
    return int(min(max(t, 1), 1 << 32))


# ------------------------------------------------- sum aggregation (§8) --

def sums_by_key(keys, values, U):
    keys = _u32(keys)
    values = _u32(values)
    sums = np.empty(U, np.uint64)
    if lib().orc_sum_by_key(_p(keys), _p(values), keys.size, U, _p(sums)) != 0:
        raise ValueError("key outside [0, U)")
    return sums


def weighted_sample(sums, s, seed, tag=0):
    """The weighted sample of §8 "Sampling": per key floor(v / v_avg) samples
    plus one with probability v / v_avg - floor(v / v_avg), v_avg = m / s."""
    sums = np.ascontiguousarray(sums, dtype=np.uint64)
    out = np.empty(sums.size, np.uint32)
    tot = lib().orc_weighted_sample(_p(sums), sums.size, s, seed, tag, _p(out))
    if tot < 0:
        raise ValueError("all sums are zero")
    return out, int(tot)


def sum_pac(keys, values, U, k, s, seed, tag=0):
    """PAC top-k sum aggregation (§8): returns (objects[k], sample counts[k])."""
    samp, _ = weighted_sample(sums_by_key(keys, values, U), s, seed, tag)
    return top_by_count(samp, k)


def sum_ec(keys, values, U, k, kstar, s, seed, tag=0):
    """With exact summation: the k* most sampled keys, the k largest of them
    by exact sum.  Returns (objects[k], exact sums[k])."""
    sums = sums_by_key(keys, values, U)
    samp, _ = weighted_sample(sums, s, seed, tag)
    cand, _ = top_by_count(samp, kstar)
    return top_by_count(sums, k, candidates=cand)


def sample_size_sum(n, eps, delta, p=1):
    """Sample size of the sum aggregation (§8, proof of Theorem "sumpac"):
    s >= (1/eps) sqrt(2 p ln(2 n / delta))."""
    return 1.0 / eps * math.sqrt(2.0 * p * math.log(2.0 * n / delta))
