"""CPU oracle for unsorted top-k selection — TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It is independent of the GPU library:
it shares no source, header, table or helper with it.

Python side of ``topk_oracle.c`` (ctypes) plus the few plain numpy oracles
(dense scatter for the gradient).  Every function states the passage of the
paper (Hübschle-Schneider, Sanders, Müller, "Communication Efficient
Algorithms for Top-k Selection Problems") it follows.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def lib():
    """Load liboracle.so, building it with gcc if it is missing."""
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path) or \
                os.path.getmtime(path) < max(os.path.getmtime(f) for f in _build.SOURCES):
            _build.build()
        L = ctypes.CDLL(path)
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        L.orc_select_sort.argtypes = [vp, i32, u64, u64, i32, vp]
        L.orc_select_brute.argtypes = [vp, i32, u64, u64, i32, vp, vp]
        L.orc_select_composite.argtypes = [vp, i32, u64, u64, i32, i32, vp]
        L.orc_check.argtypes = [vp, i32, u64, u64, i32, vp, u32, u32]
        L.orc_precedes.argtypes = [vp, i32, i32, u32, u32]
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_philox4x32_10.restype = None
        L.orc_bernoulli_sample.argtypes = [u64, ctypes.c_double, u64, u32, u32, u32, vp, u64]
        L.orc_bernoulli_sample.restype = ctypes.c_int64
        L.orc_pivot_ranks.argtypes = [u64, u64, u64, u32, vp, vp]
        L.orc_pivot_ranks.restype = None
        L.orc_take.argtypes = [u64, u32, u64, u64]
        L.orc_sample_counts.argtypes = [vp, u64, u32, u64, u32, u64, vp, vp]
        L.orc_exact_counts.argtypes = [vp, u64, u32, vp]
        L.orc_sum_by_key.argtypes = [vp, vp, u64, u32, vp]
        L.orc_weighted_sample.argtypes = [vp, u32, u64, u64, u32, vp]
        L.orc_weighted_sample.restype = ctypes.c_int64
        L.orc_rank.argtypes = [vp, i32, u64, i32, u32]
        L.orc_rank.restype = u64
        L.orc_rank_among.argtypes = [vp, i32, i32, vp, u64, vp, u64, vp]
        L.orc_rank_among.restype = None
        _lib = L
    return _lib


def _keys(keys):
    keys = np.ascontiguousarray(keys)
    if keys.dtype == np.float32:
        return keys, 1
    if keys.dtype == np.uint32:
        return keys, 0
    raise TypeError("oracle keys must be float32 or uint32, got %s" % keys.dtype)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def select_sort(keys, k, largest=False):
    """Plain oracle (§4 problem statement; §2 unique order by (value, object)).

    Sorts all positions by (value, position) and returns the first k, in that
    order: ``idx[k-1]`` is the object of rank k.
    """
    keys, f = _keys(keys)
    out = np.empty(k, np.uint32)
    rc = lib().orc_select_sort(_p(keys), f, keys.size, k, int(largest), _p(out))
    if rc != 0:
        raise ValueError("orc_select_sort rc=%d" % rc)
    return out


def select_composite(keys, k, largest=False, threads=1):
    """The same selection by a sort of 64-bit composites (value order word,
    position) on ``threads`` threads (chunk sorts, then a merge of the first k).
    The form the benchmark times; returns the first k in the unique order."""
    keys, f = _keys(keys)
    out = np.empty(k, np.uint32)
    rc = lib().orc_select_composite(_p(keys), f, keys.size, k, int(largest), int(threads), _p(out))
    if rc != 0:
        raise ValueError("orc_select_composite rc=%d" % rc)
    return out


def select_brute(keys, k, largest=False):
    """Brute-force rank counting: selected iff #{j preceding i} < k.

    Returns (selected positions ascending, position of rank k).  O(n^2).
    """
    keys, f = _keys(keys)
    out = np.empty(k, np.uint32)
    kth = np.zeros(1, np.uint32)
    rc = lib().orc_select_brute(_p(keys), f, keys.size, k, int(largest), _p(out), _p(kth))
    if rc != 0:
        raise ValueError("orc_select_brute rc=%d" % rc)
    return out, int(kth[0])


def check(keys, k, sel, kth_idx, kth_key_bits, largest=False):
    """O(n) check of a claimed result; 0 = valid, else the failing invariant.

    1 index out of range/repeated, 2 kth not selected, 3 selected above the
    k-th value, 4 unselected below it, 5 counts below/equal do not add up,
    6 tie rule broken, 7 kth_idx not the last selected tie, 8 kth key bits.
    """
    keys, f = _keys(keys)
    sel = np.ascontiguousarray(sel, dtype=np.uint32)
    if sel.size != k:
        return 1
    return int(lib().orc_check(_p(keys), f, keys.size, k, int(largest), _p(sel),
                               int(kth_idx), int(kth_key_bits)))


def precedes(keys, i, j, largest=False):
    keys, f = _keys(keys)
    return bool(lib().orc_precedes(_p(keys), f, int(largest), i, j))


def philox4x32_10(ctr, key):
    """Philox4x32-10 block function (Salmon et al., SC'11)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    kk = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(kk), _p(out))
    return out


def bernoulli_sample(n, rho, seed, tag, nseg, seg_cap):
    """Bernoulli sample of positions 0..n-1 by geometric skips (§2)."""
    cap = nseg * seg_cap
    out = np.empty(max(cap, 1), np.uint32)
    cnt = lib().orc_bernoulli_sample(n, float(rho), seed, tag, nseg, seg_cap, _p(out), cap)
    if cnt < 0:
        raise ValueError("sample buffer too small")
    return out[:cnt].copy()


def pivot_ranks(s, k, n, c_num):
    """Sample ranks (lo, hi) of the two pivots around k s / n (§2, FR-selection)."""
    lo = ctypes.c_int64()
    hi = ctypes.c_int64()
    lib().orc_pivot_ranks(s, k, n, c_num, ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def rank(keys, x, largest=False):
    """Rank of object x: the number of objects preceding it in the unique order
    (§2).  The k smallest are the objects of rank < k (§4); the counts |a| and
    |b| of a round of the Algorithm of §2 are rank differences of its pivots."""
    keys, f = _keys(keys)
    return int(lib().orc_rank(_p(keys), f, keys.size, int(largest), int(x)))


def rank_among(keys, xs, ys, largest=False):
    """For each object of xs, the number of objects of ys preceding it (O(|xs| |ys|))."""
    keys, f = _keys(keys)
    xs = np.ascontiguousarray(xs, dtype=np.uint32)
    ys = np.ascontiguousarray(ys, dtype=np.uint32)
    out = np.empty(xs.size, np.uint64)
    lib().orc_rank_among(_p(keys), f, int(largest), _p(xs), xs.size, _p(ys), ys.size, _p(out))
    return out


def topk_rows(scores, k):
    """Row-wise largest-k by the plain oracle, ordered (value desc, index asc).

    Returns (values float32[B,k], indices int64[B,k]).
    """
    scores = np.ascontiguousarray(scores, dtype=np.float32)
    B = scores.shape[0]
    idx = np.empty((B, k), np.int64)
    for b in range(B):
        idx[b] = select_sort(scores[b], k, largest=True)
    vals = np.take_along_axis(scores, idx, axis=1)
    return vals, idx


def scatter_rows(grad_out, indices, n_cols):
    """Dense gradient of row-wise top-k values: zeros except grad_out at indices."""
    g = np.zeros((grad_out.shape[0], n_cols), np.float32)
    for b in range(grad_out.shape[0]):
        for m in range(grad_out.shape[1]):
            g[b, indices[b, m]] = grad_out[b, m]
    return g


from . import freq  # noqa: E402,F401  (top-k most frequent objects and sum aggregation)
from . import msselect  # noqa: E402,F401  (selection over sorted rows: msSelect, amsSelect)
