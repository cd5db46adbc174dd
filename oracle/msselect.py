"""CPU oracle for selection over locally sorted input — TEST INFRASTRUCTURE ONLY.

§4.2 / Appendix A (Algorithm "musel", msSelect): p sorted sequences, find the
object of global rank k.  §4.3 (Algorithm "approxMusel", amsSelect): return
the k smallest objects for some k in [kmin, kmax].

On one device the p sequences are the rows of a CSR batch; an object is
identified by its position in the concatenation of the rows, so the unique
order of §2 is (value, position), and each row, sorted by value, is sorted in
that order too.  The result of a selection over sorted rows is a prefix of
every row: its lengths ("the split") determine it.

  ms_select   the plain definition: sort all objects (the plain oracle), take
              the first k, count them per row.
  ams_check   any split whose total lies in [kmin, kmax] and which equals the
              plain selection of that many objects is a valid result.
  ams_rho_*   the sampling rates of Algorithm "approxMusel", and the success
              probability they maximise (pinned in the tests).
"""
import math

import numpy as np

from . import select_composite, select_sort, precedes


def rows_sorted(keys, row_off, largest=False):
    """True iff every row is sorted in the unique order (value, position)."""
    keys = np.ascontiguousarray(keys)
    for r in range(len(row_off) - 1):
        a, b = int(row_off[r]), int(row_off[r + 1])
        for i in range(a, b - 1):
            if precedes(keys, i + 1, i, largest):
                return False
    return True


def ms_select(keys, row_off, k, largest=False, threads=0):
    """Object of global rank k and the split (selected prefix length of every
    row) by a full sort of all objects (threads > 0: the composite-key form
    of the sort on that many threads).  Returns (kth position, split)."""
    sel = select_composite(keys, k, largest, threads) if threads else select_sort(keys, k, largest)
    row_of = np.searchsorted(np.asarray(row_off, np.int64), sel.astype(np.int64), side="right") - 1
    split = np.bincount(row_of, minlength=len(row_off) - 1).astype(np.uint32)
    return int(sel[-1]), split


def ams_check(keys, row_off, kmin, kmax, split, largest=False):
    """0 if the split is a valid flexible-k selection, else 1 (total outside
    [kmin, kmax]) or 2 (not the set of the first `total` objects)."""
    split = np.asarray(split, np.int64)
    total = int(split.sum())
    if not (kmin <= total <= kmax):
        return 1
    lens = np.diff(np.asarray(row_off, np.int64))
    if np.any(split > lens) or np.any(split < 0):
        return 2
    _, ref = ms_select(keys, row_off, total, largest)
    return 0 if np.array_equal(ref.astype(np.int64), split) else 2


def ams_rho_min(kmin, kmax):
    """Rate of the min-based estimator (Algorithm "approxMusel"):
    1 - ((kmin - 1) / kmax)^(1 / (kmax - kmin + 1))."""
    return 1.0 - ((kmin - 1) / kmax) ** (1.0 / (kmax - kmin + 1))


def ams_rho_max(n, kmin, kmax):
    """Rate of the max-based estimator: 1 - ((n - kmax) / (n - kmin + 1))^(1 / (kmax - kmin + 1))."""
    return 1.0 - ((n - kmax) / (n - kmin + 1)) ** (1.0 / (kmax - kmin + 1))


def geometric_success(rho, kmin, kmax):
    """P(kmin <= X <= kmax) for X geometric on {1, 2, ...} with parameter rho:
    the probability that the smallest of a Bernoulli(rho) sample has a rank
    in [kmin, kmax] (§4.3)."""
    return (1.0 - rho) ** (kmin - 1) - (1.0 - rho) ** kmax


def geometric_success_sum(rho, kmin, kmax):
    """The same probability as the sum the proof of Theorem "approxMusel" writes."""
    return sum((1.0 - rho) ** (k - 1) * rho for k in range(kmin, kmax + 1))


def success_probe_kmin(kmin, kmax):
    """The proof's closed form for probe x = kmin (rho = 1/kmin):
    kmin/(kmin - 1) (1 - 1/kmin)^kmin - (1 - 1/kmin)^kmax."""
    q = 1.0 - 1.0 / kmin
    return kmin / (kmin - 1) * q ** kmin - q ** kmax
