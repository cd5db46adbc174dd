"""Definitional check of a device round trace (test helper).

Every recorded round of the §2 Algorithm is checked against what the paper
fixes, using only the oracle:
  * the subproblem entering a round is the interval of the unique order
    between the last lower and upper pivots (rank interval [A, B]), so
    n_cur = B - A + 1 and k_cur = k - A;
  * the pivot ranks lo, hi are the oracle's pivot_ranks(s, k_cur, n_cur, c);
  * the pivots are the sample objects of ranks lo and hi (the traced sample
    is sorted by the oracle), and every sample object lies in [A, B];
  * |a| = rank(l) - A and |b| = rank(r) - rank(l) + 1 (ranks by the oracle);
  * the round recursed into b exactly when l and r bracket rank k_cur and b
    fits its buffer and shrank the subproblem;
  * an exact round (after the attempt budget) has both pivots equal to the
    object of rank k_cur of the subproblem.
No step depends on how the device drew its sample.
"""
import numpy as np

import oracle

ROUND_EXACT = -2


def sample_order(keys, sample, largest):
    """The sample objects in the unique order of §2."""
    s = np.sort(np.asarray(sample, np.uint32))
    if s.size == 0:
        return s
    perm = oracle.select_sort(keys[s], s.size, largest)
    return s[perm]


def check_rounds(keys, k, largest, recs, band_cap, sample_of=None):
    """Check recs (dicts from trace_rounds) definitionally; sample_of(tag)
    returns the traced sample objects of a round (or None to skip that part).
    Returns the number of rounds that recursed into b."""
    n = keys.size
    A, B = 0, n - 1
    n_cur, k_cur = n, k
    oks = 0
    for r in recs:
        assert (r["n_cur"], r["k_cur"]) == (n_cur, k_cur), r
        if r["hi"] == ROUND_EXACT:      # a sampled round has hi >= 0
            assert r["lo"] == ROUND_EXACT and r["s"] == 0 and r["has_l"] and r["has_r"], r
            assert r["l_idx"] == r["r_idx"], r
            rl = rr = oracle.rank(keys, r["l_idx"], largest)
            assert rl == A + k_cur - 1, (r, A)
            has_l = has_r = True
        else:
            s = r["s"]
            lo, hi = oracle.pivot_ranks(s, k_cur, n_cur, r["c_num"])
            assert (r["lo"], r["hi"]) == (lo, hi), r
            has_l, has_r = lo >= 0, hi < s
            assert (bool(r["has_l"]), bool(r["has_r"])) == (has_l, has_r), r
            if sample_of is not None:
                S = sample_of(r["tag"])
                if S is not None:
                    S = np.asarray(S, np.uint32)
                    assert S.size == s and np.unique(S).size == s, (r, S.size)
                    srt = sample_order(keys, S, largest)
                    if has_l:
                        assert r["l_idx"] == srt[lo], r
                    if has_r:
                        assert r["r_idx"] == srt[hi], r
                    # the sample lies in the subproblem [A, B]: its first and
                    # last objects in the order do
                    if s and A > 0:
                        assert oracle.rank(keys, int(srt[0]), largest) >= A, r
                    if s and B < n - 1:
                        assert oracle.rank(keys, int(srt[-1]), largest) <= B, r
            rl = oracle.rank(keys, r["l_idx"], largest) if has_l else A
            rr = oracle.rank(keys, r["r_idx"], largest) if has_r else B
            assert A <= rl <= rr <= B, (r, A, B, rl, rr)
        na = rl - A if has_l else 0
        nb = rr - (rl if has_l else A) + 1
        assert (r["na"], r["nb"]) == (na, nb), (r, na, nb)
        ok = na < k_cur <= na + nb and nb <= band_cap and nb < n_cur
        assert bool(r["ok"]) == ok, (r, ok)
        if ok:
            oks += 1
            if has_l:
                A = rl
            if has_r:
                B = rr
            k_cur -= na
            n_cur = nb
            assert B - A + 1 == n_cur
    return oks
