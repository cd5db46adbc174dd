"""Pins of the CPU oracle against facts fixed outside it (no GPU).

Each pin is chosen so that a plausible slip in the oracle -- a flipped
comparison, a dropped tie rule, a wrong NaN/zero rule, an off-by-one rank, a
wrong Philox constant, a wrong skip law -- fails at least one test here.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load_golden(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- Philox ----

def test_philox_known_answers():
    for r in _load_golden("philox4x32_10_kat.txt"):
        v = [int(x, 16) for x in r]
        out = oracle.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_philox_uniformity_of_words():
    # 4096 blocks of 4 words: byte histogram is flat (chi-square, 255 dof).
    words = np.concatenate([oracle.philox4x32_10([i, 7, 3, 0], [11, 13]) for i in range(4096)])
    b = words.view(np.uint8)
    h = np.bincount(b, minlength=256)
    e = b.size / 256
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < 255 + 6 * math.sqrt(2 * 255)


# ------------------------------------------------------- key order & select --

def _brute_vs_sort(keys, k, largest):
    sel_b, kth_b = oracle.select_brute(keys, k, largest)
    sel_s = oracle.select_sort(keys, k, largest)
    assert np.array_equal(np.sort(sel_s), sel_b)
    assert int(sel_s[-1]) == kth_b
    bits = keys.view(np.uint32)
    assert oracle.check(keys, k, sel_s, kth_b, int(bits[kth_b]), largest) == 0


@pytest.mark.parametrize("largest", [False, True])
@pytest.mark.parametrize("seed", range(4))
def test_brute_force_small_alphabets(seed, largest):
    rng = np.random.default_rng(seed)
    for alphabet in (1, 2, 4, 256, 2**32):
        n = int(rng.integers(1, 600))
        keys = (synth.small_alphabet_u32(n, alphabet, seed) if alphabet < 2**32
                else synth.uniform_u32(n, seed))
        for k in {1, n, max(1, n // 2), max(1, n // 7)}:
            _brute_vs_sort(keys, k, largest)


@pytest.mark.parametrize("largest", [False, True])
@pytest.mark.parametrize("seed", range(4))
def test_brute_force_float_specials(seed, largest):
    n = 300 + 50 * seed
    keys = synth.specials_f32(n, seed)
    for k in (1, 2, n // 3, n // 2, n - 1, n):
        _brute_vs_sort(keys, k, largest)


def test_float_order_facts():
    # NaN above +inf, all NaNs tie, -0 ties +0, subnormal above 0, -inf lowest.
    x = np.array([np.nan, np.inf, -0.0, 0.0, 1e-45, -np.inf, np.nan], np.float32)
    x.view(np.uint32)[6] = 0xFFC00001  # negative-signed NaN with payload
    P = lambda i, j, lg=False: oracle.precedes(x, i, j, lg)
    assert P(1, 0) and not P(0, 1)            # inf < NaN
    assert P(0, 6) and not P(6, 0)            # NaN ties NaN: by position
    assert P(2, 3) and not P(3, 2)            # -0 ties +0: by position
    assert P(3, 4)                            # 0 < smallest subnormal
    assert P(5, 2)                            # -inf lowest
    assert P(0, 1, True) and P(6, 1, True)    # largest: NaNs first
    assert P(2, 3, True)                      # ties still by ascending position


@pytest.mark.parametrize("seed", range(3))
def test_numpy_stable_argsort_smallest(seed):
    # numpy's stable argsort orders by value (NaN last, -0 == +0) then position
    n = 20000
    for keys in (synth.uniform_u32(n, seed), synth.small_alphabet_u32(n, 50, seed),
                 synth.specials_f32(n, seed), synth.uniform_f32_grid(n, seed)):
        ref = np.argsort(keys, kind="stable")
        for k in (1, 17, n // 2, n):
            got = oracle.select_sort(keys, k)
            assert np.array_equal(got, ref[:k].astype(np.uint32))


@pytest.mark.parametrize("seed", range(3))
def test_numpy_stable_argsort_largest_u32(seed):
    # bitwise complement reverses the unsigned order: largest-first = argsort(~x)
    n = 20000
    keys = synth.small_alphabet_u32(n, 97, seed)
    ref = np.argsort(~keys, kind="stable")
    for k in (1, 1000, n):
        assert np.array_equal(oracle.select_sort(keys, k, largest=True), ref[:k].astype(np.uint32))


def test_numpy_partition_kth_value():
    keys = synth.uniform_f32_grid(50000, 9)
    for k in (1, 10, 25000, 50000):
        sel = oracle.select_sort(keys, k)
        assert keys[sel[-1]] == np.partition(keys, k - 1)[k - 1]


# ------------------------------------------------------------ closed forms --

def test_closed_forms():
    n = 5000
    asc = np.arange(n, dtype=np.uint32)
    for k in (1, 77, n):
        assert np.array_equal(np.sort(oracle.select_sort(asc, k)), np.arange(k))
        desc = asc[::-1].copy()
        assert np.array_equal(np.sort(oracle.select_sort(desc, k)), np.arange(n - k, n))
        perm = np.random.default_rng(k).permutation(n).astype(np.uint32)
        sel = oracle.select_sort(perm, k)
        assert np.array_equal(np.sort(sel), np.sort(np.nonzero(perm < k)[0]))
        assert perm[sel[-1]] == k - 1
        eq = np.full(n, 12345, np.uint32)
        sel = oracle.select_sort(eq, k)
        assert np.array_equal(sel, np.arange(k)) and sel[-1] == k - 1
        # largest on all-equal: still the first k positions
        assert np.array_equal(oracle.select_sort(eq, k, True), np.arange(k))


def test_closed_form_all_equal_except():
    n, C = 40000, 2**31
    keys = synth.all_equal_except(n, 0.01, C, 31)
    below = np.nonzero(keys < C)[0]
    ties = np.nonzero(keys == C)[0]
    k = len(below) + 1000
    sel = oracle.select_sort(keys, k)
    expect = np.sort(np.concatenate([below, ties[:1000]]))
    assert np.array_equal(np.sort(sel), expect)
    assert sel[-1] == ties[999]


def test_closed_form_zipf_head():
    keys = synth.zipf_u32(100000, 1.2, 2**16, 3)
    zeros = np.nonzero(keys == 0)[0]
    k = len(zeros) // 2
    sel = oracle.select_sort(keys, k)
    assert np.array_equal(sel, zeros[:k])


def test_zipf_generator_head_frequency():
    # P(rank 1) = 1 / H_{V,s}; H_{2^16,1.2} = 5.0466... (direct sum)
    V, s = 2**16, 1.2
    H = float(np.sum(np.arange(1, V + 1, dtype=np.float64) ** -s))
    keys = synth.zipf_u32(1 << 20, s, V, 5)
    f = np.mean(keys == 0)
    assert abs(f - 1 / H) < 5 * math.sqrt((1 / H) * (1 - 1 / H) / keys.size)


# ---------------------------------------------------------------- checker --

def _valid(keys, k, largest=False):
    sel = oracle.select_sort(keys, k, largest)
    return sel, int(sel[-1])


@pytest.mark.parametrize("largest", [False, True])
def test_checker_accepts_valid_and_catches_planted_mistakes(largest):
    keys = synth.small_alphabet_u32(3000, 40, 1)
    bits = keys.view(np.uint32)
    k = 1500
    sel, kth = _valid(keys, k, largest)
    assert oracle.check(keys, k, sel, kth, int(bits[kth]), largest) == 0
    # any order of the same set is fine
    assert oracle.check(keys, k, sel[::-1].copy(), kth, int(bits[kth]), largest) == 0
    # repeated index
    bad = sel.copy(); bad[0] = bad[1]
    assert oracle.check(keys, k, bad, kth, int(bits[kth]), largest) == 1
    # index out of range
    bad = sel.copy(); bad[3] = 3000
    assert oracle.check(keys, k, bad, kth, int(bits[kth]), largest) == 1
    # kth index not selected
    unsel = np.setdiff1d(np.arange(3000), sel)
    assert oracle.check(keys, k, sel, int(unsel[-1]), int(bits[unsel[-1]]), largest) in (2,)
    # swap the best-ranked selected element for the worst unselected one
    full = oracle.select_sort(keys, 3000, largest)
    bad = sel.copy(); bad[0] = full[-1]
    assert oracle.check(keys, k, bad, kth, int(bits[kth]), largest) in (3, 4)
    # tie rule: replace the last selected tie by a later-positioned tie
    t = keys[kth]
    ties_unsel = [j for j in np.nonzero(keys == t)[0] if j not in set(sel.tolist())]
    bad = sel.copy(); bad[-1] = ties_unsel[-1]
    assert oracle.check(keys, k, bad, int(ties_unsel[-1]), int(bits[ties_unsel[-1]]), largest) == 6
    # kth_idx another selected tie (not the last one)
    sel_ties = [j for j in sel.tolist() if keys[j] == t]
    if len(sel_ties) > 1:
        assert oracle.check(keys, k, sel, sel_ties[0], int(bits[sel_ties[0]]), largest) == 7
    # kth key bits wrong
    assert oracle.check(keys, k, sel, kth, int(bits[kth]) ^ 1, largest) == 8


def test_checker_float_bits_matter():
    keys = np.array([-0.0, 0.0, 1.0, np.nan], np.float32)
    sel, kth = _valid(keys, 1)
    assert kth == 0
    assert oracle.check(keys, 1, sel, 0, 0x80000000) == 0
    assert oracle.check(keys, 1, sel, 0, 0x00000000) == 8


# ---------------------------------------------------------------- sampler --

def test_sampler_positions_valid_and_rate():
    n, rho = 1 << 20, 4096 / (1 << 20)
    counts = []
    for tag in range(40):
        pos = oracle.bernoulli_sample(n, rho, 1234, tag, 1024, 64)
        assert np.all(np.diff(pos.astype(np.int64)) > 0)
        assert pos.size == 0 or pos[-1] < n
        counts.append(pos.size)
    # sample size ~ Binomial(n, rho): mean 4096, sd 64
    m = np.mean(counts)
    assert abs(m - 4096) < 5 * 64 / math.sqrt(len(counts))
    assert abs(np.std(counts) - 64) < 25


@pytest.mark.parametrize("rho", [0.5, 0.05, 0.003])
def test_sampler_skips_are_geometric(rho):
    # one segment: gaps between consecutive sampled positions ~ Geometric(rho)
    n = 2_000_000 if rho < 0.01 else 400_000
    pos = oracle.bernoulli_sample(n, rho, 99, 5, 1, 1 << 24).astype(np.int64)
    gaps = np.diff(np.concatenate([[-1], pos]))
    # bins 1..B-1 exact, B = tail; expected P(G=j) = (1-rho)^(j-1) rho
    B = 20 if rho > 0.1 else 60
    scale = 1 if rho > 0.01 else 10
    g = np.minimum((gaps - 1) // scale, B)
    obs = np.bincount(g, minlength=B + 1)
    j = np.arange(B + 1)
    p_bin = (1 - rho) ** (j * scale) - (1 - rho) ** ((j + 1) * scale)
    p_bin[B] = (1 - rho) ** (B * scale)
    exp = p_bin * gaps.size
    mask = exp > 5
    chi2 = ((obs[mask] - exp[mask]) ** 2 / exp[mask]).sum()
    dof = mask.sum() - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_sampler_segmentation_is_memoryless():
    # cutting positions into segments that restart the skip walk leaves each
    # position's inclusion probability at rho (checked per position class)
    n, rho = 5000, 0.1
    hits = np.zeros(n)
    T = 300
    for tag in range(T):
        hits[oracle.bernoulli_sample(n, rho, 7, tag, 37, 10**6)] += 1
    p = hits / T
    # segment starts and ends are not special
    L = (n + 36) // 37
    starts = np.arange(0, n, L)
    sd = math.sqrt(rho * (1 - rho) / (T * len(starts)))
    assert abs(p[starts].mean() - rho) < 5 * sd
    assert abs(p.mean() - rho) < 5 * math.sqrt(rho * (1 - rho) / (T * n))


def test_sampler_full_rate_and_caps():
    pos = oracle.bernoulli_sample(1000, 1.0, 1, 0, 10, 1000)
    assert np.array_equal(pos, np.arange(1000))
    pos = oracle.bernoulli_sample(1000, 1.0, 1, 0, 10, 7)   # 7 per segment of 100
    assert pos.size == 70 and np.all(pos % 100 < 7)
    pos = oracle.bernoulli_sample(100000, 0.5, 1, 0, 4, 3)
    assert pos.size == 12


# ---------------------------------------------------------------- pivots ----

def test_pivot_ranks_hand_worked():
    for r in _load_golden("pivot_ranks.txt"):
        s, k, n, c, lo, hi = map(int, r)
        assert oracle.pivot_ranks(s, k, n, c) == (lo, hi), r


def test_pivot_bracketing_rate():
    # With c = 4 the pivots miss rank k with probability about 2*Phi(-4) ~ 6e-5;
    # over 2000 random samples of a 2^16 permutation expect (almost) no misses,
    # and with c = 0.5 expect many.
    n, s_t = 1 << 16, 1024
    rng = np.random.default_rng(3)
    perm = rng.permutation(n).astype(np.uint32)   # key = rank - 1
    miss4 = miss05 = 0
    for t in range(2000):
        k = int(rng.integers(1, n + 1))
        pos = oracle.bernoulli_sample(n, s_t / n, 5, t, 64, 64)
        S = np.sort(perm[pos])
        for c_num, cnt in ((16, "4"), (2, "05")):
            lo, hi = oracle.pivot_ranks(S.size, k, n, c_num)
            lv = S[lo] if lo >= 0 else -1
            hv = S[hi] if hi < S.size else n
            ok = lv <= k - 1 <= hv
            if not ok:
                if cnt == "4":
                    miss4 += 1
                else:
                    miss05 += 1
    assert miss4 <= 2
    assert miss05 > 200


# ------------------------------------------------------- composite sort ---

@pytest.mark.parametrize("gen", ["u32", "alpha3", "specials", "grid"])
@pytest.mark.parametrize("largest", [False, True])
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_composite_sort_equals_plain_oracle(gen, largest, threads):
    # the timed form (composite keys, chunked over threads) is the plain
    # comparator sort: same first k, in the same order
    n = 20011
    keys = {"u32": synth.uniform_u32(n, 8), "alpha3": synth.small_alphabet_u32(n, 3, 9),
            "specials": synth.specials_f32(n, 10), "grid": synth.uniform_f32_grid(n, 11)}[gen]
    for k in (1, 2, 777, n // 2, n):
        a = oracle.select_composite(keys, k, largest, threads)
        b = oracle.select_sort(keys, k, largest)
        assert np.array_equal(a, b), (gen, k)


# ------------------------------------------------------------------ ranks ---

@pytest.mark.parametrize("gen", ["u32", "alpha3", "specials"])
@pytest.mark.parametrize("largest", [False, True])
def test_rank_is_position_in_sorted_order(gen, largest):
    # rank(x) = #{objects before x}: the position of x in the full sort, and
    # the brute-force selection of k holds exactly the objects of rank < k
    n = 700
    keys = {"u32": synth.uniform_u32(n, 3), "alpha3": synth.small_alphabet_u32(n, 3, 4),
            "specials": synth.specials_f32(n, 5)}[gen]
    perm = oracle.select_sort(keys, n, largest)
    for pos in (0, 1, 17, 350, n - 2, n - 1):
        assert oracle.rank(keys, int(perm[pos]), largest) == pos
    sel, kth = oracle.select_brute(keys, 123, largest)
    ranks = np.array([oracle.rank(keys, int(x), largest) for x in range(n)])
    assert np.array_equal(np.flatnonzero(ranks < 123), np.sort(sel))
    assert ranks[kth] == 122


def test_rank_among_counts_subset():
    keys = synth.small_alphabet_u32(500, 4, 7)
    xs = np.array([3, 99, 250, 499], np.uint32)
    ys = np.arange(0, 500, 3, dtype=np.uint32)
    got = oracle.rank_among(keys, xs, ys)
    for x, g in zip(xs, got):
        want = sum(1 for y in ys if y != x and oracle.precedes(keys, int(y), int(x)))
        assert g == want
    # among all objects it is the rank
    assert list(oracle.rank_among(keys, xs, np.arange(500, dtype=np.uint32))) == \
        [oracle.rank(keys, int(x)) for x in xs]


# ---------------------------------------------------------- rows / scatter --

def test_topk_rows_matches_torch_on_tie_free_rows():
    torch = pytest.importorskip("torch")
    s = synth.normal_f32((8, 3000), 5)
    vals, idx = oracle.topk_rows(s, 64)
    tv, ti = torch.topk(torch.from_numpy(s), 64, dim=1)
    assert np.array_equal(vals, tv.numpy()) and np.array_equal(idx, ti.numpy())


def test_scatter_rows_is_topk_values_gradient():
    torch = pytest.importorskip("torch")
    s = synth.normal_f32((4, 500), 6)
    g = synth.normal_f32((4, 16), 7)
    _, idx = oracle.topk_rows(s, 16)
    x = torch.from_numpy(s).requires_grad_(True)
    v, _ = torch.topk(x, 16, dim=1)
    v.backward(torch.from_numpy(g))
    assert np.array_equal(oracle.scatter_rows(g, idx, 500), x.grad.numpy())
