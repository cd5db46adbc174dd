"""CPU pins of the oracle for the top-k most frequent objects (§7) and the
top-k sum aggregation (§8).

Pinned against what the paper prints and what the mathematics fixes:
  * the worked example of §7.1/§7.2 (tests/golden/pac_worked_example.txt):
    the transcribed input reproduces every printed count, PAC's estimate,
    error and EC's corrected result;
  * the sample-size equation of §7.1 and Lemma "topkec" on hand-worked values;
  * rate 1: PAC and EC equal exact counting (numpy unique);
  * the per-element sampler's rate and its Philox word;
  * the weighted sample of §8 on closed forms.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth

F = oracle.freq
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "pac_worked_example.txt")


def load_example():
    rec = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val = line.split(":", 1)
            rec[key.strip()] = val.strip()
    pes = [rec["pe%d" % i].replace(" ", "") for i in range(1, 5)]
    text = "".join(pes)
    keys = np.array([ord(c.upper()) for c in text], np.uint32)
    mask = np.array([c.islower() for c in text], bool)

    def pairs(s):
        out = []
        for item in s.split(","):
            a, b = item.split()
            out.append((ord(a), int(b)))
        return out
    return rec, keys, mask, pairs


def counts_from_mask(keys, mask, U=128):
    return np.bincount(keys[mask], minlength=U).astype(np.uint32)


def test_worked_example_counts_and_pac():
    rec, keys, mask, pairs = load_example()
    assert keys.size == 100 and mask.sum() == 29          # rho = 0.3: 29 of 100 sampled
    sc = counts_from_mask(keys, mask)
    # the hash table of the figure
    assert {c: int(sc[c]) for c in np.flatnonzero(sc)} == dict(pairs(rec["sample_counts"]))
    # the exact counts printed for the result (validates the transcription)
    ex = oracle.freq.exact_counts(keys, 128)
    for obj, cnt in pairs(rec["exact_top"]) + pairs(rec["ec_counted"]):
        assert ex[obj] == cnt, chr(obj)
    k, rho = int(rec["k"]), float(rec["rho"])
    ids, cnt = F.pac_from_counts(sc, k)
    est = {int(i): int(round(c / rho)) for i, c in zip(ids, cnt)}
    assert est == dict(pairs(rec["pac_estimate"]))
    # the exact top-k, and PAC's error: D (8) missed, O (7) returned
    eids, ecnt = F.top_by_count(ex, k)
    assert dict(zip(eids.tolist(), ecnt.tolist())) == dict(pairs(rec["exact_top"]))
    assert F.error(ex, ids) == int(rec["pac_error"])


def test_worked_example_ec_is_exact():
    rec, keys, mask, pairs = load_example()
    sc = counts_from_mask(keys, mask)
    ex = oracle.freq.exact_counts(keys, 128)
    kstar = int(rec["kstar"])
    cand, _ = F.top_by_count(sc, kstar)
    assert set(cand.tolist()) == {o for o, _ in pairs(rec["ec_counted"])}
    ids, cnt = F.ec_from_counts(sc, ex, int(rec["k"]), kstar)
    assert dict(zip(ids.tolist(), cnt.tolist())) == dict(pairs(rec["exact_top"]))
    assert F.error(ex, ids) == 0


def test_top_by_count_order_and_ties():
    counts = np.array([3, 7, 7, 0, 3, 9, 7], np.uint32)
    ids, c = F.top_by_count(counts, 5)
    assert ids.tolist() == [5, 1, 2, 6, 0] and c.tolist() == [9, 7, 7, 7, 3]
    ids, c = F.top_by_count(counts, 2, candidates=[0, 4, 6])
    assert ids.tolist() == [6, 0]


def test_sample_size_equation_hand_worked():
    # §7.1: rho n >= 4/eps^2 max(3/k ln(4n/delta), 2 ln(2k/delta)); for
    # n = 2^28, k = 32, eps = 3e-4, delta = 1e-4 the second term dominates:
    # 4/9e-8 * 2 ln(640000) = 8/9e-8 * 13.369223... = 1.18837...e9
    v = F.sample_size_pac(2**28, 32, 3e-4, 1e-4)
    assert v == pytest.approx(8 / 9e-8 * math.log(640000), rel=1e-12)
    assert v == pytest.approx(1.188375e9, rel=1e-6)
    # k = 1, n = 2^40, delta = 1/2: the first term dominates (3 ln(2^43) > 2 ln 4)
    v = F.sample_size_pac(2**40, 1, 0.01, 0.5)
    assert v == pytest.approx(4e4 * 3 * 43 * math.log(2), rel=1e-12)
    # Lemma "topkec": 2/(eps^2 k*) ln(n/delta)
    v = F.sample_size_ec(2**28, 32, 3e-4, 1e-4)
    assert v == pytest.approx(2 / (9e-8 * 32) * (28 * math.log(2) + 4 * math.log(10)), rel=1e-12)
    # k* of §7.2 reduces to k on one PE; grows like sqrt(log p / p) / eps
    assert F.kstar_paper(32, 3e-4, 2**28, 1e-4, 1) == 32
    assert F.kstar_paper(32, 3e-4, 2**28, 1e-4, 16) == \
        math.ceil(1 / 3e-4 * math.sqrt(2 * 4 / 16 * math.log(2**28 / 1e-4)))
    # thresholds: rho = sample size / n as T = rho 2^32, at most 2^32
    assert F.threshold(2**28, 2**26) == 2**30
    assert F.threshold(2**28, 1e12) == 2**32
    assert F.threshold(1000, 1) == math.ceil(2**32 / 1000)


@pytest.mark.parametrize("dist", ["zipf", "alpha"])
def test_rate_one_is_exact_counting(dist):
    n, U = 20000, 300
    keys = synth.zipf_u32(n, 1.0, U, 3) if dist == "zipf" else \
        synth.small_alphabet_u32(n, 17, 4)
    vals, cnts = np.unique(keys, return_counts=True)
    order = np.lexsort((vals, -cnts))
    for k in (1, 5, 17):
        ids, c, ns = F.pac(keys, U, k, 1 << 32, seed=9)
        assert ns == n
        assert ids.tolist() == vals[order][:k].tolist() and c.tolist() == cnts[order][:k].tolist()
        for kstar in (k, 2 * k, U):
            ids2, c2, _ = F.ec(keys, U, k, kstar, 1 << 32, seed=9)
            assert ids2.tolist() == ids.tolist() and c2.tolist() == c.tolist()


def test_ec_with_all_objects_is_exact_at_any_rate():
    n, U = 30000, 500
    keys = synth.zipf_u32(n, 1.0, U, 5)
    vals, cnts = np.unique(keys, return_counts=True)
    order = np.lexsort((vals, -cnts))
    ids, c, ns = F.ec(keys, U, 10, U, F.threshold(n, 300), seed=4)
    assert ids.tolist() == vals[order][:10].tolist() and c.tolist() == cnts[order][:10].tolist()
    assert 0 < ns < n


def test_sampler_rate_and_philox_word():
    n = 40000
    T = int(0.1 * 2**32)
    m = F.take_mask(n, T, seed=77, tag=3)
    assert abs(m.mean() - 0.1) < 5 * math.sqrt(0.09 / n)
    both = np.mean(m[:-1] & m[1:])
    assert abs(both - 0.01) < 5 * math.sqrt(0.01 / n)
    # the decision is word i % 4 of Philox4x32-10 at counter (i / 4, 0, tag, 2)
    seed = 0x0123_4567_89AB_CDEF
    L = oracle.lib()
    for i in (0, 1, 2, 3, 4, 4097, 2**33 + 6):
        w = int(oracle.philox4x32_10([(i >> 2) & 0xFFFFFFFF, 0, 5, 2],
                                     [seed & 0xFFFFFFFF, seed >> 32])[i & 3])
        assert L.orc_take(seed, 5, i, w + 1) and not L.orc_take(seed, 5, i, w)
    assert not L.orc_take(seed, 5, 9, 0) and L.orc_take(seed, 5, 9, 2**32)
    # sample counts agree with the mask
    keys = synth.zipf_u32(n, 1.0, 64, 8)
    sc, ns = F.sample_counts(keys, 64, T, seed=77, tag=3)
    assert ns == m.sum() and np.array_equal(sc, np.bincount(keys[m], minlength=64))


def test_weighted_sample_closed_forms():
    # v_avg = m / s: a key holding an integer multiple j of v_avg gets exactly
    # j samples (no Bernoulli part); here m = 1000, s = 10, v_avg = 100
    sums = np.array([300, 0, 100, 600], np.uint64)
    out, tot = F.weighted_sample(sums, 10, seed=1)
    assert out.tolist() == [3, 0, 1, 6] and tot == 10
    # fractional parts: each key gets floor or floor + 1, with the expected
    # total over many seeds
    sums = np.array([150, 250, 600], np.uint64)      # 1.5, 2.5, 6.0 samples at s = 10
    tot_mean = 0.0
    for seed in range(400):
        out, tot = F.weighted_sample(sums, 10, seed=seed)
        assert out[0] in (1, 2) and out[1] in (2, 3) and out[2] == 6
        tot_mean += tot / 400
    assert abs(tot_mean - 10.0) < 0.15
    with pytest.raises(ValueError):
        F.weighted_sample(np.zeros(4, np.uint64), 10, seed=1)


def test_sum_aggregation_rate_one_and_exact_sums():
    rng = np.random.default_rng(3)
    n, U = 5000, 200
    keys = rng.integers(0, U, n).astype(np.uint32)
    values = rng.integers(0, 1000, n).astype(np.uint32)
    sums = F.sums_by_key(keys, values, U)
    ref = np.zeros(U, np.uint64)
    np.add.at(ref, keys, values.astype(np.uint64))
    assert np.array_equal(sums, ref)
    # exact summation over every key is exact whatever the sample
    ids, s = F.sum_ec(keys, values, U, 7, U, 50, seed=2)
    order = np.lexsort((np.arange(U), -ref.astype(np.int64)))[:7]
    assert ids.tolist() == order.tolist() and s.tolist() == ref[order].tolist()
    assert F.sample_size_sum(2**28, 3e-4, 1e-4) == \
        pytest.approx(1 / 3e-4 * math.sqrt(2 * math.log(2 * 2**28 / 1e-4)))
