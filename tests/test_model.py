"""CPU tests of the test-side model of the round policy (tests/model).

The model mirrors the device's sampling and retry choices; these tests check
that running it reaches the plain oracle's result (the §2 Algorithm is exact
whatever the sample) and that each policy rule does what it says.
"""
import math

import numpy as np
import pytest

import model
import oracle
import synth


def test_hash_sampler_rate_and_independence():
    # per-element decisions: P(taken) = T / 2^32, independent of the position
    T = int(0.1 * 2**32)
    taken = np.array([model.hash_taken(77, 3, x, T) for x in range(40000)])
    p = taken.mean()
    assert abs(p - 0.1) < 5 * math.sqrt(0.1 * 0.9 / taken.size)
    # pairs of neighbours are uncorrelated
    both = np.mean(taken[:-1] & taken[1:])
    assert abs(both - 0.01) < 5 * math.sqrt(0.01 / taken.size)
    # T = 0 takes nothing, T = 2^32 takes everything; another tag is another stream
    assert not any(model.hash_taken(77, 3, x, 0) for x in range(100))
    assert all(model.hash_taken(77, 3, x, 2**32) for x in range(100))
    other = np.array([model.hash_taken(77, 4, x, T) for x in range(40000)])
    assert 0 < np.sum(taken != other) and abs(np.mean(taken & other) - 0.01) < 0.003


def test_hash_sampler_matches_philox_word():
    # the decision is word 0 of Philox4x32-10 at counter (x, 0, tag, 1), key = seed
    seed = 0x1234_5678_9ABC_DEF0
    for x, tag in ((0, 0), (5, 1), (2**31 + 7, 9)):
        w = int(oracle.philox4x32_10([x, 0, tag, 1], [seed & 0xFFFFFFFF, seed >> 32])[0])
        assert model.hash_taken(seed, tag, x, w + 1) and not model.hash_taken(seed, tag, x, w)


def test_band_threshold_hand_worked():
    # pivots cover ranks [bot, top): expected b = n (top - bot) / s, rho = s_target / that
    # n = 2^28, s = 4096, lo = 1919, hi = 2177: b ~ 2^28 * 259 / 4096 = 16973824
    assert model.band_threshold(2**28, 4096, 1919, 2177, 4096) == (4096 << 32) // 16973824
    # no lower pivot (lo < 0): bot = 0; hi = 6 -> top = 7: b ~ 2^28 * 7 / 4096 = 458752
    assert model.band_threshold(2**28, 4096, -5, 6, 4096) == (4096 << 32) // 458752
    # no pivots at all: b ~ n
    assert model.band_threshold(1000, 10, -3, 12, 4096) == (4096 << 32) // 1000


# ------------------------------------------------------------------ replay --

REPLAY_CASES = [
    dict(s_target=256, c_num=16, nseg=64, seg_cap=16, t_fin=512, r_max=32),
    dict(s_target=64, c_num=16, nseg=16, seg_cap=16, t_fin=64, r_max=64),
    dict(s_target=1024, c_num=8, nseg=1024, seg_cap=4, t_fin=2048, r_max=32),
    dict(s_target=128, c_num=0, nseg=32, seg_cap=16, t_fin=100, r_max=200),  # many misses
]


def _replay_equals_plain(keys, k, largest, prm, seed, band_cap=None):
    n = keys.size
    rc, out, kth, recs = model.replay(keys, k, largest, seed=seed,
                                       band_cap=band_cap or n, **prm)
    assert rc == 0, (rc, recs[-3:])
    ref = oracle.select_sort(keys, k, largest)
    assert np.array_equal(np.sort(out), np.sort(ref))
    assert kth == int(ref[-1])
    # every round that recursed bracketed rank k_cur and shrank the problem
    for r in recs:
        if r["ok"]:
            assert r["na"] < r["k_cur"] <= r["na"] + r["nb"] and r["nb"] < r["n_cur"]
    return recs


@pytest.mark.parametrize("case", range(len(REPLAY_CASES)))
@pytest.mark.parametrize("largest", [False, True])
def test_replay_equals_plain_oracle(case, largest):
    prm = REPLAY_CASES[case]
    rng = np.random.default_rng(case)
    gens = [lambda n, s: synth.uniform_u32(n, s),
            lambda n, s: synth.small_alphabet_u32(n, 3, s),
            lambda n, s: synth.specials_f32(n, s),
            lambda n, s: synth.uniform_f32_grid(n, s),
            lambda n, s: synth.zipf_u32(n, 1.2, 2**16, s),
            lambda n, s: synth.all_equal_except(n, 0.01, 2**31, s)]
    for gi, g in enumerate(gens):
        n = int(rng.integers(1, 60000))
        keys = g(n, 100 * case + gi)
        for k in {1, n, max(1, n // 2), int(rng.integers(1, n + 1))}:
            _replay_equals_plain(keys, k, largest, prm, seed=gi * 7 + case)


def test_replay_rounds_and_output_layout():
    # a-elements of each round are written in sequence order, so the first
    # round's segment is ascending in position
    keys = synth.uniform_u32(200000, 4)
    k = 100000
    prm = dict(s_target=512, c_num=16, nseg=128, seg_cap=16, t_fin=256, r_max=32)
    rc, out, kth, recs = model.replay(keys, k, seed=1, band_cap=200000, **prm)
    assert rc == 0 and len(recs) >= 2
    na1 = recs[0]["na"]
    assert recs[0]["ok"] and np.all(np.diff(out[:na1].astype(np.int64)) > 0)


def test_replay_wide_band_halves_spread():
    # s_target = 16 at the median: Delta >= s/2 with c = 4, so b is the whole
    # subproblem; halving c restores progress
    keys = synth.small_alphabet_u32(20000, 5, 4)
    rc, out, kth, recs = model.replay(keys, 10000, s_target=16, c_num=16, nseg=1024,
                                       seg_cap=16, t_fin=512, r_max=32, band_cap=20000, seed=5)
    assert rc == 0
    assert not recs[0]["ok"] and recs[0]["nb"] == recs[0]["n_cur"]
    assert recs[1]["c_num"] == 8
    ref = oracle.select_sort(keys, 10000)
    assert np.array_equal(np.sort(out), np.sort(ref)) and kth == ref[-1]


def test_replay_miss_doubles_spread():
    keys = synth.uniform_u32(300000, 9)
    rc, out, kth, recs = model.replay(keys, 77, s_target=256, c_num=0, nseg=1024,
                                       seg_cap=16, t_fin=512, r_max=32, band_cap=300000, seed=3)
    assert rc == 0
    for a, b in zip(recs, recs[1:]):
        if not a["ok"] and (a["na"] >= a["k_cur"] or a["na"] + a["nb"] < a["k_cur"]):
            assert b["c_num"] == min(2 * a["c_num"], 4096)


def test_replay_band_cap_overflow_then_exact_round():
    # every sampled round is too wide for a band of 10: after r_max attempts
    # the exact round takes the object of rank k as both pivots and finishes
    keys = synth.uniform_u32(50000, 5)
    prm = dict(s_target=64, c_num=16, nseg=16, seg_cap=16, t_fin=64, r_max=6)
    rc, out, kth, recs = model.replay(keys, 25000, seed=1, band_cap=10, **prm)
    assert rc == 0 and len(recs) == 7 and not any(r["ok"] for r in recs[:6])
    ex = recs[6]
    assert ex["ok"] and ex["lo"] == ex["hi"] == model.ROUND_EXACT and ex["s"] == 0
    ref = oracle.select_sort(keys, 25000)
    assert ex["l_idx"] == ex["r_idx"] == ref[-1] == kth
    assert ex["na"] == 24999 and ex["nb"] == 1
    assert np.array_equal(np.sort(out), np.sort(ref))


@pytest.mark.parametrize("largest", [False, True])
def test_replay_exact_round_with_tiny_t_fin(largest):
    # t_fin = 1 and a short budget: the exact round always finishes the call
    keys = synth.small_alphabet_u32(20000, 5, 4)
    for k in (1, 2, 9999, 20000):
        rc, out, kth, recs = model.replay(keys, k, largest, s_target=16, c_num=16, nseg=1024,
                                          seg_cap=16, t_fin=1, r_max=3, band_cap=20000, seed=5)
        assert rc == 0
        ref = oracle.select_sort(keys, k, largest)
        assert np.array_equal(np.sort(out), np.sort(ref)) and kth == ref[-1]


def test_replay_direct_finish_when_small():
    keys = synth.uniform_u32(100, 6)
    rc, out, kth, recs = model.replay(keys, 40, s_target=64, c_num=16, nseg=4, seg_cap=64,
                                       t_fin=100, r_max=4, band_cap=100, seed=3)
    assert rc == 0 and recs == []
    ref = oracle.select_sort(keys, 40)
    assert kth == ref[-1]
    # the direct finish writes the selected elements in position order
    assert np.array_equal(out, np.sort(ref))




@pytest.mark.parametrize("largest", [False, True])
def test_model_traces_pass_the_definitional_round_check(largest):
    # the checker the GPU tests apply to device traces accepts the model's
    # traces (misses, too-wide rounds and the exact round included) ...
    from roundcheck import check_rounds
    keys = synth.zipf_u32(300000, 1.2, 2**16, 3)
    for k, c_num, r_max, cap in ((1, 8, 5, 300000), (1000, 0, 5, 300000),
                                 (150000, 8, 5, 300000), (150000, 16, 3, 10)):
        rc, out, kth, recs = model.replay(keys, k, largest, seed=1, band_cap=cap, s_target=256,
                                          c_num=c_num, nseg=64, seg_cap=16, t_fin=512, r_max=r_max)
        assert rc == 0
        check_rounds(keys, k, largest, recs, cap)
    # ... and rejects a trace with a miscounted |a|
    rc, out, kth, recs = model.replay(keys, 1000, largest, seed=1, band_cap=300000, s_target=256,
                                      c_num=8, nseg=64, seg_cap=16, t_fin=512, r_max=5)
    bad = [dict(r) for r in recs]
    bad[0]["na"] += 1
    with pytest.raises(AssertionError):
        check_rounds(keys, 1000, largest, bad, 300000)
