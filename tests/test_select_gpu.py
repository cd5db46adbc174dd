"""GPU parity of the single-instance selection against the CPU oracle.

Parity (exact, integer/index work):
  * the selected set, the k-th position and the k-th key bits equal the plain
    oracle's (full sort by (value, position));
  * every recorded round is checked definitionally (tests/roundcheck.py):
    counts |a|, |b| as oracle rank differences of the pivots, pivot ranks by
    the oracle's formula, pivots as the traced sample's objects of those ranks.
Beside parity, the round trace is compared with the test-side model of the
device's sampling and retry policy (tests/model), which explains the trace
but decides nothing about the result.
"""
import numpy as np
import pytest
import torch

import model
import oracle
import synth
from roundcheck import ROUND_EXACT, check_rounds

pytestmark = pytest.mark.gpu

tk = pytest.importorskip("paper_1502_03942_amd")

DISTS = {
    "u32": lambda n, s: synth.uniform_u32(n, s),
    "u32_ties3": lambda n, s: synth.small_alphabet_u32(n, 3, s),
    "f32_special": lambda n, s: synth.specials_f32(n, s),
    "f32_grid": lambda n, s: synth.uniform_f32_grid(n, s),
    "zipf": lambda n, s: synth.zipf_u32(n, 1.2, 2**16, s),
    "all_eq_1pct": lambda n, s: synth.all_equal_except(n, 0.01, 2**31, s),
}


def to_dev(a, dev):
    t = torch.from_numpy(a.view(np.int32) if a.dtype == np.uint32 else a)
    return t.to(dev)


def model_params(ctx, n):
    g = ctx.get_param
    t_fin = g("t_fin")
    cap = 0 if n <= t_fin else min(n, n // g("band_div") + 65536)
    return dict(s_target=g("s_target"), c_num=g("c_num"), nseg=1024, seg_cap=16,
                t_fin=t_fin, r_max=g("r_max"), band_cap=cap, seed=g("seed"))


def band_cap(ctx, n):
    return 0 if n <= ctx.get_param("t_fin") else min(n, n // ctx.get_param("band_div") + 65536)


def run_and_compare(ctx, keys_np, k, largest, dev, offset=0, trace=True, exact_trace=True):
    n = keys_np.size
    if offset:
        buf = to_dev(np.concatenate([np.zeros(offset, keys_np.dtype), keys_np]), dev)
        keys = buf[offset:]
    else:
        keys = to_dev(keys_np, dev)
    res = ctx.select(keys, k, largest=largest, write_keys=True, trace=trace)
    torch.cuda.synchronize()
    status = int(res["status"].item())
    got = res["idx"].cpu().numpy().view(np.uint32)
    kth_idx = int(res["kth_idx"].item())
    kth_bits = int(res["kth_key"].cpu().numpy().view(np.uint32)[0])
    got_keys = res["keys"].cpu().numpy().view(np.uint32)
    bits = keys_np.view(np.uint32)
    assert status == 0, status
    # parity with the plain oracle
    ref = oracle.select_sort(keys_np, k, largest)
    assert np.array_equal(np.sort(got), np.sort(ref)), "selected set differs from the oracle"
    assert kth_idx == int(ref[-1])
    assert kth_bits == int(bits[ref[-1]])
    assert np.array_equal(got_keys, bits[got])
    # every round, definitionally
    recs = ctx.trace_rounds(res)
    sample_of = (lambda tag: ctx.trace_sample(res, tag)) if trace else None
    check_rounds(keys_np, k, largest, recs, band_cap(ctx, n), sample_of)
    # the model of the sampling and retry policy reproduces the trace
    rc, _, mkth, mrecs = model.replay(keys_np, k, largest, **model_params(ctx, n))
    assert rc == 0 and mkth == kth_idx
    if exact_trace:
        assert recs == mrecs
    else:
        # a repeated round on a middle part samples positions of b, whose
        # physical order follows the sweep's reservations: equal up to there
        for g, r in zip(recs, mrecs):
            assert g == r, (g, r)
            if not g["ok"] and g["n_cur"] < n:
                break
    if trace and mrecs and mrecs[0]["hi"] != ROUND_EXACT:
        # round 1's sampled objects follow the skip sampler's law exactly
        p = model_params(ctx, n)
        pos = np.sort(np.array(ctx.trace_sample(res, 0), np.uint32))
        want = oracle.bernoulli_sample(n, p["s_target"] / n, p["seed"], 0, 1024, 16)
        assert np.array_equal(pos, want)
    return recs


@pytest.fixture(scope="module")
def ctx(dev):
    return tk.Context(0, seed=20240601)


@pytest.mark.parametrize("dist", sorted(DISTS))
@pytest.mark.parametrize("largest", [False, True])
def test_parity_sizes(ctx, dev, dist, largest):
    rng = np.random.default_rng(len(dist) * 31 + largest)
    for n in (1, 7, 8192, 8193, 50021, 1 << 20):
        keys = DISTS[dist](n, n % 1000 + 3)
        for k in sorted({1, n, max(1, n // 2), int(rng.integers(1, n + 1))}):
            run_and_compare(ctx, keys, k, largest, dev)


@pytest.mark.parametrize("offset", [1, 2, 3])
def test_parity_misaligned_keys(ctx, dev, offset):
    keys = synth.uniform_u32((1 << 20) + 5, 77)
    for k in (1000, 500000):
        run_and_compare(ctx, keys, k, False, dev, offset=offset)
    keysf = synth.specials_f32(300001, 78)
    run_and_compare(ctx, keysf, 150000, True, dev, offset=offset)


@pytest.mark.parametrize("r_fast", [0, 1, 2, 5])
def test_parity_round_schedules(dev, r_fast):
    # the same rounds run either as multi-workgroup sweeps or in the tail kernel
    c = tk.Context(0, seed=99).set_param("r_fast", r_fast).set_param("s_target", 512)
    keys = synth.uniform_f32_grid(1 << 21, 5)
    for k in (1, 1 << 10, 1 << 20, 1 << 21):
        recs = run_and_compare(c, keys, k, False, dev)
        assert all(r["ok"] for r in recs)


def test_parity_repeated_rounds(dev):
    # c = 0 makes the pivots miss often: rounds are repeated with c doubled
    c = tk.Context(0, seed=3).set_param("c_num", 0).set_param("s_target", 256)
    c.set_param("t_fin", 512)
    keys = synth.uniform_u32(300000, 9)
    misses = 0
    for k in (1, 77, 150000, 299999):
        recs = run_and_compare(c, keys, k, True, dev, exact_trace=False)
        misses += sum(1 for r in recs if not r["ok"])
    assert misses > 0


@pytest.mark.parametrize("largest", [False, True])
def test_exact_fallback_after_band_overflow(dev, largest):
    # every sampled round is too wide for its band (band_div 64, tiny sample,
    # huge spread): after r_max attempts the exact round finishes the call
    c = tk.Context(0, seed=3).set_param("band_div", 64).set_param("s_target", 64)
    c.set_param("c_num", 4096).set_param("r_max", 3).set_param("t_fin", 1024)
    keys = synth.uniform_u32(1 << 20, 10)
    recs = run_and_compare(c, keys, 1 << 19, largest, dev)
    assert [r["hi"] for r in recs][-1] == ROUND_EXACT and not any(r["ok"] for r in recs[:3])


@pytest.mark.parametrize("dist", ["u32", "zipf", "f32_special"])
def test_exact_fallback_on_a_band(dev, dist):
    # two sampled rounds succeed with a tiny sample, then the budget is spent
    # on a middle part (band input) and the exact round finishes it
    c = tk.Context(0, seed=8).set_param("s_target", 64).set_param("t_fin", 64)
    c.set_param("r_max", 2).set_param("r_fast", 2)
    keys = DISTS[dist](1 << 20, 41)
    exact = 0
    for k, largest in ((1, False), (5000, True), (1 << 19, False), (1 << 20, True)):
        recs = run_and_compare(c, keys, k, largest, dev, exact_trace=False)
        last = recs[-1]
        # the call ends in the exact round or in a sampled round that leaves
        # at most t_fin objects for the finisher
        assert last["hi"] == ROUND_EXACT or (last["ok"] and last["nb"] <= 64)
        exact += last["hi"] == ROUND_EXACT
    assert exact > 0


def test_exact_fallback_first_round_multi_workgroup(dev):
    # c = 0 with r_max = 1: the first (multi-workgroup) round misses often;
    # the exact round then runs over the whole input
    c = tk.Context(0, seed=1).set_param("c_num", 0).set_param("r_max", 1).set_param("r_fast", 1)
    keys = synth.uniform_f32_grid(1 << 22, 12)
    exact = 0
    for k in (1, 777, 1 << 21, (1 << 22) - 3):
        recs = run_and_compare(c, keys, k, False, dev)
        exact += sum(1 for r in recs if r["hi"] == ROUND_EXACT)
    assert exact > 0


def test_small_t_fin_and_sample(dev):
    # s_target = 16 leaves b as wide as the subproblem near the median until
    # the spread c has been halved: exercises the "too wide" repeat
    c = tk.Context(0, seed=5).set_param("t_fin", 512).set_param("s_target", 16)
    c.set_param("r_max", 32)
    keys = synth.small_alphabet_u32(20000, 5, 4)
    wide = 0
    for k in (1, 2, 10000, 20000):
        recs = run_and_compare(c, keys, k, False, dev, exact_trace=False)
        wide += sum(1 for r in recs if not r["ok"] and r["nb"] == r["n_cur"])
    assert wide > 0


def test_tiny_t_fin_finishes_exactly(dev):
    # a subproblem of 2 elements cannot shrink below t_fin = 1 by sampling
    # (every round's b keeps both); the exact round after r_max finishes it
    c = tk.Context(0, seed=5).set_param("t_fin", 1).set_param("s_target", 16)
    keys = synth.small_alphabet_u32(20000, 5, 4)
    exact = 0
    for k in (1, 10000, 20000):
        recs = run_and_compare(c, keys, k, False, dev, exact_trace=False)
        last = recs[-1]
        assert last["hi"] == ROUND_EXACT or (last["ok"] and last["nb"] <= 1)
        exact += last["hi"] == ROUND_EXACT
    assert exact > 0


def test_deterministic_repeat(ctx, dev):
    keys = to_dev(synth.zipf_u32(1 << 20, 1.2, 2**16, 8), dev)
    a = ctx.select(keys, 12345)
    b = ctx.select(keys, 12345)
    torch.cuda.synchronize()
    # the set is fixed; the order of out_idx is unspecified by the contract
    assert torch.equal(torch.sort(a["idx"])[0], torch.sort(b["idx"])[0])
    assert torch.equal(a["kth_idx"], b["kth_idx"])
    assert ctx.trace_rounds(a) == ctx.trace_rounds(b)


def test_seed_changes_trace_not_result(dev):
    keys_np = synth.uniform_u32(1 << 20, 12)
    keys = to_dev(keys_np, dev)
    sets = []
    for seed in (1, 2, 3):
        c = tk.Context(0, seed=seed)
        res = c.select(keys, 4321)
        torch.cuda.synchronize()
        sets.append(np.sort(res["idx"].cpu().numpy()))
    assert all(np.array_equal(sets[0], s) for s in sets[1:])


def test_argument_errors(ctx, dev):
    keys = torch.zeros(100, dtype=torch.float32, device=dev)
    with pytest.raises(tk.TopkError):
        ctx.select(keys, 0)
    with pytest.raises(tk.TopkError):
        ctx.select(keys, 101)
    with pytest.raises(tk.TopkError):
        ctx.select(keys, 5, workspace=torch.empty(256, dtype=torch.uint8, device=dev))
    with pytest.raises(tk.TopkError):
        ctx.set_param("s_target", 1 << 20)
