"""GPU parity of the single-instance selection against the CPU oracle.

Every comparison is exact (integer/index work):
  * the selected set, kth position and kth key bits equal the plain oracle's
    (full sort by (value, position));
  * the selected set and every round record (sample size, pivot ranks and
    objects, |a|, |b|, outcome) equal the oracle's step-by-step replay of the
    recursion run with the same parameters and seed;
  * the recorded sample positions equal the oracle's Bernoulli sampler.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

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


def replay_params(ctx, n):
    g = ctx.get_param
    t_fin = g("t_fin")
    cap = 0 if n <= t_fin else min(n, n // g("band_div") + 65536)
    return dict(s_target=g("s_target"), c_num=g("c_num"), nseg=1024, seg_cap=16,
                t_fin=t_fin, r_max=g("r_max"), band_cap=cap, seed=g("seed"))


def check_trace_chain(recs, n, k):
    """Invariants of any valid round trace (§2 Algorithm): every recursion into
    b brackets rank k_cur and shrinks the problem; a repeated round keeps it."""
    n_cur, k_cur = n, k
    for r in recs:
        assert (r["n_cur"], r["k_cur"]) == (n_cur, k_cur)
        if r["ok"]:
            assert r["na"] < r["k_cur"] <= r["na"] + r["nb"] and r["nb"] < r["n_cur"]
            n_cur, k_cur = r["nb"], r["k_cur"] - r["na"]


def run_and_compare(ctx, keys_np, k, largest, dev, offset=0, full_oracle=True, trace=True,
                    exact_trace=True):
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

    rc, rout, rkth, rrecs = oracle.replay(keys_np, k, largest, **replay_params(ctx, n))
    assert rc == 0 and status == 0, (rc, status)
    # the set is exact; the order of the sweeps' output ranges follows their reservations
    assert np.array_equal(np.sort(got), np.sort(rout)), "selected set differs from the replay"
    assert kth_idx == rkth
    assert kth_bits == int(bits[rkth])
    assert np.array_equal(got_keys, bits[got])
    recs = ctx.trace_rounds(res)
    check_trace_chain(recs, n, k)
    if exact_trace:
        assert len(recs) == len(rrecs)
        for g, r in zip(recs, rrecs):
            assert g == r, (g, r)
    else:
        # a repeated round on a middle part samples positions of b, whose
        # physical order follows the sweep's reservations: equal up to there
        for g, r in zip(recs, rrecs):
            assert g == r, (g, r)
            if not g["ok"] and g["n_cur"] < n:
                break
    if trace and rrecs:
        # sample positions of the first attempt equal the oracle's sampler
        r0 = rrecs[0]
        pos = np.array(ctx.trace_sample(res, 0), np.uint32)
        p = replay_params(ctx, n)
        ref = oracle.bernoulli_sample(n, p["s_target"] / n, p["seed"], 0, 1024, 16)
        assert pos.size == r0["s"] and np.array_equal(pos, ref)
    if full_oracle:
        ref = oracle.select_sort(keys_np, k, largest)
        assert np.array_equal(np.sort(got), np.sort(ref))
        assert kth_idx == int(ref[-1])
    else:
        assert oracle.check(keys_np, k, got, kth_idx, kth_bits, largest) == 0
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


def test_band_overflow_and_no_convergence(dev):
    c = tk.Context(0, seed=3).set_param("band_div", 64).set_param("s_target", 64)
    c.set_param("c_num", 4096).set_param("r_max", 3).set_param("t_fin", 1024)
    keys = synth.uniform_u32(1 << 20, 10)
    res = c.select(to_dev(keys, dev), 1 << 19, trace=False)
    torch.cuda.synchronize()
    assert int(res["status"].item()) == tk.STATUS_NO_CONVERGENCE
    rc, _, _, rrecs = oracle.replay(keys, 1 << 19, False, **replay_params(c, keys.size))
    assert rc == 1
    recs = c.trace_rounds(res)
    assert recs == rrecs


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


def test_tiny_t_fin_cannot_converge_on_both_sides(dev):
    # a subproblem of 2 elements cannot shrink below t_fin = 1 (every round's
    # b keeps both): device and oracle both spend the budget and say so
    c = tk.Context(0, seed=5).set_param("t_fin", 1).set_param("s_target", 16)
    keys = synth.small_alphabet_u32(20000, 5, 4)
    res = c.select(to_dev(keys, dev), 10000)
    torch.cuda.synchronize()
    rc, _, _, rrecs = oracle.replay(keys, 10000, False, **replay_params(c, keys.size))
    assert rc == 1 and int(res["status"].item()) == tk.STATUS_NO_CONVERGENCE
    recs = c.trace_rounds(res)
    assert len(recs) == len(rrecs[:32])
    check_trace_chain(recs, keys.size, 10000)


def test_deterministic_repeat(ctx, dev):
    keys = to_dev(synth.zipf_u32(1 << 20, 1.2, 2**16, 8), dev)
    a = ctx.select(keys, 12345)
    b = ctx.select(keys, 12345)
    torch.cuda.synchronize()
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
