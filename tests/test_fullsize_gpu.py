"""GPU parity at the full workload sizes.

Each selection runs twice: with the default context parameters, and with the
parameters the single-instance autotuner picks for it (the configuration
bench.py times).  Every result is compared with the oracle: the O(n) checker
confirms it against the definition (exactly k distinct positions, all at or
below the k-th key, counts below/equal adding up, ties by ascending
position), and every round is checked definitionally (oracle ranks of the
pivots give |a| and |b|).  The test-side model of the round policy must
reproduce the default-parameter trace.
"""
import numpy as np
import pytest
import torch

import model
import oracle
import synth
from roundcheck import check_rounds

pytestmark = pytest.mark.gpu

tk = pytest.importorskip("paper_1502_03942_amd")


def to_dev(a, dev):
    return torch.from_numpy(a.view(np.int32) if a.dtype == np.uint32 else a).to(dev)


def model_params(ctx, n):
    g = ctx.get_param
    t_fin = g("t_fin")
    cap = 0 if n <= t_fin else min(n, n // g("band_div") + 65536)
    return dict(s_target=g("s_target"), c_num=g("c_num"), nseg=1024, seg_cap=16,
                t_fin=t_fin, r_max=g("r_max"), band_cap=cap, seed=g("seed"))


def compare(ctx, keys_np, keys, k, largest, with_model=True):
    print("fullsize: n=%d k=%d largest=%d s_target=%d c_num=%d" % (
        keys_np.size, k, largest, ctx.get_param("s_target"), ctx.get_param("c_num")), flush=True)
    res = ctx.select(keys, k, largest=largest)
    torch.cuda.synchronize()
    assert int(res["status"].item()) == 0
    got = res["idx"].cpu().numpy().view(np.uint32)
    kth = int(res["kth_idx"].item())
    kb = int(res["kth_key"].cpu().numpy().view(np.uint32)[0])
    assert oracle.check(keys_np, k, got, kth, kb, largest) == 0
    recs = ctx.trace_rounds(res)
    p = model_params(ctx, keys_np.size)
    check_rounds(keys_np, k, largest, recs, p["band_cap"])
    if with_model:
        rc, _, mkth, mrecs = model.replay(keys_np, k, largest, **p)
        assert rc == 0 and mkth == kth and recs == mrecs


@pytest.fixture(scope="module")
def f32_2p28(dev):
    keys_np = synth.uniform_f32_grid(1 << 28, 2)
    return keys_np, to_dev(keys_np, dev)


@pytest.mark.parametrize("k", [1 << 10, 1 << 20, 1 << 27])
def test_f32_2p28(f32_2p28, k):
    keys_np, keys = f32_2p28
    compare(tk.Context(0, seed=0x5EED), keys_np, keys, k, False)


@pytest.mark.parametrize("k", [1 << 10, 1 << 20, 1 << 27])
def test_f32_2p28_tuned_as_benched(f32_2p28, k):
    # the bench's configuration: one context per k, autotuned on this selection
    keys_np, keys = f32_2p28
    ctx = tk.Context(0, seed=0x5EED)
    ctx.tune(keys, k, reps=3)
    compare(ctx, keys_np, keys, k, False, with_model=False)


def test_f32_2p28_largest(f32_2p28):
    keys_np, keys = f32_2p28
    compare(tk.Context(0, seed=0x5EED), keys_np, keys, 1 << 20, True)


@pytest.fixture(scope="module")
def zipf_2p27(dev):
    keys_np = synth.zipf_u32(1 << 27, 1.2, 1 << 16, 3)
    return keys_np, to_dev(keys_np, dev)


@pytest.mark.parametrize("largest", [False, True])
def test_zipf_2p27(zipf_2p27, largest):
    keys_np, keys = zipf_2p27
    compare(tk.Context(0, seed=0x5EED), keys_np, keys, 1 << 20, largest)


def test_all_equal_except_2p27(dev):
    keys_np = synth.all_equal_except(1 << 27, 0.01, 1 << 31, 31)
    compare(tk.Context(0, seed=0x5EED), keys_np, to_dev(keys_np, dev), 1 << 20, False)


def test_u32_2p20_k1000(dev):
    keys_np = synth.uniform_u32(1 << 20, 1)
    res = tk.Context(0, seed=0x5EED).select(to_dev(keys_np, dev), 1000)
    torch.cuda.synchronize()
    ref = oracle.select_sort(keys_np, 1000)
    got = res["idx"].cpu().numpy().view(np.uint32)
    assert np.array_equal(np.sort(got), np.sort(ref))
    assert int(res["kth_idx"].item()) == int(ref[-1])


@pytest.mark.parametrize("k", [1000, (1 << 31) + 5])
def test_positions_past_2p31(dev, k):
    # n above 2^31: positions use all 32 bits.  Too large for the oracle's
    # sort, so the result is checked by properties that hold at any size,
    # computed with torch on the device (independently of the library): k
    # distinct positions in range, every selected key at or below the k-th,
    # fewer than k keys below it and at least k at or below it, the selected
    # keys equal to it the lowest positions among the equal ones, and the
    # k-th key and position consistent.
    n = (1 << 31) + 4097
    print("positions past 2^31: n=%d k=%d" % (n, k), flush=True)
    g = torch.Generator(device=dev)
    g.manual_seed(123)
    keys = torch.rand(n, generator=g, device=dev)
    ctx = tk.Context(0, seed=7)
    res = ctx.select(keys, k)
    torch.cuda.synchronize()
    assert int(res["status"].item()) == 0
    idx = res["idx"].to(torch.int64) & 0xFFFFFFFF
    kth = res["kth_key"]
    kth_idx = int(res["kth_idx"].to(torch.int64).item()) & 0xFFFFFFFF
    assert idx.numel() == k and int(idx.max().item()) < n
    mark = torch.zeros(n, dtype=torch.bool, device=dev)
    mark[idx] = True
    assert int(mark.sum().item()) == k                    # distinct
    sel = keys[idx]
    assert bool((sel <= kth).all().item())
    below = int((keys < kth).sum().item())
    # positions of the keys equal to the k-th, ascending (nonzero in chunks:
    # one call over more than 2^31 elements is not supported)
    chunk = 1 << 30
    eq = torch.cat([torch.nonzero(keys[c0:c0 + chunk] == kth).flatten() + c0
                    for c0 in range(0, n, chunk)])
    assert below < k <= below + eq.numel()
    need = k - below
    sel_eq = torch.sort(torch.cat([idx[c0:c0 + chunk][sel[c0:c0 + chunk] == kth]
                                   for c0 in range(0, k, chunk)])).values
    assert torch.equal(sel_eq, eq[:need])                 # ties by ascending position
    assert float(keys[kth_idx].item()) == float(kth.item()) and kth_idx == int(eq[need - 1].item())
    del keys, mark, sel, idx, res
    torch.cuda.empty_cache()
