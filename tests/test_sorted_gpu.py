"""GPU parity of the canonical output order (TOPK_SORTED).

With the flag, out_idx must equal the oracle's first k positions in the
unique order by (key, position) element by element (the oracle sorts all n
positions), the keys output must follow it, and the pair of rank k must be
the last element.  At n = 2^28 the oracle's full sort is too slow; there the
order is checked by properties computed with torch: the sorted call returns
the same set as the unsorted one, and consecutive keys never decrease, with
equal keys in ascending position.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tk = pytest.importorskip("paper_1502_03942_amd")


def to_dev(a, dev):
    return torch.from_numpy(a.view(np.int32) if a.dtype == np.uint32 else a).to(dev)


def check_sorted(ctx, keys_np, k, largest, dev):
    print("sorted: n=%d k=%d largest=%d dtype=%s" % (keys_np.size, k, largest, keys_np.dtype), flush=True)
    res = ctx.select(to_dev(keys_np, dev), k, largest=largest, write_keys=True, sorted=True)
    torch.cuda.synchronize()
    assert int(res["status"].item()) == 0
    got = res["idx"].cpu().numpy().view(np.uint32)
    ref = oracle.select_sort(keys_np, k, largest)
    assert np.array_equal(got, ref)
    kb = res["keys"].cpu().numpy().view(np.uint32)
    assert np.array_equal(kb, keys_np.view(np.uint32)[ref])
    assert int(res["kth_idx"].item()) & 0xFFFFFFFF == int(ref[-1])


@pytest.mark.parametrize("largest", [False, True])
@pytest.mark.parametrize("k", [1, 2, 1000, 4096, 4097, 1 << 17, (1 << 20) - 3, 1 << 20])
def test_sorted_u32(dev, k, largest):
    keys_np = synth.uniform_u32(1 << 20, 61)
    check_sorted(tk.Context(0, seed=3), keys_np, k, largest, dev)


@pytest.mark.parametrize("largest", [False, True])
@pytest.mark.parametrize("k", [1, 777, 65536, 150000, 300001])
def test_sorted_f32_specials(dev, k, largest):
    # NaN (every payload), -0.0 and +0.0, infinities, denormals, ties
    keys_np = synth.specials_f32(300001, 62)
    check_sorted(tk.Context(0, seed=4), keys_np, k, largest, dev)


@pytest.mark.parametrize("largest", [False, True])
def test_sorted_many_ties(dev, largest):
    # five key values over 2^18 positions: the order is decided by positions
    keys_np = synth.small_alphabet_u32(1 << 18, 5, 63)
    for k in (1, 5000, 100000, 1 << 18):
        check_sorted(tk.Context(0, seed=5), keys_np, k, largest, dev)


def test_sorted_f32_2p24(dev):
    keys_np = synth.uniform_f32_grid(1 << 24, 64)
    check_sorted(tk.Context(0, seed=6), keys_np, 1 << 20, False, dev)


def test_sorted_fullsize_properties(dev):
    # n = 2^28 f32 on the 2^-24 grid (about 16 keys share each value), k = 2^27
    n, k = 1 << 28, 1 << 27
    print("sorted full size: n=%d k=%d" % (n, k), flush=True)
    keys = to_dev(synth.uniform_f32_grid(n, 2), dev)
    ctx = tk.Context(0, seed=0x5EED)
    plain = ctx.select(keys, k)
    srt = ctx.select(keys, k, sorted=True)
    torch.cuda.synchronize()
    assert int(plain["status"].item()) == 0 and int(srt["status"].item()) == 0
    a = plain["idx"].to(torch.int64) & 0xFFFFFFFF
    b = srt["idx"].to(torch.int64) & 0xFFFFFFFF
    assert torch.equal(torch.sort(a).values, torch.sort(b).values)    # the same set
    v = keys[b]
    assert bool((v[1:] >= v[:-1]).all().item())                       # keys ascending
    tie = v[1:] == v[:-1]
    assert bool((b[1:][tie] > b[:-1][tie]).all().item())              # ties by position
    assert int(srt["kth_idx"].to(torch.int64).item()) & 0xFFFFFFFF == int(b[-1].item())
    del keys, plain, srt, a, b, v, tie
    torch.cuda.empty_cache()
