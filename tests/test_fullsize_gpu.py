"""GPU parity at the full workload sizes, in the configuration bench.py times
(default context parameters).

The oracle's replay of the recursion runs in C in seconds even at 2^28 keys,
so the whole output array is compared exactly; the O(n) checker confirms it
against the definition (exactly k distinct positions, all at or below the
k-th key, counts below/equal adding up, ties by ascending position).
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


def replay_params(ctx, n):
    g = ctx.get_param
    t_fin = g("t_fin")
    cap = 0 if n <= t_fin else min(n, n // g("band_div") + 65536)
    return dict(s_target=g("s_target"), c_num=g("c_num"), nseg=1024, seg_cap=16,
                t_fin=t_fin, r_max=g("r_max"), band_cap=cap, seed=g("seed"))


def compare(ctx, keys_np, keys, k, largest):
    res = ctx.select(keys, k, largest=largest)
    torch.cuda.synchronize()
    assert int(res["status"].item()) == 0
    got = res["idx"].cpu().numpy().view(np.uint32)
    kth = int(res["kth_idx"].item())
    kb = int(res["kth_key"].cpu().numpy().view(np.uint32)[0])
    assert oracle.check(keys_np, k, got, kth, kb, largest) == 0
    rc, rout, rkth, rrecs = oracle.replay(keys_np, k, largest, **replay_params(ctx, keys_np.size))
    assert rc == 0
    assert np.array_equal(np.sort(got), np.sort(rout)) and kth == rkth
    assert ctx.trace_rounds(res) == rrecs


@pytest.fixture(scope="module")
def ctx(dev):
    return tk.Context(0, seed=0x5EED)


@pytest.fixture(scope="module")
def f32_2p28(dev):
    keys_np = synth.uniform_f32_grid(1 << 28, 2)
    return keys_np, to_dev(keys_np, dev)


@pytest.mark.parametrize("k", [1 << 10, 1 << 20, 1 << 27])
def test_f32_2p28(ctx, f32_2p28, k):
    keys_np, keys = f32_2p28
    compare(ctx, keys_np, keys, k, False)


def test_f32_2p28_largest(ctx, f32_2p28):
    keys_np, keys = f32_2p28
    compare(ctx, keys_np, keys, 1 << 20, True)


@pytest.fixture(scope="module")
def zipf_2p27(dev):
    keys_np = synth.zipf_u32(1 << 27, 1.2, 1 << 16, 3)
    return keys_np, to_dev(keys_np, dev)


@pytest.mark.parametrize("largest", [False, True])
def test_zipf_2p27(ctx, zipf_2p27, largest):
    keys_np, keys = zipf_2p27
    compare(ctx, keys_np, keys, 1 << 20, largest)


def test_all_equal_except_2p27(ctx, dev):
    keys_np = synth.all_equal_except(1 << 27, 0.01, 1 << 31, 31)
    compare(ctx, keys_np, to_dev(keys_np, dev), 1 << 20, False)


def test_u32_2p20_k1000(ctx, dev):
    keys_np = synth.uniform_u32(1 << 20, 1)
    res = ctx.select(to_dev(keys_np, dev), 1000)
    torch.cuda.synchronize()
    ref = oracle.select_sort(keys_np, 1000)
    got = res["idx"].cpu().numpy().view(np.uint32)
    assert np.array_equal(np.sort(got), np.sort(ref))
    assert int(res["kth_idx"].item()) == int(ref[-1])
