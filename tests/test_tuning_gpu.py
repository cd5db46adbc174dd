"""GPU tests of the batched autotuner and of tuning files.

The tuner may only change parameters, never results: after tuning, every row
must still equal the oracle's.  Tuning files round-trip every parameter and
are applied all or nothing.
"""
import numpy as np
import pytest

import oracle
import synth
from test_batched_gpu import check_rows, ragged, to_dev

pytestmark = pytest.mark.gpu

tk = pytest.importorskip("paper_1502_03942_amd")

S_CAND = {256, 512, 1024, 2048}
C_CAND = {8, 12, 16, 24}


def test_tune_batched_keeps_results_exact(dev):
    rng = np.random.default_rng(50)
    lens = [9000, 12000, 20000, 30000, 40000, 70000, 5000, 100, 3]
    ks = [int(rng.integers(1, min(L, 2048) + 1)) for L in lens]
    keys, off, kk = ragged(lens, ks, lambda n: synth.normal_f32(n, 51))
    ctx = tk.Context(0, seed=13)
    args = to_dev(keys, off, kk, dev)
    res = ctx.tune_batched(*args, reps=1)
    check_rows(keys, off, kk, res, False)
    present = {int(L).bit_length() for L in lens if L > 8192}
    for c in range(34):
        s, cn = ctx.get_param(f"bt_s_target@{c}"), ctx.get_param(f"bt_c_num@{c}")
        t = ctx.get_param(f"bt_tile@{c}")
        if c in present:
            assert s in S_CAND and cn in C_CAND and t in (8, 16), (c, s, cn, t)
        else:
            assert s == -1 and cn == -1 and t == -1, c
    assert ctx.get_param("bt_wg_per_cu") in (2, 3, 4)
    assert ctx.get_param("bt_attempts") in (1, 2, 4, 8)
    res = ctx.select_batched(*args)
    check_rows(keys, off, kk, res, False)
    res = ctx.select_batched(*args, largest=True)
    check_rows(keys, off, kk, res, True)


NAMES = ["s_target", "c_num", "t_fin", "r_max", "r_fast", "band_div", "tail_max",
         "bt_s_target", "bt_c_num", "bt_wg_per_cu", "bt_attempts", "bt_fast", "bt_tile", "fq_mode"]


def params(ctx):
    d = {n: ctx.get_param(n) for n in NAMES}
    for c in range(34):
        d[f"bt_s_target@{c}"] = ctx.get_param(f"bt_s_target@{c}")
        d[f"bt_c_num@{c}"] = ctx.get_param(f"bt_c_num@{c}")
        d[f"bt_tile@{c}"] = ctx.get_param(f"bt_tile@{c}")
    return d


def test_tuning_file_roundtrip(dev, tmp_path):
    a = tk.Context(0)
    defaults = params(a)
    a.set_param("s_target", 2048).set_param("c_num", 12).set_param("bt_s_target@15", 512)
    a.set_param("bt_c_num@17", 16).set_param("bt_wg_per_cu", 3).set_param("bt_tile@18", 8)
    a.set_param("bt_tile", 8)
    path = tmp_path / "t.json"
    a.save_tuning(path)
    b = tk.Context(0).load_tuning(path)
    assert params(b) == params(a)
    b.load_tuning(None)
    assert params(b) == defaults
    # all or nothing: a bad name or value leaves every parameter as it was
    for bad in ('{"s_target": 2048, "no_such": 1}', '{"c_num": 8, "t_fin": 0}',
                '{"c_num": 8,}', '{"c_num": x}', '[1]'):
        p = tmp_path / "bad.json"
        p.write_text(bad)
        before = params(a)
        with pytest.raises(tk.TopkError):
            a.load_tuning(p)
        assert params(a) == before, bad
    with pytest.raises(tk.TopkError):
        a.load_tuning(tmp_path / "missing.json")
    with pytest.raises(tk.TopkError):
        a.set_param("bt_s_target@34", 512)
    with pytest.raises(tk.TopkError):
        a.set_param("bt_c_num@3", 2)
    for bad_tile in (("bt_tile", 12), ("bt_tile@20", 12), ("bt_tile", 32)):
        with pytest.raises(tk.TopkError):
            a.set_param(*bad_tile)


def test_tune_single_keeps_results_exact(dev):
    import torch
    n = 1 << 22
    keys_np = synth.normal_f32(n, 52)
    keys = torch.from_numpy(keys_np).to(dev)
    for k, largest in ((1000, False), (1 << 20, True)):
        ctx = tk.Context(0, seed=17)
        res = ctx.tune(keys, k, largest=largest, reps=1)
        assert ctx.get_param("s_target") in (2048, 4096, 8192)
        assert ctx.get_param("c_num") in (8, 12, 16, 24)
        torch.cuda.synchronize()
        assert int(res["status"].item()) == 0
        got = res["idx"].cpu().numpy().view(np.uint32)
        kb = int(res["kth_key"].cpu().numpy().view(np.uint32)[0])
        assert oracle.check(keys_np, k, got, int(res["kth_idx"].item()), kb, largest) == 0
