"""The batched entry point that allocates nothing (static scratch) against the
workspace entry point, through the C-ABI: identical outputs on two calls in a
row, the second with a smaller batch; both checked against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tk = pytest.importorskip("paper_1502_03942_amd")


def batch(rows, seed):
    keys, off, kk = synth.lognormal_rows(rows, 2048, 1.0, 1, 1 << 18, 2048, seed)
    return keys, off, kk


def outputs(R, total, dev):
    return {"idx": torch.full((max(total, 1),), -1, dtype=torch.int32, device=dev),
            "kth_key": torch.zeros(R, dtype=torch.float32, device=dev),
            "kth_idx": torch.zeros(R, dtype=torch.int32, device=dev),
            "status": torch.full((1,), 7, dtype=torch.int32, device=dev)}


@pytest.mark.parametrize("largest", [False, True])
def test_noalloc_matches_workspace_entry_point(dev, largest):
    ctx = tk.Context(0, seed=23)
    for rows, seed in ((3000, 71), (700, 72)):           # the second call is smaller
        print("noalloc: rows=%d seed=%d largest=%d" % (rows, seed, largest), flush=True)
        keys, off, kk = batch(rows, seed)
        kd = torch.from_numpy(keys).to(dev)
        od = torch.from_numpy(off.astype(np.int64)).to(dev)
        kkd = torch.from_numpy(kk.astype(np.int32)).to(dev)
        oo = torch.zeros(rows + 1, dtype=torch.int64, device=dev)
        oo[1:] = torch.cumsum(kkd.to(torch.int64), 0)
        total = int(oo[-1].item())
        ref = ctx.select_batched(kd, od, kkd, out_off=oo, largest=largest)
        got = ctx.select_batched_noalloc(kd, od, kkd, oo, outputs(rows, total, dev), largest=largest)
        torch.cuda.synchronize()
        assert int(got["status"].item()) == 0 and int(ref["status"].item()) == 0
        for name in ("idx", "kth_key", "kth_idx"):
            a = ref[name][:total] if name == "idx" else ref[name]
            b = got[name][:total] if name == "idx" else got[name]
            assert torch.equal(a.view(torch.int32), b.view(torch.int32)), name
        idx = got["idx"].cpu().numpy().view(np.uint32)
        kth = got["kth_idx"].cpu().numpy().view(np.uint32)
        kkey = got["kth_key"].cpu().numpy().view(np.uint32)
        ooh = oo.cpu().numpy()
        for r in range(0, rows, 7):
            row = keys[int(off[r]):int(off[r + 1])]
            k = int(kk[r])
            sel = idx[int(ooh[r]):int(ooh[r]) + k]
            assert oracle.check(row, k, sel, int(kth[r]), int(kkey[r]), largest) == 0, r


def test_noalloc_rejects_what_it_cannot_do(dev):
    ctx = tk.Context(0)
    R = (1 << 20) + 1                      # one row more than the scratch holds
    off = torch.arange(R + 1, dtype=torch.int64, device=dev)
    k = torch.ones(R, dtype=torch.int32, device=dev)
    keys = torch.zeros(R, dtype=torch.float32, device=dev)
    out = outputs(R, R, dev)
    with pytest.raises(tk.TopkError, match="workspace too small"):
        ctx.select_batched_noalloc(keys, off, k, off, out)
    # TOPK_GRAPH (a graph would have to be instantiated) and unknown flags
    for flags in (tk.TOPK_GRAPH, 1 << 30):
        rc = tk.lib().topk_select_batched_f32_noalloc(
            ctx._h, tk._ptr(keys), tk._ptr(off), 10, tk._ptr(k), tk._ptr(off), flags,
            tk._ptr(out["idx"]), tk._ptr(out["kth_key"]), tk._ptr(out["kth_idx"]),
            tk._ptr(out["status"]), tk._stream(dev))
        assert rc == -1
