"""GPU test of the stream-read measurement helper: it must read every key
once (its sink is the sum of the key bits modulo 2^32), and reject lengths
that are not whole wave-tiles."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

tk = pytest.importorskip("paper_1502_03942_amd")


def test_stream_read_sums_every_key(dev):
    n = 4096 * 1000 + 4096 * 7
    keys_np = synth.uniform_u32(n, 60)
    keys = torch.from_numpy(keys_np.view(np.int32)).to(dev)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    ctx = tk.Context(0)
    ctx.stream_read(keys, sink)
    ctx.stream_read(keys, sink)
    torch.cuda.synchronize()
    want = (2 * int(keys_np.astype(np.uint64).sum())) % (1 << 32)
    assert int(sink.cpu().numpy().view(np.uint32)[0]) == want
    with pytest.raises(tk.TopkError):
        ctx.stream_read(keys[:4095], sink)
