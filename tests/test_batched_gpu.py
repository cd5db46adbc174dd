"""GPU parity of the batched selection (many rows, each with its own k).

Every row's selected set, k-th column and k-th key bits must equal the plain
oracle's (full sort by (value, column)); the full-size batch is checked row
by row with the oracle's O(n) checker and sampled rows against the sort.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tk = pytest.importorskip("paper_1502_03942_amd")


def to_dev(keys, off, kk, dev):
    return (torch.from_numpy(keys).to(dev), torch.from_numpy(off.astype(np.int64)).to(dev),
            torch.from_numpy(kk.astype(np.int32)).to(dev))


def fetch(res):
    torch.cuda.synchronize()
    return (res["idx"].cpu().numpy().view(np.uint32), res["kth_idx"].cpu().numpy().view(np.uint32),
            res["kth_key"].cpu().numpy().view(np.uint32), int(res["status"].item()),
            res["out_off"].cpu().numpy())


def check_rows(keys, off, kk, res, largest, rows=None, full=True):
    idx, kth, kkey, status, oo = fetch(res)
    assert status == 0
    R = len(kk)
    for r in (range(R) if rows is None else rows):
        row = keys[int(off[r]):int(off[r + 1])]
        k = int(kk[r])
        sel = idx[int(oo[r]):int(oo[r]) + k]
        assert oracle.check(row, k, sel, int(kth[r]), int(kkey[r]), largest) == 0, r
        if full:
            ref = oracle.select_sort(row, k, largest=largest)
            assert np.array_equal(np.sort(sel), np.sort(ref)), r
            assert int(kth[r]) == int(ref[-1]), r


def ragged(lens, ks, gen):
    off = np.zeros(len(lens) + 1, np.uint64)
    off[1:] = np.cumsum(lens)
    keys = gen(int(off[-1]))
    return keys, off, np.array(ks, np.uint32)


# lengths around every boundary: the wave mode's register blocks (1024,
# 2048 keys) and its limit (3072: longer rows of that class go to a
# workgroup), the workgroup's register rows (4096, 8192), the sampled rows
MIXED_LENS = [1, 2, 63, 64, 1000, 1024, 1025, 2047, 2048, 2049, 3071, 3072, 3073, 4095, 4096,
              4097, 5000, 8192, 20000, 65537, 150000, 300001]


def mixed_ks(lens, rng):
    out = []
    for L in lens:
        out.append([1, L, min(L, 2048), int(rng.integers(1, L + 1))][int(rng.integers(0, 4))])
    return out


@pytest.mark.parametrize("largest", [False, True])
@pytest.mark.parametrize("dist", ["normal", "specials", "alphabet"])
def test_batched_mixed(dev, largest, dist):
    rng = np.random.default_rng(21)
    lens = MIXED_LENS * 2
    ks = mixed_ks(lens, rng)
    gens = {
        "normal": lambda n: synth.normal_f32(n, 22),
        "specials": lambda n: synth.specials_f32(n, 23),
        "alphabet": lambda n: np.random.default_rng(24).integers(0, 5, n).astype(np.float32),
    }
    keys, off, kk = ragged(lens, ks, gens[dist])
    ctx = tk.Context(0, seed=7)
    res = ctx.select_batched(*to_dev(keys, off, kk, dev), largest=largest)
    check_rows(keys, off, kk, res, largest)


def edge_rows(n, seed):
    """Rows without NaN whose key ranges stress bins linear in the key value:
    extremes whose difference overflows, infinite or denormal extremes, two
    values, ties inside a bin, sorted and narrow ranges, mixed zeros."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(n).astype(np.float32)
    rows = []
    r = g.copy(); r[rng.integers(0, n)] = 3.4028235e38; r[rng.integers(0, n)] = -3.4028235e38
    rows.append(r)                                            # span overflows to inf
    r = np.abs(g); r[rng.integers(0, n)] = 3.4028235e38
    rows.append(r)                                            # finite span, one huge bin
    r = g.copy(); r[rng.integers(0, n)] = np.inf; r[rng.integers(0, n)] = -np.inf
    rows.append(r)                                            # infinite extremes
    rows.append((rng.integers(1, 900, n).astype(np.uint32)).view(np.float32))   # denormals only
    rows.append(np.where(rng.random(n) < 0.3, 0.0, 1.0).astype(np.float32))   # two values
    rows.append(np.round(g * 1000.0).astype(np.float32) / np.float32(1000.0))  # ties in bins
    rows.append(np.sort(g))                                   # sorted
    rows.append((1.0 + np.arange(n, dtype=np.float32)[::-1] * np.float32(1e-7)).astype(np.float32))
    r = g.copy(); r[rng.random(n) < 0.2] = 0.0; r[rng.random(n) < 0.2] = -0.0
    rows.append(r)                                            # +0 and -0 among the keys
    rows.append(np.exp(rng.standard_normal(n) * 8.0).astype(np.float32))       # heavy tail
    return rows


@pytest.mark.parametrize("largest", [False, True])
@pytest.mark.parametrize("n", [700, 3000, 3073, 5000, 8192])
def test_batched_value_range_edges(dev, n, largest):
    # rows of the wave mode (under 3072 keys) and of the workgroup's register
    # rows (up to 8192): every row without NaN, so each reaches the value
    # binning and, where its range allows none or a bin is too full, the
    # radix select behind it
    rows = edge_rows(n, 40 + n)
    rng = np.random.default_rng(41)
    ks = [int(x) for x in rng.integers(1, n + 1, len(rows))]
    ks[0], ks[1] = 1, n
    off = np.zeros(len(rows) + 1, np.uint64)
    off[1:] = np.cumsum([len(r) for r in rows])
    keys = np.concatenate(rows).astype(np.float32)
    kk = np.array(ks, np.uint32)
    res = tk.Context(0, seed=5).select_batched(*to_dev(keys, off, kk, dev), largest=largest)
    check_rows(keys, off, kk, res, largest)


def test_batched_every_k_small_rows(dev):
    lens = [37] * 37
    ks = list(range(1, 38))
    keys, off, kk = ragged(lens, ks, lambda n: synth.normal_f32(n, 25))
    ctx = tk.Context(0)
    res = ctx.select_batched(*to_dev(keys, off, kk, dev))
    check_rows(keys, off, kk, res, False)


def test_batched_exact_fallback(dev):
    # one sampling attempt with a tiny spread: most long rows miss and the
    # exact radix fallback over the row produces the result
    rng = np.random.default_rng(26)
    lens = [20000, 70000, 300000, 5000, 100000]
    ks = [int(rng.integers(1, min(L, 2048) + 1)) for L in lens]
    keys, off, kk = ragged(lens, ks, lambda n: synth.normal_f32(n, 27))
    ctx = tk.Context(0, seed=3)
    ctx.set_param("bt_attempts", 1).set_param("bt_c_num", 4).set_param("bt_s_target", 64)
    res = ctx.select_batched(*to_dev(keys, off, kk, dev))
    check_rows(keys, off, kk, res, False)


def test_batched_graph_replay(dev):
    rng = np.random.default_rng(28)
    lens = MIXED_LENS
    ks = mixed_ks(lens, rng)
    keys, off, kk = ragged(lens, ks, lambda n: synth.normal_f32(n, 29))
    kd, od, kd2 = to_dev(keys, off, kk, dev)
    ctx = tk.Context(0, seed=5)
    eager = ctx.select_batched(kd, od, kd2)
    e = fetch(eager)
    out = None
    for rep in range(3):
        out = ctx.select_batched(kd, od, kd2, graph=True, out=out)
        g = fetch(out)
        assert all(np.array_equal(a, b) for a, b in zip(e[:3], g[:3])) and g[3] == 0, rep
        torch.randn(1 << 20, device=dev).sum()      # unrelated eager work between replays
    # the graph reads the keys each replay: change them in place
    keys2 = synth.normal_f32(keys.size, 30)
    kd.copy_(torch.from_numpy(keys2).to(dev))
    out = ctx.select_batched(kd, od, kd2, graph=True, out=out)
    check_rows(keys2, off, kk, out, False)


def test_batched_graph_cache_eviction(dev):
    # more distinct argument sets (here: seeds) than the context keeps graphs
    # for: older graphs are dropped, every replay stays exact
    lens = [20000, 3000, 700, 9000]
    ks = [100, 3000, 1, 2048]
    keys, off, kk = ragged(lens, ks, lambda n: synth.normal_f32(n, 31))
    args = to_dev(keys, off, kk, dev)
    ctx = tk.Context(0, seed=1)
    for i in range(40):
        ctx.set_param("seed", 1000 + i)
        out = ctx.select_batched(*args, graph=True)
        if i % 13 == 0:
            check_rows(keys, off, kk, out, False)
    ctx.set_param("seed", 1000)
    check_rows(keys, off, kk, ctx.select_batched(*args, graph=True), False)


def test_batched_bad_rows(dev):
    lens = [100, 100, 100, 0]
    ks = [10, 0, 101, 0]
    keys, off, kk = ragged(lens, ks, lambda n: synth.normal_f32(n, 31))
    ctx = tk.Context(0)
    res = ctx.select_batched(*to_dev(keys, off, kk, dev))
    idx, kth, kkey, status, oo = fetch(res)
    assert status == tk.STATUS_BAD_ROW
    ref = oracle.select_sort(keys[:100], 10)
    assert np.array_equal(np.sort(idx[:10]), np.sort(ref)) and int(kth[0]) == int(ref[-1])


def test_batched_fullsize(dev):
    keys, off, kk = synth.lognormal_rows(65536, 4096, 1.0, 64, 1 << 20, 2048, 4)
    ctx = tk.Context(0)
    res = ctx.select_batched(*to_dev(keys, off, kk, dev), graph=True)
    lens = np.diff(off.astype(np.int64))
    longest = np.argsort(-lens)[:8].tolist()
    sample = sorted(set(longest + list(range(0, 65536, 997))))
    check_rows(keys, off, kk, res, False, rows=sample, full=True)
    check_rows(keys, off, kk, res, False, full=False)


@pytest.mark.parametrize("fast,tile", [(0, 16), (1, 16), (1, 8)])
@pytest.mark.parametrize("largest", [False, True])
def test_batched_fast_and_general_agree(dev, fast, tile, largest):
    # the same rows through the fast sweep (both tiles) and through the
    # general sweep; lengths with ragged last tiles of either size
    lens = [4097, 6000, 13000, 33000, 100000, 262144, 9000, 20000, 10241, 8193 + 2048]
    ks = [1, 2048, 700, 2048, 1, 1500, 9000, 20000, 333, 2048]
    keys, off, kk = ragged(lens, ks, lambda n: synth.specials_f32(n, 41))
    ctx = tk.Context(0, seed=9).set_param("bt_fast", fast).set_param("bt_tile", tile)
    res = ctx.select_batched(*to_dev(keys, off, kk, dev), largest=largest)
    check_rows(keys, off, kk, res, largest)


@pytest.mark.parametrize("largest", [False, True])
def test_batched_structured_long_rows(dev, largest):
    # sorted and reverse-sorted rows put every candidate in a few columns;
    # constant and two-valued rows tie at the pivots: region overflows and
    # band overflows fall back to the general sweep or the exact select
    n = 30000
    up = np.arange(n, dtype=np.float32)
    rows = [up, up[::-1].copy(), np.full(n, 3.0, np.float32),
            np.where(np.arange(n) % 7 == 0, 1.0, 2.0).astype(np.float32),
            np.concatenate([np.full(n // 2, -1.0, np.float32), up[: n - n // 2]])]
    ks = [2048, 1000, 1500, 2048, 700]
    off = np.zeros(len(rows) + 1, np.uint64)
    off[1:] = np.cumsum([len(r) for r in rows])
    keys = np.concatenate(rows)
    kk = np.array(ks, np.uint32)
    ctx = tk.Context(0, seed=11)
    res = ctx.select_batched(*to_dev(keys, off, kk, dev), largest=largest)
    check_rows(keys, off, kk, res, largest)


def test_batched_fullsize_tuned_as_benched(dev):
    # the configuration bench.py times: the autotuner's choice on this batch
    keys, off, kk = synth.lognormal_rows(65536, 4096, 1.0, 64, 1 << 20, 2048, 4)
    ctx = tk.Context(0, seed=0x5EED)
    args = to_dev(keys, off, kk, dev)
    ctx.tune_batched(*args, reps=3)
    tuned = {c: (ctx.get_param("bt_s_target@%d" % c), ctx.get_param("bt_c_num@%d" % c),
                 ctx.get_param("bt_tile@%d" % c))
             for c in range(34) if ctx.get_param("bt_s_target@%d" % c) >= 0}
    print("tuned:", tuned, "wg/cu", ctx.get_param("bt_wg_per_cu"),
          "attempts", ctx.get_param("bt_attempts"), flush=True)
    res = ctx.select_batched(*args, graph=True)
    res = ctx.select_batched(*args, graph=True, out=res)
    lens = np.diff(off.astype(np.int64))
    longest = np.argsort(-lens)[:8].tolist()
    sample = sorted(set(longest + list(range(0, 65536, 997))))
    check_rows(keys, off, kk, res, False, rows=sample, full=True)
    check_rows(keys, off, kk, res, False, full=False)


@pytest.mark.parametrize("largest", [False, True])
def test_batched_general_sweep_retries(dev, largest):
    # general sweep only, a narrow spread and two attempts: long rows miss,
    # retry (rewriting the part below L in out[]) and fall back to the exact
    # select, which rewrites it again
    rng = np.random.default_rng(60)
    lens = [9000, 16385, 40000, 100000, 250000, 70000, 12000, 33333]
    ks = [int(rng.integers(1, min(L, 2048) + 1)) for L in lens]
    keys, off, kk = ragged(lens * 3, ks * 3, lambda n: synth.normal_f32(n, 61))
    ctx = tk.Context(0, seed=19)
    ctx.set_param("bt_fast", 0).set_param("bt_c_num", 4).set_param("bt_attempts", 2)
    ctx.set_param("bt_s_target", 256)
    res = ctx.select_batched(*to_dev(keys, off, kk, dev), largest=largest)
    check_rows(keys, off, kk, res, largest)
