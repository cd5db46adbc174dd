"""GPU parity of the top-k most frequent objects (§7: PAC, EC) and the top-k
sum aggregation (§8) against the CPU oracle (oracle/freq.py).

Everything here is integer work, so every comparison is exact: the whole
table of sample counts (or sums and weighted samples), the sample size, and
the returned objects with their counts in order (count descending, object
ascending).  Both sides draw the sample with the same counter-based rule
(Philox4x32-10 per element, each side its own implementation).
"""
import numpy as np
import pytest
import torch

import oracle
import synth

F = oracle.freq
tk = pytest.importorskip("paper_1502_03942_amd")

DISTS = {
    "zipf1_2p20": (lambda n, s: synth.zipf_u32(n, 1.0, 1 << 20, s), 1 << 20),
    "negbin": (lambda n, s: synth.negbin_u32(n, 1000, 0.05, 1 << 15, s), 1 << 15),
    "alpha17": (lambda n, s: synth.small_alphabet_u32(n, 17, s), 17),
    "uniform": (lambda n, s: synth.uniform_u32(n, s) % np.uint32(1 << 16), 1 << 16),
}


def dev_u32(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(dev)


def run_freq(ctx, keys, U, k, kstar, T, dev):
    print("frequent: n=%d U=%d k=%d kstar=%d T=%d" % (keys.size, U, k, kstar, T), flush=True)
    out = ctx.frequent(dev_u32(keys, dev), U, k, kstar=kstar, T=T, tables=True)
    torch.cuda.synchronize()
    assert int(out["status"].item()) == 0
    seed = ctx.get_param("seed")
    sc, ns = F.sample_counts(keys, U, T, seed, 0)
    assert int(out["n_sampled"].item()) == ns
    assert np.array_equal(out["sample_counts"].cpu().numpy().view(np.uint32), sc)
    if kstar == 0:
        ids, cnt = F.pac_from_counts(sc, k)
    else:
        ids, cnt = F.ec_from_counts(sc, F.exact_counts(keys, U), k, kstar)
    assert np.array_equal(out["ids"].cpu().numpy().view(np.uint32), ids)
    assert np.array_equal(out["counts"].cpu().numpy().view(np.uint32), cnt.astype(np.uint32))


@pytest.mark.gpu
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("dist", sorted(DISTS))
@pytest.mark.parametrize("method", ["pac", "ec"])
def test_frequent_parity(dev, dist, method, mode):
    # mode 0: by universe size (direct counting for the small universes),
    # 1: LDS hash tables, 2: partitioned counting (same results)
    gen, U = DISTS[dist]
    ctx = tk.Context(0, seed=1234).set_param("fq_mode", mode)
    for n in (1, 7, 4097, (1 << 20) + 3, 1 << 22):
        keys = gen(n, n % 97 + 1)
        for k in sorted({1, min(32, U), min(U, 17)}):
            for T in (1 << 32, F.threshold(n, max(1, n // 10))):
                kstar = 0 if method == "pac" else min(U, 4096, 4 * k)
                run_freq(ctx, keys, U, k, kstar, T, dev)


@pytest.mark.gpu
def test_frequent_kstar_limits_and_small_universe(dev):
    ctx = tk.Context(0, seed=5)
    keys = synth.zipf_u32(300001, 1.0, 4096, 6)
    for k, kstar in ((1, 1), (4096, 4096), (100, 4096), (7, 7)):
        run_freq(ctx, keys, 4096, k, kstar, F.threshold(keys.size, 5000), dev)
    # k = U: every object, most frequent first (zero counts last by object)
    run_freq(ctx, synth.small_alphabet_u32(1000, 5, 2), 9, 9, 0, 1 << 32, dev)


@pytest.mark.gpu
@pytest.mark.parametrize("mode", [0, 2])
@pytest.mark.parametrize("U", [1, 2, 8191, 8192, 8193, 3 * 8192 + 5, 1 << 15, (1 << 15) + 1,
                               1 << 25, (1 << 25) + 1])
def test_frequent_partition_edges(dev, U, mode):
    # universes at the method boundaries (the largest direct universe, one
    # partition, a ragged last partition, the most partitions, the first
    # universe counted by hashing)
    ctx = tk.Context(0, seed=21).set_param("fq_mode", mode)
    n = 200003
    keys = (synth.uniform_u32(n, U % 89 + 3) % np.uint32(U)).astype(np.uint32)
    keys[: n // 3] = keys[: n // 3] % np.uint32(min(U, 5))          # a few hot objects
    for kstar, T in ((0, 1 << 32), (min(U, 64), F.threshold(n, 50000))):
        run_freq(ctx, keys, U, min(U, 10), kstar, T, dev)


@pytest.mark.gpu
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_frequent_bad_keys_are_skipped(dev, mode):
    ctx = tk.Context(0, seed=9).set_param("fq_mode", mode)
    U = 1000
    keys = synth.zipf_u32(100000, 1.0, U + 50, 3)        # some keys >= U
    out = ctx.frequent(dev_u32(keys, dev), U, 10, T=1 << 32, tables=True)
    torch.cuda.synchronize()
    assert int(out["status"].item()) == tk.STATUS_BAD_KEY
    ref = np.bincount(keys[keys < U], minlength=U)
    assert np.array_equal(out["sample_counts"].cpu().numpy(), ref)
    ids, cnt = F.top_by_count(ref, 10)
    assert np.array_equal(out["ids"].cpu().numpy().view(np.uint32), ids)


@pytest.mark.gpu
def test_frequent_argument_errors(dev):
    ctx = tk.Context(0)
    keys = torch.zeros(100, dtype=torch.int32, device=dev)
    for kw in (dict(U=10, k=0), dict(U=10, k=11), dict(U=10, k=2, kstar=1),
               dict(U=10, k=2, T=0), dict(U=10, k=2, T=(1 << 32) + 1), dict(U=0, k=1)):
        with pytest.raises(tk.TopkError):
            ctx.frequent(keys, **kw)
    with pytest.raises(tk.TopkError):                  # 16-byte alignment
        ctx.frequent(torch.zeros(101, dtype=torch.int32, device=dev)[1:], 10, 2)


@pytest.mark.gpu
@pytest.mark.parametrize("method", ["pac", "ec"])
def test_frequent_fullsize_zipf(dev, method):
    # the workload of §10.2 on one device: n = 2^28 objects, Zipf(1) over
    # 2^20 values, k = 32, (eps, delta) = (3e-4, 1e-4)
    n, U, k = 1 << 28, 1 << 20, 32
    keys = synth.zipf_u32(n, 1.0, U, 7)
    kstar = 0 if method == "pac" else k
    size = F.sample_size_pac(n, k, 3e-4, 1e-4) if method == "pac" else \
        F.sample_size_ec(n, k, 3e-4, 1e-4)
    run_freq(tk.Context(0, seed=0x5EED), keys, U, k, kstar, F.threshold(n, size), dev)


def run_sum(ctx, keys, values, U, k, kstar, s, dev):
    print("sum: n=%d U=%d k=%d kstar=%d s=%d" % (keys.size, U, k, kstar, s), flush=True)
    out = ctx.sum_top(dev_u32(keys, dev), dev_u32(values, dev), U, k, s, kstar=kstar, tables=True)
    torch.cuda.synchronize()
    assert int(out["status"].item()) == 0
    seed = ctx.get_param("seed")
    sums = F.sums_by_key(keys, values, U)
    assert np.array_equal(out["sums"].cpu().numpy().view(np.uint64), sums)
    samp, _ = F.weighted_sample(sums, s, seed, 0)
    assert np.array_equal(out["samples"].cpu().numpy().view(np.uint32), samp)
    if kstar == 0:
        ids, vals = F.top_by_count(samp, k)
    else:
        cand, _ = F.top_by_count(samp, kstar)
        ids, vals = F.top_by_count(sums, k, candidates=cand)
    assert np.array_equal(out["ids"].cpu().numpy().view(np.uint32), ids)
    assert np.array_equal(out["vals"].cpu().numpy().view(np.uint64), vals.astype(np.uint64))


@pytest.mark.gpu
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("kstar", [0, 64])
def test_sum_parity(dev, kstar, mode):
    ctx = tk.Context(0, seed=77).set_param("fq_mode", mode)
    # the last case: values up to 2^32 - 1, so per-wave partial sums carry
    # past 32 bits
    for n, U, vmax in ((5, 3, 10), (4099, 500, 1000), ((1 << 20) + 1, 1 << 16, 1 << 20),
                       (1 << 22, 1 << 20, 65535), (1 << 22, 1000, 0xFFFFFFFF)):
        keys, values = synth.keyed_values(n, U, 1.1, vmax, n % 13)
        for k, s in ((1, 10), (min(U, 16), 1000), (min(U, 32), 1 << 20)):
            kk = min(U, max(kstar, k)) if kstar else 0
            run_sum(ctx, keys, values, U, k, kk, s, dev)


@pytest.mark.gpu
def test_sum_fullsize(dev):
    n, U = 1 << 26, 1 << 20
    keys, values = synth.keyed_values(n, U, 1.0, 1000, 11)
    s = int(F.sample_size_sum(n, 3e-4, 1e-4))
    run_sum(tk.Context(0, seed=0x5EED), keys, values, U, 32, 0, s, dev)
    run_sum(tk.Context(0, seed=0x5EED), keys, values, U, 32, 256, s, dev)


def test_sample_size_helpers_match_the_oracle():
    # host arithmetic of the library (no device call) against the oracle's formulas
    if not __import__("os").path.exists(tk.LIB_PATH):
        pytest.fail("libtopk.so not built")
    for n, k, kstar, eps, delta in ((1 << 28, 32, 32, 3e-4, 1e-4), (1 << 20, 5, 40, 1e-2, 1e-3),
                                    (1 << 40, 1, 1, 0.01, 0.5)):
        assert tk.sample_size(tk.SAMPLE_PAC, n, k, 0, eps, delta) == \
            pytest.approx(F.sample_size_pac(n, k, eps, delta), rel=1e-12)
        assert tk.sample_size(tk.SAMPLE_EC, n, k, kstar, eps, delta) == \
            pytest.approx(F.sample_size_ec(n, kstar, eps, delta), rel=1e-12)
        assert tk.sample_size(tk.SAMPLE_SUM, n, k, kstar, eps, delta) == \
            pytest.approx(F.sample_size_sum(n, eps, delta), rel=1e-12)
    for n, size in ((1 << 28, 1 << 26), (1 << 28, 1e12), (1000, 1), (12345, 77.5)):
        assert tk.sample_threshold(n, size) == F.threshold(n, size)
    assert tk.sample_size(tk.SAMPLE_PAC, 0, 1, 0, 0.1, 0.1) == -1.0
