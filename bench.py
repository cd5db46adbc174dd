#!/usr/bin/env python3
"""Throughput of the sampling top-k selection on one MI355X.

One step = select the k smallest of n = 2^28 fp32 keys (uniform on [0,1) at
2^-24 resolution, seeded, resident in HBM) for each k in {2^10, 2^20, 2^27}.
Prints one JSON line on stdout; progress goes to stderr.

  value        whole-step keys processed per second (3 * 2^28 keys per step)
  roofline     the dominant kernel (the first-round sweep): algorithmic bytes
               per launch (4 B read per key + 4 B per position written below
               the lower pivot + 8 B per (ord, position) pair written to the
               band) divided by its average duration, both measured here with
               HIP events on the library's stream during the timed steps
  cpu_baseline the CPU oracle (sort by (value, position) as 64-bit composites)
               on every host thread over the whole step, plus one thread on a
               bounded sample
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Gkeys/s and % HBM roofline, top-k select n=2^28 fp32; batched vs per-row loop"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


# sources of the first-round sweep kernel (its constants, state layout and code)
TRAFFIC_SOURCES = ("select.hpp", "select_impl.hpp")


def traffic_record(kernel):
    """Measured HBM bytes per launch from a committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % kernel)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1502_03942_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    sha = h.hexdigest()
    if rec.get("source_sha256") != sha:
        return None
    return rec


def bench_select(args):
    import torch
    import paper_1502_03942_amd as tk
    import synth

    n = 1 << 28
    ks = (1 << 10, 1 << 20, 1 << 27)
    dev = torch.device("cuda:0")
    log("generating %d f32 keys" % n)
    keys_np = synth.uniform_f32_grid(n, 2)
    keys = torch.from_numpy(keys_np).to(dev)
    # one context per k: the autotuner (setup, untimed) picks s_target and
    # c_num for each selection
    ctxs = {k: tk.Context(0, seed=0x5EED) for k in ks}
    ws = {k: ctxs[k].workspace(n) for k in ks}
    tuned = {}
    for k in ks:
        if args.tuning_prefix:
            ctxs[k].load_tuning(args.tuning_prefix + "single_k%d.json" % k)
        elif not args.no_tune:
            ctxs[k].tune(keys, k, reps=10, workspace=ws[k])
        if args.save_tuning_prefix:
            ctxs[k].save_tuning(args.save_tuning_prefix + "single_k%d.json" % k)
        tuned[str(k)] = {"s_target": ctxs[k].get_param("s_target"),
                         "c_num": ctxs[k].get_param("c_num")}
        ctxs[k].set_param("timing", 1)
    if args.tuning_prefix or not args.no_tune:
        log("tuned: %s" % tuned)
    results = {}

    def step():
        for k in ks:
            results[k] = ctxs[k].select(keys, k, workspace=ws[k])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for k in ks:
        ctxs[k].kernel_times()                # drop warm-up records
    log("warmup done; timing %d steps" % args.steps)
    per_k_ms = {k: 0.0 for k in ks}
    # whole-step time: events on the stream the library launches on
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    ek = [torch.cuda.Event(enable_timing=True) for _ in range(len(ks) + 1)]
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        for i, k in enumerate(ks):
            results[k] = ctxs[k].select(keys, k, workspace=ws[k])
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    sweeps_k = {k: [ms for kind, ms in ctxs[k].kernel_times() if kind == "sweep_first"]
                for k in ks}
    sweeps = [ms for k in ks for ms in sweeps_k[k]]
    assert all(len(sweeps_k[k]) == args.steps for k in ks), {k: len(v) for k, v in sweeps_k.items()}
    # per-k whole-call times (separate short pass, same launches)
    for i, k in enumerate(ks):
        ek[0].record(stream)
        for _ in range(args.steps):
            ctxs[k].select(keys, k, workspace=ws[k])
        ek[1].record(stream)
        torch.cuda.synchronize()
        per_k_ms[k] = ek[0].elapsed_time(ek[1]) / args.steps
    for k in ks:
        ctxs[k].kernel_times()

    # the canonical output order (TOPK_SORTED), reported beside the step (not
    # part of it): the same selections with their outputs sorted by (key,
    # position), timed the same way; one workspace serves the three
    sorted_order = {}
    ws_sorted = torch.empty(max(ctxs[k].workspace_bytes(n, tk.TOPK_SORTED) for k in ks)
                            if not args.no_sorted else 256, dtype=torch.uint8, device=dev)
    for k in (ks if not args.no_sorted else ()):
        ctxs[k].set_param("timing", 0)
        r = ctxs[k].select(keys, k, workspace=ws_sorted, sorted=True)
        torch.cuda.synchronize()
        if int(r["idx"][-1].item()) != int(r["kth_idx"].item()):
            raise SystemExit("sorted output of k=%d does not end with the k-th pair" % k)
        reps = 3
        ek[0].record(stream)
        for _ in range(reps):
            ctxs[k].select(keys, k, workspace=ws_sorted, sorted=True)
        ek[1].record(stream)
        torch.cuda.synchronize()
        ms = ek[0].elapsed_time(ek[1]) / reps
        sorted_order[str(k)] = {"ms": round(ms, 4), "sort_ms": round(ms - per_k_ms[k], 4)}
    del ws_sorted
    log("sorted order: %s" % sorted_order)

    ms_per_step = total_ms / args.steps
    value = len(ks) * n / (ms_per_step * 1e-3) / 1e9

    # algorithmic bytes of each k's first sweep, from its round record
    sweep_bytes = {}
    per_k = []
    for k in ks:
        recs = ctxs[k].trace_rounds(results[k])
        r0 = recs[0]
        sweep_bytes[k] = 4 * n + 4 * r0["na"] + 8 * r0["nb"]
        b_min = 4 * n + 4 * k
        per_k.append({
            "k": k, "ms": round(per_k_ms[k], 4),
            "gkeys_s": round(n / (per_k_ms[k] * 1e-3) / 1e9, 2),
            "hbm_frac_min_bytes": round(b_min / (per_k_ms[k] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "rounds": len(recs), "band1": r0["nb"], "below1": r0["na"],
        })
    tot_bytes = sum(sweep_bytes[k] * len(sweeps_k[k]) for k in ks)
    tot_s = sum(sweeps) * 1e-3
    achieved = tot_bytes / tot_s / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_sweep<first round>",
            "avg_launch_ms": round(sum(sweeps) / len(sweeps), 5),
            "algorithmic_bytes_per_launch": round(tot_bytes / len(sweeps))}
    tr = traffic_record("sweep_first")
    if tr is not None:
        roof["traffic"] = tr["bytes_per_launch"]

    if not args.no_check:
        import oracle
        for k in ks:
            r = results[k]
            got = r["idx"].cpu().numpy().view(np.uint32)
            kth = int(r["kth_idx"].item())
            kb = int(r["kth_key"].cpu().numpy().view(np.uint32)[0])
            rc = oracle.check(keys_np, k, got, kth, kb, False)
            log("check k=%d: %s" % (k, "ok" if rc == 0 else "FAILED invariant %d" % rc))
            if rc != 0 or int(r["status"].item()) != 0:
                raise SystemExit("result check failed for k=%d" % k)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        model, ncpu = cpu_info()
        # the host's CPU share for this process: OMP_NUM_THREADS where the
        # environment sets it, else the CPUs it may run on
        threads = int(os.environ.get("OMP_NUM_THREADS") or 0) or \
            (len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else ncpu)
        # every host thread, the whole workload: the three selections of the
        # step by the oracle's composite-key sort (chunk sorts + merge of k)
        log("cpu baseline: oracle composite sort, %d threads, n=2^28" % threads)
        t0 = time.perf_counter()
        for k in ks:
            oracle.select_composite(keys_np, k, False, threads)
        dt_all = time.perf_counter() - t0
        # one thread on a bounded sample: the first 2^24 keys, k scaled by 2^-4
        m = 1 << 24
        ks_s = [max(1, k * m // n) for k in ks]
        log("cpu baseline: oracle composite sort, 1 thread, first 2^24 keys")
        t0 = time.perf_counter()
        for k in ks_s:
            oracle.select_composite(keys_np[:m], k, False, 1)
        dt_one = time.perf_counter() - t0
        cpu = {"value": round(len(ks) * n / dt_all / 1e9, 5), "unit": "Gkeys/s", "cores": threads,
               "kind": "oracle",
               "sample": "the whole step (n=2^28 f32, k in {2^10, 2^20, 2^27}) by the oracle's "
                         "sort of 64-bit (value word, position) composites on %d threads (chunk "
                         "sorts, merge of the first k): %.1f s; host %s (%d logical CPUs)"
                         % (threads, dt_all, model, ncpu),
               "single_thread": {"value": round(len(ks_s) * m / dt_one / 1e9, 5),
                                 "unit": "Gkeys/s", "cores": 1,
                                 "sample": "first 2^24 keys, k scaled by 2^-4 to %s: %.1f s"
                                           % (ks_s, dt_one)}}

    return {
        "metric": METRIC, "value": round(value, 2), "unit": "Gkeys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "select smallest k of n=2^28 f32 keys uniform on [0,1) "
                               "(2^-24 grid, seed 2), k in {2^10, 2^20, 2^27}, one step = "
                               "the three selections", "n": n, "k": list(ks),
                   "parallelism": "none (1 GPU)"},
        "per_k": per_k, "tuned": tuned if (args.tuning_prefix or not args.no_tune) else None,
        "roofline": roof, "cpu_baseline": cpu,
        "sorted_order": {"how": "the same selections with TOPK_SORTED (outputs in (key, position) "
                                "order), mean of 3 calls; sort_ms = the sorted call minus the "
                                "plain one", **sorted_order},
    }


def bench_configs(args, c2_ms_per_k):
    """The other single-instance configurations (u32 keys; parity-tested at the
    same sizes), each timed with the default parameters (median of 10 calls;
    the autotuner takes f32 keys), and the
    bandwidth of a plain stream read of the 2^28 f32 array measured on the
    same device, against which C2 is also reported."""
    import torch
    import paper_1502_03942_amd as tk
    import synth

    dev = torch.device("cuda:0")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn, reps=10):
        # back-to-back calls between the events, so that the host's launch
        # latency of each call is not counted
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {}
    # stream read: the library's plain read kernel (the first sweep's access
    # pattern) over the 1 GiB array; torch reductions beside it for context
    x = torch.from_numpy(synth.uniform_f32_grid(1 << 28, 2)).to(dev)
    sink = torch.zeros(1, dtype=torch.int32, device=dev)
    mctx = tk.Context(0)
    probes = {"topk_stream_read": lambda: mctx.stream_read(x, sink),
              "torch_sum": lambda: x.sum(), "torch_amax": lambda: torch.amax(x)}
    gbs = {}
    for name, fn in probes.items():
        for _ in range(3):
            fn()
        gbs[name] = (1 << 30) / (timed(fn) * 1e-3) / 1e9
    read_gbs = gbs["topk_stream_read"]
    out["stream_read"] = {"how": "topk_stream_read over 2^28 f32 keys (1 GiB read once, "
                                 "256-byte non-temporal column loads), mean of 10 back-to-back calls",
                          "gbs": round(read_gbs, 1),
                          "probes_gbs": {k: round(v, 1) for k, v in gbs.items()}}
    out["C2_frac_of_stream_read"] = {
        str(k): round((4 * (1 << 28) + 4 * k) / (ms * 1e-3) / 1e9 / read_gbs, 4)
        for k, ms in c2_ms_per_k.items()}
    del x
    cfgs = [
        ("C1", "u32 n=2^20 uniform, seed 1", lambda: synth.uniform_u32(1 << 20, 1), 1000, False),
        ("C3a", "u32 n=2^27 Zipf s=1.2 over 2^16 values, seed 3", lambda: synth.zipf_u32(1 << 27, 1.2, 1 << 16, 3), 1 << 20, False),
        ("C3b", "C3a data, largest", None, 1 << 20, True),
        ("C3c", "u32 n=2^27 all 2^31 but Bernoulli(0.01) uniform, seed 31", lambda: synth.all_equal_except(1 << 27, 0.01, 1 << 31, 31), 1 << 20, False),
    ]
    keys = None
    for name, what, gen, k, largest in cfgs:
        if gen is not None:
            keys_np = gen()
            keys = torch.from_numpy(keys_np.view(np.int32)).to(dev)
        n = keys.numel()
        ctx = tk.Context(0, seed=0x5EED)
        ws = ctx.workspace(n)
        for _ in range(2):
            ctx.select(keys, k, largest=largest, workspace=ws)
        ms = timed(lambda: ctx.select(keys, k, largest=largest, workspace=ws))
        res = ctx.select(keys, k, largest=largest, workspace=ws)
        torch.cuda.synchronize()
        if int(res["status"].item()) != 0:
            raise SystemExit("%s: status %d" % (name, int(res["status"].item())))
        b_min = 4 * n + 4 * k
        out[name] = {"workload": what, "n": n, "k": k, "largest": largest, "ms": round(ms, 4),
                     "gkeys_s": round(n / (ms * 1e-3) / 1e9, 2),
                     "hbm_frac_min_bytes": round(b_min / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}
        log("%s: %.4f ms" % (name, ms))
    return out


def bench_batched(args):
    """The batched form on 65,536 lognormal rows (one graph launch per step),
    next to the plain per-row loop (topk_select_f32 per row) on a sample of
    rows, scaled to the whole batch."""
    import torch
    import paper_1502_03942_amd as tk
    import synth

    dev = torch.device("cuda:0")
    R = 65536
    log("generating the batch (%d rows)" % R)
    keys_np, off_np, k_np = synth.lognormal_rows(R, 4096, 1.0, 64, 1 << 20, 2048, 4)
    keys = torch.from_numpy(keys_np).to(dev)
    off = torch.from_numpy(off_np.astype(np.int64)).to(dev)
    kk = torch.from_numpy(k_np.astype(np.int32)).to(dev)
    ctx = tk.Context(0, seed=0x5EED)
    tuned = {}
    if args.tuning_prefix:
        ctx.load_tuning(args.tuning_prefix + "batched.json")
        log("tuning loaded from %sbatched.json" % args.tuning_prefix)
    elif not args.no_tune:
        # the autotuner (setup, untimed): sample size, spread and sweep tile
        # per length class of the sampling path, attempts, workgroups per CU
        ctx.tune_batched(keys, off, kk, reps=3)
    if args.tuning_prefix or not args.no_tune:
        for c in range(34):
            sv = ctx.get_param("bt_s_target@%d" % c)
            if sv >= 0:
                tuned["class_%d" % c] = {"bt_s_target": sv, "bt_c_num": ctx.get_param("bt_c_num@%d" % c),
                                         "bt_tile": ctx.get_param("bt_tile@%d" % c)}
        tuned["bt_wg_per_cu"] = ctx.get_param("bt_wg_per_cu")
        tuned["bt_attempts"] = ctx.get_param("bt_attempts")
        log("tuned: %s" % tuned)
        if args.save_tuning_prefix:
            ctx.save_tuning(args.save_tuning_prefix + "batched.json")
    out = ctx.select_batched(keys, off, kk, graph=True)
    for _ in range(max(1, args.warmup)):
        out = ctx.select_batched(keys, off, kk, graph=True, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    steps = max(1, args.steps)
    e0.record(stream)
    for _ in range(steps):
        out = ctx.select_batched(keys, off, kk, graph=True, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    if int(out["status"].item()) != 0:
        raise SystemExit("batched status %d" % int(out["status"].item()))
    checked = None
    if not args.no_check:
        # the timed (tuned) configuration's output, every row, by the oracle's
        # checker (outside the timed region)
        import oracle
        idx = out["idx"].cpu().numpy().view(np.uint32)
        kth = out["kth_idx"].cpu().numpy().view(np.uint32)
        kkey = out["kth_key"].cpu().numpy().view(np.uint32)
        oo = out["out_off"].cpu().numpy()
        bad = []
        for r in range(R):
            row = keys_np[int(off_np[r]):int(off_np[r + 1])]
            k = int(k_np[r])
            sel = idx[int(oo[r]):int(oo[r]) + k]
            rc = oracle.check(row, k, sel, int(kth[r]), int(kkey[r]), False)
            if rc != 0:
                bad.append((r, rc))
        log("batched check: %s" % ("ok (%d rows)" % R if not bad else "FAILED %s" % bad[:5]))
        if bad:
            raise SystemExit("batched result check failed")
        checked = "every row by the oracle's checker: ok"
    total = int(off_np[-1])
    sum_k = int(k_np.astype(np.int64).sum())
    b_min = 4 * total + 4 * sum_k + 20 * R
    # plain per-row loop on a sample of rows (every 64th row), scaled by rows
    lens = np.diff(off_np.astype(np.int64))
    rows = list(range(0, R, 64))
    ws = ctx.workspace(int(lens.max()))
    for r in rows[:8]:
        ctx.select(keys[int(off_np[r]):int(off_np[r + 1])], int(k_np[r]), workspace=ws)
    torch.cuda.synchronize()
    e0.record(stream)
    for r in rows:
        ctx.select(keys[int(off_np[r]):int(off_np[r + 1])], int(k_np[r]), workspace=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    loop_ms = e0.elapsed_time(e1) * R / len(rows)
    log("batched: %.3f ms, per-row loop (scaled from %d rows): %.1f ms" % (ms, len(rows), loop_ms))
    return {"workload": "65,536 rows f32 ~N(0,1), lengths lognormal (median 4096, sigma 1, "
                        "clipped to [64, 2^20]), k ~ U{1..min(len, 2048)}, seed 4; one hipGraph "
                        "launch per step",
            "rows": R, "keys": total, "sum_k": sum_k, "ms": round(ms, 4), "check": checked,
            "tuned": tuned or None,
            "gkeys_s": round(total / (ms * 1e-3) / 1e9, 2),
            "hbm_frac_min_bytes": round(b_min / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "per_row_loop": {"ms_est": round(loop_ms, 2), "rows_timed": len(rows),
                             "how": "topk_select_f32 per row on the same stream, every 64th "
                                    "row, time scaled by 64",
                             "speedup": round(loop_ms / ms, 1)}}


def bench_rows(args):
    """Row-wise top-k forward and gradient scatter, scores [4096, 32768], k = 64."""
    import torch
    import paper_1502_03942_amd as tk

    dev = torch.device("cuda:0")
    B, N, k = 4096, 32768, 64
    g = torch.Generator(device="cpu").manual_seed(5)
    scores = torch.randn(B, N, generator=g).to(dev)
    gout = torch.randn(B, k, generator=g).to(dev)
    v, i = tk.rows_fwd(scores, k)
    gin = tk.scatter_bwd(gout, i, N)
    stream = torch.cuda.current_stream(dev)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    steps = max(1, args.steps)
    torch.cuda.synchronize()
    e[0].record(stream)
    for _ in range(steps):
        v, i = tk.rows_fwd(scores, k)
    e[1].record(stream)
    for _ in range(steps):
        gin = tk.scatter_bwd(gout, i, N)
    e[2].record(stream)
    torch.cuda.synchronize()
    fwd = e[0].elapsed_time(e[1]) / steps
    bwd = e[1].elapsed_time(e[2]) / steps
    fb = 4 * B * N + 12 * B * k
    bb = 4 * B * N + 12 * B * k
    return {"workload": "scores f32 [4096, 32768] ~N(0,1) seed 5, k = 64 largest; grad_out "
                        "f32 [4096, 64]",
            "fwd_ms": round(fwd, 4), "fwd_gbs": round(fb / (fwd * 1e-3) / 1e9, 1),
            "fwd_frac": round(fb / (fwd * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "bwd_ms": round(bwd, 4), "bwd_gbs": round(bb / (bwd * 1e-3) / 1e9, 1),
            "bwd_frac": round(bb / (bwd * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}


def _timed(fn, reps=10):
    """Mean of reps back-to-back calls (ms) on the current stream, HIP events
    around the batch (the host's launch latency of each call is not counted)."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_frequent(args):
    """Top-k most frequent objects (PAC and EC) and top-k sum aggregation on
    the workloads of the paper's most-frequent-objects experiment, one device:
    n = 2^28 objects, Zipf(1) over 2^20 values and negative binomial (r = 1000,
    p = 0.05), k = 32, (eps, delta) = (3e-4, 1e-4).  Results are checked
    against the oracle outside the timed region."""
    import torch
    import paper_1502_03942_amd as tk
    import synth
    import oracle

    dev = torch.device("cuda:0")
    n, k, eps, delta = 1 << 28, 32, 3e-4, 1e-4
    out = {}
    for name, gen, U in (("zipf1_2p20", lambda: synth.zipf_u32(n, 1.0, 1 << 20, 7), 1 << 20),
                         ("negbin_r1000_p005", lambda: synth.negbin_u32(n, 1000, 0.05, 1 << 15, 8),
                          1 << 15)):
        log("frequent: generating %s" % name)
        keys_np = gen()
        keys = torch.from_numpy(keys_np.view(np.int32)).to(dev)
        ctx = tk.Context(0, seed=0x5EED)
        nb = int(tk.lib().topk_frequent_workspace_bytes(ctx._h, n, U))
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        res = {}
        for method, kstar in (("pac", 0), ("ec", k)):
            size = tk.sample_size(tk.SAMPLE_PAC if kstar == 0 else tk.SAMPLE_EC, n, k, kstar, eps, delta)
            T = tk.sample_threshold(n, size)
            ms = _timed(lambda: ctx.frequent(keys, U, k, kstar=kstar, T=T, workspace=ws))
            r = ctx.frequent(keys, U, k, kstar=kstar, T=T, workspace=ws)
            torch.cuda.synchronize()
            ids = r["ids"].cpu().numpy().view(np.uint32)
            cnt = r["counts"].cpu().numpy().view(np.uint32)
            if not args.no_check:
                if kstar == 0:
                    rid, rc_, _ = oracle.freq.pac(keys_np, U, k, T, 0x5EED)
                else:
                    rid, rc_, _ = oracle.freq.ec(keys_np, U, k, kstar, T, 0x5EED)
                if not (np.array_equal(ids, rid) and np.array_equal(cnt, rc_.astype(np.uint32))):
                    raise SystemExit("frequent %s %s: result differs from the oracle" % (name, method))
            passes = 1 if kstar == 0 else 2
            res[method] = {"ms": round(ms, 4), "gkeys_s": round(n / (ms * 1e-3) / 1e9, 2),
                           "rho": round(min(1.0, T / 2.0**32), 6),
                           "hbm_frac_min_bytes": round(4 * n * passes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                           "check": None if args.no_check else "equal to the oracle"}
            log("frequent %s %s: %.4f ms" % (name, method, ms))
        out[name] = res
        del keys
    # sum aggregation: 2^26 (key, value) pairs, keys Zipf(1) over 2^20, values in [0, 1000]
    nn, U = 1 << 26, 1 << 20
    keys_np, vals_np = synth.keyed_values(nn, U, 1.0, 1000, 11)
    kd = torch.from_numpy(keys_np.view(np.int32)).to(dev)
    vd = torch.from_numpy(vals_np.view(np.int32)).to(dev)
    ctx = tk.Context(0, seed=0x5EED)
    ws = torch.empty(int(tk.lib().topk_sum_workspace_bytes(ctx._h, nn, U)), dtype=torch.uint8, device=dev)
    s_size = int(tk.sample_size(tk.SAMPLE_SUM, nn, k, 0, eps, delta))
    res = {}
    for method, kstar in (("pac", 0), ("exact_sums", 4 * k)):
        ms = _timed(lambda: ctx.sum_top(kd, vd, U, k, s_size, kstar=kstar, workspace=ws))
        r = ctx.sum_top(kd, vd, U, k, s_size, kstar=kstar, workspace=ws)
        torch.cuda.synchronize()
        if not args.no_check:
            if kstar == 0:
                rid, rv = oracle.freq.sum_pac(keys_np, vals_np, U, k, s_size, 0x5EED)
            else:
                rid, rv = oracle.freq.sum_ec(keys_np, vals_np, U, k, kstar, s_size, 0x5EED)
            if not (np.array_equal(r["ids"].cpu().numpy().view(np.uint32), rid) and
                    np.array_equal(r["vals"].cpu().numpy().view(np.uint64), rv.astype(np.uint64))):
                raise SystemExit("sum aggregation %s: result differs from the oracle" % method)
        res[method] = {"ms": round(ms, 4), "gpairs_s": round(nn / (ms * 1e-3) / 1e9, 2),
                       "hbm_frac_min_bytes": round(8 * nn / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}
        log("sum %s: %.4f ms" % (method, ms))
    out["sum_aggregation_2p26_pairs"] = dict(res, sample_size=s_size)
    out["workload"] = ("n = 2^28 objects per distribution, k = 32, (eps, delta) = (3e-4, 1e-4): "
                       "PAC at the rate of the sample-size equation (rho = 1 here), EC with k* = 32 "
                       "at the rate of Lemma topkec; sum aggregation on 2^26 pairs")
    return out


def bench_msselect(args):
    """Selection over 1024 sorted rows of 2^18 f32 keys (2^28 keys): msSelect
    for k in {2^10, 2^20, 2^27}, amsSelect for [k - k/8, k].  Latency-bound
    (dependent binary searches): reported in microseconds per call."""
    import torch
    import paper_1502_03942_amd as tk
    import synth
    import oracle

    dev = torch.device("cuda:0")
    p, L = 1024, 1 << 18
    keys_np = synth.uniform_f32_grid(p * L, 9).reshape(p, L)
    keys_np.sort(axis=1)
    keys_np = keys_np.reshape(-1)
    off_np = (np.arange(p + 1, dtype=np.int64) * L)
    keys = torch.from_numpy(keys_np).to(dev)
    off = torch.from_numpy(off_np).to(dev)
    ctx = tk.Context(0, seed=0x5EED)
    out = {"workload": "1024 rows of 2^18 sorted f32 keys (uniform on [0,1), 2^-24 grid, seed 9)"}
    for k in (1 << 10, 1 << 20, 1 << 27):
        ms = _timed(lambda: ctx.msselect(keys, off, k))
        r = ctx.msselect(keys, off, k)
        ra = ctx.amsselect(keys, off, k - k // 8, k)
        ms_a = _timed(lambda: ctx.amsselect(keys, off, k - k // 8, k))
        torch.cuda.synchronize()
        if not args.no_check:
            kth, split = oracle.msselect.ms_select(keys_np, off_np, k, False, threads=16)
            if not (np.array_equal(r["split"].cpu().numpy().astype(np.int64), split.astype(np.int64))
                    and int(r["kth_pos"].item()) == kth):
                raise SystemExit("msselect k=%d: result differs from the oracle" % k)
            if oracle.msselect.ams_check(keys_np, off_np, k - k // 8, k,
                                         ra["split"].cpu().numpy().astype(np.int64)) != 0:
                raise SystemExit("amsselect k=%d: invalid result" % k)
        out[str(k)] = {"msselect_us": round(ms * 1e3, 1), "msselect_rounds": int(r["rounds"].item()),
                       "amsselect_us": round(ms_a * 1e3, 1), "amsselect_rounds": int(ra["rounds"].item()),
                       "amsselect_k": int(ra["k"].item())}
        log("msselect k=%d: %.1f us (%d rounds); amsselect: %.1f us" %
            (k, ms * 1e3, int(r["rounds"].item()), ms_a * 1e3))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-sorted", action="store_true",
                    help="skip the timing of the sorted output order (TOPK_SORTED)")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched form with the default parameters (no autotuner run)")
    ap.add_argument("--tuning-prefix", metavar="PREFIX",
                    help="load the tuning files PREFIX{single_k<k>,batched}.json instead of "
                         "running the autotuners")
    ap.add_argument("--save-tuning-prefix", metavar="PREFIX",
                    help="write the parameters each selection ran with to those files")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched form (no JSON line: a profiling aid)")
    ap.add_argument("--rows-only", action="store_true",
                    help="only the row-wise forward and backward (no JSON line: a profiling aid)")
    ap.add_argument("--frequent-only", action="store_true",
                    help="only the most-frequent-objects, sum-aggregation and sorted-rows "
                         "selections (no JSON line: a profiling aid)")
    ap.add_argument("--single-only", action="store_true",
                    help="only the single-instance selection (skip the batched and row forms)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (the reference kernel "
                         "for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the selection runs on a single device "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 2^30 bytes read, 2^30 bytes written")
        del src, dst
    if args.batched_only:
        log("batched: %s" % json.dumps(bench_batched(args)))
        return
    if args.rows_only:
        log("rows: %s" % json.dumps(bench_rows(args)))
        return
    if args.frequent_only:
        log("frequent: %s" % json.dumps(bench_frequent(args)))
        log("msselect: %s" % json.dumps(bench_msselect(args)))
        return
    out = bench_select(args)
    if not args.single_only:
        out["configs"] = bench_configs(args, {p["k"]: p["ms"] for p in out["per_k"]})
        out["batched"] = bench_batched(args)
        out["rows_topk"] = bench_rows(args)
        out["frequent"] = bench_frequent(args)
        out["sorted_rows"] = bench_msselect(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
