"""Benchmark: word-count throughput on one MI355X, as GB/s of text and fraction of HBM peak.

Workload "stream-8GiB": one 8 GiB document of Zipf(s = 1.0) text over a 1,000,000-word
vocabulary (lengths 1..16), generated on the GPU from a fixed seed; global table of 2^22
slots; int64 counts. One step = one wc_count call: clear the table, scan and count the whole
corpus, compact the table into (word, count) arrays, read the sizes back. The corpus is
resident in HBM before timing starts.

Beside the headline the JSON line carries: the dominant kernel's roofline (pass 1, HIP events
on the call's stream; HBM traffic from the committed counter summary while the kernel source
is unchanged), the oracle on one core and the paper's threaded CPU design on all cores, the
measured device-copy rate, the same text from pinned host memory (copy then count, and
pieces counted while later pieces are in flight), plain-1MB, corpora-4x2000 with its top-50,
the paper's dense reduce beside the hash merge, batched-100k against one launch per document,
serving (pinned host and device-resident input) against one launch per request, and Section
4.2's float sums.

Prints one JSON line (rank 0). Runs on one GPU only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "stream-8GiB"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per launch of pass 1 from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE, scaled by a device copy of known size), or None once the kernel source has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "global_map_kernel_stream-8GiB.traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        h = hashlib.sha256()
        for src in rec["sources"]:  # the kernel's source file and the headers it includes
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        sha = h.hexdigest()
    except (OSError, ValueError, KeyError, TypeError):
        return None
    return int(rec["traffic_bytes"]) if sha == rec["sources_sha256"] else None


def cpu_baseline(corpus, sample_bytes: int):
    """Time the oracle (single-threaded CPU) on the first sample_bytes of the corpus."""
    import numpy as np
    import oracle
    host = corpus[:sample_bytes].cpu().numpy()
    # cut at a delimiter so the sample is a prefix of whole tokens
    oracle.lib()
    t0 = time.perf_counter()
    t = oracle.count(host, np.array([0, len(host)], dtype=np.int64))
    dt = time.perf_counter() - t0
    return {"value": round(len(host) / dt / 1e9, 4), "unit": "GB/s", "cores": 1,
            "kind": "oracle",
            "sample": f"first {len(host)} bytes of the {WORKLOAD} corpus "
                      f"({t.total} tokens, {len(t)} words) in {dt:.2f} s"}


def cpu_parallel_baseline(corpus, sample_bytes: int):
    """Time the paper's threaded CPU design (Section 3.1 map on threads, Section 3.2 merge;
    oracle/cpu_parallel.cpp) on all host cores available to this process, on the same sample
    as the oracle."""
    import numpy as np
    import oracle
    host = corpus[:sample_bytes].cpu().numpy()
    cores = len(os.sched_getaffinity(0))
    oracle.lib()
    _, total, secs = oracle.cpu_parallel(host, np.array([0, len(host)], dtype=np.int64), cores)
    return {"value": round(len(host) / secs / 1e9, 4), "unit": "GB/s", "cores": cores,
            "kind": "paper's CPU design (threads over byte ranges + parallel merge)",
            "sample": f"first {len(host)} bytes of the {WORKLOAD} corpus ({total} tokens) "
                      f"in {secs:.2f} s"}


def device_copy_gbs(nbytes: int = 4 << 30, reps: int = 5) -> float:
    """Measured device-to-device copy rate (read + write bytes / time), the practical HBM
    ceiling beside the 8 TB/s specification."""
    import torch
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def plain_1mb(steps: int):
    """Workload "plain-1MB" (4 documents x 250,000 bytes, 5,000 words, Zipf 1.1, int32 counts):
    microseconds per wc_count call with the text resident (host wall clock per call, which
    includes the call's size readback), and the device time of the whole call (HIP events)."""
    import torch
    from paper_2206_05269_amd import synth, wc
    c = synth.generate("plain-1MB")
    t, o = c.text.to("cuda:0"), c.offsets.to("cuda:0")
    plan = wc.count_plan(t.numel(), o.numel() - 1, count_bytes=4)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda:0")
    for _ in range(5):
        r = wc.count(t, o, count_bytes=4, workspace=ws)
    if r.as_dict() != c.expected_table():
        log("MISMATCH plain-1MB")
        sys.exit(1)
    n = max(50, steps * 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        wc.count(t, o, count_bytes=4, workspace=ws)
    dt = (time.perf_counter() - t0) / n
    dev = []
    for _ in range(20):
        r = wc.count(t, o, count_bytes=4, workspace=ws, debug_flags=wc.WC_DEBUG_TIME)
        dev.append(r.res.total_ms)
    dev_ms = sorted(dev)[len(dev) // 2]
    B = t.numel()
    res = {"workload": "plain-1MB", "bytes": B, "tokens": c.n_tokens, "words": r.n_entries,
           "us_per_call": round(dt * 1e6, 1), "GBps": round(B / dt / 1e9, 2),
           "device_us": round(dev_ms * 1e3, 1), "device_GBps": round(B / (dev_ms * 1e-3) / 1e9, 2)}
    log(f"plain-1MB: {res['us_per_call']} us per call, device {res['device_us']} us")
    return res


def corpora_top50(steps: int):
    """Workload "corpora-4x2000" (4 corpora x 2,000 documents, ~80 MB, 50,000 shared words,
    200 words x5 per corpus): the four count tables and the top-50 distinctive words per corpus.
    Times per call (host wall clock, text resident); checked against the generator."""
    import torch
    from paper_2206_05269_amd import synth, wc
    cs = synth.generate("corpora-4x2000", device="cuda:0")
    torch.cuda.synchronize()
    B = sum(c.text.numel() for c in cs)
    tabs = [wc.count(c.text, c.offsets, count_bytes=4) for c in cs]
    for c, t in zip(cs, tabs):
        if t.total_tokens != c.n_tokens or t.n_entries != int((c.expected > 0).sum()):
            log("MISMATCH corpora-4x2000")
            sys.exit(1)
    wc.topk_ratio(tabs, 50)
    n = max(5, steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        tabs = [wc.count(c.text, c.offsets, count_bytes=4) for c in cs]
    t_count = (time.perf_counter() - t0) / n
    t0 = time.perf_counter()
    for _ in range(n):
        tk = wc.topk_ratio(tabs, 50)
    t_topk = (time.perf_counter() - t0) / n
    boosted = [set(int(x) for x in c.extra["boosted"]) for c in cs]
    vocab = {bytes(cs[0].vocab[k, :cs[0].vocab_lens[k]]): k for k in range(len(cs[0].vocab_lens))}
    planted = [sum(1 for w in tk.words[i] if vocab.get(w, -1) in boosted[i]) for i in range(len(cs))]
    res = {"workload": "corpora-4x2000", "bytes": B, "tokens": sum(c.n_tokens for c in cs),
           "count_ms": round(t_count * 1e3, 3), "count_GBps": round(B / t_count / 1e9, 2),
           "topk_ms": round(t_topk * 1e3, 3), "k": 50, "vocab": int(tk.vocab_size),
           "planted_in_top50": planted}
    log(f"corpora-4x2000: counts {res['count_ms']} ms, top-50 {res['topk_ms']} ms, "
        f"planted words in the top 50: {planted}")
    return res


def dense_vs_merge(steps: int):
    """Section 3.3's reduce as the paper did it (a zero-padded words x documents matrix summed
    by a row-sum kernel, wc_merge_dense) beside the hash merge (wc_merge), both on the
    per-document table of one corpus of "corpora-4x2000" (2,000 documents, ~20 MB)."""
    import torch
    from paper_2206_05269_amd import synth, wc
    c = synth.generate("corpora-4x2000", device="cuda:0")[0]
    per = wc.count(c.text, c.offsets, per_doc=True, count_bytes=4)
    a = wc.merge([per], count_bytes=8)
    d = wc.merge_dense(per, count_bytes=8)
    if a.n_entries != d.n_entries or a.total_tokens != c.n_tokens:
        log("MISMATCH dense reduce")
        sys.exit(1)
    n = max(5, steps)
    t_m, t_d, k_d, k_m = [], [], [], []
    for _ in range(n):
        t0 = time.perf_counter()
        r = wc.merge([per], count_bytes=8, debug_flags=wc.WC_DEBUG_TIME)
        t_m.append(time.perf_counter() - t0)
        k_m.append(r.res.kernel_ms)
        t0 = time.perf_counter()
        r = wc.merge_dense(per, count_bytes=8, debug_flags=wc.WC_DEBUG_TIME)
        t_d.append(time.perf_counter() - t0)
        k_d.append(r.res.kernel_ms)
    V, D = d.n_entries, int(per.res.n_docs)
    res = {"workload": "corpora-4x2000 corpus 0", "docs": D, "doc_word_pairs": per.n_entries,
           "words": V, "matrix_bytes": V * D * 4,
           "merge_ms": round(sorted(t_m)[n // 2] * 1e3, 3),
           "merge_insert_kernel_ms": round(sorted(k_m)[n // 2], 4),
           "dense_ms": round(sorted(t_d)[n // 2] * 1e3, 3),
           "rowsum_kernel_ms": round(sorted(k_d)[n // 2], 4),
           "rowsum_GBps": round(V * D * 4 / (sorted(k_d)[n // 2] * 1e-3) / 1e9, 1),
           "paper_v100_reduce_kernel_us": 4.29}
    log(f"dense reduce: {res}")
    return res


def pinned_end_to_end(corpus, plan_kw, steps: int = 3, piece_bytes: int = 512 << 20):
    """Config-3 text from pinned host memory, GB/s of text: the copy alone; one copy of the
    whole 8 GiB, then the count; and wc_count_host, which copies 512 MiB pieces on a second
    stream while the pieces before are counted."""
    import torch
    from paper_2206_05269_amd import wc
    B = corpus.numel()
    host = torch.empty(B, dtype=torch.uint8, pin_memory=True)
    host.copy_(corpus)
    dev = torch.empty_like(corpus)
    off = torch.tensor([0, B], dtype=torch.int64, device="cuda:0")
    dev.copy_(host, non_blocking=True)
    wc.count(dev, off, **plan_kw)
    torch.cuda.synchronize()
    t_copy, t_all = [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        dev.copy_(host, non_blocking=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        wc.count(dev, off, **plan_kw)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_copy.append(t1 - t0)
        t_all.append(t2 - t0)
    t_pipe = []
    kw = {k: v for k, v in plan_kw.items() if k in ("count_bytes", "table_slots")}
    r = wc.count_host(host, piece_bytes=piece_bytes, d_text=dev, **kw)
    n_words = r.n_entries
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = wc.count_host(host, piece_bytes=piece_bytes, d_text=dev, **kw)
        torch.cuda.synchronize()
        t_pipe.append(time.perf_counter() - t0)
    del host, dev, r
    tc, ta, tp = min(t_copy), min(t_all), min(t_pipe)
    return {"h2d_GBps": round(B / tc / 1e9, 2),
            "copy_then_count_GBps": round(B / ta / 1e9, 2), "copy_then_count_ms": round(ta * 1e3, 2),
            "pipelined_GBps": round(B / tp / 1e9, 2), "pipelined_ms": round(tp * 1e3, 2),
            "piece_bytes": piece_bytes, "words": n_words}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the 8 GiB corpus")
    ap.add_argument("--cpu-sample-mb", type=int, default=1536)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-fold", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the plain-1MB and corpora legs")
    ap.add_argument("--no-pinned", action="store_true")
    ap.add_argument("--requests", type=int, default=10_000)
    ap.add_argument("--plain-docs", type=int, default=2000)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device once (calibrates HBM counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        x = torch.ones(args.copy_probe << 20, dtype=torch.uint8, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        log(f"copied {x.numel()} bytes")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the counter has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2206_05269_amd import synth, wc

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = synth.WORKLOADS[WORKLOAD]
    t0 = time.perf_counter()
    log(f"generating {WORKLOAD} (scale {args.scale}) on {dev}")
    c = synth.generate(WORKLOAD, device=dev, scale=args.scale,
                       progress=lambda done, total: None)
    torch.cuda.synchronize()
    B = c.text.numel()
    log(f"generated {B} bytes, {c.n_tokens} tokens in {time.perf_counter() - t0:.1f} s")

    slots = w.table_slots
    plan = wc.count_plan(B, 1, count_bytes=w.count_bytes, table_slots=slots)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    kw = dict(count_bytes=w.count_bytes, table_slots=slots, workspace=ws, regrow=False,
              debug_flags=wc.WC_DEBUG_TIME)

    for i in range(args.warmup):
        r = wc.count(c.text, c.offsets, **kw)
        log(f"warmup {i}: {r.res.total_ms:.3f} ms (count kernel {r.res.kernel_ms:.3f} ms)")
    # correctness guard: totals must match the generator
    r = wc.count(c.text, c.offsets, **kw)
    n_words = int((c.expected > 0).sum())
    if r.total_tokens != c.n_tokens or r.n_entries != n_words:
        log(f"MISMATCH tokens {r.total_tokens} vs {c.n_tokens}, words {r.n_entries} vs {n_words}")
        sys.exit(1)

    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = wc.count(c.text, c.offsets, **kw)
        kernel_ms.append(r.res.kernel_ms)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt * 1e3 / args.steps
    gbs = B / (dt / args.steps) / 1e9
    k_avg = sum(kernel_ms) / len(kernel_ms)
    D = r.n_entries
    # dominant kernel: pass 1 of the two-pass count (global_map_kernel), timed with HIP events
    # on the call's stream; its algorithmic traffic is the text, read once
    alg_bytes = B
    achieved = alg_bytes / (k_avg * 1e-3) / 1e9
    log(f"step {ms_step:.3f} ms, {gbs:.1f} GB/s; pass 1 avg {k_avg:.3f} ms "
        f"({achieved:.1f} GB/s algorithmic)")

    out = {
        "metric": "word-count GB/s of text (fraction of HBM peak)",
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (seeded Zipf text generated on the GPU)",
        "config": {"workload": WORKLOAD, "bytes": B, "tokens": c.n_tokens, "words": D,
                   "vocab": w.vocab, "zipf_s": w.zipf_s, "max_word_len": w.max_len,
                   "table_slots": slots, "count_bytes": w.count_bytes},
        "tokens_per_s": round(c.n_tokens / (dt / args.steps), 1),
        "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(), "kernel": "global_map_kernel",
                     "kernel_ms": round(k_avg, 4), "algorithmic_bytes": alg_bytes},
    }
    if not args.no_cpu:
        sample = min(B, args.cpu_sample_mb << 20)
        log(f"timing the oracle on {sample} bytes")
        out["cpu_baseline"] = cpu_baseline(c.text, sample)
        log(f"timing the paper's threaded CPU design on {sample} bytes")
        out["cpu_parallel"] = cpu_parallel_baseline(c.text, sample)
        log(f"parallel CPU: {out['cpu_parallel']['value']} GB/s on {out['cpu_parallel']['cores']} cores")
    if not args.no_pinned:
        kw2 = dict(count_bytes=w.count_bytes, table_slots=slots, workspace=ws, regrow=False)
        out["pinned_input"] = pinned_end_to_end(c.text, kw2)
        log(f"pinned input: {out['pinned_input']}")
    del c, ws, r
    torch.cuda.empty_cache()
    copy = device_copy_gbs()
    out["device_copy_GBps"] = round(copy, 1)
    out["roofline"]["frac_of_measured_copy"] = round(achieved / copy, 4)
    log(f"device copy {copy:.1f} GB/s")
    if not args.no_small:
        out["plain_1mb"] = plain_1mb(args.steps)
        out["corpora"] = corpora_top50(args.steps)
        out["dense_reduce"] = dense_vs_merge(args.steps)
    torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = batched_docs_per_s(args.steps, args.warmup, args.plain_docs)
    if not args.no_serving:
        out["serving"] = serving(args.requests)
    if not args.no_fold:
        out["fold_sum"] = fold_sums(args.steps)
    print(json.dumps(out), flush=True)


def fold_sums(steps: int):
    """Section 4.2's float map-reduce at the paper's largest n (10^8): sum of sqrt(i) and the
    alternating harmonic sum, binary64, no input in memory. Time per call from HIP events on
    the call's stream; the paper's own times (V100, its Section 4.2 tables) are context only."""
    import math
    import torch
    from paper_2206_05269_amd import wc
    n = 10 ** 8
    res = {"n": n, "dtype": "f64"}
    paper_ms = {wc.WC_FOLD_SQRT: 73.372, wc.WC_FOLD_ALT_HARMONIC: 65.323}
    for kind, name in ((wc.WC_FOLD_SQRT, "sqrt"), (wc.WC_FOLD_ALT_HARMONIC, "alt_harmonic")):
        f = wc.FoldSum(kind, n)
        for _ in range(2):
            f.run(n)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            out = f.run(n)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        v = float(out.cpu().item())
        if kind == wc.WC_FOLD_ALT_HARMONIC:
            check = abs(v - math.log(2) - (-1) ** (n + 1) / (2 * n)) < 1e-11
        else:
            check = abs(v / (2 / 3 * n ** 1.5 + 0.5 * n ** 0.5 - 0.2078862249773546) - 1) < 1e-13
        if not check:
            log(f"MISMATCH fold {name}: {v}")
            sys.exit(1)
        res[name] = {"ms": round(ms, 4), "terms_per_s": round(n / (ms * 1e-3), 1), "sum": v,
                     "paper_v100_ms": paper_ms[kind]}
        log(f"fold {name}: n = {n} in {ms:.3f} ms ({n / ms / 1e6:.2f} Gterms/s), sum {v!r}")
    return res


def serving(n_requests: int):
    """Workload "serving": n_requests requests of lognormal size (median 256 KiB, sigma 2,
    clipped to 1 KiB..64 MiB) cut from Zipf(1.05) text over a 500,000-word vocabulary, to a
    server with a 1 GiB device budget and 8 worker streams. Two input modes: the text in pinned
    host memory, read in place (PCIe transfer included), and device-resident text. Capacity =
    all requests queued at once; latency = completion - submission under Poisson arrivals at 70%
    of that capacity; plain = one upload and wc_count per request, one after another."""
    import numpy as np
    import torch
    from paper_2206_05269_amd import synth, wc
    w = synth.WORKLOADS["serving"]
    rng = np.random.default_rng(w.seed + 31)
    sizes = synth.lognormal_sizes(n_requests, *w.lognormal, seed=w.seed + 7919)
    total = int(sizes.sum())
    log(f"generating {total} bytes of serving text on the GPU ({n_requests} requests)")
    vocab, vlens = synth.make_vocab(w.vocab, w.max_len, w.seed)
    c = synth.gen_stream(total, vocab, vlens, synth.zipf_probs(w.vocab, w.zipf_s), w.seed + 1,
                         "cuda:0")
    dev_text = c.text
    del c
    torch.cuda.synchronize()
    log("generated; copying to pinned host memory in pieces of whole requests")
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    # pinned host copies in buffers of about 1 GiB, each holding whole requests
    host_of = [None] * n_requests
    i = 0
    while i < n_requests:
        j, acc = i, 0
        while j < n_requests and (j == i or acc + int(sizes[j]) <= (1 << 30)):
            acc += int(sizes[j])
            j += 1
        a = int(starts[i])
        buf = torch.empty(acc, dtype=torch.uint8, pin_memory=True)
        buf.copy_(dev_text[a:a + acc])
        for r in range(i, j):
            host_of[r] = (buf, int(starts[r]) - a)
        i = j
    torch.cuda.synchronize()
    log(f"pinned copies done ({len({id(b) for b, _ in host_of})} buffers)")
    budget = 1 << 30
    STREAMS = 8  # worker threads x HIP streams; more workers overlap per-request host waits

    def run(src, rate, in_place, m=n_requests):
        """Submit m requests (Poisson gaps at `rate`, or all at once); a second thread waits
        for each in submission order, reads its times and releases it, so resident tables do
        not accumulate in the budget."""
        import queue
        import threading
        srv = wc.Server(mem_budget=budget, max_streams=STREAMS)
        q = queue.Queue()
        times, errors = [], []

        def releaser():
            while True:
                i = q.get()
                if i is None:
                    return
                try:
                    srv.wait(i)
                    times.append(srv.times(i))
                    srv.release(i)
                except Exception as e:  # reported by the main thread
                    errors.append(e)

        th = threading.Thread(target=releaser)
        th.start()
        gaps = rng.exponential(1.0 / rate, size=m) if rate else np.zeros(m)
        next_t = time.perf_counter()
        try:
            for r, g in zip(range(m), gaps):
                next_t += g
                d = next_t - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                q.put(srv.submit(src(r), count_bytes=8, in_place=in_place))
        finally:
            q.put(None)
            th.join()
        if errors:
            raise errors[0]
        lat = np.array([b - a for a, _, b in times])
        span = max(b for _, _, b in times) - min(a for a, _, _ in times)
        launches = srv.launches()
        srv.close()
        return lat, span, launches

    res = {"workload": "serving", "requests": n_requests, "bytes": total,
           "budget_bytes": budget, "streams": STREAMS}
    def host_src(r):
        buf, o = host_of[r]
        return buf[o:o + int(sizes[r])]

    def dev_src(r):
        a = int(starts[r])
        return dev_text[a:a + int(sizes[r])]

    for mode, src, in_place in (("pinned_host", host_src, True), ("device", dev_src, False)):
        run(src, 0, in_place, m=max(1, n_requests // 8))  # warm-up on the first eighth
        lat0, span0, _ = run(src, 0, in_place)
        cap = n_requests / span0
        rate = 0.7 * cap
        lat, span, launches = run(src, rate, in_place)
        res[mode] = {"capacity_req_per_s": round(cap, 1),
                     "capacity_GBps": round(total / span0 / 1e9, 2),
                     "offered_req_per_s": round(rate, 1),
                     "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                     "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                     "served_req_per_s": round(n_requests / span, 1),
                     "aggregate_GBps": round(total / span / 1e9, 3), "launches": int(launches)}
        log(f"serving {mode}: {res[mode]}")
    # plain: one upload (from the same pinned memory) and one wc_count per request
    t0 = time.perf_counter()
    for r in range(n_requests):
        t = host_src(r).to("cuda:0", non_blocking=True)
        wc.count(t, count_bytes=8)
    torch.cuda.synchronize()
    res["plain_req_per_s"] = round(n_requests / (time.perf_counter() - t0), 1)
    log(f"serving plain {res['plain_req_per_s']} req/s")
    del host_of, dev_text
    torch.cuda.empty_cache()
    return res


def batched_docs_per_s(steps: int, warmup: int, plain_docs: int):
    """Workload "batched-100k": 100,000 documents (lognormal sizes, median 16 KiB, clipped to
    200 B..1 MiB; 200,000-word vocabulary, Zipf 1.1), one table per document. Batched = one
    captured graph replay per corpus; plain = one wc_count call per document."""
    import torch
    from paper_2206_05269_amd import synth, wc
    name = "batched-100k"
    log(f"generating {name} on the GPU")
    c = synth.generate(name, device="cuda:0")
    torch.cuda.synchronize()
    n_docs = c.offsets.numel() - 1
    B = c.text.numel()
    # the autotuner's choice, timed on a calibration slice of the first 5,000 documents
    cal = 5000
    off_h = c.offsets[:cal + 1].cpu()
    cal_text = c.text[:int(off_h[-1])].contiguous()
    t0 = time.perf_counter()
    tu = wc.autotune(cal_text, c.offsets[:cal + 1].contiguous(), per_doc=True, count_bytes=4,
                     use_cache=False)
    t_tune = time.perf_counter() - t0
    log(f"autotune: chunk {tu.chunk_bytes} lds {tu.lds_entries} load {tu.lds_load_pct}% "
        f"direct {tu.direct_kib} KiB in {t_tune:.1f} s")
    b = wc.Batch(max_docs=n_docs, max_bytes=B, count_bytes=4, tuning=tu,
                 **wc.output_sizes(c.text, c.offsets, count_bytes=4))
    for _ in range(warmup):
        r = b.run(c.text, c.offsets)
    if r.total_tokens != c.n_tokens:
        log(f"MISMATCH batched tokens {r.total_tokens} vs {c.n_tokens}")
        sys.exit(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = b.run(c.text, c.offsets)
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t0) / steps
    entries = r.n_entries
    recounted = r.stats["docs_recounted"]
    b.close()
    # plain: one launch (wc_count, global table of that document) per document
    off = c.offsets.cpu().numpy()
    m = min(plain_docs, n_docs)
    plan = wc.count_plan(int(off[m] - off[0]), 1, count_bytes=4)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda:0")
    doc_off = [torch.tensor([0, int(off[d + 1] - off[d])], dtype=torch.int64, device="cuda:0")
               for d in range(m)]
    for d in range(min(20, m)):
        wc.count(c.text[off[d]:off[d + 1]], doc_off[d], count_bytes=4, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d in range(m):
        wc.count(c.text[off[d]:off[d + 1]], doc_off[d], count_bytes=4, workspace=ws)
    torch.cuda.synchronize()
    dt_p = (time.perf_counter() - t0) / m
    res = {"workload": name, "docs": n_docs, "bytes": B, "tokens": c.n_tokens,
           "doc_word_pairs": entries, "docs_recounted": recounted,
           "batched_docs_per_s": round(n_docs / dt_b, 1), "batched_ms": round(dt_b * 1e3, 3),
           "batched_GBps": round(B / dt_b / 1e9, 2),
           "plain_docs_per_s": round(1.0 / dt_p, 1), "plain_sample_docs": m,
           "speedup": round((n_docs / dt_b) * dt_p, 1),
           "tuning": {"chunk_bytes": tu.chunk_bytes, "lds_entries": tu.lds_entries,
                      "lds_load_pct": tu.lds_load_pct, "direct_kib": tu.direct_kib,
                      "calibration_docs": cal,
                      "tune_s": round(t_tune, 1)}}
    log(f"batched {res['batched_docs_per_s']} docs/s vs plain {res['plain_docs_per_s']} docs/s")
    return res


if __name__ == "__main__":
    main()
