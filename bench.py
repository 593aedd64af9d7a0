"""Benchmark of the all-pairs similarity self-join on one MI355X.

One step = one apss_join_device call on the resident index: candidate
generation, bounds, verification, rescoring, pair compaction, sort and
unpack into device output buffers.  Inputs (the index) and outputs stay in
HBM.  Prints one JSON line.

After the join, the serving workload (unless --no-serve): a resident index
of 2,000,000 vectors (m = 1,000,000, nnz/vector lognormal mean 100 in
5..2000, Zipf s = 1.0) built at t = 0.5, and requests of 1..4096 queries
(log-uniform) with per-request t uniform in [0.5, 0.95], arriving as a
Poisson process.  The saturation rate is measured first with a closed-loop
burst; open-loop runs at fractions of it give p50/p99 latency at stated
queries/s.

Workload (default): 1,000,000 vectors, 1,000,000 dimensions, nnz/vector
lognormal mean 120 (5..5000), dimension popularity Zipf s = 1.0, lognormal
weights normalised to unit L2 norm (float32), t = 0.7; seeded synthetic.
"""
import argparse
import json
import math
import os
import queue
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0  # dense bf16 MFMA
TUNING = os.path.join(ROOT, "paper_1402_3010_amd", "tuning", "gfx950.json")
WORKLOADS = {
    "c1": "n=2,000 m=10,000 nnz/vector uniform 10..60, Zipf s=1.0, t=0.5",
    "c2": "n=100,000 m=200,000 nnz/vector lognormal mean 80 (5..2000), Zipf s=1.1",
    "c3": "n=1,000,000 m=1,000,000 nnz/vector lognormal mean 120 (5..5000), Zipf s=1.0, t=0.7",
    "c4": "n=500,000 m=500,000 nnz/vector lognormal mean 150 (5..2000), Zipf s=0.9, t=0.8",
}


# The paper's own figures for context (Tables 2-4).  They are sequential CPU
# wall times of its OCaml 3.12 implementation with 32-bit fixed-point weights
# (Section 7.2), on its two small text datasets (radikal: 6,883 vectors,
# 1,072,472 non-zeros; 20-newsgroups: 20,001 vectors, 2,984,809 non-zeros)
# and, in Table 4, on the five problem instances.  The hardware of Tables 2
# and 3 is not stated; Table 4 ran on the AMD Opteron 6172 (48-core nodes)
# cluster of Section 7.4.  No time unit is printed (presumably seconds).
# None of these is the metric measured here: the paper reports no GPU
# numbers, no candidate-pair rates and no serving latency.
PAPER_FIGURES = {
    "implementation": "OCaml 3.12, sequential, 32-bit fixed-point weights (Section 7.2)",
    "units": "unstated (presumably seconds)",
    "table2_radikal": {
        "hardware": "not stated", "t": [0.2, 0.3, 0.4],
        "times": {"all-pairs-0-array": [24.57, 24.44, 24.74], "all-pairs-1": [87.10, 79.05, 71.73],
                  "all-pairs-1-array": [73.02, 69.54, 64.40], "all-pairs-1-remscore": [180.55, 181.79, 182.02],
                  "all-pairs-1-upperbound": [200.96, 171.42, 145.90], "all-pairs-1-minsize": [89.57, 80.52, 72.21],
                  "all-pairs-2": [198.92, 165.64, 138.98], "all-pairs-bruteforce": [183.06, 183.32, 183.28]}},
    "table3_20newsgroups": {
        "hardware": "not stated", "t": [0.4, 0.5, 0.6],
        "times": {"all-pairs-0-array": [480.0, 495.4, 478.0], "all-pairs-1": [1169.0, 1035.6, 882.9],
                  "all-pairs-1-array": [883.8, 837.0, 757.5], "all-pairs-1-remscore": [3502.0, 3499.9, 3497.7],
                  "all-pairs-2": [1733.8, 1450.0, 1190.2], "all-pairs-bruteforce": [1866.3, 1867.2, 1871.5]}},
    "table4_problem_instances": {
        "hardware": "AMD Opteron 6172 cluster nodes, one core (Section 7.4)", "algorithm": "all-pairs-0-array",
        "rows": [{"dataset": "radikal", "t": 0.2, "time": 15.5, "matches": 16810},
                 {"dataset": "20-newsgroups", "t": 0.4, "time": 317.3, "matches": 64396},
                 {"dataset": "wikipedia", "t": 0.9, "time": 54424.0, "matches": 747999},
                 {"dataset": "facebook", "t": 0.99, "time": 10777.8, "matches": 819196},
                 {"dataset": "virginia-tech", "t": 0.99, "time": 10426.2, "matches": 13447874}]},
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(V, t, budget_s: float):
    """The CPU oracle (all-pairs-0-array, double) on the last rows of the same
    corpus, each matched against every earlier row; sized to ~budget_s.

    Each oracle call first builds the full inverted index (a fixed cost), so
    the row count is scaled from one probe whose time includes that cost.
    """
    import oracle
    n = V.n

    def run(rows):
        t0 = time.perf_counter()
        r = oracle.join_plain(V, t, n - rows, n)
        return r, time.perf_counter() - t0

    # one probe; scaling its time (which includes the fixed cost) can only
    # over-estimate the per-row cost, so the sample stays within the budget
    probe = min(n, 256)
    _, dp = run(probe)
    log("cpu baseline: probe of %d rows took %.2f s" % (probe, dp))
    rows = int(min(n, max(probe, probe * budget_s / max(dp, 1e-3))))
    r, dt = run(rows)
    log("cpu baseline: %d rows took %.2f s" % (rows, dt))
    return {
        "value": r.candidates / dt,
        "unit": "candidate pairs scored/s",
        "cores": oracle.num_threads(),
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": "rows %d..%d of the same corpus, each against all earlier rows: %d candidate pairs, "
                  "%d matches in %.1f s (includes building the full inverted index)"
                  % (n - rows, n - 1, r.candidates, len(r), dt),
        "matches_per_s": len(r) / dt,
        "posting_visits_per_s": r.visits / dt,
    }


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("join.hip", "join.h", "apss_internal.h"):
        with open(os.path.join(ROOT, "paper_1402_3010_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(config, t, n):
    """HBM bytes per k_join launch from the committed counter summary, if it
    was taken on this workload and on the kernel source as it is now."""
    path = os.path.join(ROOT, "profiles", "k_join_%s_traffic.json" % config)
    if n is not None or not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash() or abs(rec.get("t", -1) - float(t)) > 1e-6:
        return None
    return rec["traffic_bytes"]


def measured_counters(config, t, n):
    """Issue and LDS figures of the k_join dispatch from the committed counter
    summary, if it was taken on this workload at full size and on the kernel
    source as it is now."""
    path = os.path.join(ROOT, "profiles", "k_join_%s_counters.json" % config)
    if n is not None or not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash() or abs(rec.get("t", -1) - float(t)) > 1e-6:
        return None
    return rec


def percentile(x, q):
    x = sorted(x)
    if not x:
        return None
    k = min(len(x) - 1, max(0, int(math.ceil(q / 100.0 * len(x))) - 1))
    return x[k]


class ServeDriver:
    """Client side of the serving benchmark: submits prepared requests at
    given arrival times (retrying while the server answers APSS_EBUSY) and
    collects results on a second thread.  Latency of a request = time from
    its arrival to its result being ready in the server (admission wait
    included)."""

    def __init__(self, apss, srv):
        self.apss = apss
        self.srv = srv

    def run(self, reqs, arrivals):
        q = queue.Queue()
        out = []
        errors = []

        def poller():
            while True:
                item = q.get()
                if item is None:
                    return
                rid, k, wait_ms = item
                try:
                    i, j, s, info = self.srv.poll(rid)
                except Exception as e:  # keep draining; reported below
                    errors.append(e)
                    continue
                out.append((k, wait_ms + info["latency_ms"], info, len(i)))

        th = threading.Thread(target=poller)
        th.start()
        t0 = time.perf_counter()
        busy = 0
        for k, (Q, tq) in enumerate(reqs):
            at = t0 + arrivals[k]
            d = at - time.perf_counter()
            if d > 0:
                time.sleep(d)
            while True:
                rid = self.srv.try_submit(Q, t_per_row=tq)
                if rid is not None:
                    break
                busy += 1
                time.sleep(0.0005)
            q.put((rid, k, 1000.0 * (time.perf_counter() - at)))
        q.put(None)
        th.join()
        elapsed = time.perf_counter() - t0
        if errors:
            raise errors[0]
        return out, elapsed, busy


def screen_bench(args):
    """c4: the plain join and the screened join (bf16 MFMA head screen over the
    4,096 densest dimensions + sparse pass) on the same corpus and GPU; the
    outputs must be identical."""
    import numpy as np
    import torch

    import paper_1402_3010_amd as apss
    from synth.corpus import CONFIGS, make_corpus, spec_for

    spec = spec_for("c4", n=args.screen_n)
    V = make_corpus(spec)
    t = np.float32(CONFIGS["c4"]["t"][0])
    log("screen corpus c4: n=%d nnz=%d t=%.2f" % (V.n, V.nnz, t))
    dev = (V.n, V.m, torch.from_numpy(V.row_ptr).cuda(), torch.from_numpy(V.col).cuda(),
           torch.from_numpy(V.val).cuda())
    res = {}
    outs = {}
    for mode, sd in (("plain", 0), ("screened", args.screen_dims)):
        ix = apss.Index.build(dev, t, screen_dims=sd)
        torch.cuda.synchronize()
        res_tune = ix.autotune(t, budget_ms=30000.0, cache=TUNING)
        log("%s tuning: %s" % (mode, res_tune))
        i0, _, _ = ix.join(t)
        cap = len(i0) + 1024
        oi = torch.empty(cap, dtype=torch.int32, device="cuda")
        oj = torch.empty(cap, dtype=torch.int32, device="cuda")
        osim = torch.empty(cap, dtype=torch.float32, device="cuda")
        ix.join_device(t, oi, oj, osim)  # warm-up
        torch.cuda.synchronize()
        ms = []
        for _ in range(args.screen_steps):
            t0 = time.perf_counter()
            cnt = ix.join_device(t, oi, oj, osim)
            torch.cuda.synchronize()
            ms.append(1000.0 * (time.perf_counter() - t0))
        st = ix.stats()
        outs[mode] = (oi[:cnt].cpu().numpy(), oj[:cnt].cpu().numpy(), osim[:cnt].cpu().numpy())
        res[mode] = {"ms": float(np.median(ms)), "matches": cnt, "stats": st, "tuning": res_tune}
        log("%s join: %.1f ms, %d pairs" % (mode, res[mode]["ms"], cnt))
        ix.close()
        del oi, oj, osim
    a, b = outs["plain"], outs["screened"]
    identical = (len(a[0]) == len(b[0]) and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
                 and np.array_equal(a[2].view(np.uint32), b[2].view(np.uint32)))
    st = res["screened"]["stats"]
    flops = 2.0 * st["screen_tiles"] * 128 * 128 * st["screen_ld"]
    tflops = flops / (st["ms_screen"] / 1000.0) / 1e12 if st["ms_screen"] > 0 else 0.0
    return {
        "workload": "c4: n=%d m=%d nnz/vector lognormal mean 150 (5..2000), Zipf s=0.9, t=%.1f; head = %d densest "
                    "dimensions as bf16" % (V.n, V.m, float(t), args.screen_dims),
        "plain_ms": res["plain"]["ms"], "screened_ms": res["screened"]["ms"],
        "plain_tuning": res["plain"]["tuning"], "screened_tuning": res["screened"]["tuning"],
        "speedup": res["plain"]["ms"] / res["screened"]["ms"], "identical_output": bool(identical),
        "matches": res["screened"]["matches"],
        "plain_posting_visits": res["plain"]["stats"]["posting_visits"],
        "sparse_pass_posting_visits": st["posting_visits"], "sparse_pass_ms": st["ms_candidates"],
        "sparse_pass_candidates": st["candidates"], "sparse_pass_survivors": st["bound_survivors"],
        "sparse_pass_verified": st["verified"], "plain_candidates": res["plain"]["stats"]["candidates"],
        "plain_survivors": res["plain"]["stats"]["bound_survivors"], "plain_ms_kernel": res["plain"]["stats"]["ms_candidates"],
        "screen_rows": st["screen_rows"], "screen_tiles": st["screen_tiles"],
        "screen_candidates": st["screen_candidates"], "screen_ms": st["ms_screen"],
        "mfma_roofline": {"bound": "mfma", "achieved": tflops, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                          "frac": tflops / PEAK_BF16_TFLOPS, "kernel": "k_screen_mfma", "flops": flops},
    }


VARIANTS = (("partial indexing (all-pairs-1 + bounds)", {}),
            ("all-pairs-0-array (index_all)", {"index_all": True}),
            ("local pruning, 2 parts", {"local_parts": 2}),
            ("local pruning, 4 parts", {"local_parts": 4}),
            ("remscore", {"remscore": True}))


def variants_bench(args):
    """The algorithm variants on the same corpora and geometry (tile variant 1,
    16,384-row ranges): the default partial-indexing join; all-pairs-0-array,
    which indexes every component (the paper's ablation of partial indexing);
    local pruning over 2 and 4 rank ranges (Lemma 1); remscore.  Every variant
    returns the same pairs; reported are the join kernel's time and counters."""
    import numpy as np
    import torch

    import paper_1402_3010_amd as apss
    from synth.corpus import make_corpus, spec_for

    out = []
    # C2 at full size; C3 on its first 300,000 rows (same distributions),
    # where local pruning's exact rescoring of every local survivor still
    # finishes in seconds
    for name, ts, n in (("c2", (0.5, 0.7, 0.9), args.variants_n), ("c3", (0.7,), args.variants_n or 300000)):
        V = make_corpus(spec_for(name, n=n))
        dev = (V.n, V.m, torch.from_numpy(V.row_ptr).cuda(), torch.from_numpy(V.col).cuda(),
               torch.from_numpy(V.val).cuda())
        for t in ts:
            t = np.float32(t)
            base = None
            for label, kw in VARIANTS:
                ix = apss.Index.build(dev, t, variant=1, range_rows=16384, **kw)
                try:
                    # the first join sizes the pair buffers (a join whose pairs
                    # overflow them runs its kernel again); the second is timed
                    ix.join(t)
                    i, _, _ = ix.join(t)
                    cnt = len(i)
                    st = ix.stats()
                finally:
                    ix.close()
                if base is None:
                    base = cnt
                rec = {"workload": "%s n=%d t=%.1f" % (name, V.n, float(t)), "variant": label,
                       "kernel_ms": st["ms_candidates"], "join_ms": st["ms_total"],
                       "posting_visits": st["posting_visits"], "candidates": st["candidates"],
                       "bound_survivors": st["bound_survivors"], "matches": cnt, "same_pairs_count": cnt == base}
                out.append(rec)
                log("variant %s t=%.1f %-40s kernel %8.1f ms  visits %.3e  candidates %.3e  survivors %.3e  matches %d"
                    % (name, float(t), label, rec["kernel_ms"], rec["posting_visits"], rec["candidates"],
                       rec["bound_survivors"], cnt))
        del dev, V
    return out


def serve_bench(args):
    import numpy as np
    import torch

    import paper_1402_3010_amd as apss
    from synth.corpus import make_corpus, make_queries, spec_for

    spec = spec_for("c5", n=args.serve_n)
    t0 = time.perf_counter()
    V = make_corpus(spec)
    log("serve corpus c5: n=%d nnz=%d (%.1f s)" % (V.n, V.nnz, time.perf_counter() - t0))
    rp = torch.from_numpy(V.row_ptr).cuda()
    col = torch.from_numpy(V.col).cuda()
    val = torch.from_numpy(V.val).cuda()
    t_build = np.float32(0.5)
    ix = apss.Index.build((V.n, V.m, rp, col, val), t_build)
    torch.cuda.synchronize()
    del rp, col, val
    log("serve index built: %s" % ix.sizes())

    rng = np.random.default_rng(2005)

    def requests(pool, k):
        out, pos = [], 0
        for _ in range(k):
            nq = int(min(4096, max(1, math.floor(math.exp(rng.uniform(0.0, math.log(4097.0)))))))
            rows = (np.arange(pos, pos + nq) % pool.n)
            pos = (pos + nq) % pool.n
            t = np.full(nq, rng.uniform(0.5, 0.95), np.float32)
            out.append((pool.take_rows(rows), t))
        return out

    pool = make_queries(V, 32768, spec, seed=2005)
    pool_fresh = make_queries(V, 32768, spec, seed=3005, frac_copies=0.0)
    srv = apss.Server(ix, slots=args.serve_slots, max_batch_queries=args.serve_max_batch,
                      split_queries=args.serve_split)
    drv = ServeDriver(apss, srv)
    # warm-up, then saturation: all requests arrive at once
    drv.run(requests(pool, 8), [0.0] * 8)
    burst = requests(pool, args.serve_requests)
    res, el, busy = drv.run(burst, [0.0] * len(burst))
    nq_burst = sum(Q.n for Q, _ in burst)
    sat_rps = len(burst) / el
    sat_qps = nq_burst / el
    log("serve saturation: %d requests, %d queries in %.2f s: %.1f req/s, %.0f queries/s"
        % (len(burst), nq_burst, el, sat_rps, sat_qps))
    curve = []
    # open-loop runs at fractions of the saturation rate, then at fixed
    # offered query rates (request rate = query rate / mean request size)
    mean_nq = nq_burst / len(burst)
    points = [(frac, frac * sat_rps) for frac in args.serve_load]
    points += [(None, qps / mean_nq) for qps in args.serve_qps]
    for frac, rate in points:
        n_req = max(40, int(rate * args.serve_seconds))
        reqs = requests(pool, n_req)
        arr = np.cumsum(rng.exponential(1.0 / rate, size=n_req)).tolist()
        st0 = srv.stats()
        res, el, busy = drv.run(reqs, arr)
        st1 = srv.stats()
        lat = [r[1] for r in res]
        nq = sum(Q.n for Q, _ in reqs)
        small = [r[1] for r in res if reqs[r[0]][0].n <= 256]
        large = [r[1] for r in res if reqs[r[0]][0].n > 256]
        point = {"load": frac if frac is not None else rate * mean_nq / sat_qps, "rate_rps": rate,
                 "offered_qps": rate * mean_nq, "requests": n_req, "queries": nq,
                 "qps": nq / el, "rps": n_req / el, "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
                 "p99_ms_requests_le_256_queries": percentile(small, 99),
                 "p99_ms_requests_gt_256_queries": percentile(large, 99),
                 "mean_batch_requests": float(np.mean([r[2]["batch_requests"] for r in res])),
                 "batches": st1["batches"] - st0["batches"],
                 "overlapped_batches": st1["overlapped_batches"] - st0["overlapped_batches"],
                 "busy_retries": busy, "pairs": int(sum(r[3] for r in res))}
        curve.append(point)
        log("serve load %.2f: %.1f req/s offered, %.0f queries/s, p50 %.1f ms, p99 %.1f ms "
            "(requests of <= 256 queries: p99 %.1f ms)"
            % (point["load"], rate, point["qps"], point["p50_ms"], point["p99_ms"],
               point["p99_ms_requests_le_256_queries"] or 0.0))
    # the middle load once more on queries without corpus copies
    frac = args.serve_load[len(args.serve_load) // 2]
    rate = frac * sat_rps
    n_req = max(40, int(rate * args.serve_seconds))
    reqs = requests(pool_fresh, n_req)
    arr = np.cumsum(rng.exponential(1.0 / rate, size=n_req)).tolist()
    res, el, busy = drv.run(reqs, arr)
    lat = [r[1] for r in res]
    fresh = {"load": frac, "rate_rps": rate, "qps": sum(Q.n for Q, _ in reqs) / el,
             "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99), "pairs": int(sum(r[3] for r in res))}
    st = srv.stats()
    srv.close()
    ix.close()
    mid = curve[len(args.serve_load) // 2]
    return {
        "workload": "c5: resident index of %d vectors, m=%d, nnz/vector lognormal mean 100 (5..2000), Zipf s=1.0, "
                    "t_build=0.5; requests of 1..4096 queries (log-uniform), query nnz lognormal mean 100, "
                    "10%% perturbed corpus copies, per-request t ~ U[0.5, 0.95], Poisson arrivals" % (V.n, V.m),
        "slots": args.serve_slots,
        "split_queries": args.serve_split,
        "max_batch_queries": args.serve_max_batch,
        "qps": mid["qps"], "p50_ms": mid["p50_ms"], "p99_ms": mid["p99_ms"], "at_load": mid["load"],
        "saturation_qps": sat_qps, "saturation_rps": sat_rps,
        "curve": curve,
        "at_fixed_qps": [p for p in curve[len(args.serve_load):]],
        "no_copies": fresh,
        "peak_running_batches": st["peak_running"], "overlapped_batches": st["overlapped_batches"],
        "regrows": st["regrows"], "failed": st["failed"],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--t", type=float, default=None)
    ap.add_argument("--n", type=int, default=None, help="fewer rows (same distributions), for quick checks")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving workload")
    ap.add_argument("--no-screen", action="store_true", help="skip the screened-join comparison")
    ap.add_argument("--screen-only", action="store_true")
    ap.add_argument("--screen-n", type=int, default=None)
    ap.add_argument("--screen-dims", type=int, default=4096)
    ap.add_argument("--screen-steps", type=int, default=3)
    ap.add_argument("--no-variants", action="store_true", help="skip the algorithm-variant comparison")
    ap.add_argument("--variants-only", action="store_true")
    ap.add_argument("--variants-n", type=int, default=None, help="fewer rows for the variant comparison")
    ap.add_argument("--serve-only", action="store_true")
    ap.add_argument("--serve-n", type=int, default=None, help="fewer corpus rows for the serving workload")
    ap.add_argument("--serve-slots", type=int, default=2)
    ap.add_argument("--serve-max-batch", type=int, default=4096, help="queries merged into one batch at most")
    ap.add_argument("--serve-split", type=int, default=0,
                    help="queue requests of more rows as pieces of at most this many rows (0: whole requests)")
    ap.add_argument("--serve-requests", type=int, default=120, help="requests in the saturation burst")
    ap.add_argument("--serve-seconds", type=float, default=6.0, help="length of each open-loop run")
    ap.add_argument("--serve-qps", type=float, nargs="*", default=[180000.0],
                    help="also run at these offered query rates")
    ap.add_argument("--serve-load", type=float, nargs="+", default=[0.3, 0.6, 0.9],
                    help="offered load as fractions of the saturation request rate")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (3 times), to calibrate "
                         "the FETCH_SIZE / WRITE_SIZE counters against a known byte count")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n, "copies": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the join runs on a single MI355X; "
              "multi-GPU sharding is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1402_3010_amd as apss
    from synth.corpus import CONFIGS, make_corpus, spec_for

    apss.load()
    torch.cuda.set_device(0)
    if args.serve_only:
        print(json.dumps({"serve": serve_bench(args)}), flush=True)
        return
    if args.screen_only:
        print(json.dumps({"screen": screen_bench(args)}), flush=True)
        return
    if args.variants_only:
        print(json.dumps({"variants": variants_bench(args)}), flush=True)
        return
    t = np.float32(args.t if args.t is not None else CONFIGS[args.config]["t"][0])
    spec = spec_for(args.config, n=args.n)
    t0 = time.perf_counter()
    V = make_corpus(spec)
    log("corpus %s: n=%d nnz=%d (%.1f s)" % (args.config, V.n, V.nnz, time.perf_counter() - t0))
    rp = torch.from_numpy(V.row_ptr).cuda()
    col = torch.from_numpy(V.col).cuda()
    val = torch.from_numpy(V.val).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ix = apss.Index.build((V.n, V.m, rp, col, val), t)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    log("index built: %s (%.2f s)" % (ix.sizes(), build_s))
    del rp, col, val
    # tile variant and range width from the shipped tuning table (tuned here if absent)
    tune = ix.autotune(t, budget_ms=60000.0, cache=TUNING)
    log("tuning: %s" % tune)

    # size the outputs with a first call
    i0, j0, s0 = ix.join(t)
    cap = len(i0) + 1024
    del i0, j0, s0
    oi = torch.empty(cap, dtype=torch.int32, device="cuda")
    oj = torch.empty(cap, dtype=torch.int32, device="cuda")
    osim = torch.empty(cap, dtype=torch.float32, device="cuda")
    for w in range(args.warmup):
        ix.join_device(t, oi, oj, osim)
        log("warmup %d done" % w)
    torch.cuda.synchronize()
    kern_ms = []
    stats = None
    t0 = time.perf_counter()
    for k in range(args.steps):
        cnt = ix.join_device(t, oi, oj, osim)
        stats = ix.stats()
        kern_ms.append(stats["ms_candidates"])
        log("step %d: %d pairs, join %.1f ms, candidate kernel %.1f ms" % (k, cnt, stats["ms_total"],
                                                                           stats["ms_candidates"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1000.0 * elapsed / args.steps
    cand = stats["candidates"]
    value = cand / (ms_step / 1000.0)
    # algorithmic bytes of the candidate kernel: the 4-byte packed list entry
    # it streams per posting visit, 8 B per query component read, 12 B per
    # emitted pair.  (A convention that prices a visit at an unpacked posting
    # counts 8 B, an id and a float weight; that figure is reported beside it.)
    alg_bytes = 4.0 * stats["posting_visits"] + 8.0 * V.nnz + 12.0 * stats["matches"]
    alg_bytes_8b = alg_bytes + 4.0 * stats["posting_visits"]
    kms = sum(kern_ms) / len(kern_ms)
    achieved = alg_bytes / (kms / 1000.0) / 1e9
    traffic = measured_traffic(args.config, t, args.n)
    counters = measured_counters(args.config, t, args.n)
    out = {
        "metric": "candidate pairs scored/s and matches/s at 1M vectors t=0.7; serve p50/p99 latency",
        "value": value,
        "unit": "candidate pairs scored/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Zipf-popularity sparse corpus, seed %d)" % spec.seed,
        "config": {"workload": "%s: %s" % (args.config, WORKLOADS.get(args.config, "")) if args.n is None
                   else "%s with n=%d" % (args.config, V.n),
                   "n": V.n, "m": V.m, "nnz": V.nnz, "t": float(t), "parallelism": "1 GPU"},
        "matches_per_s": stats["matches"] / (ms_step / 1000.0),
        "matches": stats["matches"],
        "candidates": cand,
        "posting_visits": stats["posting_visits"],
        "bound_survivors": stats["bound_survivors"],
        "verified": stats["verified"],
        "band_rescored": stats["band"],
        "index_build_s": build_s,
        "tuning": tune,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic,
                     "frac_dram": (traffic / (kms / 1000.0) / 1e9 / PEAK_HBM_GBS) if traffic else None,
                     "frac_8b_per_visit": alg_bytes_8b / (kms / 1000.0) / 1e9 / PEAK_HBM_GBS,
                     "binding_unit": counters.get("binding_unit") if counters else None,
                     "issue": ({k: counters[k] for k in ("valu_issue_frac", "salu_issue_frac", "lds_bank_conflict_frac")
                                if k in counters} if counters else None),
                     "kernel": "k_join", "kernel_ms": kms, "algorithmic_bytes": alg_bytes,
                     "algorithmic_bytes_8b_per_visit": alg_bytes_8b,
                     "traffic_source": "profiles/k_join_%s_traffic.md" % args.config,
                     "counters_source": "profiles/k_join_%s_counters.md" % args.config},
        "paper_figures": PAPER_FIGURES,
    }
    ix.close()
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(V, t, args.cpu_budget)
    del V
    if not args.no_screen:
        out["screen"] = screen_bench(args)
    if not args.no_variants:
        out["variants"] = variants_bench(args)
    if not args.no_serve:
        sv = serve_bench(args)
        out["serve"] = sv
        out["serve_p50_ms"] = sv["p50_ms"]
        out["serve_p99_ms"] = sv["p99_ms"]
        out["serve_qps"] = sv["qps"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
