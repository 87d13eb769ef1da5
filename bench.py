"""Benchmark: weighted minwise hashes/s at k=500 on the histogram-shaped workload
(N=100000 rows, D=4096, each cell nonzero with probability 0.3, LogNormal(0,1) weights in Q8.8),
batched persistent launch (autotuned plan, hipGraph replay) vs plain one-launch-per-8192-rows,
on one GPU.

A step is one wmh_hash call over the whole batch (validation, shared position stream, walk),
with the rows already resident in HBM.  Prints one JSON line.  Beside the headline the line
carries the heavy-tail workload (batched vs plain, and the 10^4 x 10^4 all-pairs collision
counts), a row subset of the text-like workload on the component index, and the serving loop's
p50/p99 latency on the D = 2^20 corpus (skip them with --no-extras).
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_INT_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3
HBM_PEAK_GBS = 8000.0
PCIE_PEAK_GBS = 64.0  # PCIe 5.0 x16, per direction
OPS_PER_TEST = 2  # one lookup of x at the draw's component and one compare
OPS_PER_COMPARE = 2  # collision counting: one u16 equality and one accumulate per hash pair
KEY_BYTES = 8  # one component-index key
# HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by the same counters on
# a 1 GiB device-to-device copy (read x2.000, write x1.000).  Each figure is valid while its
# kernel and plan are the ones timed; the line carries null otherwise.  Keyed by wavefronts per
# workgroup (and, on the histogram, hash ids per tile) where the autotuner picks differently on
# different machines.
#   batched_kernel<unsigned short, 4, 4, true, false> (R = 4, K = 4), by (J, W), on the
#     histogram workload (N = 1e5): profiles/batched_and_ballot_kernels_histogram_k500.txt
#     (J = 256 stages every row block twice, so it reads the rows twice)
TRAFFIC_R4_HISTOGRAM = {(500, 8): 1.3025e9, (500, 16): 1.2889e9, (256, 8): 2.2311e9,
                        (256, 16): 2.1878e9}
#   ballot_kernel<unsigned short, true, false> (exact 16-bit rows), one hash group, by (J, W),
#     on the same workload (the autotuner picks it there on some boxes): the same profile
TRAFFIC_BALLOT_HISTOGRAM = {(500, 8): 1.2534e9, (500, 16): 1.2529e9, (256, 8): 2.2060e9}
#   ballot_kernel<unsigned short, true, true> (coarse codes), J = 500, one hash group, on the
#     heavy tail (depth 40704): profiles/ballot_kernel_heavy_tail_k500.txt
TRAFFIC_BALLOT_HEAVY_TAIL = {8: 13.7591e9 + 0.2114e9, 16: 13.8838e9 + 0.2115e9}
#   the row split on the heavy tail (auto: the coarse ballot walk over the walk rows, then
#     index_rows_kernel over the others), per call: the same profile
TRAFFIC_SPLIT_HEAVY_TAIL = {8: 5.0659e9, 16: 5.0617e9}
#   index_rows_kernel<false, 16>, counter claims, lists aligned to 128-byte lines, on the 1e6
#     text-like rows, by wavefronts per workgroup (the tuner picks 8 or 16 on different boxes):
#     profiles/index_rows_kernel_text_like_k1000.txt
TRAFFIC_INDEX_TEXT_LIKE = {8: 281.1099e9 + 2.0506e9, 16: 281.1544e9 + 2.0505e9}


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def alu_roofline(tests: int, kernel_ms: float, kernel: str, traffic=None, note=None) -> dict:
    """Integer-ALU roofline of a walk: 2 operations per membership test (Definition 1: a hash of
    value h is h tests) over the kernels' time."""
    achieved = OPS_PER_TEST * tests / (kernel_ms / 1e3) / 1e12
    out = {"bound": "alu", "achieved": achieved, "peak": PEAK_INT_TOPS, "unit": "TOP/s",
           "frac": achieved / PEAK_INT_TOPS, "traffic": traffic, "kernel": kernel,
           "kernel_ms": kernel_ms, "membership_tests": tests, "ops_per_test": OPS_PER_TEST}
    if note:
        out["note"] = note
    return out


def hbm_roofline(nbytes: float, kernel_ms: float, kernel: str, note=None) -> dict:
    achieved = nbytes / (kernel_ms / 1e3) / 1e9
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": kernel,
           "kernel_ms": kernel_ms, "algorithmic_bytes": nbytes}
    if note:
        out["note"] = note
    return out


def index_key_bytes(ds, k: int) -> tuple[float, dict]:
    """Algorithmic bytes of the component-index rows kernel on ds: the keys its evaluation
    order must read, in expectation (Theorem 2: Pr(h > T) = (1 - s)^T), plus the rows once and
    the signatures once.  Offset order reads every green key of a row's lists (65534 k s keys);
    step order reads the lists up to T1 (all k hashes <= T1 with probability 15/16), and again
    up to T2 when a hash is still open; the row takes the order the kernel's rule picks."""
    M = float(ds.m.astype(np.float64).sum())
    lengths = np.diff(ds.row_ptr.astype(np.int64))
    rows_of = np.repeat(np.arange(ds.n_rows), lengths)
    sx = np.bincount(rows_of, weights=ds.val.astype(np.float64), minlength=ds.n_rows)
    sm = np.bincount(rows_of, weights=np.where(ds.val > 0, ds.m[ds.col], 0).astype(np.float64),
                     minlength=ds.n_rows)
    live = sx > 0
    s = np.where(live, sx / M, 0.5)
    l1p = np.log1p(-np.minimum(s, 1 - 1e-16))
    t1 = np.ceil(np.log((1 / 16) / k) / l1p)
    t2 = np.ceil(np.log(1e-4 / k) / l1p)
    by_steps = live & (t2 < 65534) & (t2 * sm < 65534.0 * sx)
    p_open = 1.0 - (1.0 - np.power(1.0 - s, t1)) ** k
    step_keys = k * (np.minimum(t1, 65535) * sm / M + p_open * np.minimum(t2, 65535) * sm / M)
    offset_keys = k * 65534.0 * s
    keys = np.where(live, np.where(by_steps, step_keys, offset_keys), 0.0).sum()
    nbytes = KEY_BYTES * keys + 8.0 * ds.nnz + 8.0 * (ds.n_rows + 1) + 2.0 * ds.n_rows * k
    return nbytes, {"expected_keys": float(keys), "step_order_rows": int(by_steps.sum())}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rows", type=int, default=100_000)
    ap.add_argument("--plain-steps", type=int, default=None,
                    help="timed steps of the plain form (default: same as --steps, at most 5)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--rows-per-block", type=int, default=0)
    ap.add_argument("--hashes-per-tile", type=int, default=0)
    ap.add_argument("--stream-depth", type=int, default=0)
    ap.add_argument("--waves-per-block", type=int, default=0)
    ap.add_argument("--steps-per-lane", type=int, default=0)
    ap.add_argument("--hash-groups", type=int, default=0,
                    help="ballot walk: hash ids in this many groups (0: planner or autotuner)")
    ap.add_argument("--index-waves", type=int, default=0,
                    help="text-like leg: wavefronts per workgroup of the index rows kernel "
                         "(with 16 keys per trip and counter claims; 0: autotuned)")
    ap.add_argument("--values", type=int, default=0, choices=[0, 1, 2],
                    help="dense rows in LDS: 0 planner/autotuner, 1 the values, 2 coarse codes")
    ap.add_argument("--walk", type=int, default=0, choices=[0, 1, 2, 3],
                    help="batched walk: 0 planner/autotuner, 1 shared windows, 2 independent "
                         "rows, 3 ballot walk (one row per block)")
    ap.add_argument("--only", choices=["batched", "plain", "both"], default="both")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run device-to-device copies of BYTES (scales HBM counters)")
    ap.add_argument("--serve", action="store_true",
                    help="only run the serving workload (corpus of config 5, k=256)")
    ap.add_argument("--heavy-tail", action="store_true",
                    help="only run the heavy-tail workload (with --only batched: no plain "
                         "form, no collision counts)")
    ap.add_argument("--serve-requests", type=int, default=10_000,
                    help="timed open-loop requests per load level and run")
    ap.add_argument("--serve-warmup", type=int, default=500,
                    help="open-loop requests before each timed run (not counted)")
    ap.add_argument("--serve-corpus-rows", type=int, default=100_000)
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (planner default plan)")
    ap.add_argument("--text-like", action="store_true",
                    help="only run the text-like workload (component index)")
    ap.add_argument("--text-rows", type=int, default=1_000_000,
                    help="rows of the text-like workload generated for its line")
    ap.add_argument("--serve-max-rows", type=int, default=4096)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="requests/s the load levels are fractions of (0: the saturated rate "
                         "measured by the burst)")
    ap.add_argument("--serve-group-rows", type=int, default=0,
                    help="rows admitted together into one slot (0: the loop's 2048; 1: one "
                         "request per slot)")
    return ap.parse_args()


def serve_bench(args) -> dict:
    """Serving loop on the D = 2^20 corpus: saturated throughput from a closed burst, then
    open-loop Poisson arrivals at 0.5x and 0.8x of it, each level run twice with a warm-up;
    p50/p99/p999 latency from scheduled arrival to completion, and the requests' overlap on the
    device from HIP event timestamps."""
    import torch
    from paper_1602_08393_amd import serve, synth, wmh
    torch.cuda.set_device(0)
    t = time.perf_counter()
    corpus = synth.config5_corpus(n_rows=args.serve_corpus_rows)
    log(f"serve: corpus N={corpus.n_rows} D={corpus.D} nnz={corpus.nnz} "
        f"({time.perf_counter() - t:.1f}s)")
    k = corpus.k
    ctx = wmh.Context(0)
    ctx.set_bounds(corpus.m)
    out = {"workload": f"requests of 1..{args.serve_max_rows} consecutive rows (log-uniform "
                       f"sizes) of a {corpus.n_rows}-row corpus, D=2^20, tf weights Q16.16, k={k}",
           "slots": args.serve_slots, "group_rows": args.serve_group_rows or 2048,
           "request_buffers": "page-locked (wmh_host_alloc)"}

    def request_bytes(sizes, starts):
        rp = corpus.row_ptr.astype(np.int64)
        nnz = rp[starts + sizes] - rp[starts]
        h2d = 8 * (sizes + 1) + 8 * nnz
        return float(h2d.sum()), float((2 * k * sizes).sum())

    group_rows = args.serve_group_rows or 2048
    row_len = np.diff(corpus.row_ptr.astype(np.int64))
    # the most nonzeros a group of up to group_rows rows can hold
    group_nnz = int(np.sort(row_len)[::-1][:group_rows].sum())

    def reserve(srv, sizes, starts):
        # slot buffers sized up front for the largest request or group, so no admission
        # allocates
        rp = corpus.row_ptr.astype(np.int64)
        srv.reserve(max(int(sizes.max()), group_rows),
                    max(int((rp[starts + sizes] - rp[starts]).max()), group_nnz))

    # the component index is built when each loop starts, so no timed request waits for it
    with serve.Server(ctx, k, seed=0, slots=args.serve_slots, build_index=True,
                          group_rows=args.serve_group_rows) as srv:
        ring = serve.RangeRequests(srv, corpus, args.serve_max_rows)
        burst = min(500, len(ring.sig_buf))
        _, sizes, starts = synth.serving_ranges(burst, corpus.n_rows, qps=1.0, seed=3005,
                                                max_rows=args.serve_max_rows)
        reserve(srv, sizes, starts)
        reqs = [ring.make(int(a), int(n)) for a, n in zip(starts, sizes)]
        t0 = time.perf_counter()
        for r in reqs:
            srv.submit(r)
        srv.drain()
        for r in reqs:
            srv.wait(r.ticket)
        burst_s = time.perf_counter() - t0
        st = srv.stats()
        sat_qps = burst / burst_s
        h2d, d2h = request_bytes(sizes, starts)
        pcie = (h2d + d2h) / burst_s / 1e9
        out["saturated_qps"] = sat_qps
        out["saturated_hashes_per_s"] = float(sum(sizes)) * k / burst_s
        out["saturated_max_on_device"] = st["max_on_device"]
        out["saturated_max_computing"] = st["max_computing"]
        out["saturated_requests_per_load"] = st["completed"] / max(1, st["loads"])
        # the loop's bound: its requests live in host memory, so every row crosses PCIe once
        # and every signature once back
        out["roofline"] = {"bound": "pcie", "achieved": pcie, "peak": 2 * PCIE_PEAK_GBS,
                           "unit": "GB/s", "frac": pcie / (2 * PCIE_PEAK_GBS), "traffic": None,
                           "kernel": "whole loop (copies in and out, check, index rows kernel)",
                           "h2d_bytes": h2d, "d2h_bytes": d2h,
                           "note": "bytes of the burst's rows in and signatures out over its "
                                   "wall time, against PCIe 5.0 x16 both ways"}
        log(f"serve: burst of {burst} requests in {burst_s:.2f}s -> {sat_qps:.2f} req/s, "
            f"{pcie:.1f} GB/s over PCIe, on device together up to {st['max_on_device']}")
    del ring, reqs
    gc.collect()
    levels = []
    base_qps = args.serve_rate or sat_qps
    out["load_base_qps"] = base_qps
    for frac in (0.5, 0.8):
        qps = frac * base_qps
        runs = []
        for run in range(2):
            n_req = args.serve_requests + args.serve_warmup
            arrivals, sizes, starts = synth.serving_ranges(
                n_req, corpus.n_rows, qps=qps, seed=int(4005 + 100 * frac + 7 * run),
                max_rows=args.serve_max_rows)
            with serve.Server(ctx, k, seed=0, slots=args.serve_slots, build_index=True,
                          group_rows=args.serve_group_rows) as srv:
                reserve(srv, sizes, starts)
                ring = serve.RangeRequests(srv, corpus, args.serve_max_rows)
                w = args.serve_warmup
                serve.run_open_loop(srv, lambda i: ring.make(int(starts[i]), int(sizes[i])),
                                    arrivals[:w])
                srv.reset_stats()
                st = serve.run_open_loop(
                    srv, lambda i: ring.make(int(starts[w + i]), int(sizes[w + i])),
                    arrivals[w:] - arrivals[w])
                waits = ring.reused_waits
                # the ring's page-locked buffers are released here, outside any timed run
                del ring
                gc.collect()
            runs.append({"requests": st["completed"], "p50_ms": st["p50_ms"],
                         "p99_ms": st["p99_ms"], "p999_ms": st["p999_ms"],
                         "max_ms": st["max_ms"], "mean_ms": st["mean_ms"],
                         "hashes_per_s": st["hashes_per_s"], "max_queued": st["max_queued"],
                         "peak_bytes": st["peak_bytes"], "max_on_device": st["max_on_device"],
                         "max_computing": st["max_computing"], "overlap_s": st["overlap_s"],
                         "busy_s": st["busy_s"], "ring_waits": waits,
                         "requests_per_load": st["completed"] / max(1, st["loads"]),
                         "driver_late_p99_ms": st.get("driver_late_p99_ms"),
                         "driver_late_max_ms": st.get("driver_late_max_ms")})
            log(f"serve: load {frac} run {run}: {st['completed']} requests, p50 "
                f"{st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms p999 {st['p999_ms']:.2f} ms, "
                f"{st['hashes_per_s']:.3g} hashes/s, computing together up to "
                f"{st['max_computing']} ({st['overlap_s']:.2f} s with two or more), driver late "
                f"by at most {st.get('driver_late_max_ms', 0):.2f} ms")
        lv = {"load": frac, "qps": qps, "warmup_requests": args.serve_warmup, "runs": runs}
        for key in ("p50_ms", "p99_ms", "p999_ms"):
            vals = [r[key] for r in runs]
            lv[key] = float(np.mean(vals))
            lv[key + "_spread"] = [float(min(vals)), float(max(vals))]
        lv["requests"] = int(min(r["requests"] for r in runs))
        lv["hashes_per_s"] = float(np.mean([r["hashes_per_s"] for r in runs]))
        lv["max_computing"] = int(max(r["max_computing"] for r in runs))
        levels.append(lv)
    out["levels"] = levels
    ctx.close()
    return out


def copy_calibration(nbytes: int):
    """Three device-to-device copies of a known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "copies": 3}), flush=True)


def plan_args(args) -> dict:
    """Tile-plan options given on the command line (0: planner or autotuner)."""
    return dict(rows_per_block=args.rows_per_block, hashes_per_tile=args.hashes_per_tile,
                stream_depth=args.stream_depth, waves_per_block=args.waves_per_block,
                walk=args.walk, steps_per_lane=args.steps_per_lane,
                hash_groups=args.hash_groups, values=args.values)


def timed_steps(ctx, rows, k, sig, opts, steps, warmup, torch):
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        ctx.hash_into(rows, k, 0, sig, opts=opts)
    torch.cuda.synchronize()
    walk = []
    build = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.hash_into(rows, k, 0, sig, stream=stream.cuda_stream, opts=opts)
        if opts.profile:
            w, s = ctx.last_kernel_ms()
            walk.append(w)
            build.append(s)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return elapsed, walk, build


def lsh_bench(ctx, sig, torch, wmh) -> dict:
    """(K, L) banding index over the headline signatures, queried with 10000 of its rows."""
    K, L = 10, 50
    stream = torch.cuda.current_stream()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(stream)
    ix = ctx.lsh_index(sig, K, L, stream=stream.cuda_stream)
    e1.record(stream)
    q = sig[:10000].contiguous()
    out, cnt = ix.query(q, 64, stream=stream.cuda_stream)
    e2.record(stream)
    e2.synchronize()
    counts = cnt.cpu().numpy().view(np.uint32)
    rows_out = out.cpu().numpy().view(np.uint32)
    listed = [int(c) != 0xFFFFFFFF and q in rows_out[q, :min(int(c), 64)]
              for q, c in enumerate(counts)]
    ix.close()
    ok = counts[counts != 0xFFFFFFFF]
    return {"K": K, "L": L, "rows": int(sig.shape[0]), "queries": 10000,
            "build_ms": e0.elapsed_time(e1), "query_ms": e1.elapsed_time(e2),
            "queries_per_s": 10000 / (e1.elapsed_time(e2) / 1e3),
            "mean_candidates": float(ok.mean()) if len(ok) else None,
            "overflowed_queries": int((counts == 0xFFFFFFFF).sum()),
            "queries_listing_themselves": int(sum(listed))}


def heavy_tail_bench(args, torch, synth, wmh) -> dict:
    """Heavy-tail workload (N=200000, D=16384, 1% of bounds inflated 100x, k=500): batched
    (autotuned) vs plain, then exact all-pairs collision counts of rows [0, 10^4) against
    [10^4, 2*10^4)."""
    t = time.perf_counter()
    ds = synth.config4()
    gen_s = time.perf_counter() - t
    log(f"heavy-tail: N={ds.n_rows} D={ds.D} nnz={ds.nnz} ({gen_s:.1f}s)")
    k = ds.k
    ctx = wmh.Context(0)
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, "cuda:0")
    out = {"workload": "heavy-tail: N=200000, D=16384, nnz ~ U{20..2000}, weights U{1..2^24}, "
                       "1% of dims with one outlier row at 100*2^24, bounds = dataset max, "
                       "k=500, seed 0",
           "N": ds.n_rows, "D": ds.D, "k": k, "nnz": ds.nnz}
    if not args.no_tune and not any(plan_args(args).values()):
        out["autotune"] = ctx.tune(rows, k, 0, reps=1)
    sig_b = torch.empty((ds.n_rows, k), dtype=torch.int16, device="cuda:0")
    sig_p = torch.empty_like(sig_b)
    el_b, walk_b, _ = timed_steps(ctx, rows, k, sig_b,
                                  ctx.make_opts(mode="batched", profile=True, **plan_args(args)),
                                  3, 1, torch)
    out["batched_plan"] = ctx.last_plan()
    hashes = ds.n_rows * k
    tests = int(wmh.sig_to_numpy(sig_b).astype(np.int64).sum())
    out.update({"batched_hashes_per_s": hashes * 3 / el_b,
                "batched_ms_per_step": el_b / 3 * 1e3,
                "batched_walk_ms": float(np.mean(walk_b)),
                "mean_steps_per_hash": tests / hashes,
                "roofline": alu_roofline(
                    tests, float(np.mean(walk_b)), f"{out['batched_plan']['walk']} walk",
                    traffic=TRAFFIC_BALLOT_HEAVY_TAIL.get(out["batched_plan"]["waves_per_block"]) if (
                        out["batched_plan"]["walk"] == "ballot"
                        and out["batched_plan"]["values"] == "coarse"
                        and out["batched_plan"]["hashes_per_tile"] == 500
                        and out["batched_plan"]["hash_groups"] == 1 and ds.n_rows == 200_000)
                    else None)})
    bp = out["batched_plan"]
    if bp.get("values") == "coarse":
        # the same plan with the exact 32-bit values in LDS (and 8-byte stream entries)
        exact = {name: bp[name] for name in ("rows_per_block", "steps_per_lane", "waves_per_block",
                                             "hashes_per_tile", "walk", "hash_groups")}
        el_x, walk_x, _ = timed_steps(ctx, rows, k, sig_p,
                                      ctx.make_opts(mode="batched", profile=True, values="exact",
                                                    **exact), 3, 1, torch)
        out["exact_values"] = {"plan": ctx.last_plan(), "ms_per_step": el_x / 3 * 1e3,
                               "walk_ms": float(np.mean(walk_x)),
                               "coarse_walk_speedup": float(np.mean(walk_x) / np.mean(walk_b)),
                               "equals_coarse": bool(torch.equal(sig_p, sig_b))}
        log(f"heavy-tail: exact 32-bit rows {out['exact_values']['walk_ms']:.2f} ms walk against "
            f"{out['batched_walk_ms']:.2f} ms with coarse codes, equal "
            f"{out['exact_values']['equals_coarse']}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = oracle_on_head(ds, 4096, k, wmh.sig_to_numpy(sig_b[:4096]))
        log(f"heavy-tail: oracle {out['cpu_baseline']['value']:.3g} hashes/s on 4096 rows, "
            f"bit-exact {out['cpu_baseline']['bit_exact']}")
    # auto mode: the planner may split the rows between the batched walk and the index
    sig_a = torch.empty_like(sig_b)
    timed_steps(ctx, rows, k, sig_a, ctx.make_opts(mode="auto", profile=True), 1, 1, torch)
    el_a, walk_a, _ = timed_steps(ctx, rows, k, sig_a, ctx.make_opts(mode="auto", profile=True),
                                  3, 0, torch)
    ap = ctx.last_plan()
    profiled_split = (ap["mode"] == "split" and ap["walk"] == "ballot"
                      and ap["values"] == "coarse" and ap["hashes_per_tile"] == 500
                      and ds.n_rows == 200_000)
    out["auto"] = {"mode": ctx.last_mode(), "plan": ap,
                   "hashes_per_s": hashes * 3 / el_a, "ms_per_step": el_a / 3 * 1e3,
                   "kernels_ms": float(np.mean(walk_a)),
                   "equals_batched": bool(torch.equal(sig_a, sig_b)),
                   "roofline": alu_roofline(
                       tests, float(np.mean(walk_a)), "walk + index rows kernels",
                       traffic=TRAFFIC_SPLIT_HEAVY_TAIL.get(ap["waves_per_block"])
                       if profiled_split else None,
                       note="walk-equivalent tests: the index rows compute the same values "
                            "with fewer operations")}
    log(f"heavy-tail: auto ({out['auto']['mode']}) {out['auto']['ms_per_step']:.2f} ms/step, "
        f"equal {out['auto']['equals_batched']}")
    del sig_a
    if args.only == "batched":
        log(f"heavy-tail: batched {out['batched_ms_per_step']:.2f} ms/step")
        ctx.close()
        return out
    el_p, walk_p, _ = timed_steps(ctx, rows, k, sig_p, ctx.make_opts(mode="plain", profile=True),
                                  2, 1, torch)
    out.update({"plain_hashes_per_s": hashes * 2 / el_p,
                "plain_ms_per_step": el_p / 2 * 1e3,
                "batched_over_plain": (hashes * 3 / el_b) / (hashes * 2 / el_p),
                "batched_equals_plain": bool(torch.equal(sig_b, sig_p)),
                "plain_roofline": alu_roofline(tests, float(np.mean(walk_p)), "plain_kernel")})
    # the batched walk's kernels and tuned plan scheduled plainly (a launch per 8192 rows)
    el_s, walk_s, _ = timed_steps(ctx, rows, k, sig_p,
                                  ctx.make_opts(mode="plain_shared", profile=True,
                                                **plan_args(args)), 3, 1, torch)
    out.update({"plain_shared_hashes_per_s": hashes * 3 / el_s,
                "plain_shared_ms_per_step": el_s / 3 * 1e3,
                "batched_over_plain_shared": (hashes * 3 / el_b) / (hashes * 3 / el_s),
                "plain_shared_equals_batched": bool(torch.equal(sig_b, sig_p)),
                "plain_shared_roofline": alu_roofline(
                    tests, float(np.mean(walk_s)),
                    f"{out['batched_plan']['walk']} walk, one launch per 8192 rows")})
    log(f"heavy-tail: plain (shared per-step code) {out['plain_shared_ms_per_step']:.2f} ms/step, "
        f"equal {out['plain_shared_equals_batched']}")
    log(f"heavy-tail: batched {out['batched_ms_per_step']:.2f} ms/step, plain "
        f"{out['plain_ms_per_step']:.2f} ms/step, equal {out['batched_equals_plain']}")
    del sig_p
    # all-pairs collision counts
    A = sig_b[0:10000].contiguous()
    B = sig_b[10000:20000].contiguous()
    stream = torch.cuda.current_stream()
    counts = ctx.collisions(A, B, stream=stream.cuda_stream)
    times = []
    for _ in range(3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        counts = ctx.collisions(A, B, stream=stream.cuda_stream)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    rng = np.random.Generator(np.random.PCG64(77))
    a_idx = rng.integers(0, 10000, 2000)
    b_idx = rng.integers(0, 10000, 2000)
    An = wmh.sig_to_numpy(A)
    Bn = wmh.sig_to_numpy(B)
    Cn = counts.cpu().numpy().view(np.uint32)
    exact = bool(np.all((An[a_idx] == Bn[b_idx]).sum(axis=1) == Cn[a_idx, b_idx]))
    ms = float(np.median(times))
    cmp_ops = OPS_PER_COMPARE * 1e8 * k / (ms / 1e3) / 1e12
    out["collisions"] = {"pairs": 10000 * 10000, "k": k, "ms": ms,
                         "pairs_per_s": 1e8 / (ms / 1e3),
                         "compares_per_s": 1e8 * k / (ms / 1e3),
                         "sampled_pairs_exact": exact, "sampled_pairs": len(a_idx),
                         "roofline": {"bound": "alu", "achieved": cmp_ops, "peak": PEAK_INT_TOPS,
                                      "unit": "TOP/s", "frac": cmp_ops / PEAK_INT_TOPS,
                                      "traffic": None, "kernel": "collide_kernel",
                                      "kernel_ms": ms, "ops_per_compare": OPS_PER_COMPARE}}
    log(f"heavy-tail: all-pairs collisions {ms:.2f} ms, sample exact {exact}")
    # the same counts on b-bit packed signatures (lossless width)
    bits, top = ctx.sig_bits(sig_b, stream=stream.cuda_stream)
    packed, sat = ctx.pack(sig_b, bits, stream=stream.cuda_stream)
    PA, PB = packed[0:10000].contiguous(), packed[10000:20000].contiguous()
    pcounts = ctx.packed_collisions(PA, PB, k, bits, stream=stream.cuda_stream)
    ptimes = []
    for _ in range(3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        pcounts = ctx.packed_collisions(PA, PB, k, bits, stream=stream.cuda_stream)
        e1.record(stream)
        e1.synchronize()
        ptimes.append(e0.elapsed_time(e1))
    pms = float(np.median(ptimes))
    out["packed"] = {"bits": bits, "max_value": top, "saturated": sat,
                     "words_per_row": int(packed.shape[1]),
                     "bytes_per_row": int(packed.shape[1]) * 4, "u16_bytes_per_row": 2 * k,
                     "collisions_ms": pms, "speedup_over_u16": ms / pms,
                     "counts_equal_u16": bool(torch.equal(pcounts, counts))}
    log(f"heavy-tail: packed at {bits} bits: {packed.shape[1] * 4} B/row vs {2 * k}, "
        f"collisions {pms:.2f} ms, equal {out['packed']['counts_equal_u16']}")
    ctx.close()
    return out


def text_like_bench(args, torch, synth, wmh) -> dict:
    """Rows of the text-like workload (D=65536, tf weights, k=1000), where s is so small that
    the planner takes the component index; the first rows are checked against the plain walk
    on the GPU."""
    t = time.perf_counter()
    ds = synth.config3(n_rows=args.text_rows, block=20_000)
    gen_s = time.perf_counter() - t
    log(f"text-like: N={ds.n_rows} D={ds.D} nnz={ds.nnz} ({gen_s:.1f}s)")
    k = ds.k
    ctx = wmh.Context(0)
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, "cuda:0")
    sig = torch.empty((ds.n_rows, k), dtype=torch.int16, device="cuda:0")
    stream = torch.cuda.current_stream()
    opts = ctx.make_opts(mode="auto", profile=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.hash_into(rows, k, 0, sig, stream=stream.cuda_stream, opts=opts)
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - t0) * 1e3
    first_rows_ms, build_ms = ctx.last_kernel_ms()
    mode = ctx.last_mode()
    # the index rows kernel's plan, tuned on these rows (the index is already built) unless
    # given, then steady-state steps replaying it from a graph
    tune = None
    if args.index_waves:
        opts = ctx.make_opts(mode="auto", profile=True, waves_per_block=args.index_waves,
                             index_batch=16, index_claim="counter")
    elif not args.no_tune:
        tune = ctx.tune(rows, k, 0, reps=1)
        log(f"text-like: tuned {tune}")
    el, walk, _ = timed_steps(ctx, rows, k, sig, opts, 3, 1, torch)
    plan = ctx.last_plan()
    sig_np = wmh.sig_to_numpy(sig)
    head = ds.head(48)
    head_rows = wmh.upload_dataset(head, "cuda:0")
    walk_sig = torch.empty((head.n_rows, k), dtype=torch.int16, device="cuda:0")
    ctx.hash_into(head_rows, k, 0, walk_sig, stream=stream.cuda_stream,
                  opts=ctx.make_opts(mode="plain", profile=True))
    head_plain_ms = ctx.last_kernel_ms()[0]
    walk_sig = wmh.sig_to_numpy(walk_sig)
    hashes = ds.n_rows * k
    capped = float((sig_np == 65535).mean())
    out = {"workload": f"text-like: N={ds.n_rows} rows (bounds = max over these rows), D=65536, "
                       "nnz = clamp(Zipf(1.2), 10, 5000) draws, tf weights 1+ln(Zipf(1.5)) "
                       "Q16.16, k=1000, seed 0",
           "N": ds.n_rows, "D": ds.D, "k": k, "nnz": ds.nnz, "mode": mode,
           "hashes_per_s": hashes * 3 / el, "ms_per_step": el / 3 * 1e3,
           "cold_ms_per_step": cold_ms, "graph": True, "plan": plan, "autotune": tune,
           "rows_kernel_ms": float(np.mean(walk)), "index_build_ms": build_ms,
           "first_call_rows_kernel_ms": first_rows_ms,
           "walk_steps_equivalent": int(sig_np.sum(dtype=np.int64)),
           "capped_fraction": capped,
           "head_equals_plain_walk": bool(np.array_equal(sig_np[:48], walk_sig)),
           "head_plain_walk_ms": head_plain_ms,
           "head_plain_walk_rows": head.n_rows}
    key_bytes, key_info = index_key_bytes(ds, k)
    out["roofline"] = hbm_roofline(key_bytes, float(np.mean(walk)), "index_rows_kernel",
                                   note="expected keys of the rows' evaluation orders "
                                        "(Theorem 2), the rows and the signatures, once each")
    if plan["index_batch"] == 16 and plan["index_claim"] == 1 and ds.n_rows == 1_000_000:
        out["roofline"]["traffic"] = TRAFFIC_INDEX_TEXT_LIKE.get(plan["waves_per_block"])
    out["roofline"].update(key_info)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = oracle_on_head(ds, 48, k, sig_np[:48])
        log(f"text-like: oracle {out['cpu_baseline']['value']:.3g} hashes/s on 48 rows, "
            f"bit-exact {out['cpu_baseline']['bit_exact']}")
    log(f"text-like: {mode} {out['ms_per_step']:.2f} ms/step, index build {build_ms:.2f} ms, "
        f"head equals walk {out['head_equals_plain_walk']}")
    ctx.close()
    return out


def small_bench(torch, synth, wmh) -> dict:
    """The small plain workload (N=1000, D=1024, k=64): batched, plain and the batched kernels
    scheduled plainly, all checked against the oracle on every row."""
    import oracle
    ds = synth.config1()
    k = ds.k
    ctx = wmh.Context(0)
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, "cuda:0")
    want = oracle.hash_csr(ds.m, ds.row_ptr, ds.col, ds.val, k, seed=0)
    tests = int(want.astype(np.int64).sum())
    out = {"workload": "plain small: N=1000, D=1024, nnz ~ Poisson(100), weights U{1..65535}, "
                       "bounds = dataset max, k=64, seed 0",
           "N": ds.n_rows, "D": ds.D, "k": k, "nnz": ds.nnz, "membership_tests": tests}
    for mode in ("batched", "plain", "plain_shared"):
        sig = torch.empty((ds.n_rows, k), dtype=torch.int16, device="cuda:0")
        el, walk, _ = timed_steps(ctx, rows, k, sig, ctx.make_opts(mode=mode, profile=True),
                                  20, 3, torch)
        walk_ms = float(np.mean(walk))
        out[mode] = {"hashes_per_s": ds.n_rows * k * 20 / el, "ms_per_step": el / 20 * 1e3,
                     "walk_ms": walk_ms, "plan": ctx.last_plan(),
                     "equals_oracle": bool(np.array_equal(wmh.sig_to_numpy(sig), want)),
                     "roofline": alu_roofline(tests, walk_ms, f"{mode} walk")}
        log(f"small: {mode} {out[mode]['ms_per_step']:.3f} ms/step, equals oracle "
            f"{out[mode]['equals_oracle']}")
    out["batched_over_plain"] = out["batched"]["hashes_per_s"] / out["plain"]["hashes_per_s"]
    out["batched_over_plain_shared"] = (out["batched"]["hashes_per_s"] /
                                        out["plain_shared"]["hashes_per_s"])
    ctx.close()
    return out


def cpu_model() -> str:
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical CPUs visible"


def cpu_baseline(ds, k, target_s):
    import oracle
    threads = min(16, os.cpu_count() or 1)
    n = 64
    sample = ds.head(n)
    t0 = time.perf_counter()
    oracle.hash_csr(sample.m, sample.row_ptr, sample.col, sample.val, k, seed=0, threads=threads)
    dt = time.perf_counter() - t0
    n = int(min(ds.n_rows, max(n, n * target_s / max(dt, 1e-3))))
    n = max(threads, n - n % threads)
    sample = ds.head(n)
    t0 = time.perf_counter()
    sig, steps = oracle.hash_csr(sample.m, sample.row_ptr, sample.col, sample.val, k, seed=0,
                                 threads=threads, return_steps=True)
    dt = time.perf_counter() - t0
    # one thread on a tenth of the sample
    n1 = max(1, n // (10 * threads) * 1)
    one = ds.head(n1)
    t1 = time.perf_counter()
    oracle.hash_csr(one.m, one.row_ptr, one.col, one.val, k, seed=0, threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": n * k / dt, "unit": "hashes/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} rows of the workload, k={k} ({steps} membership tests, "
                      f"{dt:.1f} s, {steps / dt:.3g} tests/s)",
            "single_thread_value": n1 * k / dt1,
            "single_thread_sample": f"first {n1} rows, 1 thread, {dt1:.1f} s",
            "host": cpu_model()}, sig


def oracle_on_head(ds, n, k, gpu_sig_head):
    """The oracle timed on the first n rows (host threads as for the headline's baseline), and
    whether the GPU's signatures of those rows equal it."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    head = ds.head(n)
    t0 = time.perf_counter()
    sig, steps = oracle.hash_csr(head.m, head.row_ptr, head.col, head.val, k, seed=0,
                                 threads=threads, return_steps=True)
    dt = time.perf_counter() - t0
    return {"value": head.n_rows * k / dt, "unit": "hashes/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {head.n_rows} rows, k={k} ({steps} membership tests, {dt:.1f} s, "
                      f"{steps / dt:.3g} tests/s)",
            "bit_exact": bool(np.array_equal(sig, gpu_sig_head))}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the walk shards "
              "by rows, each GPU hashing its own rows against replicated bounds tables with no "
              "exchange step, so one GPU's figure is its share", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.serve:
        print(json.dumps({"serving": serve_bench(args)}), flush=True)
        return
    import torch
    from paper_1602_08393_amd import synth, wmh
    if args.heavy_tail:
        torch.cuda.set_device(0)
        print(json.dumps({"heavy_tail": heavy_tail_bench(args, torch, synth, wmh)}), flush=True)
        return
    if args.text_like:
        torch.cuda.set_device(0)
        print(json.dumps({"text_like": text_like_bench(args, torch, synth, wmh)}), flush=True)
        return

    if not os.path.exists(wmh.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    t = time.perf_counter()
    ds = synth.config2(n_rows=args.rows)
    k = ds.k
    log(f"generated {ds.name}: N={ds.n_rows} D={ds.D} nnz={ds.nnz} in {time.perf_counter() - t:.1f}s")
    ctx = wmh.Context(0)
    ctx.set_bounds(ds.m)
    rows = wmh.upload_dataset(ds, "cuda:0")
    sig = torch.empty((ds.n_rows, k), dtype=torch.int16, device="cuda:0")
    sig_plain = torch.empty_like(sig)
    M = int(ds.m.astype(np.uint64).sum())
    hashes = ds.n_rows * k

    plan = plan_args(args)
    result = {}
    tune = None
    if args.only in ("batched", "both") and not args.no_tune and not any(plan.values()):
        log("batched: autotuning the tile plan")
        tune = ctx.tune(rows, k, 0, reps=2)
        log(f"batched: tuned R={tune['rows_per_block']} J={tune['hashes_per_tile']} "
            f"W={tune['waves_per_block']}: {tune['best_ms']:.3f} ms vs default "
            f"{tune['default_ms']:.3f} ms over {tune['candidates']} plans")
    if args.only in ("batched", "both"):
        opts = ctx.make_opts(mode="batched", profile=True, **plan)
        log("batched: warmup + timed steps (hipGraph replay)")
        el, graph_ms, _ = timed_steps(ctx, rows, k, sig, opts, args.steps, args.warmup, torch)
        batched_plan = ctx.last_plan()
        # the same kernels launched directly, with events between them on the launch stream,
        # to time the walk kernel alone
        dopts = ctx.make_opts(mode="batched", profile=True, use_graph=False, **plan)
        _, walk, _ = timed_steps(ctx, rows, k, sig, dopts, max(3, min(args.steps, 5)), 1,
                                 torch)
        # the timed calls reuse the shared stream built by the first call; time one build with
        # another seed (into a scratch output)
        scratch = torch.empty_like(sig)
        ctx.hash_into(rows, k, 1, scratch, opts=dopts)
        torch.cuda.synchronize()
        build = [ctx.last_kernel_ms()[1]]
        del scratch
        result["batched"] = (el, walk, build, graph_ms)
        log(f"batched: {el / args.steps * 1e3:.3f} ms/step, graph {np.mean(graph_ms):.3f} ms, "
            f"walk kernel {np.mean(walk):.3f} ms, stream build {np.mean(build):.3f} ms")
    if args.only in ("plain", "both"):
        psteps = args.plain_steps or min(args.steps, 5)
        opts = ctx.make_opts(mode="plain", profile=True)
        log("plain: warmup + timed steps")
        el, walk, _ = timed_steps(ctx, rows, k, sig_plain, opts, psteps, 1, torch)
        result["plain"] = (el, walk, psteps)
        log(f"plain: {el / psteps * 1e3:.3f} ms/step, walk kernels {np.mean(walk):.3f} ms")
    if args.only == "both":
        # the batched walk's own kernels and plan, scheduled plainly: a launch per 8192 rows,
        # one workgroup per tile, no tile queue, no graph
        sig_ps = torch.empty_like(sig)
        opts = ctx.make_opts(mode="plain_shared", profile=True, **plan)
        log("plain (shared per-step code): warmup + timed steps")
        el, walk, _ = timed_steps(ctx, rows, k, sig_ps, opts, args.steps, 1, torch)
        result["plain_shared"] = (el, walk, args.steps, bool(torch.equal(sig_ps, sig)))
        del sig_ps
        log(f"plain (shared per-step code): {el / args.steps * 1e3:.3f} ms/step, walk kernels "
            f"{np.mean(walk):.3f} ms")

    main_key = "batched" if "batched" in result else "plain"
    # the walk kernel of the plan, and its HBM traffic when profiled for this workload
    walk_kernel, traffic = "plain_kernel", None
    if main_key == "batched":
        walk_kernel = {"shared": "batched_kernel", "ballot": "ballot_kernel",
                       "rows": "rows_kernel"}.get(batched_plan["walk"], "batched_kernel")
        full_size = ds.n_rows == 100_000 and k == 500
        jw = (batched_plan["hashes_per_tile"], batched_plan["waves_per_block"])
        if (full_size and batched_plan["walk"] == "shared" and batched_plan["rows_per_block"] == 4
                and batched_plan["steps_per_lane"] == 4):
            traffic = TRAFFIC_R4_HISTOGRAM.get(jw)
        if (full_size and batched_plan["walk"] == "ballot" and batched_plan["values"] == "exact"
                and batched_plan["hash_groups"] == 1):
            traffic = TRAFFIC_BALLOT_HISTOGRAM.get(jw)
    steps = args.steps if main_key == "batched" else result["plain"][2]
    el, walk, _ = result[main_key][:3]
    value = hashes * steps / el
    out_sig = sig if main_key == "batched" else sig_plain
    sig_np = wmh.sig_to_numpy(out_sig)
    tests = int(sig_np.astype(np.int64).sum())  # exact membership tests of one step
    walk_s = float(np.mean(walk)) / 1e3
    achieved = OPS_PER_TEST * tests / walk_s / 1e12
    line = {
        "metric": "weighted minwise hashes/sec at k=500 (batched vs plain, bit-exact)",
        "value": value,
        "unit": "hashes/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": el / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "histogram-shaped: N=100000 rows, D=4096, cell density 0.3, "
                               "LogNormal(0,1) weights in Q8.8, bounds = dataset max, k=500, "
                               "seed 0",
                   "N": ds.n_rows, "D": ds.D, "k": k, "nnz": ds.nnz, "M": M,
                   "mode": main_key},
        "roofline": alu_roofline(tests, walk_s * 1e3, walk_kernel, traffic=traffic),
        "mean_steps_per_hash": tests / hashes,
    }
    if "batched" in result and "plain" in result:
        pel, pwalk, psteps = result["plain"]
        plain_value = hashes * psteps / pel
        same = bool(torch.equal(sig, sig_plain))
        line["plain"] = {"value": plain_value, "ms_per_step": pel / psteps * 1e3,
                         "walk_ms": float(np.mean(pwalk)), "steps": psteps}
        line["batched_over_plain"] = value / plain_value
        line["batched_equals_plain"] = same
        line["plain"]["roofline"] = alu_roofline(tests, float(np.mean(pwalk)), "plain_kernel")
        if "plain_shared" in result:
            sel, swalk, ssteps, ssame = result["plain_shared"]
            sv = hashes * ssteps / sel
            line["plain_shared"] = {
                "value": sv, "ms_per_step": sel / ssteps * 1e3, "walk_ms": float(np.mean(swalk)),
                "steps": ssteps, "equals_batched": ssame,
                "form": "the batched walk's kernels, plan and shared stream; one launch per "
                        "8192 rows, one workgroup per tile, no tile queue, no graph",
                "roofline": alu_roofline(tests, float(np.mean(swalk)),
                                         f"{batched_plan['walk']} walk, one launch per 8192 rows")}
            line["batched_over_plain_shared"] = value / sv
        bel, bwalk, bbuild, bgraph = result["batched"]
        line["batched_detail"] = {"graph_ms": float(np.mean(bgraph)),
                                  "walk_ms": float(np.mean(bwalk)),
                                  "stream_build_ms": float(np.mean(bbuild)),
                                  "plan": batched_plan}
    if tune is not None:
        line["autotune"] = tune
    if "batched" in result and not args.no_extras:
        line["lsh"] = lsh_bench(ctx, sig, torch, wmh)
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on a sample")
        cb, want = cpu_baseline(ds, k, args.cpu_seconds)
        line["cpu_baseline"] = cb
        line["sample_bit_exact"] = bool(np.array_equal(sig_np[: want.shape[0]], want))
    ctx.close()
    if not args.no_extras and args.only == "both":
        del rows, sig, sig_plain
        torch.cuda.empty_cache()
        line["small"] = small_bench(torch, synth, wmh)
        torch.cuda.empty_cache()
        line["heavy_tail"] = heavy_tail_bench(args, torch, synth, wmh)
        torch.cuda.empty_cache()
        line["text_like"] = text_like_bench(args, torch, synth, wmh)
        torch.cuda.empty_cache()
        line["serving"] = serve_bench(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
