#!/usr/bin/env python3
"""Benchmark of the LCS library on one MI355X.

Workload (default): the batched related-pair workload -- 4096 DNA pairs,
|X| log-uniform in [256, 65536], Y = X mutated at a rate drawn from
U[5%, 30%] -- with lengths and canonical tracebacks, replayed as a HIP graph.
One step = one full pass (symbol remap, match masks, bit-parallel fill,
checkpoints, traceback) over the resident batch.

Prints ONE JSON line.  `value` is whole-job GCUPS (sum of m*n over the batch
per second, the timed passes enqueued back to back between two
synchronisations); `roofline` refers to the fill kernel, bound by integer VALU
issue, priced from the device's own compute-unit count and clock;
`cpu_baseline` is the CPU oracle timed on this host's cores on a bounded
sample of the same workload.  The same line carries the other workloads
(`workloads`: one 4096 x 4096 pair, the 262144-row related pair, 65536 short
protein pairs), the traceback in rounds (bounded history) on the long pair
and the batch, the batch end to end with host copies, and the request server
at offered loads set from its measured capacity.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# gfx950 integer-VALU roofline for the column recurrence: compute units x 64
# lanes x clock lane-instructions per second, 6 lane-instructions per 64
# cells.  The compute units and the peak clock come from the device.
LANES, OPS_PER_64 = 64, 6


def peak_tcups(cus: int, clock_mhz: float) -> float:
    return cus * LANES * clock_mhz * 1e6 * 64 / OPS_PER_64 / 1e12


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name: str):
    from paper_1306_4627_amd import inputs
    if name == "batch_related":
        ps = inputs.batch_related()
        return ps, "dna", True, {"workload": "batch_related", "pairs": 4096,
                                 "len_x": "log-uniform[256,65536]", "alphabet": "DNA",
                                 "mutation": "U[0.05,0.30] sub/ins/del", "traceback": True,
                                 "launch": "hipGraph, persistent"}
    if name == "batch_short":
        ps = inputs.batch_short()
        return ps, "protein", False, {"workload": "batch_short", "pairs": 65536,
                                      "len": "U{64..1024}", "alphabet": "protein(20)",
                                      "traceback": False, "launch": "hipGraph, persistent"}
    if name == "pair_dna_4096":
        p = inputs.pair_dna_4096()
        return [p], "dna", True, {"workload": "pair_dna_4096", "m": 4096, "n": 4096,
                                  "alphabet": "DNA", "traceback": True}
    if name == "pair_long_related":
        p = inputs.pair_long_related()
        return [p], "dna", True, {"workload": "pair_long_related", "m": int(p.x.size),
                                  "n": int(p.y.size), "alphabet": "DNA", "traceback": True}
    if name == "pair_long_related_lengths":
        p = inputs.pair_long_related()
        return [p], "dna", False, {"workload": "pair_long_related_lengths", "m": int(p.x.size),
                                   "n": int(p.y.size), "alphabet": "DNA", "traceback": False}
    raise SystemExit(f"unknown workload {name}")


def measured_traffic(workload: str, wpl: int, ckpt: int, lane_steps: int):
    """HBM bytes per fill launch from the committed rocprofv3 counter runs,
    or None when they were taken on a different kernel source, workload or
    plan (words per lane, checkpoint interval, lane-steps)."""
    import hashlib
    src = os.path.join(ROOT, "paper_1306_4627_amd", "csrc", "fill.hip")
    rec_file = os.path.join(ROOT, "profiles", "k_fill_batch_related_4096.md")
    try:
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        for line in open(rec_file):
            if line.startswith("traffic-record:"):
                rec = json.loads(line.split(":", 1)[1])
                if (rec["source_sha256_prefix"] == h and rec["workload"] == workload
                        and rec.get("words_per_lane") == wpl and rec.get("ckpt_interval") == ckpt
                        and rec.get("lane_steps") == lane_steps):
                    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


def host_info() -> dict:
    """Cores this process may run on, and the CPU model."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_model": model}


def _oracle_one(oracle, x, y, traceback: bool):
    if traceback:
        if (x.size + 1) * (y.size + 1) <= 2e8:
            oracle.lcs_traceback(x, y)
        else:
            oracle.lcs_traceback_ckpt(x, y, 512)
    else:
        oracle.lcs_length(x, y)


def cpu_baseline(pairs, traceback: bool, seconds: float, threads: int):
    """Time the oracle (built -O3 -march=native for this host) on a random
    sample of the workload's pairs spread over `threads` host threads: pairs
    are handed out in a seeded random order until `seconds` have passed
    (pairs the oracle needs more than that for alone are left out), then the
    ones started are finished; cells of the finished pairs over the time."""
    import oracle
    from concurrent.futures import FIRST_COMPLETED, wait
    g = np.random.default_rng(7)
    order = [int(k) for k in g.permutation(len(pairs))]
    per_pair_cap = seconds * (0.15e9 if traceback else 0.4e9)
    order = [k for k in order if pairs[k].cells <= per_pair_cap]
    done_cells, n_done, skipped = 0, 0, len(pairs) - len(order)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        running = {}
        it = iter(order)
        while True:
            while len(running) < threads and time.perf_counter() - t0 < seconds:
                k = next(it, None)
                if k is None:
                    break
                p = pairs[k]
                running[ex.submit(_oracle_one, oracle, p.x, p.y, traceback)] = p.cells
            if not running:
                break
            fin, _ = wait(list(running), return_when=FIRST_COMPLETED)
            for f in fin:
                f.result()
                done_cells += running.pop(f)
                n_done += 1
    dt = time.perf_counter() - t0
    return {"value": done_cells / dt / 1e9, "unit": "GCUPS", "cores": threads, "kind": "oracle",
            "sample": f"{n_done} pairs of the workload in seeded random order, {done_cells:.3e} cells, "
                      f"{'length+traceback' if traceback else 'length'}, {dt:.1f} s "
                      f"({skipped} pairs longer than the time bound left out)",
            **host_info()}


def cpu_single_thread(x, y, traceback: bool) -> dict:
    """The oracle on one pair, one thread (the plain DP is sequential)."""
    import oracle
    t0 = time.perf_counter()
    _oracle_one(oracle, x, y, traceback)
    dt = time.perf_counter() - t0
    return {"GCUPS": round(x.size * y.size / dt / 1e9, 4), "s": round(dt, 2), "threads": 1,
            "cells": int(x.size) * int(y.size)}


def _serve_once(lcs, ctx, reqs, warmup: int):
    """Submit every request at its arrival time, collect all; latency and
    throughput over the requests after the first `warmup`."""
    cells = float(sum(int(r.x.size) * int(r.y.size) for r in reqs[warmup:]))
    with lcs.Server(ctx, mem_budget_bytes=8 << 30) as srv:
        tickets = []
        t0 = time.perf_counter()
        t_meas = None
        for k, r in enumerate(reqs):
            while time.perf_counter() - t0 < r.arrival_s:
                pass
            if k == warmup:
                t_meas = time.perf_counter()
            tickets.append(srv.submit(r.x, r.y, r.alphabet, traceback=r.want_traceback))
        lat = []
        for t in tickets:
            srv.wait(t)
            lat.append(srv.result(t)[2])
        t_end = time.perf_counter()
        st = srv.stats()
    return np.array(lat[warmup:]) / 1e6, t_end - (t_meas or t0), cells, st


def serve_leg(lcs, ctx, rhos=(0.5, 0.8, 0.95), count: int = 2000, warmup: int = 200):
    """The request server under Poisson arrivals.  Capacity is measured
    first: a burst of requests all submitted at once, requests completed per
    second.  Then each offered rate is a fraction of that capacity, with
    `warmup` requests before the `count` that are measured; latency is the
    library's submit-to-completion time of each request."""
    from paper_1306_4627_amd import inputs
    burst = inputs.serve_stream(1e9, 1200, seed_offset=50)
    _, wall, _, _ = _serve_once(lcs, ctx, burst, 200)
    capacity = 1000 / wall
    log(f"serve capacity {capacity:.0f} requests/s")
    out = {"capacity_rps": round(capacity, 1), "warmup_requests": warmup, "rates": []}
    for k, rho in enumerate(rhos):
        rate = rho * capacity
        reqs = inputs.serve_stream(rate, count + warmup, seed_offset=51 + k)
        lat_ms, wall, cells, st = _serve_once(lcs, ctx, reqs, warmup)
        out["rates"].append({
            "rho": rho, "offered_rps": round(rate, 1), "requests": count,
            "achieved_rps": round(count / wall, 1),
            "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
            "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
            "GCUPS": round(cells / wall / 1e9, 2),
            "batches": st["batches"], "max_inflight": st["max_inflight"],
            "plan_ms_per_batch": round(st["plan_ns"] / max(st["batches"], 1) / 1e6, 3),
            "device_ms_per_batch": round(st["device_ns"] / max(st["batches"], 1) / 1e6, 3),
            "collect_ms_per_batch": round(st["collect_ns"] / max(st["batches"], 1) / 1e6, 3)})
        log(f"serve rho {rho}: {out['rates'][-1]}")
    return out


def batch_leg(lcs, ctx, pairs, alpha, traceback: bool, peak: float, steps: int, tuning=None,
              autotune: bool = True):
    """One resident batch: graph-replayed passes (whole pass), eager passes
    (fill kernels timed by HIP events), the plan, and for single pairs the
    fill's time per column step."""
    cells = float(sum(len(x) * len(y) for x, y in pairs))
    if tuning is None:
        tuning = {}
        if autotune:
            tuning, _ = lcs.autotune(ctx, pairs, alpha, traceback=traceback, graph=True)
    with lcs.Batch(ctx, pairs, alpha, traceback=traceback, graph=True, **tuning) as b:
        info = b.info()
        b.time()
        b.time()
        # passes enqueued back to back, one synchronisation on each side
        ctx.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            b.run()
        ctx.synchronize()
        pass_ms = (time.perf_counter() - t0) / steps * 1e3
        eager, fill = [], []
        for _ in range(max(3, steps // 2)):
            t, f = b.time(eager=True)
            eager.append(t)
            fill.append(f)
        try:
            mhz = b.clock_mhz()
        except lcs.LcsError:
            mhz = None
    fill_ms = float(np.median(fill))
    out = {"pass_ms": round(pass_ms, 4), "GCUPS": round(cells / pass_ms / 1e6, 2),
           "pass_frac": round(cells / pass_ms / 1e9 / peak, 4),
           "fill_ms": round(fill_ms, 4), "fill_TCUPS": round(cells / fill_ms / 1e9, 2),
           "fill_frac": round(cells / fill_ms / 1e9 / peak, 4),
           "eager_pass_ms": round(float(np.median(eager)), 4),
           "clock_mhz_measured": None if mhz is None else round(mhz, 1),
           "words_per_lane": info["words_per_lane"], "groups": info["groups"],
           "device_bytes": info["device_bytes"], "history_bytes": info["history_bytes"],
           "tb_rounds": info["tb_rounds"], "split_pairs": info["split_pairs"], "tuning": tuning}
    if len(pairs) == 1:
        steps_per_item = info["lane_steps"] / (info["groups"] * 64)
        out["fill_ns_per_step"] = round(fill_ms * 1e6 / steps_per_item, 2)
    return out


# Table-1 of the paper: (M, N) -> speedup on its four-processor system
PAPER_TABLE1_SPEEDUP = {(5000, 200): 3.22, (10000, 1500): 2.89}


def threshold_leg(lcs, ctx, pairs, alpha, reps: int = 5):
    """Section II's yes/no question (lengths only), graph-replayed threshold
    passes at three thresholds against the lengths-only pass of the same
    pairs, with the share of pairs whose answer came before their last
    column.  Two pair sets: the workload's own pairs, and a screening set --
    the same parents, every other child replaced by an unrelated random
    string of the same length (seeded)."""
    g = np.random.default_rng(13064627 + 61)
    symbols = np.frombuffer(lcs.DNA if alpha == "dna" else lcs.PROTEIN, dtype=np.uint8)
    screen = [(x, symbols[g.integers(0, symbols.size, len(y))] if k % 2 else y)
              for k, (x, y) in enumerate(pairs)]
    out = {}
    for name, ps in (("workload", pairs), ("screening", screen)):
        cells = float(sum(len(x) * len(y) for x, y in ps))
        with lcs.Batch(ctx, ps, alpha, graph=True) as lb:
            lb.time()
            base = float(np.median([lb.time()[0] for _ in range(reps)]))
        leg = {"lengths_only_ms": round(base, 4), "passes": []}
        with lcs.Batch(ctx, ps, alpha, graph=True, threshold=90.0) as tb:
            for pct in (80.0, 90.0, 95.0):
                tb.set_threshold(pct)
                tb.time()
                ms = float(np.median([tb.time()[0] for _ in range(reps)]))
                ok, lens = tb.decisions()
                leg["passes"].append({
                    "min_percent": pct, "ms": round(ms, 4),
                    "speedup_vs_lengths": round(base / ms, 2),
                    "pass_share": round(float(ok.mean()), 4),
                    "answered_early_share": round(float((lens == lcs.LCS_LENGTH_UNKNOWN).mean()), 4),
                    "effective_GCUPS": round(cells / (ms * 1e-3) / 1e9, 1)})
                log(f"threshold {name} {pct}%: {ms:.3f} ms vs lengths-only {base:.3f} ms")
        out[name] = leg
    return out


def striped_leg(lcs, ctx, cores: int):
    """The paper's row-striped OpenMP method on this host at Table-1 shapes
    and at 4096 x 4096, on 1, 4 and all threads, beside one GPU pass over the
    same single pair (length + traceback, inputs resident)."""
    from paper_1306_4627_amd import inputs
    from paper_1306_4627_amd.striped import striped_lcs
    g = inputs.rng(61)
    rows = []
    for m, n in ((5000, 200), (10000, 1500), (4096, 4096)):
        x = inputs.random_seq(g, m, inputs.DNA)
        y = inputs.random_seq(g, n, inputs.DNA)
        ms = {}
        for t in sorted({1, 4, cores}):
            ms[t] = min(striped_lcs(x, y, t, 64)[3] for _ in range(3)) * 1e3
        with lcs.Batch(ctx, [(x, y)], "dna", traceback=True, words_per_lane=1) as b:
            b.time(eager=True)
            gpu = min(b.time(eager=True)[0] for _ in range(3))
        rows.append({"m": m, "n": n, "cpu_ms": {str(k): round(v, 3) for k, v in ms.items()},
                     "speedup_4_threads": round(ms[1] / ms[4], 2),
                     "paper_speedup_4_processors": PAPER_TABLE1_SPEEDUP.get((m, n)),
                     "gpu_pass_ms": round(gpu, 3),
                     "gpu_over_best_cpu": round(min(ms.values()) / gpu, 1)})
        log(f"striped {m}x{n}: {rows[-1]}")
    return rows


def cpu_share() -> int:
    """Host threads this job may use: the cores it may run on, capped by the
    thread count the environment grants it (OMP_NUM_THREADS)."""
    n = len(os.sched_getaffinity(0))
    try:
        omp = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        omp = 0
    return max(1, min(n, omp) if omp > 0 else n)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch_related")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-pair leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU legs (oracle, striped method)")
    ap.add_argument("--no-serve", action="store_true", help="skip the request-server leg")
    ap.add_argument("--no-threshold", action="store_true", help="skip the threshold-pass leg")
    ap.add_argument("--no-schedule", action="store_true",
                    help="skip the traced fill pass (per-item schedule summary)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the other workloads, the rounds and the end-to-end legs")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-only", action="store_true",
                    help="only run the request-server leg and print its results")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target oracle time of the CPU baseline sample")
    ap.add_argument("--wpl", type=int, default=0)
    ap.add_argument("--ckpt", type=int, default=0)
    ap.add_argument("--tb-round-kib", type=int, default=0,
                    help="run the main workload's traceback in rounds of this many KiB")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default tuning instead of a timed search")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run one plain device-to-device copy of BYTES bytes (the "
                         "reference for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.ones(args.calibrate_copy, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": args.calibrate_copy}), flush=True)
        return 0
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU (its workload is one GPU's share; "
              "pairs are independent, so batches shard by pair); --gpus must be 1",
              file=sys.stderr)
        return 2

    if not args.no_cpu:
        # the oracle timed as a baseline is built for this host (same source)
        import oracle
        oracle.use_native_build()
    from paper_1306_4627_amd import inputs, lcs

    ctx = lcs.Context(0)
    dev = ctx.device_info()
    cus, spec_mhz = dev["compute_units"], dev["peak_clock_khz"] / 1000.0
    peak = peak_tcups(cus, spec_mhz)
    log(f"device: {cus} compute units, peak clock {spec_mhz:.0f} MHz -> roofline {peak:.1f} TCUPS")
    if args.serve_only:
        print(json.dumps({"serving": serve_leg(lcs, ctx, count=args.serve_requests,
                                               warmup=args.serve_warmup)}), flush=True)
        ctx.close()
        return 0
    ps, alpha, tb, config = make_workload(args.workload)
    pairs = [(p.x, p.y) for p in ps]
    cells = float(sum(p.cells for p in ps))
    log(f"workload {args.workload}: {len(pairs)} pairs, {cells:.3e} cells")
    tuning = {"words_per_lane": args.wpl, "ckpt_interval": args.ckpt}
    tune_s = None
    if not args.no_autotune and not args.wpl and not args.ckpt:
        t0 = time.perf_counter()
        tuning, tune_ms = lcs.autotune(ctx, pairs, alpha, traceback=tb, graph=True)
        tune_s = time.perf_counter() - t0
        log(f"autotune: {tuning} ({tune_ms:.3f} ms per pass, search {tune_s:.1f} s)")
    if args.tb_round_kib:
        tuning = dict(tuning, tb_round_kib=args.tb_round_kib)
    batch = lcs.Batch(ctx, pairs, alpha, traceback=tb, graph=True, **tuning)
    info = batch.info()
    log(f"plan: {info}")
    for _ in range(args.warmup):
        batch.time(eager=False)
    # the K passes (graph replays) enqueued back to back on the library's
    # stream, one synchronisation on each side of them
    ctx.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.run()
    ctx.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    value = cells * args.steps / wall / 1e9
    # each pass alone: graph replay, HIP events around it, synchronised
    total_ms = [batch.time(eager=False)[0] for _ in range(args.steps)]
    # the same pass with the kernels enqueued directly: HIP events on the
    # library's stream around the fill kernels give their duration
    fill_ms, eager_ms = [], []
    for _ in range(args.steps):
        t, f = batch.time(eager=True)
        eager_ms.append(t)
        fill_ms.append(f)
    fill_avg = float(np.mean(fill_ms))
    achieved = cells / (fill_avg * 1e-3) / 1e12
    # shader clock measured during the last eager fill (first wave's span)
    try:
        clock_mhz = batch.clock_mhz()
    except lcs.LcsError:
        clock_mhz = None
    log(f"step {ms_per_step:.3f} ms (graph events {np.mean(total_ms):.3f} ms, eager {np.mean(eager_ms):.3f} ms), "
        f"fill {fill_avg:.3f} ms")
    lens = batch.lengths()
    pass_tcups = value / 1e3
    at_clock = None if clock_mhz is None else peak * clock_mhz / spec_mhz

    out = {
        "metric": "LCS GCUPS batched vs plain per-pair on 1 MI355X; p50/p99 request latency",
        "value": round(value, 2), "unit": "GCUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": config,
        "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": round(peak, 1),
                     "unit": "TCUPS", "frac": round(achieved / peak, 4),
                     "traffic": measured_traffic(config["workload"], info["words_per_lane"],
                                                 info["ckpt_interval"], info["lane_steps"]),
                     "kernel": "k_fill", "fill_ms": round(fill_avg, 4),
                     "compute_units": cus, "peak_clock_mhz": round(spec_mhz, 1),
                     "clock_mhz_measured": None if clock_mhz is None else round(clock_mhz, 1),
                     "peak_at_measured_clock": None if at_clock is None else round(at_clock, 1),
                     "frac_at_measured_clock": None if at_clock is None
                     else round(achieved / at_clock, 4),
                     "pass_TCUPS": round(pass_tcups, 2), "pass_frac": round(pass_tcups / peak, 4),
                     "pass_frac_at_measured_clock": None if at_clock is None
                     else round(pass_tcups / at_clock, 4),
                     "target_frac": 0.5,
                     "eager_pass_ms": round(float(np.mean(eager_ms)), 4)},
        "plan": {k: info[k] for k in ("groups", "lanes", "lane_steps", "words_per_lane",
                                      "ckpt_interval", "classes", "device_bytes", "history_bytes",
                                      "tb_rounds", "split_pairs")},
        "tuning": {"chosen": tuning, "search_s": None if tune_s is None else round(tune_s, 2)},
    }
    if not args.no_plain and len(pairs) > 1:
        log("plain per-pair leg")
        with lcs.Batch(ctx, pairs, alpha, traceback=tb, plain=True) as pb:
            pb.time(eager=True)
            t_plain, f_plain = pb.time(eager=True)
            plain_l = pb.lengths()
        if not np.array_equal(plain_l, lens):
            log("plain and batched lengths differ!")
            out["plain_mismatch"] = True
        out["plain_per_pair"] = {"value": round(cells / (t_plain * 1e-3) / 1e9, 2), "unit": "GCUPS",
                                 "ms": round(t_plain, 3)}
        out["batched_over_plain"] = round(value / out["plain_per_pair"]["value"], 2)
    if not args.no_schedule:
        # one more eager pass of the same plan with per-item schedule records
        # (outside the timed runs above)
        log("fill schedule leg")
        from paper_1306_4627_amd import fill_schedule
        with lcs.Batch(ctx, pairs, alpha, traceback=tb, fill_trace=True, **tuning) as sb:
            sb.time(eager=True)
            _, f_tr = sb.time(eager=True)
            sm = fill_schedule.summarize(sb.fill_trace())
            same = np.array_equal(sb.lengths(), lens)
        out["fill_schedule"] = {"traced_fill_ms": round(f_tr, 4),
                                **{k: round(v, 4) if isinstance(v, float) else v
                                   for k, v in sm.items()}}
        if not same:
            log("traced and untraced lengths differ!")
            out["fill_schedule"]["lengths_mismatch"] = True
    batch.close()
    if not args.no_threshold:
        log("threshold-pass leg")
        out["threshold"] = threshold_leg(lcs, ctx, pairs, alpha)
    cores = cpu_share()
    if not args.no_workloads:
        wl = {}
        for name in ("pair_dna_4096", "pair_long_related", "batch_short"):
            if name == args.workload:
                continue
            log(f"workload leg {name}")
            wps, wal, wtb, wcfg = make_workload(name)
            wpairs = [(p.x, p.y) for p in wps]
            single = len(wpairs) == 1
            leg = batch_leg(lcs, ctx, wpairs, wal, wtb, peak, 5 if not single else 10,
                            autotune=not single)
            leg["cells"] = float(sum(p.cells for p in wps))
            leg["config"] = wcfg
            if single and not args.no_cpu:
                p0 = wps[0]
                if p0.x.size * p0.y.size <= 2e8:
                    leg["cpu_oracle_1_thread"] = cpu_single_thread(p0.x, p0.y, wtb)
                else:
                    # a bounded sample: the first 40000 symbols of X and Y
                    cs = cpu_single_thread(p0.x[:40000], p0.y[:40000], wtb)
                    cs["sample"] = "X[:40000] vs Y[:40000], length + traceback"
                    leg["cpu_oracle_1_thread"] = cs
                leg["gpu_over_cpu_1_thread"] = round(leg["GCUPS"] / leg["cpu_oracle_1_thread"]["GCUPS"], 1)
            log(f"{name}: {leg}")
            wl[name] = leg
        # the long pair's lengths-only pass: split at the middle column into
        # two half fills run side by side (the default for a lone long pair),
        # and whole
        p2 = inputs.pair_long_related()
        lw = {"config": {"workload": "pair_long_related", "m": int(p2.x.size), "n": int(p2.y.size),
                         "alphabet": "DNA", "traceback": False}}
        for key, hv in (("split", 0), ("whole", 1)):
            lw[key] = batch_leg(lcs, ctx, [(p2.x, p2.y)], "dna", False, peak, 10,
                                tuning={"words_per_lane": 1, "halves": hv})
        lw["cells"] = float(p2.x.size) * float(p2.y.size)
        lw["split_over_whole"] = round(lw["whole"]["pass_ms"] / lw["split"]["pass_ms"], 2)
        del p2
        log(f"pair_long_related lengths only: {lw}")
        wl["pair_long_related_lengths"] = lw
        out["workloads"] = wl
        # traceback in rounds (bounded history) on the long pair and the batch
        log("rounds legs")
        rl = {}
        p2 = inputs.pair_long_related()
        rl["pair_long_related_64MiB"] = batch_leg(lcs, ctx, [(p2.x, p2.y)], "dna", True, peak, 5,
                                                  tuning={"words_per_lane": 1, "tb_round_kib": 65536})
        del p2
        if args.workload == "batch_related":
            rl["batch_related_1GiB"] = batch_leg(lcs, ctx, pairs, alpha, True, peak, 3,
                                                 tuning={"tb_round_kib": 1 << 20})
        for k, v in rl.items():
            log(f"rounds {k}: {v}")
        out["traceback_rounds"] = rl
        # the batch end to end: plan, upload, run and copy the results back
        log("end-to-end leg")
        e2e = []
        for _ in range(3):
            t0 = time.perf_counter()
            if tb:
                lcs.lcs_traceback_batch(ctx, pairs, alpha)
            else:
                lcs.lcs_length_batch(ctx, pairs, alpha)
            e2e.append(time.perf_counter() - t0)
        t = float(np.median(e2e))
        out["end_to_end"] = {"s": round(t, 4), "GCUPS": round(cells / t / 1e9, 2),
                             "what": "one-call entry point from host buffers: validate, plan, "
                                     "upload, full pass, copy lengths and strings back"}
        log(f"end to end: {out['end_to_end']}")
    if not args.no_serve:
        log("request-server leg")
        sv = serve_leg(lcs, ctx, count=args.serve_requests, warmup=args.serve_warmup)
        sv["workload"] = ("Poisson arrivals at rho x measured capacity; |X|, |Y| log-uniform "
                          "[100, 100000]; alphabet DNA/protein/byte; traceback for half")
        out["serving"] = sv
    if not args.no_cpu:
        log(f"paper's striped OpenMP method on the host ({cores} threads)")
        out["paper_striped_host"] = striped_leg(lcs, ctx, cores)
        log(f"cpu oracle leg ({cores} threads)")
        cb = cpu_baseline(ps, tb, args.cpu_seconds, cores)
        out["cpu_baseline"] = cb
        out["gpu_over_cpu"] = round(value / cb["value"], 1)
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
