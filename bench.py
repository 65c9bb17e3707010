#!/usr/bin/env python3
"""Benchmark of the LCS library on one MI355X.

Workload (default): the batched related-pair workload -- 4096 DNA pairs,
|X| log-uniform in [256, 65536], Y = X mutated at a rate drawn from
U[5%, 30%] -- with lengths and canonical tracebacks, replayed as a HIP graph.
One step = one full pass (symbol remap, match masks, bit-parallel fill,
checkpoints, traceback) over the resident batch.

Prints ONE JSON line.  `value` is whole-job GCUPS (sum of m*n over the batch
per second); `roofline` refers to the fill kernel, bound by integer VALU
issue; `cpu_baseline` is the CPU oracle timed on this host on a bounded
sample of the same workload.
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

# gfx950 integer-VALU roofline for the column recurrence: 256 CUs x 64 lanes
# x 2.4 GHz lane-instructions per second, 6 lane-instructions per 64 cells.
CUS, LANES, CLOCK_HZ, OPS_PER_64 = 256, 64, 2.4e9, 6
PEAK_TCUPS = CUS * LANES * CLOCK_HZ * 64 / OPS_PER_64 / 1e12


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
    raise SystemExit(f"unknown workload {name}")


def measured_traffic(workload: str, wpl: int, ckpt: int):
    """HBM bytes per fill launch from the committed rocprofv3 counter runs,
    or None when they were taken on a different kernel source, workload or
    plan (words per lane, checkpoint interval)."""
    import hashlib
    src = os.path.join(ROOT, "paper_1306_4627_amd", "csrc", "fill.hip")
    rec_file = os.path.join(ROOT, "profiles", "k_fill_batch_related_4096.md")
    try:
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        for line in open(rec_file):
            if line.startswith("traffic-record:"):
                rec = json.loads(line.split(":", 1)[1])
                if (rec["source_sha256_prefix"] == h and rec["workload"] == workload
                        and rec.get("words_per_lane") == wpl and rec.get("ckpt_interval") == ckpt):
                    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


def cpu_baseline(pairs, traceback: bool, budget_cells: float, threads: int):
    """Time the oracle on a random sample of the workload's pairs."""
    import oracle
    g = np.random.default_rng(7)
    order = g.permutation(len(pairs))
    sample, cells = [], 0
    for k in order:
        p = pairs[k]
        if cells + p.cells > budget_cells and sample:
            continue
        sample.append(p)
        cells += p.cells
        if cells >= budget_cells:
            break

    def one(p):
        if traceback:
            if (p.x.size + 1) * (p.y.size + 1) <= 2e8:
                oracle.lcs_traceback(p.x, p.y)
            else:
                oracle.lcs_traceback_ckpt(p.x, p.y, 512)
        else:
            oracle.lcs_length(p.x, p.y)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(one, sample))
    dt = time.perf_counter() - t0
    return {"value": cells / dt / 1e9, "unit": "GCUPS", "cores": threads, "kind": "oracle",
            "sample": f"{len(sample)} random pairs of the workload, {cells:.3e} cells, "
                      f"{'length+traceback' if traceback else 'length'}, {dt:.1f} s"}


def serve_leg(lcs, ctx, rates, count: int):
    """The request server under Poisson arrivals at each offered rate: every
    request submitted at its arrival time, then collected; latency is the
    library's submit-to-completion time of each request."""
    from paper_1306_4627_amd import inputs
    out = []
    for k, rate in enumerate(rates):
        reqs = inputs.serve_stream(rate, count, seed_offset=51 + k)
        cells = float(sum(int(r.x.size) * int(r.y.size) for r in reqs))
        with lcs.Server(ctx, mem_budget_bytes=8 << 30) as srv:
            tickets = []
            t0 = time.perf_counter()
            for r in reqs:
                while time.perf_counter() - t0 < r.arrival_s:
                    pass
                tickets.append(srv.submit(r.x, r.y, r.alphabet, traceback=r.want_traceback))
            lat = []
            for t in tickets:
                srv.wait(t)
                lat.append(srv.result(t)[2])
            wall = time.perf_counter() - t0
            st = srv.stats()
        lat_ms = np.array(lat) / 1e6
        out.append({"offered_rps": rate, "requests": count,
                    "achieved_rps": round(count / wall, 1),
                    "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                    "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
                    "GCUPS": round(cells / wall / 1e9, 2),
                    "batches": st["batches"], "max_inflight": st["max_inflight"],
                    "plan_ms_per_batch": round(st["plan_ns"] / max(st["batches"], 1) / 1e6, 3),
                    "device_ms_per_batch": round(st["device_ns"] / max(st["batches"], 1) / 1e6, 3),
                    "collect_ms_per_batch": round(st["collect_ns"] / max(st["batches"], 1) / 1e6, 3)})
        log(f"serve rate {rate}/s: {out[-1]}")
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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch_related")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-pair leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the request-server leg")
    ap.add_argument("--no-threshold", action="store_true", help="skip the threshold-pass leg")
    ap.add_argument("--no-schedule", action="store_true",
                    help="skip the traced fill pass (per-item schedule summary)")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-only", action="store_true",
                    help="only run the request-server leg and print its results")
    ap.add_argument("--cpu-cells", type=float, default=6e9)
    ap.add_argument("--wpl", type=int, default=0)
    ap.add_argument("--ckpt", type=int, default=0)
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

    from paper_1306_4627_amd import lcs

    if args.serve_only:
        ctx = lcs.Context(0)
        print(json.dumps({"serving": serve_leg(lcs, ctx, (1000, 8000, 64000), args.serve_requests)}),
              flush=True)
        ctx.close()
        return 0
    ps, alpha, tb, config = make_workload(args.workload)
    pairs = [(p.x, p.y) for p in ps]
    cells = float(sum(p.cells for p in ps))
    ctx = lcs.Context(0)
    log(f"workload {args.workload}: {len(pairs)} pairs, {cells:.3e} cells")
    tuning = {"words_per_lane": args.wpl, "ckpt_interval": args.ckpt}
    tune_s = None
    if not args.no_autotune and not args.wpl and not args.ckpt:
        t0 = time.perf_counter()
        tuning, tune_ms = lcs.autotune(ctx, pairs, alpha, traceback=tb, graph=True)
        tune_s = time.perf_counter() - t0
        log(f"autotune: {tuning} ({tune_ms:.3f} ms per pass, search {tune_s:.1f} s)")
    batch = lcs.Batch(ctx, pairs, alpha, traceback=tb, graph=True, **tuning)
    info = batch.info()
    log(f"plan: {info}")
    for _ in range(args.warmup):
        batch.time(eager=False)
    total_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t, _ = batch.time(eager=False)   # graph replay + sync, HIP events around it
        total_ms.append(t)
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    value = cells * args.steps / wall / 1e9
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
    # correctness spot check against the lengths of the first run
    lens = batch.lengths()

    out = {
        "metric": "LCS GCUPS batched vs plain per-pair on 1 MI355X; p50/p99 request latency",
        "value": round(value, 2), "unit": "GCUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": config,
        "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": round(PEAK_TCUPS, 1),
                     "unit": "TCUPS", "frac": round(achieved / PEAK_TCUPS, 4),
                     "traffic": measured_traffic(config["workload"], info["words_per_lane"],
                                                 info["ckpt_interval"]),
                     "kernel": "k_fill", "fill_ms": round(fill_avg, 4),
                     "clock_mhz_measured": None if clock_mhz is None else round(clock_mhz, 1),
                     "peak_at_measured_clock": None if clock_mhz is None
                     else round(PEAK_TCUPS * clock_mhz / 2400.0, 1),
                     "frac_at_measured_clock": None if clock_mhz is None
                     else round(achieved / (PEAK_TCUPS * clock_mhz / 2400.0), 4),
                     "eager_pass_ms": round(float(np.mean(eager_ms)), 4)},
        "plan": {k: info[k] for k in ("groups", "lanes", "lane_steps", "words_per_lane",
                                      "ckpt_interval", "classes", "device_bytes")},
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
    if not args.no_threshold:
        log("threshold-pass leg")
        out["threshold"] = threshold_leg(lcs, ctx, pairs, alpha)
    if not args.no_serve:
        log("request-server leg")
        out["serving"] = {"workload": "Poisson arrivals; |X|, |Y| log-uniform [100, 100000]; "
                                      "alphabet DNA/protein/byte; traceback for half",
                          "rates": serve_leg(lcs, ctx, (1000, 8000, 64000), args.serve_requests)}
    if not args.no_cpu:
        threads = min(len(os.sched_getaffinity(0)), 16)
        log(f"paper's striped OpenMP method on the host ({threads} threads)")
        out["paper_striped_host"] = striped_leg(lcs, ctx, threads)
        log(f"cpu oracle leg ({threads} threads)")
        cb = cpu_baseline(ps, tb, args.cpu_cells, threads)
        out["cpu_baseline"] = cb
        out["gpu_over_cpu"] = round(value / cb["value"], 1)
    batch.close()
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
