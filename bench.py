"""Benchmark of the MI355X data-race check.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1]

One step is one complete check of one batch of synthetic traces through the
C ABI (sim_check_traces_device): key statistics, key generation, the radix
passes, the pair count and the download of the racing-location list.  The
records are generated on the host, copied to HBM once, and stay resident
while K steps are timed between two device synchronisations.

The library's profiling mode records HIP events around every kernel on the
stream the kernels run on; the dominant kernel's average launch time over
the timed steps gives the roofline figure.  The oracle (CPU, one thread) is
timed on a bounded sample of the same workload and its output is compared
with the GPU's, bit for bit.

Prints one JSON line.
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

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
METRIC = "access records checked/sec and achieved HBM GB/s (batched vs plain, bit-exact)"

# Algorithmic bytes per record moved by each kernel (one launch):
#   stats  reads the 16-byte record
#   keygen reads the record and writes its 8-byte key
#   sort   one radix pass reads and writes every 8-byte key
#   scan   reads every 8-byte key once (tile scan; the crossing-location
#          and output kernels touch per-tile data only)
BYTES_PER_RECORD = {"stats": 16, "keygen": 24, "sort_pass": 16, "scan_tiles": 8}
KERNEL_SYMBOL = {"stats": "k_stats", "keygen": "k_keygen or k_keygen_scatter", "sort_pass": "k_scatter",
                 "scan_tiles": "k_scan_tiles"}


def workload(name):
    import tracegen

    if name == "c1":
        recs, inj = tracegen.c1()
        desc = {"workload": "c1: plain single trace, 1024 blocks x 256 threads, 2^24 records, 75% reads, "
                            "shared window 48 KiB/block, global reads Zipf(1.1) over 64 MiB, barrier every 16 "
                            "accesses, injected races 1e-4",
                "traces": 1, "records": int(len(recs)), "threads_per_block": 256}
        return recs, np.array([0, len(recs)], dtype=np.uint64), np.array([256], dtype=np.uint32), desc
    if name == "c0":
        recs = tracegen.c0()
        desc = {"workload": "c0: shared-memory tree reduction, 1 block x 256 threads, barrier before level 3 "
                            "removed", "traces": 1, "records": int(len(recs)), "threads_per_block": 256}
        return recs, np.array([0, len(recs)], dtype=np.uint64), np.array([256], dtype=np.uint32), desc
    if name == "c2":
        recs, inj = tracegen.c2()
        desc = {"workload": "c2: plain large trace, 8192 blocks x 512 threads, 2^28 records, 5% atomics, global "
                            "reads Zipf(1.1) over 1 GiB, injected races 1e-5",
                "traces": 1, "records": int(len(recs)), "threads_per_block": 512}
        return recs, np.array([0, len(recs)], dtype=np.uint64), np.array([512], dtype=np.uint32), desc
    if name == "c3":
        shapes = tracegen.c3_shapes(4096)
        recs, off, tpb, _ = tracegen.batch(shapes, inject_rate=1e-4)
        desc = {"workload": "c3: 4096 traces, sizes log-uniform 2^8..2^20 records, 1..256 blocks x 256 threads, "
                            "c1 distributions", "traces": 4096, "records": int(len(recs)), "threads_per_block": 256}
        return recs, off, tpb, desc
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(recs, offsets, tpb, budget_records):
    """Oracle (group counts, one thread) on the first traces of the workload
    up to budget_records records (whole traces only, at least one)."""
    import oracle

    n_tr = len(offsets) - 1
    k = 1
    while k < n_tr and int(offsets[k + 1]) <= budget_records:
        k += 1
    n = int(offsets[k])
    t0 = time.perf_counter()
    races, summ = oracle.closed_form(recs[:n], offsets[: k + 1], tpb[:k])
    dt = time.perf_counter() - t0
    return races, summ, n, k, dt


KERNEL_SOURCES = ["kernels.hip", "launch.h", "keys.h", "segstate.h", "tilewalk.h"]


def kernel_source_hash():
    """SHA-256 over the device code's sources (the kernels and the headers
    they include), in a fixed order."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1905_01833_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def pmc_traffic(stage, n_records):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3
    counter runs, if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{KERNEL_SYMBOL[stage]}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernels_sha256") != kernel_source_hash() or d.get("records") != n_records:
        return None
    return d.get("bytes_per_launch")


def profile_roofline(stage_ms, stage_launches, steps, n):
    """Roofline of the dominant kernel from per-stage event times."""
    dom = max(BYTES_PER_RECORD, key=lambda s: stage_ms.get(s, 0.0))
    avg_ms = stage_ms[dom] / max(1, stage_launches[dom])
    alg_bytes = BYTES_PER_RECORD[dom] * n
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    return dom, {"bound": "hbm", "kernel": KERNEL_SYMBOL[dom], "achieved": round(achieved, 1),
                 "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                 "traffic": pmc_traffic(dom, n), "avg_launch_ms": round(avg_ms, 5),
                 "launches_per_step": stage_launches[dom] / steps, "alg_bytes_per_launch": alg_bytes}


def batched_leg(pkg, torch, steps, log):
    """The batched workload (4096 traces of uneven size): one autotuned,
    graph-replayed call over all traces against one plain call per trace
    (default shape, no graph) on the same device records."""
    log("batched: generating c3")
    recs, offsets, tpb, desc = workload("c3")
    n = int(len(recs))
    n_tr = len(offsets) - 1
    dev = torch.from_numpy(recs.view(np.uint8).reshape(-1, 16)).to("cuda:0")
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    sptr = side.cuda_stream
    bctx = pkg.Context(0, graphs=True)
    log("batched: autotune")
    with torch.cuda.stream(side):
        tuning = bctx.autotune(dev, offsets, tpb, stream=sptr, reps=1)
        races, summ = bctx.check_traces_device(dev, offsets, tpb, stream=sptr)  # capture
    torch.cuda.synchronize()
    log("batched: timed")
    t0 = time.perf_counter()
    with torch.cuda.stream(side):
        for _ in range(steps):
            races, summ = bctx.check_traces_device(dev, offsets, tpb, stream=sptr)
    torch.cuda.synchronize()
    b_s = (time.perf_counter() - t0) / steps
    bctx.close()

    # stage times of the same call shape (events, no graph)
    pctx = pkg.Context(0, profile=True)
    pctx.set_tuning(tuning["size_class"], tuning)
    stage_ms, stage_launches = {}, {}
    for _ in range(2):
        pctx.check_traces_device(dev, offsets, tpb, stream=sptr)
        for name, (ms, launches) in pctx.stage_times().items():
            stage_ms[name] = stage_ms.get(name, 0.0) + ms
            stage_launches[name] = stage_launches.get(name, 0) + launches
    pctx.close()
    _, roof = profile_roofline(stage_ms, stage_launches, 2, n)

    log("batched: plain per-trace calls")
    plain = pkg.Context(0)
    views = [dev[int(offsets[i]) : int(offsets[i + 1])] for i in range(n_tr)]
    for i in range(min(8, n_tr)):  # warm the buffers
        plain.check_traces_device(views[i], None, int(tpb[i]), stream=sptr)
    per = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_tr):
        per.append(plain.check_traces_device(views[i], None, int(tpb[i]), stream=sptr))
    torch.cuda.synchronize()
    p_s = time.perf_counter() - t0
    plain.close()
    # the batched entries are the per-trace entries with trace numbers
    parts = []
    for i, (r, _) in enumerate(per):
        r = r.copy()
        r["trace"] = i
        parts.append(r)
    joined = np.concatenate(parts) if parts else races[:0]
    same = joined.tobytes() == races.tobytes() and all(
        summ[i].tobytes() == per[i][1][0].tobytes() for i in range(n_tr))
    return {
        "workload": desc["workload"], "traces": n_tr, "records": n,
        "value": n / b_s, "unit": "records/s", "ms_per_step": 1e3 * b_s, "steps": steps,
        "plain_value": n / p_s, "plain_ms": 1e3 * p_s, "speedup_vs_plain": p_s / b_s,
        "racing_locations": int(len(races)), "tuning": tuning, "roofline": roof,
        "stage_ms_per_step": {k: round(v / 2, 4) for k, v in stage_ms.items()},
        "batched_equals_per_trace": bool(same),
    }, (recs, offsets, tpb, races, summ)


def serving_leg(pkg, log, loads=((2000.0, 3.0),), pool_size=256, seed=0x5EED0004):
    """Serving workload: Poisson arrivals at `rate` requests/s for `duration`
    seconds (one run per (rate, duration) in `loads`), each request one
    trace with a lognormal size (median 2^14 records, sigma 1.5, at most
    2^22), c1 distributions, 256 threads per block; requests cycle through
    a pool of pre-generated traces.  Every result is compared with the same
    request checked alone."""
    import tracegen

    rng = np.random.default_rng(seed)
    shapes = []
    for _ in range(pool_size):
        n = int(min(1 << 22, max(64, round(np.exp(rng.normal(np.log(1 << 14), 1.5))))))
        nb = max(1, min(256, -(-n // (256 * 64))))
        shapes.append((n, nb, -(-n // (nb * 256)), int(rng.integers(1, 1 << 62))))
    recs, off, tpb, _ = tracegen.batch(shapes, inject_rate=1e-4)
    pool = [(recs[int(off[i]) : int(off[i + 1])], np.array([0, off[i + 1] - off[i]], dtype=np.uint64), tpb[i : i + 1])
            for i in range(pool_size)]
    log("serving: requests checked alone")
    ctx = pkg.Context(0)
    alone = [ctx.check_traces(r, o, t) for r, o, t in pool]
    ctx.close()

    srv = pkg.Server(0, hbm_budget_bytes=16 << 30, slots=4, max_batch_requests=256, reserve_records=1 << 23)
    for r, o, t in pool[:16]:  # warm the workers' buffers
        srv.wait(srv.submit(r, o, t))
    out = []
    for rate, duration in loads:
        srv.stats(reset=True)
        n_req = int(rate * duration)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
        which = rng.integers(0, pool_size, n_req)
        log(f"serving: {n_req} requests over {duration:.1f} s")
        tickets = []
        t0 = time.perf_counter()
        for k in range(n_req):
            while True:
                ahead = arrivals[k] - (time.perf_counter() - t0)
                if ahead <= 0:
                    break
                if ahead > 2e-4:
                    time.sleep(ahead - 1e-4)
            r, o, t = pool[which[k]]
            tickets.append(srv.submit(r, o, t))
        late = (time.perf_counter() - t0) - arrivals[-1]
        same = True
        recs_done = 0
        for k, tk in enumerate(tickets):
            got = srv.wait(tk)
            a = alone[which[k]]
            same = same and got[0].tobytes() == a[0].tobytes() and got[1].tobytes() == a[1].tobytes()
            recs_done += len(pool[which[k]][0])
        wall = time.perf_counter() - t0
        st = srv.stats()
        out.append({
            "workload": f"c4: Poisson arrivals, {rate:.0f} requests/s, one trace per request, sizes lognormal (median "
                        "2^14, sigma 1.5, max 2^22 records), c1 distributions, 4 worker slots, 16 GiB HBM budget, "
                        "buffers reserved for batches of 2^23 records",
            "requests": n_req, "offered_rate": rate, "achieved_rate": n_req / wall,
            "submit_lag_s": round(late, 4), "records": recs_done,
            "records_per_s": st["records_per_s"], "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
            "max_ms": st["max_ms"], "mean_ms": st["mean_ms"], "batches": st["batches"],
            "mean_batch_requests": st["mean_batch_requests"], "peak_inflight_bytes": st["peak_inflight_bytes"],
            "alone_equals_mix": bool(same),
        })
    srv.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c1", choices=["c0", "c1", "c2", "c3"])
    ap.add_argument("--cpu-budget", type=int, default=1 << 24, help="records in the oracle's timed sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg (profiling runs)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain leg")
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--serving-seconds", type=float, default=3.0)
    ap.add_argument("--no-autotune", action="store_true", help="default launch shape (profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain copy kernel of known size (256 MiB read, 256 MiB written; three launches) "
                         "whose HBM counters scale the pipeline's")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this check runs on one GPU; --gpus {args.gpus} is not supported "
              "(traces shard across GPUs without exchange, but only the one-GPU path is built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1905_01833_amd as pkg

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.calibrate_copy:
        a = torch.arange(1 << 26, dtype=torch.int32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b

    recs, offsets, tpb, desc = workload(args.workload)
    n = int(len(recs))
    dev = torch.from_numpy(recs.view(np.uint8).reshape(-1, 16)).to("cuda:0")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream().cuda_stream

    # timed steps: the production configuration (autotuned launch shape,
    # launch sequence captured once and replayed as a HIP graph)
    ctx = pkg.Context(0, graphs=True)
    if args.no_autotune:
        tuning = dict(ctx.tuning(pkg.sim_size_class(n))[1], size_class=pkg.sim_size_class(n))
    else:
        log(f"{args.workload}: autotune")
        tuning = ctx.autotune(dev, offsets, tpb, stream=stream, reps=3)
    log(f"{args.workload}: warmup")
    for _ in range(args.warmup):
        ctx.check_traces_device(dev, offsets, tpb, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        races, summ = ctx.check_traces_device(dev, offsets, tpb, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"{args.workload}: timed {args.steps} steps")
    ms_per_step = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed

    # per-kernel times: the same calls with HIP events around every launch
    # (events add gaps between launches, not kernel time)
    pctx = pkg.Context(0, profile=True)
    pctx.set_tuning(tuning["size_class"], tuning)
    stage_ms, stage_launches = {}, {}
    for _ in range(args.steps):
        pctx.check_traces_device(dev, offsets, tpb, stream=stream)
        for name, (ms, launches) in pctx.stage_times().items():
            stage_ms[name] = stage_ms.get(name, 0.0) + ms
            stage_launches[name] = stage_launches.get(name, 0) + launches
    torch.cuda.synchronize()
    pctx.close()
    _, roofline = profile_roofline(stage_ms, stage_launches, args.steps, n)
    passes = stage_launches.get("sort_pass", 0) / args.steps
    pipe_bytes = n * (16 + 24 + 16 * passes + 8)
    stages = {k: round(v / args.steps, 4) for k, v in stage_ms.items()}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "records/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded generator, shapes of the workload named in config)",
        "config": desc,
        "hbm_gbps_pipeline": round(pipe_bytes / (ms_per_step * 1e-3) / 1e9, 1),
        "radix_passes": passes,
        "stage_ms_per_step": stages,
        "racing_locations": int(len(races)),
        "tuning": tuning,
        "roofline": roofline,
    }

    ok = True
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        want, wsum, n_cpu, k_cpu, dt = cpu_baseline(recs, offsets, tpb, args.cpu_budget)
        if k_cpu == len(offsets) - 1:
            parity = races.tobytes() == want.tobytes() and summ.tobytes() == wsum.tobytes()
        else:
            got, gsum = ctx.check_traces_device(dev[:n_cpu], offsets[: k_cpu + 1], tpb[:k_cpu], stream=stream)
            parity = got.tobytes() == want.tobytes() and gsum.tobytes() == wsum.tobytes()
        out["cpu_baseline"] = {"value": n_cpu / dt, "unit": "records/s", "cores": 1, "kind": "oracle",
                               "sample": f"first {k_cpu} trace(s) of the workload, {n_cpu} records, oracle group-count "
                                         f"tier, {dt:.2f} s"}
        out["parity"] = "bit-exact" if parity else "MISMATCH"
        ok = ok and parity
    ctx.close()
    del dev

    if not args.no_batched and args.workload != "c3":
        b, (brecs, boff, btpb, braces, bsumm) = batched_leg(pkg, torch, args.batched_steps, log)
        if not args.no_cpu:
            # oracle on the leading traces of the batch (about 2^21 records)
            k = 1
            while k < len(boff) - 1 and int(boff[k + 1]) <= (1 << 21):
                k += 1
            import oracle

            want, wsum = oracle.closed_form(brecs[: int(boff[k])], boff[: k + 1], btpb[:k])
            sub = braces[braces["trace"] < k]
            b["parity"] = ("bit-exact" if sub.tobytes() == want.tobytes() and bsumm[:k].tobytes() == wsum.tobytes()
                           else "MISMATCH")
            b["parity_sample"] = f"oracle on the first {k} traces ({int(boff[k])} records); all traces against " \
                                 "per-trace plain calls"
            ok = ok and b["parity"] == "bit-exact"
        ok = ok and b["batched_equals_per_trace"]
        out["batched"] = b
    if not args.no_serving:
        # the configured rate, then ten times that rate (requests queue while
        # batches run, so continuous batching merges them)
        sv, hi = serving_leg(pkg, log, loads=((2000.0, args.serving_seconds), (20000.0, 1.0)))
        ok = ok and sv["alone_equals_mix"] and hi["alone_equals_mix"]
        out["serving"] = sv
        out["serving_high_load"] = hi
    print(json.dumps(out))
    if not ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
