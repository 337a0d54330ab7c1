#!/usr/bin/env python3
"""Throughput benchmark of the batched PDHG library on one MI355X.

Default line (strong branching, Section 5.1, on the largest single-GPU shape):
a 200k x 500k base LP with 4 N(0,1) nonzeros per column, rows of mixed sense,
box [0,10], c ~ N(0,1) (the serving-stream family).  The root LP is solved on
the GPU (outside the timed region); 256 variables with fractional parts in
[0.1, 0.9] give a batch of B = 512 bound-changed LPs, each warm-started from
the root solution.  Ten draws of the candidates are staged in HBM; step i
solves draw i mod 10.  One step = set the batch from device-resident deltas
and warm start, solve every LP to 1e-4 relative KKT in FP64, copy x~ and y~ of
every LP to device buffers.

Reported beside it: the same LPs one at a time by the same library (plain
PDHG, B = 1, sampled), the dominant kernel's achieved HBM bandwidth against
8 TB/s (HIP events on the library's stream) and its measured traffic from a
committed counter summary taken on the same kernel sources, the fused product
kernels at B = 512 on the same matrix, the serving loop over four resident
bases at two Poisson rates (p50 / p99 latency, LPs/s), the 20000 x 50000
bound-tightening batch (FP32 iterates with FP64 sums, its FP64 run and the
objective difference), the 2000 x 5000 strong-branching batch, and the FP64
reference solver timed on the host cores on a sample of the same LPs.  Single
workloads: --workload fsb2 | obbt | mixed | serve | structured | sweep | copy |
trace-summary | pmc-summary.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("LPs solved/s to 1e-4 rel KKT, batched vs plain PDHG; SpMM HBM GB/s; p99 latency")
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def fused_bytes(kind, m, n, nnz, B, s_val, s_it):
    """Compulsory HBM bytes of one launch of a fused product + step kernel:
    the sparse matrix (values + int32 column indices + int32 row pointers),
    one read of the gathered block, and the streamed per-row blocks.
      primal (A'Y + primal step): Y gathered (m*B), Xbar and X0 read, Xbar written (3*n*B)
      dual   (A Xbar + dual step): Xbar gathered (n*B), Y and Y0 read, Y written (3*m*B)"""
    if kind == 0:
        return nnz * (s_val + 4) + 4 * (n + 1) + s_it * B * (m + 3 * n)
    return nnz * (s_val + 4) + 4 * (m + 1) + s_it * B * (n + 3 * m)


def kernel_source_sha() -> str:
    """SHA-256 of the library sources that decide what the kernels move (the
    kernels, their argument layout and the launch shapes)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "pdlpb_internal.h", "pdlpb.cpp"):
        with open(os.path.join(ROOT, "paper_2601_21990_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(name, kernel):
    """HBM bytes per launch of `kernel` from a committed counter summary, or
    None when the summary is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernels_sha256") != kernel_source_sha() or d.get("kernel") != kernel:
        return None
    return d["bytes_per_launch"]


def run_pmc_table(args):
    """Markdown table of L2-to-memory (EA) traffic per kernel from rocprofv3
    --pmc runs: every folder of --pmc-table (label=DIR, comma separated) holds
    one run; counters of the same label are merged, and each kernel's mean per
    dispatch is reported with the bytes the request-size counters give:
    read = 32 RDREQ_32B + 64 RDREQ_64B + 128 RDREQ_128B, write = 64 WRREQ_64B
    + 32 (WRREQ - WRREQ_64B) (on a 1 GiB copy these read exactly 1 GiB each).
    The means are over the dispatches that read at least 1 MB (a kernel with
    nothing to do, such as an evaluation of no restart cycle, returns at once
    and would dilute the mean); the runs of one label are the same program, so
    dispatch i of every run is the same launch."""
    import csv
    import glob
    runs = {}
    for item in args.pmc_table.split(","):
        label, d = item.split("=", 1)
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        per = runs.setdefault(label, {})
        for r in sorted(csv.DictReader(open(f)), key=lambda r: int(r["Dispatch_Id"])):
            name = r["Kernel_Name"]
            k = next((k for k in ("k_primal", "k_dual", "k_eval", "k_compact", "copyBuffer")
                      if k in name), None)
            if k is None:
                continue
            per.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(
                float(r["Counter_Value"]))
    lines = ["| run | kernel | dispatches (counted) | read GB | write GB | 128 B reads | 64 B reads | "
             "32 B reads | L2 hits | L2 misses |", "|---|---|---|---|---|---|---|---|---|---|"]
    for label, per in runs.items():
        for k, cs in sorted(per.items()):
            def col(c):
                return cs.get(c + "_sum") or cs.get(c)
            r128s, r64s, r32s = (col(f"TCC_EA0_RDREQ_{b}") for b in ("128B", "64B", "32B"))
            n = max(len(v) for v in cs.values())
            keep = list(range(n))
            if r128s:
                per_read = [128 * r128s[i] + 64 * (r64s[i] if r64s else 0) +
                            32 * (r32s[i] if r32s else 0) for i in range(len(r128s))]
                keep = [i for i, b in enumerate(per_read) if b >= 1e6] or keep

            def mean(c):
                v = col(c)
                if not v:
                    return None
                sel = [v[i] for i in keep if i < len(v)] if len(v) == n else v
                return sum(sel) / len(sel)
            r32, r64, r128 = (mean(f"TCC_EA0_RDREQ_{b}") for b in ("32B", "64B", "128B"))
            wr, wr64 = mean("TCC_EA0_WRREQ"), mean("TCC_EA0_WRREQ_64B")
            rd = None if r128 is None else 32 * (r32 or 0) + 64 * (r64 or 0) + 128 * r128
            wb = None if wr is None else 64 * wr64 + 32 * (wr - wr64)
            counted = f"{n} ({len(keep)})"

            def f(v, scale=1e9, nd=3):
                return "-" if v is None else f"{v / scale:.{nd}f}"
            lines.append(f"| {label} | {k} | {counted} | {f(rd)} | {f(wb)} | {f(r128, 1e6, 2)}M | "
                         f"{f(r64, 1e6, 2)}M | {f(r32, 1e6, 2)}M | {f(mean('TCC_HIT'), 1e6, 2)}M | "
                         f"{f(mean('TCC_MISS'), 1e6, 2)}M |")
    print("\n".join(lines))


def run_pmc_summary(args):
    """Per-dispatch HBM traffic of one kernel from two rocprofv3 --pmc runs of
    the same command (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), over the
    dispatches of the chosen solves (a solve starts at a k_begin_solve
    dispatch), scaled by what the same counters read for a 1 GiB device copy
    (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  Writes a JSON summary keyed by the
    hash of the kernel sources it was taken on."""
    import csv
    import glob
    solves = {int(v) for v in args.pmc_solves.split(",")}

    def per_dispatch(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        rows = sorted(csv.DictReader(open(f)), key=lambda r: int(r["Dispatch_Id"]))
        vals, solve = [], 0
        for r in rows:
            name = r["Kernel_Name"]
            if "k_begin_solve" in name:
                solve += 1
            if r["Counter_Name"] == counter and args.pmc_kernel in name and solve in solves:
                vals.append(float(r["Counter_Value"]))
        return vals

    fetch = per_dispatch(args.pmc_fetch, "FETCH_SIZE")
    write = per_dispatch(args.pmc_write, "WRITE_SIZE")
    if not fetch or len(fetch) != len(write):
        raise SystemExit(f"dispatch counts differ or are empty: {len(fetch)} vs {len(write)}")
    f_kib = sum(fetch) / len(fetch)
    w_kib = sum(write) / len(write)
    out = {"kernel": args.pmc_kernel, "solves": sorted(solves), "dispatches": len(fetch),
           "fetch_kib_per_dispatch": round(f_kib, 2), "write_kib_per_dispatch": round(w_kib, 2),
           "fetch_factor": 2.0, "write_factor": 1.0,
           "bytes_per_launch": int(round((2.0 * f_kib + 1.0 * w_kib) * 1024)),
           "kernels_sha256": kernel_source_sha(), "command": args.pmc_command}
    with open(args.pmc_out, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out), flush=True)


def spmm_leg():
    """The fused product kernels at the 200k x 500k shape (4 N(0,1) nonzeros
    per column, the serving-stream family), FP64, B = 512, default launch
    shapes, 65 iterations with every launch bracketed by HIP events: achieved
    GB/s = compulsory bytes / average launch time.  The blocks (≈2 GB each)
    exceed the 256 MB last-level cache, so this is the HBM point."""
    import paper_2601_21990_amd.pdlpb as P
    from workloads import make_cfg5, obbt_deltas, choose_vars
    inst = make_cfg5()
    m, n, nnz = inst.m, inst.n, inst.nnz
    B = 512
    ctx = P.Context.from_instance(inst, device=0)
    ctx.set_batch(obbt_deltas(choose_vars(n, B // 2, seed=B)))
    ctx.set_kernel_timing(True)
    ctx.solve(tol=0.0, max_iters=65)
    cnt, ms = ctx.kernel_times()
    cols = ctx.kernel_columns()
    ctx.set_kernel_timing(False)
    ctx.close()
    out = {"workload": f"A {m}x{n} (nnz {nnz}), FP64, B={B}, 65 iterations"}
    for kind, name in ((0, "primal"), (1, "dual")):
        nl = max(cnt[kind], 1)
        q0 = fused_bytes(kind, m, n, nnz, 0, 8, 8)
        q = q0 + (fused_bytes(kind, m, n, nnz, 1, 8, 8) - q0) * cols[kind] / nl
        avg = ms[kind] / nl
        gbs = q / (avg * 1e-3) / 1e9
        kname = "k_primal" if kind == 0 else "k_dual"
        traffic = measured_traffic(f"spmm_200kx500k_b512_fp64_{kname}_traffic.json", kname)
        out[name] = {"achieved": round(gbs, 1), "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "bytes_per_launch": int(q), "avg_launch_us": round(avg * 1e3, 2),
                     "launches": int(cnt[kind])}
        if traffic:
            # the rate of the bytes the counters saw move (gathers re-read the gathered block)
            mgbs = traffic / (avg * 1e-3) / 1e9
            out[name]["traffic_GBps"] = round(mgbs, 1)
            out[name]["traffic_frac"] = round(mgbs / HBM_PEAK_GBS, 4)
        log(f"spmm {name}: {avg*1e3:.1f} us per launch, {gbs:.1f} GB/s")
    return out


def _solve_index(rows):
    """Solve index (1-based) of every dispatch, in dispatch order: a solve
    starts at its k_begin_solve dispatch."""
    idx, cur = [], 0
    for r in rows:
        if "k_begin_solve" in r["Kernel_Name"]:
            cur += 1
        idx.append(cur)
    return idx


def run_trace_summary(args):
    """Markdown summary of a rocprofv3 --kernel-trace --stats run: the overall
    per-kernel statistics and the average duration of each kernel over the
    dispatches of the chosen solves (the benchmark's event-timed steps)."""
    import csv
    import glob
    d = args.trace_dir
    stats = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)[0]
    trace = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)[0]
    rows = sorted(csv.DictReader(open(trace)), key=lambda r: int(r["Dispatch_Id"]))
    sel = {int(v) for v in args.trace_solves.split(",")}
    per = {}
    for r, k in zip(rows, _solve_index(rows)):
        if k not in sel:
            continue
        name = r["Kernel_Name"].replace("(anonymous namespace)::", "").split("(")[0]
        name = name.split("<")[0].split("::")[-1]
        e = per.setdefault(name, [0, 0])
        e[0] += 1
        e[1] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    lines = [f"# {args.trace_title}", "", "Command:", "", "```", args.trace_command, "```", "",
             "## rocprofv3 kernel statistics (whole process)", "",
             "| kernel | calls | total ms | average us | % |", "|---|---|---|---|---|"]
    for r in list(csv.DictReader(open(stats)))[: args.trace_top]:
        lines.append(f"| {r['Name'][:60]} | {r['Calls']} | {int(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.3f} | {float(r['Percentage']):.2f} |")
    lines += ["", f"## Dispatches of solves {sorted(sel)} only", "",
              "| kernel | dispatches | average us |", "|---|---|---|"]
    for name, (cnt, ns) in sorted(per.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| {name} | {cnt} | {ns / cnt / 1e3:.3f} |")
    text = "\n".join(lines) + "\n"
    with open(args.trace_out, "w") as fh:
        fh.write(text)
    print(text)


def cpu_sample(n_lps, workers):
    """FP64 reference solver on the host cores: its own root solve, then n_lps
    branch LPs of the same family warm-started from it, one LP per task."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor
    import oracle as O
    from workloads import make_cfg2, choose_fractional, fsb_deltas, seed_for
    inst = make_cfg2()
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    base = O.solve(lp, O.Options(tol=1e-6, step_size=eta))
    vars_ = choose_fractional(base.x, n_lps // 2, seed_for(2, 1))
    D = fsb_deltas(base.x, vars_)
    tasks = [(int(d["kind"]), int(d["var"]), float(d["value"])) for d in D]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers, initializer=_cpu_init,
                             initargs=(eta, base.x, base.y, base.w)) as ex:
        res = list(ex.map(_cpu_task, tasks, chunksize=1))
    dt = time.perf_counter() - t0
    solved = sum(1 for s in res if s == O.OPTIMAL)
    return solved, dt


_CPU = {}


def _cpu_init(eta, x, y, w):
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)          # one thread per worker process
    import oracle as O
    from workloads import make_cfg2
    _CPU["lp"] = O.from_instance(make_cfg2())
    _CPU.update(eta=eta, x=x, y=y, w=w)


def _cpu_task(t):
    import oracle as O
    lpj = O.apply_delta(_CPU["lp"], *t)
    r = O.solve(lpj, O.Options(tol=1e-4, step_size=_CPU["eta"]), x_init=_CPU["x"],
                y_init=_CPU["y"], w_init=_CPU["w"])
    return r.status


def run_sweep(args):
    """Fused product kernels on a large matrix (200k x 500k, 4 N(0,1) nonzeros per
    column, the serving-stream family; or the 20k x 50k bound-tightening matrix)
    at batch widths B and both precisions:
    a fixed number of iterations per point, every launch bracketed by HIP events;
    achieved GB/s = compulsory bytes / average launch time (8 TB/s peak)."""
    import numpy as np
    import paper_2601_21990_amd.pdlpb as P
    from workloads import make_cfg3, make_cfg5, obbt_deltas, choose_vars
    # a solve replays whole blocks of C = 64 iterations: with any other count the
    # launches past the LPs' last iteration find no live column, and averaging
    # them in would overstate the rate of the ones that work
    if (args.sweep_iters - 1) % 64 != 0:
        raise SystemExit("--sweep-iters must be 64 k + 1 (65, 129, ...)")
    if args.sweep_matrix == "cfg3":
        inst = make_cfg3()
    else:
        inst = make_cfg5(m=args.sweep_m, n=int(round(2.5 * args.sweep_m)))
    m, n, nnz = inst.m, inst.n, inst.nnz
    log(f"sweep instance m={m} n={n} nnz={nnz}")
    widths = [int(b) for b in args.sweep_b.split(",")]
    points = []
    tiles = [tuple(int(v) for v in t.split("x")) for t in args.sweep_tiles.split(",")]
    caps = [int(b) for b in args.sweep_blocks.split(",")]
    eta = None
    for (prec, s_it, s_val, name), cap in ((p, c) for p in (
            (P.MIXED32, 4, 4, "fp32"), (P.FP64, 8, 8, "fp64")) for c in caps):
        if name not in args.sweep_prec.split(","):
            continue
        kw = {} if eta is None else {"step_size": eta}
        ctx = P.Context.from_instance(inst, device=0, precision=prec, use_graphs=0,
                                      max_blocks=cap, **kw)
        eta = ctx.step_size[0]
        for B in widths:
            D = obbt_deltas(choose_vars(n, max(B // 2, 1), seed=B))[:B]
            for lanes, vec in tiles:
                if vec > 1 and B % vec:
                    continue
                ctx.set_tile(lanes, vec)
                ctx.set_batch(D)
                ctx.set_kernel_timing(True)
                ctx.solve(tol=0.0, max_iters=args.sweep_iters)
                cnt, ms = ctx.kernel_times()
                ctx.set_kernel_timing(False)
                for kind, kname in ((0, "primal"), (1, "dual")):
                    avg = ms[kind] / max(cnt[kind], 1)
                    q = fused_bytes(kind, m, n, nnz, B, s_val, s_it)
                    gbs = q / (avg * 1e-3) / 1e9
                    points.append({"precision": name, "B": B, "tile": f"{lanes}x{vec}",
                                   "max_blocks": cap,
                                   "kernel": kname, "avg_us": round(avg * 1e3, 2),
                                   "bytes": int(q), "GBps": round(gbs, 1),
                                   "frac": round(gbs / HBM_PEAK_GBS, 4)})
                    log(f"{name} B={B:4d} tile={lanes}x{vec} cap={cap:5d} {kname:6s}: "
                        f"{avg*1e3:9.1f} us "
                        f"{q/1e6:9.1f} MB {gbs:8.1f} GB/s")
        ctx.close()
    best = max(points, key=lambda p: p["GBps"])
    print(json.dumps({"metric": "SpMM HBM GB/s (fused product + PDHG step)", "value": best["GBps"],
                      "unit": "GB/s", "peak": HBM_PEAK_GBS, "config": {
                          "workload": f"A {m}x{n}, nnz {nnz}",
                          "iterations_per_point": args.sweep_iters}, "best": best,
                      "points": points}), flush=True)


def run_copy(args):
    """Calibration for HBM counters: a plain device-to-device copy of a known
    size (1 GiB read + 1 GiB written per copy), repeated 4 times."""
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 4
    print(json.dumps({"metric": "device copy GB/s", "value": round(2 * nbytes / dt / 1e9, 1),
                      "unit": "GB/s", "bytes_read_per_copy": nbytes,
                      "bytes_written_per_copy": nbytes, "copies": 4}), flush=True)


def run_serve(args):
    print(json.dumps(serve_leg(args, [float(r) for r in args.serve_rates.split(",")],
                               args.serve_seconds)), flush=True)


def serve_leg(args, rates, seconds):
    """Serving stream: four resident base LPs (the 200k x 500k family by
    default, FP64; --serve-prec fp32 for FP32 iterates with FP64 sums, which
    cannot certify the infeasible branches of this family, see the design
    notes), each with its root solution kept on the device as warm start.
    Requests arrive as a Poisson process for `seconds`; each is a
    strong-branching batch of 2..512 LPs (log-uniform, even) on a random base.
    The loop admits requests whole, in arrival order, when their device-memory
    footprint fits one budget for all bases (--serve-budget-gb), serves the
    bases whose blocks finish first, and reports p50 / p99 latency, the time
    requests waited for admission and LPs/s per arrival rate.  Above capacity
    the queue grows; after the arrivals stop the loop drains for at most
    --serve-drain-s seconds, and the requests still unfinished are counted
    (their latency is at least their age, so p99 over the completed ones is
    then a lower bound, flagged `censored`)."""
    import numpy as np
    import paper_2601_21990_amd.pdlpb as P
    from paper_2601_21990_amd.serve import Server, Request, percentile
    from workloads import make_cfg5, fsb_deltas, deltas, BASE
    m = args.serve_m
    n = int(round(2.5 * m))
    prec = P.MIXED32 if args.serve_prec == "fp32" else P.FP64
    ctxs, roots = [], []
    for b in range(args.serve_bases):
        inst = make_cfg5(base=b, m=m, n=n)
        alloc = None if args.serve_hip_alloc else P.TorchAllocator(0)
        ctx = P.Context.from_instance(inst, device=0, precision=prec, max_batch=args.serve_cols,
                                      eval_every=args.serve_eval, allocator=alloc)
        ctx.set_batch(deltas([BASE], [0], [0.0]))
        ctx.solve(tol=1e-5, max_iters=50000)
        root = ctx.get(0)
        w = ctx.get_trace(0)["w"]
        log(f"base {b}: m={m} n={n} root {P.STATUS_NAMES[root['status']]} iters={root['iters']}")
        frac = root["x"] - np.floor(root["x"])
        cand = np.nonzero((frac > 0.1) & (frac < 0.9))[0]
        ctx.set_base_warm(root["x"], root["y"], w)
        ctx.serve_begin(args.serve_rows)
        ctxs.append(ctx)
        roots.append((root["x"], cand))
    if args.serve_budget_gb > 0:
        budget = int(args.serve_budget_gb * (1 << 30))
    elif args.serve_budget_gb < 0:
        # a share of the device's memory
        import torch
        budget = int(-args.serve_budget_gb * torch.cuda.get_device_properties(0).total_memory)
    else:
        budget = None
    rng = np.random.default_rng(2601021990 + 5000)
    lines = []
    for rate in rates:
        srv = Server(ctxs, warm=True, budget_bytes=budget)
        t_start = time.perf_counter()
        next_arrival = t_start + rng.exponential(1.0 / rate)
        n_req, offered = 0, 0
        submitted = []
        while True:
            now = time.perf_counter()
            while next_arrival <= now and next_arrival - t_start < seconds:
                b = int(rng.integers(0, len(ctxs)))
                size = int(round(np.exp(rng.uniform(np.log(2), np.log(512))) / 2)) * 2
                size = max(2, min(512, size))
                x, cand = roots[b]
                vars_ = np.sort(rng.choice(cand, size=size // 2, replace=False)).astype(np.int32)
                r = Request(base=b, deltas=fsb_deltas(x, vars_), arrival=next_arrival,
                            tol=1e-4, max_iters=args.serve_iters)
                srv.submit(r)
                submitted.append(r)
                n_req += 1
                offered += size
                next_arrival += rng.exponential(1.0 / rate)
            arrivals_over = next_arrival - t_start >= seconds
            if arrivals_over and (not srv.busy() or now - t_start > seconds + args.serve_drain_s):
                break
            if srv.busy():
                srv.step()
            else:
                time.sleep(max(0.0, min(next_arrival - time.perf_counter(), 0.01)))
        wall = time.perf_counter() - t_start
        unfinished = [r for r in submitted if r.done is None]
        # the loop ends here: requests never admitted are dropped, and the LPs
        # already in the library finish untimed
        srv.fifo.clear()
        srv.drain()
        done = [r for r in submitted if r.done is not None and r.done - t_start <= wall]
        lat = [r.latency for r in done]
        waits = [r.wait for r in done]
        solved = sum(sum(1 for s in r.statuses.values() if s == P.STATUS_OPTIMAL) for r in done)
        lps = sum(len(r.ids) for r in done)
        st = np.array([v for r in done for v in r.statuses.values()], dtype=np.int64)
        its = np.array([v for r in done for v in r.iters.values()], dtype=np.int64)
        line = {"rate_per_s": rate, "requests": n_req, "completed": len(done),
                "unfinished": len(unfinished), "censored": bool(unfinished),
                "offered_lps_per_s": round(offered / seconds, 1),
                "statuses": np.bincount(st, minlength=8).tolist() if st.size else [],
                "iters_median": int(np.median(its)) if its.size else 0,
                "iters_max": int(its.max()) if its.size else 0,
                "lps": lps, "lps_optimal": solved, "wall_s": round(wall, 3),
                "lps_per_s": round(lps / wall, 2),
                "p50_s": round(percentile(lat, 50), 4), "p99_s": round(percentile(lat, 99), 4),
                "admission_wait_p50_s": round(percentile(waits, 50), 4),
                "admission_wait_p99_s": round(percentile(waits, 99), 4),
                "peak_footprint_gib": round(srv.peak_bytes / (1 << 30), 2),
                "deferred_admissions": srv.blocked_on_budget, "trims": srv.trims}
        log(json.dumps(line))
        lines.append(line)
    for c in ctxs:
        c.close()
    return {"metric": "serving p50/p99 latency and LPs/s",
            "config": {"workload": f"{args.serve_bases} resident bases A {m}x{n} "
                                   f"(4 N(0,1) nnz/col), Poisson requests of 2..512 "
                                   f"strong-branching LPs, warm start, tol 1e-4",
                       "precision": args.serve_prec, "max_columns_per_base": args.serve_cols,
                       "eval_every": args.serve_eval, "result_rows": args.serve_rows,
                       "budget_gib": round(budget / (1 << 30), 2) if budget else None,
                       "torch_allocator": not args.serve_hip_alloc,
                       "seconds_per_rate": seconds,
                       "drain_cap_s": args.serve_drain_s},
            "rates": lines}


def _plain_leg(ctx, dD, X, Y, n_lps, max_iters):
    """The first n_lps LPs of a batch solved one at a time (B = 1) by the same
    context, cold start, after two untimed ones; LPs/s of those solved."""
    import torch
    import paper_2601_21990_amd.pdlpb as P
    n_lps = min(n_lps, dD.numel() // 16)

    def one(j):
        ctx.set_batch(dD[16 * j:16 * (j + 1)], mem=P.MEM_DEVICE)
        ctx.solve(tol=1e-4, max_iters=max_iters)
        r = ctx.get_batch(X=X[0:1], Y=Y[0:1], mem=P.MEM_DEVICE)
        return int(r["status"][0] == P.STATUS_OPTIMAL), int(r["iters"][0])

    for j in range(min(2, n_lps)):
        one(j)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [one(j) for j in range(n_lps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    solved = sum(r[0] for r in res)
    log(f"plain: {n_lps} LPs one at a time in {dt:.3f}s -> {solved / dt:.1f} LPs/s")
    return {"value": round(solved / dt, 2), "unit": "LPs/s", "lps": n_lps,
            "iters_median": int(sorted(r[1] for r in res)[n_lps // 2])}


def run_obbt(args):
    print(json.dumps(obbt_leg(args, args.steps, args.warmup)), flush=True)


def obbt_leg(args, steps, warmup):
    """Bound-tightening batch (Section 5.2) on the 20000 x 50000 family with 8
    U[-1,1] nonzeros per column, rows of mixed sense and box [0,5]: 256 LPs
    minimising and maximising 128 random variables, cold start.  The MIXED32
    run (FP32 iterates and products, FP64 sums) is the measured one; an FP64
    run of the same batch gives the objective difference per LP."""
    import numpy as np
    import torch
    import paper_2601_21990_amd.pdlpb as P
    from workloads import make_cfg3, obbt_deltas, choose_vars, seed_for
    inst = make_cfg3()
    D = obbt_deltas(choose_vars(inst.n, args.obbt_vars, seed_for(3, 0)))
    B = len(D)
    log(f"instance m={inst.m} n={inst.n} nnz={inst.nnz} B={B}")
    dev = torch.device("cuda:0")
    dD = torch.from_numpy(D.view(np.uint8).copy()).to(dev)
    out = {}
    for prec, name in ((P.MIXED32, "fp32"), (P.FP64, "fp64")):
        ctx = P.Context.from_instance(inst, device=0, precision=prec)
        X = torch.empty((B, inst.n), dtype=torch.float64, device=dev)
        Y = torch.empty((B, inst.m), dtype=torch.float64, device=dev)
        times = []
        for rep in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.set_batch(dD, mem=P.MEM_DEVICE)
            ctx.solve(tol=1e-4, max_iters=args.obbt_iters)
            r = ctx.get_batch(X=X, Y=Y, mem=P.MEM_DEVICE)
            torch.cuda.synchronize()
            if rep >= warmup:
                times.append(time.perf_counter() - t0)
        ok = int(np.sum(r["status"] == P.STATUS_OPTIMAL))
        dt = float(np.median(times))
        out[name] = dict(ctx=ctx, res=r, x=X.cpu().numpy(), solved=ok, s=dt,
                         lps_per_s=ok / dt)
        log(f"{name}: {ok}/{B} optimal, median {dt*1e3:.1f} ms per batch -> {ok/dt:.1f} LPs/s, "
            f"iters median {int(np.median(r['iters']))} max {int(np.max(r['iters']))}")
        if name == "fp32":
            out["plain"] = _plain_leg(ctx, dD, X, Y, args.plain_lps, args.obbt_iters)
    a, b = out["fp64"]["res"], out["fp32"]["res"]
    both = (a["status"] == P.STATUS_OPTIMAL) & (b["status"] == P.STATUS_OPTIMAL)
    dobj = np.abs(b["obj"] - a["obj"]) / (1.0 + np.abs(a["obj"]))
    vars_ = D["var"]
    xv = out["fp64"]["x"][np.arange(B), vars_]
    at_bound = np.mean((np.abs(xv - inst.l[vars_]) < 1e-6) | (np.abs(xv - inst.u[vars_]) < 1e-6))
    for k in ("fp32", "fp64"):
        out[k]["ctx"].close()
    return {
        "metric": "LPs solved/s to 1e-4 rel KKT (bound tightening, MIXED32)",
        "value": round(out["fp32"]["lps_per_s"], 2), "unit": "LPs/s",
        "fp64_lps_per_s": round(out["fp64"]["lps_per_s"], 2),
        "plain": out["plain"],
        "batched_vs_plain": round(out["fp32"]["lps_per_s"] / out["plain"]["value"], 3)
        if out["plain"]["value"] > 0 else None,
        "config": {"workload": f"A {inst.m}x{inst.n}, 8 U[-1,1] nnz/col, E/L/G rows, box [0,5], "
                               f"B={B} objectives +-e_j, cold start, tol 1e-4",
                   "B": B, "steps": steps, "warmup": warmup},
        "precision": {"lps_compared": int(both.sum()),
                      "obj_rel_diff_max": float(dobj[both].max()) if both.any() else None,
                      "obj_rel_diff_median": float(np.median(dobj[both])) if both.any() else None,
                      "fp32_rel_kkt_max": float(np.max(b["kkt"][both, 3])) if both.any() else None},
        "optimum_at_box_bound_fraction": round(float(at_bound), 4)}


def _mixed_pass(args, prec):
    """One pass of the mixed workload at one precision; returns the wall time,
    the requests (statuses, iterations, objectives per LP) and the base info."""
    import numpy as np
    import paper_2601_21990_amd.pdlpb as P
    from paper_2601_21990_amd.serve import Server, Request
    from workloads import make_cfg4, fsb_deltas, obbt_deltas, deltas, BASE, seed_for
    ctxs, roots = [], []
    for i in range(8):
        inst = make_cfg4(i)
        ctx = P.Context.from_instance(inst, device=0, precision=prec, max_batch=512)
        ctx.set_batch(deltas([BASE], [0], [0.0]))
        ctx.solve(tol=1e-5, max_iters=50000)
        root = ctx.get(0)
        w = ctx.get_trace(0)["w"]
        frac = root["x"] - np.floor(root["x"])
        cand = np.nonzero((frac > 0.1) & (frac < 0.9))[0]
        log(f"base {i}: m={inst.m} n={inst.n} nnz={inst.nnz} root "
            f"{P.STATUS_NAMES[root['status']]} iters={root['iters']} fractional={cand.size}")
        ctx.set_base_warm(root["x"], root["y"], w)
        ctx.serve_begin(1024)
        ctxs.append(ctx)
        roots.append((root["x"], cand, inst.n))
    # the request stream depends on the seed and, for bound flips, on each
    # base's fractional root values; the FP64 pass reuses the FP32 pass's stream
    reqs = getattr(args, "_mixed_reqs", None)
    if reqs is None:
        rng = np.random.default_rng(seed_for(4, 999))
        reqs, total = [], 0
        while total < args.mixed_lps:
            b = int(rng.integers(0, 8))
            size = int(round(np.exp(rng.uniform(np.log(2), np.log(512))) / 2)) * 2
            size = max(2, min(512, size, args.mixed_lps - total))
            x, cand, n = roots[b]
            if len(reqs) % 2 == 0 and cand.size >= size // 2:
                v = np.sort(rng.choice(cand, size=size // 2, replace=False)).astype(np.int32)
                d = fsb_deltas(x, v)
            else:
                v = np.sort(rng.choice(n, size=size // 2, replace=False)).astype(np.int32)
                d = obbt_deltas(v)
            reqs.append((b, d))
            total += len(d)
        args._mixed_reqs = reqs
    srv = Server(ctxs, warm=True)
    t0 = time.perf_counter()
    tagged = []
    for b, d in reqs:
        r = Request(base=b, deltas=d, arrival=t0, tol=1e-4, max_iters=args.mixed_iters)
        srv.submit(r)
        tagged.append(r)
    srv.drain()
    wall = time.perf_counter() - t0
    plain = None
    if getattr(args, "_mixed_plain", False):
        # the same loop fed one LP at a time: plain_lps LPs spread evenly over
        # the requests (both kinds, every base), after two untimed ones
        per = -(-args.plain_lps // len(reqs))
        sample = []
        for b, d in reqs:
            for j in np.linspace(0, len(d) - 1, min(per, len(d))).astype(int):
                sample.append((b, d[j:j + 1]))
        sample = sample[:args.plain_lps]

        def one(b, d):
            r = Request(base=b, deltas=d, arrival=time.perf_counter(), tol=1e-4,
                        max_iters=args.mixed_iters)
            srv.submit(r)
            srv.drain()
            return r

        for b, d in sample[:2]:
            one(b, d)
        t1 = time.perf_counter()
        done = [one(b, d) for b, d in sample]
        pdt = time.perf_counter() - t1
        ok = sum(1 for r in done for st in r.statuses.values() if st == P.STATUS_OPTIMAL)
        plain = {"value": round(ok / pdt, 2), "unit": "LPs/s", "lps": len(sample)}
        log(f"plain: {len(sample)} LPs one at a time in {pdt:.3f}s -> {ok / pdt:.1f} LPs/s")
    for c in ctxs:
        c.close()
    return wall, tagged, plain


def run_mixed(args):
    """Uneven mixed batching over eight base matrices (m = 1k ... 100k,
    n = 2.5 m, 4..12 N(0,1) nonzeros per column, box [0,10]): each base LP is
    solved on the GPU first; then 1000 LPs arrive as per-matrix batches of
    2..512 (log-uniform), half bound flips of fractional root values, half
    objectives +-e_j.  All batches are queued at once and the continuous-
    batching loop drains them, every context replaying captured blocks of
    iterations; LPs/s = LPs that reached 1e-4 / wall time.  The measured pass
    uses FP32 iterates with FP64 sums (--mixed-prec); an FP64 pass of the same
    requests gives the precision statement (objective difference per LP)."""
    import numpy as np
    import paper_2601_21990_amd.pdlpb as P
    prec = P.MIXED32 if args.mixed_prec == "fp32" else P.FP64
    args._mixed_plain = True
    wall, tagged, plain = _mixed_pass(args, prec)
    args._mixed_plain = False
    solved = sum(sum(1 for s in r.statuses.values() if s == P.STATUS_OPTIMAL) for r in tagged)
    kinds = {}
    for r in tagged:
        kind = "objective" if int(r.deltas["kind"][0]) == 3 else "bound"
        st = np.array([r.statuses[i] for i in r.ids])
        it = np.array([r.iters[i] for i in r.ids])
        e = kinds.setdefault(kind, {"lps": 0, "optimal": 0, "iters": []})
        e["lps"] += len(st)
        e["optimal"] += int(np.sum(st == P.STATUS_OPTIMAL))
        e["iters"].extend(it.tolist())
        log(f"request base={r.base} {kind} B={len(st)}: statuses {np.bincount(st, minlength=8).tolist()} "
            f"iters median {int(np.median(it))} max {int(it.max())} latency {r.latency:.2f}s")
    for e in kinds.values():
        e["iters_median"] = int(np.median(e["iters"]))
        e["iters_max"] = int(np.max(e["iters"]))
        del e["iters"]
    precision = None
    if prec == P.MIXED32 and not args.no_precision:
        wall64, tagged64, _ = _mixed_pass(args, P.FP64)
        d, both = [], 0
        for r32, r64 in zip(tagged, tagged64):
            for i32, i64 in zip(r32.ids, r64.ids):
                if r32.statuses[i32] == P.STATUS_OPTIMAL and r64.statuses[i64] == P.STATUS_OPTIMAL:
                    o32, o64 = r32.objs[i32], r64.objs[i64]
                    d.append(abs(o32 - o64) / (1.0 + abs(o64)))
        solved64 = sum(sum(1 for s in r.statuses.values() if s == P.STATUS_OPTIMAL)
                       for r in tagged64)
        precision = {"lps_compared": len(d), "obj_rel_diff_max": float(np.max(d)),
                     "obj_rel_diff_median": float(np.median(d)),
                     "fp64_lps_per_s": round(solved64 / wall64, 2)}
        log(f"precision: {json.dumps(precision)}")
    print(json.dumps({
        "metric": "LPs solved/s to 1e-4 rel KKT (uneven mixed batches over 8 bases)",
        "value": round(solved / wall, 2), "unit": "LPs/s",
        "config": {"workload": "8 bases m=1k..100k, n=2.5m, 4..12 N(0,1) nnz/col, box [0,10]; "
                               f"{sum(len(r.ids) for r in tagged)} LPs in {len(tagged)} batches "
                               "of 2..512, half bound flips, half +-e_j objectives, warm start "
                               "from each base",
                   "precision": args.mixed_prec},
        "plain": plain,
        "batched_vs_plain": round(solved / wall / plain["value"], 3) if plain and plain["value"] > 0
        else None,
        "lps": sum(len(r.ids) for r in tagged), "optimal": solved, "wall_s": round(wall, 3),
        "by_kind": kinds, "max_iters": args.mixed_iters, "precision_statement": precision}),
        flush=True)


def run_structured(args):
    """Structured LP relaxations (set covering 2000 x 4000 with 8 ones per row;
    capacitated facility location with 100 facilities, 1000 customers and 10
    candidate facilities each; packing 2000 x 5000 with 5 U[0.5,1.5] entries per
    column and box [0,10], where bound tightening moves bounds), diagonal
    preconditioning on, FP64.  Per
    family: the root LP on the GPU, then a strong-branching batch over 32
    fractional variables (64 LPs, warm start from the root) and a
    bound-tightening batch over 32 variables (64 LPs, dual feasibility checked
    at 1e-8, safe bounds with the 1e-4 improvement filter)."""
    import numpy as np
    import paper_2601_21990_amd.pdlpb as P
    from workloads import (make_setcover, make_facility, make_packing, choose_fractional,
                           fsb_deltas, obbt_deltas, choose_vars, deltas, BASE, seed_for)
    out = {}
    for inst in (make_setcover(), make_facility(), make_packing(m=2000, n=5000)):
        ctx = P.Context.from_instance(inst, device=0, scaling=1, dual_tol=1e-8)
        t0 = time.perf_counter()
        ctx.set_batch(deltas([BASE], [0], [0.0]))
        ctx.solve(tol=1e-6, max_iters=200000)
        root = ctx.get(0)
        w = ctx.get_trace(0)["w"]
        t_root = time.perf_counter() - t0
        frac = root["x"] - np.floor(root["x"])
        cand = np.nonzero((frac >= 0.1) & (frac <= 0.9))[0]
        p = min(32, cand.size)
        vars_ = choose_fractional(root["x"], p, seed_for(10, 0))
        D = fsb_deltas(root["x"], vars_)
        res = {"m": inst.m, "n": inst.n, "nnz": inst.nnz, "root_iters": int(root["iters"]),
               "root_s": round(t_root, 3), "fractional_root_values": int(cand.size)}
        for name, batch, warm in (("strong_branching", D, True),
                                  ("bound_tightening", obbt_deltas(choose_vars(inst.n, 32,
                                                                               seed_for(10, 1))),
                                   False)):
            times = []
            for rep in range(args.warmup + args.steps):
                t0 = time.perf_counter()
                if warm:
                    ctx.set_batch(batch, x_warm=root["x"], y_warm=root["y"],
                                  w_warm=np.full(len(batch), w))
                else:
                    ctx.set_batch(batch)
                ctx.solve(tol=1e-4, max_iters=100000)
                r = ctx.get_batch(want_x=False, want_y=False)
                if rep >= args.warmup:
                    times.append(time.perf_counter() - t0)
            dt = float(np.median(times))
            ok = int(np.sum(r["status"] == P.STATUS_OPTIMAL))
            e = {"lps": len(batch), "optimal": ok, "lps_per_s": round(ok / dt, 2),
                 "statuses": np.bincount(r["status"], minlength=8).tolist(),
                 "iters_median": int(np.median(r["iters"])), "iters_max": int(r["iters"].max())}
            if name == "bound_tightening":
                t = ctx.obbt_tighten(eps=1e-8, min_improve=1e-4)
                e["bounds_tightened"] = t["changed"]
            else:
                sc = ctx.branch_scores(root["obj"])
                e["best_score"] = float(np.nanmax(sc["score"][: len(batch) // 2]))
            res[name] = e
            log(f"{inst.name} {name}: {json.dumps(e)}")
        out[inst.name] = res
        ctx.close()
    print(json.dumps({"metric": "LPs solved/s to 1e-4 rel KKT (structured LP relaxations)",
                      "unit": "LPs/s", "precision": "fp64", "scaling": "ruiz+pock-chambolle",
                      "families": out}), flush=True)


def cpu_workers():
    """Worker processes for the reference solver: the CPUs this process may
    run on, at most 16 (the host share of one GPU on the measurement boxes)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail))


_CPU5 = {}


def _cpu5_init(eta, C, S, x, y, w):
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)          # one thread per worker process
    import oracle as O
    from workloads import make_cfg5
    _CPU5["lp"] = O.from_instance(make_cfg5(base=0))
    _CPU5.update(eta=eta, C=C, S=S, x=x, y=y, w=w)


def _cpu5_task(t):
    import oracle as O
    lpj = O.apply_delta(_CPU5["lp"], *t)
    r = O.solve(lpj, O.Options(tol=1e-4, step_size=_CPU5["eta"], eval_every=_CPU5["C"],
                               stop_every=_CPU5["S"], max_iters=100000),
                x_init=_CPU5["x"], y_init=_CPU5["y"], w_init=_CPU5["w"])
    return r.status, r.iters


def cpu_baseline_cfg5(sample, eta, C, S, root, w, workers):
    """The FP64 reference solver on the host cores, one LP per task, on LPs of
    the GPU batch: the same changes, the same warm start (the GPU's root
    solution), step size, evaluation interval and stopping tests."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor
    import oracle as O
    tasks = [(int(d["kind"]), int(d["var"]), float(d["value"])) for d in sample]
    with ProcessPoolExecutor(max_workers=workers, initializer=_cpu5_init,
                             initargs=(eta, C, S, root["x"], root["y"], w)) as ex:
        # the workers build the matrix before the clock starts
        list(ex.map(_cpu5_noop, range(workers), chunksize=1))
        t0 = time.perf_counter()
        res = list(ex.map(_cpu5_task, tasks, chunksize=1))
        dt = time.perf_counter() - t0
    solved = sum(1 for st, _ in res if st == O.OPTIMAL)
    iters = [it for _, it in res]
    return solved, dt, int(np.median(iters))


def _cpu5_noop(_):
    time.sleep(0.2)
    return 0


def mixed32_line(args, inst, eta, C, draws, d_draws, d_x, d_y, d_w, d_X, d_Y, fp64_by_draw):
    """The line's first draws again with FP32 iterates and products (FP64
    sums), from the same root and step size: LPs/s and the objective
    difference against the FP64 steps.  FP32 iterates cannot certify the
    infeasible branches of this family (the rounding of y~ swamps the
    displacement the test reads), so the FP32 run stops at an iteration cap
    and those LPs are reported, not counted."""
    import numpy as np
    import torch
    import paper_2601_21990_amd.pdlpb as P
    B = len(draws[0])
    ctx = P.Context.from_instance(inst, device=0, use_graphs=args.graphs, eval_every=C,
                                  stop_every=args.cfg5_stop_every, max_batch=B, step_size=eta,
                                  precision=P.MIXED32)
    cap = args.cfg5_mixed_iters

    def step(i):
        rc = P.lib.pdlpb_set_batch(ctx._h, B, d_draws[i].data_ptr(), d_x.data_ptr(),
                                   d_y.data_ptr(), d_w.data_ptr(), P.WARM_SHARED, P.MEM_DEVICE)
        ctx._check(rc)
        ctx.B = B
        ctx.solve(tol=1e-4, max_iters=cap)
        return ctx.get_batch(X=d_X, Y=d_Y, mem=P.MEM_DEVICE)

    nd = len(fp64_by_draw)
    step(0)                                # warm-up (graphs, tile choice)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [step(i) for i in range(nd)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    diffs, solved, capped, st_all = [], 0, 0, np.zeros(8, dtype=np.int64)
    for (st64, obj64), o in zip(fp64_by_draw, outs):
        both = (st64 == P.STATUS_OPTIMAL) & (o["status"] == P.STATUS_OPTIMAL)
        diffs.append(np.abs(o["obj"][both] - obj64[both]) / (1.0 + np.abs(obj64[both])))
        solved += int(np.sum(o["status"] == P.STATUS_OPTIMAL))
        capped += int(np.sum(o["status"] == P.STATUS_ITERATION_LIMIT))
        st_all += np.bincount(o["status"], minlength=8)
    d = np.concatenate(diffs) if diffs else np.zeros(0)
    res = {"value": round(solved / dt, 2), "unit": "LPs/s", "draws": nd,
           "lps_compared": int(d.size),
           "obj_rel_diff_max": float(d.max()) if d.size else None,
           "obj_rel_diff_median": float(np.median(d)) if d.size else None,
           "statuses": st_all.tolist(), "iteration_cap": cap, "capped": capped,
           "note": "FP32 iterates and products with FP64 sums, same draws, root and step size as "
                   "the FP64 steps; LPs at the iteration cap are the infeasible branches FP32 "
                   "cannot certify"}
    log(f"mixed32: {nd} draws in {dt:.3f}s, {solved} solved -> {res['value']} LPs/s; objective "
        f"difference max {res['obj_rel_diff_max']}, {capped} at the iteration cap")
    return res


def headline(args):
    """Strong branching on the 200k x 500k family (the largest single-GPU
    shape): B = 512 bound changes on 256 fractional variables of the GPU's root
    solution, warm start from it, FP64, draws cycled over the steps."""
    import numpy as np
    log("importing torch")
    import torch
    import paper_2601_21990_amd.pdlpb as P
    from workloads import make_cfg5, choose_fractional, fsb_deltas, seed_for, deltas, BASE

    dev = torch.device("cuda:0")
    torch.cuda.init()
    inst = make_cfg5(base=0)
    m, n, nnz = inst.m, inst.n, inst.nnz
    C = args.cfg5_eval
    log(f"instance m={m} n={n} nnz={nnz}")
    # the root LP (the MIP's relaxation) is solved once, with options of its
    # own, so the candidates do not depend on the batch's options
    with P.Context.from_instance(inst, device=0, eval_every=args.cfg5_root_eval,
                                 max_batch=1) as ctx_root:
        eta, norm_a = ctx_root.step_size
        log(f"eta={eta:.6g} ||A||={norm_a:.6g}")
        t0 = time.perf_counter()
        ctx_root.set_batch(deltas([BASE], [0], [0.0]))
        ctx_root.solve(tol=1e-6, max_iters=200000)
        root = ctx_root.get(0)
        root_w = ctx_root.get_trace(0)["w"]
    opts = dict(device=0, use_graphs=args.graphs, eval_every=C, max_batch=2 * args.cfg5_vars,
                stop_every=args.cfg5_stop_every, step_size=eta)
    ctx = P.Context.from_instance(inst, **opts)
    log(f"root: status={P.STATUS_NAMES[root['status']]} iters={root['iters']} "
        f"obj={root['obj']:.6f} in {time.perf_counter() - t0:.2f}s")
    draws = [fsb_deltas(root["x"], choose_fractional(root["x"], args.cfg5_vars,
                                                     seed_for(5, args.cfg5_draw_seed + r)))
             for r in range(args.fsb_draws)]
    B = len(draws[0])
    d_draws = [torch.from_numpy(D.view(np.uint8).copy()).to(dev) for D in draws]
    d_x = torch.from_numpy(root["x"]).to(dev)
    d_y = torch.from_numpy(root["y"]).to(dev)
    d_w = torch.full((B,), root_w, dtype=torch.float64, device=dev)
    d_X = torch.empty((B, n), dtype=torch.float64, device=dev)
    d_Y = torch.empty((B, m), dtype=torch.float64, device=dev)
    # the solve writes every LP's x~ and y~ into these tensors: get_batch into
    # them then copies nothing
    ctx.set_result_buffers(d_X, d_Y, B)
    torch.cuda.synchronize()

    def step(i):
        rc = P.lib.pdlpb_set_batch(ctx._h, B, d_draws[i % len(d_draws)].data_ptr(), d_x.data_ptr(),
                                   d_y.data_ptr(), d_w.data_ptr(), P.WARM_SHARED, P.MEM_DEVICE)
        ctx._check(rc)
        ctx.B = B
        ctx.solve(tol=1e-4, max_iters=100000)
        return ctx.get_batch(X=d_X, Y=d_Y, mem=P.MEM_DEVICE)

    out = None
    for i in range(max(args.warmup, 1)):
        out = step(i)
    log(f"warmup done: iters min/median/max = {out['iters'].min()}/{int(np.median(out['iters']))}/"
        f"{out['iters'].max()}, statuses {np.bincount(out['status'], minlength=8).tolist()}")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solved = 0
    iters, slowest, step_s, statuses = [], [], [], np.zeros(8, dtype=np.int64)
    fp64_by_draw = []                      # (statuses, objectives) of the first draws
    for i in range(args.steps):
        ts = time.perf_counter()
        out = step(i)                      # ends with the statuses read back to the host
        step_s.append(time.perf_counter() - ts)
        solved += int(np.sum(out["status"] == P.STATUS_OPTIMAL))
        statuses += np.bincount(out["status"], minlength=8)
        iters.append(out["iters"])
        slowest.append(int(out["iters"].max()))
        if i < len(draws) and len(fp64_by_draw) < args.cfg5_mixed_draws:
            fp64_by_draw.append((out["status"].copy(), out["obj"].copy()))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = solved / dt
    log(f"timed: {args.steps} steps in {dt:.4f}s, {solved} LPs solved -> {value:.1f} LPs/s")

    # the same steps with every fused launch bracketed by HIP events on the
    # library's stream (eager launches): per-kernel durations for the roofline
    ctx.set_kernel_timing(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    event_dt = time.perf_counter() - t1
    counts, total_ms = ctx.kernel_times()
    cols = ctx.kernel_columns()
    ctx.set_kernel_timing(False)
    log(f"event-timed pass: {event_dt:.4f}s")
    names = ["primal: A'Y + primal step", "dual: A Xbar + dual step", "evaluation",
             "control, restarts and compaction", "persistent tail"]
    dom = 0 if total_ms[0] >= total_ms[1] else 1
    nl = max(counts[dom], 1)
    avg_ms = total_ms[dom] / nl
    q0 = fused_bytes(dom, m, n, nnz, 0, 8, 8)
    q1 = fused_bytes(dom, m, n, nnz, 1, 8, 8) - q0
    q = (q0 * counts[dom] + q1 * cols[dom]) / nl
    achieved = q / (avg_ms * 1e-3) / 1e9
    kname = "k_primal" if dom == 0 else "k_dual"
    traffic = measured_traffic(f"fsb_200kx500k_b512_fp64_{kname}_traffic.json", kname)
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": traffic,
                "traffic_GBps": round(traffic / (avg_ms * 1e-3) / 1e9, 2) if traffic else None,
                "kernel": names[dom], "bytes_per_launch": int(q),
                "full_width_bytes": int(fused_bytes(dom, m, n, nnz, B, 8, 8)),
                "mean_live_columns": round(cols[dom] / nl, 2),
                "avg_launch_us": round(avg_ms * 1e3, 3), "launches": int(counts[dom])}
    kernel_ms = {names[k]: {"launches": int(counts[k]), "total_ms": round(total_ms[k], 3),
                            "avg_us": round(total_ms[k] / max(counts[k], 1) * 1e3, 2)}
                 for k in range(5)}

    # with host-memory inputs and outputs (every LP's x~ and y~ copied back)
    w_host = np.full(B, root_w)
    n_host = min(3, args.steps)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    host_solved = 0
    for i in range(n_host):
        ctx.set_batch(draws[i % len(draws)], x_warm=root["x"], y_warm=root["y"], w_warm=w_host)
        ctx.solve(tol=1e-4, max_iters=100000)
        r = ctx.get_batch()
        host_solved += int(np.sum(r["status"] == P.STATUS_OPTIMAL))
    host_dt = time.perf_counter() - t3
    host_io = {"value": round(host_solved / host_dt, 2), "unit": "LPs/s", "steps": n_host,
               "note": "inputs from and results (x~, y~ per LP, 2.9 GB) to host memory"}
    log(f"host I/O: {n_host} steps in {host_dt:.4f}s -> {host_io['value']} LPs/s")
    ctx.close()

    mixed = mixed32_line(args, inst, eta, C, draws, d_draws, d_x, d_y, d_w, d_X, d_Y,
                         fp64_by_draw) if fp64_by_draw else None

    # plain PDHG: a sample of the same LPs one at a time (B = 1), same library
    ctx_p = P.Context.from_instance(inst, device=0, use_graphs=args.graphs,
                                    eval_every=args.cfg5_plain_eval, max_batch=1, step_size=eta)
    n_plain = min(args.plain_lps, B * len(draws))
    picks = [(j % len(draws), (j * 37) % B) for j in range(n_plain)]

    def plain_ptr(j):
        r, k = picks[j]
        return d_draws[r].data_ptr() + 16 * k

    def one(j):
        rc = P.lib.pdlpb_set_batch(ctx_p._h, 1, plain_ptr(j), d_x.data_ptr(), d_y.data_ptr(),
                                   d_w.data_ptr(), P.WARM_SHARED, P.MEM_DEVICE)
        ctx_p._check(rc)
        ctx_p.B = 1
        ctx_p.solve(tol=1e-4, max_iters=100000)
        return ctx_p.get_batch(X=d_X, Y=d_Y, mem=P.MEM_DEVICE)

    for j in range(min(2, n_plain)):
        one(j)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    plain_solved, plain_iters, plain_s = 0, [], []
    for j in range(n_plain):
        tj = time.perf_counter()
        o = one(j)
        plain_s.append(time.perf_counter() - tj)
        plain_solved += int(o["status"][0] == P.STATUS_OPTIMAL)
        plain_iters.append(int(o["iters"][0]))
    torch.cuda.synchronize()
    plain_dt = time.perf_counter() - t2
    plain_value = plain_solved / plain_dt
    log(f"plain: {n_plain} LPs in {plain_dt:.4f}s -> {plain_value:.1f} LPs/s")
    ctx_p.close()

    cpu = None
    if not args.no_cpu_baseline:
        workers = cpu_workers()
        cpu_lps = np.concatenate(draws)[:args.cfg5_cpu_lps]
        n_cpu = len(cpu_lps)
        log(f"cpu baseline: reference solver, {n_cpu} LPs on {workers} processes")
        cs, cdt, cmed = cpu_baseline_cfg5(cpu_lps, eta, C, args.cfg5_stop_every, root, root_w,
                                          workers)
        cpu = {"value": round(cs / cdt, 3), "unit": "LPs/s", "cores": workers, "kind": "oracle",
               "host_cpu_count": os.cpu_count(),
               "sample": f"the {n_cpu} LPs of the first {-(-n_cpu // B)} draws (the batches of "
                         f"the first steps), same changes, warm start, step size, evaluation "
                         f"interval ({C}) and stopping tests (every {args.cfg5_stop_every}); one "
                         f"LP per process task; {cs} solved in {cdt:.2f}s, "
                         f"median {cmed} iterations"}
        log(f"cpu: {cpu['value']} LPs/s")

    it_all = np.concatenate(iters)
    return {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "LPs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"strong-branching batch on the 200k x 500k family: A {m}x{n} "
                               f"(4 N(0,1) nnz/col, E/L/G rows), box [0,10], B={B} bound changes "
                               f"on {B // 2} fractional variables of the root LP, warm start from "
                               f"it, FP64, tol 1e-4 rel KKT; step i solves draw i mod "
                               f"{len(draws)} of the candidates",
                   "m": m, "n": n, "nnz": nnz, "B": B, "tol": 1e-4, "draws": len(draws),
                   "eval_every": C, "stop_every": args.cfg5_stop_every,
                   "root_eval_every": args.cfg5_root_eval, "root_iters": int(root["iters"])},
        "plain": {"value": round(plain_value, 2), "unit": "LPs/s", "lps": n_plain,
                  "iters_median": int(np.median(plain_iters)), "eval_every": args.cfg5_plain_eval,
                  "ms_per_lp_median": round(float(np.median(plain_s)) * 1e3, 3)},
        "batched_vs_plain": round(value / plain_value, 3) if plain_value > 0 else None,
        "step_ms": {"min": round(min(step_s) * 1e3, 3),
                    "median": round(float(np.median(step_s)) * 1e3, 3),
                    "max": round(max(step_s) * 1e3, 3)},
        "statuses": statuses.tolist(),
        "event_timed_pass_s": round(event_dt, 4),
        "host_io": host_io,
        "iters": {"min": int(it_all.min()), "median": int(np.median(it_all)),
                  "max": int(it_all.max()), "slowest_per_batch_median": int(np.median(slowest))},
        "kernels": kernel_ms,
        "roofline": roofline,
        "mixed32": mixed,
        "cpu_baseline": cpu,
    }



def fsb2_leg(args, with_cpu=False):
    """Strong-branching batch on the 2000 x 5000 family (5 N(0,1) nonzeros per
    column, 1000 E + 1000 L rows, box [0,10]): B = 64 bound changes on 32
    fractional variables of the GPU's root solution, warm start from it, FP64,
    ten draws of the candidates cycled over the steps; the same LPs one at a
    time; the dual step's roofline; optionally the reference solver on the
    host cores (its own root solve)."""
    import numpy as np
    log("importing torch")
    import torch
    import paper_2601_21990_amd.pdlpb as P
    from workloads import make_cfg2, choose_fractional, fsb_deltas, seed_for, deltas, BASE

    dev = torch.device("cuda:0")
    torch.cuda.init()
    inst = make_cfg2(m=args.fsb2_m, n=args.fsb2_m * 5 // 2)
    m, n, nnz = inst.m, inst.n, inst.nnz
    log(f"instance m={m} n={n} nnz={nnz}")

    opts = dict(device=0, use_graphs=args.graphs, tail_cols=args.tail_cols,
                tile_lanes=args.tile_lanes, tile_vec=args.tile_vec,
                eval_every=args.eval_every)
    ctx = P.Context.from_instance(inst, **opts)
    # the one-LP-at-a-time leg runs at the evaluation interval that suits one LP best
    popts = {**opts, "eval_every": args.plain_eval_every}
    if args.plain_tile_lanes:
        popts.update(tile_lanes=args.plain_tile_lanes, tile_vec=1)
    ctx_plain = P.Context.from_instance(inst, **popts)
    eta, norm_a = ctx.step_size
    log(f"eta={eta:.6g} ||A||={norm_a:.6g}")

    # root LP on the GPU (untimed): the MIP's relaxation solution
    ctx.set_batch(deltas([BASE], [0], [0.0]))
    ctx.solve(tol=1e-6, max_iters=200000)
    root = ctx.get(0)
    root_w = ctx.get_trace(0)["w"]
    log(f"root: status={P.STATUS_NAMES[root['status']]} iters={root['iters']} obj={root['obj']:.6f}")
    # one batch per draw of branching candidates from the root's fractional
    # variables; step i solves draw i mod R, so the rate describes the family of
    # batches rather than the luck of one draw (the batch time is set by its
    # slowest LP, often an infeasible branch)
    draws = [fsb_deltas(root["x"], choose_fractional(root["x"], args.fsb_vars, seed_for(2, r)))
             for r in range(args.fsb_draws)]
    B = len(draws[0])

    # inputs resident in HBM before the timed region
    d_draws = [torch.from_numpy(D.view(np.uint8).copy()).to(dev) for D in draws]
    d_x = torch.from_numpy(root["x"]).to(dev)
    d_y = torch.from_numpy(root["y"]).to(dev)
    d_w = torch.full((B,), root_w, dtype=torch.float64, device=dev)
    d_X = torch.empty((B, n), dtype=torch.float64, device=dev)
    d_Y = torch.empty((B, m), dtype=torch.float64, device=dev)
    # the solve writes every LP's x~ and y~ into these tensors: get_batch into
    # them then copies nothing
    ctx.set_result_buffers(d_X, d_Y, B)
    torch.cuda.synchronize()

    def step(i):
        rc = P.lib.pdlpb_set_batch(ctx._h, B, d_draws[i % len(d_draws)].data_ptr(), d_x.data_ptr(),
                                   d_y.data_ptr(), d_w.data_ptr(), P.WARM_SHARED, P.MEM_DEVICE)
        ctx._check(rc)
        ctx.B = B
        ctx.solve(tol=1e-4, max_iters=100000)
        return ctx.get_batch(X=d_X, Y=d_Y, mem=P.MEM_DEVICE)

    out = None
    for i in range(max(args.warmup, 1)):
        out = step(i)
    log(f"warmup done: iters min/median/max = {out['iters'].min()}/{int(np.median(out['iters']))}/"
        f"{out['iters'].max()}, statuses {np.bincount(out['status'], minlength=6).tolist()}")

    # timed region: K steps as shipped (blocks of C iterations replayed as hipGraphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solved = 0
    iters, slowest, step_s = [], [], []
    for i in range(args.steps):
        ts = time.perf_counter()
        out = step(i)                      # ends with the statuses read back to the host
        step_s.append(time.perf_counter() - ts)
        solved += int(np.sum(out["status"] == P.STATUS_OPTIMAL))
        iters.append(out["iters"])
        slowest.append(int(out["iters"].max()))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = solved / dt
    log(f"timed: {args.steps} steps in {dt:.4f}s, {solved} LPs solved -> {value:.1f} LPs/s")

    # the same steps again with every product kernel bracketed by HIP events on
    # the library's stream (eager launches): per-kernel durations for the roofline
    ctx.set_kernel_timing(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    event_dt = time.perf_counter() - t1
    counts, total_ms = ctx.kernel_times()
    cols = ctx.kernel_columns()
    ctx.set_kernel_timing(False)
    log(f"event-timed pass: {event_dt:.4f}s")

    # roofline of the dominant kernel: algorithmic bytes are affine in the live
    # column count of a launch, so their sum over the timed launches follows from
    # the launch count and the summed live columns
    names = ["primal: A'Y + primal step", "dual: A Xbar + dual step", "evaluation", "control",
             "persistent tail"]
    dom = 0 if total_ms[0] >= total_ms[1] else 1
    nl = max(counts[dom], 1)
    avg_ms = total_ms[dom] / nl
    q0 = fused_bytes(dom, m, n, nnz, 0, 8, 8)
    q1 = fused_bytes(dom, m, n, nnz, 1, 8, 8) - q0
    q = (q0 * counts[dom] + q1 * cols[dom]) / nl
    achieved = q / (avg_ms * 1e-3) / 1e9
    kname = "k_primal" if dom == 0 else "k_dual"
    traffic = measured_traffic(f"fsb_2000x5000_b64_fp64_{kname}_traffic.json", kname)
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": traffic,
                "traffic_GBps": round(traffic / (avg_ms * 1e-3) / 1e9, 2) if traffic else None,
                "kernel": names[dom], "bytes_per_launch": int(q),
                "full_width_bytes": int(fused_bytes(dom, m, n, nnz, B, 8, 8)),
                "mean_live_columns": round(cols[dom] / nl, 2),
                "avg_launch_us": round(avg_ms * 1e3, 3), "launches": int(counts[dom])}
    kernel_us = {names[k]: round(total_ms[k] / max(counts[k], 1) * 1e3, 3) for k in range(5)}

    # the same steps with the inputs in host memory and the results copied back
    # to it (the boundary accepts either): the rate including the host transfers
    w_host = np.full(B, root_w)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    host_solved = 0
    for i in range(args.steps):
        ctx.set_batch(draws[i % len(draws)], x_warm=root["x"], y_warm=root["y"], w_warm=w_host)
        ctx.solve(tol=1e-4, max_iters=100000)
        r = ctx.get_batch()
        host_solved += int(np.sum(r["status"] == P.STATUS_OPTIMAL))
    host_dt = time.perf_counter() - t3
    host_io = {"value": round(host_solved / host_dt, 2), "unit": "LPs/s",
               "note": "inputs from and results (x~, y~ per LP) to host memory"}
    log(f"host I/O: {args.steps} steps in {host_dt:.4f}s -> {host_io['value']} LPs/s")

    # plain PDHG: the same LPs one at a time (B = 1) with the same library
    ctx.close()
    ctx = ctx_plain
    # LP j of the sample is LP j // R of draw j mod R
    np_plain = min(args.plain_lps, B * len(d_draws))

    def plain_ptr(j):
        return d_draws[j % len(d_draws)].data_ptr() + 16 * (j // len(d_draws))

    for j in range(min(2, np_plain)):          # untimed: graphs for B = 1
        rc = P.lib.pdlpb_set_batch(ctx._h, 1, plain_ptr(j), d_x.data_ptr(),
                                   d_y.data_ptr(), d_w.data_ptr(), P.WARM_SHARED, P.MEM_DEVICE)
        ctx._check(rc)
        ctx.B = 1
        ctx.solve(tol=1e-4, max_iters=100000)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    plain_solved = 0
    plain_iters = []
    for j in range(np_plain):
        rc = P.lib.pdlpb_set_batch(ctx._h, 1, plain_ptr(j), d_x.data_ptr(),
                                   d_y.data_ptr(), d_w.data_ptr(), P.WARM_SHARED, P.MEM_DEVICE)
        ctx._check(rc)
        ctx.B = 1
        ctx.solve(tol=1e-4, max_iters=100000)
        o = ctx.get_batch(X=d_X, Y=d_Y, mem=P.MEM_DEVICE)
        plain_solved += int(o["status"][0] == P.STATUS_OPTIMAL)
        plain_iters.append(int(o["iters"][0]))
    torch.cuda.synchronize()
    plain_dt = time.perf_counter() - t2
    plain_value = plain_solved / plain_dt
    log(f"plain: {np_plain} LPs in {plain_dt:.4f}s -> {plain_value:.1f} LPs/s")

    cpu = None
    if with_cpu and not args.no_cpu_baseline:
        workers = cpu_workers()
        log(f"cpu baseline: reference solver, {args.cpu_lps} LPs on {workers} processes")
        cs, cdt = cpu_sample(args.cpu_lps, workers)
        cpu = {"value": round(cs / cdt, 2), "unit": "LPs/s", "cores": workers, "kind": "oracle",
               "host_cpu_count": os.cpu_count(),
               "sample": f"{args.cpu_lps} strong-branching LPs of the same 2000x5000 family, "
                         f"warm-started from the reference solver's own root solve, "
                         f"one LP per process task, evaluation interval 64 (its default); "
                         f"{cs} solved in {cdt:.2f}s"}
        log(f"cpu: {cpu['value']} LPs/s")

    ctx.close()
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "LPs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"strong-branching batch: A {m}x{n} (5 N(0,1) nnz/col), {m // 2} E + "
                               f"{m - m // 2} L rows, box [0,10], B={B} bound changes on {B // 2} fractional "
                               "variables, warm start from the root LP, FP64, tol 1e-4 rel KKT; "
                               f"step i solves draw i mod {len(d_draws)} of the candidates",
                   "m": m, "n": n, "nnz": nnz, "B": B, "tol": 1e-4, "draws": len(d_draws),
                   "eval_every": args.eval_every},
        "plain": {"value": round(plain_value, 2), "unit": "LPs/s", "lps": np_plain,
                  "iters_median": int(np.median(plain_iters)),
                  "eval_every": args.plain_eval_every},
        "batched_vs_plain": round(value / plain_value, 3) if plain_value > 0 else None,
        "step_ms": {"min": round(min(step_s) * 1e3, 3), "median": round(float(np.median(step_s)) * 1e3, 3),
                    "max": round(max(step_s) * 1e3, 3)},
        "event_timed_pass_s": round(event_dt, 4),
        "host_io": host_io,
        "iters": {"min": int(np.min(np.concatenate(iters))),
                  "median": int(np.median(np.concatenate(iters))),
                  "max": int(np.max(np.concatenate(iters))),
                  "slowest_per_batch_median": int(np.median(slowest))},
        "kernel_avg_us": kernel_us,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    return line


def make_parser():
    """The command line; its defaults are the default line's options."""
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="line",
                    choices=["line", "fsb2", "sweep", "copy", "serve", "obbt", "mixed",
                             "structured", "pmc-summary", "pmc-table", "trace-summary"])
    ap.add_argument("--trace-dir", help="rocprofv3 --kernel-trace --stats output folder")
    ap.add_argument("--trace-solves", default="6,7,8")
    ap.add_argument("--trace-out", default=None)
    ap.add_argument("--trace-title", default="kernel trace")
    ap.add_argument("--trace-command", default="")
    ap.add_argument("--trace-top", type=int, default=16)
    ap.add_argument("--pmc-fetch", help="rocprofv3 output folder of the FETCH_SIZE run")
    ap.add_argument("--pmc-write", help="rocprofv3 output folder of the WRITE_SIZE run")
    ap.add_argument("--pmc-kernel", default="k_dual")
    ap.add_argument("--pmc-solves", default="2,3,4",
                    help="1-based solves (k_begin_solve dispatches) whose launches count")
    ap.add_argument("--pmc-out", default=None)
    ap.add_argument("--pmc-command", default="")
    ap.add_argument("--pmc-table", help="pmc-table: label=DIR,... of rocprofv3 --pmc runs")
    ap.add_argument("--obbt-vars", type=int, default=128)
    ap.add_argument("--obbt-iters", type=int, default=100000)
    ap.add_argument("--mixed-lps", type=int, default=1000)
    ap.add_argument("--mixed-prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--mixed-iters", type=int, default=20000)
    ap.add_argument("--no-precision", action="store_true",
                    help="mixed: skip the FP64 pass of the precision statement")
    ap.add_argument("--serve-eval", type=int, default=8,
                    help="serve: iterations between evaluations (the block length)")
    ap.add_argument("--eval-every", type=int, default=32,
                    help="fsb: iterations between evaluations of the batch")
    ap.add_argument("--fsb-vars", type=int, default=32,
                    help="fsb: branching candidates (the batch holds two LPs per candidate)")
    ap.add_argument("--fsb-draws", type=int, default=10,
                    help="fsb: independent draws of the candidates; step i solves draw i mod R")
    ap.add_argument("--plain-tile-lanes", type=int, default=0,
                    help="fsb: fixed lanes per row for the one-LP-at-a-time leg (0: the library's choice)")
    ap.add_argument("--plain-eval-every", type=int, default=64,
                    help="fsb: iterations between evaluations of the one-LP-at-a-time leg")
    ap.add_argument("--serve-m", type=int, default=200000)
    ap.add_argument("--serve-bases", type=int, default=4)
    ap.add_argument("--serve-prec", default="fp64", choices=["fp32", "fp64"])
    ap.add_argument("--serve-cols", type=int, default=256)
    ap.add_argument("--serve-rows", type=int, default=2048)
    ap.add_argument("--serve-rates", default="1,3,10")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-iters", type=int, default=20000)
    ap.add_argument("--serve-budget-gb", type=float, default=-0.75,
                    help="serve: device-memory budget of all bases: GiB if > 0, a fraction of "
                         "the device's memory if < 0, none if 0")
    ap.add_argument("--serve-hip-alloc", action="store_true",
                    help="serve: the contexts' device memory from hipMalloc instead of PyTorch's "
                         "caching allocator (growing and trimming storage then allocates anew)")
    ap.add_argument("--serve-drain-s", type=float, default=20.0,
                    help="serve: longest drain after the arrivals stop")
    ap.add_argument("--sweep-m", type=int, default=200000)
    ap.add_argument("--sweep-b", default="1,8,32,64,128,256,512")
    ap.add_argument("--sweep-iters", type=int, default=65)
    ap.add_argument("--sweep-tiles", default="0x0", help="lanes x vec per point; 0x0 = automatic")
    ap.add_argument("--sweep-prec", default="fp32,fp64")
    ap.add_argument("--sweep-matrix", default="cfg5", choices=["cfg3", "cfg5"],
                    help="cfg5: 200k x 500k (4 N(0,1) nnz/col); cfg3: 20k x 50k (8 U[-1,1] nnz/col)")
    ap.add_argument("--sweep-blocks", default="0",
                    help="workgroup caps of the step launches; 0 = the library default")
    ap.add_argument("--cfg5-vars", type=int, default=256,
                    help="default line: branching candidates on the 200k x 500k base (B = 2x)")
    ap.add_argument("--cfg5-eval", type=int, default=18,
                    help="default line: iterations between evaluations of the batch")
    ap.add_argument("--cfg5-root-eval", type=int, default=24,
                    help="default line: evaluation interval of the root solve (the candidates "
                         "come from its point, so they do not depend on the batch's options)")
    ap.add_argument("--cfg5-stop-every", type=int, default=6,
                    help="default line: stopping tests every S iterations between evaluations "
                         "(0: off)")
    ap.add_argument("--cfg5-draw-seed", type=int, default=100,
                    help="default line: first seed offset of the candidate draws (other offsets "
                         "give independent draws, e.g. to choose the evaluation interval on)")
    ap.add_argument("--cfg5-mixed-draws", type=int, default=3,
                    help="default line: draws solved again with FP32 iterates (0: none)")
    ap.add_argument("--cfg5-mixed-iters", type=int, default=3000,
                    help="default line: iteration cap of the FP32-iterate run")
    ap.add_argument("--cfg5-cpu-lps", type=int, default=1024,
                    help="default line: LPs of the first draws solved by the reference solver "
                         "on the host")
    ap.add_argument("--cfg5-plain-eval", type=int, default=8,
                    help="default line: iterations between evaluations of the one-at-a-time leg")
    ap.add_argument("--line-serve-rates", default="10,100",
                    help="default line: Poisson request rates of the serving sub-object")
    ap.add_argument("--line-serve-seconds", type=float, default=5.0)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-obbt", action="store_true")
    ap.add_argument("--no-fsb2", action="store_true")
    ap.add_argument("--fsb2-m", type=int, default=2000,
                    help="rows of the strong-branching family's matrix (n = 2.5 m; 2000 is the benchmark's)")
    ap.add_argument("--tail-cols", type=int, default=0,
                    help="persistent tail once at most this many LPs of a batch run (0: off)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # ten untimed steps: one per candidate draw of the line, so that every launch
    # shape a draw reaches is captured (and its tiles timed) before the timed steps
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-lps", type=int, default=256)
    ap.add_argument("--no-spmm", action="store_true",
                    help="skip the 200k x 500k product-kernel point")
    ap.add_argument("--tile-lanes", type=int, default=0, help="fixed lanes per row group (0: auto)")
    ap.add_argument("--tile-vec", type=int, default=0, help="fixed LPs per lane (0: auto)")
    ap.add_argument("--plain-lps", type=int, default=64, help="LPs of the batch solved one at a time")
    ap.add_argument("--graphs", type=int, default=1)
    return ap


def main():
    args = make_parser().parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; the batch shards by LP columns with no "
              "communication, so N GPUs give N independent copies of this measurement",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "sweep":
        run_sweep(args)
        return
    if args.workload == "copy":
        run_copy(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return
    if args.workload == "structured":
        run_structured(args)
        return
    if args.workload == "trace-summary":
        run_trace_summary(args)
        return
    if args.workload == "pmc-summary":
        run_pmc_summary(args)
        return
    if args.workload == "pmc-table":
        run_pmc_table(args)
        return
    if args.workload == "obbt":
        run_obbt(args)
        return
    if args.workload == "mixed":
        run_mixed(args)
        return
    if args.workload == "fsb2":
        print(json.dumps(fsb2_leg(args, with_cpu=True)), flush=True)
        return

    # the default line: the 200k x 500k strong-branching batch, then the other
    # workloads of the metric as sub-objects (each after its own warmup)
    line = headline(args)
    if not args.no_spmm:
        line["spmm_hbm"] = spmm_leg()
    if not args.no_serving:
        rates = [float(r) for r in args.line_serve_rates.split(",")]
        line["serving"] = serve_leg(args, rates, args.line_serve_seconds)
    if not args.no_obbt:
        line["bound_tightening_20kx50k"] = obbt_leg(args, steps=5, warmup=2)
    if not args.no_fsb2:
        sub = fsb2_leg(args, with_cpu=False)
        line["strong_branching_2kx5k"] = {k: sub[k] for k in (
            "value", "unit", "config", "plain", "batched_vs_plain", "step_ms", "iters",
            "roofline")}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
