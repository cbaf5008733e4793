#!/usr/bin/env python3
"""Benchmark: Torontonians/s and subset determinants/s at n = 30 (FP64).

One step = one full Torontonian of the n = 30 precision workload (2n x 2n =
60 x 60 complex128, squeezing r_i ~ U[0.3, 1.2], Haar interferometer, loss
eta = 0.9, seed 0; 2^30 subsets) through the C ABI, from a matrix already
resident in device memory: the staging kernel (validation, structure test,
packing), one persistent launch of the recursive kernel, the fixed-order
reduction and the copy of the result.  The same step from a host matrix
(its PCIe copy included) is reported beside it.  The input is synthetic
(seeded generator, no dataset).

Printed as one JSON line, with
* roofline: the recursive kernel's algorithmic FLOP (paper_2109_04528_amd/flops.py)
  over its average duration, measured with HIP events on the stream the kernel
  runs on, against the MI355X FP64 vector peak; beside it the HBM traffic and
  the FP64 FLOP the kernel issues, both from rocprofv3 counters recorded in
  profiles/ for the current kernel sources;
* plain: the per-subset-Cholesky comparison kernel on a sampled mask range;
* cpu_baseline: the CPU oracle timed on a bounded subtree of the same workload;
* with --serve, p50/p99 latency of a Poisson stream of mixed-n requests.
"""
import argparse
import gc
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Tor evals/s + subset dets/s at n=30 FP64; p50/p99 latency, mixed-n stream"
KERNEL_SOURCES = ["paper_2109_04528_amd/csrc/tor_kernels.hip", "paper_2109_04528_amd/csrc/tor_device.hpp",
                  "paper_2109_04528_amd/csrc/tor_internal.hpp"]
TRAFFIC_FILE = "profiles/tor_main_real_n30_traffic.md"
COUNTERS_FILE = "profiles/tor_main_real_n30_trace_and_counters.md"
COPY_BYTES = 256 << 20  # calibration copy for the HBM counters


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def stored_field(path, key):
    """A figure recorded in a profile summary (a "- key: value" line), valid
    only while the kernel sources hash to the summary's kernel_source_sha256."""
    path = os.path.join(ROOT, path)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(fields[key])
    except (KeyError, ValueError):
        return None


def stored_traffic():
    """HBM bytes per launch of the recursive kernel measured with rocprofv3
    (FETCH_SIZE + WRITE_SIZE, calibrated on a copy of known size)."""
    return stored_field(TRAFFIC_FILE, "hbm_bytes_per_launch")


def stored_issued_flop():
    """FP64 FLOP the recursive kernel issues per launch, from the
    SQ_INSTS_VALU_{FMA,MUL,ADD}_F64 counters (64 lanes per instruction, an FMA
    counting 2): the vector unit's own work, exclude lanes and masked lanes
    included, as opposed to the algorithmic FLOP of the method."""
    return stored_field(COUNTERS_FILE, "issued_fp64_flop_per_launch")


FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 FLOP/clk


def cpu_baseline(O, n, budget_s=12.0):
    """The CPU oracle (as it stands) on a subtree of the workload: modes
    0..k-1 fixed to an alternating include pattern, the rest enumerated."""
    from oracle import oracle as orc
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()

    def run(m):
        k = n - m
        fix_mask = (1 << k) - 1
        fix_val = sum(1 << i for i in range(0, k, 2))
        t0 = time.perf_counter()
        r = orc.tor(O, mode=orc.F64, threads=cores, fix_mask=fix_mask, fix_val=fix_val)
        return time.perf_counter() - t0, r.count, k

    # a calibration run long enough that thread start-up does not dominate,
    # then the subtree whose size is nearest the budget (0.7x..1.4x of it)
    dt, cnt, _ = run(min(18, n - 2))
    rate = cnt / max(dt, 1e-9)
    m = int(round(math.log2(max(rate * budget_s, 1 << 12))))
    m = max(12, min(m, n - 2))
    dt, cnt, k = run(m)
    dets = cnt / dt
    return {"value": dets / float(1 << n), "unit": "Tor/s", "cores": cores, "kind": "oracle",
            "subset_dets_per_s": dets, "seconds": dt,
            "sample": f"{cnt} subsets of the n={n} workload (modes 0..{k - 1} fixed, alternating "
                      f"include pattern), FP64 Cholesky per subset, __float128 sum, {cores} threads"}


def serve_requests(count, seed):
    """Click submatrices O_S of 40-mode Gaussian states (r ~ U[.5, 1],
    eta ~ U[.3, 1], one state per 8 requests), S a uniform n-subset, n ~ U{8..32}."""
    import numpy as np
    from paper_2109_04528_amd import inputs as gen
    rng = np.random.default_rng(seed)
    states = [gen.random_O(40, 5000 + i, 0.5, 1.0, float(rng.uniform(0.3, 1.0))) for i in range(count // 8 + 1)]
    reqs = []
    for i in range(count):
        n = int(rng.integers(8, 33))
        S = sorted(rng.choice(40, size=n, replace=False).tolist())
        reqs.append(gen.click_submatrix(states[i // 8], S))
    return reqs


def serve_saturated(ctx, reqs):
    """All requests submitted at once: the stream's saturated throughput."""
    t0 = time.perf_counter()
    tickets = [ctx.submit(O) for O in reqs]
    ctx.drain(-1)
    wall = time.perf_counter() - t0
    for t in tickets:
        ctx.poll(t)
    return len(reqs) / wall


def serve_stream(ctx, reqs, seed, rate_hz):
    """Poisson arrivals at rate_hz; latency = scheduled arrival to completed
    poll.  The client polls its pending tickets about every 0.1 ms (a 50 us
    sleep between rounds), so each latency includes up to that much of its
    own polling."""
    import numpy as np
    count = len(reqs)
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    t_sub = {}
    lat = []
    pending = {}
    t0 = time.perf_counter()
    nxt = t0
    i = 0
    while i < count or pending:
        now = time.perf_counter()
        while i < count and now >= nxt:
            tk = ctx.submit(reqs[i])
            t_sub[tk] = nxt  # open loop: latency counts from the scheduled arrival
            pending[tk] = i
            nxt += gaps[i]
            i += 1
        for tk in list(pending):
            r = ctx.poll(tk)
            if r is not None:
                lat.append(time.perf_counter() - t_sub[tk])
                del pending[tk]
        time.sleep(0.00005)
    wall = time.perf_counter() - t0
    lat = sorted(lat)
    return {"requests": count, "rate_hz": rate_hz, "wall_s": wall, "tor_per_s": count / wall,
            "p50_ms": 1e3 * lat[len(lat) // 2], "p99_ms": 1e3 * lat[min(len(lat) - 1, int(0.99 * len(lat)))],
            "mean_ms": 1e3 * sum(lat) / len(lat), "max_ms": 1e3 * lat[-1]}


GOLDEN = "tests/golden/oracle_values.json"


def precision_report(stream, ws):
    """Relative errors of the FP64 and the double-double factor paths against
    the stored oracle values (tests/golden/oracle_values.json: __float128 at
    n = 10, 16, 20, x87 extended at n = 24 and 30), with R, each result's
    err_est and the tolerance the tests use (6 standard deviations of
    4 sqrt(u_gpu^2 + u_oracle^2) sqrt(sum t^2)).  At n = 24 and 30 the
    double-double figure is bounded by the extended reference's own rounding
    (about 2^-64 sqrt(sum t^2))."""
    import numpy as np
    from paper_2109_04528_amd import TOR_FACTOR_DD, Context, inputs
    gold = json.load(open(os.path.join(ROOT, GOLDEN)))
    unit = {"quad": 2.0 ** -113, "ld": 2.0 ** -64, "f64": 2.0 ** -53}
    rows = []
    with Context(device=0, stream=stream, workspace=ws) as fc, \
            Context(device=0, stream=stream, workspace=ws, flags=TOR_FACTOR_DD) as qc:
        for name in sorted(gold):
            g = gold[name]
            if g["oracle_mode"] not in ("quad", "ld"):
                continue
            O = inputs.random_O(g["n"], g["seed"], g["r_lo"], g["r_hi"], g["eta"])
            if inputs.sha256(O) != g["sha256"]:
                raise RuntimeError(f"{name}: generator output differs from the stored input")
            want = g["tor_hi"] + g["tor_lo"]
            rf, rq = fc.eval(O), qc.eval(O)
            dq = (rq.tor - g["tor_hi"]) + (rq.tor_lo - g["tor_lo"])
            sq = math.sqrt(g["sum_sq"])
            rows.append({"case": name, "n": g["n"], "reference": g["oracle_mode"], "R": g["sum_abs"] / abs(want),
                         "fp64_rel_error": abs(rf.value - want) / abs(want), "fp64_err_est": rf.err_est,
                         "fp64_bound_rel": 24 * math.hypot(2.0 ** -53, unit[g["oracle_mode"]]) * sq / abs(want),
                         "dd_rel_error": abs(dq) / abs(want), "dd_err_est": rq.err_est,
                         "dd_bound_rel": 24 * math.hypot(2.0 ** -100, unit[g["oracle_mode"]]) * sq / abs(want),
                         "dd_kernel_ms": rq.device_ms})
    # one group per size and reference ("24" alone, or "24-ld" and "24-quad"
    # where a size has references of both kinds)
    refs = {}
    for row in rows:
        refs.setdefault(row["n"], set()).add(row["reference"])
    by_n = {}
    for row in rows:
        key = str(row["n"]) if len(refs[row["n"]]) == 1 else f"{row['n']}-{row['reference']}"
        by_n.setdefault(key, []).append(row)
    summary = {k: {"cases": len(v), "reference": v[0]["reference"],
                        "fp64_rel_error_max": max(x["fp64_rel_error"] for x in v),
                        "fp64_rel_error_median": float(np.median([x["fp64_rel_error"] for x in v])),
                        "dd_rel_error_max": max(x["dd_rel_error"] for x in v),
                        "R_max": max(x["R"] for x in v)}
               for k, v in sorted(by_n.items(), key=lambda kv: (int(kv[0].split("-")[0]), kv[0]))}
    return {"source": GOLDEN, "summary_by_n": summary, "cases": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--plain-masks", type=int, default=1 << 18)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--serve", type=int, default=4096, help="requests in the mixed-n stream (0: skip)")
    ap.add_argument("--batch", type=int, default=512, help="matrices in the batched launch (0: skip)")
    ap.add_argument("--n34", type=int, default=1, help="also time one n=34 Torontonian")
    ap.add_argument("--compare", type=int, default=1,
                    help="the n=24 pair workload by the append form, the paper's removal order and plain")
    ap.add_argument("--click", type=int, default=1024,
                    help="click-pattern probabilities of one 32-mode state (0: skip)")
    ap.add_argument("--click-all", type=int, default=2,
                    help="every click pattern of a 16- and a 24-mode state at once (1), and of the "
                         "32-mode state of the click block (2)")
    ap.add_argument("--quad", type=int, default=1,
                    help="also time the same n=30 Torontonian with the double-double factor")
    ap.add_argument("--precision", type=int, default=1,
                    help="errors of the FP64 and double-double paths against the stored oracle values")
    ap.add_argument("--compare-seeds", type=int, default=8, help="seeds of the n=24 method comparison")
    ap.add_argument("--profile-traffic", action="store_true",
                    help="one n=30 Torontonian and one 256 MiB device copy, for the HBM counters")
    ap.add_argument("--force-complex", action="store_true",
                    help="time the headline on the complex path (TOR_FORCE_COMPLEX), for its profile")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU only (asked for {args.gpus}); "
              "the subtree roots would shard across GPUs with one 16-byte reduction per Torontonian, "
              "but no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2109_04528_amd import TOR_FORCE_COMPLEX, TOR_INPUT_DEVICE, TOR_TUNE_REAL, Context, inputs, workspace_size
    from paper_2109_04528_amd.flops import plain_flops_per_subset, tor_flops

    n = args.n
    O = inputs.random_O(n, 0, 0.3, 1.2, 0.9)
    print(f"bench: n={n} workload staged", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    if args.profile_traffic:
        with Context(device=0) as c:
            c.eval(O)
        src = torch.empty(COPY_BYTES, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_traffic": True, "copy_bytes": COPY_BYTES,
                          "kernel_source_sha256": kernel_source_hash()}), flush=True)
        return
    stream = torch.cuda.Stream(device=dev)
    ws = torch.empty(workspace_size(max(n, 32), 0, 4), dtype=torch.uint8, device=dev)
    # the input resident in HBM before the timed region: the staging kernel
    # reads it in place
    O_dev = torch.from_numpy(O).to(dev)
    torch.cuda.synchronize()
    path_flags = TOR_FORCE_COMPLEX if args.force_complex else 0
    dctx = Context(device=0, stream=stream, workspace=ws, flags=TOR_INPUT_DEVICE | path_flags)
    # the library runs on `stream`; making it torch's current stream as well
    # orders the device input's reads without a wait per call
    torch.cuda.set_stream(stream)
    # the collector runs before the warm-up: a pause between warm-up and the
    # timed steps would let the GPU clocks fall again
    gc.collect()
    for _ in range(args.warmup):
        dctx.eval(O_dev)
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = dctx.eval(O_dev)
        kms.append(r.device_ms)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"bench: {args.steps} steps done", file=sys.stderr, flush=True)
    step_s = (t1 - t0) / args.steps
    fma_tflops, _ = dctx.fma_peak()  # the FP64 peak confirmed on this device
    dctx.close()
    # the same step from a host matrix (its PCIe copy included), for context
    ctx = Context(device=0, stream=stream, workspace=ws, flags=path_flags)
    ctx.eval(O)
    torch.cuda.synchronize()
    th = time.perf_counter()
    for _ in range(args.steps):
        ctx.eval(O)
    host_step_s = (time.perf_counter() - th) / args.steps
    tor_per_s = 1.0 / step_s
    kernel_ms = float(np.mean(kms))
    real_path = r.path == 1
    flops = tor_flops(n, real=real_path)
    achieved = flops / (kernel_ms * 1e-3) / 1e12
    # profiled figures hold for the real-path kernel on the n = 30 workload only
    profiled = real_path and n == 30
    traffic = stored_traffic() if profiled else None
    issued = stored_issued_flop() if profiled else None

    plain = None
    if args.plain_masks > 0 and n <= 34:
        m = min(args.plain_masks, 1 << n)
        lo = (1 << n) // 2 - m // 2  # a contiguous mask range from the middle
        ctx.eval_plain(O, lo, lo + m)
        p = ctx.eval_plain(O, lo, lo + m)
        plain_dets = m / (p.device_ms * 1e-3)
        plain_real = p.path == 1
        plain_tflops = plain_dets * plain_flops_per_subset(n, real=plain_real) / 1e12
        plain = {"masks": m, "kernel_ms": p.device_ms, "subset_dets_per_s": plain_dets,
                 "form": "real quadrature" if plain_real else "complex",
                 "tflops": plain_tflops, "frac": plain_tflops / FP64_PEAK_TFLOPS,
                 "recursive_speedup": ((1 << n) / (kernel_ms * 1e-3)) / plain_dets}
        print("bench: plain comparison done", file=sys.stderr, flush=True)

    batch = None
    if args.batch > 0:
        ns, mats = inputs.batch_mix(args.batch, 12, 26, seed=4)
        # median of three calls, with Python's collector run beforehand (a
        # collection pause inside one call is the interpreter's, not the
        # library's), after one call that sizes the workspace and buffers
        gc.collect()
        ctx.eval_batch(mats)
        torch.cuda.synchronize()
        calls = []
        for _ in range(3):
            t0 = time.perf_counter()
            res = ctx.eval_batch(mats)
            calls.append(time.perf_counter() - t0)
        sec = float(np.median(calls))
        # the same calls on a context whose autotuner has picked (k, waves/CU)
        # for every size of the mix on this device (tuning time reported apart)
        with Context(device=0, stream=stream) as tctx:
            ta = time.perf_counter()
            tctx.autotune(12, 26, TOR_TUNE_REAL)
            tune_s = time.perf_counter() - ta
            gc.collect()
            tctx.eval_batch(mats)
            torch.cuda.synchronize()
            tcalls = []
            for _ in range(3):
                t0 = time.perf_counter()
                tres = tctx.eval_batch(mats)
                tcalls.append(time.perf_counter() - t0)
        tsec = float(np.median(tcalls))
        subsets = sum(1 << n for n in ns)
        batch = {"matrices": args.batch, "n_range": [12, 26], "seconds": tsec,
                 "tor_per_s": args.batch / tsec, "subset_dets_per_s": subsets / tsec,
                 "kernel_ms": max(r.device_ms for r in tres), "launches": len({r.path for r in tres}),
                 "autotuned": True, "autotune_s": tune_s,
                 "untuned_seconds": sec, "untuned_kernel_ms": max(r.device_ms for r in res)}
        print("bench: batch done", file=sys.stderr, flush=True)

    big = None
    if args.n34:
        O34 = inputs.random_O(34, 0, 0.5, 1.0, 0.7)
        r34 = ctx.eval(O34)
        big = {"n": 34, "kernel_ms": r34.device_ms, "subset_dets_per_s": (1 << 34) / (r34.device_ms * 1e-3),
               "tor": r34.value, "cancellation_R": r34.cancellation, "err_est": r34.err_est,
               "note": "FP64 factor: at this R only TOR_FACTOR_DD gives a meaningful value"}
        print("bench: n=34 done", file=sys.stderr, flush=True)

    compare = None
    if args.compare:
        # the pair workload, seeds 0..7: the append form (real and complex),
        # the paper's removal order and a fresh factorisation per subset
        # (complex, as the removal order is), kernel times
        from paper_2109_04528_amd.flops import removal_flops
        rows = []
        with Context(device=0, stream=stream, workspace=ws, flags=TOR_FORCE_COMPLEX) as cc:
            for seed in range(args.compare_seeds):
                O24 = inputs.random_O(24, seed, 0.5, 1.0, 0.7)
                ctx.eval(O24)
                ra = ctx.eval(O24)
                ctx.eval_removal(O24)
                rr = ctx.eval_removal(O24)
                cc.eval(O24)
                rc_ = cc.eval(O24)
                rp = cc.eval_plain(O24)
                rows.append({"seed": seed, "append_real_ms": ra.device_ms, "append_complex_ms": rc_.device_ms,
                             "removal_order_ms": rr.device_ms, "plain_ms": rp.device_ms})
        med = {k: float(np.median([row[k] for row in rows]))
               for k in ("append_real_ms", "append_complex_ms", "removal_order_ms", "plain_ms")}
        compare = {"workload": f"n=24, r~U[0.5,1], eta=0.7, seeds 0..{args.compare_seeds - 1} (2^24 subsets each), "
                               "kernel times, medians over the seeds",
                   **med, "per_seed": rows,
                   "removal_tflops": removal_flops(24) / (med["removal_order_ms"] * 1e-3) / 1e12,
                   "removal_over_plain": med["plain_ms"] / med["removal_order_ms"],
                   "append_complex_over_removal": med["removal_order_ms"] / med["append_complex_ms"],
                   "append_real_over_removal": med["removal_order_ms"] / med["append_real_ms"],
                   "append_real_over_plain": med["plain_ms"] / med["append_real_ms"]}
        print("bench: method comparison done", file=sys.stderr, flush=True)

    quad = None
    if args.quad:
        from paper_2109_04528_amd import TOR_FACTOR_DD
        with Context(device=0, stream=stream, workspace=ws, flags=TOR_FACTOR_DD) as qc:
            qc.eval(O)
            qms = [qc.eval(O).device_ms for _ in range(3)]
            rq = qc.eval(O)
        qms_med = float(np.median(qms))
        # the FP64 result's actual error, measured against the double-double one
        quad = {"n": n, "kernel_ms": qms_med, "tor_per_s": 1e3 / qms_med,
                "subset_dets_per_s": (1 << n) / (qms_med * 1e-3),
                "alg_dd_ops_per_s": tor_flops(n, real=True) / (qms_med * 1e-3),
                "tor_hi": rq.tor, "tor_lo": rq.tor_lo, "err_est": rq.err_est,
                "fp64_path_rel_error": abs(r.value - rq.value) / abs(rq.value),
                "factor": "double-double (TOR_FACTOR_DD), real quadrature form; alg_dd_ops_per_s counts "
                          "the FP64 path's algorithmic operations, each done in double-double"}
        print("bench: double-double factor done", file=sys.stderr, flush=True)

    precision = None
    if args.precision:
        precision = precision_report(stream, ws)
        print("bench: precision report done", file=sys.stderr, flush=True)

    click = None
    if args.click > 0:
        # patterns S of a 32-mode state (r ~ U[.5, 1], eta = .7, seed 9), |S| ~ U{4..28}
        Oc = inputs.random_O(32, 9, 0.5, 1.0, 0.7)
        crng = np.random.default_rng(10)
        pats = [crng.choice(32, size=int(crng.integers(4, 29)), replace=False).tolist()
                for _ in range(args.click)]
        ctx.click_probs(Oc, pats[:8])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        probs, cres = ctx.click_probs(Oc, pats)
        t1 = time.perf_counter()
        subsets = sum(1 << len(p) for p in pats)
        click = {"modes": 32, "patterns": args.click, "clicks_range": [4, 28], "seconds": t1 - t0,
                 "patterns_per_s": args.click / (t1 - t0), "subset_dets_per_s": subsets / (t1 - t0),
                 "kernel_ms": max(r.device_ms for r in cres), "min_prob": float(probs.min())}
        print("bench: click probabilities done", file=sys.stderr, flush=True)

    click_all = None
    if args.click_all:
        # every pattern of one state at once (tor_click_all), against the same
        # patterns one by one (tor_click_probs) where that is still feasible;
        # states r ~ U[.5, 1], eta = .7
        click_all = {}
        # its own context: the terms and sums need 24 * 2^M bytes of workspace,
        # which the library grows on demand
        actx = Context(device=0, stream=stream)
        for M, direct in ((16, True), (24, False)):
            Oa = inputs.random_O(M, 11, 0.5, 1.0, 0.7)
            actx.click_all(Oa)
            t0 = time.perf_counter()
            pa, _, ra = actx.click_all(Oa)
            t1 = time.perf_counter()
            row = {"modes": M, "patterns": 1 << M, "seconds": t1 - t0, "device_ms": ra.device_ms,
                   "subset_dets": 1 << M, "subset_dets_one_by_one": 3 ** M,
                   "sum_of_probs": math.fsum(pa)}
            if direct:
                actx.click_probs(Oa, range(256))
                t0 = time.perf_counter()
                pd, _ = actx.click_probs(Oa, range(1 << M))
                t1 = time.perf_counter()
                row["one_by_one_seconds"] = t1 - t0
                row["speedup"] = row["one_by_one_seconds"] / row["seconds"]
                row["max_prob_difference"] = float(np.max(np.abs(pa - pd)))
            click_all[f"M{M}"] = row
        actx.close()
        if args.click_all > 1:
            # every pattern of the 32-mode state of the click block (r ~ U[.5, 1],
            # eta = .7, seed 9): 96 GiB of workspace, the probabilities left
            # in device memory (32 GiB), one call after a sizing call
            from paper_2109_04528_amd import TOR_OUTPUT_DEVICE, TorError
            Ob = inputs.random_O(32, 9, 0.5, 1.0, 0.7)
            try:
                with Context(device=0, stream=stream, flags=TOR_OUTPUT_DEVICE) as bctx:
                    bctx.click_all(Ob)
                    t0 = time.perf_counter()
                    pb, _, rb = bctx.click_all(Ob)
                    t1 = time.perf_counter()
                    click_all["M32"] = {"modes": 32, "patterns": 1 << 32, "seconds": t1 - t0,
                                        "device_ms": rb.device_ms, "sum_of_probs": float(torch.sum(pb).item()),
                                        "outputs": "device"}
                    del pb
            except (TorError, RuntimeError) as err:  # the library's or torch's allocation
                click_all["M32"] = {"error": str(err)}
        print("bench: every click pattern done", file=sys.stderr, flush=True)

    serve = None
    if args.serve > 0:
        reqs = serve_requests(args.serve, 5)
        sat = serve_saturated(ctx, reqs)
        rate = 0.7 * sat
        serve = serve_stream(ctx, reqs, 6, rate_hz=rate)
        serve["saturated_tor_per_s"] = sat
        serve["arrivals"] = "Poisson at 0.7 x saturated throughput of the same mix"
        print("bench: serving done", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(O, n, args.cpu_budget)
        print("bench: cpu baseline done", file=sys.stderr, flush=True)

    ctx.close()
    out = {
        "metric": METRIC,
        "value": tor_per_s,
        "unit": "Tor/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"exact Torontonian, n={n} modes (60x60 complex128 for n=30), r~U[0.3,1.2], "
                               f"Haar U, eta=0.9, seed 0, 2^{n} subsets per step", "n": n,
                   "subsets_per_step": 1 << n,
                   "path": ("recursive, real quadrature form" if real_path else "recursive, complex") +
                           " FP64 factor, double-double sum"},
        "subset_dets_per_s": (1 << n) * tor_per_s,
        "input": "device-resident (TOR_INPUT_DEVICE), staged on the GPU inside each step",
        "host_input_ms_per_step": host_step_s * 1e3,
        "kernel_ms": kernel_ms,
        "kernel_subset_dets_per_s": (1 << n) / (kernel_ms * 1e-3),
        "tor": r.value,
        "cancellation_R": r.cancellation,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                     "peak_measured": fma_tflops, "frac_of_measured": achieved / fma_tflops,
                     "flop_per_launch": flops,
                     "issued_flop_per_launch": issued,
                     "issued_frac": None if issued is None else issued / (kernel_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                     "kernel": "tor_main<double, T=5, B=6, L=2>" if real_path else "tor_main<c64, T=3, B=6, L=2>"},
        "plain": plain,
        "batch": batch,
        "n34": big,
        "quad": quad,
        "precision": precision,
        "click": click,
        "click_all": click_all,
        "compare_n24": compare,
        "serving": serve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
