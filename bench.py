#!/usr/bin/env python3
"""Benchmark: order-0 discrete Hankel transform at N = 2^20, eps = 1e-8 on one MI355X.

A step is one complete transform f = J_0(j_0 j_0^T / j_{0,N+1}) c of one
seeded synthetic coefficient vector (c_n iid N(0,1), the paper's Sec. 6.1
workload), input and output resident in HBM.  Prints one JSON line with
points/s (N output points per transform), the roofline of the dominant
kernel (HIP-event timing inside the timed region), and the CPU oracle timed
on a bounded row sample on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VECTOR_TFLOPS = 78.6      # MI355X FP64 vector peak
# measured HBM traffic per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by
# a plain copy of known size), valid while the kernel sources are unchanged
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
KERNEL_SOURCES = ["paper_1501_01652_amd/csrc/kernels.hip", "paper_1501_01652_amd/csrc/fft_device.h",
                  "paper_1501_01652_amd/csrc/device_common.h", "paper_1501_01652_amd/csrc/kernels.h"]
COPY_BYTES = 1 << 30           # the calibration copy (--only copy)
METRIC = "DHT0 points/sec at N=2^20, ε=1e-8 vs direct; batched p50/p99 latency"


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None if there is none or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    k = t.get("kernels", {}).get(kernel)
    if k is None or t.get("source_hash") != kernel_source_hash():
        return None
    return 1024.0 * (k["fetch_kib"] * t["fetch_scale"] + k["write_kib"] * t["write_scale"])


def run_copy(torch):
    """A plain device copy of COPY_BYTES, to calibrate the HBM byte counters."""
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"copy_bytes": COPY_BYTES, "copies": 3}


def write_traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, command):
    """Build TRAFFIC_FILE from rocprofv3 --pmc counter collections (csv):
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the headline run and of
    the calibration copy (--only copy), whose true traffic is COPY_BYTES each way."""
    import csv

    def per_kernel(path, counter):
        acc = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                name = r["Kernel_Name"].split("(")[0].split("<")[0].replace("void ", "").replace("hank::", "")
                acc.setdefault(name.strip(), []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}

    def copy_kib(path, counter):
        vals = per_kernel(path, counter)
        return max(vals.values())  # the copy is the largest dispatch of that run

    fscale = (COPY_BYTES / 1024.0) / copy_kib(copy_fetch_csv, "FETCH_SIZE")
    wscale = (COPY_BYTES / 1024.0) / copy_kib(copy_write_csv, "WRITE_SIZE")
    f, w = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    kernels = {k: {"fetch_kib": f[k], "write_kib": w.get(k, 0.0)} for k in f if k.startswith("k_")}
    out = {"source_hash": kernel_source_hash(), "fetch_scale": fscale, "write_scale": wscale,
           "command": command, "kernels": kernels}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--task", default="dht0")
    ap.add_argument("--N", type=int, default=1 << 20)
    ap.add_argument("--eps", type=float, default=1e-8)
    ap.add_argument("--plan-mode", type=int, default=0)
    ap.add_argument("--precision", type=int, default=1,
                    help="1: every far transform in FP64 (the headline); 0: the library's automatic choice")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-direct", action="store_true")
    ap.add_argument("--batch-count", type=int, default=1024, help="requests of the batched workload (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="arrival window of the serving run (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--only", choices=["all", "headline", "batched", "serve", "copy", "ablation", "configs"],
                    default="all")
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads (configs block)")
    ap.add_argument("--oracle-rows", type=int, default=48,
                    help="sampled output rows per large workload on which the CPU oracle is timed and "
                         "the GPU result is compared")
    ap.add_argument("--write-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write the HBM traffic summary from rocprofv3 counter csv files and exit")
    return ap.parse_args()


def run_batched(hank, inputs, torch, count):
    """1024 uneven transforms in one hank_batch call against the same requests
    one call at a time; throughput and per-request completion latency (all
    submitted at t = 0)."""
    specs = inputs.batch_specs(count)
    reqs = []
    for sp in specs:
        g = torch.Generator(device="cuda").manual_seed(sp["seed"])
        shape = (sp["nrhs"], sp["N"]) if sp["nrhs"] > 1 else (sp["N"],)
        c = torch.rand(shape, generator=g, dtype=torch.float64, device="cuda") * 2.0 - 1.0
        reqs.append({"task": sp["task"], "c": c, "out": torch.empty_like(c), "eps": sp["eps"]})
    t0 = time.perf_counter()
    hank.batch(reqs)  # builds every plan, then runs
    torch.cuda.synchronize()
    warm_s = time.perf_counter() - t0
    reps = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        hank.batch(reqs)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    # the same batch captured once as a HIP graph and replayed
    graph = hank.BatchGraph(reqs)
    graph.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        graph.launch()
    torch.cuda.synchronize()
    tg = (time.perf_counter() - t0) / reps
    graph.close()
    # one request at a time, same stream, completion stamped by events
    for r in reqs:
        hank.transform(r["task"], r["c"], r["eps"], out=r["out"])
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in reqs]
    start.record()
    for r, e in zip(reqs, evs):
        hank.transform(r["task"], r["c"], r["eps"], out=r["out"])
        e.record()
    torch.cuda.synchronize()
    lat = sorted(start.elapsed_time(e) for e in evs)
    ts = lat[-1] / 1e3
    pct = lambda q: lat[min(len(lat) - 1, int(q * (len(lat) - 1) + 0.5))]
    return {"requests": count, "rhs_total": int(sum(sp["nrhs"] for sp in specs)),
            "workload": "task 40/40/20, N log-uniform [2^8, 2^16], 1-64 rhs, eps {1e-4,1e-8,1e-14}, "
                        "c ~ U[-1,1], seed %d" % inputs.SEED_BATCH,
            "batched_transforms_per_s": count / tb, "batched_ms": tb * 1e3,
            "graph_transforms_per_s": count / tg, "graph_ms": tg * 1e3,
            "batched_latency_p50_ms": tb * 1e3, "batched_latency_p99_ms": tb * 1e3,
            "sequential_transforms_per_s": count / ts, "sequential_ms": ts * 1e3,
            "sequential_latency_p50_ms": pct(0.5), "sequential_latency_p99_ms": pct(0.99),
            "speedup": ts / tb, "first_call_incl_planning_s": warm_s}


def _median_ms(hank, torch, task, c, eps, out, reps, **kw):
    hank.transform(task, c, eps, out=out, **kw)  # plan build and warm-up
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    stream = torch.cuda.current_stream()
    evs[0].record(stream)
    for i in range(reps):
        hank.transform(task, c, eps, out=out, stream=stream, **kw)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    return sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(reps))[reps // 2]


def run_ablation(hank, inputs, torch, task, N, eps, c_host, precision=1):
    """Cost-model ablations: the tuned partition against the paper's (Table 4)
    and against one far block (P = 0, Sec. 3.3) on the headline workload; and
    the M sweep of Sec. 4.3 (Schlomilch, N = 5000, paper plan, M = 1..20)."""
    c = torch.from_numpy(c_host).to("cuda")
    out = torch.empty_like(c)
    part = {}
    for name, mode in (("tuned", 0), ("paper", 1), ("single_partition", 2)):
        info = hank.plan_info(task, N, eps, plan_mode=mode, precision=precision)
        ms = _median_ms(hank, torch, task, c, eps, out, 5, plan_mode=mode, precision=precision)
        part[name] = {"ms": ms, "points_per_s": N / (ms * 1e-3), "M": info["M"], "P": info["P"],
                      "blocks": info["nblocks"], "near_entries": info["near_entries"],
                      "far_transforms": info["far_transforms"], "fft_bytes": info["fft_bytes"]}
    del c, out
    hank.cache_clear()
    Ns = 5000
    cs = torch.from_numpy(inputs.coefficients("gauss", Ns, inputs.SEED_SCHLOMILCH)).to("cuda")
    outs = torch.empty_like(cs)
    sweep = {}
    for e in (1e-15, 1e-11, 1e-7, 1e-3):
        ms = {}
        for M in range(1, 21):
            ms[M] = _median_ms(hank, torch, "schlomilch", cs, e, outs, 5, plan_mode=1, M=M)
        best = min(ms, key=ms.get)
        table4 = hank.plan_info("schlomilch", Ns, e, plan_mode=1)["M"]
        sweep["%g" % e] = {"ms_by_M": ms, "best_M": best, "table4_M": table4,
                           "table4_over_best": ms[table4] / ms[best],
                           "tuned_ms": _median_ms(hank, torch, "schlomilch", cs, e, outs, 5)}
    direct_ms = _median_ms(hank, torch, "schlomilch", cs, 1e-15, outs, 5, direct=1)
    hank.cache_clear()
    return {"partition": part,
            "m_sweep": {"workload": "schlomilch N=%d, c_n iid N(0,1) seed %d, paper plan" % (Ns, inputs.SEED_SCHLOMILCH),
                        "by_eps": sweep, "direct_ms": direct_ms}}


def run_serve(hank, inputs, torch, seconds, rate, max_batch):
    """Open-loop Poisson arrivals through the continuous-batching server."""
    trace = inputs.serve_trace(rate=rate, seconds=seconds)
    sizes = sorted({t["N"] for t in trace})
    cin = {}
    pool = {}
    for N in sizes:
        g = torch.Generator(device="cuda").manual_seed(inputs.SEED_SERVE + N)
        cin[N] = torch.randn(N, generator=g, dtype=torch.float64, device="cuda")
        pool[N] = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in range(max_batch + 1)]
    srv = hank.Server(budget_bytes=32 << 30, max_batch=max_batch, max_pending=256)
    seen = {}
    for t in trace:  # plans on the device before the clock starts
        key = (t["task"], t["N"], t["eps"])
        if key not in seen:
            seen[key] = True
            srv.warm({"task": t["task"], "c": cin[t["N"]], "out": pool[t["N"]][0], "eps": t["eps"]})
    count = {}
    for t in trace:
        i = count.get(t["N"], 0)
        count[t["N"]] = i + 1
        srv.submit({"task": t["task"], "c": cin[t["N"]], "out": pool[t["N"]][i % (max_batch + 1)],
                    "eps": t["eps"]}, arrival_s=t["arrival"])
    srv.start()
    srv.drain()
    st = srv.stats()
    srv.close()
    st["offered_rate"] = rate
    st["window_s"] = seconds
    st["max_batch"] = max_batch
    return st


def step_times(hank, torch, task, c, eps, out, steps, warmup, **kw):
    """Per-step durations (ms) of `steps` transforms after `warmup` untimed
    ones (the first call builds the plan), with events between steps only."""
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    hank.transform(task, c, eps, out=out, **kw)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    for _ in range(warmup):
        hank.transform(task, c, eps, out=out, **kw)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(steps):
        hank.transform(task, c, eps, out=out, stream=stream, **kw)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)], wall, plan_s


def quantile(xs, q):
    ys = sorted(xs)
    return ys[min(len(ys) - 1, int(q * (len(ys) - 1) + 0.5))]


class CpuBaseline:
    """The CPU leg: the oracle (plain FP64 direct sums on the host cores) timed
    on bounded row samples of each workload.  Its rows also give the measured
    error constant C = max|f - f_oracle| / (eps sum|c|) of the GPU results on
    the same rows."""

    def __init__(self, nthreads=None):
        import oracle
        self.oracle = oracle
        self.nthreads = nthreads or oracle.default_threads()
        self.cache = {}

    def rows(self, task, c_host, rows):
        key = (task, c_host.shape[0], float(c_host[0]), np_bytes(rows))
        if key not in self.cache:
            self.oracle.eval_rows(task, c_host, rows=rows[:1], nthreads=1)  # roots set-up off the clock
            t0 = time.perf_counter()
            ref = self.oracle.eval_rows(task, c_host, rows=rows, nthreads=self.nthreads)
            self.cache[key] = (ref, time.perf_counter() - t0)
        return self.cache[key]


def np_bytes(a):
    import hashlib
    return hashlib.sha256(a.tobytes()).hexdigest()


def error_stats(np, f_rows, ref, c_host, eps):
    err = float(np.max(np.abs(f_rows - ref)))
    return {"max_abs_err": err, "C_l1": err / (eps * float(np.sum(np.abs(c_host)))),
            "C_l2": err / (eps * float(np.sqrt(np.sum(c_host * c_host))))}


def sample_rows(hank, inputs, task, N, eps, count, **kw):
    """Rows to check: first and last rows, +-2 around every far block's first
    row, and uniform ones (seeded)."""
    info = hank.plan_info(task, N, eps, **kw)
    bounds = []
    for k in range(info["nblocks"]):
        b = hank.plan_block(task, N, eps, k, **kw)
        bounds += [b["row0"], b["row1"]]
    return inputs.sampled_rows(N, count, boundaries=bounds, seed=inputs.SEED_SAMPLED_ROWS)


def run_config(hank, inputs, torch, np, cpu, task, N, eps, precision, c_host, rows, steps=10, warmup=2):
    """One workload: median/p90 time, points/s, the plan, and (with a CPU leg)
    the measured error on the sampled rows."""
    c = torch.from_numpy(c_host).to("cuda")
    out = torch.empty_like(c)
    kw = dict(precision=precision)
    ts, _, plan_s = step_times(hank, torch, task, c, eps, out, steps, warmup, **kw)
    info = hank.plan_info(task, N, eps, **kw)
    rec = {"task": task, "N": N, "eps": eps, "precision": {0: "auto", 1: "fp64", 2: "fp32"}[precision],
           "ms": quantile(ts, 0.5), "ms_p90": quantile(ts, 0.9), "points_per_s": N / (quantile(ts, 0.5) * 1e-3),
           "plan_build_s": plan_s,
           "plan": {"blocks": info["nblocks"], "near_entries": info["near_entries"],
                    "far_transforms": info["far_transforms"], "fp32_transforms": info["fp32_transforms"],
                    "fft_bytes": info["fft_bytes"]}}
    if cpu is not None:
        ref, tcpu = cpu.rows(task, c_host, rows)
        f = out.cpu().numpy()[rows - 1]
        rec["error"] = error_stats(np, f, ref, c_host, eps)
        rec["error"]["rows_checked"] = int(len(rows))
        rec["cpu_oracle_rows_per_s"] = len(rows) / tcpu
    del c, out
    return rec


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU; runs on several GPUs are not supported "
              "(got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.write_traffic:
        cmd = ("rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -- python3 bench.py "
               "--only headline --steps 2 --warmup 1 --no-cpu --no-direct; the same for --only copy")
        print(json.dumps(write_traffic(*args.write_traffic, command=cmd)))
        return
    import numpy as np
    import torch

    import paper_1501_01652_amd as hank
    from paper_1501_01652_amd import inputs

    extra = {}
    cpu = None if args.no_cpu else CpuBaseline()

    def run_extra():
        if args.only in ("all", "batched") and args.batch_count > 0:
            extra["batched"] = run_batched(hank, inputs, torch, args.batch_count)
        if args.only in ("all", "serve") and args.serve_seconds > 0:
            extra["serving"] = {
                "workload": "Poisson %g req/s for %g s, task 40/40/20, N in {2^10..2^22} log-uniform, 1 rhs, "
                            "eps {1e-4,1e-8,1e-14}, seed %d" % (args.serve_rate, args.serve_seconds,
                                                                inputs.SEED_SERVE),
                "continuous_batching": run_serve(hank, inputs, torch, args.serve_seconds, args.serve_rate, 64),
                "one_at_a_time": run_serve(hank, inputs, torch, args.serve_seconds, args.serve_rate, 1)}

    def run_configs():
        """The other workloads: Schlomilch N=4096 at 1e-14 (latency); Fourier-
        Bessel N=2^16 at 1e-14 and 1e-8 with an FP64 and an FP32 transform bulk
        side by side; the DHT at N=2^20 for eps 1e-4 (FP32 bulk, the automatic
        choice at eps >= 1e-6) and 1e-14 (FP64)."""
        out = []
        cs = inputs.workload("schlomilch", 4096)
        out.append(run_config(hank, inputs, torch, np, cpu, "schlomilch", 4096, 1e-14, 1, cs,
                              np.arange(1, 4097, dtype=np.int64), steps=50, warmup=5))
        cf = inputs.workload("fourier_bessel", 1 << 16)
        for e in (1e-14, 1e-8):
            rows = sample_rows(hank, inputs, "fourier_bessel", 1 << 16, e, 4 * args.oracle_rows, precision=1)
            for prec in (1, 2):
                out.append(run_config(hank, inputs, torch, np, cpu, "fourier_bessel", 1 << 16, e, prec, cf, rows))
        cd = inputs.workload("dht0", 1 << 20)
        for e, prec in ((1e-4, 0), (1e-14, 1)):
            rows = sample_rows(hank, inputs, "dht0", 1 << 20, e, args.oracle_rows, precision=prec)
            out.append(run_config(hank, inputs, torch, np, cpu, "dht0", 1 << 20, e, prec, cd, rows))
        hank.cache_clear()
        return out

    if args.only in ("batched", "serve"):
        run_extra()
        print(json.dumps(extra))
        return
    if args.only == "ablation":
        print(json.dumps(run_ablation(hank, inputs, torch, args.task, args.N, args.eps,
                                      inputs.workload(args.task, args.N))))
        return
    if args.only == "copy":
        print(json.dumps(run_copy(torch)))
        return
    if args.only == "configs":
        print(json.dumps({"configs": run_configs()}))
        return

    task, N, eps = args.task, args.N, args.eps
    c_host = inputs.workload(task, N)
    c = torch.from_numpy(c_host).to("cuda")
    out = torch.empty_like(c)
    stream = torch.cuda.current_stream()
    kw = dict(plan_mode=args.plan_mode, precision=args.precision)

    # timed region: K steps with events between steps only
    step_ms, elapsed, plan_s = step_times(hank, torch, task, c, eps, out, args.steps, args.warmup, **kw)
    f_head = out.cpu().numpy()
    # per-kernel durations: a second pass of K steps with HIP events around
    # every launch on the launch stream (kept out of the timed region above,
    # whose rate they would lower by about 4%)
    hank.profile(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(args.steps):
        hank.transform(task, c, eps, out=out, stream=stream, **kw)
    torch.cuda.synchronize()
    profiled_ms_per_step = 1e3 * (time.perf_counter() - t1) / args.steps
    stats = hank.profile_report()
    hank.profile(False)
    ms_per_step = 1e3 * elapsed / args.steps
    value = N * args.steps / elapsed
    step_q = lambda q: quantile(step_ms, q)
    info = hank.plan_info(task, N, eps, **kw)
    all_fp64 = info["fp32_transforms"] == 0 and not info["bulk_fp32"]

    # measured device copy bandwidth (read + write of COPY_BYTES), the
    # practical HBM ceiling beside the nominal peak
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * COPY_BYTES / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    # the whole plan against HBM: algorithmic bytes of its transforms (one read
    # and one write per FFT, two FFTs per transform) plus reading c and writing f
    plan_bytes = info["fft_bytes"] + 16.0 * N
    plan_gbs = plan_bytes / (step_q(0.5) * 1e-3) / 1e9
    plan_roofline = {"algorithmic_bytes": plan_bytes, "achieved_GBps": plan_gbs,
                     "frac_of_peak": plan_gbs / HBM_PEAK_GBS, "frac_of_copy": plan_gbs / copy_gbs,
                     "copy_GBps": copy_gbs}

    kernels = {}
    for s in stats:
        avg_ms = s["total_ms"] / max(1, s["launches"])
        k = {"launches": s["launches"], "avg_ms": avg_ms, "total_ms": s["total_ms"],
             "ms_per_step": s["total_ms"] / args.steps}
        if s["name"].startswith("pass") or s["name"] == "near_reduce":
            k["GB/s"] = s["bytes"] / (s["total_ms"] * 1e-3) / 1e9 if s["total_ms"] > 0 else None
        if s["name"] == "near":
            k["entries_per_s"] = s["work"] / (s["total_ms"] * 1e-3) if s["total_ms"] > 0 else None
        kernels[s["name"]] = k
    # the per-phase roofline of the plan: far-field passes against HBM, the
    # near field against the FP64 vector peak, summed
    far_bytes = sum(s["bytes"] for s in stats if s["name"].startswith("pass")) / args.steps
    far_ms = sum(s["total_ms"] for s in stats if s["name"].startswith("pass")) / args.steps
    near_s = [s for s in stats if s["name"] == "near"]
    near_flops = near_s[0]["work"] * NEAR_FLOPS_PER_ENTRY / args.steps if near_s else 0.0
    plan_roofline["phase_roofline_ms"] = 1e3 * (far_bytes / (HBM_PEAK_GBS * 1e9) +
                                                near_flops / (FP64_VECTOR_TFLOPS * 1e12))
    plan_roofline["far_passes_ms"] = far_ms
    plan_roofline["far_passes_GBps"] = far_bytes / (far_ms * 1e-3) / 1e9 if far_ms > 0 else None
    dom = max(stats, key=lambda s: s["total_ms"]) if stats else None
    roofline = None
    if dom is not None:
        if dom["name"] == "near":
            # FP64 ALU bound: priced at the operation count of one large-argument
            # J_0 evaluation plus the multiply-add (near-field roofline)
            flops = dom["work"] * NEAR_FLOPS_PER_ENTRY
            ach = flops / (dom["total_ms"] * 1e-3) / 1e12
            roofline = {"kernel": "near", "bound": "alu", "achieved": ach, "peak": FP64_VECTOR_TFLOPS,
                        "unit": "TFLOP/s", "frac": ach / FP64_VECTOR_TFLOPS,
                        "traffic": measured_traffic("k_near")}
        else:
            ach = dom["bytes"] / (dom["total_ms"] * 1e-3) / 1e9
            roofline = {"kernel": dom["name"], "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                        "traffic": measured_traffic("k_" + dom["name"]),
                        "bytes_per_launch": dom["bytes"] / max(1, dom["launches"])}

    direct = None
    if not args.no_direct:
        # the O(N^2) direct sum on the same GPU with the same J_0 (one transform)
        hank.transform(task, c, eps, out=out, direct=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hank.transform(task, c, eps, out=out, direct=1)
        torch.cuda.synchronize()
        td = time.perf_counter() - t0
        direct = {"points_per_s": N / td, "ms": td * 1e3, "speedup_fast_vs_direct": value / (N / td)}

    # the library's automatic precision choice on the same workload: FP64
    # bulk with the transforms whose contribution is small enough in FP32
    mixed = None
    if args.precision != 0 and args.only == "all":
        ts, _, _ = step_times(hank, torch, task, c, eps, out, args.steps, args.warmup, plan_mode=args.plan_mode,
                              precision=0)
        mi = hank.plan_info(task, N, eps, plan_mode=args.plan_mode, precision=0)
        mixed = {"ms": quantile(ts, 0.5), "points_per_s": N / (quantile(ts, 0.5) * 1e-3),
                 "fp32_transforms": mi["fp32_transforms"], "far_transforms": mi["far_transforms"],
                 "near_entries": mi["near_entries"], "blocks": mi["nblocks"]}
        f_mixed = out.cpu().numpy()

    inverse = None
    if task == "dht0" and args.only == "all":
        # the inverse DHT of Sec. 6 on the same plan, and the self-inverse
        # workload of eq. (inverseTest): c~ = dht0(dht0_inverse(c))
        back = torch.empty_like(c)
        hank.dht0_inverse(c, eps, out=back)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(11)]
        ev[0].record(stream)
        for i in range(10):
            hank.dht0_inverse(c, eps, out=back, stream=stream)
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        inv_ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(10))[5]
        hank.transform(task, back, eps, out=out)
        torch.cuda.synchronize()
        inverse = {"ms": inv_ms, "points_per_s": N / (inv_ms * 1e-3),
                   "roundtrip_max_abs_err": float(torch.max(torch.abs(out - c)).item()),
                   "c_max_abs": float(torch.max(torch.abs(c)).item())}
        del back

    cpu_line = None
    head_err = None
    if cpu is not None:
        import oracle
        nthreads = cpu.nthreads
        probe = inputs.sampled_rows(N, 4 * nthreads, seed=inputs.SEED_SAMPLED_ROWS)[:3 * nthreads]
        oracle.eval_rows(task, c_host, rows=probe[:1], nthreads=1)  # one-time set-up (roots) off the clock
        # marginal cost per row from two sample sizes (each call also has a fixed set-up)
        t0 = time.perf_counter()
        oracle.eval_rows(task, c_host, rows=probe[:nthreads], nthreads=nthreads)
        t1 = time.perf_counter()
        oracle.eval_rows(task, c_host, rows=probe, nthreads=nthreads)
        t2 = time.perf_counter()
        per_row = max(((t2 - t1) - (t1 - t0)) / (2 * nthreads), 1e-6)
        setup = max(0.0, (t1 - t0) - nthreads * per_row)
        nrows = int(max(nthreads, min(N, (args.cpu_seconds - setup) / per_row)))
        rows = np.sort(np.random.default_rng(inputs.SEED_SAMPLED_ROWS).choice(
            np.arange(1, N + 1), size=nrows, replace=False))
        t0 = time.perf_counter()
        ref = oracle.eval_rows(task, c_host, rows=rows, nthreads=nthreads)
        tc = time.perf_counter() - t0
        cpu_line = {"value": nrows / tc, "unit": "points/s", "cores": nthreads, "kind": "oracle",
                    "sample": "%d of %d output rows (uniform, seed %d), each a full %d-term FP64 direct sum; "
                              "%.1f s" % (nrows, N, inputs.SEED_SAMPLED_ROWS, N, tc)}
        # the same rows measure the error of the timed results
        head_err = error_stats(np, f_head[rows - 1], ref, c_host, eps)
        head_err["rows_checked"] = int(nrows)
        if mixed is not None:
            mixed["error"] = error_stats(np, f_mixed[rows - 1], ref, c_host, eps)
            mixed["error"]["rows_checked"] = int(nrows)

    prec_desc = ("every one of the %d far transforms in FP64" % info["far_transforms"] if all_fp64 else
                 "%d of %d far transforms in FP32" % (info["fp32_transforms"], info["far_transforms"]))
    line = {
        "metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if all_fp64 else "f64+f32", "data": "synthetic",
        "config": {"workload": "%s N=%d eps=%g, c_n iid N(0,1) seed %d, %s plan, %s; FP64 near field and roots" % (
            task, N, eps, inputs.SEED_DHT0 if task == "dht0" else 0,
            "paper" if args.plan_mode == 1 else "tuned", prec_desc),
            "task": task, "N": N, "eps": eps, "blocks": info["nblocks"],
            "near_entries": info["near_entries"], "far_transforms": info["far_transforms"],
            "fp32_transforms": info["fp32_transforms"], "plan_build_s": plan_s},
        "roofline": roofline, "cpu_baseline": cpu_line, "error": head_err, "direct_gpu": direct,
        "mixed_precision": mixed, "inverse_dht": inverse, "kernels": kernels,
        "step_ms": {"median": step_q(0.5), "p90": step_q(0.9), "min": min(step_ms), "max": max(step_ms)},
        "profiled_ms_per_step": profiled_ms_per_step,
        "plan_roofline": plan_roofline,
    }
    del c, out
    if args.only == "all" and not args.no_configs:
        line["configs"] = run_configs()
    if args.only == "all" and not args.no_ablation:
        line["ablation"] = run_ablation(hank, inputs, torch, task, N, eps, c_host, precision=args.precision)
    run_extra()
    line.update(extra)
    print(json.dumps(line))


# operation count charged per near-field entry
NEAR_FLOPS_PER_ENTRY = 60.0

if __name__ == "__main__":
    main()
