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
# counters per launch of each kernel from rocprofv3 --pmc runs of the headline
# (HBM bytes from FETCH_SIZE / WRITE_SIZE scaled by a plain copy of known
# size; FP64 VALU instruction counts), valid while the kernel sources are
# unchanged
COUNTER_FILE = os.path.join(ROOT, "profiles", "kernel_counters.json")
KERNEL_SOURCES = ["paper_1501_01652_amd/csrc/kernels.hip", "paper_1501_01652_amd/csrc/fft_device.h",
                  "paper_1501_01652_amd/csrc/device_common.h", "paper_1501_01652_amd/csrc/kernels.h"]
COPY_BYTES = 1 << 30           # the calibration copy (--only copy)
METRIC = "DHT0 points/sec at N=2^20, ε=1e-8 vs direct; batched p50/p99 latency"
# the counter passes (each its own rocprofv3 run; -d <dir>/p<i> -o p --output-format csv)
PMC_PASSES = [
    "SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_SALU SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_SMEM SQ_INSTS",
    "SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_WAIT_INST_LDS SQ_ACTIVE_INST_VALU "
    "SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_ANY",
    "SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_TRANS_F64 "
    "SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_INSTS_VALU_INT32 SQ_INSTS_VALU_INT64 SQ_INSTS_VALU_CVT",
    "SQ_LDS_BANK_CONFLICT SQ_LDS_IDX_ACTIVE SQ_THREAD_CYCLES_VALU SQ_LEVEL_WAVES SQ_BUSY_CU_CYCLES "
    "SQ_ACTIVE_INST_VMEM SQ_INSTS_VALU_FLOPS_FP64 GRBM_GUI_ACTIVE",
    "FETCH_SIZE", "WRITE_SIZE"]
PMC_HEADLINE = "python3 bench.py --only headline --steps 2 --warmup 1 --no-cpu --no-direct"
PMC_BATCHED = "python3 bench.py --only batched-kernels --steps 1"
PMC_COPY = "python3 bench.py --only copy"


def note(msg):
    """A progress line on stderr as each phase of the run ends."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_counters(kernel, workload="headline"):
    """Counters per launch of `kernel` on the headline (or the batched
    workload's one-call batch) from the committed summary, or None if there is
    none or the kernel sources changed since it was taken."""
    try:
        with open(COUNTER_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("kernels" if workload == "headline" else "kernels_batched", {}).get(kernel)


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the counter summary, or None."""
    k = kernel_counters(kernel)
    return None if k is None or "hbm_bytes" not in k else k["hbm_bytes"]


def run_copy(torch):
    """A plain device copy of COPY_BYTES, to calibrate the HBM byte counters."""
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"copy_bytes": COPY_BYTES, "copies": 3}


def write_counters(pmc_dir):
    """Build COUNTER_FILE from the rocprofv3 --pmc runs under pmc_dir: p1..p6
    the counter passes PMC_PASSES of the headline (PMC_HEADLINE), p7 and p8
    FETCH_SIZE and WRITE_SIZE of the calibration copy (PMC_COPY), whose true
    traffic is COPY_BYTES each way.  Values are per dispatch, averaged over
    the dispatches of each kernel (instantiations of one template summed per
    launch set are kept apart by their full names)."""
    import csv

    def per_kernel(path):
        acc = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("hank::", "").strip()
                acc.setdefault(name, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        return acc

    runs = {i: per_kernel(os.path.join(pmc_dir, "p%d" % i, "p_counter_collection.csv")) for i in range(1, 9)}
    p9 = os.path.join(pmc_dir, "p9", "p_counter_collection.csv")  # FP64 counters of the batched workload
    batched = per_kernel(p9) if os.path.exists(p9) else {}

    def copy_kib(i, counter):
        return max(sum(v[counter]) / len(v[counter]) for v in runs[i].values() if counter in v)

    fscale = (COPY_BYTES / 1024.0) / copy_kib(7, "FETCH_SIZE")
    wscale = (COPY_BYTES / 1024.0) / copy_kib(8, "WRITE_SIZE")
    kernels = {}
    for i in range(1, 7):
        for name, cs in runs[i].items():
            if not name.startswith("k_"):
                continue
            k = kernels.setdefault(name, {})
            for cn, v in cs.items():
                k[cn] = sum(v) / len(v)
    kernels_b = {name: {cn: sum(v) / len(v) for cn, v in cs.items()} for name, cs in batched.items()
                 if name.startswith("k_")}
    for k in list(kernels.values()) + list(kernels_b.values()):
        if "FETCH_SIZE" in k and "WRITE_SIZE" in k:
            k["hbm_bytes"] = 1024.0 * (k["FETCH_SIZE"] * fscale + k["WRITE_SIZE"] * wscale)
        if "SQ_INSTS_VALU_FMA_F64" in k:
            # FP64 operations: 64 lanes per wave instruction, an FMA two
            k["fp64_flops"] = 64.0 * (k["SQ_INSTS_VALU_ADD_F64"] + k["SQ_INSTS_VALU_MUL_F64"] +
                                      2.0 * k["SQ_INSTS_VALU_FMA_F64"] + k["SQ_INSTS_VALU_TRANS_F64"]) + \
                512.0 * k.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0)
            k["fp64_wave_insts"] = (k["SQ_INSTS_VALU_ADD_F64"] + k["SQ_INSTS_VALU_MUL_F64"] +
                                    k["SQ_INSTS_VALU_FMA_F64"] + k["SQ_INSTS_VALU_TRANS_F64"])
    cmds = ["cd /tmp && rocprofv3 --pmc %s --output-format csv -d <dir>/p%d -o p -- %s" % (c, i + 1, PMC_HEADLINE)
            for i, c in enumerate(PMC_PASSES)]
    cmds += ["cd /tmp && rocprofv3 --pmc %s --output-format csv -d <dir>/p%d -o p -- %s" % (c, i + 7, PMC_COPY)
             for i, c in enumerate(["FETCH_SIZE", "WRITE_SIZE"])]
    if batched:
        cmds.append("cd /tmp && rocprofv3 --pmc %s --output-format csv -d <dir>/p9 -o p -- %s" %
                    (PMC_PASSES[2], PMC_BATCHED))
    out = {"source_hash": kernel_source_hash(), "fetch_scale": fscale, "write_scale": wscale,
           "workload": "the headline: dht0 N=2^20 eps=1e-8, every far transform in FP64; kernels_batched: "
                       "the batched workload's one-call batch (1024 requests)",
           "commands": cmds, "kernels": kernels, "kernels_batched": kernels_b}
    with open(COUNTER_FILE, "w") as fh:
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
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-direct", action="store_true")
    ap.add_argument("--batch-count", type=int, default=1024, help="requests of the batched workload (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="arrival window of the serving run (0: skip)")
    ap.add_argument("--serve-low-seconds", type=float, default=20.0,
                    help="arrival window of the second serving trace, at 0.8 x the plain form's capacity (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--only", choices=["all", "headline", "batched", "batched-kernels", "serve", "copy", "ablation",
                                       "configs"],
                    default="all")
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads (configs block)")
    ap.add_argument("--oracle-rows", type=int, default=48,
                    help="sampled output rows per large workload on which the CPU oracle is timed and "
                         "the GPU result is compared")
    ap.add_argument("--write-counters", metavar="PMC_DIR",
                    help="write the kernel counter summary from the rocprofv3 --pmc runs under PMC_DIR and exit")
    return ap.parse_args()


def run_batched(hank, inputs, torch, count, stages=8):
    """The batched workload (1024 uneven requests, FFT splits from the
    autotuner): in one hank_batch call (its makespan), replayed as a HIP
    graph, and as `stages` consecutive hank_batch calls of requests sorted by
    the planner's modelled cost (cheapest first), each request's completion
    stamped by an event after its stage -- against the same requests one call
    at a time in the same order (completion stamped per call)."""
    import concurrent.futures
    tuned = hank.autotune()
    specs = inputs.batch_specs(count)
    with concurrent.futures.ThreadPoolExecutor(16) as ex:  # host planning only
        infos = list(ex.map(lambda sp: hank.plan_info(sp["task"], sp["N"], sp["eps"], nrhs=sp["nrhs"]), specs))
    model_s = [pi["model_s"] for pi in infos]
    # nominal FP64 work of the multi-right-hand-side near kernel: one J_0 per
    # entry, shared by the right-hand sides, and one multiply-add (2 flops)
    # per entry and right-hand side (requests of up to 3 run as single ones)
    multi_nominal = sum(pi["near_entries"] * (NEAR_FLOPS_PER_ENTRY + 2.0 * sp["nrhs"])
                        for sp, pi in zip(specs, infos) if sp["nrhs"] > SINGLE_RHS_MAX)
    reqs = []
    for sp, m in zip(specs, model_s):
        g = torch.Generator(device="cuda").manual_seed(sp["seed"])
        shape = (sp["nrhs"], sp["N"]) if sp["nrhs"] > 1 else (sp["N"],)
        c = torch.rand(shape, generator=g, dtype=torch.float64, device="cuda") * 2.0 - 1.0
        reqs.append({"task": sp["task"], "c": c, "out": torch.empty_like(c), "eps": sp["eps"],
                     "cost": m * sp["nrhs"] / (1 << (sp["nrhs"] - 1).bit_length())})
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
    # staged: cheapest first, one event per stage
    order = sorted(range(count), key=lambda i: reqs[i]["cost"])
    bounds = [round(k * count / stages) for k in range(stages + 1)]
    stage_reqs = [[reqs[i] for i in order[bounds[k]:bounds[k + 1]]] for k in range(stages)]
    for sr in stage_reqs:
        hank.batch(sr)
    torch.cuda.synchronize()
    lat_st, ts_st = [], []
    for _ in range(reps):
        start = torch.cuda.Event(enable_timing=True)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(stages)]
        start.record()
        for sr, e in zip(stage_reqs, evs):
            hank.batch(sr)
            e.record()
        torch.cuda.synchronize()
        done = [start.elapsed_time(e) for e in evs]
        lat_st = sorted(done[k] for k in range(stages) for _ in range(bounds[k + 1] - bounds[k]))
        ts_st.append(done[-1] / 1e3)
    tst = sorted(ts_st)[len(ts_st) // 2]
    # kernel times of one whole-batch call (HIP events around every launch)
    hank.profile(True)
    hank.batch(reqs)
    torch.cuda.synchronize()
    kst = hank.profile_report()
    hank.profile(False)
    kernels = {k["name"]: {"launches": k["launches"], "ms": k["total_ms"]} for k in kst}
    nm = [k for k in kst if k["name"] == "near_multi"]
    multi_roofline = None
    if nm and nm[0]["total_ms"] > 0:
        kc = kernel_counters("k_near_multi", "batched")
        counted = bool(kc and "fp64_flops" in kc)
        # FP64 operations of the launch: counted on this workload when the
        # counter summary matches the sources, else the nominal count
        flops = kc["fp64_flops"] if counted else multi_nominal
        ach = flops / (nm[0]["total_ms"] * 1e-3) / 1e12
        multi_roofline = {"kernel": "near_multi", "bound": "alu", "achieved": ach, "peak": FP64_VECTOR_TFLOPS,
                          "unit": "TFLOP/s", "frac": ach / FP64_VECTOR_TFLOPS,
                          "flops_basis": "rocprofv3 FP64 VALU and MFMA counts" if counted else
                          "nominal: 60 per entry (J_0) + 2 per entry and right-hand side"}
    # one request at a time in the same order, completion stamped per call
    for i in order:
        hank.transform(reqs[i]["task"], reqs[i]["c"], reqs[i]["eps"], out=reqs[i]["out"])
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in reqs]
    start.record()
    for i, e in zip(order, evs):
        hank.transform(reqs[i]["task"], reqs[i]["c"], reqs[i]["eps"], out=reqs[i]["out"])
        e.record()
    torch.cuda.synchronize()
    lat = sorted(start.elapsed_time(e) for e in evs)
    ts = lat[-1] / 1e3
    return {"requests": count, "rhs_total": int(sum(sp["nrhs"] for sp in specs)),
            "workload": "task 40/40/20, N log-uniform [2^8, 2^16], 1-64 rhs, eps {1e-4,1e-8,1e-14}, "
                        "c ~ U[-1,1], seed %d; FFT splits from hank_autotune" % inputs.SEED_BATCH,
            "autotuned_l2": tuned,
            "one_call_transforms_per_s": count / tb, "one_call_makespan_ms": tb * 1e3,
            "graph_transforms_per_s": count / tg, "graph_ms": tg * 1e3,
            "staged": {"stages": stages, "order": "modelled cost, cheapest first",
                       "transforms_per_s": count / tst, "makespan_ms": tst * 1e3,
                       "latency_p50_ms": quantile(lat_st, 0.5), "latency_p99_ms": quantile(lat_st, 0.99)},
            "batched_transforms_per_s": count / tst,
            "batched_latency_p50_ms": quantile(lat_st, 0.5), "batched_latency_p99_ms": quantile(lat_st, 0.99),
            "sequential_transforms_per_s": count / ts, "sequential_ms": ts * 1e3,
            "sequential_latency_p50_ms": quantile(lat, 0.5), "sequential_latency_p99_ms": quantile(lat, 0.99),
            "speedup": ts / tst, "first_call_incl_planning_s": warm_s,
            "one_call_kernels": kernels, "near_multi_roofline": multi_roofline}


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
        note("ablation: %s plan %.3f ms" % (name, ms))
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
        note("ablation: M sweep at eps %g, best M %d" % (e, best))
    direct_ms = _median_ms(hank, torch, "schlomilch", cs, 1e-15, outs, 5, direct=1)
    hank.cache_clear()
    return {"partition": part,
            "m_sweep": {"workload": "schlomilch N=%d, c_n iid N(0,1) seed %d, paper plan" % (Ns, inputs.SEED_SCHLOMILCH),
                        "by_eps": sweep, "direct_ms": direct_ms}}


def serve_buffers(torch, inputs, ring):
    """One coefficient vector of the largest size (requests use its first N
    entries) and a ring of output buffers."""
    nmax = 1 << 22
    g = torch.Generator(device="cuda").manual_seed(inputs.SEED_SERVE)
    c_all = torch.randn(nmax, generator=g, dtype=torch.float64, device="cuda")
    outs = [torch.empty(nmax, dtype=torch.float64, device="cuda") for _ in range(ring)]
    return c_all, outs


def warm_partition_tables(hank, trace):
    """Host-side start-up of a serving process: the tuned partition search at
    the grid sizes 2^(j/4) that the trace's sizes fall between (each later plan
    of a size between grid points reuses it), in parallel threads."""
    import concurrent.futures
    import math
    keys = set()
    for t in trace:
        j = int(math.floor(4 * math.log2(t["N"]) + 1e-9))
        for jj in (j, j + 1):
            keys.add((t["task"], int(round(2 ** (jj / 4.0))), t["eps"]))
    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(16) as ex:
        list(ex.map(lambda k: hank.plan_info(k[0], k[1], k[2]), sorted(keys)))
    return {"grid_plans": len(keys), "seconds": time.perf_counter() - t0}


def run_serve(hank, inputs, torch, trace, c_all, outs, max_batch=64, max_pending=512, budget=48 << 30):
    """Open-loop arrivals through the continuous-batching server (planner
    threads build unseen plans while batches run)."""
    srv = hank.Server(budget_bytes=budget, max_batch=max_batch, max_pending=max_pending)
    for k, t in enumerate(trace):
        N = t["N"]
        srv.submit({"task": t["task"], "c": c_all[:N], "out": outs[k % len(outs)][:N], "eps": t["eps"]},
                   arrival_s=t["arrival"])
    srv.start()
    srv.drain()
    st = srv.stats()
    srv.close()
    st["max_batch"] = max_batch
    st["max_pending"] = max_pending
    return st


def run_plain(hank, torch, trace, c_all, outs, max_pending=512):
    """The plain form: hank_* calls one request at a time in arrival order on
    one stream (plans built when first needed), at most two calls in flight; a
    request that arrives while max_pending requests wait is rejected."""
    import collections
    stream = torch.cuda.current_stream()
    n = len(trace)
    events = [None] * n
    rejected = 0
    queue = collections.deque()
    inflight = collections.deque()
    i_arr = 0
    start = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)

    def arrivals():
        nonlocal i_arr, rejected
        now = time.perf_counter() - t0
        while i_arr < n and trace[i_arr]["arrival"] <= now:
            if len(queue) >= max_pending:
                rejected += 1
            else:
                queue.append(i_arr)
            i_arr += 1

    while True:
        arrivals()
        if queue:
            while len(inflight) >= 2:
                inflight.popleft().synchronize()
                arrivals()
            k = queue.popleft()
            t = trace[k]
            N = t["N"]
            hank.transform(t["task"], c_all[:N], t["eps"], out=outs[k % len(outs)][:N], stream=stream)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
            events[k] = ev
            inflight.append(ev)
        elif i_arr >= n:
            break
        else:
            time.sleep(max(0.0, min(1e-3, trace[i_arr]["arrival"] - (time.perf_counter() - t0))))
    torch.cuda.synchronize()
    lat, last = [], 0.0
    for k in range(n):
        if events[k] is not None:
            done = start.elapsed_time(events[k]) / 1e3
            last = max(last, done)
            lat.append(1e3 * (done - trace[k]["arrival"]))
    lat.sort()
    wall = last - trace[0]["arrival"] if lat else 0.0
    return {"submitted": n, "completed": len(lat), "rejected": rejected,
            "p50_ms": quantile(lat, 0.5) if lat else None, "p90_ms": quantile(lat, 0.9) if lat else None,
            "p99_ms": quantile(lat, 0.99) if lat else None, "wall_s": wall,
            "throughput": len(lat) / wall if wall > 0 else 0.0, "max_pending": max_pending}


def run_serving(hank, inputs, torch, seconds, rate, low_seconds):
    """The serving workload: Poisson arrivals at `rate` for `seconds` (N
    log-uniform integers in [2^10, 2^22], so most plans are new), through the
    server and through the plain sequential form; then a second trace at 0.8 x
    the plain form's measured capacity for `low_seconds`."""
    c_all, outs = serve_buffers(torch, inputs, 1024)
    trace = inputs.serve_trace(rate=rate, seconds=seconds)
    low_rate = None
    res = {"workload": "Poisson %g req/s for %g s, task 40/40/20, N log-uniform integers in [2^10, 2^22], "
                       "1 rhs, eps {1e-4,1e-8,1e-14}, seed %d" % (rate, seconds, inputs.SEED_SERVE),
           "requests": len(trace), "distinct_sizes": len({(t["task"], t["N"], t["eps"]) for t in trace})}
    res["startup"] = warm_partition_tables(hank, trace)
    note("serving: %d requests, partition tables warmed" % len(trace))
    res["continuous_batching"] = run_serve(hank, inputs, torch, trace, c_all, outs)
    hank.cache_clear()
    note("serving: continuous batching done")
    res["plain_sequential"] = run_plain(hank, torch, trace, c_all, outs)
    hank.cache_clear()
    note("serving: plain sequential done")
    cap = res["plain_sequential"]["throughput"]
    if low_seconds > 0 and cap > 0:
        low_rate = 0.8 * cap
        low = inputs.serve_trace(rate=low_rate, seconds=low_seconds, seed=inputs.SEED_SERVE + 1)
        res["at_0.8_capacity"] = {"rate": low_rate, "seconds": low_seconds, "requests": len(low),
                                  "startup": warm_partition_tables(hank, low),
                                  "continuous_batching": run_serve(hank, inputs, torch, low, c_all, outs)}
        hank.cache_clear()
        note("serving at 0.8 x capacity: continuous batching done")
        res["at_0.8_capacity"]["plain_sequential"] = run_plain(hank, torch, low, c_all, outs)
        hank.cache_clear()
        note("serving at 0.8 x capacity: plain sequential done")
    del c_all, outs
    return res


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
    note("config %s N=%d eps=%g %s: %.4f ms" % (task, N, eps, rec["precision"], rec["ms"]))
    return rec


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU; runs on several GPUs are not supported "
              "(got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.write_counters:
        out = write_counters(args.write_counters)
        print(json.dumps({k: {c: v for c, v in d.items() if c in ("hbm_bytes", "fp64_flops")}
                          for k, d in out["kernels"].items()}))
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
            note("batched workload done")
        if args.only in ("all", "serve") and args.serve_seconds > 0:
            extra["serving"] = run_serving(hank, inputs, torch, args.serve_seconds, args.serve_rate,
                                           args.serve_low_seconds)

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
    if args.only == "batched-kernels":  # the batched workload's one-call batch, for profilers
        specs = inputs.batch_specs(args.batch_count)
        reqs = []
        for sp in specs:
            g = torch.Generator(device="cuda").manual_seed(sp["seed"])
            shape = (sp["nrhs"], sp["N"]) if sp["nrhs"] > 1 else (sp["N"],)
            c = torch.rand(shape, generator=g, dtype=torch.float64, device="cuda") * 2.0 - 1.0
            reqs.append({"task": sp["task"], "c": c, "out": torch.empty_like(c), "eps": sp["eps"]})
        for _ in range(1 + args.steps):
            hank.batch(reqs)
        torch.cuda.synchronize()
        print(json.dumps({"batches": 1 + args.steps, "requests": len(reqs)}))
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
    note("headline timed: %.4f ms per step" % (1e3 * elapsed / args.steps))
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
    near_kc = kernel_counters("k_near") if task == "dht0" and N == 1 << 20 and eps == 1e-8 else None
    # FP64 operations per near-field entry: counted by rocprofv3 on this
    # workload when the counter summary matches the kernel sources, else the
    # nominal count of one large-argument J_0 and the multiply-add
    near_fpe, near_basis = NEAR_FLOPS_PER_ENTRY, "nominal"
    if near_s and near_kc and "fp64_flops" in near_kc:
        near_fpe = near_kc["fp64_flops"] / (near_s[0]["work"] / near_s[0]["launches"])
        near_basis = "rocprofv3 FP64 VALU instruction counts"
    near_flops = near_s[0]["work"] * near_fpe / args.steps if near_s else 0.0
    plan_roofline["phase_roofline_ms"] = 1e3 * (far_bytes / (HBM_PEAK_GBS * 1e9) +
                                                near_flops / (FP64_VECTOR_TFLOPS * 1e12))
    plan_roofline["far_passes_ms"] = far_ms
    plan_roofline["far_passes_GBps"] = far_bytes / (far_ms * 1e-3) / 1e9 if far_ms > 0 else None
    dom = max(stats, key=lambda s: s["total_ms"]) if stats else None
    roofline = None
    if dom is not None:
        if dom["name"] == "near":
            # FP64 ALU bound: the kernel's FP64 operations per entry (counted, or
            # the nominal figure) times the entries, against the FP64 vector peak
            flops = dom["work"] * near_fpe
            ach = flops / (dom["total_ms"] * 1e-3) / 1e12
            roofline = {"kernel": "near", "bound": "alu", "achieved": ach, "peak": FP64_VECTOR_TFLOPS,
                        "unit": "TFLOP/s", "frac": ach / FP64_VECTOR_TFLOPS,
                        "traffic": measured_traffic("k_near"),
                        "flops_per_entry": near_fpe, "flops_basis": near_basis}
            if near_kc and "fp64_wave_insts" in near_kc:
                # FP64 issue: a wave64 FP64 instruction holds a SIMD's FP64 pipe 4 cycles
                simd_cycles = 1024 * 2.4e9 * (dom["total_ms"] / dom["launches"]) * 1e-3
                roofline["fp64_pipe_busy"] = 4.0 * near_kc["fp64_wave_insts"] / simd_cycles
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
        note("direct sum on the GPU: %.1f ms" % (td * 1e3))

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
        note("automatic precision: %.4f ms" % mixed["ms"])

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
        note("inverse DHT: %.4f ms" % inv_ms)

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
        note("oracle baseline: %d rows in %.1f s" % (nrows, tc))
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
        note("ablation done")
    run_extra()
    line.update(extra)
    print(json.dumps(line))


# operation count charged per near-field entry: one J_0 evaluation of the
# asymptotic or series form (about 60 FP64 operations) and the multiply-add
NEAR_FLOPS_PER_ENTRY = 60.0
# requests with up to this many right-hand sides run as single transforms
SINGLE_RHS_MAX = 3

if __name__ == "__main__":
    main()
