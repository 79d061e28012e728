#!/usr/bin/env python3
"""Throughput of the ensemble integrator on one MI355X.

One step = one call of the C ABI (ai_integrate_async) integrating the whole
2^20-trajectory thermal Li + Yb+ ensemble (seed 0, RelTol 1e-8, AbsTol 1e-10,
exit at r > R0 after closest approach or after 200 RF periods), inputs already
resident in device memory.  The timed configuration is the fastest one: the
plain one-trajectory-per-lane kernel on the longest-predicted-first schedule
(the call includes computing and sorting the schedule); the other
kernel/schedule combinations are timed too and reported beside it.  W untimed
warm-up steps, then K timed steps bracketed by device synchronisation; prints
one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--kernel plain|persistent]
                    [--schedule longest-first|index]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "accepted RK45 steps/s and trajectories/s per MI355X at RelTol 1e-8; p50/p99 latency"
FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters.json")
KERNEL_SYMBOL = {"persistent": "ai_persistent_kernel", "plain": "ai_plain_kernel"}


_T0 = time.perf_counter()


def progress(msg: str) -> None:
    """One line on stderr as each part of the run ends (stdout carries only the
    JSON record)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def strip_comments(src: str) -> str:
    """C/C++ source without its comments (string and character literals kept),
    each comment replaced by one space."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
            out.append(" ")
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return "".join(out)


def source_digest() -> str:
    """Digest of the kernel sources' tokens (comments and layout left out): the
    profiles are taken on code, and a change of documentation does not make
    them stale."""
    import re
    token = re.compile(r'"(?:\\.|[^"\\])*"|\'(?:\\.|[^\'\\])*\'|[^\s"\']+')
    h = hashlib.sha256()
    for p in ("paper_2509_12381_amd/csrc/ai.hip", "paper_2509_12381_amd/csrc/schedule.hip",
              "paper_2509_12381_amd/csrc/schedule.h", "include/ai.h"):
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            # the tokens, so that layout and comments do not count
            h.update(" ".join(token.findall(strip_comments(f.read()))).encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(KERNEL_SYMBOL[kernel])
    if not k or rec.get("source_digest") != source_digest():
        return None
    return k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]


def measured_counters(kernel: str):
    """Per-launch SQ counters of `kernel` from the committed rocprofv3 summary
    (profiles/counters.json), if it was taken on the current kernel source;
    else None."""
    try:
        with open(COUNTERS_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(KERNEL_SYMBOL[kernel])
    if not k or rec.get("source_digest") != source_digest():
        return None
    return k


def write_counters(dirs) -> dict:
    """profiles/counters.json from rocprofv3 --pmc runs of this script (one
    directory per pass): the mean per launch of every SQ counter, per kernel."""
    import csv
    import glob
    vals = {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*_counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                key = (r["Kernel_Name"], r["Dispatch_Id"], r["Counter_Name"])
                vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    rec = {"source_digest": source_digest(), "kernels": {}}
    for sym in KERNEL_SYMBOL.values():
        per = {}
        for (k, disp, ctr), v in vals.items():
            if f"::{sym}(" in k:
                per.setdefault(ctr, []).append(v)
        if per:
            rec["kernels"][sym] = {c: sum(v) / len(v) for c, v in per.items()}
    with open(COUNTERS_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def write_traffic(fetch_dir: str, write_dir: str, copy_mib: int) -> dict:
    """profiles/traffic.json from two rocprofv3 --pmc runs of this script (one
    with FETCH_SIZE, one with WRITE_SIZE, both with --copy-calibration-mib
    copy_mib).  Each counter is scaled by what it reads for the plain device
    copy of copy_mib MiB, the largest copy dispatch of the run."""
    import csv
    import glob

    def per_dispatch(d, counter):
        out = {}
        for f in glob.glob(os.path.join(d, "*_counter_collection.csv")):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                key = (r["Kernel_Name"], r["Dispatch_Id"])
                out[key] = out.get(key, 0.0) + float(r["Counter_Value"]) * 1024.0
        return out

    rec = {"source_digest": source_digest(), "copy_calibration_bytes": copy_mib << 20,
           "kernels": {}}
    for counter, d, field in (("FETCH_SIZE", fetch_dir, "fetch"), ("WRITE_SIZE", write_dir, "write")):
        vals = per_dispatch(d, counter)
        copies = [v for (k, _), v in vals.items() if "copyBuffer" in k]
        factor = max(copies) / float(copy_mib << 20)
        rec[f"{field}_calibration_factor"] = factor
        for sym in KERNEL_SYMBOL.values():
            mine = [v for (k, _), v in vals.items() if f"::{sym}(" in k]
            if mine:
                k = rec["kernels"].setdefault(sym, {})
                k[f"{field}_bytes_per_launch"] = sum(mine) / len(mine) / factor
                k[f"{field}_counter_bytes_per_launch"] = sum(mine) / len(mine)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def batched_grid(binding, W, flops, torch, reps: int = 3) -> dict:
    """The batched configuration: 64 uneven ensembles (collision temperature x
    trap q) in one longest-first launch of ai_integrate_batch, against the
    same ensembles as 64 separate longest-first launches on the stream."""
    grid = W.batch_grid()
    dev = []
    for wl in grid:
        d = torch.from_numpy(wl.initial_states()).cuda()
        dev.append((wl, d, torch.empty_like(d),
                    torch.empty((W.NOBS, wl.n), dtype=torch.float64, device="cuda")))
    items = [(wl.system, d, f, o, wl.t0, wl.tmax, wl.rtol, wl.atol) for wl, d, f, o in dev]

    def batched():
        binding.ai_integrate_batch_async(items, schedule="longest-first")

    def separate():
        for wl, d, f, o in dev:
            binding.ai_integrate_async(wl.system, d, wl.t0, wl.tmax, wl.rtol, wl.atol, f, o,
                                       "plain", schedule="longest-first")

    def mean_ms(fn):
        fn()
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            out.append(a.elapsed_time(b))
        return sum(out) / len(out)

    t_batch = mean_ms(batched)
    obs = [o.cpu().numpy() for *_, o in dev]
    for _ in range(reps):
        binding.ai_integrate_batch_async(items, schedule="longest-first", time_kernel=True)
    torch.cuda.synchronize()
    t_kernel = sum(binding.ai_kernel_time(back) for back in range(reps)) / reps
    t_sep = mean_ms(separate)
    # the tuner's choice for this batch, and a prepared batch captured in a HIP
    # graph and replayed
    best_kernel, best_ms = binding.ai_tune_batch(items)
    plan = binding.BatchPlan(items, schedule="longest-first")
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            plan.launch(stream=side)
    torch.cuda.current_stream().wait_stream(side)
    t_graph = mean_ms(g.replay)
    del g
    plan.close()
    n = sum(wl.n for wl, *_ in dev)
    steps = float(sum(o[W.OBS["nsteps"]].sum() for o in obs))
    flop = float(sum(flops.algorithmic_flops(o) for o in obs))
    achieved = flop / (t_kernel / 1e3) / 1e12
    return {"workload": "batch-grid-64", "ensembles": len(dev), "trajectories": n,
            "ms_per_call": t_batch, "ms_separate_launches": t_sep,
            "trajectories_per_s": n / (t_batch / 1e3), "accepted_steps_per_s": steps / (t_batch / 1e3),
            "speedup_vs_separate": t_sep / t_batch,
            "autotune": {"best_kernel_code": best_kernel, "best_ms": best_ms,
                         "what": "ai_tune_batch: index order, and longest-first with none, 256 "
                                 "or 1024 four-lane trajectories, each timed after an untimed "
                                 "run of itself (best of two rounds)"},
            "graph_replay_ms": t_graph,
            "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                         "kernel": "ai_plain_batch_kernel", "kernel_ms": t_kernel,
                         "what": f"means over {reps} timed calls each (kernel: AI_TIME_KERNEL events)"}}


def serving_requests(W, torch, count: int, rate_hz: float):
    """The first `count` requests of the serving stream (arrival times for
    `rate_hz`): each a slice of the pool moved to its own collision temperature
    and trap q (workload.retarget_thermal), prepared on the device before the
    stream starts, with its own output buffers."""
    stream = W.serving_stream(count, rate_hz=rate_hz)
    pool_wl = W.serving_pool()
    pool = torch.from_numpy(pool_wl.initial_states()).cuda()
    reqs = []
    for r in stream:
        wl = W.serving_request_workload(r)
        y0 = W.retarget_thermal(pool[:, r.offset:r.offset + r.n], pool_wl.system,
                                pool_wl.T_atom, wl.system, r.T_atom).contiguous()
        reqs.append((r, wl, y0, torch.empty_like(y0),
                     torch.empty((W.NOBS, r.n), dtype=torch.float64, device="cuda")))
    del pool
    torch.cuda.synchronize()
    return stream, reqs


def serve_stream(binding, W, torch, reqs, srv, pace: bool) -> dict:
    """Submit the requests to `srv` at their arrival times (pace) or all at
    once (from a thread of their own); latency = completion - submission of
    each request, on the host's monotonic clock."""
    import queue as queue_mod
    import threading

    import numpy as np
    tickets = queue_mod.Queue()

    def submit_all():
        t0 = time.perf_counter()
        for r, wl, y0, f, o in reqs:
            if pace:
                delay = t0 + r.arrival_s - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            tickets.put(srv.submit((wl.system, y0, f, o, wl.t0, wl.tmax, r.rtol, r.atol),
                                   r.precision))

    th = threading.Thread(target=submit_all)
    th.start()
    infos = []
    for k in range(len(reqs)):
        infos.append(srv.wait(tickets.get()))
        if (k + 1) % 250 == 0:
            progress(f"serving: {k + 1} of {len(reqs)} requests completed")
    th.join()
    lat = np.array([i["end_s"] - i["submit_s"] for i in infos]) * 1e3
    t_first = min(i["submit_s"] for i in infos)
    wall = max(i["end_s"] for i in infos) - t_first
    n = sum(r.n for r, *_ in reqs)
    steps = float(sum(o[W.OBS["nsteps"]].sum().item() for *_, o in reqs))
    bad = [i["rc"] for i in infos if i["rc"] < 0]
    rec = {"requests": len(reqs), "trajectories": n,
           "fp32_stage_requests": sum(r.precision != "fp64" for r, *_ in reqs),
           "latency_ms": {"p50": float(np.percentile(lat, 50)),
                          "p99": float(np.percentile(lat, 99)),
                          "mean": float(lat.mean()), "max": float(lat.max()),
                          "what": "request submit to completion, host monotonic clock"},
           "wall_s": wall, "trajectories_per_s": n / wall, "accepted_steps_per_s": steps / wall,
           "launches": len({i["batch_id"] for i in infos}),
           "max_requests_on_gpu": max(i["batch_size"] for i in infos),
           "failed_requests": len(bad)}
    if pace:
        rec["offered_trajectories_per_s"] = n / reqs[-1][0].arrival_s
        rec["stream_s"] = reqs[-1][0].arrival_s
    return rec


def serving(binding, W, torch, count: int, saturate: int, resident_paced: int,
            plain_traj_per_s: float, plain_steps_per_s: float) -> dict:
    """The serving configuration: the Poisson stream (200 requests/s, seed 2;
    sizes, tolerances, precision, temperature and q per request), paced,
    served by batched launches (three workers, longest-first schedule); the
    first `saturate` requests again, submitted at once, served by the resident
    kernel (continuous batching, admission by footprint, a budget that holds
    them all): the
    sustained rate, and once more through batched launches for comparison;
    and the first `resident_paced` requests of the stream
    paced through the resident kernel (idle_ms 500, so that its waves stay
    through the stream's quiet spells)."""
    stream, reqs = serving_requests(W, torch, count, W.SERVING_RATE_HZ)
    progress(f"serving: {len(reqs)} requests prepared")
    out = {"workload": f"poisson-{W.SERVING_RATE_HZ:g}rps", "seed": W.SERVING_SEED}
    with binding.Server(schedule="longest-first") as srv:
        out["paced"] = serve_stream(binding, W, torch, reqs, srv, pace=True)
        out["paced"]["mode"] = "launches"
        progress(f"serving: paced stream, p50 {out['paced']['latency_ms']['p50']:.1f} ms, "
                 f"p99 {out['paced']['latency_ms']['p99']:.1f} ms")
    if saturate:
        # a budget that admits every request at once (their footprints; the
        # buffers are device memory, integrated in place)
        need = sum(37 * ((8 * r.n + 255) // 256 * 256) for r, *_ in reqs[:saturate])
        slab = max(4 << 30, (need + (1 << 30) - 1) >> 30 << 30)
        with binding.Server(mode="resident", slab_bytes=slab) as srv:
            sat = serve_stream(binding, W, torch, reqs[:saturate], srv, pace=False)
        sat["mode"] = "resident"
        sat["slab_bytes"] = slab
        sat["vs_plain_kernel"] = sat["trajectories_per_s"] / plain_traj_per_s
        # the stream's trajectories cost more on average (RelTol down to 1e-10,
        # cold atoms), so accepted steps/s compare the work rates
        sat["steps_vs_plain_kernel"] = sat["accepted_steps_per_s"] / plain_steps_per_s
        out["saturated"] = sat
        progress(f"serving: saturated, {sat['trajectories_per_s']:.3g} trajectories/s")
        # the same requests at once through batched launches: per launch the
        # longest-first order across its requests, and one precision per launch
        with binding.Server(schedule="longest-first") as srv:
            satl = serve_stream(binding, W, torch, reqs[:saturate], srv, pace=False)
        satl["mode"] = "launches"
        satl["vs_plain_kernel"] = satl["trajectories_per_s"] / plain_traj_per_s
        satl["steps_vs_plain_kernel"] = satl["accepted_steps_per_s"] / plain_steps_per_s
        out["saturated_launches"] = satl
        progress(f"serving: saturated through launches, {satl['trajectories_per_s']:.3g} "
                 f"trajectories/s")
    if resident_paced:
        # waves that stay through the stream's quiet spells: each leaves after
        # idle_ms without work of its own (the default 20 ms lets most leave)
        idle = 500.0
        with binding.Server(mode="resident", idle_ms=idle) as srv:
            rp = serve_stream(binding, W, torch, reqs[:resident_paced], srv, pace=True)
        rp["mode"] = "resident"
        rp["idle_ms"] = idle
        out["resident_paced"] = rp
        progress(f"serving: resident paced, p50 {rp['latency_ms']['p50']:.1f} ms")
    out["plain_kernel_trajectories_per_s"] = plain_traj_per_s
    out["plain_kernel_accepted_steps_per_s"] = plain_steps_per_s
    del reqs
    torch.cuda.empty_cache()
    return out


def host_facts() -> dict:
    """The host CPU: logical CPUs online, those this process may run on, model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count()
    return {"host_nproc": os.cpu_count(), "affinity_cpus": allowed, "cpu_model": model}


def _rel(a, b):
    import numpy as np
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def _q(x, p):
    import numpy as np
    return float(np.quantile(x, p)) if x.size else None


def compare_with_oracle(oracle, W, stats, wl, y0_sub, ofin, oob, gfin, gob) -> dict:
    """Per-observable errors of a GPU run against the oracle on the same
    trajectories (columns of y0_sub): statuses and bounce counts, accepted-step
    counts, and on the direct trajectories (oracle: escaped, at most one
    bounce) the final state (block-relative, after aligning the oracle's end
    state to the GPU's end time to first order with the paper's f) and each
    observable plane (median and p99 relative difference; the angle as an
    absolute difference in radians, the transfer in units of m_atom |v_atom|)."""
    import numpy as np
    O = W.OBS
    direct = (oob[O["bounces"]] <= 1) & (oob[O["status"]] == W.ST_ESCAPED)
    al = ofin.copy()
    for i in np.nonzero(gob[O["tend"]] != oob[O["tend"]])[0]:
        al[:, i] += oracle.force(wl.system, oob[O["tend"], i], ofin[:, i]) * (
            gob[O["tend"], i] - oob[O["tend"], i])
    state = stats.block_relative_difference(gfin[:, direct], al[:, direct])
    dsteps = _rel(gob[O["nsteps"]], np.maximum(oob[O["nsteps"]], 1.0))
    out = {"trajectories": int(y0_sub.shape[1]), "direct": int(direct.sum()),
           "status_equal": float(np.mean(gob[O["status"]] == oob[O["status"]])),
           "bounces_equal": float(np.mean(gob[O["bounces"]] == oob[O["bounces"]])),
           "nsteps_equal": float(np.mean(gob[O["nsteps"]] == oob[O["nsteps"]])),
           "nsteps_rel_max": float(dsteps.max()) if dsteps.size else None,
           "final_state_aligned": {"median": _q(state, 0.5), "p99": _q(state, 0.99),
                                   "max": float(state.max()) if state.size else None}}
    speed = np.linalg.norm(ofin[9:12, direct], axis=0) * wl.system.m_atom
    planes = {}
    for name in ("tend", "dist", "rmin", "hnext", "ke", "angle", "transfer"):
        g, o = gob[O[name], direct], oob[O[name], direct]
        if name == "ke":
            o = 0.5 * wl.system.m_ion * np.sum(al[3:6, direct] ** 2, axis=0)
        if name == "angle":
            d = np.abs(g - o)
        elif name == "transfer":
            d = np.abs(g - o) / speed
        else:
            d = _rel(g, o)
        planes[name] = {"median": _q(d, 0.5), "p99": _q(d, 0.99)}
    out["observables"] = planes
    return out


def distributions_vs_oracle(W, stats, gob, oob) -> dict:
    """Complex probability (two-proportion sigma) and KS statistics of the
    scattering angle and of the complex lifetime against the oracle."""
    from scipy import stats as st
    cg, co = stats.complexes(gob), stats.complexes(oob)
    O = W.OBS
    n = gob.shape[1]
    out = {"complexes_gpu": int(cg.sum()), "complexes_oracle": int(co.sum()),
           "complex_sigma": stats.two_proportion_sigma(int(cg.sum()), n, int(co.sum()), n)}
    ks = st.ks_2samp(gob[O["angle"]], oob[O["angle"]])
    out["ks_angle"] = {"statistic": float(ks.statistic), "p": float(ks.pvalue)}
    if min(cg.sum(), co.sum()) >= 2:
        ks = st.ks_2samp(gob[O["lifetime"], cg], oob[O["lifetime"], co])
        out["ks_lifetime"] = {"statistic": float(ks.statistic), "p": float(ks.pvalue)}
    return out


def cpu_baseline(wl, y0_host, sample: int, runs: dict, subset: int = 4096):
    """The oracle as it stands, on the first `sample` trajectories of the same
    ensemble, with the host threads of this process's CPU share (the CPU
    baseline), and what the oracle's results say about the GPU runs in `runs`
    (name -> (final, obs) of the whole ensemble): per-observable errors on the
    first `subset` trajectories and, when the sample is the whole ensemble, the
    distributions."""
    import numpy as np

    import oracle
    from paper_2509_12381_amd import stats
    from paper_2509_12381_amd import workload as W
    threads = min(16, os.cpu_count() or 1)
    ys = np.ascontiguousarray(y0_host[:, :sample])
    t = time.perf_counter()
    ofin, oob, _ = oracle.integrate(wl.system, ys, wl.t0, wl.tmax, wl.rtol, wl.atol,
                                    nthreads=threads)
    wall = time.perf_counter() - t
    steps = float(oob[W.OBS["nsteps"]].sum())
    rec = {"value": steps / wall, "unit": "accepted steps/s", "cores": threads,
           "kind": "oracle", "sample": f"first {sample} trajectories of the {wl.n}-trajectory "
           f"ensemble, {wall:.1f} s wall", "trajectories_per_s": sample / wall, **host_facts()}
    sub = min(subset, wl.n)
    if sample < sub:
        sfin, sob, _ = oracle.integrate(wl.system, np.ascontiguousarray(y0_host[:, :sub]),
                                        wl.t0, wl.tmax, wl.rtol, wl.atol, nthreads=threads)
    else:
        sfin, sob = ofin[:, :sub], oob[:, :sub]
    vs = {}
    for name, (gfin, gob) in runs.items():
        vs[name] = {"subset": compare_with_oracle(oracle, W, stats, wl, y0_host[:, :sub], sfin,
                                                  sob, gfin[:, :sub], gob[:, :sub])}
        if sample == wl.n:
            vs[name]["distributions"] = distributions_vs_oracle(W, stats, gob, oob)
    rec["gpu_vs_oracle"] = vs
    return rec


def ensemble_statistics(W, stats, ob, tmax) -> dict:
    """Complex probability and the 64-bin scattering-angle (log10 bins on
    [1e-10, pi]) and complex-lifetime (linear bins on [0, tmax]) histograms of
    one ensemble's observables."""
    import math
    ha, _ = stats.angle_histogram(ob)
    hl, _ = stats.lifetime_histogram(ob, tmax)
    return {"complex_probability": stats.complex_probability(ob),
            "complexes": int(stats.complexes(ob).sum()),
            "angle_histogram": {"bins": "64 log10-spaced on [1e-10, pi] rad",
                                "lo": 1e-10, "hi": math.pi, "counts": ha.tolist()},
            "lifetime_histogram": {"bins": "64 linear on [0, tmax] (complexes only)",
                                   "lo": 0.0, "hi": tmax, "unit": "atomic time",
                                   "counts": hl.tolist()}}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--kernel", choices=("persistent", "plain"), default="plain")
    ap.add_argument("--schedule", choices=("longest-first", "index"), default="longest-first")
    ap.add_argument("--refill-min", type=int, default=0,
                    help="persistent kernel: idle lanes a wave gathers before drawing work")
    ap.add_argument("--sweep-refill", action="store_true",
                    help="also time the persistent kernel at several refill thresholds")
    ap.add_argument("--n", type=int, default=None, help="ensemble size (default 2^20)")
    ap.add_argument("--no-compare", action="store_true", help="skip timing the other kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip timing the batched 64-ensemble grid")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="requests of the serving stream to run, paced, by batched launches "
                         "(0: skip serving)")
    ap.add_argument("--serving-saturate", type=int, default=1000,
                    help="requests of the stream the resident kernel serves submitted at once "
                         "(the sustained rate)")
    ap.add_argument("--serving-resident-paced", type=int, default=400,
                    help="requests of the stream to serve paced by the resident kernel "
                         "(0: skip)")
    ap.add_argument("--cpu-sample", type=int, default=1 << 20,
                    help="trajectories the oracle baseline integrates (default: the whole ensemble)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a plain device copy of this size first (HBM counter calibration)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic.json from two rocprofv3 counter runs and exit")
    ap.add_argument("--write-counters", nargs="+", metavar="PMC_DIR",
                    help="write profiles/counters.json from rocprofv3 SQ counter runs and exit")
    args = ap.parse_args()
    if args.write_traffic:
        print(json.dumps(write_traffic(*args.write_traffic, args.copy_calibration_mib or 512)))
        return 0
    if args.write_counters:
        print(json.dumps(write_counters(args.write_counters)))
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU (asked for {max(args.gpus, world)}): the "
              "trajectories are independent and this build measures one GPU's share",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2509_12381_amd import binding, flops, stats
    from paper_2509_12381_amd import workload as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 3
    binding.load()
    dev = torch.device("cuda:0")

    wl = W.full_ensemble()
    if args.n is not None:
        wl = W.thermal_workload(args.n, 0, name=f"liyb-thermal-{args.n}")
    y0_host = wl.initial_states()
    y0 = torch.from_numpy(y0_host).to(dev)
    fin = torch.empty_like(y0)
    obs = torch.empty((W.NOBS, wl.n), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    if args.copy_calibration_mib:
        nel = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def call(kernel, schedule, refill, precision="fp64"):
        return binding.ai_integrate_async(wl.system, y0, wl.t0, wl.tmax, wl.rtol, wl.atol, fin,
                                          obs, kernel=kernel, stream=stream, schedule=schedule,
                                          refill_min=refill, precision=precision)

    def timed(kernel, steps, warmup, schedule=args.schedule, refill=args.refill_min,
              precision="fp64"):
        for _ in range(warmup):
            call(kernel, schedule, refill, precision)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        t_start.record(stream)
        for a, b in ev:
            a.record(stream)
            call(kernel, schedule, refill, precision)
            b.record(stream)
        t_end.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        per = [a.elapsed_time(b) for a, b in ev]
        return t_start.elapsed_time(t_end), per, wall

    progress(f"{wl.name}: inputs on the device")
    total_ms, per_ms, wall = timed(binding.KERNELS[args.kernel] | binding.TIME_KERNEL,
                                   args.steps, args.warmup)
    progress(f"timed {args.steps} calls: {total_ms / args.steps:.3f} ms each")
    ob = obs.cpu().numpy()
    fin64 = fin.cpu().numpy()
    nsteps = float(ob[W.OBS["nsteps"]].sum())
    nfailed = float(ob[W.OBS["nfailed"]].sum())
    flop = flops.algorithmic_flops(ob)
    ms_per_step = total_ms / args.steps
    value = nsteps * args.steps / (total_ms / 1e3)
    call_ms = float(np.mean(per_ms))
    # the integration kernel's own duration in the timed calls: HIP events the
    # library records on the launch stream around it (AI_TIME_KERNEL)
    kernel_ms_each = [binding.ai_kernel_time(back) for back in range(min(args.steps, 64))]
    kernel_ms = float(np.mean(kernel_ms_each))
    achieved = flop / (kernel_ms / 1e3) / 1e12
    status = np.bincount(ob[W.OBS["status"]].astype(int), minlength=6)[1:].tolist()

    info = binding.ai_get_kernel_info(args.kernel)
    runs = {"fp64": (fin64, ob)}
    other = None
    if not args.no_compare:
        other = []
        for okernel in ("plain", "persistent"):
            for osched in ("index", "longest-first"):
                if (okernel, osched) == (args.kernel, args.schedule):
                    continue
                k = max(1, min(args.steps, 5))
                o_total, o_per, _ = timed(okernel, k, 1, osched)
                o_ms = o_total / k
                other.append({"kernel": okernel, "schedule": osched, "ms_per_step": o_ms,
                              "steps_per_s": nsteps / (o_ms / 1e3),
                              "timed_kernel_speedup": o_ms / ms_per_step})
                progress(f"{okernel}/{osched}: {o_ms:.3f} ms per call")
        # the precision variant: single-precision stages (plain kernel)
        k = max(1, min(args.steps, 5))
        o_total, _, _ = timed("plain", k, 1, "longest-first", 0, "fp32-stages")
        o_ms = o_total / k
        runs["fp32-stages"] = (fin.cpu().numpy(), obs.cpu().numpy())
        other.append({"kernel": "plain", "schedule": "longest-first",
                      "precision": "fp32-stages", "ms_per_step": o_ms,
                      "accepted_steps_per_call": float(obs[W.OBS["nsteps"]].sum().item()),
                      "timed_kernel_speedup": o_ms / ms_per_step,
                      "ensemble": ensemble_statistics(W, stats, runs["fp32-stages"][1], wl.tmax)})
        if args.sweep_refill:
            for k_ in (1, 8, 16, 32, 64):
                o_total, _, _ = timed("persistent", 3, 1, "longest-first", k_)
                other.append({"kernel": "persistent", "schedule": "longest-first",
                              "refill_min": k_, "ms_per_step": o_total / 3})

    tuned = None
    if not args.no_compare:
        t_fin = torch.empty_like(y0)
        t_obs = torch.empty_like(obs)
        best, best_ms = binding.ai_tune(wl.system, y0, wl.t0, wl.tmax, wl.rtol, wl.atol,
                                        t_fin, t_obs)
        progress(f"ai_tune: kernel code {best}, {best_ms:.3f} ms")
        tuned = {"best_kernel_code": best, "best_ms": best_ms,
                 "what": "ai_tune: each configuration timed twice on this ensemble, each after an untimed run of itself"}
        del t_fin, t_obs

    batched = None
    if not args.no_batch and args.n is None:
        batched = batched_grid(binding, W, flops, torch)
        progress("batched grid done")

    served = None
    if args.serving_requests > 0 and args.n is None:
        served = serving(binding, W, torch, args.serving_requests,
                         min(args.serving_saturate, args.serving_requests),
                         min(args.serving_resident_paced, args.serving_requests),
                         wl.n * args.steps / (total_ms / 1e3), value)
        progress("serving done")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, y0_host, min(args.cpu_sample, wl.n), runs)
        progress("cpu baseline done")

    traffic = measured_traffic(args.kernel)
    counters = measured_counters(args.kernel)
    counter_rate = None
    if counters and counters.get("SQ_INSTS_VALU") and counters.get("SQ_INSTS_VALU_FLOPS_FP64"):
        util = counters["SQ_THREAD_CYCLES_VALU"] / (64.0 * counters["SQ_INSTS_VALU"])
        hw_flop = 64.0 * counters["SQ_INSTS_VALU_FLOPS_FP64"] * util
        counter_rate = {"counter_tflops": hw_flop / (kernel_ms / 1e3) / 1e12,
                        "counter_frac": hw_flop / (kernel_ms / 1e3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                        "counter_flop_per_launch": hw_flop, "lane_utilisation": util,
                        "valu_insts_per_launch": counters["SQ_INSTS_VALU"],
                        "counter_what": "hardware FP64 FLOPs per launch = 64 x SQ_INSTS_VALU_FLOPS_FP64 "
                                        "x lane utilisation (SQ_THREAD_CYCLES_VALU / 64 SQ_INSTS_VALU), "
                                        "from profiles/counters.json, over this run's kernel_ms"}
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "accepted steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded thermal Li(6 amu) + Yb+(171 amu) ensemble, impact-parameter "
                "sampling, generated on the host",
        "config": {"workload": wl.name, "trajectories": wl.n, "seed": wl.seed,
                   "rtol": wl.rtol, "atol": wl.atol, "kernel": args.kernel,
                   "schedule": args.schedule, "refill_min": args.refill_min,
                   "tmax_rf_periods": 200, "R0_a0": wl.R0, "b_max_a0": wl.b_max},
        "trajectories_per_s": wl.n * args.steps / (total_ms / 1e3),
        "latency_ms": {"p50": float(np.percentile(per_ms, 50)),
                       "p99": float(np.percentile(per_ms, 99)),
                       "what": "one ensemble call, enqueue to completion on the stream"},
        "accepted_steps_per_call": nsteps,
        "rejected_attempts_per_call": nfailed,
        "status_counts": dict(zip(("escaped", "tmax", "maxsteps", "hmin", "nonfinite"), status)),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": traffic, "kernel": KERNEL_SYMBOL[args.kernel],
                     "flop_per_launch": flop, "kernel_ms": kernel_ms, "call_ms": call_ms,
                     "kernel_ms_each": [round(x, 4) for x in reversed(kernel_ms_each)],
                     "call_ms_each": [round(x, 4) for x in per_ms],
                     "what": "achieved: algorithmic FLOPs (the 12-component Dormand-Prince "
                             "attempt, 922 per attempt) over kernel_ms, the integration kernel "
                             "alone (AI_TIME_KERNEL events on the launch stream), the mean of "
                             "kernel_ms_each (the timed calls in order); call_ms: the whole "
                             "call with the schedule, the mean of call_ms_each",
                     **(counter_rate or {"counter_tflops": None})},
        "ensemble": ensemble_statistics(W, stats, ob, wl.tmax),
        "kernel_info": info,
        "other_variants": other,
        "autotune": tuned,
        "batched_grid": batched,
        "serving": served,
        "cpu_baseline": cpu,
        "wall_s_timed_region": wall,
    }
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
