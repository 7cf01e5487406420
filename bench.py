"""Benchmark: PT2 contributions/s of the MI355X engine on a synthetic workload.

Default: workload C5, the largest that one GPU holds: (18a,18b) electrons in
100 orbitals, 300,000 reference determinants, 959,326,200,000 single+double
contributions, FP64, hash records, split into the 256 subsets of a hash split
(Algorithm 2; the fewest whose two record buffers fit the device: 3.75e9
records, 90 GB each).  The timed region evaluates every subset exactly once, as
--steps contiguous groups of subsets (one pt2_evaluate_parts_device call per
step, each a complete pass of generation, sort and single pass over its
subsets); the subset energies are summed in subset order.  Inputs are
resident in HBM before the timed region starts; --warmup single-subset calls
run before it.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 8] [--warmup 1] [--workload c5|c3|c2]

The roofline entry is for the dominant kernel, the radix rank-and-scatter
kernel of each digit pass: algorithmic bytes per launch (each record read once
and written once: 2 x record_bytes per record) over its average duration,
measured with HIP events on the stream the passes run on, inside the timed
region.  Beside the headline: the FP64 oracle timed on the host cores on a
sample of the same workload (with the engine's result on that sample), the
energy of one subset against the stored oracle result (evaluated alone when
the stored records form a subset of a finer split than the timed one), a few
subsets in the FP32-payload form, and workload C2 (one subset, 1.3e9
contributions) as a second line.

Workload C2 alone (--workload c2): one step = one complete pt2_evaluate.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "PT2 contributions/s at |dE_PT2| <= 1e-6 Eh vs FP64 oracle; p50/p99 latency"
SORT_SRC = os.path.join(ROOT, "paper_1808_02049_amd", "csrc", "sort.hip")
GOLDENS = os.path.join(ROOT, "tests", "golden", "oracle_goldens.json")
# default hash split and oracle sample per workload
SPLIT = {"c2": 0, "c3": 5, "c5": 8}
CPU_SAMPLE = {"c2": 2000, "c3": 150, "c5": 24}


def counters_md(workload, precision):
    return os.path.join(ROOT, "profiles", f"radix_scatter_{workload}_{precision}_hbm_counters.md")


def measured_traffic(workload, precision, record_bytes):
    """HBM bytes per scatter launch from the committed rocprofv3 counter
    summary of this workload, or None if there is none, if the sort kernel
    source changed since those counters were taken, or if the summary covers
    another record format."""
    import hashlib
    import re
    path = counters_md(workload, precision)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"scatter_traffic_bytes_per_launch=(\S+) .*source_sha256_16=([0-9a-f]+)", text)
    r = re.search(r"record_bytes=(\d+)", text)
    if not m or not r or int(r.group(1)) != record_bytes:
        return None
    cur = hashlib.sha256(open(SORT_SRC, "rb").read()).hexdigest()[:16]
    return float(m.group(1)) if cur == m.group(2) else None


def load_workload(name):
    import synth
    w = synth.WORKLOADS[name]
    h, eri, rng = synth.make_integrals(w.norb, w.n_chol, w.seed)
    f = np.load(os.path.join(ROOT, "tests", "golden", f"inputs_{name}.npz"))
    dets, e0 = f["dets"], float(f["e0"])
    c = f["c"] if "c" in f else synth.decaying_coefficients(w.n_ref, w.decay,
                                                            synth.draw_signs(rng, w.n_ref))
    return w, h, eri, dets, c, e0


def host_threads():
    """CPUs this process may run on: its affinity set, capped by a cgroup
    CPU quota if one is set."""
    n = len(os.sched_getaffinity(0))
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()
        if q != "max":
            n = max(1, min(n, int(int(q) // int(per))))
    except (OSError, ValueError):
        pass
    return n


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def neumaier(values):
    s, comp = 0.0, 0.0
    for x in values:
        t = s + x
        comp += (s - t) + x if abs(s) >= abs(x) else (x - t) + s
        s = t
    return s + comp


def golden(name):
    if not os.path.exists(GOLDENS):
        return None
    g = json.load(open(GOLDENS)).get(name)
    if g:
        g = dict(g)
        g["e"] = float.fromhex(g["e_pt2_hex"])
    return g


def cpu_baseline(w, h, eri, dets, c, e0, nref_sample, log2p, gpu_ctx):
    """The FP64 oracle on the first nref_sample references (all their
    contributions), timed on the host cores; the same sample on the GPU gives
    a parity check.  The oracle expands the references on all threads and
    groups 2^log2p hash subsets side by side (one per thread)."""
    import oracle
    threads = host_threads()
    O = oracle.Oracle(h, eri, w.norb, w.nalpha, w.nbeta)
    d, cc = dets[:nref_sample], c[:nref_sample]
    t0 = time.perf_counter()
    ref, _ = O.pt2(d, cc, e0, log2p=log2p, nthreads=threads)
    dt = time.perf_counter() - t0
    got = gpu_ctx.evaluate(d, cc, e0)
    return {"value": ref["n_contrib"] / dt, "unit": "contributions/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {nref_sample} of {len(dets)} references (rank order), all "
                      f"{ref['n_contrib']} of their contributions, {1 << log2p} hash subsets, {dt:.1f} s",
            "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count(),
                     "affinity": len(os.sched_getaffinity(0))},
            "parity_abs_dE": abs(got["e_pt2"] - ref["e_pt2"]),
            "parity_counts_equal": all(got[k] == ref[k] for k in
                                       ("n_contrib", "n_unique", "n_external", "n_in_ref_hit",
                                        "key_xor", "key_sum"))}


def serving_bench(args):
    """Workload C4: 200 requests of different active spaces (10-24 electrons,
    20-60 orbitals, 1e3-5e4 references, FP32-payload form), each on its own
    context.  First all requests are submitted at once (closed loop) to
    measure capacity; then they are replayed open loop with Poisson arrivals
    at 0.7 x that capacity.  Latency runs from a request's arrival (before its
    context is created and its integrals uploaded) to its result."""
    import concurrent.futures as cf
    import threading
    import torch
    import paper_1808_02049_amd as pt2
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    stored = json.load(open(os.path.join(ROOT, "tests", "golden", "serving_requests.json")))
    reqs = synth.serving_requests(count=args.serving_count)
    t_gen = time.perf_counter()
    inputs = [synth.request_inputs(r) for r in reqs]
    nper = [synth.n_excitations_per_det(r.norb, r.nalpha, r.nalpha) for r in reqs]
    contrib = [r.n_ref * k for r, k in zip(reqs, nper)]
    total = sum(contrib)
    print(f"bench: serving {len(reqs)} requests, {total} contributions, inputs in "
          f"{time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    keep = []          # contexts stay resident until the end (no device-wide free mid-run)
    lock = threading.Lock()
    progress = {"done": 0, "t0": time.perf_counter()}

    def one(j):
        r = reqs[j]
        h, eri, dets, c = inputs[j]
        ctx = pt2.Context(h, eri, r.norb, r.nalpha, r.nalpha, precision=args.precision,
                          n_streams=args.serving_streams, timing=args.serving_timing)
        res = ctx.wait(ctx.submit(dets, c, stored[r.index]["e0"]))
        done = time.perf_counter()
        with lock:
            keep.append(ctx)
            progress["done"] += 1
            if progress["done"] % 10 == 0:
                print(f"bench: {progress['done']} requests done, {done - progress['t0']:.1f} s",
                      file=sys.stderr, flush=True)
        return res, done

    pool = cf.ThreadPoolExecutor(max_workers=64)
    # warm-up: the four smallest requests (library load, worker streams)
    for f in [pool.submit(one, j) for j in sorted(range(len(reqs)), key=lambda j: contrib[j])[:4]]:
        f.result()

    # closed loop
    t0 = time.perf_counter()
    futs = [pool.submit(one, j) for j in range(len(reqs))]
    closed = [f.result() for f in futs]
    makespan = max(d for _, d in closed) - t0
    cap_rps = len(reqs) / makespan
    print(f"bench: closed loop {makespan:.1f} s, {total / makespan:.3e} contributions/s",
          file=sys.stderr, flush=True)

    if args.serving_closed_only:
        busy = sorted(((r["ms_total"], j, r["n_partitions"], contrib[j]) for j, (r, _) in enumerate(closed)),
                      reverse=True)
        print(json.dumps({"closed_loop": {"makespan_s": makespan, "contributions_per_s": total / makespan},
                          "request_ms_sum": sum(b[0] for b in busy),
                          "phase_ms_sum": {k: round(sum(r[k] for r, _ in closed), 1)
                                           for k in ("ms_gen", "ms_hist", "ms_sort", "ms_reduce")},
                          "sort_passes": sum(r["n_sort_passes"] for r, _ in closed),
                          "key_bits": sorted({r["key_bits"] for r, _ in closed}),
                          "streams": args.serving_streams}), flush=True)
        pool.shutdown()
        for ctx in keep:
            ctx.close()
        return

    # open loop at 0.7 x capacity
    lam = 0.7 * cap_rps
    arrivals = [r.arrival_s for r in synth.serving_requests(count=args.serving_count, rate_per_s=lam)]
    t0 = time.perf_counter()
    futs = []
    for j, a in enumerate(arrivals):
        dt = t0 + a - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        futs.append(pool.submit(one, j))
        if j % 20 == 0:
            print(f"bench: open loop submitted {j}", file=sys.stderr, flush=True)
    opened = [f.result() for f in futs]
    lat = [(d - (t0 + a)) * 1e3 for (_, d), a in zip(opened, arrivals)]
    busy = sorted(((r["ms_total"], j, r["n_partitions"], contrib[j]) for j, (r, _) in enumerate(closed)),
                  reverse=True)
    span = max(d for _, d in opened) - t0
    same = all(a[0]["e_pt2"] == b[0]["e_pt2"] and a[0]["n_unique"] == b[0]["n_unique"]
               for a, b in zip(closed, opened))
    pool.shutdown()
    torch.cuda.synchronize()
    for ctx in keep:
        ctx.close()
    line = {
        "metric": "PT2 contributions/s at |dE_PT2| <= 1e-6 Eh vs FP64 oracle; p50/p99 latency",
        "value": total / span,
        "unit": "contributions/s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": span * 1e3,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(max(lat))},
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-payload/f64-accumulate",
        "data": "synthetic (seeded integrals and references per request)",
        "config": {"workload": f"c4 serving: {len(reqs)} requests, 10-24 electrons, 20-60 orbitals, "
                               f"1e3-5e4 references, {total} contributions, Poisson arrivals at "
                               f"0.7 x closed-loop capacity",
                   "precision": args.precision, "scheduler_streams": args.serving_streams},
        "arrival_rate_per_s": lam,
        "closed_loop": {"makespan_s": makespan, "contributions_per_s": total / makespan,
                        "requests_per_s": cap_rps},
        "deterministic_across_runs": same,
        "closed_loop_request_ms_sum": sum(b[0] for b in busy),
        "closed_loop_phase_ms_sum": {k: round(sum(r[k] for r, _ in closed), 1)
                                     for k in ("ms_gen", "ms_hist", "ms_sort", "ms_reduce")},
        "closed_loop_sort_passes": sum(r["n_sort_passes"] for r, _ in closed),
        "slowest_requests": [{"index": j, "ms": round(ms, 1), "subsets": p, "contributions": n}
                             for ms, j, p, n in busy[:5]],
    }
    print(json.dumps(line), flush=True)


def split_scope(P, nsub, steps):
    """How much of a split workload a line covers."""
    if nsub == P:
        return f"all {P} subsets of a hash split once, in {steps} steps"
    return (f"PARTIAL: the first {nsub} of the {P} subsets of a hash split "
            f"(a profiling run, not the whole workload), in {steps} steps")


def split_bench(args):
    """A workload evaluated as the 2^log2p subsets of its hash split, every
    subset once in the timed region, as args.steps contiguous groups."""
    import torch
    import paper_1808_02049_amd as pt2

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w, h, eri, dets, c, e0 = load_workload(args.workload)
    log2p = args.log2p if args.log2p >= 0 else SPLIT[args.workload]
    P = 1 << log2p
    stream = torch.cuda.current_stream()
    ctx = pt2.Context(h, eri, w.norb, w.nalpha, w.nbeta, precision=args.precision, timing=True,
                      stream=stream, compress_keys=args.compress_keys, cutoff=args.cutoff)
    d_dets = torch.from_numpy(np.ascontiguousarray(dets).view(np.int64)).cuda()
    d_c = torch.from_numpy(np.ascontiguousarray(c)).cuda()
    torch.cuda.synchronize()
    # --subsets K (profiling runs): only the first K subsets; the line then
    # covers that part of the workload and says so
    nsub = P if args.subsets <= 0 else min(args.subsets, P)
    steps = max(1, min(args.steps, nsub))
    groups = np.array_split(np.arange(nsub), steps)
    print(f"bench: {args.workload} {args.precision}, {P} subsets in {steps} steps, warmup {args.warmup}",
          file=sys.stderr, flush=True)
    for i in range(args.warmup):
        ctx.evaluate_parts(d_dets, d_c, e0, log2p, [i % P])
    torch.cuda.synchronize()
    res, eparts, lat = [], [], []
    t0 = time.perf_counter()
    for i, g in enumerate(groups):
        ts = time.perf_counter()
        r, ep = ctx.evaluate_parts(d_dets, d_c, e0, log2p, g)
        lat.append((time.perf_counter() - ts) * 1e3)
        res.append(r)
        eparts.append(ep)
        print(f"bench: step {i} subsets {g[0]}-{g[-1]} {lat[-1]:.0f} ms, elapsed "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    eparts = np.concatenate(eparts)
    e_total = neumaier(eparts)
    tot = {k: sum(r[k] for r in res) for k in ("n_contrib", "n_after_cutoff", "n_unique", "n_external",
                                               "n_in_ref_hit", "n_sort_passes", "ms_gen", "ms_hist",
                                               "ms_sort", "ms_sort_scatter", "ms_reduce", "ref_cross",
                                               "bytes_sort")}
    rec = res[0]["record_bytes"]
    # every record of a subset is read and written once per digit pass of
    # that subset; the subsets of one call take the same passes
    scatter_bytes = sum(2.0 * rec * r["n_after_cutoff"] * r["n_sort_passes"] / len(g)
                        for r, g in zip(res, groups))
    launches = tot["n_sort_passes"]
    scatter_ms = tot["ms_sort_scatter"] / launches
    achieved = scatter_bytes / launches / (scatter_ms * 1e-3) / 1e9
    pass_gbs = tot["bytes_sort"] / (tot["ms_sort"] * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": tot["n_contrib"] / elapsed, "unit": "contributions/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": elapsed / steps * 1e3,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-payload/f64-accumulate",
        "data": "synthetic (seeded integrals and reference, stand-in for molecular inputs)",
        "config": {"workload": f"{args.workload}: ({w.nalpha}a,{w.nbeta}b) electrons in {w.norb} orbitals, "
                               f"{len(dets)} reference determinants, {tot['n_contrib']} contributions, "
                               + split_scope(P, nsub, steps),
                   "precision": args.precision, "key_bits": res[0]["key_bits"], "record_bytes": rec,
                   "subsets": P},
        "e_pt2": e_total,
        "counts": {k: int(tot[k]) for k in ("n_unique", "n_external", "n_in_ref_hit")},
        "phases_ms": {k: round(tot[k], 1) for k in ("ms_gen", "ms_hist", "ms_sort", "ms_sort_scatter",
                                                    "ms_reduce")},
        "sort_passes": int(launches),
        "roofline": {"kernel": "k_scatter (radix rank-and-scatter, one per digit pass)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, args.precision, rec),
                     "bytes_per_launch": scatter_bytes / launches, "avg_launch_ms": scatter_ms,
                     "whole_digit_pass": {"avg_ms": tot["ms_sort"] / launches, "achieved_GBs": pass_gbs}},
    }
    if args.cutoff > 0:
        # the paper's screening (Section V): terms with |H_ai c_i| below the
        # cutoff are dropped; the contribution count stays the structural one
        line["cutoff"] = {"value": args.cutoff, "n_after_cutoff": int(tot["n_after_cutoff"]),
                          "kept_fraction": tot["n_after_cutoff"] / tot["n_contrib"]}
    # one benchmarked subset against the stored oracle result of its records
    # (with a cutoff: the cutoff's effect on that subset, against the exact
    # cutoff-0 oracle value)
    g = golden(f"{args.workload}_parts12")
    if g and log2p <= 12 and args.precision == "fp64":
        sh = 12 - log2p
        top = {p >> sh for p in g["parts"]}
        whole = len(top) == 1 and sorted(g["parts"]) == list(range(min(top) << sh, (min(top) + 1) << sh))
        key = "parity_vs_oracle" if args.cutoff <= 0 else "cutoff_dE_vs_cutoff0_oracle"
        if whole and min(top) < nsub:
            p = min(top)
            line[key] = {"subset": int(p), "of": P, "engine": float(eparts[p]),
                         "oracle": g["e"], "abs_dE": abs(float(eparts[p]) - g["e"])}
        elif nsub == P:
            # the stored records are one whole subset of a finer split:
            # evaluate that subset alone, after the timed region (not in
            # profiling runs of a few subsets, whose traces it would mix)
            gk = 12 - (len(g["parts"]).bit_length() - 1)
            gp = min(g["parts"]) >> (12 - gk)
            if len(g["parts"]) == 1 << (12 - gk) and sorted(g["parts"]) == list(range(gp << (12 - gk),
                                                                                       (gp + 1) << (12 - gk))):
                _, ep = ctx.evaluate_parts(d_dets, d_c, e0, gk, [gp])
                torch.cuda.synchronize()
                line[key] = {"subset": int(gp), "of": 1 << gk, "engine": float(ep[0]),
                             "oracle": g["e"], "abs_dE": abs(float(ep[0]) - g["e"])}
    ctx.close()
    torch.cuda.synchronize()
    extra = {}
    if args.fp32_subsets > 0 and args.precision == "fp64" and nsub == P and args.cutoff <= 0:
        sel = sorted({5 % P} | set(np.linspace(0, P - 1, args.fp32_subsets).astype(int).tolist()))
        ctx32 = pt2.Context(h, eri, w.norb, w.nalpha, w.nbeta, precision="fp32", timing=True, stream=stream,
                            compress_keys=args.compress_keys)
        ctx32.evaluate_parts(d_dets, d_c, e0, log2p, [sel[0]])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r32, e32 = ctx32.evaluate_parts(d_dets, d_c, e0, log2p, sel)
        torch.cuda.synchronize()
        el32 = time.perf_counter() - t1
        ctx32.close()
        extra["fp32_payload_form"] = {
            "subsets": sel, "value": r32["n_contrib"] / el32, "unit": "contributions/s",
            "max_abs_dE_vs_fp64_path_per_subset": float(np.max(np.abs(e32 - eparts[sel]))),
            "record_bytes": r32["record_bytes"]}
        pv = line.get("parity_vs_oracle")
        if pv and pv["of"] == P and pv["subset"] in sel:
            j = sel.index(pv["subset"])
            extra["fp32_payload_form"]["abs_dE_vs_oracle_subset"] = abs(float(e32[j]) - g["e"])
        elif pv:
            # the oracle's subset belongs to a finer split: evaluated alone
            ctx32 = pt2.Context(h, eri, w.norb, w.nalpha, w.nbeta, precision="fp32", stream=stream,
                                compress_keys=args.compress_keys)
            _, eo = ctx32.evaluate_parts(d_dets, d_c, e0, pv["of"].bit_length() - 1, [pv["subset"]])
            ctx32.close()
            extra["fp32_payload_form"]["abs_dE_vs_oracle_subset"] = abs(float(eo[0]) - g["e"])
            extra["fp32_payload_form"]["oracle_subset"] = {"subset": pv["subset"], "of": pv["of"]}
    del d_dets, d_c
    torch.cuda.synchronize()
    cpu = None
    n_sample = args.cpu_sample if args.cpu_sample >= 0 else CPU_SAMPLE[args.workload]
    if n_sample > 0:
        ctx = pt2.Context(h, eri, w.norb, w.nalpha, w.nbeta, precision="fp64", compress_keys=args.compress_keys)
        cpu = cpu_baseline(w, h, eri, dets, c, e0, n_sample, 4, ctx)
        ctx.close()
    line["cpu_baseline"] = cpu
    if args.c2_line and args.workload != "c2":
        extra["c2_fp64"] = c2_line(args.c2_steps)
    line.update(extra)
    print(json.dumps(line), flush=True)


def c2_run(steps, warmup, precision="fp64", compress_keys=-1):
    """Workload C2 as one subset: steps complete evaluations, device inputs."""
    import torch
    import paper_1808_02049_amd as pt2
    w, h, eri, dets, c, e0 = load_workload("c2")
    stream = torch.cuda.current_stream()
    ctx = pt2.Context(h, eri, w.norb, w.nalpha, w.nbeta, precision=precision,
                      stream=stream, allocator="torch", timing=True, compress_keys=compress_keys)
    d_dets = torch.from_numpy(np.ascontiguousarray(dets).view(np.int64)).cuda()
    d_c = torch.from_numpy(np.ascontiguousarray(c)).cuda()
    torch.cuda.synchronize()
    for _ in range(warmup):
        ctx.evaluate(d_dets, d_c, e0)
    torch.cuda.synchronize()
    lat, results = [], []
    t0 = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        results.append(ctx.evaluate(d_dets, d_c, e0))
        lat.append((time.perf_counter() - ts) * 1e3)
        print(f"bench: c2 step {i} {lat[-1]:.1f} ms E={results[-1]['e_pt2']:.12f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return ctx, w, h, eri, dets, c, e0, results, lat, elapsed


def c2_line(steps):
    ctx, w, h, eri, dets, c, e0, results, lat, elapsed = c2_run(steps, 1)
    ctx.close()
    r = results[0]
    g = golden("c2_full")
    passes = sum(x["n_sort_passes"] for x in results)
    scatter_ms = sum(x["ms_sort_scatter"] for x in results) / passes
    achieved = 2.0 * r["record_bytes"] * r["n_after_cutoff"] / (scatter_ms * 1e-3) / 1e9
    return {"workload": f"c2: (10a,10b) electrons in 40 orbitals, {len(dets)} reference determinants, "
                        f"{r['n_contrib']} contributions, one subset",
            "value": r["n_contrib"] * steps / elapsed, "unit": "contributions/s",
            "ms_per_step": elapsed / steps * 1e3, "steps": steps, "e_pt2": r["e_pt2"],
            "abs_dE_vs_oracle": None if not g else abs(r["e_pt2"] - g["e"]),
            "deterministic": len({x["e_pt2"] for x in results}) == 1,
            "phases_ms": {k: round(sum(x[k] for x in results) / steps, 3)
                          for k in ("ms_gen", "ms_hist", "ms_sort", "ms_sort_scatter", "ms_reduce")},
            "scatter": {"achieved_GBs": achieved, "frac": achieved / HBM_PEAK_GBS, "avg_launch_ms": scatter_ms,
                        "record_bytes": r["record_bytes"]}}


def c2_bench(args):
    """Workload C2 alone: one step = one complete evaluation of its single subset."""
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    ctx, w, h, eri, dets, c, e0, results, lat, elapsed = c2_run(args.steps, args.warmup, args.precision,
                                                                args.compress_keys)
    r = results[0]
    rec = r["record_bytes"]
    passes = sum(x["n_sort_passes"] for x in results)
    n_per_pass = r["n_after_cutoff"] / max(1, r["n_partitions"])
    scatter_ms = sum(x["ms_sort_scatter"] for x in results) / passes
    pass_ms = sum(x["ms_sort"] for x in results) / passes
    bytes_per_pass = 2.0 * rec * n_per_pass
    achieved = bytes_per_pass / (scatter_ms * 1e-3) / 1e9
    pass_gbs = r["bytes_sort"] / r["n_sort_passes"] / (pass_ms * 1e-3) / 1e9
    g = golden("c2_full")
    line = {
        "metric": METRIC, "value": r["n_contrib"] * args.steps / elapsed, "unit": "contributions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-payload/f64-accumulate",
        "data": "synthetic (seeded integrals and reference, stand-in for molecular inputs)",
        "config": {"workload": f"c2: (10a,10b) electrons in 40 orbitals, {len(dets)} reference determinants, "
                               f"{r['n_contrib']} contributions, {r['n_partitions']} subset(s)",
                   "precision": args.precision, "key_bits": r["key_bits"], "record_bytes": rec},
        "e_pt2": r["e_pt2"], "deterministic": len({x["e_pt2"] for x in results}) == 1,
        "phases_ms": {k: round(sum(x[k] for x in results) / args.steps, 3)
                      for k in ("ms_gen", "ms_hist", "ms_sort", "ms_sort_scatter", "ms_reduce")},
        "sort_passes_per_step": passes // args.steps,
        "roofline": {"kernel": "k_scatter (radix rank-and-scatter, one per digit pass)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("c2", args.precision, rec),
                     "bytes_per_launch": bytes_per_pass, "avg_launch_ms": scatter_ms,
                     "whole_digit_pass": {"avg_ms": pass_ms, "achieved_GBs": pass_gbs}},
    }
    if g and args.precision == "fp64":
        line["parity_vs_oracle"] = {"engine": r["e_pt2"], "oracle": g["e"], "abs_dE": abs(r["e_pt2"] - g["e"])}
    n_sample = args.cpu_sample if args.cpu_sample >= 0 else CPU_SAMPLE["c2"]
    line["cpu_baseline"] = cpu_baseline(w, h, eri, dets, c, e0, n_sample, 4, ctx) if n_sample > 0 else None
    print(json.dumps(line), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5", choices=["c2", "c3", "c5"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--cutoff", type=float, default=0.0,
                    help="drop terms with |H_ai c_i| below this (the paper's production setting is 1e-8)")
    ap.add_argument("--log2p", type=int, default=-1, help="hash split (default: 8 for c5, 5 for c3)")
    ap.add_argument("--cpu-sample", type=int, default=-1,
                    help="reference determinants in the oracle's timed sample (0: skip; default per workload)")
    ap.add_argument("--fp32-subsets", type=int, default=4,
                    help="subsets also evaluated in the FP32-payload form after the timed region")
    ap.add_argument("--no-c2-line", dest="c2_line", action="store_false",
                    help="skip the workload C2 line")
    ap.add_argument("--c2-steps", type=int, default=5)
    ap.add_argument("--subsets", type=int, default=0,
                    help="profiling: evaluate only the first K subsets of the split (0: all)")
    ap.add_argument("--compress-keys", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="record keys: -1 library default, 0 bitstrings, 1 combinatorial ranks, 2 hash records")
    ap.add_argument("--serving", action="store_true",
                    help="the serving workload (C4) instead of the single large evaluation")
    ap.add_argument("--serving-count", type=int, default=200)
    ap.add_argument("--serving-streams", type=int, default=4)
    ap.add_argument("--serving-timing", action="store_true",
                    help="time each request's phases with HIP events (serving diagnostics)")
    ap.add_argument("--serving-closed-only", action="store_true",
                    help="measure the closed loop only (diagnostics)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="counter runs: first copy 1 GiB device to device (the reference that scales "
                         "FETCH_SIZE and WRITE_SIZE to bytes)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.gpus != 1:
        print(f"bench.py: this engine runs on one GPU; --gpus {args.gpus} is not supported "
              "(the subsets of the hash split are independent units of work)",
              file=sys.stderr)
        sys.exit(2)
    if args.serving:
        if args.precision == "fp64" and "--precision" not in sys.argv:
            args.precision = "fp32"
        return serving_bench(args)
    if args.workload == "c2" and args.log2p <= 0:
        return c2_bench(args)
    return split_bench(args)


if __name__ == "__main__":
    main()
