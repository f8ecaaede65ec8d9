#!/usr/bin/env python3
"""Benchmark of the round-synchronous innermost rewriter on one MI355X.

One step = one ``trs_normalize`` of the whole workload: the pool is restored
on the device from the resident initial image (no host transfer), then the
rounds run until the fixpoint.  ``value`` is rule applications per second of
the whole job (the paper's "rewritten terms per second"), with the inputs
already in HBM when the timed region starts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg3]
                       [--mode learned|plain|frontier] [--compare plain,frontier]
                       [--weights PATH] [--no-cpu-baseline]

The default workload is the batched configuration: 4096 independent terms
(plus/times trees, g(S^n(0)) and merge sorts in equal parts) in one 2^27-slot
pool, whose full sweeps exceed the 256 MB Infinity Cache.  The timed mode is
the learned frontier (the predictor's parameters come from --weights or the
packaged file, else they are trained on the device first, outside the timed
region); the same workload is also run once in each --compare mode and
reported under ``compare``: the plain sweep (the paper's method) and the
parent-notification frontier without the network (the ablation).  The printed JSON line carries a
``roofline`` object for the round kernel (algorithmic bytes of the run /
device time of the round loop, against 8 TB/s) and a ``cpu_baseline``
object: the CPU oracle timed on a bounded sample of the same workload on one
host core.  The same CPU leg also runs the oracle on every term and compares
its normal forms, element by element, and its per-rule counts with those read
back from the device after each mode's run (``parity``); the script exits
with status 3 when any differs.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str):
    from trs_workloads import generators as G
    if name == "cfg0":
        return G.cfg0()
    if name.startswith("cfg1"):
        n = int(name.split("_")[1]) if "_" in name else 25
        return G.cfg1(n)
    if name == "cfg2":
        return G.cfg2()
    if name == "cfg3":
        return G.cfg3()
    if name == "cfg4":
        return G.cfg4()
    if name.startswith("ttree"):
        d = int(name.split("_")[1]) if "_" in name else 22
        return G.ttree(d)
    if name.startswith("tmsort"):
        parts = name.split("_")[1:]
        d = int(parts[0]) if parts else 23
        k = int(parts[1]) if len(parts) > 1 else 5
        return G.tmsort(d, k)
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes(st: dict, A: int) -> dict:
    """Bytes the method itself must move, from the run's counters, whatever
    shortcut the kernel takes: 1 B state per visited slot; per live
    non-normal-form slot 4 B symbol + 4A B argument indices + A one-byte
    argument-state reads; per rule application A 4-byte argument-symbol reads
    for matching and the rewritten root (4 + 4A + 1 B); per created node
    4 + 4A + 4 + 1 B; per reference-count atomic 8 B (read and write of a
    4-byte count); per collected node its argument indices and free-list
    entry (its count decrements are among the atomics)."""
    parts = {
        "sweep": st["node_visits"] * 1,
        "active": st["active_visits"] * (4 + 4 * A + A),
        "match": st["rule_apps"] * 4 * A,
        "rewrite": st["rule_apps"] * (4 + 4 * A + 1),
        "alloc": st["allocs"] * (4 + 4 * A + 4 + 1),
        "rc_atomics": st["rc_atomics"] * 8,
        "collect": st["frees"] * (4 * A + 4),
    }
    parts["total"] = sum(parts.values())
    return parts


def load_predictor(w, path):
    """Predictor parameters for the workload's system: from path (or the
    packaged default), else trained on the device now from plain-run traces
    (outside the timed region)."""
    from paper_2009_07174_amd import predictor as PR
    path = path or PR.DEFAULT_WEIGHTS
    if os.path.exists(path):
        log(f"[bench] predictor parameters from {path}")
        return PR.load(path, w.trs.symbols)
    log(f"[bench] no predictor at {path}: training one on the device")
    recs = [PR.collect(trs, terms, pool, 1_000_000, log=log)
            for _, trs, terms, pool, _ in PR.training_sets("full")]
    import numpy as np
    params, _ = PR.train(len(w.trs.symbols), np.concatenate(recs), log=log)
    return params


KERNEL_SOURCES = ["paper_2009_07174_amd/csrc/trs_kernels.hip",
                  "paper_2009_07174_amd/csrc/trs_layout.h",
                  "paper_2009_07174_amd/csrc/trs_kernels.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_profile(workload: str, mode: str, block: int, npt: int):
    """The committed counter summary (profiles/*.md, a fenced json block) of
    the round kernel on this workload, mode and launch shape, or None unless
    it was taken with the current kernel source."""
    import glob
    import re
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        m = re.search(r"```json\n(.*?)\n```", open(f).read(), re.S)
        if not m:
            continue
        try:
            d = json.loads(m.group(1))
        except ValueError:
            continue
        if (d.get("workload"), d.get("mode"), d.get("block"), d.get("npt")) != (workload, mode, block, npt):
            continue
        return d if d.get("source_sha256") == kernel_source_hash() else None
    return None


def atomics_roofline(workload: str, mode: str, block: int, npt: int, avg_launch_us: float):
    """Atomic throughput of the round kernel: the atomics per launch that
    the L2 counted (rocprofv3 TCC_ATOMIC, calibrated against a kernel of
    known atomic count) over this run's average launch time, against the
    random-atomic rate trs_membench measured on the same GPU."""
    d = measured_profile(workload, mode, block, npt)
    if not d or d.get("atomics_per_launch") is None or not avg_launch_us:
        return None
    ach = d["atomics_per_launch"] / (avg_launch_us * 1e-6)
    peak = d.get("membench_atomic_peak_per_s")
    return {"achieved": ach, "peak": peak, "unit": "atomics/s",
            "frac": ach / peak if peak else None,
            "per_launch": d["atomics_per_launch"],
            "source": "rocprofv3 --pmc TCC_ATOMIC (profiles/), trs_membench random atomics"}


def measured_traffic(workload: str, mode: str, block: int, npt: int):
    """HBM bytes per launch of the round kernel from the committed counter
    summary: FETCH_SIZE and WRITE_SIZE per launch, each scaled by what the
    counter reads for a copy of known size.  None unless the summary was
    taken on this workload, mode and launch shape with the current kernel
    source."""
    d = measured_profile(workload, mode, block, npt)
    if not d or d.get("fetch_bytes_per_launch") is None or d.get("write_bytes_per_launch") is None:
        return None
    return d["fetch_bytes_per_launch"] + d["write_bytes_per_launch"]


def cpu_baseline(w, budget_s: float = 15.0):
    """The oracle, as it stands, on a bounded sample of the same workload:
    terms in a fixed seeded order until about budget_s of normalisation time
    has accumulated (one host core)."""
    import numpy as np
    from oracle import oracle as O
    o = O.Oracle.from_trs(w.trs)
    order = np.random.default_rng(7174).permutation(len(w.terms))
    apps, secs, used = 0, 0.0, 0
    t_wall = time.time()
    for i in order:
        r = o.run(w.terms[int(i)], with_nf=False)
        apps += r.steps
        secs += r.seconds
        used += 1
        if secs >= budget_s or time.time() - t_wall > 3 * budget_s:
            break
    o.close()
    return {"value": apps / secs if secs > 0 else None, "unit": "rule applications/s",
            "cores": 1, "kind": "oracle",
            "sample": f"{used} of {len(w.terms)} terms of {w.name} in a seeded order, "
                      f"{apps} rule applications, {secs:.2f} s of normalisation on one core"}


def cpu_baseline_all_cores(w, budget_s: float = 15.0, max_threads: int = 16):
    """The oracle on every core the process may use (at most max_threads): a
    thread per core with an oracle of its own (the oracle's library releases
    the interpreter lock while it normalises), taking the workload's terms,
    which are independent, in the same seeded order until about budget_s of
    wall time.  Rate = rule applications / wall time."""
    import threading
    import numpy as np
    from oracle import oracle as O
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, max_threads))
    order = np.random.default_rng(7174).permutation(len(w.terms))
    lock = threading.Lock()
    state = {"next": 0, "apps": 0, "used": 0}
    t0 = time.perf_counter()

    def worker():
        o = O.Oracle.from_trs(w.trs)
        try:
            while True:
                with lock:
                    k = state["next"]
                    if k >= len(order) or time.perf_counter() - t0 > budget_s:
                        return
                    state["next"] = k + 1
                r = o.run(w.terms[int(order[k])], with_nf=False)
                with lock:
                    state["apps"] += r.steps
                    state["used"] += 1
        finally:
            o.close()

    threads = [threading.Thread(target=worker) for _ in range(cores)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    wall = time.perf_counter() - t0
    return {"value": state["apps"] / wall if wall > 0 else None, "unit": "rule applications/s",
            "cores": cores, "kind": "oracle",
            "sample": f"{state['used']} of {len(w.terms)} terms of {w.name} in a seeded order, "
                      f"{state['apps']} rule applications, {wall:.2f} s wall on {cores} threads"}


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def oracle_normal_forms(w, max_threads: int = 16):
    """The oracle's normal forms and per-rule counts for every term of the
    workload (untimed; a thread per host core over the independent terms,
    each with an oracle of its own)."""
    import threading
    import numpy as np
    from oracle import oracle as O
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    nt = max(1, min(cores, max_threads, w.n_terms))
    nfs = [None] * w.n_terms
    counts = [np.zeros(len(w.trs.rules), np.int64) for _ in range(nt)]
    lock = threading.Lock()
    nxt = {"i": 0}

    def worker(k):
        o = O.Oracle.from_trs(w.trs)
        try:
            while True:
                with lock:
                    i = nxt["i"]
                    nxt["i"] = i + 1
                if i >= w.n_terms:
                    return
                r = o.run(w.terms[i])
                nfs[i] = r.nf
                counts[k] += r.counts
        finally:
            o.close()

    ts = [threading.Thread(target=worker, args=(k,)) for k in range(nt)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    return nfs, np.sum(counts, axis=0)


def parity_against_oracle(w, runs: dict) -> dict:
    """Every mode's normal forms (read back from the device after its run)
    compared element by element with the oracle's, and the per-rule counts."""
    import numpy as np
    t0 = time.perf_counter()
    onfs, ocounts = oracle_normal_forms(w)
    out = {"terms": w.n_terms, "compared": "canonical serialisation of every term, element by "
                                           "element, and rule applications per rule",
           "modes": {}}
    for mode, (nfs, counts) in runs.items():
        bad = [i for i in range(w.n_terms) if not np.array_equal(nfs[i], onfs[i])]
        ok_counts = bool(np.array_equal(counts, ocounts))
        out["modes"][mode] = {"ok": not bad and ok_counts, "differing_terms": len(bad),
                              "first_differing_term": bad[0] if bad else None,
                              "counts_equal": ok_counts}
    out["ok"] = all(v["ok"] for v in out["modes"].values())
    out["oracle_wall_s"] = time.perf_counter() - t0
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--mode", default="learned", choices=["plain", "frontier", "learned"])
    ap.add_argument("--compare", default="plain,frontier",
                    help="comma-separated modes run once more for comparison ('' = none)")
    ap.add_argument("--weights", default=None, help="predictor parameters (.npz)")
    ap.add_argument("--threshold", type=float, default=0.1)
    ap.add_argument("--sweep-every", type=int, default=0,
                    help="learned mode: full sweep every k rounds (0 = library default)")
    ap.add_argument("--persistent", action="store_true")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--npt", type=int, default=0)
    ap.add_argument("--max-grid", type=int, default=0, help="workgroups per launch cap (0 = default)")
    ap.add_argument("--pf-depth", type=int, default=0, help="sweep tiles prefetched (0 = as fit)")
    ap.add_argument("--place-fresh", type=int, default=0,
                    help="fresh slots first while the extent is below this %% of the pool")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default (or given) block and nodes per thread")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); the batched "
              "workload would shard by giving each GPU its own pool and share of the terms, "
              "which is not built.", file=sys.stderr)
        sys.exit(2)

    os.environ.setdefault("TRS_PROGRESS", "1")  # round progress on stderr in long runs
    import torch
    from paper_2009_07174_amd import trs as T

    log(f"[bench] building workload {args.workload}")
    w = make_workload(args.workload)
    log(f"[bench] {w.name}: {w.n_terms} terms, {w.initial_nodes} initial nodes, "
        f"pool {w.pool_slots} slots")
    ctx = T.Context(w.pool_slots, w.maxarity)
    ctx.load_trs(w.trs)
    off, code = w.packed()
    ctx.load_terms(off, code)
    MODES = {"plain": T.TRS_MODE_PLAIN, "frontier": T.TRS_MODE_FRONTIER,
             "learned": T.TRS_MODE_LEARNED}
    compare = [m for m in args.compare.split(",") if m and m != args.mode]
    if args.mode == "learned" or "learned" in compare:
        ctx.set_predictor(load_predictor(w, args.weights))
    opts = T.Options(block=args.block, nodes_per_thread=args.npt, mode=MODES[args.mode],
                     persistent=1 if args.persistent else 0, threshold=args.threshold, sweep_every=args.sweep_every,
                     max_grid=args.max_grid, pf_depth=args.pf_depth, place_fresh=args.place_fresh)
    tune = None
    if not args.no_autotune and not args.block and not args.npt:
        # the launch shape is tuned on complete runs (seconds each): on the
        # parent-notification frontier for the frontier and learned modes,
        # on the plain sweep for plain mode
        tmode = T.TRS_MODE_PLAIN if args.mode == "plain" else T.TRS_MODE_FRONTIER
        log(f"[bench] autotuning the launch shape (mode {tmode})")
        tuned, tune = ctx.autotune(T.Options(mode=tmode, threshold=args.threshold,
                                                    sweep_every=args.sweep_every))
        opts.block, opts.nodes_per_thread = tuned.block, tuned.nodes_per_thread
        opts.max_grid = tuned.max_grid
        log(f"[bench] autotune: {tune}")
    stream = torch.cuda.current_stream()
    for i in range(args.warmup):
        st = ctx.normalize(opts)
        log(f"[bench] warmup {i}: {st['rounds']} rounds, {st['rule_apps']} rule apps, "
            f"{st['device_ms']:.1f} ms")
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    stats = []
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        st = ctx.normalize(opts)
        stats.append(st)
        log(f"[bench] step {i}: {st['rounds']} rounds, {st['rule_apps']} rule apps, "
            f"{st['device_ms']:.1f} ms")
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # every normal form of the last timed step, read back through the C-ABI
    # (checked against the oracle in the CPU leg below)
    runs = {args.mode: ([ctx.read_nf(i) for i in range(w.n_terms)], ctx.rule_counts())}
    ev_ms = ev0.elapsed_time(ev1)
    ms_per_step = 1e3 * wall / args.steps
    st = stats[-1]
    apps = st["rule_apps"]
    value = apps * args.steps / wall
    dev_ms = sum(s["device_ms"] for s in stats) / len(stats)
    A = w.maxarity
    ab = algorithmic_bytes(st, A)
    # round kernel: average over the rounds of the step, from the HIP events
    # bracketing the timed region on the library's stream
    rounds = st["rounds"]
    ev_ms_step = ev_ms / args.steps
    achieved = ab["total"] / (ev_ms_step * 1e-3) / 1e9
    res = {
        "metric": "rule applications/s + node-visits/s (HBM GB/s), plain vs learned frontier",
        "value": value,
        "unit": "rule applications/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": w.name, "terms": w.n_terms, "initial_nodes": w.initial_nodes,
                   "pool_slots": w.pool_slots, "maxarity": A, "mode": args.mode,
                   "persistent": bool(args.persistent), "block": opts.block,
                   "max_grid": opts.max_grid,
                   "nodes_per_thread": opts.nodes_per_thread},
        "autotune": tune,
        "rule_apps": apps,
        "node_visits_per_s": st["node_visits"] * args.steps / wall,
        "rounds": rounds,
        "device_ms_per_step": dev_ms,
        "event_ms_per_step": ev_ms_step,
        "us_per_round": 1e3 * ev_ms_step / max(rounds, 1),
        "peak_slots": st["peak_slots"],
        "rc_atomics_per_s": st["rc_atomics"] * args.steps / wall,
        "algorithmic_bytes": ab,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": measured_traffic(w.name, args.mode, opts.block, opts.nodes_per_thread),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "copy-calibrated)",
                     "kernel": "k_round", "launches_per_step": st["launches"],
                     "bytes_per_launch": ab["total"] / max(st["launches"], 1),
                     "avg_launch_us": 1e3 * ev_ms_step / max(st["launches"], 1),
                     "atomics": atomics_roofline(w.name, args.mode, opts.block,
                                                 opts.nodes_per_thread,
                                                 1e3 * ev_ms_step / max(st["launches"], 1))},
        "stats": st,
    }
    if compare:
        res["compare"] = {}
        for m in compare:
            o = T.Options(block=opts.block, nodes_per_thread=opts.nodes_per_thread, mode=MODES[m],
                          persistent=1 if args.persistent else 0, threshold=args.threshold, sweep_every=args.sweep_every,
                          max_grid=opts.max_grid)
            if m == "plain" and tune is not None:
                # the plain sweep has candidate shapes of its own (its round
                # launch examines the scan kernel's lists)
                log("[bench] autotuning the plain sweep's launch shape")
                o, tune_m = ctx.autotune(o)
                log(f"[bench] autotune plain: {tune_m}")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sm = ctx.normalize(o)
            torch.cuda.synchronize()
            wm = time.perf_counter() - t1
            log(f"[bench] compare {m}: {sm['rounds']} rounds, {sm['device_ms']:.1f} ms")
            runs[m] = ([ctx.read_nf(i) for i in range(w.n_terms)], ctx.rule_counts())
            if sm["rule_apps"] != apps:
                raise SystemExit(f"compare {m}: {sm['rule_apps']} rule applications, "
                                 f"expected {apps}")
            res["compare"][m] = {
                "value": sm["rule_apps"] / wm, "ms_per_step": 1e3 * wm, "rounds": sm["rounds"],
                "node_visits": sm["node_visits"], "node_visits_per_s": sm["node_visits"] / wm,
                "full_sweeps": sm["full_sweeps"], "speedup_of_" + args.mode: wm / (wall / args.steps),
                "algorithmic_gbps": algorithmic_bytes(sm, A)["total"] / wm / 1e9,
                "roofline_frac": algorithmic_bytes(sm, A)["total"] / wm / 1e9 / HBM_PEAK_GBPS,
                "block": o.block, "nodes_per_thread": o.nodes_per_thread,
                "max_grid": o.max_grid, "us_per_round": 1e6 * wm / max(sm["rounds"], 1)}
            if m == "plain":
                # the full-sweep round (the paper's method) over the library's
                # device time: per round, the scan kernel's classification
                # and the round kernel's examination of the listed slots
                abm = algorithmic_bytes(sm, A)["total"]
                dev_s = sm["device_ms"] * 1e-3
                R = max(sm["rounds"], 1)
                res["roofline_full_sweep"] = {
                    "bound": "hbm", "achieved": abm / dev_s / 1e9, "peak": HBM_PEAK_GBPS,
                    "unit": "GB/s", "frac": abm / dev_s / 1e9 / HBM_PEAK_GBPS,
                    "traffic": measured_traffic(w.name, "plain", o.block, o.nodes_per_thread),
                    "traffic_unit": "bytes per round launch (k_scan + k_round, copy-calibrated)",
                    "kernel": "k_scan + k_round", "mode": "plain", "rounds": sm["rounds"],
                    "round_launches_per_step": sm["launches"],
                    "bytes_per_round": abm / R, "us_per_round": 1e6 * dev_s / R,
                    "basis": "algorithmic bytes: an estimate of what the method must move "
                             "(per visited slot, active visit and rule application), "
                             "not measured traffic"}
                rf = res["roofline_full_sweep"]
                if rf["traffic"]:
                    rf["measured_frac"] = rf["traffic"] / (rf["us_per_round"] * 1e-6) / 1e9 / HBM_PEAK_GBPS
    if compare:
        # speedups over the plain sweep (the paper's method), from the time
        # of one normalisation in each mode
        times = {args.mode: wall / args.steps}
        times.update({m: v["ms_per_step"] / 1e3 for m, v in res["compare"].items()})
        if "plain" in times:
            res["speedup_over_plain"] = {m: times["plain"] / t for m, t in times.items()
                                         if m != "plain"}
    ctx.close()
    parity_ok = True
    if not args.no_cpu_baseline:
        # the CPU leg: the oracle timed on the host (cpu_baseline), and its
        # normal forms compared with every mode's (parity)
        cpu = host_cpu_model()
        log("[bench] CPU baseline (oracle, one core)")
        res["cpu_baseline"] = cpu_baseline(w)
        res["cpu_baseline"]["cpu"] = cpu
        if w.n_terms > 1:  # independent terms: the oracle on every core as well
            log("[bench] CPU baseline (oracle, all cores)")
            res["cpu_baseline_all_cores"] = cpu_baseline_all_cores(w)
            res["cpu_baseline_all_cores"]["cpu"] = cpu
        log("[bench] parity: every normal form against the oracle's")
        res["parity"] = parity_against_oracle(w, runs)
        parity_ok = res["parity"]["ok"]
        log(f"[bench] parity: {res['parity']}")
    print(json.dumps(res))
    if not parity_ok:
        sys.exit(3)


if __name__ == "__main__":
    main()
