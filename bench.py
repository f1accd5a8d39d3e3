#!/usr/bin/env python3
"""Benchmark of the DovetailSort hot path on one MI355X.

One "step" = one complete sort (every level: sampling, counting sort,
recursion, leaf sorts, dovetail merges) of each input of the workload, with
the inputs already resident in HBM.  Before every sort its input is restored
from a pristine device copy (outside the timed region); each sort is
bracketed by stream synchronisations and timed with HIP events on the sort's
stream; the step time is the sum.

Prints ONE JSON line (rank 0, N=1):
  value      G keys/s of the primary workload: 10^9 uint32 keys in two inputs
             (uniform, and Zipf s = 1 over ranks 1..10^9); a step sorts both
  roofline   the scatter kernel (the dominant kernel): algorithmic bytes per
             launch / its average launch time, measured with HIP events in a
             profiled extra run of each input, against the 8 TB/s HBM peak
  roofline_whole_sort  the whole sort: the method's algorithmic bytes (from
             the sorts' own counters) / the measured step time, against 8 TB/s
  cpu_baseline  the CPU oracle's multicore stable sort (all host threads it is
             given) on a bounded sample of the same inputs; cpu_baseline_1core
             the one-thread numpy definition
  extra      the other workloads (64-bit pairs, batched vs per-instance calls,
             learned vs sampling partitioner)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed_sorts(sortfn, src, work, steps, warmup, extra_src=None, extra_work=None):
    """Restore + sort, warmup then `steps` timed sorts; returns per-step ms."""
    import torch
    s = torch.cuda.current_stream()
    times = []
    for i in range(warmup + steps):
        work.copy_(src)
        if extra_src is not None:
            extra_work.copy_(extra_src)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        sortfn()
        e1.record(s)
        torch.cuda.synchronize()
        if i >= warmup:
            times.append(e0.elapsed_time(e1))
    return times


def roofline_from_stats(stats, kind=3):
    """Dominant kernel (the scatter): algorithmic bytes per launch / average
    launch time, over the launches of the given profiled sorts."""
    ms = sum(st.kernel_ms[kind] for st in stats)
    nb = sum(st.kernel_bytes[kind] for st in stats)
    launches = sum(int(st.kernel_launches[kind]) for st in stats)
    if ms <= 0 or launches == 0:
        return None
    gbs = nb / (ms / 1e3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        # counters taken on an older version of the kernel source do not count
        try:
            import hashlib
            tr = json.load(open(TRAFFIC_FILE))
            h = hashlib.sha256()
            for f in tr["kernel_sources"]:
                h.update(open(os.path.join(ROOT, f), "rb").read())
            if h.hexdigest() == tr["kernel_sources_sha256"]:
                traffic = tr.get("k_scatter_bytes_per_launch")
        except (OSError, ValueError, KeyError):
            traffic = None
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_scatter", "launches": launches,
            "bytes_per_launch": nb / launches, "avg_launch_ms": ms / launches}


def cpu_baseline(srcs, n_sample):
    """The CPU oracle's multicore stable sort (libstdc++ parallel mode on every
    host thread OpenMP is given) on the first n_sample keys of each input,
    scaled to G keys/s."""
    import numpy as np
    from oracle import psort  # the CPU oracle, timed as the reported baseline
    dt, threads = 0.0, 0
    for src in srcs.values():
        k = src[:n_sample].cpu().numpy().view(np.uint32).copy()
        t0 = time.perf_counter()
        threads = psort.sort_u32_(k)
        dt += time.perf_counter() - t0
    cnt = n_sample * len(srcs)
    return {"value": round(cnt / dt / 1e9, 5), "unit": "Gkeys/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_sample} keys of each of the {len(srcs)} inputs (parallel stable sort on "
                      f"{threads} threads, {dt:.2f} s wall)"}


def cpu_baseline_1core(srcs, n_sample):
    """The CPU oracle's definition (numpy stable sort, one thread) on the first
    n_sample keys of each input."""
    import numpy as np
    from oracle import sort as S  # the CPU oracle
    dt = 0.0
    for src in srcs.values():
        k = src[:n_sample].cpu().numpy().view(np.uint32).copy()
        t0 = time.perf_counter()
        S.stable_sort_keys(k)
        dt += time.perf_counter() - t0
    cnt = n_sample * len(srcs)
    return {"value": round(cnt / dt / 1e9, 5), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_sample} keys of each of the {len(srcs)} inputs (numpy stable sort, {dt:.2f} s)"}


def algorithmic_bytes(st, key_bytes, rec_bytes):
    """Bytes the method itself moves in one sort, from the sort's own counters:
    2 s per record of every distribution (scatter read + write), of every
    base-case sort, of every paired base case's merge, of every dovetail-merged
    zone and of every copy between buffers; plus the histogram's read of the
    keys of every distributed record (reported apart)."""
    moved = 2 * rec_bytes * (st.records_distributed + st.records_leaf_sorted + st.records_pair_merged +
                             st.records_merged + st.records_copied)
    hist = key_bytes * st.records_distributed
    return moved, hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=float, default=1e9)
    ap.add_argument("--digit-bits", type=int, default=-1, help="-1: autotuned table; 0: the paper's rule")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 27, help="keys per input for the multicore baseline")
    ap.add_argument("--cpu-sample-1core", type=int, default=1 << 24, help="keys per input for the one-core baseline")
    ap.add_argument("--grid", action="store_true",
                    help="the paper's synthetic grid (Tab. synthetic) as 32+32 and 64+64 records, heavy-key "
                         "detection on (sampling) and off (plain); prints one JSON line")
    ap.add_argument("--merge-study", action="store_true",
                    help="the paper's merge study (Section 6.3): seven distributions, 32+32 and 64+64 records, "
                         "the dovetail merge as a gather, PLMerge-style, Alg. 3 in place, and no merge")
    ap.add_argument("--apps", action="store_true",
                    help="the paper's applications (Section 6.2) on synthetic stand-ins: graph transpose of a "
                         "power-law graph and Morton order of varying-density points")
    ap.add_argument("--once", default=None, metavar="WORKLOAD",
                    help="for profilers: generate WORKLOAD, sort it once (tuned), print its time and exit; one of "
                         + ", ".join(ONCE))
    args = ap.parse_args()
    if args.once:
        return run_once(args.once, int(args.n))
    if args.grid:
        return run_grid(args)
    if args.merge_study:
        return run_merge_study(args)
    if args.apps:
        return run_apps(args)
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus above 1 is not supported "
                                   "(the sort has no multi-GPU path)"}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2401_00710_amd as dt
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = int(args.n)
    tuned = 1 if args.digit_bits < 0 else 0
    dbits = max(args.digit_bits, 0)

    def opts(**kw):
        base = dict(tuned=tuned, digit_bits=dbits)
        base.update(kw)
        return dt.make_opts(**base)

    # ---------------- primary workload: 10^9 uint32 keys in two inputs,
    # uniform and Zipf (s = 1 over ranks 1..10^9); a step sorts both
    log(f"generating uniform and Zipf u32 n={n}")
    srcs = {"uniform": W.uniform_u32(n, seed=0, device=dev).to(torch.int32),
            "zipf1": W.zipf_u32(n, 1.0, n, seed=0, device=dev).to(torch.int32)}
    work = torch.empty_like(srcs["uniform"])
    st = {k: dt.Stats() for k in srcs}
    log("timing the two inputs")
    per = {k: [] for k in srcs}
    for i in range(args.warmup + args.steps):
        for k, src in srcs.items():
            t = timed_sorts(lambda: dt.sort_u32(work, opts(stats=st[k])), src, work, 1, 0)[0]
            if i >= args.warmup:
                per[k].append(t)
    times = [a + b for a, b in zip(per["uniform"], per["zipf1"])]
    ms = statistics.mean(times)
    # correctness spot check of the last output (Zipf): sorted, same sum
    w64 = work.to(torch.int64) & 0xFFFFFFFF
    ok = bool((w64[1:] >= w64[:-1]).all().item()) and int(w64.sum()) == int(
        (srcs["zipf1"].to(torch.int64) & 0xFFFFFFFF).sum())
    # profiled extra run of each input for the roofline
    prof = {}
    for k, src in srcs.items():
        work.copy_(src)
        torch.cuda.synchronize()
        prof[k] = dt.Stats()
        dt.sort_u32(work, opts(stats=prof[k], profile=1))
        torch.cuda.synchronize()
    roof = roofline_from_stats(list(prof.values()))
    kern = {}
    for i, kd in enumerate(dt.Stats.KINDS):
        ms_k = sum(p.kernel_ms[i] for p in prof.values())
        nb = sum(p.kernel_bytes[i] for p in prof.values())
        ln = sum(int(p.kernel_launches[i]) for p in prof.values())
        if ln:
            kern[kd] = {"ms": round(ms_k, 4), "GBs": round(nb / max(ms_k, 1e-9) / 1e6, 1), "launches": ln}
    alg_bytes = sum(p.kernel_bytes[i] for p in prof.values() for i in (1, 3, 5, 6, 7))
    # the whole sort against the HBM peak: the method's algorithmic bytes (from
    # the timed sorts' own counters) over the measured step time
    moved = sum(algorithmic_bytes(st[k], 4, 4)[0] for k in srcs)
    hist = sum(algorithmic_bytes(st[k], 4, 4)[1] for k in srcs)
    whole = {"bound": "hbm", "achieved": round((moved + hist) / (ms / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": round((moved + hist) / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
             "frac_without_hist_reads": round(moved / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
             "bytes_per_step": moved + hist, "hist_read_bytes_per_step": hist, "hist_reads_counted": True,
             "ms_per_step": round(ms, 4),
             "terms": "2 s x (records distributed + leaf-sorted + pair-merged + dovetail-merged + copied) "
                      "+ key bytes x records distributed (histogram reads); s = 4 B"}
    # practical ceiling: the library's own copy kernel (the one the sorts use
    # for finished buckets) on the same buffers, reading and writing 4 B a key
    log("device copy")

    def copy_ms(fn):
        cts = []
        for _ in range(6):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            cts.append(e0.elapsed_time(e1))
        return statistics.median(cts[1:])
    lib_copy_gbs = 2 * 4 * n / (copy_ms(lambda: dt.copy_u32(work, srcs["uniform"])) / 1e3) / 1e9
    torch_copy_gbs = 2 * 4 * n / (copy_ms(lambda: work.copy_(srcs["uniform"])) / 1e3) / 1e9
    ceiling = {"library_copy_kernel_GBs": round(lib_copy_gbs, 1), "torch_copy_GBs": round(torch_copy_gbs, 1),
               "scatter_frac_of_copy": round(roof["achieved"] / lib_copy_gbs, 4) if roof else None,
               "whole_sort_frac_of_copy": round(whole["achieved"] / lib_copy_gbs, 4),
               "sort_floor_frac": None}
    log("cpu baseline")
    cpu = cpu_baseline(srcs, min(args.cpu_sample, n))
    cpu1 = cpu_baseline_1core(srcs, min(args.cpu_sample_1core, n))

    extra = {}
    if not args.no_extra:
        del work, srcs
        extra = run_extra(dt, W, torch, np, n, args, opts)

    # one read and one write of every key per step, against the HBM peak
    ceiling["sort_floor_frac"] = round(2 * 4 * 2 * n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    per_input = {k: {"ms": round(statistics.mean(v), 4), "Gkeys_s": round(n / (statistics.mean(v) / 1e3) / 1e9, 3),
                     "levels": int(st[k].levels), "heavy_keys": int(st[k].heavy_keys)} for k, v in per.items()}
    out = {
        "metric": "G keys/s sorted at n=1e9 + % HBM roofline (dominant kernel; whole sort beside it)",
        "value": round(2 * n / (ms / 1e3) / 1e9, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "u32_1e9_uniform_and_zipf1", "n_per_input": n, "key": "uint32",
                   "inputs": ["uniform over [0, 2^32)", "Zipf s=1.0 over ranks 1..1e9, seeded bijection to keys"],
                   "step": "one stable sort of each input (2e9 keys)", "seed": 0,
                   "parameters": "tuning table" if tuned else f"digit_bits={dbits}", "mode": "sampling"},
        "roofline": roof,
        "roofline_whole_sort": whole,
        "cpu_baseline": cpu,
        "cpu_baseline_1core": cpu1,
        "per_input": per_input,
        "step_ms_all": [round(t, 4) for t in times],
        "sorted_ok": ok,
        "kernels": kern,
        "whole_sort_alg_GBs": round(alg_bytes / (ms / 1e3) / 1e9, 1),
        "practical_ceiling": ceiling,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


ONCE = ("u32_1e9_uniform_and_zipf1", "uniform_u32_1e9", "zipf1_u32_1e9", "exp_pairs_u64_1e9", "bexp_pairs_u64_1e9",
        "bexp_pairs_u64_1e9_split", "uniform_u64_1e9", "bexp_pairs_u64_1e9_learned", "mixture_u64_1e9",
        "mixture_u64_1e9_learned", "mixture_u64_1e9_learned_forced", "batched_4096_segments_graph",
        "batched_4096_segments", "uniform_u32_2p20", "uniform_u32_2p20_graph")


def run_once(name, n):
    """One tuned sort of a named workload (input generated and restored outside
    the sort), for kernel traces and counters; prints the sort's time."""
    import torch

    import paper_2401_00710_amd as dt
    import workloads as W
    if name not in ONCE:
        raise SystemExit(f"unknown workload {name}; one of {', '.join(ONCE)}")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if name == "u32_1e9_uniform_and_zipf1":  # the primary workload: one sort of each input
        for sub in ("uniform_u32_1e9", "zipf1_u32_1e9"):
            run_once(sub, n)
        return
    vals = vsrc = off = None
    kw = {}
    if name.startswith("uniform_u32_2p20"):
        src = W.make_config("uniform_u32_2p20", seed=0, device=dev)["keys"].to(torch.int32)
        kw = dict(graph=1 if name.endswith("graph") else 0)
    elif name.startswith("batched"):
        c = W.make_config("segmented_u32", seed=0, device=dev)
        src, off = c["keys"].to(torch.int32), c["offsets"]
        kw = dict(graph=1 if name.endswith("graph") else 0)
    elif name.startswith("uniform_u32"):
        src = W.uniform_u32(n, seed=0, device=dev).to(torch.int32)
    elif name.startswith("zipf1_u32"):
        src = W.zipf_u32(n, 1.0, n, seed=0, device=dev).to(torch.int32)
    elif name.startswith("uniform_u64"):
        src = W.uniform_u64(n, seed=0, device=dev)
    elif name.startswith("mixture"):
        src = W.mixture_u64(n, seed=0, device=dev)
        if "learned" in name:
            kw = dict(mode=dt.MODE_LEARNED, learned_judge=1 if name.endswith("forced") else 0)
    else:
        src = (W.exponential_keys(n, 1e-5, seed=0, device=dev) if name.startswith("exp")
               else W.bit_exponential_keys(n, 0.1, seed=0, device=dev))
        vsrc = torch.arange(n, dtype=torch.int64, device=dev)
        vals = torch.empty_like(vsrc)
        if name.endswith("learned"):
            kw = dict(mode=dt.MODE_LEARNED)
        elif name.endswith("split"):
            kw = dict(merge_variant=dt.MERGE_SPLIT)
    work = torch.empty_like(src)
    o = dt.make_opts(tuned=1, **kw)
    times = []
    # a graph is recorded on its first call; the small workload is timed as in the bench (six calls)
    for _ in range(6 if name.startswith("uniform_u32_2p20") else (2 if name.startswith("batched") else 1)):
        work.copy_(src)
        if vals is not None:
            vals.copy_(vsrc)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        if off is not None:
            dt.sort_segmented(work, off, opts=o)
        elif vals is not None:
            dt.sort_pairs_u64(work, vals, o)
        elif src.element_size() == 4:
            dt.sort_u32(work, o)
        else:
            dt.sort_u64(work, o)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    print(json.dumps({"once": name, "ms": round(times[-1], 4)}), flush=True)


# The paper's times on its 96-core machine (Tab. synthetic, seconds for 10^9
# records), quoted as context: family -> (32+32 times, 64+64 times) in the
# parameter order of workloads.PAPER_GRID.
PAPER_GRID_S = {
    "unif": ((0.308, 0.506, 0.478, 0.501, 0.500), (0.581, 0.795, 0.859, 1.03, 0.994)),
    "exp": ((0.526, 0.502, 0.435, 0.419, 0.402), (0.976, 0.919, 0.819, 0.782, 0.763)),
    "zipf": ((0.493, 0.524, 0.601, 0.516, 0.446), (1.00, 1.00, 1.04, 0.918, 0.883)),
    "bexp": ((1.11, 0.643, 0.550, 0.512, 0.616), (3.30, 2.75, 1.85, 1.42, 1.32)),
}


def run_grid(args):
    """Every instance of the paper's synthetic grid at n records (default
    10^9) as (32-bit key, 32-bit value) and (64-bit key, 64-bit value)
    records with value = index: one warm-up and `steps` timed sorts each
    (median), tuned parameters, with heavy-key detection (sampling) and
    without it (plain, the paper's ablation)."""
    import numpy as np
    import torch

    import paper_2401_00710_amd as dt
    import workloads as W
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = int(args.n)
    steps = max(1, min(args.steps, 5))
    res = {}
    for bits in (32, 64):
        vt = torch.int32 if bits == 32 else torch.int64
        srt = dt.sort_pairs_u32 if bits == 32 else dt.sort_pairs_u64
        k = v = kw = vw = None
        for fam, params in W.PAPER_GRID.items():
            for i, prm in enumerate(params):
                name = f"{fam}-{prm:g}/{bits}"
                log(f"grid {name}")
                del k, v, kw, vw
                torch.cuda.empty_cache()
                k = W.paper_keys(fam, prm, n, bits, seed=0, device=dev)
                k = k.to(torch.int32) if bits == 32 else k
                v = torch.arange(n, dtype=vt, device=dev)
                kw, vw = torch.empty_like(k), torch.empty_like(v)
                row = {}
                for mode, mname in ((dt.MODE_SAMPLING, "sampling"), (dt.MODE_PLAIN, "plain")):
                    st = dt.Stats()
                    o = dt.make_opts(tuned=1, mode=mode, stats=st)
                    ts = timed_sorts(lambda: srt(kw, vw, o), k, kw, steps, 1, v, vw)
                    m = statistics.median(ts)
                    row[mname] = {"ms": round(m, 3), "Grec_s": round(n / (m / 1e3) / 1e9, 3),
                                  "levels": int(st.levels), "heavy_keys": int(st.heavy_keys),
                                  "merged_records": int(st.records_merged)}
                w64 = kw.to(torch.int64) & (0xFFFFFFFF if bits == 32 else -1)
                if bits == 32:
                    ok = bool((w64[1:] >= w64[:-1]).all().item())
                else:  # unsigned order of int64 bit patterns
                    ws = w64 ^ (-(2 ** 63))
                    ok = bool((ws[1:] >= ws[:-1]).all().item())
                row["sorted_ok"] = ok
                row["plain_over_sampling"] = round(row["plain"]["ms"] / row["sampling"]["ms"], 3)
                ps = PAPER_GRID_S[fam][0 if bits == 32 else 1][i]
                row["paper_96core_s"] = ps
                row["vs_paper_96core"] = round(ps * 1e3 / row["sampling"]["ms"], 2)
                res[name] = row
        del k, v, kw, vw
        torch.cuda.empty_cache()

    def gm(xs):
        return round(math.exp(sum(math.log(x) for x in xs) / len(xs)), 3)
    summary = {}
    for bits in (32, 64):
        for grp, fams in (("standard", ("unif", "exp", "zipf")), ("bexp", ("bexp",))):
            rows = [r for kname, r in res.items() if kname.endswith(f"/{bits}") and kname.split("-")[0] in fams]
            summary[f"{grp}/{bits}"] = {
                "geomean_ms_sampling": gm([r["sampling"]["ms"] for r in rows]),
                "geomean_ms_plain": gm([r["plain"]["ms"] for r in rows]),
                "geomean_plain_over_sampling": gm([r["plain_over_sampling"] for r in rows]),
                "geomean_paper_96core_s": gm([r["paper_96core_s"] for r in rows])}
    print(json.dumps({"grid": "paper synthetic distributions (Tab. synthetic), records with value = index",
                      "n": n, "steps": steps, "timing": "median of steps after one warm-up, HIP events",
                      "summary": summary, "instances": res}), flush=True)


MERGE_STUDY = (("unif", 1000), ("exp", 1), ("exp", 10), ("zipf", 0.6), ("zipf", 1.5), ("bexp", 10), ("bexp", 300))


def run_merge_study(args):
    """The paper's merge study (Section 6.3, Fig. scale c-d): for its seven
    distributions (Unif-10^3, and the lightest and heaviest of Exp, Zipf and
    BExp), sorts of n records with each Step 4 implementation, with
    dovetailing during distribution (no merge step at all) and with no merge
    (the time of the other steps); the merge share is (t - t_none) / t."""
    import torch

    import paper_2401_00710_amd as dt
    import workloads as W
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = int(args.n)
    steps = max(1, min(args.steps, 5))
    variants = (("dtmerge_gather", dt.MERGE_GATHER), ("plmerge", dt.MERGE_PLMERGE),
                ("dtmerge_inplace", dt.MERGE_INPLACE), ("split_at_distribution", dt.MERGE_SPLIT),
                ("no_merge", dt.MERGE_NONE))
    res = {}
    for bits in (32, 64):
        vt = torch.int32 if bits == 32 else torch.int64
        srt = dt.sort_pairs_u32 if bits == 32 else dt.sort_pairs_u64
        k = v = kw = vw = None
        for fam, prm in MERGE_STUDY:
            name = f"{fam}-{prm:g}/{bits}"
            log(f"merge study {name}")
            del k, v, kw, vw
            torch.cuda.empty_cache()
            k = W.paper_keys(fam, prm, n, bits, seed=0, device=dev)
            k = k.to(torch.int32) if bits == 32 else k
            v = torch.arange(n, dtype=vt, device=dev)
            kw, vw = torch.empty_like(k), torch.empty_like(v)
            row = {}
            for vname, mv in variants:
                st = dt.Stats()
                o = dt.make_opts(tuned=1, merge_variant=mv, stats=st)
                ts = timed_sorts(lambda: srt(kw, vw, o), k, kw, steps, 1, v, vw)
                row[vname] = {"ms": round(statistics.median(ts), 3)}
                if mv == dt.MERGE_GATHER:
                    row["merged_records"] = int(st.records_merged)
                    row["merges"] = int(st.merges)
            t0 = row["no_merge"]["ms"]
            for vname, _ in variants[:4]:
                t = row[vname]["ms"]
                row[vname]["merge_ms"] = round(t - t0, 3)
                row[vname]["merge_share"] = round((t - t0) / t, 3)
            row["plmerge_over_gather"] = round(row["plmerge"]["ms"] / row["dtmerge_gather"]["ms"], 3)
            row["inplace_over_gather"] = round(row["dtmerge_inplace"]["ms"] / row["dtmerge_gather"]["ms"], 3)
            row["split_over_gather"] = round(row["split_at_distribution"]["ms"] / row["dtmerge_gather"]["ms"], 3)
            res[name] = row
        del k, v, kw, vw
        torch.cuda.empty_cache()
    print(json.dumps({"merge_study": "Section 6.3 merge study, records with value = index", "n": n,
                      "steps": steps, "timing": "median of steps after one warm-up, HIP events",
                      "instances": res}), flush=True)


def run_apps(args):
    """Graph transpose (CSR in, CSR out) of a synthetic power-law graph of
    2^25 vertices and n edges (Zipf out-degrees s = 0.8, in-degrees s = 1),
    and Morton order of n varying-density points in 2-D and 3-D: whole
    application calls (preparation kernels + the 32+32-bit sort), median of
    `steps` after one warm-up."""
    import torch

    import paper_2401_00710_amd as dt
    import workloads as W
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = int(args.n)
    steps = max(1, min(args.steps, 5))
    o = dt.make_opts(tuned=1)
    res = {}

    def timed(fn):
        ts = []
        for i in range(steps + 1):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            if i:
                ts.append(e0.elapsed_time(e1))
        return statistics.median(ts)
    V = 1 << 25
    log(f"graph: {V} vertices, {n} edges")
    off, tgt = W.power_law_graph(V, n, s_out=0.8, s_in=1.0, seed=0, device=dev)
    tgt = tgt.to(torch.int32)
    ms = timed(lambda: dt.graph_transpose(off, tgt, V, opts=o))
    indeg = torch.bincount(tgt.to(torch.int64), minlength=V)
    res["graph_transpose_powerlaw"] = {"vertices": V, "edges": n, "ms": round(ms, 3),
                                       "Gedges_s": round(n / (ms / 1e3) / 1e9, 3),
                                       "max_in_degree": int(indeg.max()), "paper_context": "TW (1.47e9 edges) 0.888 s, "
                                       "SD (2.04e9) 1.10 s on 96 cores"}
    del off, tgt, indeg
    torch.cuda.empty_cache()
    for dims in (2, 3):
        log(f"morton {dims}-D: {n} points")
        c = W.varden_points(n, dims, seed=0, device=dev).to(torch.int32)
        ms = timed(lambda: dt.morton_sort(c, opts=o))
        res[f"morton_{dims}d_varden"] = {"points": n, "ms": round(ms, 3), "Gpoints_s": round(n / (ms / 1e3) / 1e9, 3),
                                         "paper_context": f"Varden SS{dims}d (1e9 points) "
                                                          f"{0.498 if dims == 2 else 0.512} s on 96 cores"}
        del c
        torch.cuda.empty_cache()
    print(json.dumps({"apps": "Section 6.2 applications on synthetic stand-ins", "n": n, "steps": steps,
                      "results": res}), flush=True)


def run_extra(dt, W, torch, np, n, args, opts):
    dev = torch.device("cuda:0")
    res = {}
    steps = max(1, min(args.steps, 3))

    def one(name, sortfn, src, work, vsrc=None, vwork=None, **info):
        log(f"timing {name}")
        ts = timed_sorts(sortfn, src, work, steps, 1, vsrc, vwork)
        m = statistics.mean(ts)
        res[name] = dict(ms=round(m, 3), Gkeys_s=round(info.pop("count", n) / (m / 1e3) / 1e9, 3), **info)
        return m

    # the small workload (2^20 uniform u32, cache-resident): latency, six runs, median of the last five
    small = W.make_config("uniform_u32_2p20", seed=0, device=dev)["keys"].to(torch.int32)
    sw = torch.empty_like(small)
    ts = timed_sorts(lambda: dt.sort_u32(sw, opts()), small, sw, 5, 1)
    m = statistics.median(ts)
    res["uniform_u32_2p20"] = dict(us=round(m * 1e3, 1), Gkeys_s=round(small.numel() / (m / 1e3) / 1e9, 3),
                                   protocol="6 runs, median of the last 5")
    # the same in the graph form (the first call records; then one graph launch per sort, no host read-back)
    og = opts(graph=1)
    ts = timed_sorts(lambda: dt.sort_u32(sw, og), small, sw, 5, 1)
    m = statistics.median(ts)
    res["uniform_u32_2p20_graph"] = dict(us=round(m * 1e3, 1), Gkeys_s=round(small.numel() / (m / 1e3) / 1e9, 3),
                                         protocol="6 runs, median of the last 5; the first records the graph")
    # n sweep of uniform u32 (where launch overhead stops mattering): prefixes of one 2^30 input
    big = W.uniform_u32(1 << 30, seed=0, device=dev).to(torch.int32)
    bw = torch.empty_like(big)
    sweep = {}
    for lg in (20, 22, 24, 26, 28, 30):
        m_ = 1 << lg
        src_, w_ = big[:m_], bw[:m_]
        ts = timed_sorts(lambda: dt.sort_u32(w_, opts()), src_, w_, 3, 1)
        t_ = statistics.median(ts)
        sweep[f"2^{lg}"] = dict(ms=round(t_, 4), Gkeys_s=round(m_ / (t_ / 1e3) / 1e9, 3))
    res["n_sweep_uniform_u32"] = sweep
    del small, sw, big, bw

    # 64-bit pairs: exponential and bit-exponential keys, value = index
    for name, gen in (("exp_pairs_u64_1e9", lambda: W.exponential_keys(n, 1e-5, seed=0, device=dev)),
                      ("bexp_pairs_u64_1e9", lambda: W.bit_exponential_keys(n, 0.1, seed=0, device=dev))):
        log(f"generating {name}")
        k = gen()
        v = torch.arange(n, dtype=torch.int64, device=dev)
        kw, vw = torch.empty_like(k), torch.empty_like(v)
        st = dt.Stats()
        one(name, lambda: dt.sort_pairs_u64(kw, vw, opts(stats=st)), k, kw, v, vw)
        res[name]["levels"] = int(st.levels)
        res[name]["merged_records"] = int(st.records_merged)
        # dovetailing during distribution: no merge step
        ss = dt.Stats()
        one(name + "_split", lambda: dt.sort_pairs_u64(kw, vw, opts(stats=ss, merge_variant=dt.MERGE_SPLIT)), k, kw,
            v, vw)
        res[name + "_split"].update(levels=int(ss.levels), merges=int(ss.merges), copied_records=int(ss.records_copied))
        if name.startswith("bexp"):
            # the learned partitioner on the input whose bit lengths are geometric
            sl = dt.Stats()
            one(name + "_learned", lambda: dt.sort_pairs_u64(kw, vw, opts(stats=sl, mode=dt.MODE_LEARNED)), k, kw,
                v, vw)
            res[name + "_learned"].update(learned_trained=int(sl.learned_trained), learned_used=int(sl.learned_used),
                                          balance_learned=round(sl.learned_balance, 3),
                                          balance_digit=round(sl.sampling_balance, 3),
                                          cost_learned=round(sl.learned_cost / n, 3),
                                          cost_digit=round(sl.sampling_cost / n, 3),
                                          cost_ideal=round(sl.ideal_cost / n, 3),
                                          judge_ms=round(sl.learned_ms, 3), levels=int(sl.levels))
            res[name + "_learned"]["ms_without_judge"] = round(res[name + "_learned"]["ms"] - sl.learned_ms, 3)
            res["bexp_learned_speedup_vs_sampling"] = round(res[name]["ms"] / res[name + "_learned"]["ms"], 3)
        del k, v, kw, vw
    # n sweep of the exponential pairs (64-bit key, value = index): prefixes of one 2^30 input
    log("n sweep of exponential pairs")
    nb_ = 1 << 30
    big = W.exponential_keys(nb_, 1e-5, seed=0, device=dev)
    bv = torch.arange(nb_, dtype=torch.int64, device=dev)
    bkw, bvw = torch.empty_like(big), torch.empty_like(bv)
    sweep = {}
    for lg in (20, 22, 24, 26, 28, 30):
        m_ = 1 << lg
        kw_, vw_ = bkw[:m_], bvw[:m_]
        ts = timed_sorts(lambda: dt.sort_pairs_u64(kw_, vw_, opts()), big[:m_], kw_, 3, 1, bv[:m_], vw_)
        t_ = statistics.median(ts)
        sweep[f"2^{lg}"] = dict(ms=round(t_, 4), Grec_s=round(m_ / (t_ / 1e3) / 1e9, 3))
    res["n_sweep_exp_pairs_u64"] = sweep
    del big, bv, bkw, bvw
    # batched: 4096 instances in one call vs one call per instance
    log("generating segmented")
    c = W.make_config("segmented_u32", seed=0, device=dev)
    keys, off = c["keys"].to(torch.int32), c["offsets"]
    total = keys.numel()
    kw = torch.empty_like(keys)
    one("batched_4096_segments_graph", lambda: dt.sort_segmented(kw, off, opts=opts(graph=1)), keys, kw,
        count=total, n_total=total, form="one HIP graph launch (device-driven levels, recorded once)")
    one("batched_4096_segments", lambda: dt.sort_segmented(kw, off, opts=opts()), keys, kw, count=total,
        n_total=total, form="one call, level loop with a host read-back per level")
    offh = off.cpu().tolist()
    o_plain = opts()

    def per_instance():
        for i in range(len(offh) - 1):
            a, b = offh[i], offh[i + 1]
            if b - a > 1:
                dt.sort_u32(kw[a:b], o_plain)
    one("per_instance_calls_4096", per_instance, keys, kw, count=total)
    res["batched_speedup_vs_per_instance"] = round(res["per_instance_calls_4096"]["ms"] /
                                                   res["batched_4096_segments"]["ms"], 2)
    res["batched_graph_speedup_vs_per_instance"] = round(res["per_instance_calls_4096"]["ms"] /
                                                         res["batched_4096_segments_graph"]["ms"], 2)
    del keys, kw, off
    # learned partitioner vs sampling partitioner on the 64-bit mixture
    log("generating mixture u64")
    mk = W.mixture_u64(n, seed=0, device=dev)
    mw = torch.empty_like(mk)
    st_s = dt.Stats()
    one("mixture_u64_1e9_sampling", lambda: dt.sort_u64(mw, opts(stats=st_s)), mk, mw)
    for tag, judge in (("", 0), ("_forced", 1)):
        st_l = dt.Stats()
        nm = "mixture_u64_1e9_learned" + tag
        one(nm, lambda: dt.sort_u64(mw, opts(stats=st_l, mode=dt.MODE_LEARNED, learned_judge=judge)), mk, mw)
        res[nm].update(judge="cost judge" if judge == 0 else "model's zones forced",
                       learned_trained=int(st_l.learned_trained), learned_used=int(st_l.learned_used),
                       balance_learned=round(st_l.learned_balance, 3), balance_digit=round(st_l.sampling_balance, 3),
                       cost_learned=round(st_l.learned_cost / n, 3), cost_digit=round(st_l.sampling_cost / n, 3),
                       cost_ideal=round(st_l.ideal_cost / n, 3), judge_ms=round(st_l.learned_ms, 3),
                       ms_without_judge=round(res[nm]["ms"] - st_l.learned_ms, 3), levels=int(st_l.levels))
    res["mixture_u64_1e9_sampling"]["levels"] = int(st_s.levels)
    res["learned_speedup_vs_sampling"] = round(res["mixture_u64_1e9_sampling"]["ms"] /
                                               res["mixture_u64_1e9_learned"]["ms"], 3)
    res["learned_forced_speedup_vs_sampling"] = round(res["mixture_u64_1e9_sampling"]["ms"] /
                                                      res["mixture_u64_1e9_learned_forced"]["ms"], 3)
    # the paper's own multicore numbers, as context only (96-core Xeon, 8-byte pairs)
    res["paper_context_96core_xeon"] = {"unif_1e9_32bit_pairs_s": 0.500, "zipf1_32bit_pairs_s": 0.601,
                                        "exp1_64bit_pairs_s": 0.976, "bexp10_64bit_pairs_s": 3.30}
    return res


if __name__ == "__main__":
    main()
