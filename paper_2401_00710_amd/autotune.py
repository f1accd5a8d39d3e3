"""Autotuner of libdtsort's launch parameters on the current GPU.

For every record layout (32-bit keys, 64-bit keys, 64-bit pairs, the batched
32-bit form) and size class it times whole sorts of seeded synthetic inputs
through the C ABI (the score of a parameter set is the summed time of the two
input distributions the layout is benchmarked on, at the class size) and
picks, by coordinate descent, the scatter tile shape, then the digit width,
then the digit width of the levels below the root, then the base-case
cutoff.  The winners are written as rows of the text table the library reads
when dtsort_opts.tuned = 1:

    key_bytes val_bytes segmented log2n_lo log2n_hi digit_bits lds_cutoff tile_shape digit_bits_below

Usage (on a GPU):  python -m paper_2401_00710_amd.autotune --out tune_table.txt
The output is only a speed choice: every parameter set sorts identically.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

TILES = (1, 2, 3, 4, 5, 6)
DIGITS = (8, 9, 10)
DIGITS_BELOW = (8, 9)  # 0 (the start) = as digit_bits
MIN_GAIN = 0.01  # a candidate replaces the current best only when it is at least this much faster


def _cutoffs(kb, vb):
    return (4096, 8192) if (kb == 8 and vb) else (4096, 8192, 16384)


def _inputs(torch, W, kb, vb, seg, n, dev):
    """Seeded inputs a candidate is timed on (its score is the summed time),
    the distributions each record layout is benchmarked on: 32-bit keys
    uniform and Zipf (s = 1); 64-bit keys uniform and the three-part mixture;
    64-bit pairs with exponential and bit-exponential keys; the batched
    workload for the segmented form."""
    if seg:
        # a different seed from the benchmark's batched workload (seed 0), so
        # that the choice is not fitted to the input it is measured on
        c = W.make_config("segmented_u32", seed=1, device=dev)
        return [dict(keys=c["keys"].to(torch.int32), offsets=c["offsets"], vals=None)]
    out = []
    if kb == 4 and vb == 4:
        # 32-bit records of the paper's 32-bit experiments: uniform and Zipf keys
        gens = (lambda: W.uniform_u32(n, seed=1, device=dev).to(torch.int32),
                lambda: W.zipf_u32(n, 1.0, n, seed=2, device=dev).to(torch.int32))
    elif kb == 4:
        gens = (lambda: W.uniform_u32(n, seed=1, device=dev).to(torch.int32),
                lambda: W.zipf_u32(n, 1.0, n, seed=2, device=dev).to(torch.int32))
    elif not vb:
        gens = (lambda: W.uniform_u64(n, seed=1, device=dev),
                lambda: W.mixture_u64(n, seed=2, device=dev))
    else:
        gens = (lambda: W.exponential_keys(n, 1e-5, seed=1, device=dev),
                lambda: W.bit_exponential_keys(n, 0.1, seed=2, device=dev))
    for g in gens:
        v = torch.arange(n, dtype=torch.int32 if vb == 4 else torch.int64, device=dev) if vb else None
        out.append(dict(keys=g(), offsets=None, vals=v))
    return out


def _time(dt, torch, case, inp, work, vwork, params, reps):
    kb, vb, seg = case
    o = dt.make_opts(**params)

    def run():
        if seg:
            dt.sort_segmented(work, inp["offsets"], opts=o)
        elif kb == 4 and vb:
            dt.sort_pairs_u32(work, vwork, o)
        elif kb == 4:
            dt.sort_u32(work, o)
        elif vb:
            dt.sort_pairs_u64(work, vwork, o)
        else:
            dt.sort_u64(work, o)

    ts = []
    for r in range(reps + 1):
        work.copy_(inp["keys"])
        if vwork is not None:
            vwork.copy_(inp["vals"])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        if r:
            ts.append(e0.elapsed_time(e1))
    return statistics.median(ts)


ALL_CASES = [(4, 0, 0), (8, 0, 0), (8, 8, 0), (4, 4, 0), (4, 0, 1)]


def tune(sizes, reps, log, cases=None):
    import torch

    import paper_2401_00710_amd as dt
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rows, report = [], []
    cases = ALL_CASES if cases is None else cases
    # size classes: [lo, hi] of floor(log2 n) and the n timed for the class
    # (the cutoff matters only relative to the bucket sizes the levels leave,
    # so each class is timed at a size inside it)
    classes = [(0, 21, sizes[0]), (22, 25, sizes[1]), (26, 28, sizes[2]), (29, 29, sizes[3]), (30, 63, sizes[4])]
    plan = [(c, cl) if not c[2] else (c, (0, 63, 0)) for c in cases for cl in (classes if not c[2] else classes[:1])]
    for case, (lo, hi, n) in plan:
        kb, vb, seg = case
        inps = _inputs(torch, W, kb, vb, seg, n, dev)
        work = torch.empty_like(inps[0]["keys"])
        vwork = torch.empty_like(inps[0]["vals"]) if inps[0]["vals"] is not None else None

        def score(p):
            return sum(_time(dt, torch, case, inp, work, vwork, p, reps) for inp in inps)

        best = dict(digit_bits=8, lds_cutoff=0, tile_shape=1)
        if seg:
            best["graph"] = 1
        t_best = score(best)
        tried = {json.dumps(best, sort_keys=True): t_best}
        for key, values in (("tile_shape", TILES), ("digit_bits", DIGITS), ("digit_bits_below", DIGITS_BELOW),
                            ("lds_cutoff", _cutoffs(kb, vb))):
            for v in values:
                p = dict(best)
                p[key] = v
                tag = json.dumps(p, sort_keys=True)
                if tag in tried:
                    continue
                t = score(p)
                tried[tag] = t
                log(f"  {case} n={work.numel()} {p} {t:.3f} ms")
                if t < t_best * (1.0 - MIN_GAIN):  # ties within timing noise keep the earlier choice
                    best, t_best = p, t
        log(f"{case} log2n [{lo},{hi}] best {best} {t_best:.3f} ms")
        rows.append((kb, vb, seg, lo, hi, best["digit_bits"], best["lds_cutoff"], best["tile_shape"],
                     best.get("digit_bits_below", 0)))
        report.append(dict(case=case, n=int(work.numel()), best=best, ms=t_best,
                           tried={k: round(v, 4) for k, v in tried.items()}))
        del inps, work, vwork
        torch.cuda.empty_cache()
    return rows, report


def read_table(path):
    """Rows of an existing table (empty if there is none)."""
    rows = []
    if os.path.exists(path):
        for line in open(path):
            if line.startswith("#") or not line.strip():
                continue
            r = tuple(int(x) for x in line.split())
            rows.append(r + (0,) * (9 - len(r)))  # tables written before the last column: 0 there
    return rows


def merge_rows(old, new):
    """The new rows replace every old row of the same record layout; layouts
    not tuned this time keep their rows."""
    layouts = {r[:3] for r in new}
    return [r for r in old if r[:3] not in layouts] + list(new)


def write_table(rows, path, device_name):
    with open(path, "w") as f:
        f.write("# Tuning table of libdtsort (read when dtsort_opts.tuned = 1).\n")
        f.write("# Columns: key_bytes val_bytes segmented log2n_lo log2n_hi digit_bits lds_cutoff tile_shape "
                "digit_bits_below\n")
        f.write("# (0 = automatic).  First matching row wins.\n")
        f.write(f"# Written by python -m paper_2401_00710_amd.autotune on {device_name}, "
                f"{time.strftime('%Y-%m-%d')}.\n")
        for r in rows:
            f.write(" ".join(str(x) for x in r) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tune_table.txt"))
    ap.add_argument("--report", default=None, help="JSON file with every timing")
    ap.add_argument("--sizes", default="1048576,16777216,134217728,1000000000,1073741824",
                    help="n timed for the classes log2n <= 21, 22..25, 26..28, 29, >= 30")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--cases", default=None,
                    help="layouts to tune as kb:vb:seg,... (default all); the table keeps the other layouts' rows")
    args = ap.parse_args()
    import torch

    def log(m):
        print(m, flush=True)

    sizes = [int(x) for x in args.sizes.split(",")]
    cases = None
    if args.cases:
        cases = [tuple(int(x) for x in c.split(":")) for c in args.cases.split(",")]
    rows, report = tune(sizes, args.reps, log, cases)
    write_table(merge_rows(read_table(args.out), rows), args.out, torch.cuda.get_device_name(0))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)
    log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
