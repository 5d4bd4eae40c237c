#!/usr/bin/env python3
"""Summaries of rocprofv3 output for profiles/ (kernel time, HBM traffic, LDS).

    python bench_profile.py stats DIR                 kernel-time table from *_kernel_stats.csv
    python bench_profile.py counters DIR [DIR ...]    per-kernel counter means from
                                                      *_counter_collection.csv
    python bench_profile.py traffic FETCH_DIR WRITE_DIR [--json OUT]
        HBM bytes per dispatch of every kernel: FETCH_SIZE and WRITE_SIZE (KiB
        per dispatch) each scaled by what the same counter reads for the plain
        copy kernel k_copy16 moving exactly 1 GiB (bench.py's copy ceiling) in
        the same run; with --json, the bench step's kernels go to a file that
        bench.py reports as roofline "traffic" while the kernel sources match.

DIR is a rocprofv3 output directory (-d); every CSV below it is read.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os
import re
import sys

COPY_KERNEL = "k_copy16"
COPY_BYTES = 1 << 30
# bench step kernel -> the kernel that does its work (the sums' combine levels
# are tiny and separate)
STEP_KERNELS = {"tpose_f32_16384x16384": (r"^k_tpose<4,", 2 * 16384 * 16384 * 4),
                "tpose_bf16_12288x20000": (r"^k_tpose<2,", 2 * 12288 * 20000 * 2),
                "sum_f32_2^28": (r"^k_reduce_parts<0,", (1 << 28) * 4),
                "sum_i64_2^28": (r"^k_reduce_parts<5,", (1 << 28) * 8)}


def _rows(d: str, suffix: str):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    for f in files:
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                yield {k.strip().lower(): (v or "").strip() for k, v in r.items() if k}


def short(name: str) -> str:
    name = re.sub(r"^void ", "", name)
    name = name.replace("(anonymous namespace)::", "")
    name = re.sub(r"\(.*$", "", name)          # drop the argument list
    return name.replace("xtr::", "").replace("tpk::", "")


def stats(d: str):
    agg = collections.OrderedDict()
    for r in _rows(d, "kernel_stats.csv"):
        n = short(r["name"])
        calls = int(r["calls"])
        tot = float(r["totaldurationns"])
        e = agg.setdefault(n, [0, 0.0, float("inf"), 0.0])
        e[0] += calls
        e[1] += tot
        e[2] = min(e[2], float(r.get("minns", "inf") or "inf"))
        e[3] = max(e[3], float(r.get("maxns", "0") or 0))
    total = sum(v[1] for v in agg.values()) or 1.0
    print(f"{'kernel':60s} {'calls':>7s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'%time':>6s}")
    for n, (c, t, mn, mx) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        print(f"{n[:60]:60s} {c:7d} {t / c / 1e3:10.2f} {mn / 1e3:10.2f} {mx / 1e3:10.2f} "
              f"{100 * t / total:6.2f}")


def counter_means(d: str):
    """{kernel: {counter: [values per dispatch]}}"""
    out = collections.defaultdict(lambda: collections.defaultdict(list))
    per_dispatch = collections.defaultdict(float)
    names = {}
    for r in _rows(d, "counter_collection.csv"):
        key = (r.get("dispatch_id") or r.get("correlation_id"), r["counter_name"])
        per_dispatch[key] += float(r["counter_value"])   # summed over dimensions
        names[key[0]] = short(r["kernel_name"])
    for (disp, cname), v in per_dispatch.items():
        out[names[disp]][cname].append(v)
    return out


def counters(dirs):
    for d in dirs:
        m = counter_means(d)
        print(f"# {d}")
        cn = sorted({c for k in m.values() for c in k})
        print(f"{'kernel':60s} {'dispatches':>10s} " + " ".join(f"{c:>22s}" for c in cn))
        for k in sorted(m):
            n = max(len(v) for v in m[k].values())
            vals = " ".join(f"{(sum(m[k][c]) / len(m[k][c]) if m[k][c] else float('nan')):22.1f}"
                            for c in cn)
            print(f"{k[:60]:60s} {n:10d} {vals}")


def traffic(fetch_dir: str, write_dir: str, json_out: str | None):
    f = counter_means(fetch_dir)
    w = counter_means(write_dir)
    fc = f[COPY_KERNEL]["FETCH_SIZE"]
    wc = w[COPY_KERNEL]["WRITE_SIZE"]
    fkib = sum(fc) / len(fc)
    wkib = sum(wc) / len(wc)
    fscale = COPY_BYTES / (fkib * 1024)
    wscale = COPY_BYTES / (wkib * 1024)
    print(f"Calibration: {COPY_KERNEL} FETCH_SIZE {fkib:.1f} KiB, WRITE_SIZE {wkib:.1f} KiB for "
          f"{COPY_BYTES // 1024} KiB read and written -> fetch scale {fscale:.4f}, "
          f"write scale {wscale:.4f}\n")
    print(f"{'kernel':60s} {'dispatches':>10s} {'fetch MB':>10s} {'write MB':>10s} {'HBM MB':>10s}")
    per = {}
    for k in sorted(set(f) | set(w)):
        fv = f[k].get("FETCH_SIZE", [])
        wv = w[k].get("WRITE_SIZE", [])
        if not fv or not wv:
            continue
        fb = sum(fv) / len(fv) * 1024 * fscale
        wb = sum(wv) / len(wv) * 1024 * wscale
        per[k] = (fb, wb)
        print(f"{k[:60]:60s} {len(fv):10d} {fb / 1e6:10.1f} {wb / 1e6:10.1f} {(fb + wb) / 1e6:10.1f}")
    if json_out:
        sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
        import bench
        ks = {}
        print(f"\n{'step call':28s} {'alg MB':>10s} {'HBM MB':>10s} {'HBM/alg':>8s}")
        for call, (pat, alg) in STEP_KERNELS.items():
            hit = [k for k in per if re.search(pat, k)]
            if len(hit) != 1:
                print(f"{call}: {len(hit)} kernels match {pat!r}; skipped")
                continue
            fb, wb = per[hit[0]]
            ks[call] = {"kernel": hit[0], "hbm_bytes_per_launch": int(round(fb + wb)),
                        "fetch_bytes": int(round(fb)), "write_bytes": int(round(wb)),
                        "algorithmic_bytes": alg}
            print(f"{call:28s} {alg / 1e6:10.1f} {(fb + wb) / 1e6:10.1f} {(fb + wb) / alg:8.4f}")
        with open(json_out, "w") as fh:
            json.dump({"source_hash": bench.kernel_source_hash(),
                       "note": "HBM bytes per call from rocprofv3 FETCH_SIZE/WRITE_SIZE scaled by a "
                               "1 GiB copy; valid only for the kernel sources with this hash",
                       "calibration": {"fetch_scale": round(fscale, 5), "write_scale": round(wscale, 5),
                                       "copy_bytes": COPY_BYTES},
                       "kernels": ks}, fh, indent=1)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    b = sub.add_parser("counters")
    b.add_argument("dirs", nargs="+")
    c = sub.add_parser("traffic")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--json", default=None)
    args = ap.parse_args()
    if args.cmd == "stats":
        stats(args.dir)
    elif args.cmd == "counters":
        counters(args.dirs)
    else:
        traffic(args.fetch_dir, args.write_dir, args.json)


if __name__ == "__main__":
    main()
