"""Summaries of rocprofv3 output for the libensdns kernels.

* ``stats``: per-kernel calls / total / average duration from a
  ``rocprofv3 --kernel-trace --stats`` database (rocpd SQLite).
* ``traffic``: per-launch HBM bytes of each kernel from two ``--pmc`` runs
  (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), each scaled by what the same
  counter reads for a plain device copy of known size.  The result records a
  hash of the kernel sources, so a later change of the kernels invalidates it.

Command line::

    python -m paper_2506_23712_amd.profiling stats DB_DIR --out FILE.md [--title T] [--command C]
    python -m paper_2506_23712_amd.profiling traffic --copy-fetch D --copy-write D --copy-bytes B \
        --fetch D --write D --out FILE.json [--command C]
"""
from __future__ import annotations

import argparse
import collections
import glob
import hashlib
import json
import os
import re
import sqlite3
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))


# sources of the time-step kernels whose traffic the summaries record
STEP_SOURCES = ("kernels_step.hip", "fft.hpp", "gmem.hpp", "ens_internal.h")


def source_hash() -> str:
    """sha256 over the sources of the time-step kernels."""
    h = hashlib.sha256()
    for name in STEP_SOURCES:
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def pass_bytes(n: int, prec: str) -> dict:
    """Algorithmic HBM bytes of one launch of each pass for one member: the
    pass's inputs read once and outputs written once, truncated storage
    without the line padding of the pencil buffers."""
    K = n // 3
    cs = 16 if prec == "fp64" else 8
    S = (2 * K + 1) ** 2 * (K + 1)
    zl = n * (2 * K + 1) * (K + 1)          # one field of z-pencils
    yl = n * n * (K + 1)                    # one field of y-pencils
    return {
        "zinv": (3 * S + 5 * zl) * cs,
        "yinv": (5 * zl + 6 * yl) * cs,
        "xpass": (6 * yl + 3 * yl) * cs,
        "yfwd": (3 * yl + 3 * zl) * cs,
        # stages 2 and 3 read the RK register, stages 1 and 2 write it;
        # average over the 3 stages
        "zfwd_update": (3 * zl + 3 * S + 2 * 3 * S / 3 + 3 * S + 2 * 3 * S / 3) * cs,
    }


def zfwd_stage_bytes(n: int, prec: str, stage: int, fused: bool = False) -> tuple:
    """(read, write) algorithmic bytes of the z forward + update of one RK
    stage for one member: the 3 z-line fields and u_hat read, u_hat written;
    the RK register read in stages 1 and 2 and written in stages 0 and 1; a
    fused kernel (stages 0 and 1, and stage 2 of a step followed by another
    in the same call) also writes the next stage's 5 z-inverse fields."""
    K = n // 3
    cs = 16 if prec == "fp64" else 8
    S, zl = (2 * K + 1) ** 2 * (K + 1), n * (2 * K + 1) * (K + 1)
    r = 3 * zl + 3 * S + (3 * S if stage > 0 else 0)
    w = 3 * S + (3 * S if stage < 2 else 0) + (5 * zl if fused else 0)
    return r * cs, w * cs


def kernel_name(pass_name: str, n: int, prec: str, variant) -> str:
    """Symbol (as rocprofv3 prints it, without arguments) of a pass's kernel."""
    p = "float" if prec == "fp32" else "double"
    if pass_name == "zfwd_update":                             # the kernel of the middle RK stage
        return f"ens::k_zfwd_update<{p}, {n}, 1, {'true' if variant == 1 else 'false'}>"
    ea = 16 if prec == "fp32" else 8
    if pass_name == "xpass" and variant == 6 and n >= 64:
        return f"ens::k_xpass_wave2<{p}, {n}, {ea}>"
    if pass_name == "xpass" and variant in (4, 5) and n >= 64:
        return f"ens::k_xpass_wave<{p}, {n}, {ea if variant == 4 else ea // 2}>"
    if pass_name == "xpass" and variant == 3 and 128 <= n <= 512 and prec == "fp32":
        return f"ens::k_xpass_dma<{p}, {n}, 16>"
    if pass_name == "xpass" and variant in (2, 3) and n >= 64:
        return f"ens::k_xpass_dma<{p}, {n}, 8>"
    if pass_name in ("zinv", "yinv", "yfwd"):                  # variants 2, 3: twice the lines per workgroup
        return f"ens::k_{pass_name}<{p}, {n}, {16 if variant in (1, 3) else 8}, {2 if variant in (2, 3) else 1}>"
    return f"ens::k_{pass_name}<{p}, {n}, {16 if variant == 1 else 8}>"


def _db(path: str) -> sqlite3.Connection:
    if os.path.isdir(path):
        found = glob.glob(os.path.join(path, "**", "*.db"), recursive=True)
        if not found:
            raise FileNotFoundError(f"no rocpd database under {path}")
        path = found[0]
    return sqlite3.connect(path)


def short_name(name: str) -> str:
    n = re.sub(r"\(.*", "", name)
    return n.replace("void ", "").strip()


def kernel_stats(path: str):
    """[(kernel, calls, total_us, average_us, percent)] sorted by total time."""
    db = _db(path)
    rows = db.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    return [(short_name(r[0]), int(r[1]), float(r[2]), float(r[3]), float(r[4])) for r in rows]


def pmc_per_kernel(path: str, counter: str) -> dict:
    """kernel -> list of per-dispatch counter values."""
    out = collections.defaultdict(list)
    for name, val in _db(path).execute("select name, counter_value from pmc_events where counter_name = ?", (counter,)):
        out[short_name(name)].append(float(val))
    return dict(out)


def copy_factor(path: str, counter: str, true_bytes: int) -> float:
    """true bytes / counter bytes for the device copy kernel of the calibration run."""
    vals = [v for k, vs in pmc_per_kernel(path, counter).items() if "copyBuffer" in k or "copy" in k.lower()
            for v in vs]
    if not vals:
        raise ValueError(f"no copy kernel in {path}")
    return true_bytes / (statistics.median(vals) * 1024.0)


def traffic(copy_fetch: str, copy_write: str, copy_bytes: int, fetch: str, write: str) -> dict:
    ff = copy_factor(copy_fetch, "FETCH_SIZE", copy_bytes)
    fw = copy_factor(copy_write, "WRITE_SIZE", copy_bytes)
    f = pmc_per_kernel(fetch, "FETCH_SIZE")
    w = pmc_per_kernel(write, "WRITE_SIZE")
    kernels = {}
    for k in sorted(set(f) | set(w)):
        fb = statistics.mean(f.get(k, [0.0])) * 1024.0 * ff
        wb = statistics.mean(w.get(k, [0.0])) * 1024.0 * fw
        kernels[k] = {"fetch_bytes": round(fb), "write_bytes": round(wb), "bytes_per_launch": round(fb + wb),
                      "launches": max(len(f.get(k, [])), len(w.get(k, [])))}
    return {"source_hash": source_hash(), "fetch_factor": round(ff, 4), "write_factor": round(fw, 4),
            "kernels": kernels}


def trace_averages(path: str) -> dict:
    """kernel -> average duration (us) from a kernel-statistics table written
    by ``stats`` (rows ``| `kernel` | calls | total us | average us | % |``)."""
    out = {}
    with open(path) as f:
        for line in f:
            m = re.match(r"\|\s*`([^`]+)`\s*\|\s*(\d+)\s*\|\s*([\d.]+)\s*\|\s*([\d.]+)\s*\|", line)
            if m:
                out[m.group(1)] = float(m.group(4))
    return out


PEAK_GBS = 8000.0


DEFAULT_WORKLOADS = (("single256_fp64", "fp64", 1), ("ens96_mixed_fp32", "fp32", 25))


def write_summary(n: int, counts, out: str, trace: str | None = None, workloads=None) -> None:
    """Markdown table: measured HBM bytes per launch (profiles/traffic_*.json)
    against the algorithmic bytes of each pass, for the n^3 kernels; with a
    kernel-statistics table of the same kernel sources, each kernel's
    achieved HBM rate (measured and algorithmic bytes over its average
    duration) against the MI355X peak."""
    rows = []
    prof = os.path.join(os.path.dirname(HERE), "profiles")
    avg = trace_averages(trace) if trace else {}
    wls = workloads if workloads else [(w, p, c) for (w, p, _), c in zip(DEFAULT_WORKLOADS, counts)]
    for wl, prec, cnt in wls:
        path = os.path.join(prof, f"traffic_{wl}.json")
        t = json.load(open(path))
        pb = pass_bytes(n, prec)
        K = n // 3
        cs = 16 if prec == "fp64" else 8
        S, zl, yl = (2 * K + 1) ** 2 * (K + 1), n * (2 * K + 1) * (K + 1), n * n * (K + 1)
        rw = {"zinv": (3 * S, 5 * zl), "yinv": (5 * zl, 6 * yl), "xpass": (6 * yl, 3 * yl), "yfwd": (3 * yl, 3 * zl),
              "zfwd_update": (3 * zl + 3 * S + 2 * S, 3 * S + 2 * S)}
        for k in ("zinv", "yinv", "xpass", "yfwd", "zfwd_update"):
            for name, v in sorted(t["kernels"].items()):
                short = name.replace("ens::", "")
                if not (short.startswith(f"k_{k}<") or (k == "xpass" and short.startswith(("k_xpass_dma<", "k_xpass_wave<",
                                                                                          "k_xpass_wave2<")))):
                    continue
                if f", {n}" not in short or ("float" in short) != (prec == "fp32"):
                    continue
                ar, aw = rw[k][0] * cs * cnt, rw[k][1] * cs * cnt
                st = re.match(r"k_zfwd_update<\w+, \d+, (\d)(?:, (true|false))?>", short)
                if st:                                     # one RK stage: its own register traffic
                    r1, w1 = zfwd_stage_bytes(n, prec, int(st.group(1)), st.group(2) == "true")
                    ar, aw = r1 * cnt, w1 * cnt
                us = avg.get(name)
                rows.append((wl, short, ar / 1e9, aw / 1e9, v["fetch_bytes"] / 1e9, v["write_bytes"] / 1e9,
                             (v["fetch_bytes"] + v["write_bytes"]) / (ar + aw), t["source_hash"], us,
                             (v["fetch_bytes"] + v["write_bytes"]) / (us * 1e3) if us else None,
                             (ar + aw) / (us * 1e3) if us else None))
    with open(out, "w") as f:
        f.write(f"# HBM traffic per launch vs algorithmic bytes ({n}^3 members)\n\n")
        f.write("Made by `python -m paper_2506_23712_amd.profiling summary"
                + (f" --n {n}" if n != 256 else "")
                + "".join(f" --workload {w}:{p}:{c}" for w, p, c in (workloads or []))
                + " --out " + os.path.relpath(out, os.path.dirname(HERE))
                + (" --trace " + os.path.relpath(trace, os.path.dirname(HERE)) if trace else "")
                + "` from " + " and ".join(f"`profiles/traffic_{w}.json`" for w, _, _ in wls)
                + " (their commands are recorded inside).  Counters: FETCH_SIZE and WRITE_SIZE (rocprofv3 `--pmc`, one "
                  "counter per run), KiB per dispatch, scaled by what the same counter reads for a plain 1 GiB device "
                  "copy.  Algorithmic bytes: each pass's inputs read once and outputs written once, truncated storage "
                  "(a `zfwd_update` kernel of one RK stage: stage 0 does not read the RK register, stage 2 does not "
                  "write it, and a fused kernel (`true` in its name) also writes the next stage's "
                  "5 z-inverse fields; the stage-averaged figure where the stage is not in the name).  The pencil buffers hold no row "
                  "padding; what the measured bytes add comes from loads that straddle 128-byte lines (the y inverse "
                  "and the z forward read rows of K + 1 values that start anywhere in a line) and from the z planes' "
                  "pad of at most one line.\n\n")
        if trace:
            f.write("Durations: kernel-trace averages from `" + os.path.relpath(trace, os.path.dirname(HERE)) +
                    "` (same kernel sources; averages include the autotuner's launches of each variant).  "
                    f"Rates against the MI355X HBM peak of {PEAK_GBS:.0f} GB/s.\n\n")
        f.write("| workload | kernel | algorithmic read / write GB | measured read / write GB | measured / algorithmic |"
                " average us | measured GB/s (frac) | algorithmic GB/s (frac) | kernel source hash |\n")
        f.write("|---|---|---|---|---|---|---|---|---|\n")
        for r in rows:
            rate = (f"{r[8]:.1f} | {r[9]:.0f} ({r[9] / PEAK_GBS:.2f}) | {r[10]:.0f} ({r[10] / PEAK_GBS:.2f})"
                    if r[8] else "— | — | —")
            f.write(f"| {r[0]} | `{r[1]}` | {r[2]:.3f} / {r[3]:.3f} | {r[4]:.3f} / {r[5]:.3f} | {r[6]:.2f} | {rate} | `{r[7]}` |\n")


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2506_23712_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--out", required=True)
    s.add_argument("--title", default="Kernel statistics")
    s.add_argument("--command", default="")
    s.add_argument("--top", type=int, default=25)
    t = sub.add_parser("traffic")
    for a in ("--copy-fetch", "--copy-write", "--fetch", "--write", "--out"):
        t.add_argument(a, required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--command", default="")
    m = sub.add_parser("summary")
    m.add_argument("--n", type=int, default=256)
    m.add_argument("--counts", type=int, nargs=2, default=(1, 25), metavar=("FP64", "FP32"),
                   help="members of that size per launch in the two workloads")
    m.add_argument("--workload", action="append", default=None, metavar="NAME:PREC:COUNT",
                   help="workload of profiles/traffic_NAME.json, its precision and members per launch of the n^3 "
                        "kernels (repeatable; default single256_fp64 and ens96_mixed_fp32)")
    m.add_argument("--trace", default=None,
                   help="kernel-statistics table (from `stats`) of the same kernel sources, for the rate columns")
    m.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "summary":
        wls = None
        if a.workload:
            wls = [(w.split(":")[0], w.split(":")[1], int(w.split(":")[2])) for w in a.workload]
        write_summary(a.n, a.counts, a.out, a.trace, wls)
        return
    if a.cmd == "stats":
        rows = kernel_stats(a.db)[: a.top]
        with open(a.out, "w") as f:
            f.write(f"# {a.title}\n\n")
            if a.command:
                f.write("Command:\n\n```\n" + a.command + "\n```\n\n")
            f.write(f"Kernel source hash: `{source_hash()}`. Durations in microseconds.\n\n")
            f.write("| kernel | calls | total us | average us | % |\n|---|---|---|---|---|\n")
            for r in rows:
                f.write(f"| `{r[0]}` | {r[1]} | {r[2]:.0f} | {r[3]:.1f} | {r[4]:.2f} |\n")
    else:
        res = traffic(a.copy_fetch, a.copy_write, a.copy_bytes, a.fetch, a.write)
        res["command"] = a.command
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
