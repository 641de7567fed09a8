#!/usr/bin/env python3
"""Throughput of the ensemble-DNS hot path on one MI355X.

Metric: grid-point RK steps per second, sum over members of N^3 x RK3 steps
per wall second (the cost unit N^3 M of the paper's cost-ratio estimate,
section "Extrapolating to the frontier of current turbulence simulations").

A timed step is one RK3 step of every member of the workload; gradient
statistics are accumulated every 10th step (as in the workloads' recipe) and
the Gaussian mixture of all members is formed once at the end, all inside the
timed region.  Inputs are seeded synthetic fields (E(k) ~ k^4 exp(-2(k/2)^2),
energy 0.5) resident in HBM before timing starts.

Workloads
  ens96_mixed_fp32 : 96 members, lambda = linspace(-5, 6, 96), eps = e^lambda,
                     nu = 0.03395, band |m| <= 2.5, CFL 0.5, grid = smallest of
                     64/128/256 with K eta(lambda) >= 1.5 (47 x 64^3, 24 x 128^3,
                     25 x 256^3), FP32 transforms/RHS with FP64 reductions.
  single256_fp64   : one 256^3 member, nu = 4.594e-3 (k_max eta ~ 1.5),
                     eps = 1, band |m| <= 2.5, CFL 0.5, FP64.
The JSON line reports the first as `value` and the second beside it, and for
each workload the rate of RK steps alone (`rk_only`: median and interquartile
range of five repeats, without statistics snapshots or the mixture).
  ens48_128_fp64   : (only with --only ens48_128_fp64) the 48-member 128^3 FP64
                     set of the ensemble driver: lambda = i ln2/3, i = -22..25,
                     band [1.4, 2.3], CFL 0.2, k_M eta = 3 for lambda = 0.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def ens96_specs(ens):
    nu, specs = 0.03395, []
    lams = [-5.0 + 11.0 * i / 95 for i in range(96)]
    for i, lam in enumerate(lams):
        eta = (nu ** 3 / math.exp(lam)) ** 0.25
        n = next((g for g in (64, 128, 256) if (g // 3) * eta >= 1.5), 256)
        specs.append(ens.MemberSpec(n=n, nu=nu, eps_ref=1.0, lam=lam, kf_lo=0.0, kf_hi=2.5, dt=0.0, cfl=0.5,
                                    precision="fp32", seed=23712 + i))
    return specs


def single256_specs(ens):
    return [ens.MemberSpec(n=256, nu=4.594e-3, eps_ref=1.0, lam=0.0, kf_lo=0.0, kf_hi=2.5, dt=0.0, cfl=0.5,
                           precision="fp64", seed=23712)]


def ens48_128_specs(ens):
    from paper_2506_23712_amd import run_ensemble
    return run_ensemble.ens128_specs(ens, n=128, precision="fp64")


def hist_for(ens, nu):
    return ens.HistSpec(qr_bins=256, q_lo=-30, q_hi=30, r_lo=-60, r_hi=60, log_bins=512, log10_lo=-8,
                        log10_hi=5, a_bins=1024, a_lo=-100, a_hi=100, eps_ref=1.0, nu_ref=nu)


def pass_bytes(n: int, prec: str) -> dict:
    from paper_2506_23712_amd import profiling
    return profiling.pass_bytes(n, prec)


def run_workload(ens, torch, name, specs, steps, warmup, stats_every, hist_nu, autotune=True, develop=0):
    E = ens.Ensemble(hist=hist_for(ens, hist_nu), graphs=True)
    members = [E.add_member(s) for s in specs]
    torch.cuda.synchronize()
    variants = E.autotune() if autotune else E.variants()

    def advance(k):
        """k steps with a statistics snapshot after every stats_every-th; the
        steps between snapshots are one library call (inside a call, each step
        but the last hands its final z inverse to the next)."""
        done = 0
        while done < k:
            chunk = min(stats_every - done % stats_every, k - done) if stats_every else k - done
            E.step(chunk)
            done += chunk
            if stats_every and done % stats_every == 0:
                E.accumulate_stats()

    advance(warmup)
    for m in members:
        m.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    advance(steps)
    mix = E.mix(0.023, math.log(8), mode=0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pts = sum(s.n ** 3 for s in specs)
    # RK steps alone (no statistics, no mixture): five repeats of a quarter of the
    # timed steps each, for the median and the interquartile range
    rk = []
    for _ in range(5):
        k = max(1, steps // 4)
        torch.cuda.synchronize()
        r0 = time.perf_counter()
        E.step(k)
        torch.cuda.synchronize()
        rk.append(pts * k / (time.perf_counter() - r0))
    rk.sort()
    diverged = [m.id for m in members if m.diag()["diverged"]]
    # per-kernel times with HIP events on the launch stream, per grid size
    groups = sorted({(s.n, s.precision) for s in specs}, reverse=True)
    prof = {}
    for (n, prec) in groups:
        sel = [m for m in members if m.spec.n == n and m.spec.precision == prec]
        acc = None
        reps = 3
        for _ in range(reps):
            p = E.profile_step(sel)
            acc = p if acc is None else {k: acc[k] + p[k] for k in p}
        prof[(n, prec)] = ({k: v / reps for k, v in acc.items()}, len(sel))
    # one statistics snapshot of the whole workload, HIP events on the launch stream
    # (optionally after `develop` more steps, so that the gradients have their
    # developed, heavy-tailed distribution)
    if develop:
        E.step(develop)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    E.accumulate_stats()
    ev1.record()
    torch.cuda.synchronize()
    stats_ms = ev0.elapsed_time(ev1)
    E.close()
    return {"name": name, "seconds": t1 - t0, "points": pts, "rate": pts * steps / (t1 - t0), "variants": variants,
            "ms_per_step": 1e3 * (t1 - t0) / steps, "prof": prof, "diverged": diverged,
            "mix_weight_sum": float(mix["weights"].sum()), "stats_snapshot_ms": stats_ms,
            "rk_only": {"median": rk[2], "iqr": [rk[1], rk[3]], "repeats": 5, "steps_each": max(1, steps // 4)}}


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary of
    this workload, if it was taken on the current kernel sources; else None."""
    from paper_2506_23712_amd import profiling
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("source_hash") != profiling.source_hash():
        return None
    for name, v in t["kernels"].items():
        if name.replace(" ", "").startswith(kernel.replace(" ", "")):
            return v["bytes_per_launch"]
    return None


def dominant_kernel(res):
    """The kernel with the largest summed event time per step, from the
    per-pass times: the y inverse, x pass and y forward launch one kernel in
    every RK stage; the z inverse too, or only in the first stage where the z
    forward performs the next stage's (its variant 1); the z forward launches
    a different kernel in each stage (its time split evenly over the three,
    the middle stage's kernel standing for them).  Returns ((n, prec), pass,
    members, ms per launch, launches per step, fused)."""
    best = None
    for (n, prec), (ms, count) in res["prof"].items():
        fused = res["variants"].get(f"zfwd_update:{n}:{prec}", 0) == 1
        for k, v in ms.items():
            if k not in pass_bytes(n, prec):
                continue
            launches = 1 if (k == "zinv" and fused) else 3
            per_kernel = v / 3 if k == "zfwd_update" else v
            if best is None or per_kernel > best[0]:
                best = (per_kernel, (n, prec), k, count, v / launches, launches, fused)
    return best[1:]


def roofline(res):
    """Roofline point of the dominant kernel: its algorithmic bytes per launch
    over its average launch duration."""
    from paper_2506_23712_amd import profiling
    (n, prec), k, count, avg_ms, launches, fused = dominant_kernel(res)
    if k == "zfwd_update":
        bytes_launch = sum(profiling.zfwd_stage_bytes(n, prec, 1, fused)) * count
    else:
        bytes_launch = pass_bytes(n, prec)[k] * count
    gbs = bytes_launch / (avg_ms * 1e-3) / 1e9
    v = res["variants"].get(f"{k}:{n}:{prec}")
    pname = profiling.kernel_name(k, n, prec, v)
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(res["name"], pname),
            "kernel": pname.replace("ens::", ""), "avg_launch_ms": round(avg_ms, 4),
            "bytes_per_launch": int(bytes_launch), "members_per_launch": count}


def cpu_baseline(specs, steps=3):
    """The oracle, as it stands, on `steps` RK3 steps of one member of each grid size
    (about 10 s of host work; the field set-up is outside the timed region)."""
    import oracle
    sizes = sorted({s.n for s in specs})
    threads = oracle.num_threads()
    work = []
    for n in sizes:
        s = next(x for x in specs if x.n == n)
        u = oracle.init_field(n, s.seed, k_peak=s.k_peak, e0=s.e0)
        m = oracle.Member(n=n, nu=s.nu, eps=s.eps_ref * math.exp(s.lam), kf_lo=s.kf_lo, kf_hi=s.kf_hi, dt=s.dt,
                          cfl=s.cfl)
        work.append((m, u))
    t0 = time.perf_counter()
    pts = 0
    for m, u in work:
        oracle.run(m, u, steps)
        pts += m.n ** 3 * steps
    dt = time.perf_counter() - t0
    # the same on one thread, smallest grid only
    m, u = work[0]
    oracle.set_threads(1)
    s0 = time.perf_counter()
    oracle.run(m, u, steps)
    d1 = time.perf_counter() - s0
    oracle.set_threads(threads)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": round(pts / dt, 1), "unit": "grid-pt RK steps/s", "cores": threads, "kind": "oracle",
            "host_cpu": model,
            "sample": f"{steps} FP64 RK3 steps of one member at each of {sizes} (oracle, {threads} OpenMP threads), "
                      f"{dt:.1f} s",
            "one_thread": {"value": round(m.n ** 3 * steps / d1, 1), "sample": f"{steps} steps at {m.n}^3, {d1:.1f} s"}}


def diagnostics(ens, torch, reps=20):
    """HIP-event times of the spectral diagnostics on 256^3 members (FP32 and FP64):
    shell spectrum, integral scales (each reads the 3 velocity components once),
    and refinement of a 128^3 member onto 256^3 (reads the 128^3 field, writes
    the 256^3 field and clears its RK register)."""
    out = {}
    stream = torch.cuda.current_stream()
    for prec, cs in (("fp32", 8), ("fp64", 16)):
        E = ens.Ensemble()
        a = E.add_member(ens.MemberSpec(n=128, nu=0.02, eps_ref=1.0, kf_hi=2.5, precision=prec, seed=1))
        b = E.add_member(ens.MemberSpec(n=256, nu=0.02, eps_ref=1.0, kf_hi=2.5, precision=prec, seed=2))
        E.step(2)
        S = lambda n: (2 * (n // 3) + 1) ** 2 * (n // 3 + 1)
        cases = {"spectrum": (b.spectrum, 3 * S(256) * cs),
                 "integral_scales": (b.integral_scales, 3 * S(256) * cs),
                 "refine_128_to_256": (lambda: b.refine_from(a), 3 * S(128) * cs + 6 * S(256) * cs)}
        for name, (fn, nbytes) in cases.items():
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) / reps * 1e3
            gbs = nbytes / (us * 1e-6) / 1e9
            out[f"{name}_{prec}"] = {"us": round(us, 2), "bytes": nbytes, "GB/s": round(gbs, 1),
                                     "frac": round(gbs / HBM_PEAK_GBS, 4)}
        E.close()
    return out


def tail_probs(counts_log, lo, hi, nbins, n_samples, xs):
    """P(X >= 10^b) from a log10 histogram (counts per bin, then under, over,
    nan), at the bin edges nearest to log10 of each threshold in `xs`."""
    import numpy as np
    c = np.asarray(counts_log, dtype=np.float64)
    w = (hi - lo) / nbins
    out = {}
    for x in xs:
        b = int(round((math.log10(x) - lo) / w))
        out[f"{x:g}"] = float((c[b:nbins].sum() + c[nbins + 1]) / n_samples)
    return out


def mixed_tail_probs(pdf_log, lo, hi, nbins, xs):
    """The same from a mixed log10 PDF (density per log10 unit)."""
    import numpy as np
    p = np.asarray(pdf_log, dtype=np.float64)
    w = (hi - lo) / nbins
    return {f"{x:g}": float(p[int(round((math.log10(x) - lo) / w)):].sum() * w) for x in xs}


def config5(ens, torch, args):
    """Single member 1024^3 FP32, band |m| <= 2.5, nu set for R_lambda ~ 280,
    500 steps with statistics every 10 into 512-bin log10 histograms of
    eps/<eps> and omega^2/<omega^2>; beside it the 96-member FP32 set run to a
    developed state and mixed (c = 0.023) at the scale gap Z whose reference
    R_lambda is the 1024^3 member's.  nu is calibrated from the 96-member set:
    R_lambda = A e^(lambda/6) fitted over lambda >= 0, R_lambda ~ nu^(-1/2) at
    fixed injection and band, so nu = nu_96 (A / 280)^2."""
    import numpy as np
    xs = (3, 10, 30, 100, 300, 1000, 3000)
    nu96 = 0.03395
    t_start = time.perf_counter()
    log = lambda msg: print(f"[config5 {time.perf_counter() - t_start:7.1f}s] {msg}", file=sys.stderr, flush=True)
    h96 = hist_for(ens, nu96)
    E96 = ens.Ensemble(hist=h96, graphs=True)
    ms96 = [E96.add_member(sp) for sp in ens96_specs(ens)]
    E96.autotune()
    for k in range(args.c5_ens_transient // 500):
        E96.step(500)
        torch.cuda.synchronize()
        log(f"ens96 transient {500 * (k + 1)} steps")
    for m in ms96:
        m.reset_stats()
    for k in range(args.c5_ens_measure // 10):
        E96.step(10)
        E96.accumulate_stats()
        if (k + 1) % 50 == 0:
            torch.cuda.synchronize()
            log(f"ens96 measured {10 * (k + 1)} steps")
    gap = E96.scale_gap(280.0)
    A = gap["prefactor"]
    nu = nu96 * (A / 280.0) ** 2
    log(f"ens96: R_lambda(0) fit A = {A:.2f}; 1024^3 nu = {nu:.4e}")
    # The large scales develop over several integral times, which the 1024^3
    # grid would spend minutes on: the member starts on 256^3 (the same nu,
    # under-resolved), is refined onto 512^3 and then onto 1024^3 (spectral
    # refinement keeps every mode), and each grid runs long enough for its
    # new small scales to fill in.
    E = ens.Ensemble(hist=hist_for(ens, nu), graphs=True)
    chain = [(256, args.c5_coarse_steps), (512, args.c5_mid_steps), (1024, args.c5_transient)]
    prev = None
    for n, steps in chain:
        spec = ens.MemberSpec(n=n, nu=nu, eps_ref=1.0, lam=0.0, kf_lo=0.0, kf_hi=2.5, dt=0.0, cfl=0.5,
                              precision="fp32", seed=23712)
        m = E.add_member(spec)
        if prev is not None:
            m.refine_from(prev)
        for k in range(0, steps, 500):
            E.step(min(500, steps - k), members=[m])
            torch.cuda.synchronize()
            d = m.diag()
            log(f"{n}^3 transient {min(k + 500, steps)} steps: t {d['t']:.3f} E {d['E']:.4f} D {d['D']:.4f} "
                f"R_lambda {d['rlambda']:.1f} kmax_eta {d['kmax_eta']:.3f}")
            if d["diverged"]:
                raise RuntimeError(f"config5: the {n}^3 stage diverged")
        prev = m
    E.autotune(members=[m])
    log("1024^3 variants tuned")
    m.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.c5_steps):
        E.step(1, members=[m])
        if (i + 1) % 10 == 0:
            E.accumulate_stats(members=[m])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d = m.diag()
    own = E.scale_gap(280.0, members=[m])["rlambda"][0]   # from the snapshot-averaged E and D
    counts, mom, npts = m.stats()
    h = E.hist
    hg = {"qr": h.qr_bins ** 2 + 3, "le": h.log_bins + 3}
    c = counts.numpy()
    le = c[hg["qr"]:hg["qr"] + hg["le"]]
    lw = c[hg["qr"] + hg["le"]:hg["qr"] + 2 * hg["le"]]
    mean_eps, mean_ens = float(mom[12] / npts), float(mom[16] / npts)
    # thresholds in units of each member's own mean (eps_ref = 1 = injection; Omega* = omega^2 nu / eps_ref)
    member = {"eps": tail_probs(le, h.log10_lo, h.log10_hi, h.log_bins, npts, [x * mean_eps for x in xs]),
              "enstrophy": tail_probs(lw, h.log10_lo, h.log10_hi, h.log_bins, npts, [x * mean_ens for x in xs])}
    Z = E96.scale_gap(own)["Z"]
    mix = E96.mix(0.023, Z, mode=0)
    pred = {"eps": mixed_tail_probs(mix["log_eps"].numpy(), h96.log10_lo, h96.log10_hi, h96.log_bins, xs),
            "enstrophy": mixed_tail_probs(mix["log_ens"].numpy(), h96.log10_lo, h96.log10_hi, h96.log_bins, xs)}
    pts = 1024 ** 3
    out = {"metric": "grid-pt RK steps/s (single 1024^3 FP32 member)", "value": round(pts * args.c5_steps / (t1 - t0), 1),
           "unit": "grid-pt RK steps/s", "n_gpus": 1, "steps": args.c5_steps, "warmup": args.c5_transient,
           "ms_per_step": round(1e3 * (t1 - t0) / args.c5_steps, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded random solenoidal field developed on "
           f"256^3 for {args.c5_coarse_steps} steps, refined to 512^3 for {args.c5_mid_steps} and to 1024^3 for "
           f"{args.c5_transient} steps before timing)",
           "config": {"workload": "single1024_fp32", "members": 1, "grid_points_per_step": pts, "stats_every": 10,
                      "nu": nu, "band": "|m| <= 2.5", "cfl": 0.5},
           "member": {"t_end": d["t"], "rlambda_snapshot_mean": own, "rlambda_last": d["rlambda"],
                      "kmax_eta_last": d["kmax_eta"], "snapshots": int(mom[28]), "samples": int(npts),
                      "mean_eps": mean_eps, "mean_enstrophy_nu": mean_ens, "tail_P(X>=x<X>)": member},
           "ens96_mixture": {"transient_steps": args.c5_ens_transient, "measured_steps": args.c5_ens_measure,
                             "rlambda_fit_A": A, "Z": Z, "c": 0.023, "weights": "Gaussian, open end bins",
                             "tail_P(X>=x)": pred, "mean_eps": mix["mean_eps"], "mean_enstrophy_nu": mix["mean_ens"]},
           "wall_s": round(time.perf_counter() - t_start, 1)}
    E.close()
    E96.close()
    return out


def member_moments(E, m):
    """A member's moment sums (FP64 tensor), without copying its histograms."""
    import ctypes
    import torch
    from paper_2506_23712_amd import _lib
    mom = torch.zeros(_lib.ENS_NMOM, dtype=torch.float64)
    _lib.check(_lib.lib().ens_get_stats(E.ctx, m.id, None, ctypes.cast(mom.data_ptr(), ctypes.POINTER(ctypes.c_double)),
                                        None))
    return mom.numpy()


def precision_report(ens, torch, args):
    """FP32 against FP64 on the 96-member benchmark set: both runs start from
    the same seeded fields, decorrelate by chaos after the transient, and are
    compared statistically over non-overlapping windows of `window` steps
    (statistics every 10 steps; about one to two integral times of most
    members): each member's mean dissipation over its injection, and the
    Gaussian mixture (c = 0.023, Z = ln 8) -- skewness, flatness and
    hyper-flatness of the gradient components, mean dissipation, and every
    QR-PDF bin holding at least 5e-4 of the mass -- with two-sample BCa
    bootstrap intervals of the FP32 - FP64 difference of the window means."""
    import numpy as np
    from scipy import stats as sps
    t_start = time.perf_counter()
    log = lambda msg: print(f"[precision {time.perf_counter() - t_start:7.1f}s] {msg}", file=sys.stderr, flush=True)
    nu = 0.03395
    h = hist_for(ens, nu)
    runs = {}
    for prec in ("fp32", "fp64"):
        specs = [dataclasses.replace(sp, precision=prec) for sp in ens96_specs(ens)]
        E = ens.Ensemble(hist=h, graphs=True)
        ms = [E.add_member(sp) for sp in specs]
        E.autotune()
        runs[prec] = (E, ms, specs)
    for k in range(args.pr_transient // 500):
        for prec, (E, ms, _) in runs.items():
            E.step(500)
        torch.cuda.synchronize()
        log(f"transient {500 * (k + 1)} steps")
    win = {p: {"eps": [], "mix": [], "qr": []} for p in runs}
    area = ((h.q_hi - h.q_lo) / h.qr_bins) * ((h.r_hi - h.r_lo) / h.qr_bins)
    for w in range(args.pr_windows):
        for prec, (E, ms, specs) in runs.items():
            for m in ms:
                m.reset_stats()
            for _ in range(args.pr_window // 10):
                E.step(10)
                E.accumulate_stats()
            eps = []
            for m, sp in zip(ms, specs):
                mom = member_moments(E, m)
                eps.append(mom[12] / (mom[28] * sp.n ** 3) / math.exp(sp.lam))   # <eps>/injection (eps_ref = 1)
            win[prec]["eps"].append(eps)
            mx = E.mix(0.023, math.log(8), mode=0)
            win[prec]["mix"].append([mx["S_long"], mx["F_long"], mx["H_long"], mx["F_trans"], mx["H_trans"],
                                     mx["mean_eps"]])
            win[prec]["qr"].append((mx["qr"].numpy() * area).ravel())
        log(f"window {w + 1}/{args.pr_windows}")
    diverged = {p: [m.id for m in ms if m.diag()["diverged"]] for p, (E, ms, _) in runs.items()}
    for E, _, _ in runs.values():
        E.close()
    rng = np.random.default_rng(0)
    boot = lambda a, b, cl: sps.bootstrap((a, b), lambda x, y: np.mean(x) - np.mean(y), method="BCa",
                                          confidence_level=cl, random_state=rng).confidence_interval
    e32, e64 = np.array(win["fp32"]["eps"]), np.array(win["fp64"]["eps"])     # [window][member]
    specs = runs["fp32"][2]
    members, inside = [], 0
    for i, sp in enumerate(specs):
        ci = boot(e32[:, i], e64[:, i], 0.95)
        ok = bool(ci.low <= 0.0 <= ci.high)
        inside += ok
        members.append({"lambda": round(sp.lam, 4), "n": sp.n, "eps_over_inj_fp32": float(e32[:, i].mean()),
                        "eps_over_inj_fp64": float(e64[:, i].mean()), "ci95_diff": [float(ci.low), float(ci.high)],
                        "zero_inside": ok})
    names = ("S_long", "F_long", "H_long", "F_trans", "H_trans", "mean_eps")
    m32, m64 = np.array(win["fp32"]["mix"]), np.array(win["fp64"]["mix"])
    mix = {}
    for j, nm in enumerate(names):
        ci = boot(m32[:, j], m64[:, j], 0.95)
        mix[nm] = {"fp32": float(m32[:, j].mean()), "fp64": float(m64[:, j].mean()),
                   "ci95_diff": [float(ci.low), float(ci.high)], "zero_inside": bool(ci.low <= 0.0 <= ci.high)}
    q32, q64 = np.array(win["fp32"]["qr"]), np.array(win["fp64"]["qr"])
    mean_q = 0.5 * (q32.mean(0) + q64.mean(0))
    bins = np.flatnonzero(mean_q >= 5e-4)
    qin = sum(bool(ci.low <= 0.0 <= ci.high) for ci in (boot(q32[:, b], q64[:, b], 0.99) for b in bins))
    return {"report": "fp32_vs_fp64_ens96", "windows": args.pr_windows, "window_steps": args.pr_window,
            "transient_steps": args.pr_transient, "stats_every": 10,
            "member_mean_dissipation": {"members": len(specs), "zero_inside_ci95": inside, "per_member": members},
            "mixture_Z_ln8_c0.023": mix,
            "mixed_qr_pdf": {"bins_tested": int(len(bins)), "zero_inside_ci99": int(qin)},
            "diverged": diverged, "wall_s": round(time.perf_counter() - t_start, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--stats-every", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--only", choices=["ens96_mixed_fp32", "single256_fp64", "ens48_128_fp64", "single1024_fp32",
                                       "ens96_fp32_vs_fp64"],
                    default=None,
                    help="one workload; ens48_128_fp64 (the 48-member 128^3 FP64 set of the ensemble driver) and "
                         "single1024_fp32 (one 1024^3 FP32 member at R_lambda ~ 280 with tail statistics, beside "
                         "the developed 96-member set's mixture) run only when named")
    ap.add_argument("--pr-transient", type=int, default=2000,
                    help="ens96_fp32_vs_fp64: steps of both runs before the windows")
    ap.add_argument("--pr-windows", type=int, default=16, help="ens96_fp32_vs_fp64: number of windows")
    ap.add_argument("--pr-window", type=int, default=150, help="ens96_fp32_vs_fp64: steps per window")
    ap.add_argument("--c5-coarse-steps", type=int, default=3000,
                    help="single1024_fp32: steps of the member on 256^3 before refinement")
    ap.add_argument("--c5-mid-steps", type=int, default=1000,
                    help="single1024_fp32: steps on 512^3 before the second refinement")
    ap.add_argument("--c5-transient", type=int, default=2500,
                    help="single1024_fp32: steps on 1024^3 before the timed steps")
    ap.add_argument("--c5-steps", type=int, default=500, help="single1024_fp32: timed steps (statistics every 10)")
    ap.add_argument("--c5-ens-transient", type=int, default=2500,
                    help="single1024_fp32: steps of the 96-member set before its statistics")
    ap.add_argument("--c5-ens-measure", type=int, default=2500,
                    help="single1024_fp32: steps of the 96-member set with statistics every 10")
    ap.add_argument("--develop", type=int, default=0, metavar="STEPS",
                    help="step the workload this many more steps before the timed statistics snapshot")
    ap.add_argument("--diagnostics", action="store_true",
                    help="only time the spectral diagnostics (spectrum, integral scales, refinement) and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (reference for HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (an ensemble would shard across GPUs by member, "
              "not implemented here); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": n * 4, "bytes_written": n * 4, "launches": 3}))
        return
    import paper_2506_23712_amd as ens
    if args.diagnostics:
        print(json.dumps({"diagnostics_256": diagnostics(ens, torch), "peak_GB/s": HBM_PEAK_GBS}))
        return

    if args.only == "single1024_fp32":
        print(json.dumps(config5(ens, torch, args)))
        return
    if args.only == "ens96_fp32_vs_fp64":
        print(json.dumps(precision_report(ens, torch, args)))
        return
    res = {}
    if args.only in (None, "ens96_mixed_fp32"):
        res["ens"] = run_workload(ens, torch, "ens96_mixed_fp32", ens96_specs(ens), args.steps, args.warmup,
                                  args.stats_every, 0.03395, not args.no_autotune, args.develop)
    if args.only in (None, "single256_fp64"):
        res["single"] = run_workload(ens, torch, "single256_fp64", single256_specs(ens), args.steps, args.warmup,
                                     args.stats_every, 4.594e-3, not args.no_autotune, args.develop)
    if args.only == "ens48_128_fp64":
        specs = ens48_128_specs(ens)
        res["ens48"] = run_workload(ens, torch, "ens48_128_fp64", specs, args.steps, args.warmup,
                                    args.stats_every, specs[0].nu, not args.no_autotune, args.develop)
    head = res.get("ens") or res.get("single") or res["ens48"]
    out = {
        "metric": "grid-pt RK steps/s (batched FP32 ensemble; FP64 single member beside it)",
        "value": round(head["rate"], 1),
        "unit": "grid-pt RK steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head["name"].endswith("fp32") else "f64",
        "data": "synthetic (seeded random solenoidal fields)",
        "config": {"workload": head["name"],
                   "members": {"ens96_mixed_fp32": 96, "single256_fp64": 1, "ens48_128_fp64": 48}[head["name"]],
                   "grid_points_per_step": head["points"], "stats_every": args.stats_every,
                   "mixture": "c=0.023, Z=ln 8, open end bins"},
        "roofline": roofline(head),
    }
    if "ens" in res and "single" in res:
        out["fp64_single_256"] = {"value": round(res["single"]["rate"], 1),
                                  "ms_per_step": round(res["single"]["ms_per_step"], 4),
                                  "roofline": roofline(res["single"]),
                                  "per_pass_ms": {k: round(v, 4) for k, v in res["single"]["prof"][(256, "fp64")][0].items()}}
        out["ratio_fp32_ensemble_vs_fp64_single"] = round(res["ens"]["rate"] / res["single"]["rate"], 3)
    out["per_pass_ms"] = {f"{n}_{p}": {k: round(v, 4) for k, v in ms.items()}
                          for (n, p), (ms, c) in head["prof"].items()}
    out["diverged_members"] = head["diverged"]
    out["stats_snapshot_ms"] = {r["name"]: round(r["stats_snapshot_ms"], 3) for r in res.values()}
    if args.develop:
        out["stats_snapshot_after_steps"] = args.develop
    out["rk_only"] = {r["name"]: {"median": round(r["rk_only"]["median"], 1),
                                  "iqr": [round(x, 1) for x in r["rk_only"]["iqr"]],
                                  "repeats": r["rk_only"]["repeats"], "steps_each": r["rk_only"]["steps_each"]}
                      for r in res.values()}
    out["kernel_variants"] = {k: v for r in res.values() for k, v in r["variants"].items()}
    if not args.no_cpu_baseline:
        specs = {"ens96_mixed_fp32": ens96_specs, "single256_fp64": single256_specs,
                 "ens48_128_fp64": ens48_128_specs}[head["name"]](ens)
        out["cpu_baseline"] = cpu_baseline(specs)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
