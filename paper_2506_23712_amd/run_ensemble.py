"""Driver for a paper-faithful ensemble at one GPU's scale (the ens128 set of
Table I: 48 members on 128^3 in a (2 pi)^3 box, lambda = i ln2/3 for
i = -22 .. 25 (the spacing 0.23 and range of the paragraph after Table II),
forcing band [1.4, 2.3] dk, CFL 0.2, viscosity set by k_M eta = 3 for the
central member, section "Description of the ensemble simulations").

Every member is stepped by the library in one batched, graph-captured step per
call.  Time is counted per member in its own integral times T = L / u' (from
``Member.integral_scales``): the transient ends when every member has run
``transient`` integral times, the measurement when every member has run
``measure`` more, with statistics snapshots about ``snaps_per_T`` times per
integral time.  The result collects, per member, the snapshot-averaged energy,
dissipation, R_lambda and k_M eta, and the mixture predictions (Gaussian and
truncated-Gaussian weights) of skewness, flatness and hyper-flatness of the
gradient components against the scale gap Z, the mixed gradient PDFs, and Z for
the reference Reynolds numbers of Table II.  All arithmetic on fields and
statistics runs in the library; this module only schedules calls.

    python -m paper_2506_23712_amd.run_ensemble --n 128 --precision fp64 --out run.json
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import sys
import time

LAMBDA_STEP = math.log(2) / 3


def ens128_specs(ens, n: int = 128, precision: str = "fp64", i_lo: int = -22, i_hi: int = 25,
                 kmeta: float = 3.0, cfl: float = 0.2, seed0: int = 23712):
    """Member specs: lambda_i = i ln2/3, eps = e^lambda, nu from k_M eta of the
    central member (k_M = K dk, dk = 1, eps = 1: nu = (kmeta / K)^(4/3))."""
    K = n // 3
    nu = (kmeta / K) ** (4.0 / 3.0)
    return [ens.MemberSpec(n=n, nu=nu, eps_ref=1.0, lam=i * LAMBDA_STEP, kf_lo=1.4, kf_hi=2.3, dt=0.0, cfl=cfl,
                           precision=precision, seed=seed0 + (i - i_lo)) for i in range(i_lo, i_hi + 1)]


def hist_spec(ens, nu: float):
    """Axes in Kolmogorov units of the central member (eps = 1, nu)."""
    return ens.HistSpec(qr_bins=256, q_lo=-25.0, q_hi=25.0, r_lo=-50.0, r_hi=50.0, log_bins=256, log10_lo=-8.0,
                        log10_hi=5.0, a_bins=2048, a_lo=-120.0, a_hi=120.0, eps_ref=1.0, nu_ref=nu)


def _scales(members, record=None, phase="", steps=0):
    """(t, T) of every member: its time and current integral time.  With
    `record` (a text file), one JSON line of every member's diagnostics."""
    out, rows = [], []
    for m in members:
        T = float(m.integral_scales()[3].item())
        d = m.diag()
        out.append((d["t"], T))
        if record is not None:
            rows.append({"lambda": m.spec.lam, "n": m.spec.n, "t": d["t"], "dt": d["dt"], "E": d["E"], "D": d["D"],
                         "E_f": d["E_f"], "cfl": d["cfl"], "rlambda": d["rlambda"], "kmax_eta": d["kmax_eta"], "T": T,
                         "diverged": d["diverged"]})
    if record is not None:
        record.write(json.dumps({"phase": phase, "steps": steps, "members": rows}) + "\n")
        record.flush()
    return out


def refine_members(E, members, lam_min: float):
    """Replace every member with lambda >= lam_min by a member on twice its grid
    that takes over its field (the paper reruns its lambda >= 3.2 members at
    twice the resolution, section "Extrapolating to the frontier of current
    turbulence simulations").  Returns the new member list (same order); the
    replaced members stay in the context, unused."""
    out = []
    for m in members:
        if m.spec.lam >= lam_min:
            m2 = E.add_member(dataclasses.replace(m.spec, n=2 * m.spec.n))
            m2.refine_from(m)
            out.append(m2)
        else:
            out.append(m)
    return out


def run(E, members, transient: float, measure: float, snaps_per_T: float, chunk: int = 50, log=print,
        c: float = 0.023, zs=(0.0, 0.25, math.log(2), 1.0, math.log(4), 1.75, math.log(8)),
        rlambda_refs=(103.0, 173.0, 261.0), max_steps: int = 10 ** 7, refine_lambda: float | None = None,
        refine_transient: float = 1.0, record=None):
    """Run transient and measurement; returns the result dictionary.  With
    `refine_lambda`, the members with lambda >= refine_lambda move to twice
    their grid after the transient and run `refine_transient` more of their
    integral times before the measurement.  `record` (a text file) receives one
    JSON line of all members' diagnostics per check."""
    t_start = time.perf_counter()
    steps = 0
    members = list(members)
    central = min(members, key=lambda m: abs(m.spec.lam))
    # transient: every member runs `transient` of its own integral times
    while True:
        E.step(chunk, members=members)
        steps += chunk
        sc = _scales(members, record, "transient", steps)
        prog = min((t / T if T > 0 else 0.0) for t, T in sc)
        log(f"transient: step {steps}, slowest member at {prog:.2f} T, {time.perf_counter() - t_start:.0f} s")
        if prog >= transient or steps >= max_steps:
            break
    refined, refined_at = [], None
    if refine_lambda is not None:
        refined_at = steps
        members = refine_members(E, members, refine_lambda)
        refined = [k for k, m in enumerate(members) if m.spec.lam >= refine_lambda]
        t_ref = {k: t for k, (t, _) in zip(range(len(members)), _scales(members)) if k in refined}
        log(f"refined {len(refined)} members with lambda >= {refine_lambda} onto twice their grid")
        while refined:
            E.step(chunk, members=members)
            steps += chunk
            sc = _scales(members, record, "refined transient", steps)
            prog = min(((sc[k][0] - t_ref[k]) / sc[k][1] if sc[k][1] > 0 else 0.0) for k in refined)
            log(f"refined transient: step {steps}, slowest refined member at {prog:.2f} T, "
                f"{time.perf_counter() - t_start:.0f} s")
            if prog >= refine_transient or steps >= max_steps:
                break
    # steps per integral time (median over members) sets the snapshot interval
    rates = sorted(T / d for d, (t, T) in ((m.diag()["dt"], s) for m, s in zip(members, sc)) if d > 0 and T > 0)
    if not rates:
        raise RuntimeError("no member has a positive time step and integral time after the transient")
    per_T = rates[len(rates) // 2]
    every = max(1, int(round(per_T / snaps_per_T)))
    for m in members:
        m.reset_stats()
    t0 = [t for t, _ in sc]
    Tsum = [0.0] * len(members)
    nsnap = 0
    e_central = []
    m_steps = 0
    while True:
        E.step(every, members=members)
        m_steps += every
        E.accumulate_stats(members=members)
        sc = _scales(members, record, "measure", steps + m_steps)
        nsnap += 1
        for k, (_, T) in enumerate(sc):
            Tsum[k] += T
        e_central.append(central.diag()["E"])
        prog = min(((t - t0[k]) / (Tsum[k] / nsnap) if Tsum[k] > 0 else 0.0) for k, (t, _) in enumerate(sc))
        if nsnap % 10 == 0:
            log(f"measure: step {steps + m_steps}, {nsnap} snapshots, slowest member at {prog:.2f} T, "
                f"{time.perf_counter() - t_start:.0f} s")
        if prog >= measure or steps + m_steps >= max_steps:
            break
    wall = time.perf_counter() - t_start
    res = {"steps": steps + m_steps, "transient_steps": steps, "snapshot_every": every, "snapshots": nsnap,
           "wall_s": wall, "refined_members": refined,
           "refined_at_step": refined_at}
    gap = E.scale_gap(rlambda_refs[0], members=members)
    res["rlambda_prefactor"] = gap["prefactor"]
    res["scale_gap"] = {str(r): E.scale_gap(r, members=members)["Z"] for r in rlambda_refs}
    per = []
    for k, m in enumerate(members):
        _, mom, npts = m.stats()
        mom = mom.numpy()
        Em, Dm = mom[26] / mom[28], mom[27] / mom[28]
        K = m.spec.n // 3
        per.append({"lambda": m.spec.lam, "n": m.spec.n, "E": Em, "D": Dm, "rlambda": gap["rlambda"][k],
                    "kmeta": K * (2 * math.pi / m.spec.box) * (m.spec.nu ** 3 / Dm) ** 0.25,
                    "T": Tsum[k] / nsnap,
                    "measured_T": (m.diag()["t"] - t0[k]) / (Tsum[k] / nsnap) if Tsum[k] > 0 else 0.0})
    res["members"] = per
    # stationarity of the central member: mean energy of the two halves of the record
    h = len(e_central) // 2
    res["central_energy_halves"] = [sum(e_central[:h]) / max(h, 1), sum(e_central[h:]) / max(len(e_central) - h, 1)]
    preds = []
    for Z in zs:
        for mode, name in ((0, "gaussian"), (3, "truncated")):
            mx = E.mix(c, Z, mode=mode, members=members)
            preds.append({"Z": Z, "weights": name, "S_long": mx["S_long"], "F_long": mx["F_long"],
                          "H_long": mx["H_long"], "F_trans": mx["F_trans"], "H_trans": mx["H_trans"],
                          "mean_eps": mx["mean_eps"], "weight_sum": float(mx["weights"].sum())})
    res["predictions"] = preds
    mx = E.mix(c, math.log(4), mode=0, members=members)
    res["pdf_Z_ln4"] = {"a_long": mx["a_long"].tolist(), "a_trans": mx["a_trans"].tolist()}
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2506_23712_amd.run_ensemble")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--i-lo", type=int, default=-22)
    ap.add_argument("--i-hi", type=int, default=25)
    ap.add_argument("--transient", type=float, default=5.0, help="integral times before measuring")
    ap.add_argument("--measure", type=float, default=18.0, help="integral times measured")
    ap.add_argument("--snaps-per-T", type=float, default=10.0)
    ap.add_argument("--chunk", type=int, default=100)
    ap.add_argument("--refine-lambda", type=float, default=None,
                    help="after the transient, move the members with lambda >= this onto twice their grid")
    ap.add_argument("--refine-transient", type=float, default=1.0,
                    help="integral times the refined members run before the measurement")
    ap.add_argument("--record", default=None, help="JSON-lines file of every member's diagnostics per check")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    import torch
    import paper_2506_23712_amd as ens
    specs = ens128_specs(ens, a.n, a.precision, a.i_lo, a.i_hi)
    E = ens.Ensemble(hist=hist_spec(ens, specs[0].nu), graphs=True)
    members = [E.add_member(s) for s in specs]
    E.autotune()
    torch.cuda.synchronize()
    rec = open(a.record, "w") if a.record else None
    try:
        res = run(E, members, a.transient, a.measure, a.snaps_per_T, a.chunk,
                  log=lambda s: print(s, flush=True), refine_lambda=a.refine_lambda,
                  refine_transient=a.refine_transient, record=rec)
    finally:
        if rec is not None:
            rec.close()
    res["config"] = {"n": a.n, "precision": a.precision, "members": len(specs), "nu": specs[0].nu,
                     "lambda": [s.lam for s in specs], "band": [1.4, 2.3], "cfl": 0.2}
    diverged = [m.id for m in E.members if m.diag()["diverged"]]
    res["diverged"] = diverged
    E.close()
    with open(a.out, "w") as f:
        json.dump(res, f)
    cen = min(res["members"], key=lambda r: abs(r["lambda"]))
    print(json.dumps({"steps": res["steps"], "wall_s": round(res["wall_s"], 1), "central_rlambda": cen["rlambda"],
                      "central_kmeta": cen["kmeta"], "scale_gap": res["scale_gap"], "diverged": diverged}), flush=True)
    return 1 if diverged else 0


if __name__ == "__main__":
    sys.exit(main())
