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

Options: the ens256 set (n = 256 in a box of 4 pi: --box-scale 2), moving the
largest-lambda members onto twice their grid after the transient
(--refine-lambda), a JSON-lines record of every member's diagnostics
(--record), and stopping at a wall-time limit with a checkpoint that a later
process resumes exactly (--wall-limit, --checkpoint, --resume).

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


def max_resolved_wavenumber(n: int, box: float = 2 * math.pi, convention: str = "cubic") -> float:
    """k_M of an n^3 grid.  The paper calls it the maximum resolved wavenumber
    without a formula.  "cubic": the largest retained |m_i| of the cubic 2/3
    truncation, K dk with K = floor(n/3); "sqrt2": sqrt(2) n/3 dk, the radius of
    the spherical truncation that phase-shift dealiased codes keep (a reading
    that reproduces Table I's R_lambda, see the design notes)."""
    dk = 2 * math.pi / box
    if convention == "cubic":
        return (n // 3) * dk
    if convention == "sqrt2":
        return math.sqrt(2.0) * n / 3.0 * dk
    raise ValueError(f"unknown k_M convention {convention!r}")


def ens128_specs(ens, n: int = 128, precision: str = "fp64", i_lo: int = -22, i_hi: int = 25,
                 kmeta: float = 3.0, cfl: float = 0.2, seed0: int = 23712, box: float = 2 * math.pi,
                 km: str = "cubic"):
    """Member specs: lambda_i = i ln2/3, eps = e^lambda, nu from k_M eta of the
    central member (eps = 1: nu = (kmeta / k_M)^(4/3), k_M from
    max_resolved_wavenumber).  The ens256 set of Table I is n = 256 in a box
    of 4 pi (dk = 1/2), the band still [1.4, 2.3] dk."""
    nu = (kmeta / max_resolved_wavenumber(n, box, km)) ** (4.0 / 3.0)
    return [ens.MemberSpec(n=n, nu=nu, eps_ref=1.0, lam=i * LAMBDA_STEP, kf_lo=1.4, kf_hi=2.3, dt=0.0, cfl=cfl,
                           precision=precision, seed=seed0 + (i - i_lo), box=box) for i in range(i_lo, i_hi + 1)]


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
        refine_transient: float = 1.0, record=None, state: dict | None = None, stop=None):
    """Run transient and measurement; returns the result dictionary.  With
    `refine_lambda`, the members with lambda >= refine_lambda move to twice
    their grid after the transient and run `refine_transient` more of their
    integral times before the measurement.  `record` (a text file) receives one
    JSON line of all members' diagnostics per check.

    The run can be split over processes: `stop()` is asked after every check
    that does not end a phase; when it returns True the run returns
    {"stopped": True, "state": ..., "members": ...} at that step boundary, and
    a later call with the members restored from their checkpoint and
    `state=` that state continues it exactly as if uninterrupted."""
    t_start = time.perf_counter()
    members = list(members)
    central = min(members, key=lambda m: abs(m.spec.lam))
    st = dict(state) if state else {"phase": "transient", "steps": 0, "wall": 0.0}

    def elapsed():
        return st["wall"] + time.perf_counter() - t_start

    def stopped():
        out = dict(st)
        out["wall"] = elapsed()
        return {"stopped": True, "state": out, "members": members}

    # transient: every member runs `transient` of its own integral times
    if st["phase"] == "transient":
        while True:
            E.step(chunk, members=members)
            st["steps"] += chunk
            sc = _scales(members, record, "transient", st["steps"])
            prog = min((t / T if T > 0 else 0.0) for t, T in sc)
            log(f"transient: step {st['steps']}, slowest member at {prog:.2f} T, {elapsed():.0f} s")
            if prog >= transient or st["steps"] >= max_steps:
                st["phase"] = "refine" if refine_lambda is not None else "measure setup"
                break
            if stop is not None and stop():
                return stopped()
    if st["phase"] == "refine":
        st["refined_at"] = st["steps"]
        members = refine_members(E, members, refine_lambda)
        st["refined"] = [k for k, m in enumerate(members) if m.spec.lam >= refine_lambda]
        sc = _scales(members)
        st["t_ref"] = [sc[k][0] for k in st["refined"]]
        log(f"refined {len(st['refined'])} members with lambda >= {refine_lambda} onto twice their grid")
        st["phase"] = "refined transient"
    if st["phase"] == "refined transient":
        refined, t_ref = st["refined"], st["t_ref"]
        while refined:
            E.step(chunk, members=members)
            st["steps"] += chunk
            sc = _scales(members, record, "refined transient", st["steps"])
            prog = min(((sc[k][0] - t0) / sc[k][1] if sc[k][1] > 0 else 0.0) for k, t0 in zip(refined, t_ref))
            log(f"refined transient: step {st['steps']}, slowest refined member at {prog:.2f} T, {elapsed():.0f} s")
            if prog >= refine_transient or st["steps"] >= max_steps:
                break
            if stop is not None and stop():
                return stopped()
        st["phase"] = "measure setup"
    if st["phase"] == "measure setup":
        # steps per integral time (median over members) sets the snapshot interval
        sc = _scales(members)
        rates = sorted(T / d for d, (t, T) in ((m.diag()["dt"], s) for m, s in zip(members, sc)) if d > 0 and T > 0)
        if not rates:
            raise RuntimeError("no member has a positive time step and integral time after the transient")
        per_T = rates[len(rates) // 2]
        st["every"] = max(1, int(round(per_T / snaps_per_T)))
        for m in members:
            m.reset_stats()
        st.update(t0=[t for t, _ in sc], Tsum=[0.0] * len(members), nsnap=0, e_central=[], m_steps=0,
                  phase="measure")
    every, t0, Tsum, e_central = st["every"], st["t0"], st["Tsum"], st["e_central"]
    steps = st["steps"]
    while st["phase"] == "measure":
        E.step(every, members=members)
        st["m_steps"] += every
        E.accumulate_stats(members=members)
        sc = _scales(members, record, "measure", steps + st["m_steps"])
        st["nsnap"] += 1
        nsnap = st["nsnap"]
        for k, (_, T) in enumerate(sc):
            Tsum[k] += T
        e_central.append(central.diag()["E"])
        prog = min(((t - t0[k]) / (Tsum[k] / nsnap) if Tsum[k] > 0 else 0.0) for k, (t, _) in enumerate(sc))
        if nsnap % 10 == 0:
            log(f"measure: step {steps + st['m_steps']}, {nsnap} snapshots, slowest member at {prog:.2f} T, "
                f"{elapsed():.0f} s")
        if prog >= measure or steps + st["m_steps"] >= max_steps:
            st["phase"] = "done"
        elif stop is not None and stop():
            return stopped()
    m_steps, nsnap = st["m_steps"], st["nsnap"]
    refined, refined_at = st.get("refined", []), st.get("refined_at")
    wall = elapsed()
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


RUN_KEYS = ("n", "precision", "i_lo", "i_hi", "box_scale", "transient", "measure", "snaps_per_T", "chunk",
            "refine_lambda", "refine_transient", "km_convention")


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2506_23712_amd.run_ensemble")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--i-lo", type=int, default=-22)
    ap.add_argument("--i-hi", type=int, default=25)
    ap.add_argument("--box-scale", type=float, default=1.0, help="box = box_scale * 2 pi (2 for the ens256 set)")
    ap.add_argument("--km-convention", choices=["cubic", "sqrt2"], default="cubic",
                    help="k_M in k_M eta = 3 (sets nu): K dk of the cubic truncation, or sqrt(2) n/3 dk")
    ap.add_argument("--transient", type=float, default=5.0, help="integral times before measuring")
    ap.add_argument("--measure", type=float, default=18.0, help="integral times measured")
    ap.add_argument("--snaps-per-T", type=float, default=10.0)
    ap.add_argument("--chunk", type=int, default=100)
    ap.add_argument("--refine-lambda", type=float, default=None,
                    help="after the transient, move the members with lambda >= this onto twice their grid")
    ap.add_argument("--refine-transient", type=float, default=1.0,
                    help="integral times the refined members run before the measurement")
    ap.add_argument("--record", default=None, help="JSON-lines file of every member's diagnostics per check")
    ap.add_argument("--wall-limit", type=float, default=None,
                    help="stop at the first check after this many seconds and write --checkpoint")
    ap.add_argument("--checkpoint", default=None, help=".npz file written when the run stops early")
    ap.add_argument("--resume", default=None, help="continue a stopped run from its checkpoint (its settings apply)")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.wall_limit is not None and not a.checkpoint:
        ap.error("--wall-limit needs --checkpoint")
    import torch
    import paper_2506_23712_amd as ens
    state = None
    if a.resume:
        extra = ens.Ensemble.read_checkpoint_extra(a.resume)
        state, cfg = extra["driver"], extra["run"]
        for k in RUN_KEYS:
            setattr(a, k, cfg.get(k, getattr(a, k)))
        E, members = ens.Ensemble.load_checkpoint(a.resume)
    else:
        specs = ens128_specs(ens, a.n, a.precision, a.i_lo, a.i_hi, box=a.box_scale * 2 * math.pi,
                             km=a.km_convention)
        E = ens.Ensemble(hist=hist_spec(ens, specs[0].nu), graphs=True)
        members = [E.add_member(s) for s in specs]
        E.autotune()
    torch.cuda.synchronize()
    t_proc = time.perf_counter()
    stop = (lambda: time.perf_counter() - t_proc > a.wall_limit) if a.wall_limit is not None else None
    rec = open(a.record, "a" if a.resume else "w") if a.record else None
    try:
        res = run(E, members, a.transient, a.measure, a.snaps_per_T, a.chunk,
                  log=lambda s: print(s, flush=True), refine_lambda=a.refine_lambda,
                  refine_transient=a.refine_transient, record=rec, state=state, stop=stop)
    finally:
        if rec is not None:
            rec.close()
    if res.get("stopped"):
        E.save_checkpoint(a.checkpoint, members=res["members"],
                          extra={"driver": res["state"], "run": {k: getattr(a, k) for k in RUN_KEYS}})
        E.close()
        print(json.dumps({"stopped": True, "phase": res["state"]["phase"], "steps": res["state"]["steps"]
                          + res["state"].get("m_steps", 0), "checkpoint": a.checkpoint}), flush=True)
        return 0
    specs = [m.spec for m in members]
    res["config"] = {"n": a.n, "precision": a.precision, "km_convention": a.km_convention, "members": len(specs),
                     "nu": specs[0].nu,
                     "box": specs[0].box, "lambda": [s.lam for s in specs], "band": [1.4, 2.3], "cfl": 0.2}
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
