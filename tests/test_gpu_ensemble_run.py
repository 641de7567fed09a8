"""The ensemble driver on a small ensemble (8 members at 32^3, a short run):
its schedule and its self-consistency.  The same driver runs the 48-member
128^3 set; this test keeps to seconds."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_small_ensemble_run_is_self_consistent(orc):
    import paper_2506_23712_amd as ens
    from paper_2506_23712_amd import run_ensemble as rd
    from oracle import mixture as mx
    specs = rd.ens128_specs(ens, n=32, precision="fp64", i_lo=-4, i_hi=3)
    assert [round(s.lam / rd.LAMBDA_STEP) for s in specs] == list(range(-4, 4))
    assert abs((32 // 3) * (specs[0].nu ** 3) ** 0.25 - 3.0) < 1e-12          # k_M eta = 3 at eps = 1
    E = ens.Ensemble(hist=rd.hist_spec(ens, specs[0].nu))
    members = [E.add_member(s) for s in specs]
    import io
    import json
    rec = io.StringIO()
    res = rd.run(E, members, transient=0.5, measure=1.0, snaps_per_T=5, chunk=20, log=print, record=rec)
    lines = [json.loads(x) for x in rec.getvalue().splitlines()]
    assert [x["phase"] for x in lines].count("measure") == res["snapshots"]
    assert lines[0]["phase"] == "transient" and lines[-1]["steps"] == res["steps"]
    assert all(len(x["members"]) == len(members) for x in lines)
    assert all(a["steps"] < b["steps"] for a, b in zip(lines, lines[1:]))
    assert lines[-1]["members"][4]["t"] == members[4].diag()["t"]
    central = members[4]
    assert central.spec.lam == 0.0
    # every member measured at least one of its integral times, nothing diverged
    assert all(r["measured_T"] >= 1.0 for r in res["members"])
    assert not any(m.diag()["diverged"] for m in members)
    assert res["snapshots"] >= 5
    # R_lambda from the snapshot sums, as the oracle forms it; the scale gaps from the fit
    rls = []
    for m, r in zip(members, res["members"]):
        _, mom, _ = m.stats()
        mom = mom.numpy()
        assert mom[28] == res["snapshots"]
        rl = mx.rlambda_from_means(mom[26] / mom[28], mom[27] / mom[28], m.spec.nu)
        assert math.isclose(r["rlambda"], rl, rel_tol=1e-13)
        rls.append(rl)
    A = mx.rlambda_prefactor([s.lam for s in specs], rls)
    assert math.isclose(res["rlambda_prefactor"], A, rel_tol=1e-13)
    for r, Z in res["scale_gap"].items():
        assert math.isclose(Z, mx.scale_gap(float(r), A), rel_tol=1e-12, abs_tol=1e-13)
    # Z = 0: the prediction is the central member's own statistics
    _, mom, npts = central.stats()
    mom = mom.numpy()
    z0 = [p for p in res["predictions"] if p["Z"] == 0.0]
    assert len(z0) == 2
    for p in z0:
        assert p["weight_sum"] == 1.0
        m1, m2 = mom[1] / (3 * npts), mom[2] / (3 * npts)
        assert math.isclose(p["S_long"], mx.skewness(m1, m2), rel_tol=1e-12)
        assert math.isclose(p["mean_eps"], mom[12] / npts, rel_tol=1e-12)
    for p in res["predictions"]:
        assert abs(p["weight_sum"] - 1.0) < 1e-13
        assert p["F_long"] > 1.0 and p["F_trans"] > 1.0
    # the gradient PDFs of the mixture are normalised over the table
    h = rd.hist_spec(ens, specs[0].nu)
    width = (h.a_hi - h.a_lo) / h.a_bins
    for name in ("a_long", "a_trans"):
        s = float(np.sum(res["pdf_Z_ln4"][name]) * width)
        assert 0.99 < s <= 1.0 + 1e-12
    E.close()


def test_small_ensemble_run_with_refined_members():
    """The largest-lambda members move onto twice their grid after the
    transient, run on there, and are measured and mixed on the finer grid."""
    import paper_2506_23712_amd as ens
    from paper_2506_23712_amd import run_ensemble as rd
    specs = rd.ens128_specs(ens, n=32, precision="fp64", i_lo=-2, i_hi=3)
    E = ens.Ensemble(hist=rd.hist_spec(ens, specs[0].nu))
    members = [E.add_member(s) for s in specs]
    res = rd.run(E, members, transient=0.5, measure=1.0, snaps_per_T=5, chunk=20, log=print,
                 refine_lambda=0.4, refine_transient=0.25)
    assert res["refined_members"] == [4, 5]
    assert [r["n"] for r in res["members"]] == [32, 32, 32, 32, 64, 64]
    assert [r["lambda"] for r in res["members"]] == [s.lam for s in specs]
    assert len(E.members) == 8                                     # the two replaced members stay, unused
    assert not any(m.diag()["diverged"] for m in E.members)
    assert all(r["measured_T"] >= 1.0 for r in res["members"])
    fine = E.members[6:]
    for m in fine:
        _, mom, npts = m.stats()
        assert m.spec.n == 64 and npts == 64 ** 3 * res["snapshots"]
        assert mom.numpy()[28] == res["snapshots"]
    # the coarse originals stopped at the end of the transient
    assert 0 < res["refined_at_step"] < res["transient_steps"]
    assert all(E.members[k].diag()["step"] == res["refined_at_step"] for k in (4, 5))
    assert all(E.members[k].diag()["step"] == res["steps"] for k in (0, 1, 2, 3))
    for p in res["predictions"]:
        assert abs(p["weight_sum"] - 1.0) < 1e-13
    E.close()


def test_run_split_over_three_contexts_equals_the_uninterrupted_run(tmp_path):
    """The driver stopped twice (once in the transient, once later) and
    resumed each time in a fresh context from the .npz checkpoint with its
    state gives the uninterrupted run's results exactly (all but wall time)."""
    import paper_2506_23712_amd as ens
    from paper_2506_23712_amd import run_ensemble as rd
    specs = rd.ens128_specs(ens, n=32, precision="fp64", i_lo=-2, i_hi=3)
    kw = dict(transient=0.5, measure=1.0, snaps_per_T=5, chunk=20, log=print, refine_lambda=0.4,
              refine_transient=0.25)

    def fresh():
        E = ens.Ensemble(hist=rd.hist_spec(ens, specs[0].nu))
        return E, [E.add_member(s) for s in specs]

    def stop_after(k):
        n = [0]

        def stop():
            n[0] += 1
            return n[0] >= k
        return stop

    E, ms = fresh()
    ref = rd.run(E, ms, **kw)
    E.close()
    E, ms = fresh()
    state, phases = None, []
    for k in (2, 6, None):
        res = rd.run(E, ms, state=state, stop=stop_after(k) if k else None, **kw)
        if not res.get("stopped"):
            break
        phases.append(res["state"]["phase"])
        path = str(tmp_path / f"ck{len(phases)}.npz")
        E.save_checkpoint(path, members=res["members"], extra=res["state"])
        E.close()
        E, ms = ens.Ensemble.load_checkpoint(path)
        state = ens.Ensemble.read_checkpoint_extra(path)
    E.close()
    assert phases[0] == "transient" and len(phases) == 2
    for key in ref:
        if key != "wall_s":
            assert res[key] == ref[key], key
