"""The byte model and kernel names the benchmark's roofline uses (CPU): the
per-pass algorithmic bytes add up to the per-step totals, scale with the
complex size, and the kernel named for each variant exists in the library's
sources."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pass_bytes_model():
    from paper_2506_23712_amd import profiling as p
    for n in (64, 128, 256, 512):
        K = n // 3
        S = (2 * K + 1) ** 2 * (K + 1)
        zl, yl = n * (2 * K + 1) * (K + 1), n * n * (K + 1)
        b64, b32 = p.pass_bytes(n, "fp64"), p.pass_bytes(n, "fp32")
        assert set(b64) == {"zinv", "yinv", "xpass", "yfwd", "zfwd_update"}
        for k in b64:
            assert abs(b64[k] - 2 * b32[k]) < 1e-6                  # 16 vs 8 bytes per complex value
        assert b64["xpass"] == 9 * yl * 16                             # 6 fields read, 3 written
        assert b64["zinv"] == (3 * S + 5 * zl) * 16
        # z forward + update: 3 z-line fields, u_hat read and written, q read in 2 and written in 2 of 3 stages
        assert abs(b64["zfwd_update"] - (3 * zl + 3 * S + 2 * S + 3 * S + 2 * S) * 16) < 1e-6
    per_pt = sum(p.pass_bytes(256, "fp64").values()) / 256 ** 3
    assert 180 < per_pt < 190                                          # about 185 B per point and stage


def test_kernel_names_exist_in_the_sources():
    from paper_2506_23712_amd import profiling as p
    src = open(os.path.join(ROOT, "paper_2506_23712_amd", "csrc", "kernels_step.hip")).read()
    for (pass_name, n, prec, v) in (("xpass", 256, "fp32", 3), ("xpass", 256, "fp32", 2), ("xpass", 512, "fp64", 3),
                                    ("xpass", 32, "fp32", 2), ("yinv", 256, "fp32", 1), ("zfwd_update", 128, "fp64", 0)):
        name = p.kernel_name(pass_name, n, prec, v)
        base = re.sub(r"<.*", "", name.replace("ens::", ""))
        assert re.search(r"\b" + base + r"\b", src), name
    assert p.kernel_name("xpass", 256, "fp32", 3).endswith(", 16>")
    assert p.kernel_name("xpass", 256, "fp64", 3).endswith(", 8>")   # FP64 falls back to 8 values per thread
    assert p.kernel_name("xpass", 32, "fp32", 2) == "ens::k_xpass<float, 32, 8>"
    assert p.kernel_name("yinv", 256, "fp32", 1) == "ens::k_yinv<float, 256, 16, 1>"
    assert p.kernel_name("zinv", 256, "fp32", 2) == "ens::k_zinv<float, 256, 8, 2>"
    assert p.kernel_name("zfwd_update", 256, "fp32", 1) == "ens::k_zfwd_update<float, 256, 1, true>"
    assert p.kernel_name("zfwd_update", 256, "fp64", 0) == "ens::k_zfwd_update<double, 256, 1, false>"
    # every y/z name appears in the committed trace of the same sources
    table = open(os.path.join(ROOT, "profiles", "ens96_mixed_fp32_and_single256_fp64_kernel_stats.md")).read()
    assert "`" + p.kernel_name("yfwd", 256, "fp32", 3) + "`" in table



def test_trace_averages_read_the_committed_kernel_table():
    """The rate columns of the traffic summary take each kernel's average
    duration from the committed kernel-statistics table."""
    from paper_2506_23712_amd import profiling as p
    path = os.path.join(ROOT, "profiles", "ens96_mixed_fp32_and_single256_fp64_kernel_stats.md")
    avg = p.trace_averages(path)
    assert "ens::k_xpass_dma<float, 256, 16>" in avg
    rows = [l for l in open(path) if l.startswith("| `")]
    assert len(avg) == len(rows)
    for l in rows:
        cells = [c.strip() for c in l.strip().strip("|").split("|")]
        name = cells[0].strip("`")
        assert avg[name] == float(cells[3])
        assert abs(float(cells[2]) - int(cells[1]) * float(cells[3])) <= 0.01 * float(cells[2]) + 1


def test_summary_uses_each_rk_stage_own_bytes_for_the_z_forward():
    """The z forward + update of RK stage 0 reads no RK register, that of
    stage 2 writes none, and a fused kernel (stages 0 and 1, `true` in its
    name) also writes the next stage's 5 z-inverse fields: the committed
    summary's algorithmic bytes of each stage's kernel follow that, and the
    unfused stages average to the pass model's figure."""
    from paper_2506_23712_amd import profiling as p
    path = os.path.join(ROOT, "profiles", "traffic_summary_256.md")
    n, K, cs, cnt = 256, 256 // 3, 8, 25
    S, zl = (2 * K + 1) ** 2 * (K + 1), n * (2 * K + 1) * (K + 1)
    got = {}
    for l in open(path):
        cells = [c.strip() for c in l.strip().strip("|").split("|")]
        if len(cells) > 2 and cells[0] == "ens96_mixed_fp32":
            m = re.fullmatch(r"`k_zfwd_update<float, 256, (\d), (true|false)>`", cells[1])
            if m:
                r, w = (float(x) for x in cells[2].split("/"))
                got[(int(m.group(1)), m.group(2) == "true")] = (r, w)
    assert {st for st, _ in got} == {0, 1, 2}
    for (st, fused), (r, w) in got.items():
        want_r = (3 * zl + 3 * S + (3 * S if st > 0 else 0)) * cs * cnt
        want_w = (3 * S + (3 * S if st < 2 else 0) + (5 * zl if fused else 0)) * cs * cnt
        assert abs(r - want_r / 1e9) < 1e-3 and abs(w - want_w / 1e9) < 1e-3, (st, fused, r, w)
        assert tuple(x * cnt for x in p.zfwd_stage_bytes(n, "fp32", st, fused)) == (want_r, want_w)
    avg = sum(sum(p.zfwd_stage_bytes(n, "fp32", st)) for st in range(3)) / 3
    assert abs(avg - p.pass_bytes(n, "fp32")["zfwd_update"]) < 1e-6 * avg


def test_dominant_kernel_counts_launches_per_kernel():
    """The benchmark's roofline kernel: the largest summed time of one kernel
    per step.  The z forward's time is spread over three stage kernels, and
    with the fused z forward the z inverse launches once per step."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    ms = {"band": 0.03, "zinv": 0.91, "yinv": 5.8, "xpass": 5.9, "yfwd": 2.9, "zfwd_update": 6.3, "end_step": 0.01}
    res = {"prof": {(256, "fp32"): (ms, 25)}, "variants": {"zfwd_update:256:fp32": 1, "xpass:256:fp32": 6}}
    (n, prec), k, count, avg, launches, fused = bench.dominant_kernel(res)
    assert (n, prec, k, count, launches, fused) == (256, "fp32", "xpass", 25, 3, True)
    assert abs(avg - 5.9 / 3) < 1e-12
    ms2 = {"zinv": 3.0, "yinv": 2.5, "xpass": 2.9, "yfwd": 1.0, "zfwd_update": 4.0}
    r = bench.dominant_kernel({"prof": {(128, "fp64"): (ms2, 2)}, "variants": {"zfwd_update:128:fp64": 1}})
    assert r[1] == "zinv" and r[4] == 1 and r[3] == 3.0
    r = bench.dominant_kernel({"prof": {(128, "fp64"): (ms2, 2)}, "variants": {"zfwd_update:128:fp64": 0}})
    assert r[1] == "zinv" and r[4] == 3 and abs(r[3] - 1.0) < 1e-12
