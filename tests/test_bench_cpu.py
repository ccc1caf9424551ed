"""Host logic of bench.py: the roofline entry, the traffic summary lookup and
the extrapolated optimum of the full-size time-to-tolerance leg."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_aitken_limit_of_a_geometric_sequence():
    import bench
    f = 3.0 + 2.0 * 0.93 ** np.arange(40)
    assert abs(bench.aitken_limit(f) - 3.0) < 1e-12
    assert bench.aitken_limit(np.array([1.0, 1.0, 1.0])) == 1.0


def test_roofline_picks_the_dominant_kernel_and_its_bound():
    import bench
    k = {"launches": 10, "tiles": 100, "ms": 0.0, "bytes": 0.0, "flops": 0.0}
    ks = {name: dict(k) for name in bench.STAGE_KERNELS["mixed"]}
    ks["lambda_update"].update(ms=10.0, bytes=4.0e10, flops=4.0e11)     # 4 TB/s, 10 flop/B
    ks["lambda_snapshot"].update(ms=5.0, bytes=1.0e10, flops=1.0e11)
    out, name = bench.roofline(ks, "mixed")
    assert name == "lambda_update" and out["kernel"] == "lambda_u_update32_kernel"
    assert out["bound"] == "hbm" and abs(out["achieved"] - 4000.0) < 1e-6
    assert abs(out["frac"] - 0.5) < 1e-9
    out64, _ = bench.roofline(ks, "fp64")        # 10 flop/B is right of the FP64 balance
    assert out64["bound"] == "mfma" and out64["kernel"] == "lambda_u_update_kernel<double>"


def test_traffic_summary_matches_the_current_source():
    import bench
    vals = {}
    for line in open(bench.TRAFFIC_FILE):
        if line.startswith("<!-- ") and "=" in line:
            key, v = line[5:].split("-->")[0].strip().split("=", 1)
            vals[key.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_1509_04681_amd", "csrc", "cd.hip")
    digest = bench.code_digest(src)
    got = bench.measured_traffic(vals["kernel"])
    if vals["cd_hip_code_sha256"] == digest:
        assert got == float(vals["bytes_per_launch"])
    else:
        assert got is None
    assert bench.measured_traffic("no_such_kernel") is None


def test_code_digest_ignores_comments_and_whitespace_only(tmp_path):
    import bench
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text('int f(int x) {  // one\n  return x + 1; /* two */ }\nconst char *s = "// kept";\n')
    b.write_text('// header\nint f(int x) {\n    return x + 1;\n}\nconst char *s = "// kept";\n')
    c.write_text('int f(int x) { return x + 2; }\nconst char *s = "// kept";\n')
    assert bench.code_digest(str(a)) == bench.code_digest(str(b))
    assert bench.code_digest(str(a)) != bench.code_digest(str(c))
