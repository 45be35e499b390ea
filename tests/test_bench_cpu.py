"""bench.py contract pieces that need no GPU: more than one GPU is refused
with a message before anything touches a device, and the CPU-baseline leg
(the oracle timed on the host) returns the fields the JSON line carries."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_cpu_baseline_leg_reports_the_oracle_rate():
    sys.path.insert(0, ROOT)
    import bench
    import oracle as O
    from paper_2504_00998_amd import workloads as W

    wl = W.CFG1
    om = O.Mesh.from_workload(wl)
    op = O.Operator(om, W.workload_potential(wl, om.quad_points()), wl.E, wl.z0)
    a0, b, _ = O.lanczos_bounds(op.apply, wl.lanczos_start(op.n), 10)
    a = O.weyl_cut(a0, b, wl.N, op.n)
    rec = bench.cpu_baseline(wl, a, b, a0, ncols=4)
    assert rec["kind"] == "oracle" and rec["unit"] == bench.UNIT
    assert rec["value"] > 0 and rec["cores"] >= 1
    assert "4 of 16 columns" in rec["sample"]
