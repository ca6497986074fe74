"""CPU-side checks of the measurement helpers: the counter-traffic
conversion (calibration by a copy of known size, per-kernel averages, the
source hash and workload that scope a figure) and bench.py's refusal of
more than one GPU. No GPU is used."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2609_07204_amd import traffic  # noqa: E402

HEADER = ('"Correlation_Id","Dispatch_Id","Agent_Id","Queue_Id","Process_Id","Thread_Id","Grid_Size","Kernel_Id",'
          '"Kernel_Name","Workgroup_Size","LDS_Block_Size","Scratch_Size","VGPR_Count","Accum_VGPR_Count",'
          '"SGPR_Count","Counter_Name","Counter_Value","Start_Timestamp","End_Timestamp"\n')


def write_run(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w") as f:
        f.write(HEADER)
        for i, (name, value) in enumerate(rows):
            f.write('%d,%d,"Agent 1",1,1,1,1,1,"%s",256,0,0,8,0,16,"%s",%f,0,1\n' % (i, i, name, counter, value))


def test_traffic_scales_by_the_copy_and_averages_per_launch(tmp_path):
    mib = 16
    nbytes = mib << 20
    # the copy reads nbytes in FETCH units of 2048 B and writes in 1024 B units
    write_run(str(tmp_path / "f"), "FETCH_SIZE", [
        ("__amd_rocclr_copyBuffer", nbytes / 2048),
        ("(anonymous namespace)::k_big_insert(DGraph)", 1000.0),
        ("(anonymous namespace)::k_big_insert(DGraph)", 3000.0),
        ("(anonymous namespace)::k_other(int)", 5.0)])
    write_run(str(tmp_path / "w"), "WRITE_SIZE", [
        ("__amd_rocclr_copyBuffer", nbytes / 1024),
        ("(anonymous namespace)::k_big_insert(DGraph)", 10.0),
        ("(anonymous namespace)::k_big_insert(DGraph)", 30.0)])
    out = str(tmp_path / "traffic.json")
    res = traffic.main(str(tmp_path / "f"), str(tmp_path / "w"), str(mib), "rhg", out)
    cal = res["_calibration"]
    assert cal["fetch_factor"] == pytest.approx(2048.0) and cal["write_factor"] == pytest.approx(1024.0)
    assert cal["workload"] == "rhg"
    k = res["k_big_insert"]
    assert k["launches"] == 2
    assert k["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 2048)
    assert k["write_bytes_per_launch"] == pytest.approx(20.0 * 1024)
    assert k["bytes_per_launch"] == pytest.approx(2000.0 * 2048 + 20.0 * 1024)
    src = os.path.join(ROOT, k["source"])
    assert k["source_sha256"] == hashlib.sha256(open(src, "rb").read()).hexdigest()
    assert "k_other" not in res           # only the timed kernels are kept
    assert json.load(open(out)) == {"rhg": json.loads(json.dumps(res))}
    # a run of another workload adds its own section and keeps this one
    traffic.main(str(tmp_path / "f"), str(tmp_path / "w"), str(mib), "chung_lu", out)
    assert set(json.load(open(out))) == {"rhg", "chung_lu"}


def test_bench_reports_traffic_only_for_its_workload_and_source():
    import bench
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        pytest.skip("no committed traffic summary")
    full = json.load(open(path))
    for measured, tab in full.items():
        assert tab["_calibration"]["workload"] == measured
        others = [w for w in ("chung_lu", "rhg", "batch", "served") if w not in full]
        for kernel in [k for k in tab if not k.startswith("_")]:
            for w in others:
                assert bench.traffic_for(kernel, w) is None
            rec = tab[kernel]
            same = hashlib.sha256(open(os.path.join(ROOT, rec["source"]), "rb").read()).hexdigest() == \
                rec["source_sha256"]
            got = bench.traffic_for(kernel, measured)
            assert (got == rec["bytes_per_launch"]) if same else got is None
        assert bench.traffic_for("k_no_such_kernel", measured) is None


def test_traffic_kernels_name_their_defining_sources():
    # every kernel of the committed summary is keyed to the file that
    # defines it (template instances by their base name)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        pytest.skip("no committed traffic summary")
    srcs = traffic.kernel_sources()
    for w, tab in json.load(open(path)).items():
        for kernel, rec in tab.items():
            if kernel.startswith("_"):
                continue
            assert srcs.get(kernel.split("<")[0]) == rec["source"], (w, kernel)


def test_headline_roofline_kernel_has_current_traffic():
    # the hyperbolic solve's dominant kernel (the roofline's) has a counter
    # figure measured on its current source
    import bench
    if not os.path.exists(os.path.join(ROOT, "profiles", "traffic.json")):
        pytest.skip("no committed traffic summary")
    got = bench.traffic_for("k_lp_flat", "rhg")
    assert got is not None and got > 0


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""
