"""Host logic of bench.py (no GPU): the one-GPU contract, kernel-name parsing, the calibrated
traffic summary and its source-hash guard, and the per-launch algorithmic bytes."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("sig, name", [
    ("void dgp::k_relax<float, 256>(dgp::cx<float> const*, unsigned long, float*)", "dgp::k_relax<float, 256>"),
    ("dgp::k_p3<double, 256, (dgp::SpecMode)0>(dgp::cx<double> const*, int)", "dgp::k_p3<double, 256, (dgp::SpecMode)0>"),
    ("__amd_rocclr_copyBuffer", "__amd_rocclr_copyBuffer"),
])
def test_kernel_name(sig, name):
    assert bench.kernel_name(sig) == name


def test_algorithmic_bytes_of_the_roofline_kernel():
    # 256^3 float32 relaxation launch: six spectra read and one written (complex float), the
    # field and source read and the field written (float)
    hs = 129 * 256 * 256
    assert bench.algorithmic_bytes("relax", 256, 4) == 7 * hs * 8 + 3 * 256 ** 3 * 4 == 674758656
    # split Hessian: the axis-1 inverse pass reads three spectra and writes six
    assert bench.algorithmic_bytes("axis1_inv", 256, 8) == 9 * hs * 16
    assert bench.algorithmic_bytes("fanout", 256, 4) == 4 * hs * 8


def _counter_csv(path, rows):
    with open(path, "w") as fh:
        fh.write("Kernel_Name,Counter_Name,Counter_Value\n")
        for name, value in rows:
            fh.write('"%s",X,%r\n' % (name, value))


def test_pmc_summary_calibration_and_working_dispatches(tmp_path, monkeypatch):
    mib = 1024.0   # counter values are KiB
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    # the calibration copy reads half (fetch) and all (write) of its 512 MiB in the counters;
    # the second relaxation dispatch exited at once (below 5 % of the largest)
    _counter_csv(fetch, [("__amd_rocclr_copyBuffer", 256 * mib), ("void dgp::k_relax<float, 256>(int)", 300 * mib),
                         ("void dgp::k_relax<float, 256>(int)", 1.0)])
    _counter_csv(write, [("__amd_rocclr_copyBuffer", 512 * mib), ("void dgp::k_relax<float, 256>(int)", 70 * mib),
                         ("void dgp::k_relax<float, 256>(int)", 0.5)])
    text = bench.pmc_summary(str(fetch), str(write))
    blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    k = blob["kernels"]["dgp::k_relax<float, 256>"]
    assert k["dispatches"] == 2 and k["working"] == 1
    assert k["fetch_bytes"] == pytest.approx(600 * 2 ** 20)   # scaled x2
    assert k["write_bytes"] == pytest.approx(70 * 2 ** 20)    # scaled x1
    assert blob["source_sha256"] == bench.kernel_source_digest()
    # the stored figure is used only while the device sources hash to the recorded value
    stored = tmp_path / "traffic.md"
    stored.write_text(text)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stored))
    assert bench.stored_traffic("relax_fp32") == pytest.approx(670 * 2 ** 20)
    stored.write_text(text.replace(blob["source_sha256"], "0" * 64))
    assert bench.stored_traffic("relax_fp32") is None


def test_trace_summary_working_average(tmp_path):
    trace = tmp_path / "t.csv"
    with open(trace, "w") as fh:
        fh.write("Kernel_Name,Start_Timestamp,End_Timestamp\n")
        for start, dur_ns in ((0, 160000), (1000000, 170000), (2000000, 3000)):
            fh.write('"void dgp::k_relax<float, 256>(int)",%d,%d\n' % (start, start + dur_ns))
    row = [l for l in bench.trace_summary(str(trace)).splitlines() if "k_relax" in l][0].split("|")
    assert int(row[2]) == 3 and int(row[4]) == 2          # calls, working dispatches
    assert float(row[5]) == pytest.approx(165.0)           # working average, us
