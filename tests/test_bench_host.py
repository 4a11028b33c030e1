"""Host logic of bench.py (no GPU): the one-GPU refusal, the counter
summary's copy-kernel calibration, and the rule that measured traffic is
reported only for the kernel source and workload size it was taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def _counter_csv(path, counter, rows):
    with open(path, "w") as f:
        f.write("Kernel_Name,Counter_Name,Counter_Value\n")
        for name, value in rows:
            f.write(f'"{name}",{counter},{value}\n')


def test_pmc_summary_scales_by_the_copy_kernel(tmp_path):
    """A 1 MiB copy kernel reads as 512 KiB FETCH_SIZE and 1 024 KiB
    WRITE_SIZE: fetch counts are doubled, write counts kept."""
    step = "void swe::swe_step_kernel<256, 256, false, false>(swe::StepArgs)"
    neg = "at::native::vectorized_elementwise_kernel<neg_kernel_cuda>"
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(f, "FETCH_SIZE", [(neg, 512.0), (step, 100.0),
                                   (step, 300.0)])
    _counter_csv(w, "WRITE_SIZE", [(neg, 1024.0), (step, 50.0)])
    out = tmp_path / "t.json"
    bench.pmc_summary(str(f), str(w), 1, 1000, str(out))
    t = json.loads(out.read_text())
    assert t["reference"]["fetch_scale"] == 2.0
    assert t["reference"]["write_scale"] == 1.0
    assert t["fetch_bytes_per_launch"] == 200.0 * 1024 * 2.0
    assert t["write_bytes_per_launch"] == 50.0 * 1024
    assert t["bytes_per_cell"] == (200.0 * 2048 + 50.0 * 1024) / 1000
    assert t["dispatches"] == {"fetch": 2, "write": 1}
    assert t["kernel_sha256"] == bench.kernel_hash()


def test_traffic_only_for_its_kernel_and_size(tmp_path, monkeypatch):
    path = tmp_path / "t.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.counter_record(10) is None   # no file
    path.write_text(json.dumps(dict(kernel_sha256=bench.kernel_hash(),
                                    n_cells=10, bytes_per_launch=123.0)))
    assert bench.counter_record(10)["bytes_per_launch"] == 123.0
    assert bench.counter_record(11) is None   # other size
    path.write_text(json.dumps(dict(kernel_sha256="0" * 64, n_cells=10,
                                    bytes_per_launch=123.0)))
    assert bench.counter_record(10) is None   # other source


def test_pmc_summary_leaves_out_the_fresh_slot_step(tmp_path):
    """The adjoint's fresh-slot instantiation of the step kernel is not the
    plain step: its dispatches do not enter the summary; VALU counters give
    instructions per launch and the issue share."""
    step = ("void swe::(anonymous namespace)::swe_step_kernel<256, 256, "
            "false, false, false>(swe::StepArgs)")
    slot = step.replace("false, false, false>", "false, false, true>")
    neg = "at::native::vectorized_elementwise_kernel<neg_kernel_cuda>"
    f, w, v = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "v.csv"
    _counter_csv(f, "FETCH_SIZE", [(neg, 512.0), (step, 100.0),
                                   (slot, 900.0)])
    _counter_csv(w, "WRITE_SIZE", [(neg, 1024.0), (step, 50.0),
                                   (slot, 900.0)])
    with open(v, "w") as fh:
        fh.write("Kernel_Name,Counter_Name,Counter_Value\n")
        for c, val in (("SQ_INSTS_VALU", 1024.0),
                       ("SQ_INSTS_VALU_TRANS_F64", 0.0),
                       ("SQ_BUSY_CU_CYCLES", 256.0 * 8)):
            fh.write(f'"{step}",{c},{val}\n')
            fh.write(f'"{slot}",{c},{10 * val}\n')
    out = tmp_path / "t.json"
    bench.pmc_summary(str(f), str(w), 1, 1000, str(out), str(v), "1..12")
    t = json.loads(out.read_text())
    assert t["fetch_bytes_per_launch"] == 100.0 * 1024 * 2.0
    assert t["write_bytes_per_launch"] == 50.0 * 1024
    assert t["steps"] == "1..12"
    # 1 024 instructions x 4 cycles / 1 024 SIMDs = 4 cycles of 8 per CU
    assert t["valu"]["insts_per_launch"] == 1024.0
    assert t["valu"]["issue_frac"] == 0.5
