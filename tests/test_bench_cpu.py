"""Host-side logic of bench.py and of the rocprofv3 summary tool (no GPU)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_0909_0928_amd import profile_summary as PS  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_workload_size():
    # 256x256x100 -> 128x128x50 -> 64x64x25 with 25/50/100 iterations (finest first)
    assert bench.voxel_iters((256, 256, 100), [100, 50, 25]) == 25 * 6553600 + 50 * 819200 + 100 * 102400
    assert bench.voxel_iters(bench.SHAPE, bench.ITERS) == 215040000
    assert bench.level_dims((5, 4, 3), 3) == [(5, 4, 3), (3, 2, 2), (2, 1, 1)]


def test_algorithmic_bytes():
    # images + field in (3) + x-smoothed field out (3), each operand once
    assert bench.algo_bytes_per_voxel("force", 4) == 32 and bench.algo_bytes_per_voxel("force", 2) == 16
    assert bench.algo_bytes_per_voxel("smooth_yz", 4) == 24
    assert bench.algo_bytes_per_voxel("warp", 4) == 24
    assert bench.algo_bytes_per_voxel("warp_pair", 4) == 28 and bench.algo_bytes_per_voxel("warp_pair", 2) == 16
    assert bench.algo_bytes_per_voxel("compose", 4) is None
    # force and smoothing run for every setting; the pre-warps for their variants only
    per_reg = bench.voxel_iters(bench.SHAPE, bench.ITERS)
    assert bench.launch_units("force", bench.SHAPE, bench.ITERS, 1, 3, 6) == 6 * per_reg
    assert bench.launch_units("warp", bench.SHAPE, bench.ITERS, 1, 3, 6) == 3 * per_reg
    assert bench.launch_units("warp_pair", bench.SHAPE, bench.ITERS, 1, 3, 6) == per_reg


def _write_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)


def test_trace_summary_solo_launches(tmp_path):
    k = "void dir::(anonymous namespace)::k_force_x<0, 256, 5, dir::dev::StF32>(dir::(anonymous namespace)::ForceArgs)"
    y = "void dir::(anonymous namespace)::k_smooth_yz<5, 8, dir::dev::StF32>(void const*)"
    trace = [  # two force launches alone, one overlapped by a smoothing launch
        {"Kernel_Name": k, "Start_Timestamp": 0, "End_Timestamp": 10000, "Grid_Size_X": 256, "Grid_Size_Y": 1,
         "Grid_Size_Z": 1},
        {"Kernel_Name": k, "Start_Timestamp": 20000, "End_Timestamp": 40000, "Grid_Size_X": 256, "Grid_Size_Y": 1,
         "Grid_Size_Z": 1},
        {"Kernel_Name": k, "Start_Timestamp": 50000, "End_Timestamp": 60000, "Grid_Size_X": 256, "Grid_Size_Y": 1,
         "Grid_Size_Z": 1},
        {"Kernel_Name": y, "Start_Timestamp": 55000, "End_Timestamp": 58000, "Grid_Size_X": 64, "Grid_Size_Y": 4,
         "Grid_Size_Z": 1},
    ]
    _write_csv(tmp_path / "x_kernel_trace.csv", trace)
    _write_csv(tmp_path / "x_kernel_stats.csv", [{"Name": k, "Calls": 3, "TotalDurationNs": 40000,
                                                   "AverageNs": 13333.3, "Percentage": 90.0}])
    out = tmp_path / "s.md"
    PS.trace_summary(str(tmp_path), "cmd", str(out))
    text = out.read_text()
    solo = [l for l in text.splitlines() if l.startswith("| `k_force_x` | all |")]
    assert solo and solo[0].split("|")[3].strip() == "2" and solo[0].split("|")[4].strip() == "15.00"


def test_traffic_summary_scales_by_the_copy(tmp_path):
    kib = PS.COPY_BYTES / 1024.0
    name = "void dir::(anonymous namespace)::k_force_x<0, 256, 5, dir::dev::StF32>(dir::ForceArgs)"
    for d, copy_reading, kernel_reading in (("f", kib / 2, 100.0), ("w", kib, 40.0)):
        os.makedirs(tmp_path / d)
        os.makedirs(tmp_path / (d + "c"))
        _write_csv(tmp_path / d / "b_counter_collection.csv",
                   [{"Kernel_Name": name, "Counter_Value": kernel_reading, "Grid_Size": 1}])
        _write_csv(tmp_path / (d + "c") / "c_counter_collection.csv",
                   [{"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Value": copy_reading, "Grid_Size": 1}])
    r = PS.traffic_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "fc"), str(tmp_path / "wc"),
                           "force", "cmd", str(tmp_path / "t.json"))
    assert r["fetch_factor"] == pytest.approx(2.0) and r["write_factor"] == pytest.approx(1.0)
    assert r["traffic_bytes_per_launch"] == pytest.approx(100.0 * 1024 * 2 + 40.0 * 1024)
    assert r["source_sha256"] == PS.source_fingerprint("force")


def test_rounded_field_oracle_is_the_oracle_without_rounding():
    """The parity envelope's rounded-field registration, run without rounding,
    is bitwise the oracle's registration (same primitives in the same order)."""
    import numpy as np
    import oracle as O
    from paper_0909_0928_amd import phantom as P
    ph = P.make_phantom((20, 18, 10), seed=5, max_u=2.0)
    for variant in ("passive", "inverse_consistent"):
        ref, _, _, _ = O.register(ph.static, ph.moving, O.VARIANTS[variant], [3, 2], sigma=1.0, radius=3,
                                  alpha=0.4)
        got = bench.register_f32_field(O, ph.static, ph.moving, variant, [3, 2], 1.0, 3, 0.4, round_field=False)
        assert np.array_equal(got, ref)
        r = bench.register_f32_field(O, ph.static, ph.moving, variant, [3, 2], 1.0, 3, 0.4)
        assert 0 < bench.rms_vox(r, ref) < 1e-4


def test_perturbed_pair_is_one_rounding():
    import numpy as np
    S = np.full((4, 5, 6), -1000.0)
    Sp, Mp = bench.perturbed_pair(S, S + 1.0, 99)
    assert 0 < np.abs(Sp / S - 1).max() <= bench.PERTURB_REL
