"""Host logic of bench.py: the sort plan, the algorithmic byte counts and the conversion of
two rocprofv3 counter files into HBM bytes per launch (calibrated by the 1 GiB copy)."""
import csv
import json

import pytest

import bench


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_sort_plan_covers_the_key_range():
    for C in (1, 3, 1000, 1600, 4096, 262144, 1 << 20, 2250000, 1 << 22):
        bits = bench.sort_plan(C)
        assert sum(bits) == max(1, C.bit_length())      # keys 0..C, C = outside the grid
        assert max(bits) <= 11 and max(bits) - min(bits) <= 1
    assert bench.sort_plan(262144) == [10, 9]
    assert bench.sort_plan(1 << 22) == [8, 8, 7]


def test_cycle_budget_matches_the_per_unit_figures():
    # 156 B per persistent particle, 28 per new-born slot, 92 per cell
    assert bench.b_alg(2 ** 21, 2 ** 18, 512 * 512) == 358612992
    # the sort is one ideal pass over the 24-byte record, shared by its scatter launches
    assert bench.algorithmic_bytes("k_sort_scatter", 1000, 0, 4096) == 1000 * 48 / 2


def test_traffic_from_counter_files(tmp_path):
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    scatter = "dogm::k_sort_scatter(dogm::Batch, unsigned int)"
    # the copy fetches half its bytes as counted by FETCH_SIZE, writes them 1:1
    _counter_csv(fetch, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 2.0),
                                       ("__amd_rocclr_copyBuffer", 524288.0),
                                       (scatter, 1000.0), (scatter, 3000.0),
                                       ("unrelated_kernel", 5.0)])
    _counter_csv(write, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 0.0),
                                       ("__amd_rocclr_copyBuffer", 1048576.0),
                                       (scatter, 500.0), (scatter, 1500.0)])
    bench.write_traffic(str(fetch), str(write), "c512", ["cmd-f", "cmd-w"], outdir=str(tmp_path))
    rec = json.loads((tmp_path / "traffic_c512.json").read_text())
    assert rec["fetch_factor"] == pytest.approx(2.0) and rec["write_factor"] == pytest.approx(1.0)
    k = rec["kernels"]["k_sort_scatter"]
    assert k["launches"] == 2
    assert k["read_bytes"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert k["written_bytes"] == pytest.approx(1000.0 * 1024)
    assert k["source_sha256"] == bench.source_digest("k_sort_scatter")
    assert "unrelated_kernel" not in rec["kernels"]
    assert bench.measured_traffic("k_sort_scatter", "c512", outdir=str(tmp_path)) == \
        pytest.approx(k["read_bytes"] + k["written_bytes"])
    # a record whose source digest no longer matches is not reported
    rec["kernels"]["k_sort_scatter"]["source_sha256"] = "0" * 64
    (tmp_path / "traffic_c512.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("k_sort_scatter", "c512", outdir=str(tmp_path)) is None
    assert "k_sort_scatter" in (tmp_path / "hbm_traffic_c512.md").read_text()


def test_traffic_needs_the_calibration_copy(tmp_path):
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(fetch, "FETCH_SIZE", [("dogm::k_predict(dogm::Batch)", 10.0)])
    _counter_csv(write, "WRITE_SIZE", [("dogm::k_predict(dogm::Batch)", 10.0)])
    with pytest.raises(SystemExit):
        bench.write_traffic(str(fetch), str(write), "c512", [], outdir=str(tmp_path))


def test_more_than_one_gpu_is_refused(monkeypatch, capsys):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
