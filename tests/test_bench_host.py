"""Host logic of bench.py that needs no GPU: the one-GPU guard and the HBM
traffic summary (counter means scaled by the calibration copy)."""
import csv
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode != 0
    assert "one GPU" in res.stdout


def write_counters(directory, counter, rows):
    os.makedirs(directory, exist_ok=True)
    with open(os.path.join(directory, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow(dict(Kernel_Name=name, Counter_Name=counter, Counter_Value=value))


def test_traffic_summary_scaling(tmp_path, capsys):
    b = load_bench()
    b.TRAFFIC_JSON = str(tmp_path / "traffic.json")
    pair = "void lub::k_pairs<float, false>(lub::CallDesc, ...)"
    tangent = "void lub::k_pairs<float, true>(lub::CallDesc, ...)"
    nbr = "void lub::k_neighbors<32, 0, 4>(lub::CallDesc, ...)"
    probe = "void lub::k_neighbors<16, 0, 4>(lub::CallDesc, ...)"
    copy = "__amd_rocclr_copyBuffer"
    # the copy reads 512 MiB: FETCH_SIZE shows half (scale 2), WRITE_SIZE all
    write_counters(tmp_path / "f", "FETCH_SIZE",
                   [(copy, 262144.0), (copy, 10.0), (pair, 100.0), (pair, 300.0),
                    (tangent, 5.0), (nbr, 1000.0), (nbr, 1000.0), (nbr, 1000.0),
                    (probe, 7.0)])
    write_counters(tmp_path / "w", "WRITE_SIZE",
                   [(copy, 524288.0), (pair, 50.0), (pair, 50.0), (tangent, 1.0),
                    (nbr, 20.0), (nbr, 20.0), (nbr, 20.0), (probe, 1.0)])
    b.traffic_summary(str(tmp_path / "f"), str(tmp_path / "w"), "wl", "mixed")
    rec = json.load(open(b.TRAFFIC_JSON))
    m = rec["k_pairs"]["wl/mixed"]
    assert m["kernel"] == pair and m["dispatches"] == 2
    assert abs(m["scale_fetch"] - 2.0) < 1e-12 and abs(m["scale_write"] - 1.0) < 1e-12
    # mean fetch 200 KiB x 2 + mean write 50 KiB x 1
    assert abs(m["bytes_per_launch"] - (400.0 + 50.0) * 1024.0) < 1e-6
    assert rec["k_pairs"]["source_sha256"] == b.kernel_source_hash("k_pairs")
    # the most frequent instantiation of the neighbour search is taken
    n = rec["k_neighbors"]["wl/mixed"]
    assert n["kernel"] == nbr and abs(n["bytes_per_launch"] - 2020.0 * 1024.0) < 1e-6
    # the bench line takes it only while the kernel source is unchanged
    assert b.kernel_traffic("k_pairs", "wl", "mixed") == m["bytes_per_launch"]
    assert b.kernel_traffic("k_pairs", "other", "mixed") is None
    rec["k_pairs"]["source_sha256"] = "0" * 64
    json.dump(rec, open(b.TRAFFIC_JSON, "w"))
    assert b.kernel_traffic("k_pairs", "wl", "mixed") is None


def test_advance_goes_through_the_library():
    """The trajectory's step is the library's kinematic advance (its
    arithmetic is pinned with the oracle's in test_oracle_integrate.py and
    compared on the GPU in test_gpu_integrate.py), with the bench's dt."""
    b = load_bench()
    calls = []

    class Handle:
        def advance(self, r, q, v, w, dt):
            calls.append((r, q, v, w, dt))

    b.advance(Handle(), "r", "q", "v", "w", 0.5)
    assert calls == [("r", "q", "v", "w", 0.5)]
