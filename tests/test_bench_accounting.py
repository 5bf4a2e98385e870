"""The benchmark's roofline accounting and its recorded-traffic lookup, on the CPU.

The roofline object charges the dominant kernel with its share of the layer's algorithmic
bytes, (N_in + N_out) B per layer call split over the gates of that call, and keeps the
per-pass rate and the counted DRAM traffic apart.  The traffic figure must only be reported
for the kernel sources it was counted on.
"""
import bench


def _stats():
    # two kernels; the second has the larger device time and is the dominant one
    return [
        {"name": "noise", "launches": 10, "total_ms": 5.0, "layer_bytes": 4.0e9, "algo_bytes": 4.0e9},
        {"name": "gate_tile_256", "launches": 100, "total_ms": 10.0, "layer_bytes": 2.0e9, "algo_bytes": 1.0e11},
    ]


def test_roofline_charges_the_dominant_kernel_its_layer_bytes():
    r = bench.roofline(_stats(), "tfim7x8_pna", "f64", copy_gbs=5000.0)
    assert r["kernel"] == "gate_tile_256"
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == bench.HBM_PEAK_GBS
    # 2e9 layer bytes over 100 launches of 0.1 ms each: 2e7 B / 1e-4 s = 200 GB/s
    assert abs(r["achieved"] - 200.0) < 1e-9
    assert abs(r["frac"] - 200.0 / bench.HBM_PEAK_GBS) < 1e-9
    # the pass's own rate: 1e9 B per launch / 1e-4 s = 10 TB/s, against the copy ceiling
    assert abs(r["pass_gbs"] - 10000.0) < 1e-6
    assert abs(r["pass_frac_of_copy"] - 2.0) < 1e-9
    assert r["launches"] == 100 and abs(r["avg_launch_ms"] - 0.1) < 1e-12
    assert abs(r["share_of_device_time"] - 10.0 / 15.0) < 1e-3


def test_recorded_traffic_needs_matching_sources(tmp_path, monkeypatch):
    src = bench.kernel_source_hash()
    f = tmp_path / "traffic.md"
    f.write_text("notes\n"
                 f"traffic: tfim7x8_pna gate_tile_256 f64 1070000000 {src}\n"
                 "traffic: tfim7x8_pna gate_tile_128 f64 777 0000000000000000\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.recorded_traffic("tfim7x8_pna", "gate_tile_256", "f64") == 1.07e9
    assert bench.recorded_traffic("tfim7x8_pna", "gate_tile_256", "f32k") is None     # other precision
    assert bench.recorded_traffic("tfim8x16", "gate_tile_256", "f64") is None         # other workload
    assert bench.recorded_traffic("tfim7x8_pna", "gate_tile_128", "f64") is None      # stale sources
    r = bench.roofline(_stats(), "tfim7x8_pna", "f64")
    assert r["traffic"] == 1070000000
    assert abs(r["traffic_over_pass_bytes"] - 1.07) < 1e-9        # against 1e9 pass bytes a launch
    assert abs(r["traffic_gbs"] - 10700.0) < 1e-6
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.md"))
    assert bench.recorded_traffic("tfim7x8_pna", "gate_tile_256", "f64") is None

