"""The benchmark's algorithmic-byte model (CPU): the step totals of the three workloads."""
import importlib.util
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_step_bytes_match_the_measurement_plan():
    b = _bench()
    # 36 N_p + 32 M + 16 M_h + 8 J B, in MB
    assert round(b.step_algorithmic_bytes(256, 256 ** 3, 1, 64, 200) / 1e6, 1) == 1276.2
    assert round(b.step_algorithmic_bytes(512, 512 ** 3, 1, 128, 400) / 1e6, 1) == 10205.2
    assert round(b.step_algorithmic_bytes(64, 64 ** 3, 64, 48, 100) / 1e6, 1) == 1281.7


def test_stage_bytes_sum_covers_the_step():
    b = _bench()
    sb = b.stage_bytes(256, 256 ** 3, 1, 64, 200, 1032)
    assert sb["cic_interp"] == 24 * 256 ** 3 + 12 * 256 ** 3
    assert sb["cic_deposit"] == 12 * 256 ** 3 + 4 * 256 ** 3
    sp = b.stage_bytes(256, 256 ** 3, 1, 64, 200, 1032, deposit_mode=6)
    assert sp["cic_deposit"] + sp["patch_reduce"] == sb["cic_deposit"]


def test_traffic_table_from_counter_csvs(tmp_path):
    """bench_traffic scales the counters by the plain copy and files them per stage."""
    sys.path.insert(0, ROOT)
    import bench
    import bench_traffic
    hdr = '"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n'
    dep = "void pmnu::(anonymous namespace)::deposit_tiled_kernel<2048, 5120, 256>(float const*)"
    fz = "void pmnu::(anonymous namespace)::fwd_z_kernel<256>(unsigned long long const*)"
    cp = "__amd_rocclr_copyBuffer"

    def write(name, counter, rows):
        p = tmp_path / name
        p.write_text(hdr + "".join(f'{i},"{k}","{counter}",{v}\n' for i, (k, v) in enumerate(rows)))
        return str(p)
    f = write("f.csv", "FETCH_SIZE", [(dep, 100.0), (dep, 300.0), (fz, 50.0)])
    w = write("w.csv", "WRITE_SIZE", [(dep, 400.0), (dep, 400.0), (fz, 25.0)])
    cf = write("cf.csv", "FETCH_SIZE", [(cp, 1.0), (cp, 512.0)])     # copy of 1 MiB reads half
    cw = write("cw.csv", "WRITE_SIZE", [(cp, 1024.0)])
    out = tmp_path / "traffic.json"
    argv = sys.argv
    sys.argv = ["bench_traffic.py", "--workload", "pm256", "--fetch", f, "--write", w,
                "--copy-fetch", cf, "--copy-write", cw, "--copy-mib", "1", "--out", str(out)]
    try:
        bench_traffic.main()
    finally:
        sys.argv = argv
    t = json.loads(out.read_text())["pm256"]
    assert t["calibration"]["fetch_factor"] == 2.0 and t["calibration"]["write_factor"] == 1.0
    rec = t["kernels"]["cic_deposit"]["deposit_tiled_kernel<2048, 5120, 256>"]
    assert rec["fetch_bytes"] == 2.0 * 1024 * 200.0 and rec["write_bytes"] == 1024 * 400.0
    assert t["kernels"]["fft_fwd_z"]["fwd_z_kernel<256>"]["bytes_per_launch"] == 1024 * 125.0
    assert bench.kernel_name("cic_deposit", {"deposit_mode": 2}, 256) == \
        "deposit_tiled_kernel<2048, 5120, 256>"
    tiles = {"fft_tiles": {"fwd_z": 32, "fwd_y": 16, "fwd_x": 16, "inv_x": 8, "inv_y": 4,
                           "inv_z": 8}}
    assert bench.kernel_name("fft_inv_z", tiles, 512) == "inv_z_kernel<512, 8>"
    assert bench.kernel_name("fft_fwd_z", dict(tiles, deposit_mode=6), 256) == \
        "fwd_z_kernel<256, true, 32>"
    assert bench.kernel_name("fft_fwd_x_bin", tiles, 256) == \
        "fwd_x_bin_kernel<256, false, true, 16>"
    assert bench.kernel_name("cic_deposit", {"deposit_mode": 6}, 256) == \
        "deposit_patch_kernel<4096, 6144, 512>"
    assert bench.kernel_name("cic_deposit", {"deposit_mode": 7}, 256) == \
        "deposit_patch_kernel<4096, 9216, 512>"
    assert bench.kernel_name("fft_fwd_z", dict(tiles, deposit_mode=7), 256) == \
        "fwd_z_kernel<256, true, 32>"
