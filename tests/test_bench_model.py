"""The benchmark's algorithmic-byte model (CPU): the step totals of the three workloads."""
import importlib.util
import os

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
