"""Host logic of bench.py (no GPU): the one-GPU contract, the algorithmic byte and
flop counts the roofline figures use, and the traffic records' source check."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_algorithmic_counts(bench):
    # LU of the 55 x 55 system, four right-hand sides, 35^2 PHS entries in 3D
    assert bench.weights_flops(35, 20, 3, 4) == pytest.approx((2 / 3) * 55 ** 3 + 8 * 55 ** 2 + 10 * 35 ** 2)
    assert bench.knn_bytes(35, 3) == 24 + 140
    assert bench.csr_bytes(35, 4) == 2 * (140 + 1120) + 8
    # BiCGStab: two row products and three vector passes; block-Jacobi adds two
    # block products (64 float16 entries, the scale, the order and the output)
    assert bench.bicgstab_bytes_per_row(35) == 2 * (8 + 420 + 32) + 112
    assert bench.bicgstab_bytes_per_row(9) == 408
    assert bench.bicgstab_bytes_per_row(35, "block_jacobi") == bench.bicgstab_bytes_per_row(35) + 2 * (128 + 16)


def test_traffic_records_follow_their_sources(bench, tmp_path, monkeypatch):
    for wl, (path, files) in bench.TRAFFIC.items():
        assert os.path.exists(os.path.join(ROOT, path)), path
        for f in files:
            assert os.path.exists(os.path.join(ROOT, f)), f
    # a record taken on other sources (or another form) is not used
    rec = os.path.join(ROOT, bench.TRAFFIC["cube_sphere3d"][0])
    text = open(rec).read()
    fake = tmp_path / "rec.txt"
    fake.write_text(text.replace("source_hash: ", "source_hash: 0"))
    monkeypatch.setitem(bench.TRAFFIC, "cube_sphere3d", (str(fake), bench.TRAFFIC["cube_sphere3d"][1]))
    assert bench.recorded_traffic("cube_sphere3d", "f32_ir") is None
    fake.write_text(text)
    v = bench.recorded_traffic("cube_sphere3d", "f32_ir")
    if v is not None:  # the committed record matches the committed sources
        assert v > 1e9
        assert bench.recorded_traffic("cube_sphere3d", "f64") is None
