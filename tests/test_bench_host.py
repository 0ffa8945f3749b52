"""Host-side pieces of bench.py: the kernel-source digest that ties the committed
counter summary to the kernel it was measured on."""
import os
import shutil

import bench


def _copy_sources(tmp_path):
    for rel in bench.KERNEL_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, rel), dst)
    return tmp_path


def test_digest_ignores_comments_and_blank_lines(tmp_path, monkeypatch):
    root = _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(root))
    d0 = bench.kernel_source_digest()
    p = root / bench.KERNEL_SOURCES[0]
    text = p.read_text()
    p.write_text("// a new comment line\n\n" + text.replace("\n", "  // trailing note\n", 1))
    assert bench.kernel_source_digest() == d0


def test_digest_sees_code_changes(tmp_path, monkeypatch):
    root = _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(root))
    d0 = bench.kernel_source_digest()
    p = root / bench.KERNEL_SOURCES[1]
    p.write_text(p.read_text() + "\nstatic const int lbmz_digest_probe = 1;\n")
    assert bench.kernel_source_digest() != d0


def test_traffic_is_dropped_for_another_kernel(tmp_path, monkeypatch):
    root = _copy_sources(tmp_path)
    prof = root / bench.TRAFFIC_FILE
    prof.parent.mkdir(parents=True, exist_ok=True)
    prof.write_text(f"# header\nsource_digest {'0' * 16}\nbytes_per_launch 123\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.measured_traffic() is None
    prof.write_text(f"# header\nsource_digest {bench.kernel_source_digest()}\nbytes_per_launch 123\n")
    assert bench.measured_traffic() == 123


def test_byte_model_matches_the_stated_per_update_figures():
    # per lattice update at 2048^2: 78.2 B at density 1, 26.2 B at 0.3, 11.3 B at
    # 0.1, 4.9 B at 0.03, 2.7 B at 0.01 (records read + written, halo, table)
    npatch = (2048 // 64) ** 2
    lups = 2048 * 2048
    for rho, want in ((1.0, 78.2), (0.3, 26.2), (0.1, 11.3), (0.03, 4.9), (0.01, 2.7)):
        assert abs(bench.bytes_model(rho, npatch) / lups - want) < 0.06, rho


def test_fixed_error_ratio_interpolates_and_reports_saturation():
    pts = [{"eps": 1e-5, "rel_l2": 1e-4, "ratio": 100.0}, {"eps": 1e-4, "rel_l2": 4e-4, "ratio": 200.0},
           {"eps": 1e-3, "rel_l2": 8e-4, "ratio": 220.0}]
    r = bench.cr_at_error(pts, 2e-4)
    assert r["bracket_eps"] == [1e-5, 1e-4] and 100.0 < r["ratio"] < 200.0
    r = bench.cr_at_error(pts, 1e-3)
    assert r["bracket_eps"] is None and r["ratio"] == 220.0
    assert bench.cr_at_error(pts, 1e-5)["ratio"] is None


def test_cpu_baseline_harness_gives_the_oracle_result():
    out = bench.cpu_baseline(steps=1, workers=2, n=128)
    assert out["identical_results"] and out["cores"] == 2 and out["kind"] == "oracle"
    assert out["value"] > 0 and out["one_core"]["value"] > 0 and out["cpu"]["nproc"] >= 1
