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
