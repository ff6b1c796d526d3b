"""Host logic of bench.py (no GPU): the kernel-source hash that keys the committed counter
summary, and the lookup of HBM bytes per launch from it."""
import json
import os
import shutil

import pytest

import bench


def _copy_sources(tmp_path):
    root = tmp_path / "repo"
    shutil.copytree(os.path.join(bench.ROOT, "paper_2602_21242_amd", "csrc"),
                    root / "paper_2602_21242_amd" / "csrc")
    return root


def test_strip_comments():
    src = "int a; // one\n/* two\n three */ int b;   \n\n  // only a comment\nint c; /* x */ int d;\n"
    assert bench._strip_comments(src) == "int a;\n int b;\nint c;  int d;"


def test_source_hash_ignores_comments_and_host_only_file(tmp_path, monkeypatch):
    root = _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(root))
    h0 = bench.kernel_source_hash()
    dev = root / "paper_2602_21242_amd" / "csrc" / "lbm_device.h"
    dev.write_text(dev.read_text() + "\n// a comment added at the end\n\n/* and a block\n comment */\n")
    api = root / "paper_2602_21242_amd" / "csrc" / "lbm_api.hip"
    api.write_text(api.read_text() + "\nstatic int host_side_change = 1;\n")
    assert bench.kernel_source_hash() == h0


def test_source_hash_follows_device_code(tmp_path, monkeypatch):
    root = _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(root))
    h0 = bench.kernel_source_hash()
    step = root / "paper_2602_21242_amd" / "csrc" / "lbm_step.h"
    step.write_text(step.read_text().replace("constexpr int kAuxNT = 2;", "constexpr int kAuxNT = 0;"))
    assert bench.kernel_source_hash() != h0


def test_traffic_lookup(tmp_path, monkeypatch):
    """The committed summary is used only while its hash matches the sources."""
    path = os.path.join(bench.ROOT, "profiles", "traffic.json")
    with open(path) as fh:
        data = json.load(fh)
    ent = data["entries"]["tg4096/complete/f32/ab"]
    # bytes per launch = scaled FETCH_SIZE + WRITE_SIZE (KiB per dispatch)
    expect = (ent["FETCH_SIZE_KiB"] * 1024 * data["copy_scale"]["FETCH_SIZE"]
              + ent["WRITE_SIZE_KiB"] * 1024 * data["copy_scale"]["WRITE_SIZE"])
    assert ent["hbm_bytes_per_launch"] == pytest.approx(expect, rel=1e-6)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: data["kernel_source_hash"])
    assert bench.load_traffic("tg4096", "complete", "f32", "ab") == ent["hbm_bytes_per_launch"]
    assert bench.load_traffic("tg4096", "complete", "f32", "no-such-pattern") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.load_traffic("tg4096", "complete", "f32", "ab") is None


def test_section_merges_results_and_records_failures():
    var = {"kept": 1}
    bench.section(var, "ok", lambda: {"a": 2.0})
    assert var == {"kept": 1, "a": 2.0}

    def boom():
        raise RuntimeError("device allocation failed")

    bench.section(var, "big", boom)
    assert var["kept"] == 1 and var["a"] == 2.0
    assert "device allocation failed" in var["big_error"]
