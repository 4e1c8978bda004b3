"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic bytes
per cell the roofline uses, and the lookup of committed counter summaries,
which must refuse figures taken on other kernel sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1", "--warmup", "0"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_unknown_extra_sections_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--extras", "variants,nonsense"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "nonsense" in r.stderr


@pytest.mark.parametrize("elem,force,want", [(4, 12, 228), (2, 12, 120), (8, 24, 456), (8, 0, 432), (4, 0, 216)])
def test_algorithmic_bytes_per_cell(elem, force, want):
    """27 populations read and written once, plus the force field read once."""
    assert bench.bytes_per_cell(elem, force) == want


def test_counter_summaries_match_only_their_own_sources(tmp_path, monkeypatch):
    key = "k_step<f32,periodic,les,force_field>@256^3"
    entry = {"bytes_per_launch": 1000, "cells": 10, "bytes_per_cell": 100.0, "source_hash": bench.kernel_hash()}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps({key: entry}))
    for p in bench.KERNEL_SOURCES:   # the same sources under the temporary root
        os.makedirs(os.path.dirname(tmp_path / p), exist_ok=True)
        with open(os.path.join(ROOT, p), "rb") as src, open(tmp_path / p, "wb") as dst:
            dst.write(src.read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic(key) == {"bytes_per_launch": 1000, "cells_per_launch": 10, "bytes_per_cell": 100.0}
    assert bench.measured_traffic("k_step<f64,periodic,les,force_field>@512^3") is None
    with open(tmp_path / bench.KERNEL_SOURCES[1], "ab") as fh:   # any change to a kernel source
        fh.write(b"\n")
    assert bench.traffic_entry(key) is None and bench.measured_traffic(key) is None
