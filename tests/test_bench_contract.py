"""bench.py on the host: the one-GPU rule, the traffic record and the algorithmic byte count."""
import os
import subprocess
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_is_reported_only_for_the_profiled_sources_and_shape(tmp_path, monkeypatch):
    import shutil
    root = tmp_path / "repo"
    (root / "profiles").mkdir(parents=True)
    (root / "paper_2104_11404_amd" / "csrc").mkdir(parents=True)
    for f in ("rom.hip", "internal.hpp"):
        shutil.copy(os.path.join(ROOT, "paper_2104_11404_amd", "csrc", f), root / "paper_2104_11404_amd" / "csrc" / f)
    import hashlib
    h = hashlib.sha1()
    for f in ("rom.hip", "internal.hpp"):
        h.update((root / "paper_2104_11404_amd" / "csrc" / f).read_bytes())
    prof = root / "profiles" / "rom_step_kernel_sedov2d_64x64_traffic.md"
    prof.write_text(f"machine-readable: traffic_bytes_per_launch=123456 source_sha1={h.hexdigest()} workgroups=20\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.measured_traffic(20) == 123456.0
    assert bench.measured_traffic(24) is None  # another launch shape: other exchange traffic
    with open(root / "paper_2104_11404_amd" / "csrc" / "rom.hip", "a") as fh:
        fh.write("// changed\n")
    assert bench.measured_traffic(20) is None


def test_every_headline_form_with_traffic_names_a_committed_counter_summary():
    import re
    for form, name in bench.HEADLINE_TRAFFIC.items():
        text = open(os.path.join(ROOT, "profiles", name)).read()
        m = re.search(r"traffic_bytes_per_launch=(\d+) source_sha1=([0-9a-f]{40}) workgroups=(\d+)", text)
        assert m, form
        assert int(m.group(1)) > 0 and int(m.group(3)) >= 1
        # the command that made it runs the same form
        assert f"--headline-form {form}" in text, form


def test_rom_step_bytes_counts_tiles_offsets_and_operators():
    nx, nv, ne, ns1, ns2 = 3, 5, 4, 10, 8
    wd = {"phi": [torch.zeros(nx, 7), torch.zeros(nv, 7), torch.zeros(ne, 7)],
          "z1": torch.zeros(ns1), "z2": torch.zeros(ns2)}
    n_el, n_own = 6, 2
    got = bench.rom_step_bytes(None, [(wd, n_el, n_own)])
    nkd, nt = 18, 4
    per_stage = 8 * (n_el * (nkd * (nx + nv) + nt * ne + 2 * nkd + nt) + n_own * nkd * nv + nv * ns1 + ne * ns2
                     + nx * nv)
    assert got == [2 * per_stage]
