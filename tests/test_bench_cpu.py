"""Host-side checks of bench.py: the one-GPU contract, the algorithmic byte
counts it prices the roofline with, and the traffic record it reads."""

import json
import os
import re
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_csr_halfsweep_bytes_count_the_27_point_pattern():
    n = 128
    avg, per_colour = bench.csr_halfsweep_bytes(n)
    # both colours together hold every nonzero of the 27-point pattern once:
    # nnz = (3n - 5)^3 (3 entries per direction at interior nodes, 2 next
    # to the boundary)
    NI = (n - 1) ** 3
    nnz = (3 * n - 5) ** 3
    rows = NI
    total = 12 * nnz + 4 * (rows + 2) + 4 * rows + 16 * rows + 2 * 8 * NI
    assert sum(per_colour) == total
    assert avg == total / 2


def test_stencil_halfsweep_bytes():
    n = 256
    NI = (n - 1) ** 3
    assert bench.stencil_halfsweep_bytes(n, 8) == 8 * NI + 8 * NI
    assert bench.stencil_halfsweep_bytes(n, 4, kappa=True) == 4 * NI + 4 * NI + 4 * n ** 3


def test_traffic_record_is_checked_against_the_kernel_sources(tmp_path, monkeypatch):
    text = open(os.path.join(ROOT, "profiles", "traffic.md")).read()
    rec = json.loads(re.search(r"```json\n(.*?)```", text, re.S).group(1))
    assert "poisson3d_128_csr_rbgs" in rec
    for name, r in rec.items():
        got = bench.measured_traffic(name)
        # either the sources are unchanged (the recorded bytes come back) or
        # they changed since the counters were taken (None)
        assert got in (None, r["bytes_per_launch"])
        assert np.isclose(r["bytes_per_launch"],
                          1024 * (r["fetch_kib"] * r["fetch_scale"] + r["write_kib"] * r["write_scale"]),
                          rtol=1e-4)
    # a copy of the tree whose kernel source differs reports None
    fake = tmp_path / "repo"
    (fake / "profiles").mkdir(parents=True)
    (fake / "profiles" / "traffic.md").write_text(text)
    for src in rec["poisson3d_128_csr_rbgs"]["sources"]:
        p = fake / src
        p.parent.mkdir(parents=True, exist_ok=True)
        p.write_text("// changed\n")
    monkeypatch.setattr(bench, "ROOT", str(fake))
    assert bench.measured_traffic("poisson3d_128_csr_rbgs") is None
    assert bench.measured_traffic("no_such_workload") is None
