"""Host-side logic of bench.py (CPU): the one-GPU refusal, the algorithmic byte
counts behind the roofline, and the lookup of measured HBM traffic, which must
only be used while the committed counter summary matches the kernel sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_kernel_bytes_counts_every_datum_once():
    A = dict(nv_total=120, nv_real=100, ne_flux=330, nnz_v=1900, nnz_e=4400)
    nb = bench.kernel_bytes(A)
    # edge: ids (24 B) + geometry (48 B) + flux out (32 B) per flux edge, every state row once
    assert nb["edge"] == 330 * (24 + 48 + 32) + 120 * 32
    # vertex: pointers, c_O, w_n, out per real vertex; id + 2 weights per vertex entry,
    # id + weight per edge entry; state rows and flux rows once
    assert nb["vertex"] == 100 * (8 + 16 + 32 + 32) + 1900 * (4 + 16) + 4400 * (4 + 8) + 120 * 32 + 330 * 32
    blocks = dict(n_blocks=7, halo_rows=900, rows_max=300)
    nl = bench.kernel_bytes(A, blocks=blocks)
    # block variants: 16-bit local ids, plus per block 3 pointers and its row lists
    assert nl["vertex"] == nb["vertex"] - (1900 + 4400) * 2 + 7 * 12 + 900 * 4
    assert nl["edge"] == nb["edge"]
    # packed-id variants: a 12-byte record per real vertex and lane for the first
    # round's ids, 16-bit ids only for the entries past it
    npk = bench.kernel_bytes(A, blocks=blocks, packed=(5, 7))
    assert npk["vertex"] == nl["vertex"] - (1900 + 4400) * 2 + 100 * 8 * 12 + (5 + 7) * 2
    # FP32 storage halves the state rows and weights, never the FP64 flux rows
    n4 = bench.kernel_bytes(A, precision_bytes=4)
    assert n4["edge"] == 330 * (24 + 24 + 32) + 120 * 16


def test_blueprint_unit_count():
    """The roofline's per-vertex-stage bytes: 1,132 B for the vertex step with a
    19-vertex, 44-edge stencil and 3 flux edges per vertex (w_n in every stage),
    w_n's 32 B in two of three stages for a whole step, and 392 B for the edge step."""
    n = 1000
    A = dict(nv_total=n, nv_real=n, ne_flux=3 * n, nnz_v=19 * n, nnz_e=44 * n)
    assert bench.survey_bytes_per_vertex_stage(A, 8, wn_stages=3) == pytest.approx(1132.0)
    assert bench.survey_bytes_per_vertex_stage(A, 8, wn_stages=2) == pytest.approx(1132.0 - 32.0 / 3)
    assert bench.survey_edge_bytes_per_vertex_stage(A, 8) == pytest.approx(392.0)
    # stage-averaged w_n in the stored count as well
    A2 = dict(A, nv_total=n)
    assert bench.kernel_bytes(A2, wn_stages=2)["vertex"] == pytest.approx(bench.kernel_bytes(A2)["vertex"] - n * 32 / 3)


def test_entries_past_first_round():
    import numpy as np
    # three real vertices with 30, 10, 24 vertex entries and 50, 48, 60 edge entries, one ghost
    A = dict(nv_real=3, vptr=np.array([0, 30, 40, 64, 64]), eptr=np.array([0, 50, 98, 158, 158]))
    assert bench.entries_past_first_round(A) == (6, 2 + 12)


def test_every_variant_names_a_kernel():
    assert set(bench.EDGE_KERNELS) == {0, 1}
    assert set(bench.VERTEX_KERNELS) == set(range(6))
    assert set(bench.PACKED_VERTEX_VARIANTS) <= set(bench.BLOCK_VERTEX_VARIANTS) <= set(bench.VERTEX_KERNELS)
    assert all(k.startswith("k_") for k in list(bench.EDGE_KERNELS.values()) + list(bench.VERTEX_KERNELS.values()))


def test_traffic_lookup_follows_the_source_hash(tmp_path, monkeypatch):
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    with open(path) as fh:
        d = json.load(fh)
    kernel = next(iter(d["kernels"]))
    grid = next(iter(d["kernels"][kernel]))
    if d["source_hash"] == bench.source_hash():
        assert (bench.traffic_from_profiles(kernel, d["N"], d["reorder"], int(grid))
                == d["kernels"][kernel][grid]["bytes_per_launch"])
    # another workload size, vertex order or grid never borrows the measurement
    assert bench.traffic_from_profiles(kernel, d["N"] + 1, d["reorder"], int(grid)) is None
    assert bench.traffic_from_profiles(kernel, d["N"], (d["reorder"] + 1) % 3, int(grid)) is None
    assert bench.traffic_from_profiles(kernel, d["N"], d["reorder"], int(grid) + 256) is None
    # a summary taken on other sources is ignored
    fake_root = tmp_path
    (fake_root / "profiles").mkdir()
    d2 = dict(d, source_hash="0" * 16)
    (fake_root / "profiles" / "hbm_traffic.json").write_text(json.dumps(d2))
    monkeypatch.setattr(bench, "ROOT", str(fake_root))
    monkeypatch.setattr(bench, "source_hash", lambda: "f" * 16)
    assert bench.traffic_from_profiles(kernel, d["N"], d["reorder"], int(grid)) is None


def test_kernel_names_shorten_to_template_instances():
    assert bench.short_kernel_name("void fdu::k_edge_flux_lean<double, double>(double const*, int const*, "
                                   "double const*, double*, int, fdu::Scheme)") == "k_edge_flux_lean<double, double>"
    assert bench.short_kernel_name("fdu::k_cfl_final(double const*, int, double, double*)") == "k_cfl_final"
