"""The benchmark's accounting: the algorithmic operation and byte counts that
the roofline fractions divide by, the peak they are taken against, and the
rule that measured HBM traffic is reported only for the kernel source it was
measured on.  Host only."""
import json
import os

import pytest

import bench


def test_axis_operation_count_per_leaf_and_substep():
    # 3 axes x 64 pencils x (355 per field + 9 faces x (80 + 7 per species))
    # + 512 cells x 11 fields x (8, + 3 with U0)
    assert bench.ops_per_leaf_stage(11, True) == 1_010_432
    assert bench.ops_per_leaf_stage(11, False) == 1_010_432 - 512 * 11 * 3
    assert bench.ops_per_leaf_stage(6, True) == 3 * 64 * (355 * 6 + 9 * 80) + 512 * 6 * 11


def test_ghost_fill_bytes_per_leaf():
    # the 14^3 tile written and the leaf's own 8^3 cells read once, per field
    assert bench.fill_bytes_per_leaf(11, 8) == (14 * 14 * 14 + 8 * 8 * 8) * 11 * 8 == 286_528
    assert bench.fill_bytes_per_leaf(11, 4) * 2 == bench.fill_bytes_per_leaf(11, 8)


def _distinct_cell_lines():
    """(cell, line direction) pairs whose PPM the 9-point face quadrature
    reads, over every face of one 8^3 leaf: face point (pu, pv) on side
    sd of a face normal to D lies at offset p/2 from its cell, p the point
    vector; its value comes from the line along p or -p, whichever has its
    first non-zero component positive."""
    pairs = set()
    pts = [(-1, -1), (1, 1), (1, -1), (-1, 1), (0, -1), (0, 1), (-1, 0), (1, 0), (0, 0)]
    for D in range(3):
        for k in range(-1, 8):  # face between cells k and k+1 along D
            for a in range(8):
                for b in range(8):
                    for sd, kk in ((1, k), (-1, k + 1)):
                        for pu, pv in pts:
                            p = [0, 0, 0]
                            t = [0, 0, 0]
                            p[D], t[D] = sd, kk
                            u, v = [i for i in range(3) if i != D]
                            p[u], p[v] = pu, pv
                            t[u], t[v] = a, b
                            first = next(c for c in p if c != 0)
                            e = tuple(p) if first > 0 else tuple(-c for c in p)
                            pairs.add((tuple(t), e))
    return pairs


def test_3d_line_count_is_the_enumerated_set():
    assert len(_distinct_cell_lines()) == bench.LINES_PER_LEAF_3D == 10_112


def test_3d_operation_count():
    nf = 11
    per_face = 9 * (80 + 7 * (nf - 6)) + 11 * nf
    assert bench.ops_per_leaf_stage_3d(nf, True) == (
        10_112 * nf * 58 + 3 * 576 * per_face + 512 * nf * 11)
    assert bench.ops_per_leaf_stage_3d(11, True) == 8_510_976


def test_algorithmic_bytes_and_peaks():
    assert bench.hbm_bytes_per_leaf_stage(11, 8, True) == 512 * 11 * 8 * 3
    assert bench.hbm_bytes_per_leaf_stage(11, 4, False) == 512 * 11 * 4 * 2
    # 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz, one operation per lane and clock
    assert bench.ALU_PEAK == pytest.approx(256 * 4 * 16 * 2.4e9)
    assert bench.HBM_PEAK == pytest.approx(8e12)


def test_traffic_is_reported_only_for_the_measured_source(tmp_path, monkeypatch):
    digest = bench.source_digest()
    assert len(digest) == 64 and digest == bench.source_digest()
    good = tmp_path / "good.json"
    good.write_text(json.dumps({"traffic_bytes": 123.0, "source_sha256": digest}))
    monkeypatch.setattr(bench, "TRAFFIC_PATH", str(good))
    assert bench.measured_traffic() == 123.0
    stale = tmp_path / "stale.json"
    stale.write_text(json.dumps({"traffic_bytes": 123.0, "source_sha256": "0" * 64}))
    monkeypatch.setattr(bench, "TRAFFIC_PATH", str(stale))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_PATH", str(tmp_path / "missing.json"))
    assert bench.measured_traffic() is None


def test_source_digest_covers_every_kernel_source(tmp_path, monkeypatch):
    """Changing any source the substep kernel is built from changes the
    digest that gates the measured traffic."""
    import shutil
    pkg = os.path.join(os.path.dirname(bench.__file__), "paper_2210_06437_amd")
    root = tmp_path / "repo"
    (root / "paper_2210_06437_amd" / "csrc").mkdir(parents=True)
    (root / "include").mkdir()
    for name in bench.STEP_SOURCES:
        src = os.path.normpath(os.path.join(pkg, "csrc", name))
        dst = os.path.normpath(os.path.join(root, "paper_2210_06437_amd", "csrc", name))
        shutil.copyfile(src, dst)
    monkeypatch.setattr(bench, "KERNEL_DIR", str(root / "paper_2210_06437_amd" / "csrc"))
    base = bench.source_digest()
    assert base == bench.source_digest()
    monkeypatch.undo()
    assert base == bench.source_digest()  # the copy hashes like the tree
    for name in bench.STEP_SOURCES:
        path = os.path.normpath(os.path.join(root, "paper_2210_06437_amd", "csrc", name))
        data = open(path, "rb").read()
        with open(path, "ab") as f:
            f.write(b"\n// changed\n")
        monkeypatch.setattr(bench, "KERNEL_DIR", str(root / "paper_2210_06437_amd" / "csrc"))
        assert bench.source_digest() != base, name
        monkeypatch.undo()
        with open(path, "wb") as f:
            f.write(data)
