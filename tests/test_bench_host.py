"""Host-side logic of the benchmark (no GPU): the per-kernel summaries and the
calibrated traffic computed from rocprofv3 counter databases, on small
synthetic databases with the same table layout."""

import json
import sqlite3

import pytest

import bench

COPY_KIB_FETCH = 4.0 * bench.COPY_FLOATS / 1024.0 / 2.0   # FETCH_SIZE reads half the bytes
COPY_KIB_WRITE = 4.0 * bench.COPY_FLOATS / 1024.0


def _db(path, counter, rows):
    """rows: (kernel name, grid, duration ns, counter value in KiB)."""
    c = sqlite3.connect(path)
    c.execute("create table counters_collection (kernel_name text, grid_size int, duration int, "
              "counter_name text, value real)")
    c.executemany("insert into counters_collection values (?,?,?,?,?)",
                  [(n, g, d, counter, v) for n, g, d, v in rows])
    c.commit()
    c.close()
    return str(path)


def _rows(copy_kib, fwd_kib, bwd_kib):
    finest, coarse = bench.FINEST_VOXELS, bench.FINEST_VOXELS // 8
    rows = []
    # copies: the finest-level velocity (the calibration), a 2x-level one and a
    # small one, all with one launch shape; the longest are the calibration
    rows += [("k_copy(float const*, float*, long long)", 4194304, 410000, copy_kib)] * 3
    rows += [("k_copy(float const*, float*, long long)", 4194304, 52000, copy_kib / 8)] * 2
    rows += [("k_copy(float const*, float*, long long)", 1260032, 7000, copy_kib / 64)] * 2
    # forward sweep: finest (long) and coarse (short) levels of one launch shape
    rows += [("void lddmm::k_forward<1, false, false, false>(lddmm::FwdArgs)", 262144, 206000,
              fwd_kib)] * 4
    rows += [("void lddmm::k_forward<1, false, false, false>(lddmm::FwdArgs)", 262144, 26000,
              fwd_kib / 8)] * 4
    # plane-marching forward: the finest level (long), a coarser level whose grid
    # is larger (short), and two trial launches of another shape at the finest level
    zm = "void lddmm::k_forward<1, false, false, false, true>(lddmm::FwdArgs)"
    rows += [(zm, 448512, 187000, fwd_kib)] * 5
    rows += [(zm, 450560, 22000, fwd_kib / 8)] * 6
    rows += [(zm, 897024, 185000, 1.5 * fwd_kib)] * 2
    # staged backward at the finest level only; a map-only step at the finest level
    # (60 % of the bytes, another profile class); a grid-stride body-force variant
    # that runs only on a coarser level (left out)
    rows += [("void lddmm::k_backward_staged<1, true, false>(lddmm::BwdArgs)", 737280, 205000,
              bwd_kib)] * 4
    rows += [("void lddmm::k_backward<1, true, true, false, false>(lddmm::BwdArgs)", 262144,
              41000, 0.6 * bwd_kib)] * 2
    rows += [("void lddmm::k_backward<1, true, false, true, false>(lddmm::BwdArgs)", 262144,
              29000, bwd_kib / 8)] * 6
    return rows


def test_traffic_is_calibrated_on_the_finest_copies(tmp_path):
    # counters that read the copy at half its bytes (fetch) and at all of them
    # (write): the kernels' figures come back at twice and once their values
    fwd_bytes, bwd_bytes = 61.0 * bench.FINEST_VOXELS, 50.0 * bench.FINEST_VOXELS
    fetch = _db(tmp_path / "f.db", "FETCH_SIZE",
                _rows(COPY_KIB_FETCH, fwd_bytes / 2 / 1024, bwd_bytes / 2 / 1024))
    write = _db(tmp_path / "w.db", "WRITE_SIZE",
                _rows(COPY_KIB_WRITE, 16.0 * bench.FINEST_VOXELS / 1024,
                      30.0 * bench.FINEST_VOXELS / 1024))
    out = tmp_path / "t.json"
    bench.compute_traffic(fetch, write, str(out))
    t = json.load(open(out))
    assert t["fetch_factor"] == pytest.approx(2.0) and t["write_factor"] == pytest.approx(1.0)
    assert t["source_sha"] == bench.library_sources_sha()
    k = t["kernels"]
    # the coarse launches and the trial shape left out: 4 grid-stride + 5 marching
    assert k["forward"]["launches"] == 9
    assert k["forward"]["fetch_bytes_per_voxel"] == pytest.approx(61.0)
    assert k["forward"]["write_bytes_per_voxel"] == pytest.approx(16.0)
    # the backward class is the body-force step with a map: the map-only step and the
    # coarse-level variant are left out
    assert k["backward"]["launches"] == 4
    assert k["backward"]["fetch_bytes_per_voxel"] == pytest.approx(50.0)
    assert k["backward"]["write_bytes_per_voxel"] == pytest.approx(30.0)
    assert k["forward"]["mean_us_under_counters"] == pytest.approx((4 * 206.0 + 5 * 187.0) / 9)


def test_missing_copy_is_an_error(tmp_path):
    rows = [r for r in _rows(1.0, 1.0, 1.0) if not r[0].startswith("k_copy")]
    f = _db(tmp_path / "f.db", "FETCH_SIZE", rows)
    w = _db(tmp_path / "w.db", "WRITE_SIZE", rows)
    with pytest.raises(SystemExit):
        bench.compute_traffic(f, w, str(tmp_path / "t.json"))


def test_summary_names_and_levels(tmp_path):
    db = _db(tmp_path / "f.db", "FETCH_SIZE", _rows(1.0, 2.0, 3.0))
    out = bench.summarize_profile(db, str(tmp_path / "s.txt"), "cmd")
    names = {k[0] for k in out}
    assert "void k_forward<1, false, false, false>" in names      # namespaces and args dropped
    assert "k_copy" in names
    tags = {k[2] for k in out if k[0] == "void k_forward<1, false, false, false>"}
    assert tags == {" (short)", " (long)"}                         # two levels split
    tags = {k[2] for k in out if k[0] == "void k_forward<1, false, false, false, true>"}
    assert tags == {""}                                            # one level per shape
    assert open(tmp_path / "s.txt").readline().startswith("# rocprofv3 summary of: cmd")


def test_last_accepted_D_skips_rejected_and_stopped_rows():
    import numpy as np
    nan = float("nan")
    tr = np.array([[3.0, 0.0, 3.0, 0.1, nan, nan, 1.0, 3.0],
                   [2.0, 0.5, 1.5, 0.1, 0.9, nan, 1.0, 2.0],
                   [2.5, 0.6, 1.9, 0.1, 0.9, nan, 0.0, 2.0],     # rejected trial
                   [nan, nan, nan, 0.05, 0.9, nan, 0.0, 2.0]])   # stopped
    assert bench.last_accepted_D(tr) == 1.5


def test_kernel_names_follow_the_launch_choice():
    assert bench.kernel_name("backward", {"staged_min_blocks": 2048}, False) == \
        "k_backward_staged<1, true, false>"
    assert bench.kernel_name("backward", {"staged_min_blocks": 1 << 30}, True) == \
        "k_backward<1, true, false, true, true>"
    assert bench.kernel_name("forward", {"fwd_tiles": 3584}, False) == \
        "k_forward<1, false, false, false, true>"
    assert bench.kernel_name("forward", {"fwd_tiles": 0}, False) == \
        "k_forward<1, false, false, false, false>"
