"""Host logic of the profile summaries on a synthetic rocpd database: kernel names lose
namespace, return type and call arguments; the issue share is VALU instructions x
4 cycles over 1024 SIMDs x 2.4 GHz x the mean kernel-trace duration; the copy
calibration scales the traffic counters."""
import json
import sqlite3

import pytest

from paper_2204_14167_amd import rocprof_summary as rs


def _db(path, kernels, counters):
    c = sqlite3.connect(path)
    c.execute("create table kernels (name text, duration real)")
    c.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    c.executemany("insert into kernels values (?, ?)", kernels)
    c.executemany("insert into counters_collection values (?, ?, ?)", counters)
    c.commit()
    c.close()
    return str(path)


def test_short_names():
    assert rs._short("void discos::near_list_kernel<2>(discos::GridDev, int)") == "near_list_kernel<2>"
    assert rs._short("discos::spread_charge_kernel(discos::GridDev)") == "spread_charge_kernel"


def test_issue_share(tmp_path, capsys):
    name = "void discos::near_list_kernel<2>(discos::GridDev)"
    kt = _db(tmp_path / "kt.db", [(name, 200e3), (name, 300e3)], [])
    waves, valu = 16384.0, 16384.0 * 8000
    sq = _db(tmp_path / "sq.db", [], [(name, "SQ_WAVES", waves), (name, "SQ_INSTS_VALU", valu),
                                      (name, "SQ_INSTS_SALU", waves * 3000)])
    rs.main(["issue", sq, kt, "--command", "a", "--command", "b"])
    out = capsys.readouterr().out
    data = json.loads(out.split("```json", 1)[1].split("```", 1)[0])
    k = data["kernels"]["near_list_kernel<2>"]
    assert k["valu_per_wave"] == 8000.0
    assert k["valu_issue_share"] == pytest.approx(round(valu * 4 / (1024 * 2.4e9 * 250e-6), 3))
    assert data["source_sha256"] == rs.source_hashes()


def test_traffic_calibration(tmp_path, capsys):
    copy = "__amd_rocclr_copyBuffer"
    kern = "discos::interp_es_kernel(discos::GridDev)"
    f = _db(tmp_path / "f.db", [], [(copy, "FETCH_SIZE", 2.0 * (1 << 20)), (kern, "FETCH_SIZE", 1000.0)])
    w = _db(tmp_path / "w.db", [], [(copy, "WRITE_SIZE", 1 << 20), (kern, "WRITE_SIZE", 10.0)])
    rs.main(["traffic", f, w, "--command", "c"])
    data = json.loads(capsys.readouterr().out.split("```json", 1)[1].split("```", 1)[0])
    # the 1 GiB copy read 2 GiB of FETCH_SIZE (factor 1/2) and 1 GiB of WRITE_SIZE
    assert data["kernels"]["interp_es_kernel"]["hbm_bytes_per_launch"] == round(1000 * 1024 * 0.5 + 10 * 1024)


def test_source_check(tmp_path):
    """A profile entry holds for a kernel while the file defining it and every header are
    unchanged; edits elsewhere leave it valid."""
    (tmp_path / "a.h").write_text("#pragma once\n")
    (tmp_path / "k.hip").write_text("template <int R>\n__global__ void\n  foo_kernel(int x) {}\n")
    (tmp_path / "o.hip").write_text("__global__ void bar_kernel() {}\n")
    data = {"source_sha256": rs.source_hashes(tmp_path)}
    assert rs.kernel_files("foo_kernel<3>", tmp_path) == ["a.h", "k.hip"]
    assert rs.sources_unchanged(data, "foo_kernel<3>", tmp_path)
    (tmp_path / "o.hip").write_text("__global__ void bar_kernel() { }\n")
    assert rs.sources_unchanged(data, "foo_kernel<3>", tmp_path)
    assert not rs.sources_unchanged(data, "bar_kernel", tmp_path)
    (tmp_path / "a.h").write_text("#pragma once // x\n")
    assert not rs.sources_unchanged(data, "foo_kernel<3>", tmp_path)
    assert not rs.sources_unchanged(data, "missing_kernel", tmp_path)
    assert not rs.sources_unchanged({"source_sha256": "0" * 64}, "foo_kernel<3>", tmp_path)
