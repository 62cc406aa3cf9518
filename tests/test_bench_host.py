"""bench.py's host-side logic, no GPU: the one-GPU guard, the counter records
in profiles/ keyed on the current kernels' code, and the host-range summary
of a rocprofv3 marker database (a small synthetic one here)."""
import json
import os
import sqlite3
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_committed_counter_records_match_the_current_kernels():
    # the roofline's `traffic` and `counters` come from these records only when
    # they were taken on the kernels as they are now (comments aside)
    h = bench.kernel_source_hash()
    names = [n for n in os.listdir(os.path.join(ROOT, "profiles")) if n.startswith("counters_")]
    assert names
    for n in names:
        rec = json.load(open(os.path.join(ROOT, "profiles", n)))
        assert rec["kernel_source_sha256_16"] == h, n
        assert bench._profile_record(n) is not None, n


def test_kernel_source_hash_ignores_comments(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_2012_06925_amd", "csrc")
    fake = tmp_path / "paper_2012_06925_amd" / "csrc"
    fake.mkdir(parents=True)
    for name in bench.KERNEL_SOURCES:
        (fake / name).write_text(open(os.path.join(src, name)).read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    with open(fake / bench.KERNEL_SOURCES[0], "a") as f:
        f.write("// a comment line\n   \n")
    assert bench.kernel_source_hash() == h0
    with open(fake / bench.KERNEL_SOURCES[0], "a") as f:
        f.write("static int bench_hash_probe = 1;\n")
    assert bench.kernel_source_hash() != h0


def test_marker_summary_groups_ranges_by_message(tmp_path, capsys):
    db = tmp_path / "m.db"
    con = sqlite3.connect(db)
    con.execute("create table regions (category text, extdata text, start integer, end integer)")
    rows = [("MARKER_CORE_RANGE_API", {"message": "bldtt:traversal"}, 0, 4_000_000),
            ("MARKER_CORE_RANGE_API", {"message": "bldtt:traversal"}, 10_000_000, 16_000_000),
            ("MARKER_CORE_RANGE_API", {"message": "bldtt_compute"}, 0, 30_000_000),
            ("HIP_RUNTIME_API", {"message": "ignored"}, 0, 1)]
    con.executemany("insert into regions values (?, ?, ?, ?)", [(c, json.dumps(m), s, e) for c, m, s, e in rows])
    con.commit()
    con.close()
    bench.summarize_markers(str(db))
    out = capsys.readouterr().out.splitlines()
    assert out[0].startswith("| host range |")
    body = {l.split("|")[1].strip(): l for l in out[2:]}
    assert set(body) == {"`bldtt:traversal`", "`bldtt_compute`"}
    assert "| 2 | 5.000 | 4.000 | 6.000 |" in body["`bldtt:traversal`"]
    assert "| 1 | 30.000 |" in body["`bldtt_compute`"]
