"""The counter-traffic summarizer on hand-made rocprofv3 counter tables: the probe kernel's
reading sets the scale, a kernel's bytes per launch are the median of its dispatches, or
for a launch of n dispatches their mean times n."""
import csv

import pytest

from paper_1601_06274_amd import traffic


def _table(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value"])
        for name, v in rows:
            w.writerow([name, counter, v])


def _pair(tmp_path, fetch_rows, write_rows):
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _table(fp, "FETCH_SIZE", fetch_rows)
    _table(wp, "WRITE_SIZE", write_rows)
    return str(fp), str(wp)


def test_scale_and_median(tmp_path):
    probe = "void at::native::MulFunctor<float>"
    f, w = _pair(tmp_path, [(probe, 512.0), ("k_alpha", 100.0), ("k_alpha", 300.0), ("k_alpha", 200.0)],
                 [(probe, 1024.0), ("k_alpha", 50.0), ("k_alpha", 50.0), ("k_alpha", 70.0)])
    r = traffic.summarize(f, w, copy_bytes=1024.0 * 1024, kernel="k_alpha", sources="sweep")
    # the probe moves 1 MiB each way: 2048 B per fetch unit, 1024 B per write unit
    assert r["fetch_bytes_per_launch"] == pytest.approx(200.0 * 2048)
    assert r["write_bytes_per_launch"] == pytest.approx(50.0 * 1024)
    assert r["dispatches"] == [3, 3] and r["dispatches_per_launch"] == 1


def test_launch_of_two_dispatches(tmp_path):
    probe = "MulFunctor"
    f, w = _pair(tmp_path, [(probe, 1024.0), ("hier", 10.0), ("hier", 90.0), ("hier", 12.0), ("hier", 88.0)],
                 [(probe, 1024.0), ("hier", 1.0), ("hier", 9.0), ("hier", 1.0), ("hier", 9.0)])
    r = traffic.summarize(f, w, copy_bytes=1024.0 * 1024, kernel="hier", sources="hier", per_launch=2)
    assert r["fetch_bytes_per_launch"] == pytest.approx(100.0 * 1024)
    assert r["write_bytes_per_launch"] == pytest.approx(10.0 * 1024)
    with pytest.raises(ValueError):
        traffic.summarize(f, w, copy_bytes=1024.0 * 1024, kernel="hier", sources="hier", per_launch=3)
