"""Host logic of bench.py (no GPU): the committed HBM-counter summaries are matched to the
kernel source and launch shape they were taken on, and the launch-shape codes name the
kernel instantiations the library builds."""
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _summary(tmp_path, precision, sha, entries):
    lines = ["# counters", "", f"- precision: `{precision}`", f"- kernel_source_sha256: `{sha}`"]
    for name, fetch, write in entries:
        lines += [f"- kernel: `{name}` (elimination)", f"- fetch_bytes_per_launch: `{fetch}`",
                  f"- write_bytes_per_launch: `{write}`"]
    p = tmp_path / "summary.md"
    p.write_text("\n".join(lines) + "\n")
    return str(p)


def test_measured_traffic_picks_the_entry_of_the_shape(tmp_path, monkeypatch):
    sha = bench.source_digest("eliminate")
    path = _summary(tmp_path, "mixed", sha, [("gemm_whole_kernel<2, 2, 3, 3, 16, true>", 100, 20),
                                             ("gemm_whole_kernel<4, 4, 3, 3, 32, false>", 300, 40)])
    _, start, fn = bench.COUNTERS["eliminate"]
    monkeypatch.setitem(bench.COUNTERS, "eliminate", (path, start, fn))
    assert bench.measured_traffic("eliminate", "mixed", "gemm_whole_kernel<2, 2, 3, 3, 16, true>") == 120.0
    assert bench.measured_traffic("eliminate", "mixed", "gemm_whole_kernel<4, 4, 3, 3, 32, false>") == 340.0
    # a shape that was not measured, another precision: no figure
    assert bench.measured_traffic("eliminate", "mixed", "gemm_whole_kernel<2, 4, 3, 3, 16, true>") is None
    assert bench.measured_traffic("eliminate", "fp64", "gemm_whole_kernel<2, 2, 3, 3, 16, true>") is None


def test_measured_traffic_rejects_another_source(tmp_path, monkeypatch):
    path = _summary(tmp_path, "mixed", "0" * 64, [("gemm_whole_kernel<2, 2, 3, 3, 16, true>", 100, 20)])
    _, start, fn = bench.COUNTERS["eliminate"]
    monkeypatch.setitem(bench.COUNTERS, "eliminate", (path, start, fn))
    assert bench.measured_traffic("eliminate", "mixed", "gemm_whole_kernel<2, 2, 3, 3, 16, true>") is None
    monkeypatch.setitem(bench.COUNTERS, "eliminate", (str(tmp_path / "missing.md"), start, fn))
    assert bench.measured_traffic("eliminate", "mixed", "gemm_whole_kernel<2, 2, 3, 3, 16, true>") is None


def test_whole_shape_names_match_the_kernel_table():
    """bench.WHOLE_SHAPES (the template arguments a shape code runs) agrees with the
    whole_shape table of the HIP source, field by field."""
    src = open(os.path.join(ROOT, "paper_2607_16044_amd", "csrc", "hdg.hip")).read()
    table = dict(re.findall(r"code == (\d{4}) \? WholeShape\{([^}]*)\}", src))
    assert sorted(int(c) for c in table) == sorted(bench.WHOLE_SHAPES)
    for code, args in table.items():
        want = [a.strip() for a in args.split(",")]
        got = [a.strip() for a in bench.WHOLE_SHAPES[int(code)].split(",")]
        assert got == want, (code, got, want)
        if len(want) == 7 and want[6] == "true":
            assert bench.gemm_kernel_name(int(code), "float") == f"gemm_bf3_kernel<{', '.join(want[:5])}>"
        else:
            assert bench.gemm_kernel_name(int(code), "float") == f"gemm_whole_kernel<{', '.join(want)}>"
