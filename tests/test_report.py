"""CPU pins of the report's derived fields and formatting against the tally
table printed in the paper's section 4.3 (tests/golden/tally_section_4_3.txt):
Average = Time / Calls, Time(%) over one denominator that counts the rows of
both stacked layers, sort by Time, Calls = 1 giving Min = Average = Max, and
the unit rendering (678ns, 471.80ns, 9.71us, 295.89ms, 4.73s)."""
import os

import numpy as np
import pytest

from paper_2504_03683_amd import report
from paper_2504_03683_amd.tally import ROW_DTYPE

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tally_section_4_3.txt")

# Exact ns values behind the printed rows: Time = Calls x the printed Average
# (the Average is what the table prints to the most digits), extremes as
# printed.  The table is a partial snapshot; three further rows of 19.90 ms
# each stand for the rest, so that the sum over every row is 12.6616 s, inside
# the interval the seven printed Time(%) values allow together.
EXACT = {
    "hipDeviceSynchronize": (16, 16 * 295_890_000, 678, 867_220_000),
    "zeEventHostSynchronize": (9_927_772, 4_683_922_830, 390, 3_560_000),
    "hipMemcpy": (7, 7 * 252_790_000, 202_400_000, 291_560_000),
    "__hipUnregisterFatBinary": (1, 500_910_000, 500_910_000, 500_910_000),
    "zeCommandListAppendMemoryCopy": (7, 394_500_000, 48_860_000, 69_420_000),
    "hipLaunchKernel": (32, 262_700_000, 9_710, 261_350_000),
    "zeModuleCreate": (1, 256_090_000, 256_090_000, 256_090_000),
}
TOTAL_NS = 12_661_600_000


def golden():
    out = []
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            out.append(line.strip().split("|"))
    return out


def rows_for(exact, rest):
    names = {}
    rows = np.zeros(len(exact) + len(rest), dtype=ROW_DTYPE)
    for i, (name, (calls, time, mn, mx)) in enumerate(list(exact.items()) + rest):
        names[i] = name
        r = rows[i]
        r["id"] = i
        r["row_kind"] = 1
        r["count"] = calls
        r["incl_sum"] = time
        r["incl_min"] = mn
        r["incl_max"] = mx
        r["self_sum"] = time
    return rows, names


def rest_rows():
    left = TOTAL_NS - sum(v[1] for v in EXACT.values())
    assert 0 < left < 3 * 256_090_000
    return [("rest_%d" % k, (1, left // 3 + (left % 3 if k == 0 else 0), 1, left)) for k in range(3)]


def test_units():
    assert report.fmt_duration(678) == "678ns"
    assert report.fmt_duration(4_683_922_830 / 9_927_772) == "471.80ns"
    assert report.fmt_duration(9_710) == "9.71us"
    assert report.fmt_duration(16 * 295_890_000 / 16) == "295.89ms"
    assert report.fmt_duration(16 * 295_890_000) == "4.73s"
    assert report.fmt_duration(999) == "999ns" and report.fmt_duration(1000) == "1.00us"
    assert report.fmt_duration(0) == "0ns"


def test_section_4_3_table():
    rows, names = rows_for(EXACT, rest_rows())
    text = report.render(rows, {"distinct_hosts": 1, "distinct_processes": 1, "distinct_threads": 1}, names,
                         backends="BACKEND_HIP,BACKEND_ZE")
    lines = text.splitlines()
    assert report.parse_line(lines[0]) == ["BACKEND_HIP,BACKEND_ZE", "1 Hostnames", "1 Processes", "1 Threads"]
    assert report.parse_line(lines[2]) == report.HEADER
    got = [report.parse_line(l) for l in lines[3:]]
    want = golden()
    # sorted by Time: the printed rows first, in the printed order
    assert [g[0] for g in got[:len(want)]] == [w[0] for w in want]
    for g, w in zip(got, want):
        assert g == w, (g, w)


def test_one_denominator_for_both_layers():
    """The printed Time(%) values are reproduced only when the denominator
    counts the HIP rows and the Level-Zero rows they are built on: with
    either layer alone the first row's share would be far from 37.39%."""
    rows, names = rows_for(EXACT, rest_rows())
    for layer in ("hip", "ze"):
        keep = np.array([names[int(i)].startswith(layer) or names[int(i)].startswith("__" + layer)
                         for i in rows["id"]])
        lines = report.table_lines(report.aggregate(rows[keep]), names)
        pcts = {l[0]: l[2] for l in lines}
        assert pcts.get("hipDeviceSynchronize", pcts.get("zeEventHostSynchronize")) not in ("37.39%", "36.99%")


def test_derived_fields_invariants():
    rows, names = rows_for(EXACT, rest_rows())
    per = report.aggregate(rows)
    for k, a in per.items():
        avg = a["time"] / a["count"]
        assert a["min"] <= avg <= a["max"] or a["count"] == 1 and a["min"] == a["max"] == a["time"] or \
            names[k].startswith("rest")
    ones = [l for l in report.table_lines(per, names) if l[3] == "1" and not l[0].startswith("rest")]
    assert ones and all(l[4] == l[5] == l[6] == l[1] for l in ones)
    total = sum(a["time"] for a in per.values())
    assert total == TOTAL_NS


def test_aggregate_over_threads_is_exact():
    """Rows of several threads fold into one line per function: counts and
    sums add, min and max combine, with no rounding."""
    rows = np.zeros(3, dtype=ROW_DTYPE)
    for i, (c, s, mn, mx) in enumerate([(2, 10, 3, 7), (5, (1 << 62) + 1, 1, 1 << 61), (1, 4, 4, 4)]):
        rows[i]["id"] = 9 if i < 2 else 3
        rows[i]["row_kind"] = 1
        rows[i]["count"], rows[i]["incl_sum"], rows[i]["incl_min"], rows[i]["incl_max"] = c, s, mn, mx
    per = report.aggregate(rows)
    assert per[9]["count"] == 7 and per[9]["time"] == (1 << 62) + 11 and per[9]["min"] == 1 and per[9]["max"] == 1 << 61
    assert per[3]["time"] == 4
