"""Text report of a tally, in the layout of the paper's Tally view (section 4.3:
a header with the backends and the numbers of hosts, processes and threads,
then one line per function with Time, Time(%), Calls, Average, Min and Max,
sorted by Time).

Presentation only: the exact integer tallies come from the library
(`tally.Tally.read`); this module derives Average = Time / Calls and
Time(%) = Time / (sum of Time over every row of the table), which is the
reading the section 4.3 numbers fix (nested rows of two layers are both
counted in the same denominator), and formats durations with a unit.
"""
from __future__ import annotations

from typing import Dict, Iterable, List, Optional

import numpy as np

_UNITS = ((1e9, "s"), (1e6, "ms"), (1e3, "us"))


def fmt_duration(ns: float) -> str:
    """Duration in ns with the largest unit that keeps the value >= 1:
    two decimals for s, ms and us; whole numbers of ns print without
    decimals, fractional ones (averages) with two."""
    for scale, unit in _UNITS:
        if ns >= scale:
            return "%.2f%s" % (ns / scale, unit)
    if float(ns).is_integer():
        return "%dns" % int(ns)
    return "%.2fns" % ns


def fmt_percent(frac: float) -> str:
    return "%.2f%%" % (100.0 * frac)


def aggregate(rows: np.ndarray) -> Dict[int, dict]:
    """Rows (any scope, API rows only) folded per function id: counts and sums
    add, mins and maxes combine (exact integers)."""
    out: Dict[int, dict] = {}
    for r in rows:
        if int(r["row_kind"]) != 1 or int(r["count"]) == 0:
            continue
        k = int(r["id"])
        a = out.get(k)
        if a is None:
            out[k] = {"count": int(r["count"]), "time": int(r["incl_sum"]), "min": int(r["incl_min"]),
                      "max": int(r["incl_max"]), "self": int(r["self_sum"]), "bytes": int(r["bytes_sum"])}
        else:
            a["count"] += int(r["count"])
            a["time"] += int(r["incl_sum"])
            a["self"] += int(r["self_sum"])
            a["bytes"] += int(r["bytes_sum"])
            a["min"] = min(a["min"], int(r["incl_min"]))
            a["max"] = max(a["max"], int(r["incl_max"]))
    return out


def table_lines(per_fn: Dict[int, dict], names: Optional[Dict[int, str]] = None) -> List[List[str]]:
    """[Name, Time, Time(%), Calls, Average, Min, Max] cells, sorted by Time
    (descending; ties by name)."""
    names = names or {}
    total = sum(a["time"] for a in per_fn.values())
    items = sorted(per_fn.items(), key=lambda kv: (-kv[1]["time"], names.get(kv[0], "fn_%d" % kv[0])))
    out = []
    for k, a in items:
        out.append([names.get(k, "fn_%d" % k), fmt_duration(a["time"]),
                    fmt_percent(a["time"] / total if total else 0.0), "%d" % a["count"],
                    fmt_duration(a["time"] / a["count"]), fmt_duration(a["min"]), fmt_duration(a["max"])])
    return out


HEADER = ["Name", "Time", "Time(%)", "Calls", "Average", "Min", "Max"]


def render(rows: np.ndarray, stats: dict, names: Optional[Dict[int, str]] = None, backends: str = "",
           limit: Optional[int] = None) -> str:
    """The report of rows read from the library (e.g. the FN scope of one
    trace) and the read's stats."""
    lines = table_lines(aggregate(rows), names)
    if limit is not None:
        lines = lines[:limit]
    widths = [max([len(HEADER[c])] + [len(l[c]) for l in lines]) for c in range(len(HEADER))]

    def fmt(cells: Iterable[str]) -> str:
        return " | ".join(c.rjust(w) for c, w in zip(cells, widths)) + " |"

    head = "%s | %d Hostnames | %d Processes | %d Threads |" % (
        backends or "BACKEND", stats.get("distinct_hosts", 0), stats.get("distinct_processes", 0),
        stats.get("distinct_threads", 0))
    return "\n".join([head, "", fmt(HEADER)] + [fmt(l) for l in lines]) + "\n"


def parse_line(line: str) -> List[str]:
    """Cells of one rendered table line."""
    return [c.strip() for c in line.strip().rstrip("|").split("|")]
