"""Summaries of rocprofv3 output for the PDHG kernels (text for profiles/).

    python -m paper_2305_03945_amd.profsum trace <dir> <prefix>
    python -m paper_2305_03945_amd.profsum traffic <fetch_dir> <write_dir> <prefix> <copy_bytes>

``trace`` reads ``<prefix>_kernel_trace.csv`` of a ``--kernel-trace --stats`` run
and prints a per-kernel table.  Launches that found their slot finished return
at once (the host enqueues iterations speculatively); the "working" columns
keep only launches longer than half the kernel's median duration.  The mixed
row pass (last template argument 5) makes either the FP32 inner iteration or,
once an inner loop has stopped, the FP64 outer update: its launches above 1.6x
the median (duration, or counter value) are listed apart as ``<kernel>:outer``.

``counters`` reads the ``<prefix>_counter_collection.csv`` of one ``--pmc`` run
and prints, per kernel, the average of every listed counter over the working
dispatches, chosen (and the mixed row pass's outer updates split off) by the
first listed counter, e.g. SQ_WAVE_CYCLES: a launch that found its slot finished
has all its waves exit at once.

    python -m paper_2305_03945_amd.profsum counters <dir> <prefix> <counter> [<counter> ...]

``traffic`` reads the ``<prefix>_counter_collection.csv`` of two ``--pmc`` runs
(FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) and scales both by what the same
counter reads for the calibration copy (``bench.py --calib-copy-mb``: a float32
negation of known size, ``copy_bytes`` read and as many written), then prints
HBM bytes per working launch of every kernel and a JSON line with the figures.
"""
import csv
import hashlib
import json
import os
import re
import statistics
import sys

CALIB_KERNEL = "neg_kernel"


def short_name(full):
    m = re.match(r"void rdk::(\w+)<([^>]*)>", full)
    if m:
        return "%s<%s>" % (m.group(1), m.group(2).replace(" ", ""))
    if CALIB_KERNEL in full:
        return "calib_copy(neg)"
    return full.split("(")[0][:60]


def _working(values):
    med = statistics.median(values)
    return [v for v in values if v >= 0.5 * med]


MIXED_ROW = re.compile(r"row_forward<.*,5>$")


def _split_outer(by):
    """Move the outer-update launches of the mixed row pass to a key of their own.
    by: kernel -> {launch id: value}."""
    for k in [k for k in by if MIXED_ROW.search(k)]:
        med = statistics.median(by[k].values())
        outer = {i: v for i, v in by[k].items() if v > 1.6 * med}
        if outer:
            by[k + ":outer"] = outer
            by[k] = {i: v for i, v in by[k].items() if v <= 1.6 * med}
    return by


def trace_table(path):
    rows = list(csv.DictReader(open(path)))
    by = {}
    for i, r in enumerate(rows):
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        by.setdefault(short_name(r["Kernel_Name"]), {})[i] = d
    by = {k: list(v.values()) for k, v in _split_outer(by).items()}
    out = []
    for k, v in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        w = _working(v)
        out.append(dict(kernel=k, calls=len(v), avg_us=sum(v) / len(v), working_calls=len(w),
                        working_avg_us=sum(w) / len(w), min_us=min(v), max_us=max(v), total_us=sum(v)))
    return out


def counter_table(path, counter):
    rows = list(csv.DictReader(open(path)))
    by = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        by.setdefault(short_name(r["Kernel_Name"]), {}).setdefault(r["Dispatch_Id"], 0.0)
        by[short_name(r["Kernel_Name"])][r["Dispatch_Id"]] += float(r["Counter_Value"])
    by = _split_outer(by)
    out = {}
    for k, d in by.items():
        w = _working(list(d.values()))
        out[k] = dict(dispatches=len(d), working=len(w), kib=sum(w) / len(w))
    return out


def counters_table(path, counters):
    """kernel -> {counter: average over working dispatches, dispatches, working}; the
    working dispatches and the outer-update split follow counters[0]."""
    vals = {}
    for r in csv.DictReader(open(path)):
        c = r.get("Counter_Name")
        if c not in counters:
            continue
        d = vals.setdefault(short_name(r["Kernel_Name"]), {}).setdefault(r["Dispatch_Id"], {})
        d[c] = d.get(c, 0.0) + float(r["Counter_Value"])
    by = _split_outer({k: {i: d.get(counters[0], 0.0) for i, d in disp.items()} for k, disp in vals.items()})
    out = {}
    for k, sel in by.items():
        disp = vals[k[:-len(":outer")] if k.endswith(":outer") else k]
        med = statistics.median(sel.values())
        ids = [i for i, v in sel.items() if v >= 0.5 * med]
        row = {c: sum(disp[i].get(c, 0.0) for i in ids) / len(ids) for c in counters}
        row.update(dispatches=len(sel), working=len(ids))
        out[k] = row
    return out


def _code_only(text):
    """Source text without // comments and blank lines (comments do not change kernels)."""
    out = []
    for line in text.splitlines():
        code = re.sub(r"//.*$", "", line).rstrip()
        if code:
            out.append(code)
    return "\n".join(out)


def source_hash(root=None):
    """Hash of the HIP sources (code only): counter figures are valid only for these kernels."""
    root = root or os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(root)):
        if name.endswith((".h", ".hip")):
            h.update(name.encode())
            h.update(_code_only(open(os.path.join(root, name)).read()).encode())
    return h.hexdigest()[:16]


def main(argv):
    if argv[0] == "trace":
        d, prefix = argv[1], argv[2]
        t = trace_table(os.path.join(d, prefix + "_kernel_trace.csv"))
        print("| kernel | calls | avg us (all) | working calls | avg us (working) | min us | max us |")
        print("|---|---|---|---|---|---|---|")
        for r in t:
            print("| %s | %d | %.1f | %d | %.1f | %.1f | %.1f |" % (r["kernel"], r["calls"], r["avg_us"],
                                                               r["working_calls"], r["working_avg_us"],
                                                               r["min_us"], r["max_us"]))
        return
    if argv[0] == "counters":
        d, prefix, counters = argv[1], argv[2], argv[3:]
        t = counters_table(os.path.join(d, prefix + "_counter_collection.csv"), counters)
        print("| kernel | working dispatches | " + " | ".join(counters) + " |")
        print("|---|---|" + "---|" * len(counters))
        for k in sorted(t):
            print("| %s | %d | " % (k, t[k]["working"]) + " | ".join("%.0f" % t[k][c] for c in counters) + " |")
        print()
        print(json.dumps(dict(source_hash=source_hash(), kernels=t)))
        return
    if argv[0] == "traffic":
        fdir, wdir, prefix, copy_bytes = argv[1], argv[2], argv[3], float(argv[4])
        f = counter_table(os.path.join(fdir, prefix + "_counter_collection.csv"), "FETCH_SIZE")
        w = counter_table(os.path.join(wdir, prefix + "_counter_collection.csv"), "WRITE_SIZE")
        cal = "calib_copy(neg)"
        ffac = copy_bytes / (f[cal]["kib"] * 1024.0)
        wfac = copy_bytes / (w[cal]["kib"] * 1024.0)
        print("Calibration copy: %.0f bytes read and written; FETCH_SIZE reads %.0f KiB (factor %.4f), "
              "WRITE_SIZE reads %.0f KiB (factor %.4f)." % (copy_bytes, f[cal]["kib"], ffac, w[cal]["kib"], wfac))
        print()
        print("| kernel | FETCH KiB/launch | WRITE KiB/launch | scaled HBM MB/launch (read + write) |")
        print("|---|---|---|---|")
        res = {}
        for k in sorted(set(f) & set(w)):
            if k == cal:
                continue
            mb = (f[k]["kib"] * 1024.0 * ffac + w[k]["kib"] * 1024.0 * wfac) / 1e6
            res[k] = dict(fetch_kib=f[k]["kib"], write_kib=w[k]["kib"], hbm_bytes=mb * 1e6)
            print("| %s | %.0f | %.0f | %.2f |" % (k, f[k]["kib"], w[k]["kib"], mb))
        print()
        print(json.dumps(dict(source_hash=source_hash(), fetch_factor=ffac, write_factor=wfac, kernels=res)))
        return
    raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
