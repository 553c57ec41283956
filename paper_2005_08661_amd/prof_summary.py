"""Summaries of rocprofv3 output (CSV format) for the committed profiles.

  python -m paper_2005_08661_amd.prof_summary trace  <kt_dir> <out.md> <command...>
  python -m paper_2005_08661_amd.prof_summary counters <fetch_dir> <write_dir> <copy_fetch_dir>
         <copy_write_dir> <copy_bytes> <out.md> <out.json> <command...>

The counter summary scales FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by what
the same counters read for a plain device copy of known size, and records a
hash of the HIP sources' code (comments ignored) so that stale counters can be
recognised.
"""
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def _code_only(text):
    """C++ source without comments and blank or trailing whitespace (string and
    character literals kept as they are), so that the hash changes with the code
    the compiler sees and not with its commentary."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    lines = (ln.rstrip() for ln in "".join(out).split("\n"))
    return "\n".join(ln for ln in lines if ln)


def source_hash():
    """Hash of the HIP sources' code (comments and blank lines ignored)."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) + glob.glob(os.path.join(HERE, "csrc", "*.hpp")) +
                    glob.glob(os.path.join(HERE, "csrc", "*.inc"))):
        with open(p, encoding="utf-8") as fh:
            h.update(os.path.basename(p).encode())
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def _short(name):
    name = name.replace("void ", "")
    return name.split("(")[0]


def _one(pattern):
    got = sorted(glob.glob(pattern))
    if not got:
        raise SystemExit("no file matches %s" % pattern)
    return got[0]


def trace_summary(kt_dir, out_md, command):
    stats = _one(os.path.join(kt_dir, "*kernel_stats.csv"))
    rows = list(csv.DictReader(open(stats)))
    lines = ["# Kernel durations (rocprofv3 --kernel-trace --stats)", "",
             "Command: `%s`" % command, "", "Source hash: `%s`" % source_hash(), "",
             "| kernel | calls | avg (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append("| `%s` | %s | %.2f | %.2f | %.2f | %s%% |" % (
            _short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, r["Percentage"]))
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def _counter_avgs(d, counter):
    f = _one(os.path.join(d, "*counter_collection.csv"))
    acc = {}
    for r in csv.DictReader(open(f)):
        if r["Counter_Name"] != counter:
            continue
        acc.setdefault(_short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def counters_summary(fetch_dir, write_dir, cfetch_dir, cwrite_dir, copy_bytes, out_md, out_json, command):
    fetch = _counter_avgs(fetch_dir, "FETCH_SIZE")
    write = _counter_avgs(write_dir, "WRITE_SIZE")
    cf = _counter_avgs(cfetch_dir, "FETCH_SIZE")
    cw = _counter_avgs(cwrite_dir, "WRITE_SIZE")
    # the copy kernel is the one with the largest counter value
    ckf = max(cf, key=cf.get)
    ckw = max(cw, key=cw.get)
    f_factor = copy_bytes / (cf[ckf] * 1024.0)
    w_factor = copy_bytes / (cw[ckw] * 1024.0)
    lines = ["# HBM traffic per dispatch (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)", "",
             "Command: `%s`" % command, "", "Source hash: `%s`" % source_hash(), "",
             "Calibration: a device copy of %d bytes read %.1f KiB (FETCH_SIZE) and wrote %.1f KiB "
             "(WRITE_SIZE); scale factors %.4f (fetch) and %.4f (write) turn KiB into bytes." % (
                 copy_bytes, cf[ckf], cw[ckw], f_factor, w_factor), "",
             "| kernel | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | traffic (MB, scaled) |", "|---|---|---|---|"]
    out = {"source_hash": source_hash(), "copy_bytes": copy_bytes, "fetch_factor": f_factor,
           "write_factor": w_factor, "kernels": {}}
    for k in sorted(set(fetch) | set(write)):
        fv, wv = fetch.get(k, 0.0), write.get(k, 0.0)
        traffic = fv * 1024.0 * f_factor + wv * 1024.0 * w_factor
        out["kernels"][k] = {"fetch_kib": fv, "write_kib": wv, "traffic_bytes": traffic}
        lines.append("| `%s` | %.1f | %.1f | %.2f |" % (k, fv, wv, traffic / 1e6))
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(out_json, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace_summary(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif sys.argv[1] == "counters":
        counters_summary(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], int(sys.argv[6]), sys.argv[7],
                         sys.argv[8], " ".join(sys.argv[9:]))
    else:
        raise SystemExit(__doc__)
