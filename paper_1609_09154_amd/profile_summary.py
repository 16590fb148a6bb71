"""Writes a short Markdown summary of a rocprofv3 kernel-trace database.

    python -m paper_1609_09154_amd.profile_summary DB OUT.md "TITLE" "COMMAND" [PATTERNS]

PATTERNS: comma-separated kernel-name fragments whose dispatches are listed
split at 1 ms (default: the dense product kernels).

Reads the `top_kernels` view (name, calls, total and average duration in
microseconds) and the per-dispatch `kernels` view of a rocpd SQLite file.
"""
import sqlite3
import sys


def summarize(db, out, title, command, top=14, patterns=("gemm_tn_kernel", "gemm_nn_kernel")):
    con = sqlite3.connect(db)
    cur = con.cursor()
    rows = list(cur.execute("select name, total_calls, total_duration, average, percentage "
                            "from top_kernels limit %d" % top))
    with open(out, "w") as f:
        f.write("# %s\n\nCommand (repository root on the MI355X box, R = its path):\n\n" % title)
        f.write("    %s\n\n" % command)
        f.write("Summary of the `top_kernels` view of the rocpd database; durations in "
                "microseconds.\n\n| kernel | calls | total us | average us | % |\n|---|---|---|---|---|\n")
        for name, calls, tot, avg, pct in rows:
            f.write("| `%s` | %d | %.1f | %.1f | %.2f |\n"
                    % (name[:120].replace("|", "/"), calls, tot, avg, pct))
        # dispatches of the product kernels, split by duration (products vs Grams)
        for pat in patterns:
            d = [r[0] / 1000.0 for r in cur.execute(
                "select (end - start) from kernels where name like ? order by start", ("%" + pat + "%",))]
            big = [x for x in d if x > 1000.0]
            small = [x for x in d if x <= 1000.0]
            if d:
                f.write("\n`%s`: %d launches; %d above 1 ms averaging %.1f us, "
                        "%d at or below averaging %.1f us.\n"
                        % (pat, len(d), len(big), sum(big) / max(len(big), 1), len(small),
                           sum(small) / max(len(small), 1)))


def _per_dispatch(db, counter):
    """{dispatch_id: (kernel_name, duration_ns, value)} summed over instances."""
    con = sqlite3.connect(db)
    cur = con.cursor()
    out = {}
    for did, name, dur, val in cur.execute(
            "select dispatch_id, kernel_name, duration, value from counters_collection "
            "where counter_name = ?", (counter,)):
        n0, d0, v0 = out.get(did, (name, dur, 0.0))
        out[did] = (name, dur, v0 + float(val))
    return out


def traffic(fetch_db, write_db, out_json, kernel_pattern, src_hash, copy_bytes, command):
    """HBM bytes per launch of the product kernel from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads
    for a device copy of copy_bytes (the largest copy dispatch)."""
    import json

    res = {}
    for tag, db, ctr in (("fetch", fetch_db, "FETCH_SIZE"), ("write", write_db, "WRITE_SIZE")):
        d = _per_dispatch(db, ctr)
        copies = [v for (nm, du, v) in d.values() if "rocclr_copyBuffer" in nm]
        prods = [v for (nm, du, v) in d.values() if kernel_pattern in nm and du > 1e6]
        cal = max(copies)
        factor = (copy_bytes / 1024.0) / cal
        res[tag] = dict(counter=ctr, copy_kib=cal, factor=factor, launches=len(prods),
                        kib_per_launch_raw=sum(prods) / max(len(prods), 1),
                        bytes_per_launch=factor * 1024.0 * sum(prods) / max(len(prods), 1))
    total = res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]
    rec = {"kernel": kernel_pattern, "kernel_source_hash": src_hash,
           "hbm_bytes_per_launch": total, "fetch": res["fetch"], "write": res["write"],
           "copy_calibration_bytes": copy_bytes, "command": command}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


if __name__ == "__main__":
    if sys.argv[1] == "traffic":
        print(traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6],
                      int(sys.argv[7]), sys.argv[8]))
    else:
        pats = tuple(sys.argv[5].split(",")) if len(sys.argv) > 5 else ("gemm_tn_kernel",
                                                                         "gemm_nn_kernel")
        summarize(*sys.argv[1:5], patterns=pats)
