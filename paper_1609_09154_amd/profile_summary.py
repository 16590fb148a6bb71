"""Writes a short Markdown summary of a rocprofv3 kernel-trace database.

    python -m paper_1609_09154_amd.profile_summary DB OUT.md "TITLE" "COMMAND"

Reads the `top_kernels` view (name, calls, total and average duration in
microseconds) and the per-dispatch `kernels` view of a rocpd SQLite file.
"""
import sqlite3
import sys


def summarize(db, out, title, command, top=14):
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
        for pat in ("gemm_tn_kernel", "gemm_nn_kernel"):
            d = [r[0] / 1000.0 for r in cur.execute(
                "select (end - start) from kernels where name like ? order by start", ("%" + pat + "%",))]
            big = [x for x in d if x > 1000.0]
            small = [x for x in d if x <= 1000.0]
            if d:
                f.write("\n`%s`: %d launches; %d above 1 ms averaging %.1f us (the large products), "
                        "%d at or below averaging %.1f us (Grams and small launches).\n"
                        % (pat, len(d), len(big), sum(big) / max(len(big), 1), len(small),
                           sum(small) / max(len(small), 1)))


if __name__ == "__main__":
    summarize(*sys.argv[1:5])
