"""Summaries of rocprofv3 output.

Kernel trace (rocpd SQLite database, `--kernel-trace`): per kernel and launch
grid, the number of dispatches, total and average duration.
Counters (`--pmc ... --output-format csv`, the counter_collection CSV): per
kernel and counter, the number of dispatches and the average value.

Usage: python -m paper_0711_0999_amd.profsummary <results.db> [N]
       python -m paper_0711_0999_amd.profsummary <counter_collection.csv> [N]"""
import csv
import sqlite3
import sys


def summarize(db, top=15):
    con = sqlite3.connect(db)
    rows = con.execute(
        "select name, grid_x, count(*), sum(duration), avg(duration) "
        "from kernels group by name, grid_x order by sum(duration) desc").fetchall()
    total = sum(r[3] for r in rows) or 1.0
    out = ["kernel | grid_x (work-items) | calls | total ms | avg ms | % of GPU time",
           "---|---|---|---|---|---"]
    for name, gx, n, tot, avg in rows[:top]:
        short = name.split("(")[0].replace("void ", "")
        out.append(f"{short} | {gx} | {n} | {tot / 1e6:.3f} | {avg / 1e6:.4f} | "
                   f"{100.0 * tot / total:.2f}")
    return "\n".join(out)


def _col(header, *names):
    low = [h.strip().lower() for h in header]
    for n in names:
        if n in low:
            return low.index(n)
    raise KeyError(f"none of {names} in {header}")


def summarize_counters(path, top=15):
    with open(path, newline="") as f:
        rd = csv.reader(f)
        header = next(rd)
        ik = _col(header, "kernel_name", "kernel-name", "name")
        ic = _col(header, "counter_name", "counter-name")
        iv = _col(header, "counter_value", "counter-value", "value")
        ig = None
        for n in ("grid_size", "grid_size_x", "grid-size"):
            try:
                ig = _col(header, n)
                break
            except KeyError:
                pass
        acc = {}
        for r in rd:
            key = (r[ik].split("(")[0].replace("void ", ""),
                   r[ig] if ig is not None else "", r[ic])
            s = acc.setdefault(key, [0, 0.0])
            s[0] += 1
            s[1] += float(r[iv])
    rows = sorted(acc.items(), key=lambda kv: -kv[1][1])
    out = ["kernel | grid | counter | dispatches | average per dispatch | total",
           "---|---|---|---|---|---"]
    for (name, grid, ctr), (n, tot) in rows[:top]:
        out.append(f"{name} | {grid} | {ctr} | {n} | {tot / n:.1f} | {tot:.1f}")
    return "\n".join(out)


if __name__ == "__main__":
    top = int(sys.argv[2]) if len(sys.argv) > 2 else 15
    if sys.argv[1].endswith(".csv"):
        print(summarize_counters(sys.argv[1], top))
    else:
        print(summarize(sys.argv[1], top))
