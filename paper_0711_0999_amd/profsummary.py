"""Summarize a rocprofv3 kernel-trace database (rocpd SQLite output):
per kernel and launch grid, the number of dispatches, total and average
duration.  Usage: python -m paper_0711_0999_amd.profsummary <results.db> [N]"""
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


if __name__ == "__main__":
    print(summarize(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 15))
