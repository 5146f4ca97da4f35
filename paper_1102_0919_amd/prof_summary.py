"""Summarise a rocprofv3 kernel-trace database into a short markdown table.

    python -m paper_1102_0919_amd.prof_summary DB_OR_DIR --title T --cmd "C" [--kernel NAME ...] [--pmc]

Prints, for the whole run: calls, total and average duration of every kernel; then, for each kernel
named with --kernel (a substring of the full name, template arguments included), its launches grouped
by grid size, largest total time first.
With --pmc the database holds counter samples (rocprofv3 --pmc): their per-dispatch averages are
listed per kernel and grid size instead.
"""
from __future__ import annotations

import argparse
import glob
import os
import sqlite3


def _short(name: str) -> str:
    s = name.split("(")[0].replace("void ", "").replace("slamg::", "")
    return s.strip()


def _find_db(path: str) -> str:
    if os.path.isfile(path):
        return path
    dbs = sorted(glob.glob(os.path.join(path, "**", "*_results.db"), recursive=True))
    if not dbs:
        raise SystemExit(f"no rocprofv3 results database under {path}")
    return dbs[-1]


def kernel_table(con) -> list[str]:
    rows = list(con.execute("select name, count(*), sum(duration), avg(duration) from kernels group by name"))
    rows.sort(key=lambda r: -r[2])
    tot = sum(r[2] for r in rows)
    out = [f"Total kernel time: {tot / 1e6:.3f} ms over {sum(r[1] for r in rows)} dispatches", "",
           "| kernel | calls | total (ms) | average (us) | share |", "|---|---|---|---|---|"]
    for n, c, t, a in rows[:30]:
        out.append(f"| `{_short(n)}` | {c} | {t / 1e6:.3f} | {a / 1e3:.2f} | {100.0 * t / tot:.1f}% |")
    return out


def grid_table(con, kernel: str) -> list[str]:
    rows = list(con.execute(
        "select name, grid_x, count(*), sum(duration), avg(duration), min(duration), max(duration) from kernels "
        "where name like ? group by name, grid_x order by sum(duration) desc", (f"%{kernel}%",)))
    out = [f"Launches of `{kernel}` by launch shape (grid in threads), the 12 largest by total time:", "",
           "| instance | grid_x | calls | total (ms) | average (us) | min (us) | max (us) |",
           "|---|---|---|---|---|---|---|"]
    for n, g, c, t, a, lo, hi in rows[:12]:
        out.append(f"| `{_short(n)}` | {g} | {c} | {t / 1e6:.3f} | {a / 1e3:.2f} | {lo / 1e3:.2f} | {hi / 1e3:.2f} |")
    return out


def pmc_table(con, kernel: str | None) -> list[str]:
    q = ("select kernel_name, grid_size, counter_name, count(*), avg(value) from counters_collection ")
    args: tuple = ()
    if kernel:
        q += "where kernel_name like ? "
        args = (f"%{kernel}%",)
    q += "group by kernel_name, grid_size, counter_name order by grid_size desc"
    try:
        rows = list(con.execute(q, args))
    except sqlite3.Error as e:   # schema differences between rocprofv3 versions
        return [f"(counter table not readable: {e})"]
    title = f"`{kernel}`" if kernel else "all kernels"
    out = [f"Counters of {title} by grid size (threads):", "",
           "| kernel | grid | counter | dispatches | average per dispatch |", "|---|---|---|---|---|"]
    for n, g, cn, c, v in rows[:40]:
        out.append(f"| `{_short(n)}` | {g} | {cn} | {c} | {v:.1f} |")
    # all matching dispatches together
    tot: dict = {}
    for n, g, cn, c, v in rows:
        d, s_ = tot.get(cn, (0, 0.0))
        tot[cn] = (d + c, s_ + c * v)
    if tot:
        out += ["", "| counter | dispatches | average per dispatch (all shapes) |", "|---|---|---|"]
        for cn, (d, s_) in sorted(tot.items()):
            out.append(f"| {cn} | {d} | {s_ / d:.1f} |")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("path")
    ap.add_argument("--title", required=True)
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--kernel", action="append", default=[])
    ap.add_argument("--pmc", action="store_true")
    a = ap.parse_args(argv)
    con = sqlite3.connect(_find_db(a.path))
    lines = [f"# {a.title}", "", "Command (repository root, one MI355X):", "", "    " + a.cmd, ""]
    if a.pmc:
        for k in a.kernel or [None]:
            lines += pmc_table(con, k) + [""]
    else:
        lines += kernel_table(con) + [""]
        for k in a.kernel:
            lines += grid_table(con, k) + [""]
    print("\n".join(lines))


if __name__ == "__main__":
    main()
