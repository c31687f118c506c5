"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite) as text.

Dispatches are grouped by kernel name and grid shape, so launches of one
kernel with different roles (e.g. probe and main-loop hashes) stay apart.

    python -m paper_1908_02461_amd.profsum RESULTS.db [--match atsfft] [--title ...]
"""
from __future__ import annotations

import argparse
import sqlite3
from collections import defaultdict


def summarize(db: str, match: str = "") -> list[dict]:
    c = sqlite3.connect(db)
    names = {r[0]: r[1] for r in c.execute("select id, kernel_name from rocpd_info_kernel_symbol")}
    groups = defaultdict(list)
    q = ("select kernel_id, start, end, grid_size_x, grid_size_y, grid_size_z, "
         "workgroup_size_x from rocpd_kernel_dispatch")
    for kid, s, e, gx, gy, gz, wx in c.execute(q):
        name = names.get(kid, str(kid))
        if match and match not in name:
            continue
        groups[(name, gx, gy, gz, wx)].append(e - s)
    rows = []
    for (name, gx, gy, gz, wx), d in groups.items():
        rows.append(dict(kernel=name, grid=(gx, gy, gz), block=wx, calls=len(d), total_us=sum(d) / 1e3,
                         avg_us=sum(d) / len(d) / 1e3, min_us=min(d) / 1e3, max_us=max(d) / 1e3))
    rows.sort(key=lambda r: -r["total_us"])
    return rows


def render(rows: list[dict], title: str = "") -> str:
    out = []
    if title:
        out.append(title)
    out.append(f"{'total_us':>11} {'calls':>6} {'avg_us':>10} {'min_us':>9} {'max_us':>9}  grid(threads)      kernel")
    for r in rows:
        g = "x".join(str(v) for v in r["grid"])
        out.append(f"{r['total_us']:11.1f} {r['calls']:6d} {r['avg_us']:10.2f} {r['min_us']:9.2f} {r['max_us']:9.2f}  "
                   f"{g:18s} {r['kernel'][:110]}")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--match", default="")
    ap.add_argument("--title", default="")
    a = ap.parse_args()
    print(render(summarize(a.db, a.match), a.title))


if __name__ == "__main__":
    main()
