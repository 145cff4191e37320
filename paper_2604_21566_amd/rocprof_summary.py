"""Turn a rocprofv3 results database into a short per-kernel text summary (the files
under profiles/).  Usage: python -m paper_2604_21566_amd.rocprof_summary <results.db> "<command>" > out.txt"""
import re
import sqlite3
import sys


def short(name: str) -> str:
    name = re.sub(r"\(anonymous namespace\)::", "", name)
    return name.split("(")[0]


def main(db, cmd):
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), sum(duration), avg(duration), min(duration), max(duration), "
                       "max(vgpr_count), max(accum_vgpr_count), max(lds_size), max(grid_x), max(workgroup_x) "
                       "from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows)
    print(f"# command: {cmd}")
    print("# durations in microseconds (rocprofv3 --kernel-trace --stats, kernel dispatch records)")
    print(f"{'kernel':70s} {'calls':>6s} {'total_us':>10s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} "
          f"{'pct':>6s} {'vgpr':>5s} {'agpr':>5s} {'lds':>6s} {'grid_x':>9s} {'wg':>4s}")
    for r in rows:
        name, n, tot, avg, mn, mx, vg, ag, lds, gx, wg = r
        print(f"{short(name)[:70]:70s} {n:6d} {tot/1e3:10.1f} {avg/1e3:9.2f} {mn/1e3:9.2f} {mx/1e3:9.2f} "
              f"{100*tot/total:6.2f} {vg:5d} {ag:5d} {lds:6d} {gx:9d} {wg:4d}")


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2])
