"""Short text summaries of rocprofv3 output (the files under profiles/).

  python -m paper_2604_21566_amd.rocprof_summary <results.db> "<command>" > out.txt
      per-kernel durations from a --kernel-trace --stats run
  python -m paper_2604_21566_amd.rocprof_summary launches <results.db> "<command>" > out.txt
      chained add/sub launches in dispatch order, each scan dispatch together with the
      status scan and fill pass that follow it (deferred launches), grouped into runs
      of consecutive launches of the same kernel and form
  python -m paper_2604_21566_amd.rocprof_summary pmc <counter_collection.csv> "<command>" > out.txt
      per-kernel mean of every counter of a --pmc run (one row per kernel and counter)
  python -m paper_2604_21566_amd.rocprof_summary traffic <fetch.csv> <write.csv> "<fetch cmd>" "<write cmd>" > out.txt
      HBM bytes per launch of the add/sub scan kernel on the batched workload
      (2^20 pairs x 64 limbs) from one FETCH_SIZE and one WRITE_SIZE --pmc run of
      `bench.py --calibrate`, each scaled by what the counter reads for the 512 MiB
      device-to-device copies that run makes
"""
import csv
import hashlib
import os
import re
import sqlite3
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
COPY_BYTES = 512 << 20
C2_PAIRS, C2_LIMBS = 1 << 20, 64


INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")


def kernel_source_hash() -> str:
    """Hash of the scan kernel's source file and the headers it includes: a counter
    summary is valid only for the source it was taken on."""
    h = hashlib.sha256()
    for path in (os.path.join(CSRC, "k_addsub.hip"), os.path.join(CSRC, "bn_internal.h"),
                 os.path.join(INCLUDE, "bn.h")):
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


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


def launches(db, cmd):
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end from kernels order by start").fetchall()
    groups = []  # [kernel, deferred?, main_us, scan_us, fill_us, start, end]
    for name, st, en in rows:
        n = short(name)
        if "k_flat_scan" in n and n.rstrip(">").split(",")[-2].strip() == "true":
            groups.append([n, False, (en - st) / 1e3, 0.0, 0.0, st, en])
        elif groups and ("k_defer_scan" in n or "k_defer_fill" in n):
            g = groups[-1]
            g[1] = True
            g[3 if "scan" in n else 4] += (en - st) / 1e3
            g[6] = en
    blocks = []  # consecutive launches of one kernel and form with similar duration
    for g in groups:
        b = blocks[-1] if blocks else None
        if b and b[0] == g[0] and b[1] == g[1] and abs(g[2] - b[2][-1][2]) < 0.25 * b[2][-1][2]:
            b[2].append(g)
        else:
            blocks.append([g[0], g[1], [g]])
    print(f"# command: {cmd}")
    print("# chained add/sub launches in dispatch order (rocprofv3 --kernel-trace); a deferred launch")
    print("# is the scan kernel + k_defer_scan + k_defer_fill; first to last is the first dispatch's")
    print("# start to the fill's end; microseconds, means over the block")
    print(f"{'block':>5s} {'kernel':44s} {'form':9s} {'launches':>8s} {'scan_kernel':>11s} {'status_scan':>11s} "
          f"{'fill':>8s} {'first_to_last':>13s}")
    for i, (name, deferred, gs) in enumerate(blocks):
        k = len(gs)
        m = lambda j: sum(g[j] for g in gs) / k
        span = sum((g[6] - g[5]) / 1e3 for g in gs) / k
        print(f"{i:5d} {name[:44]:44s} {'deferred' if deferred else 'waiting':9s} {k:8d} {m(2):11.1f} {m(3):11.1f} "
              f"{m(4):8.1f} {span:13.1f}")


def _counter_rows(path):
    with open(path, newline="") as fh:
        return [(r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])) for r in csv.DictReader(fh)]


def pmc(path, cmd):
    per = {}
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            k = (short(r["Kernel_Name"]), r["Counter_Name"])
            per.setdefault(k, []).append(float(r["Counter_Value"]))
    print(f"# command: {cmd}")
    print("# mean (min, max) over the kernel's dispatches of each counter, as rocprofv3 --pmc reports it")
    print(f"{'kernel':60s} {'counter':30s} {'dispatches':>10s} {'mean':>14s} {'min':>14s} {'max':>14s}")
    for (name, ctr), v in sorted(per.items()):
        print(f"{name[:60]:60s} {ctr:30s} {len(v):10d} {sum(v) / len(v):14.6g} {min(v):14.6g} {max(v):14.6g}")


def traffic(fetch_csv, write_csv, fetch_cmd, write_cmd):
    F, W = _counter_rows(fetch_csv), _counter_rows(write_csv)
    copy_kib = COPY_BYTES / 1024

    def split(rows):
        # the calibration copies are the three largest rocclr copy dispatches
        copies = sorted((v for n, g, v in rows if "copyBuffer" in n), reverse=True)[:3]
        scans = [v for n, g, v in rows if "k_flat_scan" in n]
        names = sorted({re.sub(r"\(anonymous namespace\)::", "", n).split("(")[0] for n, g, v in rows
                        if "k_flat_scan" in n})
        return copies, scans, names

    fc, fs, names = split(F)
    wc, ws, _ = split(W)
    if len(fc) < 3 or len(wc) < 3 or not fs or not ws:
        raise SystemExit("counter files lack the calibration copies or the scan dispatches")
    fcm, wcm = sum(fc) / len(fc), sum(wc) / len(wc)
    fscale, wscale = copy_kib / fcm, copy_kib / wcm
    fm, wm = sum(fs) / len(fs), sum(ws) / len(ws)
    fb, wb = fm * 1024 * fscale, wm * 1024 * wscale
    alg = C2_PAIRS * C2_LIMBS * 24 + C2_PAIRS * 8
    print("# HBM traffic of the add/sub scan kernel on the batched workload (2^20 pairs x 64 limbs)")
    print("# commands (run from the repository root on an MI355X host):")
    print(f"#   {fetch_cmd}")
    print(f"#   {write_cmd}")
    print("#   python -m paper_2604_21566_amd.rocprof_summary traffic <fetch csv> <write csv> ...")
    print("# Counter values are KiB per dispatch.  Calibration: --calibrate runs three plain")
    print("# device-to-device copies of 512 MiB (524288 KiB read and 524288 KiB written); the")
    print("# counters for those copies give the scale factors below.")
    print(f"copy_fetch_kib_measured = {fcm:.1f}")
    print(f"copy_write_kib_measured = {wcm:.1f}")
    print(f"fetch_scale = {fscale:.5f}")
    print(f"write_scale = {wscale:.5f}")
    print(f"scan_dispatches = {len(fs)} ({', '.join(names)})")
    print(f"scan_fetch_kib_measured = {fm:.1f}  (min {min(fs):.1f}, max {max(fs):.1f})")
    print(f"scan_write_kib_measured = {wm:.1f}  (min {min(ws):.1f}, max {max(ws):.1f})")
    print(f"scan_fetch_bytes = {fb:.4e}")
    print(f"scan_write_bytes = {wb:.4e}")
    print(f"algorithmic_bytes_per_launch = {alg:.4e}  (24 B per limb + 8 B per pair)")
    print(f"traffic_over_algorithmic = {(fb + wb) / alg:.4f}")
    print(f"traffic_bytes_per_launch = {fb + wb:.6e}")
    print(f"kernel_src_sha = {kernel_source_hash()}")


if __name__ == "__main__":
    if sys.argv[1] == "traffic":
        traffic(*sys.argv[2:6])
    elif sys.argv[1] == "launches":
        launches(sys.argv[2], sys.argv[3])
    elif sys.argv[1] == "pmc":
        pmc(sys.argv[2], sys.argv[3])
    else:
        main(sys.argv[1], sys.argv[2])
