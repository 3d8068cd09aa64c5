"""Per-kernel summary (calls, total, average, min, max, share, VGPR/SGPR/LDS) of a
rocprofv3 --kernel-trace database (results.db written by rocprofv3 in ROCm 7)."""
import re
import sqlite3
import sys


def main(path):
    cur = sqlite3.connect(path).cursor()
    rows = cur.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration), "
        "max(vgpr_count), max(sgpr_count), max(lds_size) from kernels group by name "
        "order by sum(duration) desc").fetchall()
    tot = sum(r[2] for r in rows)
    print(f"| kernel | calls | total ms | avg us | min us | max us | % | VGPR | SGPR | LDS B |")
    print("|---|---|---|---|---|---|---|---|---|---|")
    for n, c, s, a, mn, mx, v, sg, lds in rows:
        m = re.search(r"(k_[a-z0-9_]+)", n)
        short = m.group(1) if m else n.split("(")[0][-40:]
        print(f"| {short} | {c} | {s / 1e6:.3f} | {a / 1e3:.2f} | {mn / 1e3:.2f} | {mx / 1e3:.2f} | "
              f"{100 * s / tot:.2f} | {v} | {sg} | {lds} |")


if __name__ == "__main__":
    main(sys.argv[1])
