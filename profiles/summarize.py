"""Print a per-kernel summary (count, total ms, average us) from a rocprofv3
results database (rocpd SQLite output of `rocprofv3 --kernel-trace --stats`)."""
import sqlite3
import sys


def main(db, top=25):
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), sum(end-start)/1e6, avg(end-start)/1e3 from kernels "
                       "group by name order by sum(end-start) desc").fetchall()
    tot = sum(r[2] for r in rows)
    print(f"{'kernel':70s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s} {'share':>6s}")
    for name, n, ms, us in rows[:top]:
        short = name.replace("ncl::(anonymous namespace)::", "").split("(")[0]
        print(f"{short:70s} {n:7d} {ms:10.3f} {us:10.2f} {100*ms/tot:5.1f}%")
    print(f"{'TOTAL':70s} {'':7s} {tot:10.3f}")


if __name__ == "__main__":
    main(sys.argv[1])
