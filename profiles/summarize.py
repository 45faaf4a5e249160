"""Summaries of rocprofv3 result databases (rocpd SQLite output).

  python profiles/summarize.py kernels DB          per-kernel calls / total ms / avg us
  python profiles/summarize.py pmc DB COUNTER REGEX  per-dispatch counter values of the
                                                     kernels matching REGEX (mean, sum)
  python profiles/summarize.py split DB REGEX N       average duration of the kernels matching
                                                     REGEX over N equal consecutive phases of
                                                     the run (e.g. warmup / timed / evented)
"""
import re
import sqlite3
import sys


def kernels(db, top=25):
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), sum(end-start)/1e6, avg(end-start)/1e3 from kernels "
                       "group by name order by sum(end-start) desc").fetchall()
    tot = sum(r[2] for r in rows)
    print(f"{'kernel':70s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s} {'share':>6s}")
    for name, n, ms, us in rows[:top]:
        short = name.replace("ncl::(anonymous namespace)::", "").split("(")[0]
        print(f"{short:70s} {n:7d} {ms:10.3f} {us:10.2f} {100*ms/tot:5.1f}%")
    print(f"{'TOTAL':70s} {'':7s} {tot:10.3f}")


def pmc(db, counter, regex):
    con = sqlite3.connect(db)
    cols = [r[1] for r in con.execute("pragma table_info(counters_collection)").fetchall()]
    q = "select * from counters_collection"
    rows = con.execute(q).fetchall()
    idx = {c: i for i, c in enumerate(cols)}
    name_col = "kernel_name" if "kernel_name" in idx else "name"
    vals = {}
    for r in rows:
        nm = r[idx[name_col]]
        if not re.search(regex, nm):
            continue
        if r[idx["counter_name"]] != counter:
            continue
        key = nm.replace("ncl::(anonymous namespace)::", "").split("(")[0]
        vals.setdefault(key, []).append(float(r[idx["value"]]))
    for k, v in sorted(vals.items()):
        print(f"{k:60s} {counter} dispatches={len(v):6d} mean={sum(v)/len(v):14.1f} sum={sum(v):16.1f}")


def split(db, regex, nphase):
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end-start from kernels order by start").fetchall()
    by = {}
    for name, _, dur in rows:
        if re.search(regex, name):
            key = name.replace("ncl::(anonymous namespace)::", "").split("(")[0]
            by.setdefault(key, []).append(dur / 1e3)
    for k, v in sorted(by.items()):
        per = len(v) // nphase
        parts = [sum(v[i * per:(i + 1) * per]) / per for i in range(nphase)] if per else []
        print(f"{k:40s} calls={len(v):6d} avg_us per phase: " + " ".join(f"{x:8.2f}" for x in parts))


if __name__ == "__main__":
    if sys.argv[1] == "kernels":
        kernels(sys.argv[2])
    elif sys.argv[1] == "split":
        split(sys.argv[2], sys.argv[3], int(sys.argv[4]))
    elif sys.argv[1] == "pmc":
        pmc(sys.argv[2], sys.argv[3], sys.argv[4])
    else:
        kernels(sys.argv[1])
