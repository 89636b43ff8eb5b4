"""Condense a rocprofv3 kernel-trace database into a short text summary
(kernel, calls, average and total duration), for the committed profiles."""
import re
import sqlite3
import sys


def summarize(db_path: str) -> str:
    db = sqlite3.connect(db_path)
    rows = db.execute("select name, count(*), avg(duration), sum(duration), min(duration), max(duration) "
                      "from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[3] for r in rows) or 1
    out = [f"{'kernel':<48} {'calls':>5} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'pct':>6}"]
    for name, n, avg, tot, mn, mx in rows:
        short = name.replace("vp::(anonymous namespace)::", "")
        short = re.sub(r"^void ", "", short)
        short = re.sub(r"\(.*", "", short)
        out.append(f"{short[:48]:<48} {n:>5} {avg / 1e3:>10.2f} {mn / 1e3:>10.2f} {mx / 1e3:>10.2f} "
                   f"{100.0 * tot / total:>6.1f}")
    return "\n".join(out)


if __name__ == "__main__":
    print(summarize(sys.argv[1]))
