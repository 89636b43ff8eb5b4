"""Condense a rocprofv3 --pmc database: per kernel, the mean of each counter
over its dispatches, plus derived VALU figures (for the committed profiles)."""
import re
import sqlite3
import sys
from collections import defaultdict


def summarize(db_path: str) -> str:
    db = sqlite3.connect(db_path)
    rows = db.execute("select kernel_name, dispatch_id, counter_name, sum(value), avg(duration) "
                      "from counters_collection group by kernel_name, dispatch_id, counter_name").fetchall()
    agg = defaultdict(lambda: defaultdict(list))
    dur = defaultdict(list)
    for kname, did, cname, val, d in rows:
        short = re.sub(r"\(.*", "", kname.replace("vp::(anonymous namespace)::", "").replace("void ", ""))
        agg[short][cname].append(val)
        dur[short].append(d)
    out = []
    for k, cs in agg.items():
        out.append(f"{k}  ({len(next(iter(cs.values())))} dispatches)")
        m = {c: sum(v) / len(v) for c, v in cs.items()}
        for c in sorted(m):
            out.append(f"  {c:<24} {m[c]:>16.4g}")
        if "SQ_INSTS_VALU" in m and "SQ_WAVES" in m and m["SQ_WAVES"]:
            out.append(f"  VALU instr / wave        {m['SQ_INSTS_VALU'] / m['SQ_WAVES']:>16.1f}")
        if "SQ_ACTIVE_INST_VALU" in m and "SQ_BUSY_CYCLES" in m and m["SQ_BUSY_CYCLES"]:
            out.append(f"  ACTIVE_INST_VALU/BUSY    {m['SQ_ACTIVE_INST_VALU'] / m['SQ_BUSY_CYCLES']:>16.3f}")
    return "\n".join(out)


if __name__ == "__main__":
    print(summarize(sys.argv[1]))
