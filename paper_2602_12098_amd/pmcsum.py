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


def _per_dispatch(db_path: str, regex: str):
    db = sqlite3.connect(db_path)
    rows = db.execute("select kernel_name, dispatch_id, counter_name, sum(value), avg(duration) "
                      "from counters_collection group by kernel_name, dispatch_id, counter_name").fetchall()
    per = defaultdict(dict)
    for kname, did, cname, val, d in rows:
        if re.search(regex, kname):
            per[did][cname] = val
            per[did]["duration_ns"] = d
    if not per:
        raise SystemExit(f"no dispatch of /{regex}/ in {db_path}")
    return per


def clocks_per_valu(db_path: str, regex: str):
    """(shader clock in GHz, SIMD clocks per VALU wave-instruction, VALU
    instructions, dispatches, duration in s) of one kernel from a run with
    SQ_INSTS_VALU and GRBM_GUI_ACTIVE: the clock is GRBM_GUI_ACTIVE (summed
    over the 8 XCDs) / 8 over the dispatch's duration; the clocks per
    instruction are 1024 SIMDs x those cycles over SQ_INSTS_VALU."""
    per = _per_dispatch(db_path, regex)
    n = len(per)
    mean = lambda c: sum(v[c] for v in per.values()) / n
    dur = mean("duration_ns") * 1e-9
    cycles = mean("GRBM_GUI_ACTIVE") / 8.0
    valu = mean("SQ_INSTS_VALU")
    return cycles / dur / 1e9, 1024.0 * cycles / valu, valu, n, dur


def valu_record(db_path: str, regex: str, vectors: int, sources, ref_db: str) -> dict:
    """Clock and VALU issue of one kernel, set against the reference stream of
    independent fp32 FMAs (valuref.py, profiled the same way): issue_vs_fma_stream
    is the stream's clocks per VALU instruction over the kernel's."""
    import hashlib
    ghz, cpi, valu, n, dur = clocks_per_valu(db_path, regex)
    rghz, rcpi, _, _, _ = clocks_per_valu(ref_db, "fma_stream")
    h = hashlib.sha256()
    for f in sources:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return {"kernel_regex": regex, "dispatches": n, "duration_us": dur * 1e6, "sclk_ghz": ghz,
            "valu_instr": valu, "simd_clocks_per_valu_instr": cpi,
            "fma_stream_clocks_per_valu_instr": rcpi, "fma_stream_sclk_ghz": rghz,
            "issue_vs_fma_stream": rcpi / cpi,
            "valu_instr_per_vector": valu / vectors, "vectors": vectors, "source_files": list(sources),
            "source_sha256": h.hexdigest()}


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "--valu-json":
        # --valu-json OUT DB REF_DB REGEX VECTORS SOURCE...
        import json
        out, db, ref_db, regex, vec = sys.argv[2:7]
        rec = valu_record(db, regex, int(vec), sys.argv[7:], ref_db)
        with open(out, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec, indent=1))
    else:
        print(summarize(sys.argv[1]))
