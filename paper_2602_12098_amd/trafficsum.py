"""HBM traffic of one kernel from rocprofv3 --pmc runs: FETCH_SIZE and
WRITE_SIZE (KiB per dispatch, summed over the TCC channels) of the kernel,
each scaled by what the same counter reads for the reference copy kernel of
known size (copyref.py: 1 GiB read + 1 GiB written per dispatch).  Writes a
small JSON with the per-launch bytes and the hash of the kernel sources, so
that a consumer can tell when the counters are stale.

Usage: python -m paper_2602_12098_amd.trafficsum KERNEL_REGEX FETCH_DB WRITE_DB
           COPY_FETCH_DB COPY_WRITE_DB OUT.json SOURCE...
"""
import hashlib
import json
import re
import sqlite3
import sys


def per_dispatch(db_path, counter, regex):
    db = sqlite3.connect(db_path)
    rows = db.execute("select kernel_name, dispatch_id, sum(value) from counters_collection "
                      "where counter_name = ? group by kernel_name, dispatch_id", (counter,)).fetchall()
    vals = [v for k, d, v in rows if re.search(regex, k)]
    if not vals:
        raise SystemExit(f"no dispatch of /{regex}/ with {counter} in {db_path}")
    return sum(vals) / len(vals), len(vals)


def sources_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def main():
    regex, fdb, wdb, cfdb, cwdb, out = sys.argv[1:7]
    srcs = sys.argv[7:]
    f, nf = per_dispatch(fdb, "FETCH_SIZE", regex)
    w, nw = per_dispatch(wdb, "WRITE_SIZE", regex)
    cf, _ = per_dispatch(cfdb, "FETCH_SIZE", "elementwise")
    cw, _ = per_dispatch(cwdb, "WRITE_SIZE", "elementwise")
    ref = float(1 << 30)
    sf, sw = ref / (cf * 1024.0), ref / (cw * 1024.0)   # true bytes per counted byte
    rec = {"kernel_regex": regex, "dispatches": [nf, nw],
           "fetch_kib_raw": f, "write_kib_raw": w, "copy_fetch_kib_raw": cf, "copy_write_kib_raw": cw,
           "fetch_scale": sf, "write_scale": sw,
           "fetch_bytes_per_launch": f * 1024.0 * sf, "write_bytes_per_launch": w * 1024.0 * sw,
           "source_files": srcs, "source_sha256": sources_hash(srcs)}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
