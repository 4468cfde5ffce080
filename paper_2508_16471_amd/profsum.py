#!/usr/bin/env python3
"""Summarise rocprofv3 output databases (SQLite, ``*_results.db``).

  python -m paper_2508_16471_amd.profsum stats DIR [FILTER]
      per-kernel dispatch count, total / average / min / max duration
  python -m paper_2508_16471_amd.profsum counters DIR [FILTER]
      per-kernel mean value of every collected counter per dispatch
  python -m paper_2508_16471_amd.profsum traffic FETCH_DIR WRITE_DIR KERNEL KIND RCAL WCAL OUT.json
      HBM bytes per dispatch of KERNEL (a name substring; KIND is the
      library's timing name for it) from a FETCH_SIZE run and a WRITE_SIZE
      run, each scaled so that a calibration kernel of known traffic reads
      its true byte count: RCAL reads 512 MiB per dispatch (a device sum),
      WCAL writes 512 MiB per dispatch (a device fill).  Writes a JSON
      record stamped with the SHA-256 of the operator-product sources so that
      a later change invalidates it.
"""

import glob
import hashlib
import json
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PRODUCT_SOURCES = ["paper_2508_16471_amd/csrc/fft_passes.hip", "paper_2508_16471_amd/csrc/fft_xc.hip",
                   "paper_2508_16471_amd/csrc/fft_common.h", "paper_2508_16471_amd/csrc/fft.h",
                   "paper_2508_16471_amd/csrc/common.h", "paper_2508_16471_amd/csrc/kernels.h"]
COPY_BYTES = 512 << 20


def sources_sha():
    h = hashlib.sha256()
    for rel in PRODUCT_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _db(d):
    found = glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True)
    if not found:
        raise SystemExit(f"no *_results.db under {d}")
    return sqlite3.connect(found[0])


def kernel_stats(d, flt=""):
    cur = _db(d).cursor()
    rows = cur.execute("select name, count(*), sum(duration), avg(duration), min(duration), "
                       "max(duration) from kernels group by name order by sum(duration) desc").fetchall()
    return [r for r in rows if flt in r[0]]


def counters(d, flt=""):
    cur = _db(d).cursor()
    cols = [r[1] for r in cur.execute("pragma table_info(counters_collection)")]
    kn = "kernel_name" if "kernel_name" in cols else "name"
    cn = "counter_name" if "counter_name" in cols else "counter"
    vn = "value" if "value" in cols else "counter_value"
    rows = cur.execute(f"select {kn}, {cn}, sum({vn}), count(distinct dispatch_id) from "
                       f"counters_collection group by {kn}, {cn}").fetchall()
    out = {}
    for k, c, s, n in rows:
        if flt in k:
            out.setdefault(k, {})[c] = s / n
    return out


def _short(name, n=90):
    return name if len(name) <= n else name[:n - 3] + "..."


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        flt = argv[2] if len(argv) > 2 else ""
        print(f"{'kernel':90s} {'calls':>7s} {'total ms':>10s} {'avg us':>10s} {'min us':>10s} "
              f"{'max us':>10s}")
        for name, n, tot, avg, mn, mx in kernel_stats(argv[1], flt):
            print(f"{_short(name):90s} {n:7d} {tot / 1e6:10.3f} {avg / 1e3:10.2f} {mn / 1e3:10.2f} "
                  f"{mx / 1e3:10.2f}")
        return 0
    if len(argv) >= 2 and argv[0] == "counters":
        flt = argv[2] if len(argv) > 2 else ""
        for k, cs in counters(argv[1], flt).items():
            print(_short(k))
            for c, v in sorted(cs.items()):
                print(f"    {c:36s} {v:.6g}")
        return 0
    if len(argv) == 8 and argv[0] == "traffic":
        fdir, wdir, kern, kind, rcal, wcal, out = argv[1:]
        f = counters(fdir)
        w = counters(wdir)

        def pick(tab, key, counter):
            hits = [v[counter] for k, v in tab.items() if key in k and counter in v]
            if not hits:
                raise SystemExit(f"{counter} for '{key}' not found")
            return sum(hits) / len(hits)

        fk, wk = pick(f, kern, "FETCH_SIZE"), pick(w, kern, "WRITE_SIZE")
        fc, wc = pick(f, rcal, "FETCH_SIZE"), pick(w, wcal, "WRITE_SIZE")
        fscale = COPY_BYTES / (fc * 1024.0)
        wscale = COPY_BYTES / (wc * 1024.0)
        rec = {"kernel": kern, "kind": kind, "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
               "calib_read_kernel": rcal, "calib_write_kernel": wcal,
               "calib_fetch_kib": fc, "calib_write_kib": wc, "fetch_scale": fscale,
               "write_scale": wscale,
               "bytes_per_dispatch": fk * 1024.0 * fscale + wk * 1024.0 * wscale,
               "sources_sha256": sources_sha(), "sources": PRODUCT_SOURCES}
        with open(out, "w") as fo:
            json.dump(rec, fo, indent=1)
            fo.write("\n")
        print(json.dumps(rec))
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
