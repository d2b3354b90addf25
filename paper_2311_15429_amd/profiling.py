"""Summaries of rocprofv3 output for the lag-sum kernel (reporting only).

HBM traffic per launch comes from two counter passes, FETCH_SIZE and
WRITE_SIZE (KiB per dispatch).  Each is scaled by what the same counter reads
for a device copy of known size in the same run (the largest
__amd_rocclr_copyBuffer dispatch, `bench.py --calib-copy-mib N`), because the
derived counters need not count every request size.

    python -m paper_2311_15429_amd.profiling FETCH.csv WRITE.csv --copy-mib 1024 \
        --key config2|fp32 --out profiles/lagsum_traffic.json
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import sys
from collections import defaultdict


def kernel_source_sha():
    """Hash of the lag-sum kernel's source: lagsum.hip and the lag-sum tables'
    declarations.  Counter figures taken on another source are stale."""
    import hashlib
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha1()
    h.update(open(os.path.join(here, "lagsum.hip"), "rb").read())
    hdr = open(os.path.join(here, "rpot_internal.hpp")).read()
    a, b = hdr.index("// Lag-sum multiply-accumulate."), hdr.index("// Launchers")
    h.update(hdr[a:b].encode())
    return h.hexdigest()


def _read(path):
    rows = list(csv.DictReader(open(path)))
    per = defaultdict(list)
    copy = 0.0
    for r in rows:
        v = float(r["Counter_Value"])
        per[r["Kernel_Name"]].append(v)
        if r["Kernel_Name"].startswith("__amd_rocclr_copyBuffer"):
            copy = max(copy, v)
    return per, copy


def traffic(fetch_csv, write_csv, copy_mib, kernel_substr="k_lagsum"):
    """Calibrated HBM bytes per launch of the kernel whose name contains
    kernel_substr: (fetch_bytes, write_bytes, fetch_scale, write_scale, launches)."""
    fper, fcopy = _read(fetch_csv)
    wper, wcopy = _read(write_csv)
    true_kib = copy_mib * 1024.0
    fscale = true_kib / fcopy if fcopy > 0 else float("nan")
    wscale = true_kib / wcopy if wcopy > 0 else float("nan")
    fk = [v for k, vs in fper.items() if kernel_substr in k for v in vs]
    wk = [v for k, vs in wper.items() if kernel_substr in k for v in vs]
    if not fk or not wk:
        raise ValueError(f"no dispatch of {kernel_substr} in the counter files")
    f = sum(fk) / len(fk) * 1024.0 * fscale
    w = sum(wk) / len(wk) * 1024.0 * wscale
    return f, w, fscale, wscale, len(fk)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv")
    ap.add_argument("--copy-mib", type=float, required=True)
    ap.add_argument("--key", required=True)
    ap.add_argument("--kernel-sha", default=None, help="default: the current lag-sum source")
    ap.add_argument("--kernel", default="k_lagsum")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    f, w, fs, ws, n = traffic(a.fetch_csv, a.write_csv, a.copy_mib, a.kernel)
    rec = {}
    if os.path.exists(a.out):
        rec = json.load(open(a.out))
    rec[a.key] = {"kernel_source_sha": a.kernel_sha or kernel_source_sha(), "traffic_bytes_per_launch": f + w,
                  "fetch_bytes": f, "write_bytes": w, "fetch_scale": fs, "write_scale": ws,
                  "launches": n}
    json.dump(rec, open(a.out, "w"), indent=1, sort_keys=True)
    print(json.dumps(rec[a.key]))
    return 0


if __name__ == "__main__":
    sys.exit(main())
