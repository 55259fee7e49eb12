"""Turn two rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE) of
`bench.py --calibrate-copy BYTES ...` into HBM bytes per launch of a kernel.

Both counters are read per dispatch in KiB.  The run's largest plain
device-to-device copy (`__amd_rocclr_copyBuffer`, BYTES read and BYTES
written) calibrates each counter: scale = BYTES / (counter KiB * 1024).  The
kernel's mean counter value per dispatch times that scale is the traffic.

usage: python -m paper_2604_12902_amd.counters FETCH_DIR WRITE_DIR BYTES KERNEL_SUBSTRING OUT_JSON
"""
import glob
import hashlib
import json
import os
import sqlite3
import sys


def per_dispatch(d, counter):
    db = glob.glob(os.path.join(d, "*.db"))[0]
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, dispatch_id, value from counters_collection "
                       "where counter_name = ?", (counter,)).fetchall()
    out = {}
    for name, disp, val in rows:
        out.setdefault((name, disp), 0.0)
        out[(name, disp)] += val
    return out


def main():
    fdir, wdir, nbytes, ksub, out = sys.argv[1], sys.argv[2], int(sys.argv[3]), sys.argv[4], sys.argv[5]
    res = {"copy_bytes": nbytes, "kernel": ksub}
    for tag, d, c in (("fetch", fdir, "FETCH_SIZE"), ("write", wdir, "WRITE_SIZE")):
        vals = per_dispatch(d, c)
        copies = [v for (n, _), v in vals.items() if "copyBuffer" in n]
        kern = [v for (n, _), v in vals.items() if ksub in n]
        ref = max(copies)
        scale = nbytes / (ref * 1024.0)
        res[tag + "_copy_kib"] = ref
        res[tag + "_scale"] = scale
        res[tag + "_kernel_kib_mean"] = sum(kern) / len(kern)
        res[tag + "_kernel_dispatches"] = len(kern)
        res[tag + "_bytes_per_launch"] = sum(kern) / len(kern) * 1024.0 * scale
    res["bytes_per_launch"] = res["fetch_bytes_per_launch"] + res["write_bytes_per_launch"]
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "rasp_kernels.hip")
    res["kernels_sha256"] = hashlib.sha256(open(src, "rb").read()).hexdigest()
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
