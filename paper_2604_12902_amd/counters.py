"""HBM bytes per launch of a kernel from two rocprofv3 counter runs.

The two runs (FETCH_SIZE, then WRITE_SIZE, each in KiB per dispatch) profile
`bench.py --calibrate-copy BYTES ...`.  The run's largest plain device-to-device
copy (`__amd_rocclr_copyBuffer`, BYTES read and BYTES written) calibrates each
counter: scale = BYTES / (counter KiB * 1024).  A kernel's mean counter value
per dispatch times that scale is its traffic.

The result is recorded in profiles/<workload>_<kernel>_traffic.json under the
scheduling knobs of the profiled run (the traffic of a launch depends on
them) together with the SHA-256 of the kernel source's code (comments and
whitespace aside); bench.py reports it only for the same kernel code and a
run that agrees on the knobs that affect that kernel (KNOBS_OF_KERNEL).

usage: python -m paper_2604_12902_amd.counters FETCH_DIR WRITE_DIR BYTES KERNEL_SUBSTRING OUT_JSON KNOBS_JSON [LAST]
"""
import glob
import hashlib
import json
import os
import re
import sqlite3
import sys

KERNELS_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "rasp_kernels.hip")


def code_sha256(text: str) -> str:
    """SHA-256 of C++ source with comments removed and whitespace collapsed,
    so that a record outlives edits to comments but not to code."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return hashlib.sha256(" ".join(text.split()).encode()).hexdigest()


def kernels_sha256() -> str:
    with open(KERNELS_SRC, encoding="utf-8") as f:
        return code_sha256(f.read())


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


def measure(fdir, wdir, nbytes, ksub, last=0):
    """Bytes per launch of the kernels whose name contains `ksub`: the mean
    over their dispatches, or over the `last` latest ones (a run that times
    two modes one after the other).  `ksub` may list several substrings
    separated by '|' (launches that run side by side as one step, such as
    the fits' and the misfits' launches of a hot-cell run): the result is the
    sum of their per-launch means."""
    res = {"copy_bytes": nbytes, "kernel": ksub}
    if last:
        res["last_dispatches"] = last
    parts = ksub.split("|")
    for tag, d, c in (("fetch", fdir, "FETCH_SIZE"), ("write", wdir, "WRITE_SIZE")):
        vals = per_dispatch(d, c)
        copies = [v for (n, _), v in vals.items() if "copyBuffer" in n]
        ref = max(copies)
        scale = nbytes / (ref * 1024.0)
        res[tag + "_copy_kib"] = ref
        res[tag + "_scale"] = scale
        kib = 0.0
        for part in parts:
            kern = [v for (n, disp), v in sorted(vals.items(), key=lambda e: e[0][1]) if part in n]
            if last:
                kern = kern[-last:]
            kib += sum(kern) / len(kern)
            res[tag + "_kernel_dispatches"] = len(kern)
        res[tag + "_kernel_kib_mean"] = kib
        res[tag + "_bytes_per_launch"] = kib * 1024.0 * scale
    res["bytes_per_launch"] = res["fetch_bytes_per_launch"] + res["write_bytes_per_launch"]
    return res


# the knobs that can change the bytes a kernel moves per launch: k_pack runs
# before any step (only how c0 is built and the CU share matter); the first
# pass also depends on its length and on whether it profiles hot cells; the
# persistent kernels (and the hot-cell pair of launches) on every knob
KNOBS_OF_KERNEL = {
    "pack": ("c0_in_run", "batches_in_flight", "cu_partition"),
    "plain": ("first_pass", "first_pass_kind", "c0_in_run", "batches_in_flight", "cu_partition",
              "hot_cells", "profile_steps"),
}


def lookup(path, knobs, kernel=None):
    """Bytes per launch recorded for the current kernel code and knobs that
    agree with `knobs` on every knob that affects `kernel` (all knobs when
    the kernel is not in KNOBS_OF_KERNEL), or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernels_sha256") != kernels_sha256():
        return None
    keys = KNOBS_OF_KERNEL.get(kernel)
    for run in t.get("runs", []):
        rk = run.get("knobs", {})
        if keys is None:
            if rk == knobs:
                return run["bytes_per_launch"]
        elif all(rk.get(k) == knobs.get(k) for k in keys):
            return run["bytes_per_launch"]
    return None


def main():
    fdir, wdir, nbytes, ksub, out = sys.argv[1], sys.argv[2], int(sys.argv[3]), sys.argv[4], sys.argv[5]
    knobs = json.loads(sys.argv[6])
    last = int(sys.argv[7]) if len(sys.argv) > 7 else 0
    res = measure(fdir, wdir, nbytes, ksub, last)
    res["knobs"] = knobs
    sha = kernels_sha256()
    t = {"kernels_sha256": sha, "runs": []}
    if os.path.exists(out):
        with open(out) as f:
            old = json.load(f)
        if old.get("kernels_sha256") == sha:
            t["runs"] = [r for r in old.get("runs", []) if r.get("knobs") != knobs]
    t["runs"].append(res)
    with open(out, "w") as f:
        json.dump(t, f, indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
