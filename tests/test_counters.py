"""The traffic records bench.py reports: keyed by the scheduling knobs and
by the kernel source's code (comments and whitespace aside)."""
import json
import os

from paper_2604_12902_amd import counters


def test_code_hash_ignores_comments_and_whitespace_only():
    a = "int f(int x) {  // doubles\n    return 2 * x; /* the\n result */\n}\n"
    b = "int f(int x)\n{\n  return 2 * x;\n}  // edited comment\n"
    c = "int f(int x) { return 3 * x; }"
    assert counters.code_sha256(a) == counters.code_sha256(b)
    assert counters.code_sha256(a) != counters.code_sha256(c)


def test_lookup_needs_the_same_knobs_and_kernel_code(tmp_path):
    knobs = {"schedule": 2, "lds_words": 256, "epoch": 256}
    path = tmp_path / "w_k_traffic.json"
    path.write_text(json.dumps({"kernels_sha256": counters.kernels_sha256(),
                                "runs": [{"knobs": knobs, "bytes_per_launch": 123.0}]}))
    assert counters.lookup(str(path), knobs) == 123.0
    assert counters.lookup(str(path), dict(knobs, epoch=1024)) is None
    path.write_text(json.dumps({"kernels_sha256": "0" * 64,
                                "runs": [{"knobs": knobs, "bytes_per_launch": 123.0}]}))
    assert counters.lookup(str(path), knobs) is None
    assert counters.lookup(str(tmp_path / "missing.json"), knobs) is None


def test_committed_records_of_the_headline_match_the_current_kernels():
    """The records of the default workload (uneven) were taken on the kernel
    code in the tree, so the bench line's traffic is not null; records of
    other workloads taken on older code are ignored by lookup()."""
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for k in ("persistent+misfit", "pack", "plain"):
        with open(os.path.join(root, "profiles", "uneven_%s_traffic.json" % k)) as f:
            rec = json.load(f)
        assert rec["kernels_sha256"] == counters.kernels_sha256(), k
        assert rec["runs"]


def test_cached_headline_knobs_find_a_traffic_record():
    """The knobs the autotune cache holds for the headline (uneven, four
    batches in flight) have a record of the concurrent fits' and misfits'
    launches."""
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(root, "paper_2604_12902_amd", "tune_cache.json")) as f:
        cache = json.load(f)
    entries = [(json.loads(k), v) for k, v in cache.items() if json.loads(k)["num_vms"] == 1 << 22]
    assert entries
    path = os.path.join(root, "profiles", "uneven_persistent+misfit_traffic.json")
    for key, v in entries:
        t = dict(v["autotune"])
        knobs = {k: t[k] for k in ("schedule", "lds_words", "first_pass", "epoch", "waves_per_cu",
                                   "first_pass_kind", "hot_cells", "profile_steps", "misfit_waves")}
        knobs.update(first_pass=v["inflight_first_pass"], epoch=v["inflight_epoch"], c0_in_run=False)
        knobs.update(hot_cells=v.get("inflight_hot_cells", knobs["hot_cells"]),
                     misfit_waves=v.get("inflight_misfit_waves", knobs["misfit_waves"]))
        if v["inflight"] > 1:
            knobs.update(batches_in_flight=v["inflight"], cu_partition="split")
        assert counters.lookup(path, knobs, "persistent+misfit") is not None, knobs


def test_pack_records_ignore_the_step_loop_knobs(tmp_path):
    """k_pack runs before any step: its record serves any epoch, slot or
    first pass, but not another CU share or lazy c0."""
    rec = {"schedule": 2, "lds_words": 256, "first_pass": 64, "epoch": 256, "waves_per_cu": 16,
           "first_pass_kind": 0, "c0_in_run": False, "batches_in_flight": 4, "cu_partition": "split"}
    path = tmp_path / "w_pack_traffic.json"
    path.write_text(json.dumps({"kernels_sha256": counters.kernels_sha256(),
                                "runs": [{"knobs": rec, "bytes_per_launch": 7.0}]}))
    assert counters.lookup(str(path), dict(rec, epoch=64, lds_words=128), "pack") == 7.0
    assert counters.lookup(str(path), dict(rec, batches_in_flight=2), "pack") is None
    assert counters.lookup(str(path), dict(rec, c0_in_run=True), "pack") is None
    assert counters.lookup(str(path), dict(rec, epoch=64), "persistent") is None
    assert counters.lookup(str(path), dict(rec, epoch=64), "plain") == 7.0
    assert counters.lookup(str(path), dict(rec, first_pass=16), "plain") is None


def _counter_db(d, counter, rows):
    """A rocprofv3-shaped result: one counters_collection row per (kernel,
    dispatch, counter instance), values in KiB."""
    import sqlite3
    os.makedirs(d, exist_ok=True)
    con = sqlite3.connect(os.path.join(d, "pmc_results.db"))
    con.execute("create table counters_collection (kernel_name text, dispatch_id integer, "
                "counter_name text, value real, duration integer)")
    for name, disp, val in rows:
        con.execute("insert into counters_collection values (?, ?, ?, ?, 0)", (name, disp, counter, val))
    con.commit()
    con.close()


def test_measure_scales_by_the_copy_and_averages_dispatches(tmp_path):
    """A 1 GiB copy that reads 512 Ki KiB of FETCH_SIZE scales fetch by 2; a
    kernel's counter instances are summed per dispatch and averaged over
    dispatches (or over the last N)."""
    gib = 1 << 30
    f, w = str(tmp_path / "f"), str(tmp_path / "w")
    copy = "__amd_rocclr_copyBuffer"
    _counter_db(f, "FETCH_SIZE", [(copy, 1, 262144.0), (copy, 1, 262144.0),
                                  ("k_pack(x)", 2, 100.0), ("k_pack(x)", 2, 50.0),
                                  ("k_pack(x)", 3, 300.0), ("k_plain(x)", 4, 7.0)])
    _counter_db(w, "WRITE_SIZE", [(copy, 1, 1048576.0), ("k_pack(x)", 2, 10.0),
                                  ("k_pack(x)", 3, 30.0)])
    res = counters.measure(f, w, gib, "k_pack")
    assert res["fetch_scale"] == 2.0 and res["write_scale"] == 1.0
    assert res["fetch_kernel_dispatches"] == 2
    assert res["fetch_bytes_per_launch"] == (150.0 + 300.0) / 2 * 1024 * 2
    assert res["write_bytes_per_launch"] == (10.0 + 30.0) / 2 * 1024
    assert res["bytes_per_launch"] == res["fetch_bytes_per_launch"] + res["write_bytes_per_launch"]
    last = counters.measure(f, w, gib, "k_pack", last=1)
    assert last["fetch_bytes_per_launch"] == 300.0 * 1024 * 2
    assert last["write_bytes_per_launch"] == 30.0 * 1024


def test_measure_sums_launches_that_run_side_by_side(tmp_path):
    """'a|b': the per-launch means of both kernels, added (one step of the
    path is one launch of each)."""
    gib = 1 << 30
    f, w = str(tmp_path / "f"), str(tmp_path / "w")
    copy = "__amd_rocclr_copyBuffer"
    _counter_db(f, "FETCH_SIZE", [(copy, 1, 524288.0), ("k_hot(x)", 2, 100.0), ("k_hot(x)", 4, 300.0),
                                  ("k_mis(x)", 3, 10.0), ("k_mis(x)", 5, 30.0)])
    _counter_db(w, "WRITE_SIZE", [(copy, 1, 1048576.0), ("k_hot(x)", 2, 1.0), ("k_hot(x)", 4, 3.0),
                                  ("k_mis(x)", 3, 5.0), ("k_mis(x)", 5, 5.0)])
    res = counters.measure(f, w, gib, "k_hot|k_mis")
    assert res["fetch_bytes_per_launch"] == (200.0 + 20.0) * 1024 * 2
    assert res["write_bytes_per_launch"] == (2.0 + 5.0) * 1024
