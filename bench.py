#!/usr/bin/env python3
"""Benchmark: VM instructions retired per second on one MI355X, bit-exact.

One step = one pass of the whole hot path over one batch of synthetic
machines whose packed programs and tapes are already resident in HBM:
  rasp_load_batch (device descriptor: checks, offsets, c0 pack)
  rasp_run(budget) (plain, or first plain pass + persistent work-queue kernel)
  rasp_fetch_outputs into device-resident buffers (status, steps, i, a, u0,
  y0 and the output words)
  rasp_free_batch.
The value is the sum of retired transitions of a batch divided by the mean
time per batch over the timed batches, with up to four batches in flight:
one context per batch in flight, each with its own host thread and its own
share of the compute units (rasp_create_on_cus), the count chosen from 1, 2
and 4 by short untimed trials, after which the first-pass length, the epoch
and the hot-cell knobs are tried again the same way in flight (and, when one
of them moved, the other counts once more).  The same schedule one batch at a time
(single_batch) and the plain one-machine-per-lane schedule are reported
beside it.  Before reporting, the final state of every machine is checked
against the CPU oracle (the oracle is run on the same batch on the host; its
timing is the cpu_baseline).

Workloads (sizes of the stated populations):
  uneven       4,194,304 programs of 8..512 instructions (lengths log-uniform),
               n = 64..1,024 words, budget 65,536 (default: the largest
               population that fits one GPU)
  plain-scale  1,048,576 random programs x 64 instructions, n = 256,
               tape 32 words, output capacity 16, budget 4,096
  plain-small  4,096 x 16 instructions, n = 32, budget 256
  rollouts     262,144 counted-loop array programs (each machine its own), n = 2,048,
               budget 2^20
  fig1         262,144 uniform Sec. 2.2 programs of 100 terminals, word RASP,
               n = 250, l = 10, s = 2, budget 10^6 (the Sec. 3 evaluation)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uneven",
                    choices=["plain-scale", "plain-small", "uneven", "rollouts", "fig1", "serve"])
    ap.add_argument("--requests", type=int, default=500, help="serve: requests per run")
    ap.add_argument("--loads", default="0.5,0.8,1.0", help="serve: offered load, fractions of capacity")
    ap.add_argument("--cap-gb", type=float, default=200.0, help="serve: arena footprint cap")
    ap.add_argument("--serve-epoch", type=int, default=4096, help="serve: transitions per epoch")
    ap.add_argument("--serve-graph", type=int, default=0, choices=[0, 1],
                    help="serve: replay each epoch's launch sequence as a HIP graph while the admitted set "
                         "is unchanged (RASP_OPT_GRAPH)")
    ap.add_argument("--serve-partitions", type=int, default=0,
                    help="serve: servers, each with its own context on its own CU share (0: one "
                         "or four, whichever serves the closed loop faster)")
    ap.add_argument("--num-vms", type=int, default=0, help="override the population size")
    ap.add_argument("--batch-file", default="",
                    help="keep the generated batch in this .npz file and read it from there when it "
                         "holds the same workload (saves generating it again, e.g. under a profiler)")
    ap.add_argument("--gen-workers", type=int, default=0,
                    help="processes generating the fig1 and rollout programs (0: up to 16; 1 under "
                         "a profiler, which would otherwise follow every child process)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-schedule comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verify", choices=["full", "sample", "none"], default="full")
    ap.add_argument("--first-pass", type=int, default=None)
    ap.add_argument("--lds-words", type=int, default=None)
    ap.add_argument("--epoch", type=int, default=None)
    ap.add_argument("--waves-per-cu", type=int, default=None)
    ap.add_argument("--first-pass-kind", type=int, default=None, choices=[0, 1])
    ap.add_argument("--hot-cells", type=int, default=None, choices=[0, 8, 16, 32, 64],
                    help="slots of the hot-cell LDS table per machine (0: off)")
    ap.add_argument("--profile-steps", type=int, default=None,
                    help="transitions profiled at the end of a hot-cell first pass")
    ap.add_argument("--misfit-waves", type=int, default=None,
                    help="waves per CU of the hot-cell misfits' launch")
    ap.add_argument("--inflight", type=int, default=0,
                    help="the headline times the persistent schedule with this many batches in "
                         "flight, one context, stream and host thread each (1: one batch at a "
                         "time; 0: the best of 1, 2 and 4 in short untimed trials); the "
                         "one-batch run is always timed and reported as single_batch")
    ap.add_argument("--inflight-shares", type=int, default=0,
                    help="CU shares the batches in flight are spread over (0: one share per batch); "
                         "with fewer shares than batches, batch k runs on share k mod shares")
    ap.add_argument("--inflight-cus", choices=["shared", "split"], default="split",
                    help="with --inflight N: all contexts share every CU, or each context's stream "
                         "gets its own contiguous 1/N of them")
    ap.add_argument("--lazy", action="store_true",
                    help="build c0 inside the run (RASP_DESC_LAZY) instead of in rasp_load_batch")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default knobs instead of running rasp_autotune")
    ap.add_argument("--retune", action="store_true",
                    help="search the knobs again even when the autotune cache holds them for this "
                         "device, batch and library code")
    ap.add_argument("--tune-cache", default=None,
                    help="autotune cache file (default: the package's tune_cache.json)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="bytes of one plain device-to-device copy run before the workload "
                         "(the reference dispatch for HBM byte counters)")
    ap.add_argument("--json-extra", default="", help="path to write the full report")
    return ap.parse_args()


def make_batch(args):
    from paper_2604_12902_amd import workloads as W
    if args.batch_file and os.path.exists(args.batch_file):
        b = W.load_batch(args.batch_file)
        if b.meta.get("workload") == args.workload and (not args.num_vms or b.N == args.num_vms):
            return b
    b = _generate(args)
    if args.batch_file:
        b.meta["workload"] = args.workload
        W.save_batch(b, args.batch_file)
    return b


def _generate(args):
    from paper_2604_12902_amd import workloads as W
    kw = {}
    if args.num_vms:
        kw["num_vms"] = args.num_vms
    if args.workload == "plain-scale":
        return W.config2(**kw)
    if args.workload == "plain-small":
        return W.config1(**kw)
    if args.workload == "uneven":
        return W.config3(**kw)
    if args.workload == "fig1":
        return W.fig1(workers=args.gen_workers or min(16, os.cpu_count() or 1), **kw)
    return W.config4(workers=args.gen_workers or min(16, os.cpu_count() or 1), **kw)


def cpu_model() -> str:
    """The host CPU's model name and logical CPU count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return "%s (%d logical CPUs)" % (name, os.cpu_count() or 0)


def oracle_compiler() -> str:
    """Version of the C compiler that builds the oracle."""
    import subprocess
    try:
        out = subprocess.run(["gcc", "--version"], capture_output=True, text=True, timeout=10).stdout
        return out.splitlines()[0].strip() + " -O3"
    except (OSError, subprocess.SubprocessError, IndexError):
        return "unknown"


def bytes_per_step(mix: np.ndarray) -> float:
    """Algorithmic bytes per retired step for a retired-opcode mix:
    8 B fetch (opcode + operand) always; +4 B data read for ADD/SUB/MUL;
    +4 B data write for STORE; READ +4 B tape read +4 B memory write; a
    PRINT that appends +4 B data read +4 B output write (a PRINT past the
    output capacity moves no word)."""
    steps = float(mix[1:9].sum())
    if steps == 0:
        return 0.0
    extra = 4.0 * (mix[2] + mix[3]) + 4.0 * mix[4] + 8.0 * mix[6] + 8.0 * mix[9]
    return 8.0 + float(extra) / steps


def pack_bytes(batch) -> int:
    """Algorithmic bytes of building c0: read the program and input words,
    write n + l + s words and the 25 B of scalars (i, a, u0, y0, steps,
    status) per machine."""
    N = batch.N
    return int(4 * batch.prog.size + 4 * batch.tape.size +
               4 * (batch.mem_words.astype(np.int64).sum() + batch.tape_cap.astype(np.int64).sum()
                    + batch.out_cap.astype(np.int64).sum()) + 25 * N)


def serve_bench(args):
    """Serving: a Poisson stream of rollout requests (1,024-262,144 machines,
    family uniform over plain-small / plain-scale / uneven, budgets 4,096-65,536)
    served with continuous batching under a footprint cap.  Capacity is first
    measured closed-loop (every request queued at t = 0); the stream is then
    replayed at fixed fractions of that rate.  Reports retired steps/s and
    p50/p99 request latency (arrival to outputs on the host)."""
    import torch
    import oracle
    from paper_2604_12902_amd import rasp as R, serving

    t0 = time.time()
    reqs = serving.poisson_requests(args.requests, 1.0, seed=4)
    base_arrivals = [q.arrival for q in reqs]
    print("serve: %d requests generated in %.1f s (%d machines)" % (
        len(reqs), time.time() - t0, sum(q.size for q in reqs)), flush=True)
    free, _ = torch.cuda.mem_get_info()
    cap = int(min(args.cap_gb * 1e9, 0.85 * free))
    state = {}

    def open_partitions(k):
        """k servers: one context each (k > 1: on its own CU share), sharing the cap."""
        close_partitions()
        if k == 1:
            state["ctxs"] = [R.Context(cap + (256 << 20))]
        else:
            cus = torch.cuda.get_device_properties(0).multi_processor_count
            state["ctxs"] = [R.Context(cap // k + (256 << 20), cus=R.cu_share(i, k, cus)) for i in range(k)]
        for c in state["ctxs"]:
            c.set(R.RASP_OPT_GRAPH, args.serve_graph)
        state["k"] = k

    def close_partitions():
        for c in state.get("ctxs", []):
            c.close()
        state.clear()

    def run(qps):
        for q, a in zip(reqs, base_arrivals):
            q.arrival = 0.0 if qps is None else a / qps
            q.result = None
        exs = [serving.RaspExecutor(c) for c in state["ctxs"]]
        if len(exs) == 1:
            return serving.Server(exs[0], cap, epoch=args.serve_epoch).serve(reqs)
        return serving.serve_partitioned(exs, reqs, cap, epoch=args.serve_epoch)

    # partitions: one server on the whole chip, or (chosen when the closed
    # loop is at least 3% faster) one per CU share; each closed loop after a
    # warm-up pass
    closed = None
    for k in ([1, SERVE_PARTITIONS] if args.serve_partitions == 0 else [args.serve_partitions]):
        open_partitions(k)
        run(None)                                       # warm-up
        st = run(None)
        print("serve: %d partition(s): closed loop %.3f s, %.1f requests/s, %.3e steps/s" % (
            k, st.wall_s, st.requests / st.wall_s, st.steps_per_s), flush=True)
        if closed is None or st.steps_per_s > closed[1].steps_per_s / 0.97:
            closed = (k, st)
    if state["k"] != closed[0]:
        open_partitions(closed[0])
    parts, closed = closed
    # the results checked below are those of the chosen configuration
    closed = run(None)
    cap_qps = closed.requests / closed.wall_s
    print("serve: closed loop %.3f s, %.1f requests/s, %.3e steps/s (%d partition(s))" % (
        closed.wall_s, cap_qps, closed.steps_per_s, parts), flush=True)
    # bit-exactness of a sample of every request's machines against the oracle
    for q in reqs[:: max(1, len(reqs) // 6)]:
        idx = np.arange(0, q.batch.N, max(1, q.batch.N // 300))
        want = oracle.run(q.batch.subset(idx), q.budget, threads=16)
        for k in ("status", "steps", "i", "a", "u0", "y0"):
            if not np.array_equal(np.asarray(q.result[k])[idx], getattr(want, k)):
                raise SystemExit("serve: NOT bit-exact (request %d, %s)" % (q.rid, k))
    runs = []
    for f in [float(x) for x in args.loads.split(",") if x]:
        st = run(f * cap_qps)
        runs.append(dict(load=f, qps=f * cap_qps, wall_s=st.wall_s, steps_per_s=st.steps_per_s,
                         p50_ms=st.p50_ms, p99_ms=st.p99_ms, mean_ms=st.mean_ms,
                         epochs=st.epochs, max_active=st.max_active))
        print("serve: load %.2f qps %.1f: %.3e steps/s  p50 %.1f ms  p99 %.1f ms  epochs %d  "
              "max active %d" % (f, f * cap_qps, st.steps_per_s, st.p50_ms, st.p99_ms, st.epochs,
                                 st.max_active), flush=True)
    close_partitions()
    head = runs[-1] if runs else None
    line = {"metric": "VM instructions retired/sec (1 GPU), bit-exact; served; p50/p99 request latency",
            "value": head["steps_per_s"] if head else closed.steps_per_s,
            "unit": "VM instructions retired/s", "n_gpus": 1, "steps": len(reqs), "warmup": 1,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
            "data": "synthetic (seeded Poisson stream of random RASP programs)",
            "config": {"workload": "serving: Poisson stream, %d requests of 1,024-262,144 machines, "
                                   "budgets 4,096-65,536, cap %.1f GB" % (len(reqs), cap / 1e9),
                       "epoch": args.serve_epoch, "partitions": parts, "graph": args.serve_graph},
            "closed_loop": {"requests_per_s": cap_qps, "steps_per_s": closed.steps_per_s,
                            "p50_ms": closed.p50_ms, "p99_ms": closed.p99_ms},
            "open_loop": runs}
    print(json.dumps(line), flush=True)


def measured_traffic(workload: str, kernel: str, knobs: dict):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known size)
    for a run with these knobs, or None when there is none or the kernels have
    changed since."""
    from paper_2604_12902_amd import counters
    return counters.lookup(os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (workload, kernel)), knobs,
                           kernel)


def TUNED_OPTIONS(R):
    """The context options the autotuner chooses (copied to in-flight contexts)."""
    return (R.RASP_OPT_SCHEDULE, R.RASP_OPT_LDS_WORDS, R.RASP_OPT_FIRST_PASS, R.RASP_OPT_EPOCH,
            R.RASP_OPT_WAVES_PER_CU, R.RASP_OPT_FIRST_PASS_KIND, R.RASP_OPT_HOT_CELLS,
            R.RASP_OPT_PROFILE_STEPS, R.RASP_OPT_MISFIT_WAVES)


def current_knobs(R, ctx, lazy):
    """The knobs of a run, as recorded beside traffic measurements."""
    return dict(schedule=int(ctx.get(R.RASP_OPT_SCHEDULE)), lds_words=int(ctx.get(R.RASP_OPT_LDS_WORDS)),
                first_pass=int(ctx.get(R.RASP_OPT_FIRST_PASS)), epoch=int(ctx.get(R.RASP_OPT_EPOCH)),
                waves_per_cu=int(ctx.get(R.RASP_OPT_WAVES_PER_CU)),
                first_pass_kind=int(ctx.get(R.RASP_OPT_FIRST_PASS_KIND)),
                hot_cells=int(ctx.get(R.RASP_OPT_HOT_CELLS)),
                profile_steps=int(ctx.get(R.RASP_OPT_PROFILE_STEPS)),
                misfit_waves=int(ctx.get(R.RASP_OPT_MISFIT_WAVES)), c0_in_run=lazy)


# batches in flight tried (five to eight were slower on plain-scale)
INFLIGHT_CANDIDATES = (1, 2, 4)
# knobs tried again once several batches are in flight: the ones whose best
# value depends on how many lanes a batch has
INFLIGHT_FIRST_PASSES = (16, 64, 256)
INFLIGHT_EPOCHS = (64, 256, 1024)
# hot-cell runs: the misfits' waves per CU and the table size, tried again in
# flight (on a CU share the misfits outnumber their lanes several times over)
INFLIGHT_MISFIT_WAVES = (6, 8, 12, 16)
INFLIGHT_HOT_CELLS = (16, 32)
SERVE_PARTITIONS = 4


def arena_inflight(fp):
    """Arena of a context that only loads, runs and fetches (no autotune snapshot)."""
    return int(fp * 1.25) + (256 << 20)


def timed_inflight(args, R, torch, ctx, desc, batch, budget, arena, ref, total_steps, n, steps=None,
                   warmup=None, verify=True, quiet=False, ref_digest=None):
    """The persistent schedule with `n` batches in flight: one
    context per batch in flight, each with its own stream and its own host
    thread that loads, runs and fetches its share of the batches one after
    another, so the load and first pass of one batch run beside the long tail
    of another.  Every batch does the whole work (load, run, fetch); the
    outputs of the last batch of each context are checked against the
    oracle.  Returns throughput and per-batch latency (load issued to outputs
    fetched)."""
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    if args.inflight_cus == "split":
        # each context's stream runs on its own contiguous 1/n of the compute
        # units, so one batch's latency-bound tail does not share SIMDs with
        # the next batch's load and first pass
        cus = R.rasp_device_info(ctx.handle)["compute_units"]
        shares = args.inflight_shares if 0 < args.inflight_shares < n else n
        ctxs = [R.Context(arena, cus=R.cu_share(k % shares, shares, cus)) for k in range(n)]
    else:
        ctxs = [ctx] + [R.Context(arena) for _ in range(n - 1)]
    for c in ctxs:
        if c is ctx:
            continue
        for o in TUNED_OPTIONS(R):
            c.set(o, ctx.get(o))
    dev = torch.device("cuda", 0)
    N = batch.N
    ny = int(batch.out_cap.astype(np.int64).sum())

    def new_outs():
        return dict(status=torch.empty(N, dtype=torch.uint8, device=dev),
                    steps=torch.empty(N, dtype=torch.int64, device=dev),
                    i=torch.empty(N, dtype=torch.int32, device=dev),
                    a=torch.empty(N, dtype=torch.int32, device=dev),
                    u0=torch.empty(N, dtype=torch.int32, device=dev),
                    y0=torch.empty(N, dtype=torch.int32, device=dev),
                    y=torch.empty(ny, dtype=torch.int32, device=dev))
    outs = [new_outs() for _ in range(n)]
    # with a reference digest, each context's last timed batch is kept until
    # after the timed region, when every machine's final memory is compared
    # as its FNV-1a-64 digest (untimed)
    kept = [None] * n

    def drive(c, count, lat, errors, keep_last):
        # one host thread per context: load, run, fetch, free, one batch after
        # another (the library's calls release the interpreter lock)
        try:
            for it in range(count):
                t_issue = time.perf_counter()
                h = R.rasp_load_batch(ctxs[c].handle, desc)
                R.rasp_run(ctxs[c].handle, h, budget)
                R.rasp_fetch_outputs_into(ctxs[c].handle, h, outs[c], device=True)
                if keep_last and it == count - 1:
                    kept[c] = h
                else:
                    R.rasp_free_batch(ctxs[c].handle, h)
                lat.append(time.perf_counter() - t_issue)
        except Exception as e:                          # re-raised by run()
            errors.append(e)

    def run(steps, keep_last=False):
        lat, errors = [[] for _ in range(n)], []
        threads = [threading.Thread(target=drive, args=(c, steps // n + (c < steps % n), lat[c], errors,
                                                        keep_last))
                   for c in range(n)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if errors:
            raise errors[0]
        return np.array([x for part in lat for x in part])

    run(max(warmup, n))
    torch.cuda.synchronize()
    for c in ctxs:
        c.set(R.RASP_OPT_PROFILE, 1)
        R.rasp_kernel_times(c.handle)                   # reset
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    lat = run(steps, keep_last=ref_digest is not None)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    # kernel times of the timed region, summed over the contexts (HIP events
    # on each context's own stream)
    kt = {}
    for c in ctxs:
        for k, (ms, cnt) in R.rasp_kernel_times(c.handle).items():
            a, b = kt.get(k, (0.0, 0))
            kt[k] = (a + ms, b + cnt)
        c.set(R.RASP_OPT_PROFILE, 0)
    if verify and args.verify != "none":
        for c in range(n):
            for k in ("status", "steps", "i", "a", "u0", "y0"):
                got = outs[c][k].cpu().numpy()
                if not np.array_equal(got.astype(getattr(ref, k).dtype), getattr(ref, k)):
                    raise SystemExit("bench: NOT bit-exact with %d batches in flight: %s" % (n, k))
            if not np.array_equal(outs[c]["y"].cpu().numpy(), ref.Y):
                raise SystemExit("bench: NOT bit-exact with %d batches in flight: output words" % n)
            if kept[c] is not None:
                dg = {"mem_digest": torch.empty(N, dtype=torch.int64, device=dev)}
                R.rasp_fetch_outputs_into(ctxs[c].handle, kept[c], dg, device=True)
                R.rasp_free_batch(ctxs[c].handle, kept[c])
                kept[c] = None
                if not np.array_equal(dg["mem_digest"].cpu().numpy().view(np.uint64), ref_digest):
                    raise SystemExit("bench: NOT bit-exact with %d batches in flight: memory digests" % n)
    for c in range(n):
        if kept[c] is not None:
            R.rasp_free_batch(ctxs[c].handle, kept[c])
    for c in ctxs:
        if c is not ctx:
            c.close()
    knobs = dict(current_knobs(R, ctx, args.lazy), batches_in_flight=n, cu_partition=args.inflight_cus)
    res = {"batches_in_flight": n, "cus": args.inflight_cus, "value": total_steps / (wall / steps),
           "ms_per_step": 1e3 * wall / steps,
           "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "bit_exact": args.verify != "none", "kernels": kt, "knobs": knobs}
    if quiet:
        return res
    print("bench: inflight=%d %.3f ms/step  %.3e steps/s  batch latency p50 %.3f p99 %.3f ms  kernels %s" % (
        n, res["ms_per_step"], res["value"], res["p50_ms"], res["p99_ms"],
        {k: "%.3f ms x%d" % (v[0] / max(1, v[1]), v[1]) for k, v in kt.items() if v[1]}), flush=True)
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the hot path is data-parallel over "
              "independent machines and this build has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "serve":
        serve_bench(args)
        return

    import torch
    import oracle
    from paper_2604_12902_amd import rasp as R

    t_gen = time.time()
    batch = make_batch(args)
    budget = batch.budget
    gen_s = time.time() - t_gen
    print("bench: workload %s N=%d budget=%d (generated in %.1f s, sha256 %s)" % (
        args.workload, batch.N, budget, gen_s, batch.sha256()[:16]), flush=True)

    # ---- CPU oracle: the reference result and the CPU baseline ----
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 64))
    # c0 is built outside the timer: the baseline times the step loop only
    ref = oracle.init(batch)
    t0 = time.time()
    mix = oracle.advance_mix(ref, budget, threads=cores)
    cpu_s = time.time() - t0
    total_steps = int(ref.steps.sum())
    bstep = bytes_per_step(mix)
    print("bench: oracle %d threads %.2f s, %d retired steps, %.2f algorithmic B/step" % (
        cores, cpu_s, total_steps, bstep), flush=True)
    one = None
    if not args.no_cpu_baseline:
        # one host thread on every cores-th machine: about the CPU work of the run above
        sub = batch.subset(np.arange(0, batch.N, cores))
        st1 = oracle.init(sub)
        t1 = time.time()
        oracle.advance(st1, budget, threads=1)
        one_s = time.time() - t1
        one = {"value": float(st1.steps.sum()) / one_s,
               "sample": "every %d-th machine (%d machines, %d retired steps), 1 host thread"
                         % (cores, sub.N, int(st1.steps.sum()))}
        print("bench: oracle 1 thread %.2f s on %d machines: %.3e steps/s" % (
            one_s, sub.N, one["value"]), flush=True)

    dev = torch.device("cuda", 0)
    # inputs resident in HBM; c0 is packed by rasp_load_batch (with --lazy the
    # first launch of the run builds it)
    desc = R.make_desc(batch, dev, lazy=args.lazy)
    N = batch.N
    outs = dict(status=torch.empty(N, dtype=torch.uint8, device=dev),
                steps=torch.empty(N, dtype=torch.int64, device=dev),
                i=torch.empty(N, dtype=torch.int32, device=dev),
                a=torch.empty(N, dtype=torch.int32, device=dev),
                u0=torch.empty(N, dtype=torch.int32, device=dev),
                y0=torch.empty(N, dtype=torch.int32, device=dev),
                y=torch.empty(int(batch.out_cap.astype(np.int64).sum()), dtype=torch.int32, device=dev))
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    fp = R.rasp_batch_footprint(desc)
    # tune on the whole batch (up to 4M machines): occupancy effects only show
    # at the batch's real size
    tune_vms = min(N, 1 << 22)
    # the batch, its autotune snapshot and trial copy of a prefix, room to
    # stage a dense memory dump for the verification fetch, and slack
    arena = int(fp * (2.25 + 2.0 * tune_vms / N)) + (256 << 20)
    ctx = R.Context(arena)
    torch.cuda.synchronize()

    # knobs: from the autotune cache when it holds this device, batch and
    # library code, else searched (untimed) and stored there
    from paper_2604_12902_amd import tune_cache
    props = torch.cuda.get_device_properties(0)
    cache_key = tune_cache.make_key(getattr(props, "gcnArchName", "unknown"), props.multi_processor_count,
                                    batch, budget, extra="lazy=%d cus=%s" % (args.lazy, args.inflight_cus))
    cache_path = args.tune_cache or tune_cache.PATH
    cached = None if (args.retune or args.no_autotune) else tune_cache.get(cache_key, cache_path)
    tuned = None
    if cached is not None:
        tuned = cached["autotune"]
        print("bench: knobs from the autotune cache: %s" % cached, flush=True)
    elif not args.no_autotune:
        # the library's autotuner picks the knobs on a snapshot (untimed)
        h = R.rasp_load_batch(ctx.handle, desc)
        tuned = R.rasp_autotune(ctx.handle, h, budget, max_vms=tune_vms)
        R.rasp_free_batch(ctx.handle, h)
        print("bench: autotune chose %s" % tuned, flush=True)

    def configure(schedule):
        if tuned is not None and schedule == R.RASP_SCHED_PERSISTENT:
            ctx.set(R.RASP_OPT_LDS_WORDS, tuned["lds_words"])
            ctx.set(R.RASP_OPT_FIRST_PASS, tuned["first_pass"])
            ctx.set(R.RASP_OPT_EPOCH, tuned["epoch"])
            ctx.set(R.RASP_OPT_WAVES_PER_CU, tuned["waves_per_cu"])
            ctx.set(R.RASP_OPT_FIRST_PASS_KIND, tuned["first_pass_kind"])
            ctx.set(R.RASP_OPT_HOT_CELLS, tuned.get("hot_cells", 0))
            ctx.set(R.RASP_OPT_PROFILE_STEPS, tuned.get("profile_steps", 256))
            ctx.set(R.RASP_OPT_MISFIT_WAVES, tuned.get("misfit_waves", 6))
        ctx.set(R.RASP_OPT_SCHEDULE, schedule)
        if args.first_pass is not None:
            ctx.set(R.RASP_OPT_FIRST_PASS, args.first_pass)
        if args.lds_words is not None:
            ctx.set(R.RASP_OPT_LDS_WORDS, args.lds_words)
        if args.epoch is not None:
            ctx.set(R.RASP_OPT_EPOCH, args.epoch)
        if args.waves_per_cu is not None:
            ctx.set(R.RASP_OPT_WAVES_PER_CU, args.waves_per_cu)
        if args.first_pass_kind is not None:
            ctx.set(R.RASP_OPT_FIRST_PASS_KIND, args.first_pass_kind)
        if args.hot_cells is not None:
            ctx.set(R.RASP_OPT_HOT_CELLS, args.hot_cells if schedule == R.RASP_SCHED_PERSISTENT else 0)
        if args.profile_steps is not None:
            ctx.set(R.RASP_OPT_PROFILE_STEPS, args.profile_steps)
        if args.misfit_waves is not None:
            ctx.set(R.RASP_OPT_MISFIT_WAVES, args.misfit_waves)

    def one_step(keep=False):
        h = R.rasp_load_batch(ctx.handle, desc)
        R.rasp_run(ctx.handle, h, budget)
        R.rasp_fetch_outputs_into(ctx.handle, h, outs, device=True)
        if keep:
            return h
        R.rasp_free_batch(ctx.handle, h)
        return None

    def timed(schedule):
        configure(schedule)
        for _ in range(args.warmup):
            one_step()
        torch.cuda.synchronize()
        ctx.set(R.RASP_OPT_PROFILE, 1)
        R.rasp_kernel_times(ctx.handle)                 # reset
        per = []
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(args.steps):
            s0 = time.perf_counter()
            one_step()
            per.append(time.perf_counter() - s0)        # fetch_outputs waits for the step
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        kt = R.rasp_kernel_times(ctx.handle)
        ctx.set(R.RASP_OPT_PROFILE, 0)
        return wall, np.array(per), kt

    def verify():
        h = one_step(keep=True)
        got = R.rasp_fetch_outputs(ctx.handle, h, mem=(args.verify == "full"))
        R.rasp_free_batch(ctx.handle, h)
        for k in ("status", "steps", "i", "a", "u0", "y0"):
            if not np.array_equal(got[k], getattr(ref, k)):
                bad = np.flatnonzero(got[k] != getattr(ref, k))
                raise SystemExit("bench: NOT bit-exact: %s differs at %d machines (first %s)" % (
                    k, bad.size, bad[:5]))
        if not np.array_equal(got["y"], ref.Y):
            raise SystemExit("bench: NOT bit-exact: output words differ")
        if args.verify == "full" and not np.array_equal(got["mem"], ref.mem):
            raise SystemExit("bench: NOT bit-exact: memory differs")

    results = {}
    for name, sched in (("persistent", R.RASP_SCHED_PERSISTENT), ("plain", R.RASP_SCHED_PLAIN)):
        if name == "plain" and args.no_plain:
            continue
        wall, per, kt = timed(sched)
        knobs = current_knobs(R, ctx, args.lazy)
        if args.verify != "none":
            verify()
        ms = 1e3 * wall / args.steps
        results[name] = dict(ms_per_step=ms, value=total_steps / (wall / args.steps),
                             p50_ms=float(np.percentile(per, 50) * 1e3),
                             p99_ms=float(np.percentile(per, 99) * 1e3), kernels=kt, knobs=knobs)
        print("bench: %-10s %.3f ms/step  %.3e steps/s  p50 %.3f p99 %.3f ms  kernels %s" % (
            name, ms, results[name]["value"], results[name]["p50_ms"], results[name]["p99_ms"],
            {k: "%.3f ms x%d" % (v[0] / max(1, v[1]), v[1]) for k, v in kt.items() if v[1]}),
            flush=True)

    inflight = None
    n_flight = args.inflight
    configure(R.RASP_SCHED_PERSISTENT)                  # the knobs the contexts copy
    from_cache = cached is not None and n_flight == 0
    if from_cache:
        n_flight = int(cached["inflight"])
        if args.first_pass is None:
            ctx.set(R.RASP_OPT_FIRST_PASS, int(cached["inflight_first_pass"]))
        if args.epoch is None:
            ctx.set(R.RASP_OPT_EPOCH, int(cached["inflight_epoch"]))
        if args.hot_cells is None and "inflight_hot_cells" in cached:
            ctx.set(R.RASP_OPT_HOT_CELLS, int(cached["inflight_hot_cells"]))
        if args.misfit_waves is None and "inflight_misfit_waves" in cached:
            ctx.set(R.RASP_OPT_MISFIT_WAVES, int(cached["inflight_misfit_waves"]))
    if n_flight == 0:
        # batches in flight chosen like the other knobs: a short untimed trial
        # of each candidate (2n batches after n warm-up ones); a larger count
        # must be at least 3% faster
        best = None
        for cand in INFLIGHT_CANDIDATES:
            if cand == 1:
                rate = results["persistent"]["value"]
            else:
                rate = timed_inflight(args, R, torch, ctx, desc, batch, budget, arena_inflight(fp), ref,
                                      total_steps, cand, steps=2 * cand, warmup=cand, verify=False,
                                      quiet=True)["value"]
            print("bench: trial %d in flight: %.3e steps/s" % (cand, rate), flush=True)
            if best is None or rate > best[1] / 0.97:
                best = (cand, rate)
        n_flight = best[0]
    if n_flight > 1 and not from_cache:
        # the autotuner picks the first-pass length and the epoch one batch
        # at a time on the whole chip, where the first pass's survivors may
        # all fit the resident lanes; on a 1/n share of the CUs the first pass
        # takes n times as long and the survivors may not fit, so finished
        # lanes wait for the next refill check.  Both are tried again with the
        # batches in flight, one after the other (the current value stays
        # unless another is at least 3% faster); a knob given on the command
        # line is kept.
        retune = []
        # (a hot-cell first pass is as long as its profile needs: kept)
        if args.first_pass is None and int(ctx.get(R.RASP_OPT_HOT_CELLS)) == 0:
            retune.append(("first pass", R.RASP_OPT_FIRST_PASS, INFLIGHT_FIRST_PASSES))
        if args.epoch is None:
            retune.append(("epoch", R.RASP_OPT_EPOCH, INFLIGHT_EPOCHS))
        if int(ctx.get(R.RASP_OPT_HOT_CELLS)) > 0:
            if args.hot_cells is None:
                retune.append(("hot cells", R.RASP_OPT_HOT_CELLS, INFLIGHT_HOT_CELLS))
            if args.misfit_waves is None:
                retune.append(("misfit waves", R.RASP_OPT_MISFIT_WAVES, INFLIGHT_MISFIT_WAVES))
        moved = False
        last = None
        for name, opt, cands in retune:
            cur = int(ctx.get(opt))
            best = None
            for v in (cur,) + tuple(x for x in cands if x != cur):
                ctx.set(opt, v)
                rate = timed_inflight(args, R, torch, ctx, desc, batch, budget, arena_inflight(fp), ref,
                                      total_steps, n_flight, steps=4 * n_flight, warmup=n_flight,
                                      verify=False, quiet=True)["value"]
                print("bench: trial %s %d with %d in flight: %.3e steps/s" % (name, v, n_flight, rate),
                      flush=True)
                if best is None or rate > best[1] / 0.97:
                    best = (v, rate)
            ctx.set(opt, best[0])
            moved |= best[0] != cur
            last = best[1]
        # a knob that moved can change which count in flight is best (a
        # table size chosen one batch at a time may lose on a CU share):
        # the other counts are tried once more with the retuned knobs
        if moved and args.inflight == 0:
            best = (n_flight, last)
            for cand in INFLIGHT_CANDIDATES:
                if cand in (1, n_flight):
                    continue
                rate = timed_inflight(args, R, torch, ctx, desc, batch, budget, arena_inflight(fp), ref,
                                      total_steps, cand, steps=4 * cand, warmup=cand, verify=False,
                                      quiet=True)["value"]
                print("bench: trial %d in flight, retuned knobs: %.3e steps/s" % (cand, rate), flush=True)
                if rate > best[1] / 0.97:
                    best = (cand, rate)
            n_flight = best[0]
    if tuned is not None and cached is None and args.inflight == 0:
        tune_cache.put(cache_key, {"autotune": tuned, "inflight": n_flight,
                                   "inflight_first_pass": int(ctx.get(R.RASP_OPT_FIRST_PASS)),
                                   "inflight_epoch": int(ctx.get(R.RASP_OPT_EPOCH)),
                                   "inflight_hot_cells": int(ctx.get(R.RASP_OPT_HOT_CELLS)),
                                   "inflight_misfit_waves": int(ctx.get(R.RASP_OPT_MISFIT_WAVES))},
                       cache_path)
    if n_flight > 1:
        inflight = timed_inflight(args, R, torch, ctx, desc, batch, budget, arena_inflight(fp), ref,
                                  total_steps, n_flight,
                                  ref_digest=oracle.digest(ref) if args.verify == "full" else None)

    # the headline: the persistent schedule with the batches in flight the
    # run was asked for (one: results["persistent"])
    head = inflight if inflight is not None else results["persistent"]
    kt = head["kernels"]
    # dominant kernel of the headline schedule: largest total time; with
    # hot-cell tables the fits' and the misfits' launches run side by side
    # over the survivors of the first pass, and count as one (their common
    # span is the longer of the two)
    dom = max((k for k in kt if kt[k][1] > 0), key=lambda k: kt[k][0])
    dom_ms = kt[dom][0] / kt[dom][1]
    if kt.get("misfit", (0, 0))[1] and kt["persistent"][1] and dom in ("persistent", "misfit"):
        dom = "persistent+misfit"
        dom_ms = max(kt["persistent"][0] / kt["persistent"][1], kt["misfit"][0] / kt["misfit"][1])
    fp_pass = head["knobs"]["first_pass"]
    # which launch built c0: the pack kernel, the first pass (plain or LDS
    # persistent kernel) or the persistent kernel itself
    first_kind = "first" if kt["first"][1] else ("plain" if kt["plain"][1] else None)
    if first_kind is None:
        fp_pass = 0
    c0_in = "pack" if kt["pack"][1] else (first_kind or "persistent")
    steps_first = int(np.minimum(ref.steps.astype(np.int64), fp_pass).sum())
    c0_note = "c0 built in the launch (programs + inputs read, n+l+s words + 25 B scalars written per machine)"
    if dom == "pack":
        algo = pack_bytes(batch)
        unit_note = "c0 bytes: programs + inputs read, n+l+s words + 25 B scalars written per machine"
    elif dom == first_kind:
        if c0_in == dom:
            algo = pack_bytes(batch) + bstep * steps_first + 25.0 * N
            unit_note = "%s + %.2f B per retired step + 25 B final state per machine" % (c0_note, bstep)
        else:
            algo = bstep * steps_first + 50.0 * N
            unit_note = "%.2f B per retired step x steps retired by the launch + 50 B state per machine" % bstep
    elif dom == "persistent" and c0_in == "persistent":
        algo = pack_bytes(batch) + bstep * total_steps + 25.0 * N
        unit_note = "%s + %.2f B per retired step + 25 B final state per machine" % (c0_note, bstep)
    elif dom in ("persistent", "persistent+misfit"):
        algo = bstep * (total_steps - steps_first) + 50.0 * int((ref.steps > fp_pass).sum())
        unit_note = "%.2f B per retired step x steps retired by the launch + 50 B state per machine" % bstep
    else:
        algo = 0.0
        unit_note = "n/a"
    achieved = algo / (dom_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, dom, head["knobs"])
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
            "kernel": dom, "kernel_ms": round(dom_ms, 4), "algorithmic_bytes": int(algo),
            "per_unit": unit_note,
            # the whole path: retired steps/s x algorithmic bytes per step against the peak
            "path_frac": round(head["value"] * bstep / (HBM_PEAK_GBS * 1e9), 5)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = {"value": total_steps / cpu_s, "unit": "VM instructions retired/s", "cores": cores,
               "kind": "oracle",
               "sample": "the whole batch (%d machines, %d retired steps), %d host threads, "
                         "static round-robin striping; the step loop timed (c0 built before the "
                         "timer), with the retired-opcode histogram counted" % (N, total_steps, cores),
               "one_thread": one, "cpu_model": cpu_model(), "compiler": oracle_compiler()}

    line = {
        "metric": "VM instructions retired/sec (1 GPU), bit-exact; persistent vs plain; p50/p99",
        "value": head["value"], "unit": "VM instructions retired/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded random RASP programs)",
        "config": {"workload": batch.name, "num_vms": N, "budget": budget,
                   "retired_steps_per_batch": total_steps, "schedule": "persistent",
                   "first_pass": fp_pass, "lds_words": head["knobs"]["lds_words"],
                   "c0_in_run": args.lazy, "autotuned": tuned is not None, "knobs_from_cache": cached is not None,
                   "epoch": head["knobs"]["epoch"], "waves_per_cu": head["knobs"]["waves_per_cu"],
                   "first_pass_kind": head["knobs"]["first_pass_kind"],
                   "batches_in_flight": n_flight if inflight is not None else 1,
                   "cu_partition": args.inflight_cus if inflight is not None else "shared"},
        # p50/p99: per-batch latency, load issued to outputs fetched
        "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
        "single_batch": {k: results["persistent"][k] for k in ("value", "ms_per_step", "p50_ms", "p99_ms")},
        "plain": ({k: results["plain"][k] for k in ("value", "ms_per_step", "p50_ms", "p99_ms")}
                  if "plain" in results else None),
        "bit_exact": args.verify,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if args.json_extra:
        with open(args.json_extra, "w") as f:
            json.dump(dict(line=line, results={k: {kk: vv for kk, vv in v.items()}
                                               for k, v in results.items()}), f, indent=1)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
