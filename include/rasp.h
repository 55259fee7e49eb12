/*
 * rasp.h -- C ABI of librasp, a GPU hypervisor for word-RASP machines on
 * AMD MI355X (gfx950).
 *
 * The library advances many independent RASP machines in lockstep: the lifted
 * transition map Phi : C^d -> C^d of Sec. 2 ("Method"), each coordinate being
 * the one-step transition of the word RASP (Sec. 2.1) or of the classic RASP
 * (Sec. 1.1).  A machine's configuration is <i, a, M, u, y>: instruction
 * counter, accumulator, n memory words holding the program and its data,
 * the input tape (pointer u0 and l words) and the output (count y0 and s
 * words).  A machine halts when it reaches a fixed point (F = { c : c -> c },
 * Sec. 1.1 and Sec. 2.1).
 *
 * Conventions for every call:
 *   - the return value is RASP_OK (0) or a negative RASP_E_* code; no C++
 *     exception crosses this boundary; rasp_last_error() describes the last
 *     failure on a context;
 *   - RASP_E_INVAL leaves the context and all batches exactly as they were;
 *   - RASP_E_DEVICE (a HIP runtime error) is sticky: the context refuses all
 *     further work except rasp_last_error and rasp_destroy;
 *   - a context is driven by one host thread at a time; different contexts
 *     (each with its own stream, which may carry a CU mask) may be driven
 *     from different host threads at the same time;
 *   - words are w-bit two's complement, w = word_bits of the batch (32 by
 *     default, the w = 32 of Sec. 3); + and * wrap mod 2^w.
 *
 * Semantics fixed by this library where the paper leaves a choice:
 *   - the program is stored in memory: P occupies M[0 .. 2m), n >= 2m words
 *     in total (Sec. 2: each machine stores its program in memory; Sec. 2.1:
 *     P in W^(2m <= n), c0 = <0, 0, P 0^(n-2m), x 0^(l-|x|), 0^(s+1)>);
 *   - memory is addressed circularly by the Euclidean remainder of the signed
 *     word, M[v mod n] with v mod n in [0, n), for fetch (<M[i mod n],
 *     M[(i+1) mod n]>, Sec. 2.1) and for data;
 *   - LOAD is immediate (a <- j) in both instruction sets;
 *   - READ stores tape word u0 (0-based) into M[j mod n] and increments u0; it
 *     is a fixed point once u0 >= l (Sec. 2.1 guard);
 *   - PRINT appends M[j mod n] while y0 < s and is otherwise a no-op that still
 *     advances i (Sec. 2.1, y :: z);
 *   - a taken jump is a fixed point exactly when its target word equals i;
 *   - a retired step is a transition that changes the configuration; a run of
 *     budget B applies exactly min(B, steps to the fixed point) transitions
 *     (the halting number tau_h of Sec. 3 when it is below B).
 */
#ifndef RASP_H
#define RASP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RASP_ABI_VERSION 4u

typedef struct rasp_ctx rasp_ctx;
typedef uint64_t rasp_batch;                 /* 0 is never a valid handle */

enum {
    RASP_OK = 0,
    RASP_E_INVAL = -1,     /* bad argument or descriptor; nothing changed   */
    RASP_E_NOMEM = -2,     /* the context's arena cannot hold the request   */
    RASP_E_DEVICE = -3,    /* HIP runtime error; sticky for the context     */
    RASP_E_STATE = -4,     /* unknown or freed handle, wrong call order     */
    RASP_E_BUSY = -5       /* resource in use by queued work                */
};

/* Instruction sets.  Both keep the paper's opcode numbers. */
enum {
    RASP_ISA_WORD = 0,     /* Sec. 2.1: 1 LOD, 2 ADD, 3 MUL, 4 STO, 5 BNZ (jump if a != 0),
                              6 RD, 7 PRI; every other value is stuck (halts)          */
    RASP_ISA_CLASSIC = 1   /* Sec. 1.1: 1 LOAD, 2 ADD, 3 SUB, 4 STORE, 5 JPOS (jump if
                              a > 0, signed), 6 READ, 7 PRINT; plus 8 JMP (the JMP of
                              Sec. 2.2 as one instruction); 0 (HALT, the pair 0 0 of
                              Sec. 2.2) and every other value is stuck                 */
};

enum { RASP_RUNNING = 0, RASP_HALTED = 1 };

/* rasp_batch_desc.flags */
enum {
    RASP_DESC_DEVICE_PTRS = 1u,  /* every array of the descriptor is device memory */
    RASP_DESC_LAZY = 2u          /* with DEVICE_PTRS: build c0 inside the first rasp_run
                                    (each machine's c0 is written straight into its LDS
                                    slot by the step kernel and then to the arena); the
                                    descriptor arrays are read until that run, or the
                                    first call that needs the state, has finished */
};

/* rasp_outputs.flags */
enum {
    RASP_OUT_DEVICE_PTRS = 1u,       /* every destination is device memory */
    RASP_OUT_ASYNC = 2u              /* rasp_fetch_outputs queues the fetch and returns */
};

/*
 * rasp_create: open a context on HIP device `device`.
 *   arena, arena_bytes: device memory the context sub-allocates batches from.
 *     If arena is NULL the library allocates arena_bytes itself (hipMalloc) and
 *     frees them in rasp_destroy; otherwise the caller owns the buffer (e.g. a
 *     torch tensor) and must keep it alive until rasp_destroy returns.
 *   stream: the hipStream_t all work of this context is queued on (NULL: the
 *     context creates its own).  The caller keeps a passed stream alive.
 * Errors: INVAL (out == NULL, arena_bytes < 1 MiB), DEVICE.
 */
int rasp_create(rasp_ctx **out, int device, void *arena, uint64_t arena_bytes,
                void *stream);

/*
 * rasp_create_on_cus: rasp_create on a stream the library creates, restricted
 * by a CU mask (hipExtStreamCreateWithCUMask) to compute units
 * [cu_first, cu_first + cu_count) of the device; rasp_destroy destroys it.
 * Several contexts on disjoint CU ranges, each driven from its own host
 * thread, run independent batches side by side: one batch's latency-bound
 * tail then does not share SIMDs with another batch's bandwidth-bound load.
 * Each such stream takes a hardware queue of its own (HIP gives a process 4
 * by default).  arena, arena_bytes as for rasp_create.
 * Errors: INVAL (out == NULL, cu_count == 0, or the range not within the
 * device's compute units), DEVICE (the runtime refused the mask), and those
 * of rasp_create.
 */
int rasp_create_on_cus(rasp_ctx **out, int device, void *arena, uint64_t arena_bytes,
                       uint32_t cu_first, uint32_t cu_count);

/* rasp_destroy: wait for queued work, release the context (NULL is a no-op). */
int rasp_destroy(rasp_ctx *ctx);

/* rasp_last_error: message for the last failing call on ctx ("" if none).
 * Valid until the next call on ctx.  ctx may be NULL (message of the last
 * failed rasp_create). */
const char *rasp_last_error(const rasp_ctx *ctx);

/*
 * A batch of machines in packed form.  Machine v (0 <= v < num_vms):
 *   program words  prog[prog_off[v] .. prog_off[v+1])      (2 m_v words: opcode,
 *                                                             operand, ...)
 *   memory size    n_v = mem_words ? mem_words[v] : default_mem_words,
 *                  1 <= n_v <= 2^30 and n_v >= 2 m_v
 *   input x_v      tape[tape_off[v] .. tape_off[v+1])
 *   tape capacity  l_v = tape_cap ? tape_cap[v] : |x_v|, l_v >= |x_v|
 *   output cap.    s_v = out_cap ? out_cap[v] : default_out_cap
 * prog_off and tape_off hold num_vms + 1 non-decreasing entries.
 * With RASP_DESC_DEVICE_PTRS every pointer is device memory on the context's
 * device; otherwise host memory.  The arrays are only read, and only until the
 * call that takes the descriptor returns (host) or until the work it queues
 * has finished on the context stream (device; with RASP_DESC_LAZY until the
 * batch's first run or fetch has finished).
 * Word width (Sec. 2.1, W = F_2^w): word_bits w in [2, 32] (0 means 32).
 * Every word of the machine is then a w-bit two's-complement value held
 * sign-extended in an int32: ADD, SUB, MUL and the advance i + 2 (and the
 * operand position i + 1) wrap mod 2^w.  Program and input words must already
 * be w-bit values (RASP_E_INVAL otherwise); App. B's halting numbers are
 * quoted at w = 29.
 */
typedef struct {
    uint32_t abi_version;            /* RASP_ABI_VERSION */
    uint32_t isa;                    /* RASP_ISA_* */
    uint64_t num_vms;                /* >= 1 */
    const int32_t *prog;
    const uint64_t *prog_off;
    const uint32_t *mem_words;       /* NULL: default_mem_words for every machine */
    uint32_t default_mem_words;
    uint32_t default_out_cap;
    const int32_t *tape;
    const uint64_t *tape_off;
    const uint32_t *tape_cap;        /* NULL: l_v = |x_v| */
    const uint32_t *out_cap;         /* NULL: default_out_cap */
    uint32_t flags;                  /* RASP_DESC_* */
    uint32_t word_bits;              /* w: 0 or 32 for 32-bit words, else 2..31 */
} rasp_batch_desc;

/*
 * Per-machine results.  Every pointer may be NULL (that field is not
 * fetched).  Layouts: the scalar arrays hold num_vms entries; y holds
 * sum_v s_v words, machine-major (machine v's s_v words after those of
 * machines 0..v-1), zero beyond y0; mem holds sum_v n_v words, machine-major;
 * mem_digest holds num_vms FNV-1a-64 hashes of each machine's n_v memory
 * words taken as little-endian bytes.  Host memory unless flags has
 * RASP_OUT_DEVICE_PTRS.  For rasp_load_state the same struct carries a state
 * to load (status is ignored, mem is required, y and steps may be NULL).
 */
typedef struct {
    uint8_t *status;                 /* RASP_RUNNING / RASP_HALTED: is c a fixed point */
    uint64_t *steps;                 /* transitions retired since load (cumulative) */
    int32_t *i;
    int32_t *a;
    uint32_t *u0;
    uint32_t *y0;
    int32_t *y;
    int32_t *mem;
    uint64_t *mem_digest;
    uint32_t flags;                  /* RASP_OUT_* */
    uint32_t reserved;
} rasp_outputs;

/*
 * rasp_batch_footprint: bytes of arena a batch with this descriptor occupies
 * (state, shapes and the n + l + s words of every machine), for admission
 * control.  Pure: touches no context.  A device descriptor is read with
 * synchronous copies on the null stream.
 * Errors: INVAL (malformed descriptor).
 */
int rasp_batch_footprint(const rasp_batch_desc *d, uint64_t *bytes);

/*
 * rasp_load_batch: allocate a batch in the arena and build c0(P_v, x_v) for
 * every machine (Sec. 2.1): i = a = 0, M = P 0^(n-2m), tape = x 0^(l-|x|),
 * u0 = y0 = 0, y = 0^s, steps = 0; status = whether c0 is already a fixed
 * point.  All or nothing: on error no batch exists.  Queues work on the
 * context stream and waits only for the descriptor checks.
 * Errors: INVAL (descriptor), NOMEM (arena), DEVICE.
 */
int rasp_load_batch(rasp_ctx *ctx, const rasp_batch_desc *d, rasp_batch *out);

/*
 * rasp_load_state: like rasp_load_batch (the descriptor gives shapes, tapes and
 * the isa; its program words are ignored beyond validation), then overwrite
 * every machine's i, a, u0, y0, steps, y and memory from `state` (host or
 * device per state->flags).  status is recomputed.  u0 <= l and y0 <= s are
 * required, and with w < 32 every word (i, a, memory, output) must be a
 * w-bit value.  Used to resume from a checkpoint and to test arbitrary states.
 * Errors: INVAL, NOMEM, DEVICE.
 */
int rasp_load_state(rasp_ctx *ctx, const rasp_batch_desc *d, const rasp_outputs *state,
                    rasp_batch *out);

/*
 * rasp_run: queue the advance of every machine of batch b by at most `budget`
 * more transitions (Phi^budget, Sec. 2).  Runs compose: run(b1) then run(b2)
 * equals run(b1 + b2).  Halted machines never change.  Returns once the work
 * is queued; use rasp_sync / rasp_fetch_outputs to wait.
 * Errors: STATE (bad handle), DEVICE.
 */
int rasp_run(rasp_ctx *ctx, rasp_batch b, uint64_t budget);

/*
 * rasp_run_multi: one persistent launch that advances k batches together,
 * batch bs[t] by at most budgets[t] transitions (continuous batching: machines
 * of every batch share the device work queue).  k <= 64.  Equivalent to
 * rasp_run on each batch in turn.
 * Errors: INVAL (k), STATE, DEVICE.
 */
int rasp_run_multi(rasp_ctx *ctx, const rasp_batch *bs, const uint64_t *budgets, uint32_t k);

/*
 * rasp_run_async: the same call as rasp_run_multi under the name a serving
 * loop uses for it (one launch over k batches, returning once queued; wait
 * with rasp_poll / rasp_sync per batch or rasp_running_counts_async).
 */
int rasp_run_async(rasp_ctx *ctx, const rasp_batch *bs, const uint64_t *budgets, uint32_t k);

/*
 * rasp_run_noalloc: rasp_run for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * allocation).  The same kernels and results as rasp_run, but the queue
 * counters, batch tables and first-pass survivor list live in one fixed
 * device array of the library (16 MiB per GPU, held until the process ends)
 * instead of the context arena; the call allocates nothing, creates no
 * events (kernel timing is off for it) and never captures a graph.  The
 * batch (inputs and outputs) is the caller's, loaded as usual.  Every call on
 * one GPU shares that array: calls that overlap on one GPU, from any context
 * or thread, race and must be serialised by the caller.  The queue counters
 * are cleared by a fill kernel at the start of every launch.
 * Limit: at most 4,194,304 machines in the batch.
 * Errors: INVAL (batch above the limit), STATE (bad handle), DEVICE.
 */
int rasp_run_noalloc(rasp_ctx *ctx, rasp_batch b, uint64_t budget);

/*
 * rasp_poll: *done = 1 when the work queued so far for batch b (its load and
 * runs) has finished, else 0; never waits.  b = 0 asks about all work queued
 * on the context.
 * Errors: INVAL (done NULL), STATE (bad handle), DEVICE.
 */
int rasp_poll(rasp_ctx *ctx, rasp_batch b, int *done);

/*
 * rasp_sync: wait until the work queued so far for batch b has finished
 * (b = 0: all work queued on the context).
 * Errors: STATE (bad handle), DEVICE.
 */
int rasp_sync(rasp_ctx *ctx, rasp_batch b);

/*
 * rasp_fetch_outputs: wait for the batch's queued work, then copy the requested
 * fields into caller-owned buffers (layouts above): each machine's
 * configuration after the transitions applied so far, Phi^tau(c0) of Sec. 2
 * (i, a, memory M, tape head u0, output head y0 and the output words y that
 * PRINT appended, Sec. 1.1 and 2.1), whether it is at a fixed point (status:
 * F of Sec. 1.1/2.1) and how many transitions it retired.
 * With RASP_OUT_ASYNC in out->flags the fetch is queued on the context's copy
 * stream (created on first use, on the context's compute units), behind the
 * work already queued for the batch, and the call returns at once: the fields
 * are in place when rasp_poll reports the batch done or rasp_sync returns.
 * Host destinations must then be page-locked (hipHostMalloc, pinned torch
 * tensors) for the copies to run in the background, and stay valid until
 * then.  mem cannot be fetched this way.  Digests go through a buffer of the
 * batch (8 bytes a machine of arena, taken at its first asynchronous fetch,
 * returned with the batch).  Later runs of the batch are ordered after the
 * fetch, and rasp_free_batch waits for it.  A serving loop hands one
 * request's results back this way while the next epoch of the others runs.
 * Errors: INVAL (mem with RASP_OUT_ASYNC), NOMEM (digest buffer), STATE, DEVICE.
 */
int rasp_fetch_outputs(rasp_ctx *ctx, rasp_batch b, const rasp_outputs *out);

/*
 * rasp_batch_info: num_vms, total memory words, total output words and the
 * retired-step sum of a batch (the sum needs a device reduction and a wait;
 * pass NULL to skip it).
 */
int rasp_batch_info(rasp_ctx *ctx, rasp_batch b, uint64_t *num_vms, uint64_t *mem_words,
                    uint64_t *out_words, uint64_t *steps_sum);

/*
 * rasp_running_counts: for k batches (k <= 64), counts[t] = number of machines
 * of bs[t] not at a fixed point, from one device launch and one wait.  Used by
 * a serving loop to retire requests whose machines have all halted.
 * Errors: INVAL, STATE, DEVICE.
 */
int rasp_running_counts(rasp_ctx *ctx, const rasp_batch *bs, uint32_t k, uint64_t *counts);

/*
 * rasp_running_counts_async: queue the computation of rasp_running_counts for
 * bs[0..k) behind the work queued so far on the context and return at once
 * with a ticket; the counts land in page-locked memory of the context.
 * rasp_running_counts_wait: wait until the counts of `ticket` are there and
 * copy them to counts (k entries); a ticket is claimed once.  At most 4
 * tickets are in flight per context: a fifth request waits for the oldest
 * unclaimed one, which is then dropped (its wait fails with RASP_E_STATE).
 * A serving loop queues the counts right behind an epoch's launch and does
 * its host work (admission, loads, fetches) before it waits.
 * Errors: INVAL (k, NULL pointers), STATE (bad handle or ticket), DEVICE.
 */
int rasp_running_counts_async(rasp_ctx *ctx, const rasp_batch *bs, uint32_t k, uint64_t *ticket);
int rasp_running_counts_wait(rasp_ctx *ctx, uint64_t ticket, uint64_t *counts);

/* rasp_free_batch: release a batch's arena space after its queued work (and
 * after an asynchronous fetch of it still in flight, which it waits for). */
int rasp_free_batch(rasp_ctx *ctx, rasp_batch b);

/*
 * Scheduling knobs (per context).  The library's autotuner sets them; they can
 * also be forced.
 *   RASP_OPT_SCHEDULE      RASP_SCHED_PLAIN: one machine per lane, every lane
 *                          runs its machine to the end, no compaction;
 *                          RASP_SCHED_PERSISTENT: resident waves refill lanes
 *                          of halted machines from a device queue;
 *                          RASP_SCHED_AUTO (default): the autotuned choice.
 *   RASP_OPT_EPOCH         steps a lane runs between refill checks (q), >= 1
 *   RASP_OPT_LDS_WORDS     memory words per machine staged in LDS by the
 *                          persistent kernel (0 = none), a multiple of 4 in
 *                          [4, 1024]; -1 (default): n rounded up to 4 when
 *                          two waves of such slots fit in LDS, else 0
 *   RASP_OPT_WAVES_PER_CU  resident waves per compute unit for the persistent
 *                          kernel
 *   RASP_OPT_GRAPH         1: capture the launch sequence of a run (queue reset,
 *                          plain pass, persistent kernel) once per (batches,
 *                          budgets, knobs) and replay it as a HIP graph; graphs
 *                          of a batch are dropped when it is freed
 *   RASP_OPT_FIRST_PASS    persistent schedule only: transitions every machine
 *                          first runs in a first pass; the machines still
 *                          running then go through the persistent kernel
 *                          (0: persistent kernel only)
 *   RASP_OPT_FIRST_PASS_KIND  0 (default): the first pass is the plain
 *                          kernel (memory in HBM, one machine per lane); 1: the
 *                          persistent kernel with every machine's memory in
 *                          its LDS slot, when every memory fits a slot
 *                          (otherwise the plain kernel)
 *   RASP_OPT_HOT_CELLS     persistent schedule with a plain first pass, memories
 *                          of at most 2,048 words: 0 (default) off; S in
 *                          {8, 16, 32, 64}: the first pass profiles the 2-word
 *                          cells each machine touches in its last
 *                          RASP_OPT_PROFILE_STEPS transitions, and the persistent
 *                          kernel keeps a machine's profiled cells (up to S,
 *                          hashed into S slots) in LDS, every other word in HBM;
 *                          a cell missed later whose slot is empty joins the
 *                          table (replaces RASP_OPT_LDS_WORDS for that launch)
 *   RASP_OPT_PROFILE_STEPS transitions profiled at the end of a hot-cell first
 *                          pass, >= 1 (default 256)
 *   RASP_OPT_MISFIT_WAVES  resident waves per compute unit of the launch that
 *                          runs the survivors of a hot-cell first pass whose
 *                          cells do not fit (memory in HBM, on a second stream
 *                          of the context beside the fits' launch), 1..32
 *                          (default 6)
 */
enum {
    RASP_OPT_SCHEDULE = 1,
    RASP_OPT_EPOCH = 2,
    RASP_OPT_LDS_WORDS = 3,
    RASP_OPT_WAVES_PER_CU = 4,
    RASP_OPT_GRAPH = 5,
    RASP_OPT_FIRST_PASS = 6,
    RASP_OPT_FIRST_PASS_KIND = 8,
    RASP_OPT_HOT_CELLS = 9,
    RASP_OPT_PROFILE_STEPS = 10,
    RASP_OPT_MISFIT_WAVES = 11
};
enum { RASP_SCHED_AUTO = 0, RASP_SCHED_PLAIN = 1, RASP_SCHED_PERSISTENT = 2 };

int rasp_set_option(rasp_ctx *ctx, int option, int64_t value);
int rasp_get_option(rasp_ctx *ctx, int option, int64_t *value);

/*
 * Kernel timing.  With RASP_OPT_PROFILE set to 1 the context records a pair of
 * HIP events on its stream around every kernel it launches.  rasp_kernel_times
 * waits for the stream, then adds the elapsed time (ms) and the launch count
 * of each kernel kind into ms[RASP_KERNEL_COUNT] and launches[RASP_KERNEL_COUNT]
 * (either may be NULL) and forgets the recorded pairs.
 */
enum {
    RASP_KERNEL_PACK = 0,          /* c0 construction                           */
    RASP_KERNEL_PLAIN = 1,         /* one machine per lane step loop            */
    RASP_KERNEL_PERSISTENT = 2,    /* work-queue step loop                      */
    RASP_KERNEL_DIGEST = 3,        /* memory digests                            */
    RASP_KERNEL_OTHER = 4,         /* checks, scans, copies, queue reset        */
    RASP_KERNEL_FIRST = 5,         /* work-queue first pass with LDS memory     */
    RASP_KERNEL_MISFIT = 6,        /* hot-cell misfits' work-queue step loop    */
    RASP_KERNEL_COUNT = 7
};
enum { RASP_OPT_PROFILE = 7 };
int rasp_kernel_times(rasp_ctx *ctx, double *ms, uint64_t *launches);

/*
 * rasp_autotune: choose the scheduling knobs for batches shaped like b.
 * Copies the first min(num_vms, max_vms) machines of b into a scratch batch
 * (b itself is not changed), then times rasp_run(budget) on fresh copies of
 * that snapshot while searching one knob at a time (LDS words per machine,
 * first-pass length, epoch, waves per compute unit, first-pass kind), then
 * hot-cell tables (slots per machine and misfit waves per CU on a grid, then
 * the profile length) when memories have at most 2,048 words, and the plain
 * schedule; keeps the fastest setting in the context and writes it to
 * chosen[0..8] = {schedule, lds_words, first_pass, epoch, waves_per_cu,
 * first_pass_kind, hot_cells, profile_steps, misfit_waves} (chosen may be
 * NULL); a knob leaves its current setting only for a setting at least 3%
 * faster.  Returns the
 * best time in *best_ms (may be NULL).  A lazily loaded batch stays lazy:
 * each trial builds c0 of the prefix again from the descriptor.
 * Errors: STATE, NOMEM (no room for the snapshot), DEVICE.
 */
int rasp_autotune(rasp_ctx *ctx, rasp_batch b, uint64_t budget, uint64_t max_vms,
                  int64_t *chosen, double *best_ms);

/* Device properties the context saw: compute units, LDS bytes per workgroup. */
int rasp_device_info(rasp_ctx *ctx, int *compute_units, int *lds_bytes, int *wave_size);

#ifdef __cplusplus
}
#endif
#endif /* RASP_H */
