// rasp_internal.h -- structures shared by the host runtime and the kernels of
// librasp (never exposed through the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rasp {

constexpr int kWave = 64;              // CDNA wavefront width
constexpr int kMaxMulti = 64;          // batches per multi-batch launch
constexpr uint32_t kMaxMemWords = 1u << 30;
constexpr uint32_t kNoCap = 0xffffffffu;   // a persistent launch that is not a first pass

// Device view of one batch: struct-of-arrays machine state plus the packed
// per-machine shapes and the three word arenas (memory, tape, output), each
// machine's slice contiguous.  Memory slices start on 16-byte boundaries.
struct DevBatch {
    int32_t *i;
    int32_t *a;
    uint32_t *u0;
    uint32_t *y0;
    uint64_t *steps;
    uint8_t *status;
    uint32_t *n;
    uint32_t *ell;
    uint32_t *s;
    uint64_t *mem_off;                 // word offset of M_v in M
    uint64_t *t_off;                   // word offset of tape_v in T
    uint64_t *y_off;                   // word offset of y_v in Y
    // words of M_v at or above hw[v] are zero and not stored (c0's zero tail
    // before anything is written there); a multiple of 4, at most n_v
    // rounded up to 4, which means every word is stored
    uint32_t *hw;
    int32_t *M;
    int32_t *T;
    int32_t *Y;
    uint64_t N;
    uint32_t isa;
    uint32_t fresh;                    // 1: state is c0, built from the packed inputs below
    uint32_t wshift;                   // 32 - w: words are w-bit values, sign-extended
    uint32_t pad;
    const int32_t *prog;               // packed programs / inputs of a fresh batch
    const uint64_t *prog_off;
    const int32_t *tape;
    const uint64_t *tape_off;
};

// Table of batches advanced together by one launch.  Machine g of the launch
// is machine g - start[k] of batch k, for the k with start[k] <= g < start[k+1].
struct BatchTable {
    DevBatch b[kMaxMulti];
    uint64_t start[kMaxMulti + 1];
    uint32_t budget[kMaxMulti];        // transitions this launch may apply per machine
    uint32_t count;
    uint32_t pad;
};

// Counters of one persistent launch (device memory, zeroed by a fill kernel
// before every launch so that the launch can sit in a HIP graph).
struct QueueState {
    unsigned long long head;           // next unclaimed work item
    unsigned long long survivors;      // items appended to the survivor list
    unsigned long long retired;        // transitions retired (statistics)
    unsigned long long pad;
    unsigned long long misfits;        // hot-cell first pass: survivors whose hot cells do not all fit
    unsigned long long head_m;         // next unclaimed misfit
    unsigned long long pad2[2];
};

// Hot-cell tables.  A first pass profiles the last R transitions of every
// machine it leaves running: the 2-word cells (words 2x, 2x + 1) its
// fetches and data accesses touch.  A survivor whose cells can be placed in
// S slots without two sharing one (slot of cell x = bits [16, 16 + log2 S)
// of x * c, c chosen per machine) is a fit; the persistent kernel then keeps
// exactly those cells in LDS and every access of its steady loop is an LDS
// hit.  Fit p of the survivor list has multiplier mult[p] and cells
// tags[p S + s] (0xffff: empty slot); misfits go to a list of their own
// (count q->misfits), run with their memory in HBM by a second persistent
// launch beside the fits' launch, so that no wave mixes the two.
struct HotArgs {
    uint32_t S;                        // slots per machine (power of two, 8..64); 0: off
    uint32_t lgS;
    uint32_t R;                        // profiled transitions at the end of the first pass
    uint32_t bw;                       // profile bitmap words per lane
    uint32_t *mult;
    uint16_t *tags;
    uint32_t *mis;                     // misfit list
};

// Descriptor-check error bits.
enum : uint32_t {
    kErrOffsets = 1u,                  // prog_off / tape_off decreasing
    kErrProgTooLong = 2u,              // 2m > n
    kErrTapeTooLong = 4u,              // |x| > l
    kErrMemSize = 8u,                  // n == 0 or n > 2^30
    kErrStateRange = 16u,              // u0 > l or y0 > s in a loaded state
    kErrWordRange = 32u                // a word outside the w-bit range
};

struct LaunchShape {
    int cus;
    int lds_bytes;
};

// kernel launchers (rasp_kernels.hip)
// Layout of a batch from a device descriptor: n, l, s per machine (b.n,
// b.ell, b.s), the exclusive offsets b.mem_off (padded n), b.t_off, b.y_off,
// totals[0..3] = sums of padded n, l, s and n, err |= descriptor error bits,
// mx[0] = max n, mx[1] != 0 iff some n is not a power of two, mx[2] = max l.
// sums holds layout_scratch_words(N) words; mx and totals start at zero.
hipError_t launch_layout(const uint64_t *prog_off, const uint64_t *tape_off, const uint32_t *mem_words,
                         uint32_t def_mem, const uint32_t *tape_cap, const uint32_t *out_cap, uint32_t def_out,
                         uint64_t N, DevBatch b, uint64_t *sums, uint64_t *totals, uint32_t *err, uint32_t *mx,
                         hipStream_t st);
uint64_t layout_scratch_words(uint64_t N);
hipError_t launch_scan_u64(const uint64_t *in, uint64_t *out_excl, uint64_t N,
                           uint64_t *block_sums, uint64_t *total, hipStream_t st);
hipError_t launch_scan_u32(const uint32_t *in, uint64_t *out_excl, uint64_t N,
                           uint64_t *block_sums, uint64_t *total, hipStream_t st);
uint64_t scan_scratch_words(uint64_t N);
hipError_t launch_pack(DevBatch b, const int32_t *prog, const uint64_t *prog_off,
                       const int32_t *tape, const uint64_t *tape_off, hipStream_t st);
hipError_t launch_check_state(DevBatch b, uint32_t *err, hipStream_t st);  // u0, y0, and i, a when w < 32
hipError_t launch_probe(DevBatch b, hipStream_t st);
// wm: some batch of the launch has words narrower than 32 bits
hipError_t launch_plain(const BatchTable *tab, uint64_t total, uint32_t cap,
                        uint32_t isa, bool pow2, bool pack, bool wm, uint32_t *surv, QueueState *q,
                        hipStream_t st, const HotArgs *hot = nullptr);
// cap < UINT32_MAX with surv non-null: a first pass (machines still running
// after cap transitions are appended to surv, q->survivors counts them)
hipError_t launch_persistent(const BatchTable *tab, uint64_t total, const uint32_t *work,
                             uint32_t already, uint32_t isa, bool pow2, bool wm, uint32_t epoch,
                             uint32_t lds_words, uint32_t max_n, uint32_t max_ell,
                             uint32_t waves_per_block, uint32_t blocks, uint32_t cap, uint32_t *surv,
                             QueueState *q, hipStream_t st, bool misfits = false);
// (misfits: the work list is a hot-cell first pass's misfit list, counted by
// q->misfits and claimed through q->head_m)
// the persistent kernel over the fits of a hot-cell first pass, each
// machine's hot cells in its lane's LDS table
hipError_t launch_persistent_hot(const BatchTable *tab, const uint32_t *work, uint32_t already, uint32_t isa,
                                 bool pow2, bool wm, uint32_t epoch, const HotArgs &hot,
                                 uint32_t waves_per_block, uint32_t blocks, QueueState *q, hipStream_t st);
// LDS words per lane of a hot-cell table of S slots (two words and a 16-bit
// cell tag per slot)
constexpr uint32_t hot_slot_words(uint32_t S) { return 2u * S + S / 2u; }
// profile bitmap words per lane for memories of at most max_n words
constexpr uint32_t hot_bitmap_words(uint32_t max_n) { return ((max_n + 1u) / 2u + 31u) / 32u; }
constexpr uint32_t kHotMaxN = 2048;     // largest memory a hot-cell launch profiles
// err |= kErrWordRange if some of the `count` words is not a w-bit value
hipError_t launch_check_words(const int32_t *w, uint64_t count, uint32_t wshift, uint32_t *err,
                              hipStream_t st);
// the same for words [off[0], off[N]) of w, the offsets in device memory
hipError_t launch_check_words_off(const int32_t *w, const uint64_t *off, uint64_t N, uint32_t wshift,
                                  uint32_t *err, hipStream_t st);
// LDS words of one lane's slot for a launch (memory words, four spare words
// and, when every memory fits and tapes are short, the tape); 0 for memory in HBM
uint32_t slot_words(uint32_t lds_words, uint32_t max_n, uint32_t max_ell);
constexpr uint32_t kTapeLdsMax = 64;     // tapes up to this many words are staged in LDS
hipError_t launch_zero_queue(QueueState *q, hipStream_t st);
hipError_t launch_reset_head(QueueState *q, hipStream_t st);     // head = 0, counts kept
void init_kernel_attributes();
hipError_t launch_running(const BatchTable *tab, uint64_t total, unsigned long long *counts,
                          hipStream_t st);
hipError_t launch_digest(DevBatch b, uint64_t *out, hipStream_t st);
// every machine's zero tail stored (zero_fill) or declared stored: hw = n rounded up to 4
hipError_t launch_tails(DevBatch b, bool zero_fill, hipStream_t st);
// per-machine scalars into device buffers (null pointers skipped)
hipError_t launch_fetch_scalars(DevBatch b, uint8_t *status, uint64_t *steps, int32_t *i, int32_t *a,
                                uint32_t *u0, uint32_t *y0, hipStream_t st);
hipError_t launch_steps_sum(DevBatch b, unsigned long long *out, hipStream_t st);
hipError_t launch_gather_words(const int32_t *src, const uint64_t *off, const uint32_t *len,
                               uint64_t N, int32_t *dst, const uint64_t *dst_off,
                               hipStream_t st);
hipError_t launch_scatter_words(const int32_t *src, const uint64_t *src_off,
                                const uint32_t *len, uint64_t N, int32_t *dst,
                                const uint64_t *dst_off, hipStream_t st);

}  // namespace rasp
