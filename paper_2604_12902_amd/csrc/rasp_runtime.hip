// rasp_runtime.hip -- host side of librasp: contexts, the device arena
// sub-allocator, batch loading, run scheduling and output fetching behind the
// C ABI of include/rasp.h.
#include "rasp_internal.h"
#include "../../include/rasp.h"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace rasp;

namespace {

constexpr uint64_t kAlign = 256;
constexpr int kTableRing = 16;
constexpr int kTickets = 4;              // running-count requests in flight per context
static_assert(sizeof(BatchTable) >= 8 * kMaxMulti * kTickets, "device count slots fit one table slot");
constexpr uint64_t kStageWords = 32ull << 20;    // host-load staging: program + input words per chunk
constexpr uint64_t kStageVms = 1ull << 20;       // and machines per chunk

constexpr uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// First-fit allocator over [0, size) with coalescing free list.
class Arena {
public:
    void reset(uint64_t size) { free_.clear(); if (size) free_[0] = size; size_ = size; }
    bool alloc(uint64_t bytes, uint64_t *off)
    {
        bytes = align_up(bytes ? bytes : 1, kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes)
    {
        bytes = align_up(bytes ? bytes : 1, kAlign);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t largest() const
    {
        uint64_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }
private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t size_ = 0;
};

struct Alloc {
    uint64_t off = 0, bytes = 0;
    bool live = false;
};

struct Batch {
    DevBatch dev{};
    Alloc meta, words;
    uint64_t N = 0;
    uint64_t sum_n = 0, sum_n_pad = 0, sum_ell = 0, sum_s = 0;
    uint32_t max_n = 0, max_ell = 0;
    uint32_t wbits = 32;                 // word width w
    bool all_pow2 = false;               // every n a power of two
    bool uniform_dense = false;          // every n a multiple of 4: padded == dense
    bool status_stale = true;            // status not yet computed since the load
    bool tails = false;                  // some memory's zero tail is not stored (hw below n)
    hipEvent_t done = nullptr;           // recorded after the batch's latest queued work
    bool fetch_pending = false;          // `done` was last recorded on the copy stream
    Alloc fetch_tmp;                     // digests of asynchronous fetches (8 bytes a machine)
    ~Batch() { if (done) (void)hipEventDestroy(done); }
};

uint64_t meta_bytes(uint64_t N)
{
    // i a u0 y0 (4 each) steps (8) status (1) n ell s (4 each) mem_off t_off y_off (8 each) hw (4)
    uint64_t b = 0;
    b += align_up(4 * N, kAlign) * 4;
    b += align_up(8 * N, kAlign);
    b += align_up(N, kAlign);
    b += align_up(4 * N, kAlign) * 3;
    b += align_up(8 * N, kAlign) * 3;
    b += align_up(4 * N, kAlign);
    return b;
}

void carve_meta(char *base, uint64_t N, DevBatch *d)
{
    char *p = base;
    auto take = [&](uint64_t bytes) { char *q = p; p += align_up(bytes, kAlign); return q; };
    d->i = reinterpret_cast<int32_t *>(take(4 * N));
    d->a = reinterpret_cast<int32_t *>(take(4 * N));
    d->u0 = reinterpret_cast<uint32_t *>(take(4 * N));
    d->y0 = reinterpret_cast<uint32_t *>(take(4 * N));
    d->steps = reinterpret_cast<uint64_t *>(take(8 * N));
    d->status = reinterpret_cast<uint8_t *>(take(N));
    d->n = reinterpret_cast<uint32_t *>(take(4 * N));
    d->ell = reinterpret_cast<uint32_t *>(take(4 * N));
    d->s = reinterpret_cast<uint32_t *>(take(4 * N));
    d->mem_off = reinterpret_cast<uint64_t *>(take(8 * N));
    d->t_off = reinterpret_cast<uint64_t *>(take(8 * N));
    d->y_off = reinterpret_cast<uint64_t *>(take(8 * N));
    d->hw = reinterpret_cast<uint32_t *>(take(4 * N));
    d->N = N;
}

uint64_t words_bytes(uint64_t sum_n_pad, uint64_t sum_ell, uint64_t sum_s)
{
    return align_up(4 * sum_n_pad, kAlign) + align_up(4 * sum_ell, kAlign) + align_up(4 * sum_s, kAlign);
}

void carve_words(char *base, uint64_t sum_n_pad, uint64_t sum_ell, DevBatch *d)
{
    d->M = reinterpret_cast<int32_t *>(base);
    d->T = reinterpret_cast<int32_t *>(base + align_up(4 * sum_n_pad, kAlign));
    d->Y = reinterpret_cast<int32_t *>(base + align_up(4 * sum_n_pad, kAlign) + align_up(4 * sum_ell, kAlign));
}

thread_local std::string g_create_error;

}  // namespace

struct rasp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *arena = nullptr;
    uint64_t arena_bytes = 0;
    bool own_arena = false;
    Arena alloc;
    std::map<uint64_t, std::unique_ptr<Batch>> batches;
    uint64_t next_handle = 1;
    std::string err;
    bool sticky = false;
    // device properties
    int cus = 0, lds_bytes = 0, wave = 64;
    // options
    int64_t schedule = RASP_SCHED_AUTO, epoch = 256, lds_words = -1, waves_per_cu = 16, graph = 0;
    int64_t first_pass = 64;
    int64_t first_pass_kind = 0;         // 1: LDS-resident first pass when memories fit
    int64_t hot_cells = 0;               // slots of a hot-cell table (0: off)
    int64_t profile_steps = 256;         // transitions profiled at the end of a hot-cell first pass
    int64_t misfit_waves = 6;            // waves per CU of the hot-cell misfits' launch
    Alloc hot;                           // hot-cell multipliers, tags and misfit list
    uint64_t hot_cap = 0, hot_S = 0;
    // second stream (same CU mask as the first) and its two events: the
    // misfits' launch runs there beside the fits' launch
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_first = nullptr, ev_second = nullptr;
    std::vector<uint32_t> cu_mask;       // empty: the context's stream has no CU mask
    // scratch: queue counters, batch tables (device ring + pinned host ring)
    Alloc scratch;
    QueueState *queue = nullptr;
    BatchTable *tables = nullptr;       // kTableRing device slots
    BatchTable *host_tables = nullptr;  // pinned
    hipEvent_t table_ev[kTableRing] = {};
    bool table_used[kTableRing] = {};
    int table_next = 0;
    Alloc work;                          // survivor list
    uint64_t work_cap = 0;
    uint32_t *err_host = nullptr;        // pinned: error word and totals
    uint64_t *tot_host = nullptr;
    uint64_t *count_host = nullptr;      // pinned: running counts, kTickets x kMaxMulti
    hipEvent_t count_ev[kTickets] = {};
    uint64_t ticket_next = 1;            // ticket t uses slot t % kTickets
    uint64_t ticket_of[kTickets] = {};   // the ticket a slot holds (0: none)
    uint32_t ticket_k[kTickets] = {};
    // copy stream (same CU mask as the first): asynchronous fetches
    hipStream_t cstream = nullptr;
    // captured launch sequences (RASP_OPT_GRAPH)
    struct GraphEntry {
        std::vector<uint64_t> key;         // handles, budgets, knobs
        std::vector<uint64_t> handles;
        Alloc table;                       // the graph's own device batch table
        hipGraphExec_t exec = nullptr;
    };
    std::vector<GraphEntry> graphs;
    // kernel timing (RASP_OPT_PROFILE)
    int64_t profile = 0;
    bool no_events = false;              // set while rasp_run_noalloc runs: no timing events
    char *noalloc_scratch = nullptr;     // this device's no-allocation scratch (device address)
    struct Timed { int kind; hipEvent_t a, b; };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> ev_pool;
};

namespace {

int fail(rasp_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) {
        c->err = buf;
        if (code == RASP_E_DEVICE) c->sticky = true;
    } else {
        g_create_error = buf;
    }
    return code;
}

#define HIPCHK(c, expr)                                                              \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess)                                                        \
            return fail((c), RASP_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

bool arena_alloc(rasp_ctx *c, uint64_t bytes, Alloc *a)
{
    if (!c->alloc.alloc(bytes, &a->off)) return false;
    a->bytes = bytes;
    a->live = true;
    return true;
}

void arena_free(rasp_ctx *c, Alloc *a)
{
    if (a->live) c->alloc.release(a->off, a->bytes);
    a->live = false;
}

template <class T>
T *at(rasp_ctx *c, const Alloc &a, uint64_t byte_off = 0)
{
    return reinterpret_cast<T *>(c->arena + a.off + byte_off);
}

int check_ctx(rasp_ctx *c)
{
    if (!c) return RASP_E_INVAL;
    if (c->sticky) return RASP_E_DEVICE;
    HIPCHK(c, hipSetDevice(c->device));
    return RASP_OK;
}

Batch *find(rasp_ctx *c, rasp_batch b)
{
    auto it = c->batches.find(b);
    return it == c->batches.end() ? nullptr : it->second.get();
}

template <class F> hipError_t timed_launch(rasp_ctx *c, int kind, F fn, hipStream_t st = nullptr);

// Build c0 of a lazily loaded batch (RASP_DESC_LAZY) in the arena.
int mark_queued(rasp_ctx *c, Batch *b);

int materialize(rasp_ctx *c, Batch *b)
{
    if (!b->dev.fresh) return RASP_OK;
    DevBatch d = b->dev;
    HIPCHK(c, timed_launch(c, RASP_KERNEL_PACK, [&] {
        return launch_pack(d, d.prog, d.prog_off, d.tape, d.tape_off, c->stream); }));
    b->dev.fresh = 0;
    b->status_stale = true;
    b->tails = true;
    return mark_queued(c, b);
}

// store every zero tail of the batch that is not stored yet
int store_tails(rasp_ctx *c, Batch *b)
{
    if (!b->tails) return RASP_OK;
    HIPCHK(c, timed_launch(c, RASP_KERNEL_OTHER, [&] { return launch_tails(b->dev, true, c->stream); }));
    b->tails = false;
    return RASP_OK;
}

hipEvent_t pooled_event(rasp_ctx *c)
{
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch `fn` (returning hipError_t) on the context stream (or `st`),
// bracketed by timing events when profiling is on.
template <class F>
hipError_t timed_launch(rasp_ctx *c, int kind, F fn, hipStream_t st)
{
    if (!c->profile || c->no_events) return fn();
    if (!st) st = c->stream;
    hipEvent_t a = pooled_event(c), b = pooled_event(c);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, st);
    if (!e) e = fn();
    if (!e) e = hipEventRecord(b, st);
    if (!e) c->timed.push_back({kind, a, b});
    return e;
}

// Host-side checks of a descriptor with host arrays; fills shapes and totals.
struct HostShapes {
    std::vector<uint32_t> n, ell, s;
    std::vector<uint64_t> mem_off, t_off, y_off;
    uint64_t sum_n = 0, sum_n_pad = 0, sum_ell = 0, sum_s = 0;
    uint64_t prog_words = 0, tape_words = 0;
    uint32_t max_n = 0, max_ell = 0;
    bool all_n_mult4 = true;
    bool all_pow2 = true;
};

int host_shapes(rasp_ctx *c, const rasp_batch_desc *d, HostShapes *h)
{
    const uint64_t N = d->num_vms;
    h->n.resize(N); h->ell.resize(N); h->s.resize(N);
    h->mem_off.resize(N); h->t_off.resize(N); h->y_off.resize(N);
    for (uint64_t v = 0; v < N; ++v) {
        const uint64_t p0 = d->prog_off[v], p1 = d->prog_off[v + 1];
        const uint64_t t0 = d->tape_off[v], t1 = d->tape_off[v + 1];
        if (p1 < p0 || t1 < t0) return fail(c, RASP_E_INVAL, "machine %llu: offsets decrease", (unsigned long long)v);
        const uint64_t plen = p1 - p0, tlen = t1 - t0;
        const uint32_t n = d->mem_words ? d->mem_words[v] : d->default_mem_words;
        const uint64_t ell = d->tape_cap ? d->tape_cap[v] : tlen;
        const uint32_t s = d->out_cap ? d->out_cap[v] : d->default_out_cap;
        if (n == 0 || n > kMaxMemWords)
            return fail(c, RASP_E_INVAL, "machine %llu: memory size %u outside [1, 2^30]", (unsigned long long)v, n);
        if (plen > n)
            return fail(c, RASP_E_INVAL, "machine %llu: program of %llu words exceeds memory of %u", (unsigned long long)v, (unsigned long long)plen, n);
        if (tlen > ell || ell > 0x7fffffffull)
            return fail(c, RASP_E_INVAL, "machine %llu: input of %llu words exceeds tape capacity %llu", (unsigned long long)v, (unsigned long long)tlen, (unsigned long long)ell);
        if (s > 0x7fffffffu) return fail(c, RASP_E_INVAL, "machine %llu: output capacity too large", (unsigned long long)v);
        h->n[v] = n; h->ell[v] = static_cast<uint32_t>(ell); h->s[v] = s;
        h->mem_off[v] = h->sum_n_pad; h->t_off[v] = h->sum_ell; h->y_off[v] = h->sum_s;
        h->sum_n += n; h->sum_n_pad += (n + 3u) & ~3ull; h->sum_ell += ell; h->sum_s += s;
        if (n & 3u) h->all_n_mult4 = false;
        h->max_n = std::max(h->max_n, n);
        if (n & (n - 1u)) h->all_pow2 = false;
        h->max_ell = std::max(h->max_ell, static_cast<uint32_t>(ell));
    }
    h->prog_words = d->prog_off[N] - d->prog_off[0];
    h->tape_words = d->tape_off[N] - d->tape_off[0];
    return RASP_OK;
}

int basic_desc_checks(rasp_ctx *c, const rasp_batch_desc *d)
{
    if (!d) return fail(c, RASP_E_INVAL, "descriptor is NULL");
    if (d->abi_version != RASP_ABI_VERSION) return fail(c, RASP_E_INVAL, "abi_version %u, library has %u", d->abi_version, RASP_ABI_VERSION);
    if (d->isa != RASP_ISA_WORD && d->isa != RASP_ISA_CLASSIC) return fail(c, RASP_E_INVAL, "unknown isa %u", d->isa);
    if (d->num_vms == 0 || d->num_vms >= (1ull << 32)) return fail(c, RASP_E_INVAL, "num_vms must be in [1, 2^32)");
    if (!d->prog_off || !d->tape_off) return fail(c, RASP_E_INVAL, "prog_off and tape_off are required");
    if (d->flags & ~(RASP_DESC_DEVICE_PTRS | RASP_DESC_LAZY)) return fail(c, RASP_E_INVAL, "unknown descriptor flags");
    if ((d->flags & RASP_DESC_LAZY) && !(d->flags & RASP_DESC_DEVICE_PTRS))
        return fail(c, RASP_E_INVAL, "RASP_DESC_LAZY needs a device descriptor");
    if (d->word_bits == 1 || d->word_bits > 32) return fail(c, RASP_E_INVAL, "word_bits %u outside [2, 32]", d->word_bits);
    return RASP_OK;
}

uint32_t word_bits_of(const rasp_batch_desc *d) { return d->word_bits == 0 ? 32u : d->word_bits; }

// is every host word a w-bit value
bool host_words_fit(const int32_t *w, uint64_t count, uint32_t bits)
{
    if (bits >= 32) return true;
    const int64_t lo = -(int64_t(1) << (bits - 1)), hi = (int64_t(1) << (bits - 1)) - 1;
    for (uint64_t k = 0; k < count; ++k)
        if (w[k] < lo || w[k] > hi) return false;
    return true;
}

// Allocate and fill a batch's metadata and word arenas, then queue the pack.
int load_common(rasp_ctx *c, const rasp_batch_desc *d, std::unique_ptr<Batch> &out)
{
    int rc = basic_desc_checks(c, d);
    if (rc) return rc;
    const uint64_t N = d->num_vms;
    auto B = std::make_unique<Batch>();
    B->N = N;
    const bool dev = (d->flags & RASP_DESC_DEVICE_PTRS) != 0;
    hipStream_t st = c->stream;

    if (!arena_alloc(c, meta_bytes(N), &B->meta))
        return fail(c, RASP_E_NOMEM, "arena cannot hold state of %llu machines", (unsigned long long)N);
    carve_meta(at<char>(c, B->meta), N, &B->dev);
    B->dev.isa = d->isa;
    B->wbits = word_bits_of(d);
    B->dev.wshift = 32u - B->wbits;

    const int32_t *prog_dev = nullptr, *tape_dev = nullptr;
    const uint64_t *poff_dev = nullptr, *toff_dev = nullptr;
    Alloc staging;

    auto bail = [&](int code) {
        (void)hipStreamSynchronize(st);
        arena_free(c, &staging);
        arena_free(c, &B->words);
        arena_free(c, &B->meta);
        return code;
    };

    if (!dev) {
        HostShapes h;
        if ((rc = host_shapes(c, d, &h))) return bail(rc);
        if (h.prog_words && !d->prog) { fail(c, RASP_E_INVAL, "prog is NULL"); return bail(RASP_E_INVAL); }
        if (h.tape_words && !d->tape) { fail(c, RASP_E_INVAL, "tape is NULL"); return bail(RASP_E_INVAL); }
        if (!host_words_fit(d->prog + d->prog_off[0], h.prog_words, B->wbits) ||
            !host_words_fit(d->tape + d->tape_off[0], h.tape_words, B->wbits)) {
            fail(c, RASP_E_INVAL, "a program or input word is not a %u-bit value", B->wbits);
            return bail(RASP_E_INVAL);
        }
        B->sum_n = h.sum_n; B->sum_n_pad = h.sum_n_pad; B->sum_ell = h.sum_ell; B->sum_s = h.sum_s;
        B->uniform_dense = h.all_n_mult4;
        B->max_n = h.max_n;
        B->max_ell = h.max_ell;
        B->all_pow2 = h.all_pow2;
        if (!arena_alloc(c, words_bytes(h.sum_n_pad, h.sum_ell, h.sum_s), &B->words)) {
            fail(c, RASP_E_NOMEM, "arena cannot hold the batch (%llu memory words)", (unsigned long long)h.sum_n);
            return bail(RASP_E_NOMEM);
        }
        carve_words(at<char>(c, B->words), B->sum_n_pad, B->sum_ell, &B->dev);
        auto H2D = [&](void *dst, const void *src, uint64_t bytes) {
            return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
        };
        hipError_t e = hipSuccess;
        if (!e) e = H2D(B->dev.n, h.n.data(), 4 * N);
        if (!e) e = H2D(B->dev.ell, h.ell.data(), 4 * N);
        if (!e) e = H2D(B->dev.s, h.s.data(), 4 * N);
        if (!e) e = H2D(B->dev.mem_off, h.mem_off.data(), 8 * N);
        if (!e) e = H2D(B->dev.t_off, h.t_off.data(), 8 * N);
        if (!e) e = H2D(B->dev.y_off, h.y_off.data(), 8 * N);
        // programs and inputs go through a bounded staging buffer, a chunk of
        // machines at a time; each chunk is packed from its staged copy
        const uint64_t budget_words = std::max<uint64_t>(kStageWords, 0);
        uint64_t max_chunk_words = 0;
        {
            uint64_t v0 = 0;
            while (v0 < N) {
                uint64_t v1 = v0, words = 0;
                while (v1 < N) {
                    const uint64_t w = (d->prog_off[v1 + 1] - d->prog_off[v1]) + (d->tape_off[v1 + 1] - d->tape_off[v1]);
                    if (v1 > v0 && (words + w > budget_words || v1 - v0 >= kStageVms)) break;
                    words += w;
                    ++v1;
                }
                max_chunk_words = std::max(max_chunk_words, words);
                v0 = v1;
            }
        }
        const uint64_t sb = align_up(4 * max_chunk_words, kAlign) + 2 * align_up(8 * (std::min<uint64_t>(N, kStageVms) + 1), kAlign) + kAlign;
        if (!e && !arena_alloc(c, sb, &staging)) {
            fail(c, RASP_E_NOMEM, "arena cannot hold the load staging buffer");
            return bail(RASP_E_NOMEM);
        }
        std::vector<uint64_t> po_h, to_h;
        uint64_t v0 = 0;
        while (!e && v0 < N) {
            uint64_t v1 = v0, words = 0;
            while (v1 < N) {
                const uint64_t w = (d->prog_off[v1 + 1] - d->prog_off[v1]) + (d->tape_off[v1 + 1] - d->tape_off[v1]);
                if (v1 > v0 && (words + w > budget_words || v1 - v0 >= kStageVms)) break;
                words += w;
                ++v1;
            }
            const uint64_t cn = v1 - v0;
            const uint64_t pw = d->prog_off[v1] - d->prog_off[v0], tw = d->tape_off[v1] - d->tape_off[v0];
            char *sp = at<char>(c, staging);
            int32_t *pg = reinterpret_cast<int32_t *>(sp);
            int32_t *tp = pg + pw;
            uint64_t *po = reinterpret_cast<uint64_t *>(sp + align_up(4 * max_chunk_words, kAlign));
            uint64_t *to = reinterpret_cast<uint64_t *>(reinterpret_cast<char *>(po) + align_up(8 * (std::min<uint64_t>(N, kStageVms) + 1), kAlign));
            po_h.resize(cn + 1); to_h.resize(cn + 1);
            for (uint64_t v = 0; v <= cn; ++v) {
                po_h[v] = d->prog_off[v0 + v] - d->prog_off[v0];
                to_h[v] = d->tape_off[v0 + v] - d->tape_off[v0] + pw;   // tape words follow the program words
            }
            if (!e) e = H2D(pg, d->prog + d->prog_off[v0], 4 * pw);
            if (!e) e = H2D(tp, d->tape + d->tape_off[v0], 4 * tw);
            if (!e) e = H2D(po, po_h.data(), 8 * (cn + 1));
            if (!e) e = H2D(to, to_h.data(), 8 * (cn + 1));
            DevBatch view = B->dev;
            view.i += v0; view.a += v0; view.u0 += v0; view.y0 += v0; view.steps += v0; view.status += v0;
            view.n += v0; view.ell += v0; view.s += v0; view.mem_off += v0; view.t_off += v0; view.y_off += v0;
            view.hw += v0;
            view.N = cn;
            if (!e) e = timed_launch(c, RASP_KERNEL_PACK, [&] { return launch_pack(view, pg, po, pg, to, st); });
            // the staging buffer and the host offset vectors are reused: wait
            if (!e) e = hipStreamSynchronize(st);
            B->tails = true;
            v0 = v1;
        }
        if (e) { fail(c, RASP_E_DEVICE, "loading batch: %s", hipGetErrorString(e)); return bail(RASP_E_DEVICE); }
        arena_free(c, &staging);
    } else {
        // device descriptor: checks, shapes and offsets computed on the device
        const uint64_t tb = align_up(8 * layout_scratch_words(N), kAlign) + kAlign;
        if (!arena_alloc(c, tb, &staging)) { fail(c, RASP_E_NOMEM, "arena cannot hold load scratch"); return bail(RASP_E_NOMEM); }
        char *sp = at<char>(c, staging);
        uint64_t *sums = reinterpret_cast<uint64_t *>(sp);
        uint64_t *tots = reinterpret_cast<uint64_t *>(sp + align_up(8 * layout_scratch_words(N), kAlign));
        uint32_t *errw = reinterpret_cast<uint32_t *>(tots + 4);
        hipError_t e = hipMemsetAsync(tots, 0, kAlign, st);
        if (!e) e = launch_layout(d->prog_off, d->tape_off, d->mem_words, d->default_mem_words, d->tape_cap,
                                  d->out_cap, d->default_out_cap, N, B->dev, sums, tots, errw, errw + 1, st);
        if (!e) e = launch_check_words_off(d->prog, d->prog_off, N, B->dev.wshift, errw, st);
        if (!e) e = launch_check_words_off(d->tape, d->tape_off, N, B->dev.wshift, errw, st);
        if (!e) e = hipMemcpyAsync(c->tot_host, tots, 4 * sizeof(uint64_t) + 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, st);
        if (!e) e = hipStreamSynchronize(st);
        if (e) { fail(c, RASP_E_DEVICE, "loading batch: %s", hipGetErrorString(e)); return bail(RASP_E_DEVICE); }
        uint32_t errbits;
        std::memcpy(&errbits, reinterpret_cast<char *>(c->tot_host) + 32, 4);
        if (errbits) {
            fail(c, RASP_E_INVAL, "descriptor check failed (bits 0x%x: 1 offsets, 2 program > memory, 4 input > tape, "
                                  "8 memory size, 32 a word wider than %u bits)", errbits, B->wbits);
            return bail(RASP_E_INVAL);
        }
        B->sum_n_pad = c->tot_host[0]; B->sum_ell = c->tot_host[1]; B->sum_s = c->tot_host[2]; B->sum_n = c->tot_host[3];
        std::memcpy(&B->max_n, reinterpret_cast<char *>(c->tot_host) + 36, 4);
        uint32_t nonpow2 = 0;
        std::memcpy(&nonpow2, reinterpret_cast<char *>(c->tot_host) + 40, 4);
        B->all_pow2 = nonpow2 == 0;
        std::memcpy(&B->max_ell, reinterpret_cast<char *>(c->tot_host) + 44, 4);
        B->uniform_dense = (B->sum_n == B->sum_n_pad);
        if (!arena_alloc(c, words_bytes(B->sum_n_pad, B->sum_ell, B->sum_s), &B->words)) {
            fail(c, RASP_E_NOMEM, "arena cannot hold the batch (%llu memory words)", (unsigned long long)B->sum_n);
            return bail(RASP_E_NOMEM);
        }
        carve_words(at<char>(c, B->words), B->sum_n_pad, B->sum_ell, &B->dev);
        prog_dev = d->prog; tape_dev = d->tape; poff_dev = d->prog_off; toff_dev = d->tape_off;
        B->dev.prog = prog_dev; B->dev.prog_off = poff_dev; B->dev.tape = tape_dev; B->dev.tape_off = toff_dev;
        if (d->flags & RASP_DESC_LAZY) {
            B->dev.fresh = 1;              // c0 is built by the first run (or on demand)
        } else {
            e = timed_launch(c, RASP_KERNEL_PACK, [&] { return launch_pack(B->dev, prog_dev, poff_dev, tape_dev, toff_dev, st); });
            B->tails = true;
        }
        if (e) { fail(c, RASP_E_DEVICE, "pack: %s", hipGetErrorString(e)); return bail(RASP_E_DEVICE); }
        // scratch is only used by work queued before this point: stream order makes reuse safe
        arena_free(c, &staging);
    }
    out = std::move(B);
    return RASP_OK;
}

// LDS words per machine slot for a launch whose largest memory is max_n:
// the option, or (option -1) the whole memory rounded up to 4 words if two
// waves of such slots fit a compute unit, else none
uint32_t lds_words_for(rasp_ctx *c, uint32_t max_n, uint32_t max_ell = 0)
{
    const uint64_t lds = static_cast<uint64_t>(c->lds_bytes);
    uint32_t P;
    if (c->lds_words >= 0) {
        P = static_cast<uint32_t>(c->lds_words);
    } else {
        P = max_n <= 1024 ? std::max<uint32_t>(4, (max_n + 3u) & ~3u) : 0u;
        if (P && 2ull * kWave * slot_words(P, max_n, max_ell) * 4 > lds) P = 0;
    }
    while (P && static_cast<uint64_t>(kWave) * slot_words(P, max_n, max_ell) * 4 > lds) P = (P >> 1) & ~3u;
    return P;
}

// waves per block (1..4) of a persistent launch whose lanes hold slots of SPw
// LDS words: the one that keeps the most waves of a compute unit resident
// (ties to the larger block).  With 208-word slots, for instance, three
// one-wave blocks fit where one two-wave block does.
uint32_t waves_per_block_for(uint32_t SPw, uint64_t lds)
{
    if (SPw == 0) return 4;
    uint32_t wpb = 1;
    uint64_t best = 0;
    for (uint32_t w = 4; w >= 1; --w) {
        const uint64_t resident = lds / (static_cast<uint64_t>(w) * kWave * SPw * 4) * w;
        if (resident > best) { best = resident; wpb = w; }
    }
    return wpb;
}

// blocks of a persistent launch: the waves asked for (waves per CU x CUs),
// in blocks of wpb waves, but no more than the LDS of the context's compute
// units holds at once (lanes with SPw-word slots): blocks beyond that would
// only start as resident ones exit
uint32_t resident_blocks(const rasp_ctx *c, uint32_t wpb, uint32_t SPw, uint32_t waves)
{
    uint32_t blocks = std::max<uint32_t>(1, waves / wpb);
    if (SPw > 0) {
        const uint64_t per_cu = static_cast<uint64_t>(c->lds_bytes) / (static_cast<uint64_t>(wpb) * kWave * SPw * 4);
        const uint64_t most = std::max<uint64_t>(1, per_cu * static_cast<uint64_t>(c->cus));
        blocks = static_cast<uint32_t>(std::min<uint64_t>(blocks, most));
    }
    return blocks;
}

// drop captured graphs (all of them, or those that use batch h)
void drop_graphs(rasp_ctx *c, bool all, uint64_t h = 0)
{
    std::vector<rasp_ctx::GraphEntry> keep;
    bool synced = false;
    for (auto &g : c->graphs) {
        bool uses = all;
        for (auto x : g.handles) uses |= (x == h);
        if (!uses) { keep.push_back(std::move(g)); continue; }
        if (!synced) { (void)hipStreamSynchronize(c->stream); synced = true; }
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        arena_free(c, &g.table);
    }
    c->graphs = std::move(keep);
}

// ensure the survivor list holds `items` entries
int ensure_work(rasp_ctx *c, uint64_t items)
{
    if (items <= c->work_cap) return RASP_OK;
    if (c->work.live) {
        drop_graphs(c, true);                  // captured launches point at the old list
        HIPCHK(c, hipStreamSynchronize(c->stream));
        arena_free(c, &c->work);
    }
    if (!arena_alloc(c, 4 * items, &c->work)) {
        c->work_cap = 0;
        return fail(c, RASP_E_NOMEM, "arena cannot hold the work list of %llu machines", (unsigned long long)items);
    }
    c->work_cap = items;
    return RASP_OK;
}

// ensure the hot-cell arrays hold `items` survivor-list entries of S slots
int ensure_hot(rasp_ctx *c, uint64_t items, uint64_t S)
{
    if (items <= c->hot_cap && S <= c->hot_S) return RASP_OK;
    if (c->hot.live) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        arena_free(c, &c->hot);
    }
    const uint64_t bytes = 2 * align_up(4 * items, kAlign) + 2 * items * S;
    if (!arena_alloc(c, bytes, &c->hot)) {
        c->hot_cap = c->hot_S = 0;
        return fail(c, RASP_E_NOMEM, "arena cannot hold the hot-cell tables of %llu machines", (unsigned long long)items);
    }
    c->hot_cap = items;
    c->hot_S = S;
    return RASP_OK;
}

// the context's second stream and its events (created on first use, with
// the first stream's CU mask)
int ensure_stream2(rasp_ctx *c)
{
    if (c->stream2) return RASP_OK;
    hipError_t e = c->cu_mask.empty()
                       ? hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking)
                       : hipExtStreamCreateWithCUMask(&c->stream2, static_cast<uint32_t>(c->cu_mask.size()),
                                                      c->cu_mask.data());
    if (!e) e = hipEventCreateWithFlags(&c->ev_first, hipEventDisableTiming);
    if (!e) e = hipEventCreateWithFlags(&c->ev_second, hipEventDisableTiming);
    if (e) return fail(c, RASP_E_DEVICE, "second stream: %s", hipGetErrorString(e));
    return RASP_OK;
}

// the copy stream, created on first use with the context's CU mask
int ensure_cstream(rasp_ctx *c)
{
    if (c->cstream) return RASP_OK;
    hipError_t e = c->cu_mask.empty()
                       ? hipStreamCreateWithFlags(&c->cstream, hipStreamNonBlocking)
                       : hipExtStreamCreateWithCUMask(&c->cstream, static_cast<uint32_t>(c->cu_mask.size()),
                                                      c->cu_mask.data());
    if (e) return fail(c, RASP_E_DEVICE, "copy stream: %s", hipGetErrorString(e));
    return RASP_OK;
}

// work about to be queued for b on the context stream comes after an
// asynchronous fetch of b still in flight on the copy stream
int after_fetch(rasp_ctx *c, Batch *b)
{
    if (!b->fetch_pending) return RASP_OK;
    HIPCHK(c, hipStreamWaitEvent(c->stream, b->done, 0));
    b->fetch_pending = false;
    return RASP_OK;
}

// grab a device batch-table slot and its pinned host mirror
int table_slot(rasp_ctx *c, BatchTable **host, BatchTable **devp, int *slot)
{
    const int k = c->table_next;
    c->table_next = (k + 1) % kTableRing;
    if (c->table_used[k]) HIPCHK(c, hipEventSynchronize(c->table_ev[k]));
    *host = &c->host_tables[k];
    *devp = &c->tables[k];
    *slot = k;
    return RASP_OK;
}

// record the batch's event after the work queued for it so far (the event is
// created with the batch's first queued work)
int mark_queued(rasp_ctx *c, Batch *b)
{
    if (!b->done) HIPCHK(c, hipEventCreateWithFlags(&b->done, hipEventDisableTiming));
    HIPCHK(c, hipEventRecord(b->done, c->stream));
    return RASP_OK;
}

// Device memory a run needs beyond its batches: the queue counters, the
// batch tables a launch reads and the survivor list of a first pass.
struct RunScratch {
    QueueState *queue;
    BatchTable *table[2];                // the launch's table and, after a first pass, its successor
    uint32_t *work;
    uint64_t work_cap;                   // survivor-list entries
};

int run_batches(rasp_ctx *c, Batch **bs, const uint32_t *budgets, uint32_t k, const RunScratch *rs = nullptr)
{
    const uint32_t isa = bs[0]->dev.isa;
    for (uint32_t t = 1; t < k; ++t)
        if (bs[t]->dev.isa != isa) return fail(c, RASP_E_INVAL, "batches of one launch must share the instruction set");
    for (uint32_t t = 0; t < k; ++t) {
        int rc0 = after_fetch(c, bs[t]);
        if (rc0) return rc0;
    }
    // lazily loaded batches are built inside the persistent kernel when every
    // machine of the launch fits its LDS slot; otherwise c0 is packed first
    bool any_fresh = false;
    uint32_t mx = 0, mxl = 0;
    for (uint32_t t = 0; t < k; ++t) {
        any_fresh |= bs[t]->dev.fresh != 0;
        mx = std::max(mx, bs[t]->max_n);
        mxl = std::max(mxl, bs[t]->max_ell);
    }
    const uint32_t Pq = lds_words_for(c, mx, mxl);
    const int64_t schedq = c->schedule == RASP_SCHED_AUTO ? RASP_SCHED_PERSISTENT : c->schedule;
    // every memory fits its LDS slot: the persistent kernel can build c0 itself
    const bool lds_ok = Pq > 0 && Pq >= mx;
    // the first pass is the persistent kernel in LDS (else the plain kernel)
    const bool lds_first = schedq == RASP_SCHED_PERSISTENT && c->first_pass > 0 &&
                           c->first_pass_kind == 1 && lds_ok;
    // (a) first pass 0 and every memory fits: c0 is built by the persistent
    //     kernel; (b) an LDS first pass builds c0 the same way; (c) a plain
    //     first pass packs c0 of its wave's machines before stepping them;
    //     (d) otherwise pack first.  A batch that runs 0 transitions in the
    //     launch is never claimed by the persistent kernel: pack it first
    const bool fused = any_fresh && schedq == RASP_SCHED_PERSISTENT && lds_ok && c->first_pass == 0;
    const bool pack_in_plain = any_fresh && !fused && !lds_first &&
                               (schedq == RASP_SCHED_PLAIN || c->first_pass > 0);
    for (uint32_t t = 0; t < k; ++t)
        if (bs[t]->dev.fresh && ((!fused && !lds_first && !pack_in_plain) ||
                                 ((fused || lds_first) && budgets[t] == 0))) {
            int rc = materialize(c, bs[t]);
            if (rc) return rc;
        }
    // c0's zero tails: the plain pass reads unstored ones as zeros (and stores
    // them for the machines it hands on); any other opening launch reads and
    // writes whole memories, so they are stored first
    const bool plain_first = schedq == RASP_SCHED_PLAIN || (!fused && !lds_first && c->first_pass > 0);
    for (uint32_t t = 0; t < k; ++t) {
        if (bs[t]->dev.fresh && pack_in_plain) bs[t]->tails = true;
        if (!plain_first && !bs[t]->dev.fresh) {
            int rc = store_tails(c, bs[t]);
            if (rc) return rc;
        }
    }
    // queue counters: the context's, or the caller-independent scratch
    QueueState *const qs = rs ? rs->queue : c->queue;
    const bool graphed = c->graph && !any_fresh && !rs && c->hot_cells == 0;
    BatchTable *ht, *dt;
    int slot;
    int rc = table_slot(c, &ht, &dt, &slot);
    if (rc) return rc;
    if (rs) dt = rs->table[0];
    std::memset(ht, 0, sizeof(BatchTable));
    uint64_t total = 0;
    uint32_t maxb = 0, max_n = 0, max_ell = 0;
    bool pow2 = true, wm = false;
    for (uint32_t t = 0; t < k; ++t) {
        max_n = std::max(max_n, bs[t]->max_n);
        max_ell = std::max(max_ell, bs[t]->max_ell);
        // v mod n = v & (n - 1) on w-bit words needs n | 2^w
        pow2 &= bs[t]->all_pow2 && (bs[t]->wbits >= 32 || bs[t]->max_n <= (1u << bs[t]->wbits));
        wm |= bs[t]->wbits < 32;
        ht->b[t] = bs[t]->dev;
        ht->start[t] = total;
        ht->budget[t] = budgets[t];
        total += bs[t]->N;
        maxb = std::max(maxb, budgets[t]);
    }
    ht->start[k] = total;
    ht->count = k;
    if (total >= (1ull << 32)) return fail(c, RASP_E_INVAL, "too many machines in one launch");
    if (maxb == 0) {
        for (uint32_t t = 0; t < k; ++t) { int rc2 = materialize(c, bs[t]); if (rc2) return rc2; }
        return RASP_OK;
    }
    for (uint32_t t = 0; t < k; ++t)
        if (budgets[t] > 0) bs[t]->status_stale = false;    // every run recomputes status
    hipStream_t st = c->stream;
    int64_t sched = c->schedule;
    if (sched == RASP_SCHED_AUTO) sched = RASP_SCHED_PERSISTENT;
    if (!graphed) {
        HIPCHK(c, hipMemcpyAsync(dt, ht, sizeof(BatchTable), hipMemcpyHostToDevice, st));
        HIPCHK(c, hipEventRecord(c->table_ev[slot], st));
        c->table_used[slot] = true;
        HIPCHK(c, timed_launch(c, RASP_KERNEL_OTHER, [&] { return launch_zero_queue(qs, st); }));
    }
    if (sched == RASP_SCHED_PLAIN && !graphed) {
        HIPCHK(c, timed_launch(c, RASP_KERNEL_PLAIN, [&] {
            return launch_plain(dt, total, maxb, isa, pow2, pack_in_plain, wm, nullptr, qs, st); }));
        for (uint32_t t = 0; t < k; ++t) bs[t]->dev.fresh = 0;
        return RASP_OK;
    }
    // persistent: a first plain pass of `first_pass` steps retires the short
    // runners; the survivors go through the persistent kernel (the plain
    // schedule is a first pass as long as the budget)
    const uint32_t cap = sched == RASP_SCHED_PLAIN ? maxb : static_cast<uint32_t>(std::max<int64_t>(0, c->first_pass));
    // waves per block: as many (up to 4) as the LDS slots of one block allow
    const uint32_t P = lds_words_for(c, max_n, max_ell);
    const uint64_t lds = static_cast<uint64_t>(c->lds_bytes);
    const uint32_t SPw = slot_words(P, max_n, max_ell);
    const uint32_t wpb = waves_per_block_for(SPw, lds);
    const uint32_t waves = static_cast<uint32_t>(std::max<int64_t>(1, c->waves_per_cu)) * static_cast<uint32_t>(c->cus);
    const uint32_t blocks = resident_blocks(c, wpb, SPw, waves);
    const uint32_t epoch = static_cast<uint32_t>(std::max<int64_t>(1, c->epoch));
    // hot-cell tables: a plain first pass shorter than the budget, memories of
    // at most kHotMaxN words, a launch that may allocate
    const uint32_t S_hot = static_cast<uint32_t>(c->hot_cells);
    const bool hot = S_hot > 0 && sched == RASP_SCHED_PERSISTENT && cap > 0 && cap < maxb && !lds_first &&
                     !fused && max_n <= kHotMaxN && rs == nullptr;
    if (graphed) {
        // replay (capturing on first use) the launch sequence for this key
        std::vector<uint64_t> key;
        for (uint32_t t = 0; t < k; ++t) { key.push_back(reinterpret_cast<uint64_t>(bs[t])); key.push_back(budgets[t]); }
        const uint64_t knobs[] = {static_cast<uint64_t>(c->schedule), P, epoch, cap, wpb, blocks,
                                  pow2 ? 1u : 0u, isa, maxb, wm ? 1u : 0u, lds_first ? 1u : 0u};
        key.insert(key.end(), knobs, knobs + 11);
        rasp_ctx::GraphEntry *ge = nullptr;
        for (auto &g : c->graphs) if (g.key == key) ge = &g;
        if (!ge) {
            if (cap > 0 && cap < maxb && (rc = ensure_work(c, total))) return rc;
            rasp_ctx::GraphEntry g;
            g.key = key;
            if (!arena_alloc(c, sizeof(BatchTable), &g.table)) return fail(c, RASP_E_NOMEM, "arena cannot hold a graph table");
            BatchTable *gt = at<BatchTable>(c, g.table);
            HIPCHK(c, hipMemcpyAsync(gt, ht, sizeof(BatchTable), hipMemcpyHostToDevice, st));
            HIPCHK(c, hipStreamSynchronize(st));
            uint32_t *work = (cap > 0 && cap < maxb) ? at<uint32_t>(c, c->work) : nullptr;
            hipGraph_t graph = nullptr;
            HIPCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            hipError_t e = launch_zero_queue(qs, st);
            if (!e && cap > 0 && cap < maxb && lds_first) {
                e = launch_persistent(gt, total, nullptr, 0, isa, pow2, wm, epoch, P, max_n, max_ell, wpb, blocks, cap, work, qs, st);
                if (!e) e = launch_reset_head(qs, st);
                if (!e) e = launch_persistent(gt, total, work, cap, isa, pow2, wm, epoch, P, max_n, max_ell, wpb, blocks, kNoCap, nullptr, qs, st);
            } else if (!e && cap > 0 && cap < maxb) {
                e = launch_plain(gt, total, cap, isa, pow2, false, wm, work, qs, st);
                if (!e) e = launch_persistent(gt, total, work, cap, isa, pow2, wm, epoch, P, max_n, max_ell, wpb, blocks, kNoCap, nullptr, qs, st);
            } else if (!e && cap >= maxb && !lds_first) {
                e = launch_plain(gt, total, maxb, isa, pow2, false, wm, nullptr, qs, st);
            } else if (!e) {
                e = launch_persistent(gt, total, nullptr, 0, isa, pow2, wm, epoch, P, max_n, max_ell, wpb, blocks, kNoCap, nullptr, qs, st);
            }
            hipError_t e2 = hipStreamEndCapture(st, &graph);
            if (!e) e = e2;
            if (!e) e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e) { arena_free(c, &g.table); return fail(c, RASP_E_DEVICE, "graph capture: %s", hipGetErrorString(e)); }
            for (uint32_t t = 0; t < k; ++t) g.handles.push_back(reinterpret_cast<uint64_t>(bs[t]));
            c->graphs.push_back(std::move(g));
            ge = &c->graphs.back();
        }
        hipGraphExec_t ex = ge->exec;
        HIPCHK(c, timed_launch(c, RASP_KERNEL_PERSISTENT, [&] { return hipGraphLaunch(ex, st); }));
        return RASP_OK;
    }
    if (fused) {
        // fresh batches present: one persistent launch over every machine
        HIPCHK(c, timed_launch(c, RASP_KERNEL_PERSISTENT, [&] {
            return launch_persistent(dt, total, nullptr, 0, isa, pow2, wm, epoch, P, max_n, max_ell, wpb, blocks, kNoCap, nullptr, qs, st); }));
        for (uint32_t t = 0; t < k; ++t) bs[t]->dev.fresh = 0;
    } else if (hot) {
        // hot-cell first pass (plain, profiling its last transitions), then
        // the persistent kernel over fits and misfits with their LDS tables
        if ((rc = ensure_work(c, total)) || (rc = ensure_hot(c, total, S_hot))) return rc;
        uint32_t *work = at<uint32_t>(c, c->work);
        HotArgs ha{};
        ha.S = S_hot;
        ha.lgS = static_cast<uint32_t>(__builtin_ctz(S_hot));
        ha.R = static_cast<uint32_t>(std::min<int64_t>(c->profile_steps, cap));
        ha.bw = hot_bitmap_words(max_n);
        ha.mult = at<uint32_t>(c, c->hot);
        ha.mis = at<uint32_t>(c, c->hot, align_up(4 * c->hot_cap, kAlign));
        ha.tags = at<uint16_t>(c, c->hot, 2 * align_up(4 * c->hot_cap, kAlign));
        if ((rc = ensure_stream2(c))) return rc;
        HIPCHK(c, timed_launch(c, RASP_KERNEL_PLAIN, [&] {
            return launch_plain(dt, total, cap, isa, pow2, pack_in_plain, wm, work, qs, st, &ha); }));
        BatchTable *dt2 = dt;
        if (any_fresh) {
            BatchTable *ht2;
            int slot2;
            if ((rc = table_slot(c, &ht2, &dt2, &slot2))) return rc;
            std::memcpy(ht2, ht, sizeof(BatchTable));
            for (uint32_t t = 0; t < k; ++t) ht2->b[t].fresh = 0;
            HIPCHK(c, hipMemcpyAsync(dt2, ht2, sizeof(BatchTable), hipMemcpyHostToDevice, st));
            HIPCHK(c, hipEventRecord(c->table_ev[slot2], st));
            c->table_used[slot2] = true;
        }
        const uint32_t SPh = hot_slot_words(S_hot);
        const uint32_t wpb_h = waves_per_block_for(SPh, lds);
        const uint32_t blocks_h = resident_blocks(c, wpb_h, SPh, waves);
        // the misfits on the second stream, after the first pass; the first
        // stream's later work waits for them
        hipStream_t st2 = c->stream2;
        const uint32_t blocks_m = std::max<uint32_t>(
            1, static_cast<uint32_t>(std::max<int64_t>(1, c->misfit_waves)) * static_cast<uint32_t>(c->cus) / 4u);
        HIPCHK(c, hipEventRecord(c->ev_first, st));
        HIPCHK(c, hipStreamWaitEvent(st2, c->ev_first, 0));
        HIPCHK(c, timed_launch(c, RASP_KERNEL_MISFIT, [&] {
            return launch_persistent(dt2, total, ha.mis, cap, isa, pow2, wm, epoch, 0u, max_n, max_ell, 4u, blocks_m,
                                     kNoCap, nullptr, qs, st2, true); }, st2));
        HIPCHK(c, hipEventRecord(c->ev_second, st2));
        HIPCHK(c, timed_launch(c, RASP_KERNEL_PERSISTENT, [&] {
            return launch_persistent_hot(dt2, work, cap, isa, pow2, wm, epoch, ha, wpb_h, blocks_h, qs, st); }));
        HIPCHK(c, hipStreamWaitEvent(st, c->ev_second, 0));
        for (uint32_t t = 0; t < k; ++t) bs[t]->dev.fresh = 0;
    } else if (cap > 0 && cap < maxb) {
        if (rs) {
            if (total > rs->work_cap)
                return fail(c, RASP_E_INVAL, "%llu machines exceed the survivor list of %llu entries",
                            (unsigned long long)total, (unsigned long long)rs->work_cap);
        } else if ((rc = ensure_work(c, total))) {
            return rc;
        }
        uint32_t *work = rs ? rs->work : at<uint32_t>(c, c->work);
        if (lds_first) {
            HIPCHK(c, timed_launch(c, RASP_KERNEL_FIRST, [&] {
                return launch_persistent(dt, total, nullptr, 0, isa, pow2, wm, epoch, P, max_n, max_ell, wpb, blocks, cap, work, qs, st); }));
            HIPCHK(c, timed_launch(c, RASP_KERNEL_OTHER, [&] { return launch_reset_head(qs, st); }));
        } else {
            HIPCHK(c, timed_launch(c, RASP_KERNEL_PLAIN, [&] {
                return launch_plain(dt, total, cap, isa, pow2, pack_in_plain, wm, work, qs, st); }));
        }
        BatchTable *dt2 = dt;
        if (any_fresh) {
            // the survivors' c0 now sits in the arena: their table says so
            BatchTable *ht2;
            int slot2;
            if ((rc = table_slot(c, &ht2, &dt2, &slot2))) return rc;
            if (rs) dt2 = rs->table[1];
            std::memcpy(ht2, ht, sizeof(BatchTable));
            for (uint32_t t = 0; t < k; ++t) ht2->b[t].fresh = 0;
            HIPCHK(c, hipMemcpyAsync(dt2, ht2, sizeof(BatchTable), hipMemcpyHostToDevice, st));
            HIPCHK(c, hipEventRecord(c->table_ev[slot2], st));
            c->table_used[slot2] = true;
        }
        HIPCHK(c, timed_launch(c, RASP_KERNEL_PERSISTENT, [&] {
            return launch_persistent(dt2, total, work, cap, isa, pow2, wm, epoch, P, max_n, max_ell, wpb, blocks, kNoCap, nullptr, qs, st); }));
        for (uint32_t t = 0; t < k; ++t) bs[t]->dev.fresh = 0;
    } else if (cap >= maxb && !lds_first) {
        HIPCHK(c, timed_launch(c, RASP_KERNEL_PLAIN, [&] {
            return launch_plain(dt, total, maxb, isa, pow2, pack_in_plain, wm, nullptr, qs, st); }));
        for (uint32_t t = 0; t < k; ++t) bs[t]->dev.fresh = 0;
    } else {
        // no first pass (or one as long as the budget): one persistent launch;
        // fresh machines here fit their slots and are built by the kernel
        HIPCHK(c, timed_launch(c, RASP_KERNEL_PERSISTENT, [&] {
            return launch_persistent(dt, total, nullptr, 0, isa, pow2, wm, epoch, P, max_n, max_ell, wpb, blocks, kNoCap, nullptr, qs, st); }));
        for (uint32_t t = 0; t < k; ++t) bs[t]->dev.fresh = 0;
    }
    return RASP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of rasp_run_noalloc: one fixed device array per GPU, held until the
// process ends.  Layout: queue counters, two batch tables, then the survivor
// list of up to kNoAllocMaxVms machines.  Host code never passes `scratch`
// itself to a kernel or copy (in host code the name stands for a host-side
// shadow, not a device address): each device's address is taken once, with
// that device current, by hipGetSymbolAddress when a context is created on it.
// ---------------------------------------------------------------------------
namespace {
constexpr uint64_t kNoAllocMaxVms = 1ull << 22;
constexpr uint64_t kNoAllocQueueOff = 0;
constexpr uint64_t kNoAllocTableOff = align_up(sizeof(QueueState), kAlign);
constexpr uint64_t kNoAllocWorkOff = kNoAllocTableOff + 2 * align_up(sizeof(BatchTable), kAlign);
constexpr uint64_t kNoAllocBytes = kNoAllocWorkOff + 4 * kNoAllocMaxVms;
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
char *g_noalloc_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
// this device's address of `scratch` (the device must be current)
hipError_t noalloc_scratch_of(int device, char **out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_noalloc_ptr[device] = static_cast<char *>(ptr);
    }
    *out = g_noalloc_ptr[device];
    return hipSuccess;
}
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

int rasp_create(rasp_ctx **out, int device, void *arena, uint64_t arena_bytes, void *stream)
{
    if (!out) return fail(nullptr, RASP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (arena_bytes < (1ull << 20)) return fail(nullptr, RASP_E_INVAL, "arena must be at least 1 MiB");
    int ndev = 0;
    const hipError_t ec = hipGetDeviceCount(&ndev);
    if (ec != hipSuccess) return fail(nullptr, RASP_E_DEVICE, "hipGetDeviceCount: %s", hipGetErrorString(ec));
    if (device < 0 || device >= ndev) return fail(nullptr, RASP_E_INVAL, "no HIP device %d", device);
    auto c = std::unique_ptr<rasp_ctx>(new (std::nothrow) rasp_ctx());
    if (!c) return fail(nullptr, RASP_E_NOMEM, "host allocation failed");
    c->device = device;
    hipError_t e = hipSetDevice(device);
    hipDeviceProp_t prop;
    if (!e) e = hipGetDeviceProperties(&prop, device);
    if (e) return fail(nullptr, RASP_E_DEVICE, "device query: %s", hipGetErrorString(e));
    c->cus = prop.multiProcessorCount;
    c->wave = prop.warpSize;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) lds = 65536;
    c->lds_bytes = lds;
    if (c->wave != kWave) return fail(nullptr, RASP_E_DEVICE, "wavefront size %d, library built for 64", c->wave);
    if (stream) {
        c->stream = static_cast<hipStream_t>(stream);
    } else {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e) return fail(nullptr, RASP_E_DEVICE, "stream: %s", hipGetErrorString(e));
        c->own_stream = true;
    }
    if (arena) {
        c->arena = static_cast<char *>(arena);
    } else {
        e = hipMalloc(reinterpret_cast<void **>(&c->arena), arena_bytes);
        if (e) {
            if (c->own_stream) (void)hipStreamDestroy(c->stream);
            return fail(nullptr, RASP_E_NOMEM, "arena hipMalloc(%llu): %s", (unsigned long long)arena_bytes, hipGetErrorString(e));
        }
        c->own_arena = true;
    }
    c->arena_bytes = arena_bytes;
    c->alloc.reset(arena_bytes);
    init_kernel_attributes();
    e = noalloc_scratch_of(device, &c->noalloc_scratch);
    if (e) {
        if (c->own_arena) (void)hipFree(c->arena);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        return fail(nullptr, RASP_E_DEVICE, "no-allocation scratch address: %s", hipGetErrorString(e));
    }
    const uint64_t sbytes = align_up(sizeof(QueueState), kAlign) + (kTableRing + 1) * align_up(sizeof(BatchTable), kAlign);
    bool ok = arena_alloc(c.get(), sbytes, &c->scratch);
    if (ok) {
        c->queue = at<QueueState>(c.get(), c->scratch);
        c->tables = at<BatchTable>(c.get(), c->scratch, align_up(sizeof(QueueState), kAlign));
    }
    e = ok ? hipHostMalloc(reinterpret_cast<void **>(&c->host_tables), kTableRing * sizeof(BatchTable), hipHostMallocDefault) : hipErrorOutOfMemory;
    if (!e) e = hipHostMalloc(reinterpret_cast<void **>(&c->tot_host), 64, hipHostMallocDefault);
    if (!e) e = hipHostMalloc(reinterpret_cast<void **>(&c->count_host), 8 * kMaxMulti * kTickets, hipHostMallocDefault);
    for (int k = 0; k < kTickets && !e; ++k) e = hipEventCreateWithFlags(&c->count_ev[k], hipEventDisableTiming);
    for (int k = 0; k < kTableRing && !e; ++k) e = hipEventCreateWithFlags(&c->table_ev[k], hipEventDisableTiming);
    if (e) {
        rasp_destroy(c.release());
        return fail(nullptr, RASP_E_DEVICE, "context scratch: %s", hipGetErrorString(e));
    }
    *out = c.release();
    return RASP_OK;
}

int rasp_create_on_cus(rasp_ctx **out, int device, void *arena, uint64_t arena_bytes, uint32_t cu_first,
                       uint32_t cu_count)
{
    if (!out) return fail(nullptr, RASP_E_INVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    const hipError_t ec = hipGetDeviceCount(&ndev);
    if (ec != hipSuccess) return fail(nullptr, RASP_E_DEVICE, "hipGetDeviceCount: %s", hipGetErrorString(ec));
    if (device < 0 || device >= ndev) return fail(nullptr, RASP_E_INVAL, "no HIP device %d", device);
    hipDeviceProp_t prop;
    hipError_t e = hipSetDevice(device);
    if (!e) e = hipGetDeviceProperties(&prop, device);
    if (e) return fail(nullptr, RASP_E_DEVICE, "device query: %s", hipGetErrorString(e));
    const uint32_t cus = static_cast<uint32_t>(prop.multiProcessorCount);
    if (cu_count == 0 || cu_first >= cus || cu_count > cus - cu_first)
        return fail(nullptr, RASP_E_INVAL, "compute units [%u, %u + %u) are not within the device's %u",
                    cu_first, cu_first, cu_count, cus);
    std::vector<uint32_t> mask((cus + 31) / 32, 0u);
    for (uint32_t k = cu_first; k < cu_first + cu_count; ++k) mask[k / 32] |= 1u << (k % 32);
    hipStream_t st = nullptr;
    e = hipExtStreamCreateWithCUMask(&st, static_cast<uint32_t>(mask.size()), mask.data());
    if (e) return fail(nullptr, RASP_E_DEVICE, "stream on compute units [%u, %u): %s", cu_first,
                       cu_first + cu_count, hipGetErrorString(e));
    const int rc = rasp_create(out, device, arena, arena_bytes, st);
    if (rc) {
        (void)hipStreamDestroy(st);
        return rc;
    }
    (*out)->own_stream = true;
    // launches of this context size their grids to its share of the CUs
    (*out)->cus = static_cast<int>(cu_count);
    (*out)->cu_mask = mask;
    return RASP_OK;
}

int rasp_destroy(rasp_ctx *c)
{
    if (!c) return RASP_OK;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->cstream) (void)hipStreamSynchronize(c->cstream);
    for (auto &g : c->graphs) if (g.exec) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
    for (int k = 0; k < kTableRing; ++k)
        if (c->table_ev[k]) (void)hipEventDestroy(c->table_ev[k]);
    for (auto &t : c->timed) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->host_tables) (void)hipHostFree(c->host_tables);
    if (c->tot_host) (void)hipHostFree(c->tot_host);
    if (c->count_host) (void)hipHostFree(c->count_host);
    if (c->own_arena && c->arena) (void)hipFree(c->arena);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    if (c->stream2) {
        (void)hipStreamSynchronize(c->stream2);
        (void)hipStreamDestroy(c->stream2);
    }
    if (c->ev_first) (void)hipEventDestroy(c->ev_first);
    if (c->ev_second) (void)hipEventDestroy(c->ev_second);
    if (c->cstream) (void)hipStreamDestroy(c->cstream);
    for (int k = 0; k < kTickets; ++k)
        if (c->count_ev[k]) (void)hipEventDestroy(c->count_ev[k]);
    delete c;
    return RASP_OK;
}

const char *rasp_last_error(const rasp_ctx *c)
{
    return c ? c->err.c_str() : g_create_error.c_str();
}

int rasp_batch_footprint(const rasp_batch_desc *d, uint64_t *bytes)
{
    rasp_ctx tmp;                       // only for error text
    int rc = basic_desc_checks(&tmp, d);
    if (rc) return rc;
    if (!bytes) return RASP_E_INVAL;
    const uint64_t N = d->num_vms;
    uint64_t sum_n_pad = 0, sum_ell = 0, sum_s = 0;
    if (d->flags & RASP_DESC_DEVICE_PTRS) {
        std::vector<uint64_t> to(N + 1);
        std::vector<uint32_t> nn, tc, oc;
        if (hipMemcpy(to.data(), d->tape_off, 8 * (N + 1), hipMemcpyDeviceToHost) != hipSuccess) return RASP_E_DEVICE;
        if (d->mem_words) { nn.resize(N); if (hipMemcpy(nn.data(), d->mem_words, 4 * N, hipMemcpyDeviceToHost)) return RASP_E_DEVICE; }
        if (d->tape_cap) { tc.resize(N); if (hipMemcpy(tc.data(), d->tape_cap, 4 * N, hipMemcpyDeviceToHost)) return RASP_E_DEVICE; }
        if (d->out_cap) { oc.resize(N); if (hipMemcpy(oc.data(), d->out_cap, 4 * N, hipMemcpyDeviceToHost)) return RASP_E_DEVICE; }
        for (uint64_t v = 0; v < N; ++v) {
            const uint64_t n = nn.empty() ? d->default_mem_words : nn[v];
            sum_n_pad += (n + 3) & ~3ull;
            sum_ell += tc.empty() ? (to[v + 1] - to[v]) : tc[v];
            sum_s += oc.empty() ? d->default_out_cap : oc[v];
        }
    } else {
        HostShapes h;
        if ((rc = host_shapes(&tmp, d, &h))) return rc;
        sum_n_pad = h.sum_n_pad; sum_ell = h.sum_ell; sum_s = h.sum_s;
    }
    *bytes = meta_bytes(N) + words_bytes(sum_n_pad, sum_ell, sum_s);
    return RASP_OK;
}

int rasp_load_batch(rasp_ctx *c, const rasp_batch_desc *d, rasp_batch *out)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!out) return fail(c, RASP_E_INVAL, "out is NULL");
    std::unique_ptr<Batch> B;
    if ((rc = load_common(c, d, B))) return rc;
    const rasp_batch h = c->next_handle++;
    if ((rc = mark_queued(c, B.get()))) return rc;
    c->batches[h] = std::move(B);
    *out = h;
    return RASP_OK;
}

int rasp_load_state(rasp_ctx *c, const rasp_batch_desc *d, const rasp_outputs *s, rasp_batch *out)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!out || !s || !s->mem || !s->i || !s->a || !s->u0 || !s->y0)
        return fail(c, RASP_E_INVAL, "state needs i, a, u0, y0 and mem");
    std::unique_ptr<Batch> B;
    if ((rc = load_common(c, d, B))) return rc;
    Batch &b = *B;
    hipStream_t st = c->stream;
    const hipMemcpyKind kind = (s->flags & RASP_OUT_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const uint64_t N = b.N;
    Alloc tmp;
    auto undo = [&](int code) {
        (void)hipStreamSynchronize(st);
        arena_free(c, &tmp);
        arena_free(c, &b.words);
        arena_free(c, &b.meta);
        return code;
    };
    hipError_t e = hipMemcpyAsync(b.dev.i, s->i, 4 * N, kind, st);
    if (!e) e = hipMemcpyAsync(b.dev.a, s->a, 4 * N, kind, st);
    if (!e) e = hipMemcpyAsync(b.dev.u0, s->u0, 4 * N, kind, st);
    if (!e) e = hipMemcpyAsync(b.dev.y0, s->y0, 4 * N, kind, st);
    if (!e && s->steps) e = hipMemcpyAsync(b.dev.steps, s->steps, 8 * N, kind, st);
    if (!e && s->y && b.sum_s) e = hipMemcpyAsync(b.dev.Y, s->y, 4 * b.sum_s, kind, st);
    if (e) { fail(c, RASP_E_DEVICE, "state copy: %s", hipGetErrorString(e)); return undo(RASP_E_DEVICE); }
    if (b.uniform_dense) {
        e = hipMemcpyAsync(b.dev.M, s->mem, 4 * b.sum_n, kind, st);
    } else {
        // dense machine-major memory -> padded arena
        const uint64_t nsc = scan_scratch_words(N);
        const uint64_t tb = align_up(8 * N, kAlign) + align_up(8 * nsc, kAlign) + kAlign + align_up(4 * b.sum_n, kAlign);
        if (!arena_alloc(c, tb, &tmp)) { fail(c, RASP_E_NOMEM, "arena cannot stage the state"); return undo(RASP_E_NOMEM); }
        uint64_t *doff = at<uint64_t>(c, tmp);
        uint64_t *sums = at<uint64_t>(c, tmp, align_up(8 * N, kAlign));
        uint64_t *tot = at<uint64_t>(c, tmp, align_up(8 * N, kAlign) + align_up(8 * nsc, kAlign));
        int32_t *dense = at<int32_t>(c, tmp, align_up(8 * N, kAlign) + align_up(8 * nsc, kAlign) + kAlign);
        e = launch_scan_u32(b.dev.n, doff, N, sums, tot, st);
        if (!e) e = hipMemcpyAsync(dense, s->mem, 4 * b.sum_n, kind, st);
        if (!e) e = launch_scatter_words(dense, doff, b.dev.n, N, b.dev.M, b.dev.mem_off, st);
    }
    if (!e) e = launch_tails(b.dev, false, st);            // every memory word is stored
    uint32_t *errw = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(c->tot_host) + 32);
    if (!e) { *errw = 0; }
    // the error word lives in the queue scratch to avoid another allocation
    uint32_t *derr = reinterpret_cast<uint32_t *>(&c->queue->pad);
    if (!e) e = hipMemsetAsync(derr, 0, 4, st);
    if (!e) e = launch_check_state(b.dev, derr, st);
    if (!e) e = launch_check_words(b.dev.M, b.sum_n_pad, b.dev.wshift, derr, st);
    if (!e) e = launch_check_words(b.dev.Y, b.sum_s, b.dev.wshift, derr, st);
    if (!e) e = launch_probe(b.dev, st);
    if (!e) b.status_stale = false;
    if (!e) e = hipMemcpyAsync(errw, derr, 4, hipMemcpyDeviceToHost, st);
    if (!e) e = hipStreamSynchronize(st);
    if (e) { fail(c, RASP_E_DEVICE, "state load: %s", hipGetErrorString(e)); return undo(RASP_E_DEVICE); }
    if (*errw & kErrStateRange) { fail(c, RASP_E_INVAL, "state has u0 > l or y0 > s"); return undo(RASP_E_INVAL); }
    if (*errw) { fail(c, RASP_E_INVAL, "a word of the state is not a %u-bit value", b.wbits); return undo(RASP_E_INVAL); }
    arena_free(c, &tmp);
    const rasp_batch h = c->next_handle++;
    if ((rc = mark_queued(c, B.get()))) return rc;
    c->batches[h] = std::move(B);
    *out = h;
    return RASP_OK;
}

int rasp_run(rasp_ctx *c, rasp_batch h, uint64_t budget)
{
    return rasp_run_multi(c, &h, &budget, 1);
}

int rasp_run_multi(rasp_ctx *c, const rasp_batch *hs, const uint64_t *budgets, uint32_t k)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!hs || !budgets || k == 0 || k > static_cast<uint32_t>(kMaxMulti))
        return fail(c, RASP_E_INVAL, "rasp_run_multi takes 1..%d batches", kMaxMulti);
    std::vector<Batch *> bs(k);
    std::vector<uint64_t> left(budgets, budgets + k);
    for (uint32_t t = 0; t < k; ++t) {
        bs[t] = find(c, hs[t]);
        if (!bs[t]) return fail(c, RASP_E_STATE, "unknown batch handle %llu", (unsigned long long)hs[t]);
        for (uint32_t u = 0; u < t; ++u)
            if (hs[u] == hs[t]) return fail(c, RASP_E_INVAL, "batch %llu listed twice", (unsigned long long)hs[t]);
    }
    // budgets above 2^31 - 1 are applied in several launches (runs compose)
    const uint64_t chunk = 0x7fffffffull;
    for (;;) {
        std::vector<uint32_t> b32(k);
        bool any = false;
        for (uint32_t t = 0; t < k; ++t) {
            const uint64_t x = std::min(left[t], chunk);
            b32[t] = static_cast<uint32_t>(x);
            left[t] -= x;
            any |= x > 0;
        }
        if (!any) break;
        if ((rc = run_batches(c, bs.data(), b32.data(), k))) return rc;
    }
    for (uint32_t t = 0; t < k; ++t)
        if ((rc = mark_queued(c, bs[t]))) return rc;
    return RASP_OK;
}

int rasp_run_async(rasp_ctx *c, const rasp_batch *hs, const uint64_t *budgets, uint32_t k)
{
    return rasp_run_multi(c, hs, budgets, k);
}

int rasp_run_noalloc(rasp_ctx *c, rasp_batch h, uint64_t budget)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    Batch *b = find(c, h);
    if (!b) return fail(c, RASP_E_STATE, "unknown batch handle %llu", (unsigned long long)h);
    if (b->N > kNoAllocMaxVms)
        return fail(c, RASP_E_INVAL, "rasp_run_noalloc takes at most %llu machines; the batch has %llu",
                    (unsigned long long)kNoAllocMaxVms, (unsigned long long)b->N);
    if (!c->noalloc_scratch) return fail(c, RASP_E_DEVICE, "no-allocation scratch is not available");
    RunScratch rs;
    rs.queue = reinterpret_cast<QueueState *>(c->noalloc_scratch + kNoAllocQueueOff);
    rs.table[0] = reinterpret_cast<BatchTable *>(c->noalloc_scratch + kNoAllocTableOff);
    rs.table[1] = reinterpret_cast<BatchTable *>(c->noalloc_scratch + kNoAllocTableOff + align_up(sizeof(BatchTable), kAlign));
    rs.work = reinterpret_cast<uint32_t *>(c->noalloc_scratch + kNoAllocWorkOff);
    rs.work_cap = kNoAllocMaxVms;
    // budgets above 2^31 - 1 are applied in several launches (runs compose)
    uint64_t left = budget;
    c->no_events = true;
    while (left > 0 && rc == RASP_OK) {
        const uint32_t b32 = static_cast<uint32_t>(std::min<uint64_t>(left, 0x7fffffffull));
        left -= b32;
        rc = run_batches(c, &b, &b32, 1, &rs);
    }
    c->no_events = false;
    // the batch's completion event was created by its load: recording it
    // allocates nothing
    if (rc == RASP_OK && b->done) HIPCHK(c, hipEventRecord(b->done, c->stream));
    return rc;
}

int rasp_poll(rasp_ctx *c, rasp_batch h, int *done)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!done) return fail(c, RASP_E_INVAL, "done is NULL");
    hipError_t e;
    if (h == 0) {
        e = hipStreamQuery(c->stream);
    } else {
        Batch *b = find(c, h);
        if (!b) return fail(c, RASP_E_STATE, "unknown batch handle %llu", (unsigned long long)h);
        e = b->done ? hipEventQuery(b->done) : hipSuccess;
    }
    if (e == hipSuccess) { *done = 1; return RASP_OK; }
    if (e == hipErrorNotReady) { *done = 0; return RASP_OK; }
    return fail(c, RASP_E_DEVICE, "completion query: %s", hipGetErrorString(e));
}

int rasp_sync(rasp_ctx *c, rasp_batch h)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (h == 0) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return RASP_OK;
    }
    Batch *b = find(c, h);
    if (!b) return fail(c, RASP_E_STATE, "unknown batch handle %llu", (unsigned long long)h);
    if (b->done) HIPCHK(c, hipEventSynchronize(b->done));
    return RASP_OK;
}

int rasp_fetch_outputs(rasp_ctx *c, rasp_batch h, const rasp_outputs *o)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    Batch *b = find(c, h);
    if (!b) return fail(c, RASP_E_STATE, "unknown batch handle %llu", (unsigned long long)h);
    if (!o) return fail(c, RASP_E_INVAL, "outputs is NULL");
    const bool async = (o->flags & RASP_OUT_ASYNC) != 0;
    if (async && o->mem) return fail(c, RASP_E_INVAL, "memories are not fetched asynchronously");
    if (async && (rc = ensure_cstream(c))) return rc;
    if ((rc = materialize(c, b))) return rc;
    hipStream_t st = c->stream;
    const hipMemcpyKind kind = (o->flags & RASP_OUT_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const uint64_t N = b->N;
    if (o->status && b->status_stale) {
        if ((rc = after_fetch(c, b))) return rc;
        HIPCHK(c, timed_launch(c, RASP_KERNEL_OTHER, [&] { return launch_probe(b->dev, st); }));
        b->status_stale = false;
        if ((rc = mark_queued(c, b))) return rc;
    }
    if (async) {
        // the copy stream takes over behind the batch's own queued work (its
        // event, recorded after its load, runs and probes), not behind work
        // queued since for other batches
        if (!b->done && (rc = mark_queued(c, b))) return rc;
        if (!b->fetch_pending) HIPCHK(c, hipStreamWaitEvent(c->cstream, b->done, 0));
        st = c->cstream;
    } else if ((rc = after_fetch(c, b))) {
        return rc;
    }
    if (kind == hipMemcpyDeviceToDevice) {
        if (o->status || o->steps || o->i || o->a || o->u0 || o->y0)
            HIPCHK(c, timed_launch(c, RASP_KERNEL_OTHER, [&] {
                return launch_fetch_scalars(b->dev, o->status, o->steps, o->i, o->a, o->u0, o->y0, st); }, st));
    } else {
        if (o->status) HIPCHK(c, hipMemcpyAsync(o->status, b->dev.status, N, kind, st));
        if (o->steps) HIPCHK(c, hipMemcpyAsync(o->steps, b->dev.steps, 8 * N, kind, st));
        if (o->i) HIPCHK(c, hipMemcpyAsync(o->i, b->dev.i, 4 * N, kind, st));
        if (o->a) HIPCHK(c, hipMemcpyAsync(o->a, b->dev.a, 4 * N, kind, st));
        if (o->u0) HIPCHK(c, hipMemcpyAsync(o->u0, b->dev.u0, 4 * N, kind, st));
        if (o->y0) HIPCHK(c, hipMemcpyAsync(o->y0, b->dev.y0, 4 * N, kind, st));
    }
    if (o->y && b->sum_s) HIPCHK(c, hipMemcpyAsync(o->y, b->dev.Y, 4 * b->sum_s, kind, st));
    Alloc tmp;
    if (o->mem_digest) {
        if (kind == hipMemcpyDeviceToDevice) {
            HIPCHK(c, timed_launch(c, RASP_KERNEL_DIGEST, [&] { return launch_digest(b->dev, o->mem_digest, st); }, st));
        } else if (async) {
            // the batch's own digest buffer, kept (and reused by later
            // asynchronous fetches) until the batch is released
            if (!b->fetch_tmp.live && !arena_alloc(c, 8 * N, &b->fetch_tmp))
                return fail(c, RASP_E_NOMEM, "arena cannot hold digests");
            uint64_t *dd = at<uint64_t>(c, b->fetch_tmp);
            HIPCHK(c, timed_launch(c, RASP_KERNEL_DIGEST, [&] { return launch_digest(b->dev, dd, st); }, st));
            HIPCHK(c, hipMemcpyAsync(o->mem_digest, dd, 8 * N, kind, st));
        } else {
            if (!arena_alloc(c, 8 * N, &tmp)) return fail(c, RASP_E_NOMEM, "arena cannot hold digests");
            HIPCHK(c, timed_launch(c, RASP_KERNEL_DIGEST, [&] { return launch_digest(b->dev, at<uint64_t>(c, tmp), st); }));
            HIPCHK(c, hipMemcpyAsync(o->mem_digest, at<uint64_t>(c, tmp), 8 * N, kind, st));
            HIPCHK(c, hipStreamSynchronize(st));
            arena_free(c, &tmp);
        }
    }
    if (o->mem) {
        if ((rc = store_tails(c, b))) return rc;
        if (b->uniform_dense) {
            HIPCHK(c, hipMemcpyAsync(o->mem, b->dev.M, 4 * b->sum_n, kind, st));
        } else {
            // padded arena -> dense machine-major, through an arena buffer
            const uint64_t nsc = scan_scratch_words(N);
            const uint64_t tb = align_up(8 * N, kAlign) + align_up(8 * nsc, kAlign) + kAlign +
                                (kind == hipMemcpyDeviceToDevice ? 0 : align_up(4 * b->sum_n, kAlign));
            if (!arena_alloc(c, tb, &tmp)) return fail(c, RASP_E_NOMEM, "arena cannot stage the memory dump");
            uint64_t *doff = at<uint64_t>(c, tmp);
            uint64_t *sums = at<uint64_t>(c, tmp, align_up(8 * N, kAlign));
            uint64_t *tot = at<uint64_t>(c, tmp, align_up(8 * N, kAlign) + align_up(8 * nsc, kAlign));
            int32_t *dense = kind == hipMemcpyDeviceToDevice
                                 ? o->mem
                                 : at<int32_t>(c, tmp, align_up(8 * N, kAlign) + align_up(8 * nsc, kAlign) + kAlign);
            HIPCHK(c, launch_scan_u32(b->dev.n, doff, N, sums, tot, st));
            HIPCHK(c, launch_gather_words(b->dev.M, b->dev.mem_off, b->dev.n, N, dense, doff, st));
            if (kind != hipMemcpyDeviceToDevice)
                HIPCHK(c, hipMemcpyAsync(o->mem, dense, 4 * b->sum_n, kind, st));
            HIPCHK(c, hipStreamSynchronize(st));
            arena_free(c, &tmp);
        }
    }
    if (async) {
        HIPCHK(c, hipEventRecord(b->done, st));
        b->fetch_pending = true;
        return RASP_OK;
    }
    HIPCHK(c, hipStreamSynchronize(st));
    return RASP_OK;
}

int rasp_batch_info(rasp_ctx *c, rasp_batch h, uint64_t *num_vms, uint64_t *mem_words,
                    uint64_t *out_words, uint64_t *steps_sum)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    Batch *b = find(c, h);
    if (!b) return fail(c, RASP_E_STATE, "unknown batch handle %llu", (unsigned long long)h);
    if (num_vms) *num_vms = b->N;
    if (mem_words) *mem_words = b->sum_n;
    if (out_words) *out_words = b->sum_s;
    if (steps_sum) {
        if ((rc = materialize(c, b))) return rc;
        unsigned long long *d = reinterpret_cast<unsigned long long *>(&c->queue->retired);
        HIPCHK(c, hipMemsetAsync(d, 0, 8, c->stream));
        HIPCHK(c, launch_steps_sum(b->dev, d, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->tot_host, d, 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *steps_sum = c->tot_host[0];
    }
    return RASP_OK;
}

int rasp_running_counts_async(rasp_ctx *c, const rasp_batch *hs, uint32_t k, uint64_t *ticket)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!hs || !ticket || k == 0 || k > static_cast<uint32_t>(kMaxMulti))
        return fail(c, RASP_E_INVAL, "running counts take 1..%d batches and a ticket", kMaxMulti);
    hipStream_t st = c->stream;
    Batch *bb[kMaxMulti];
    for (uint32_t t = 0; t < k; ++t) {
        bb[t] = find(c, hs[t]);
        if (!bb[t]) return fail(c, RASP_E_STATE, "unknown batch handle %llu", (unsigned long long)hs[t]);
    }
    // the slot of this ticket: one still unclaimed there is waited for and dropped
    const uint64_t tk = c->ticket_next;
    const int s = static_cast<int>(tk % kTickets);
    if (c->ticket_of[s]) {
        HIPCHK(c, hipEventSynchronize(c->count_ev[s]));
        c->ticket_of[s] = 0;
    }
    BatchTable *ht, *dt;
    int slot;
    if ((rc = table_slot(c, &ht, &dt, &slot))) return rc;
    std::memset(ht, 0, sizeof(BatchTable));
    uint64_t total = 0;
    for (uint32_t t = 0; t < k; ++t) {
        Batch *b = bb[t];
        if ((rc = materialize(c, b))) return rc;
        if (b->status_stale) {
            if ((rc = after_fetch(c, b))) return rc;
            HIPCHK(c, timed_launch(c, RASP_KERNEL_OTHER, [&] { return launch_probe(b->dev, st); }));
            b->status_stale = false;
            if ((rc = mark_queued(c, b))) return rc;
        }
        ht->b[t] = b->dev;
        ht->start[t] = total;
        total += b->N;
    }
    ht->start[k] = total;
    ht->count = k;
    unsigned long long *dcount = reinterpret_cast<unsigned long long *>(&c->tables[kTableRing]) + s * kMaxMulti;
    uint64_t *hcount = c->count_host + s * kMaxMulti;
    HIPCHK(c, hipMemcpyAsync(dt, ht, sizeof(BatchTable), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipEventRecord(c->table_ev[slot], st));
    c->table_used[slot] = true;
    HIPCHK(c, hipMemsetAsync(dcount, 0, 8 * kMaxMulti, st));
    HIPCHK(c, timed_launch(c, RASP_KERNEL_OTHER, [&] { return launch_running(dt, total, dcount, st); }));
    HIPCHK(c, hipMemcpyAsync(hcount, dcount, 8 * k, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipEventRecord(c->count_ev[s], st));
    c->ticket_of[s] = tk;
    c->ticket_k[s] = k;
    ++c->ticket_next;
    *ticket = tk;
    return RASP_OK;
}

int rasp_running_counts_wait(rasp_ctx *c, uint64_t ticket, uint64_t *counts)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!counts) return fail(c, RASP_E_INVAL, "counts is NULL");
    const int s = static_cast<int>(ticket % kTickets);
    if (ticket == 0 || c->ticket_of[s] != ticket)
        return fail(c, RASP_E_STATE, "ticket %llu is unknown, already claimed or dropped (at most %d in flight)",
                    (unsigned long long)ticket, kTickets);
    HIPCHK(c, hipEventSynchronize(c->count_ev[s]));
    std::memcpy(counts, c->count_host + s * kMaxMulti, 8 * c->ticket_k[s]);
    c->ticket_of[s] = 0;
    return RASP_OK;
}

int rasp_running_counts(rasp_ctx *c, const rasp_batch *hs, uint32_t k, uint64_t *counts)
{
    uint64_t tk = 0;
    int rc = rasp_running_counts_async(c, hs, k, &tk);
    if (rc) return rc;
    return rasp_running_counts_wait(c, tk, counts);
}

int rasp_free_batch(rasp_ctx *c, rasp_batch h)
{
    if (!c) return RASP_E_INVAL;
    auto it = c->batches.find(h);
    if (it == c->batches.end()) return fail(c, RASP_E_STATE, "unknown or freed batch handle %llu", (unsigned long long)h);
    if (it->second->fetch_pending) HIPCHK(c, hipEventSynchronize(it->second->done));
    arena_free(c, &it->second->fetch_tmp);
    drop_graphs(c, false, reinterpret_cast<uint64_t>(it->second.get()));
    // later work on the same stream may reuse the space only after this batch's
    // queued work: stream order guarantees it
    arena_free(c, &it->second->words);
    arena_free(c, &it->second->meta);
    c->batches.erase(it);
    return RASP_OK;
}

int rasp_set_option(rasp_ctx *c, int option, int64_t value)
{
    if (!c) return RASP_E_INVAL;
    switch (option) {
    case RASP_OPT_SCHEDULE:
        if (value < RASP_SCHED_AUTO || value > RASP_SCHED_PERSISTENT) return fail(c, RASP_E_INVAL, "bad schedule");
        c->schedule = value; return RASP_OK;
    case RASP_OPT_EPOCH:
        if (value < 1 || value > 0x7fffffff) return fail(c, RASP_E_INVAL, "epoch must be >= 1");
        c->epoch = value; return RASP_OK;
    case RASP_OPT_LDS_WORDS:
        if (value < -1 || value > 1024 || (value > 0 && (value & 3)))
            return fail(c, RASP_E_INVAL, "lds words must be -1 (auto), 0 or a multiple of 4 in [4, 1024]");
        c->lds_words = value; return RASP_OK;
    case RASP_OPT_WAVES_PER_CU:
        if (value < 1 || value > 32) return fail(c, RASP_E_INVAL, "waves per CU must be in [1, 32]");
        c->waves_per_cu = value; return RASP_OK;
    case RASP_OPT_GRAPH:
        c->graph = value ? 1 : 0;
        if (!c->graph) drop_graphs(c, true);
        return RASP_OK;
    case RASP_OPT_FIRST_PASS:
        if (value < 0 || value > 0x7fffffff) return fail(c, RASP_E_INVAL, "first pass must be >= 0");
        c->first_pass = value; return RASP_OK;
    case RASP_OPT_PROFILE:
        c->profile = value ? 1 : 0; return RASP_OK;
    case RASP_OPT_FIRST_PASS_KIND:
        if (value != 0 && value != 1) return fail(c, RASP_E_INVAL, "first pass kind must be 0 or 1");
        c->first_pass_kind = value; return RASP_OK;
    case RASP_OPT_HOT_CELLS:
        if (value != 0 && value != 8 && value != 16 && value != 32 && value != 64)
            return fail(c, RASP_E_INVAL, "hot cells must be 0, 8, 16, 32 or 64");
        c->hot_cells = value; return RASP_OK;
    case RASP_OPT_PROFILE_STEPS:
        if (value < 1 || value > 0x7fffffff) return fail(c, RASP_E_INVAL, "profile steps must be >= 1");
        c->profile_steps = value; return RASP_OK;
    case RASP_OPT_MISFIT_WAVES:
        if (value < 1 || value > 32) return fail(c, RASP_E_INVAL, "misfit waves per CU must be in [1, 32]");
        c->misfit_waves = value; return RASP_OK;
    default:
        return fail(c, RASP_E_INVAL, "unknown option %d", option);
    }
}

int rasp_get_option(rasp_ctx *c, int option, int64_t *value)
{
    if (!c || !value) return RASP_E_INVAL;
    switch (option) {
    case RASP_OPT_SCHEDULE: *value = c->schedule; return RASP_OK;
    case RASP_OPT_EPOCH: *value = c->epoch; return RASP_OK;
    case RASP_OPT_LDS_WORDS: *value = c->lds_words; return RASP_OK;
    case RASP_OPT_WAVES_PER_CU: *value = c->waves_per_cu; return RASP_OK;
    case RASP_OPT_GRAPH: *value = c->graph; return RASP_OK;
    case RASP_OPT_FIRST_PASS: *value = c->first_pass; return RASP_OK;
    case RASP_OPT_PROFILE: *value = c->profile; return RASP_OK;
    case RASP_OPT_FIRST_PASS_KIND: *value = c->first_pass_kind; return RASP_OK;
    case RASP_OPT_HOT_CELLS: *value = c->hot_cells; return RASP_OK;
    case RASP_OPT_PROFILE_STEPS: *value = c->profile_steps; return RASP_OK;
    case RASP_OPT_MISFIT_WAVES: *value = c->misfit_waves; return RASP_OK;
    default: return fail(c, RASP_E_INVAL, "unknown option %d", option);
    }
}

int rasp_kernel_times(rasp_ctx *c, double *ms, uint64_t *launches)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto &t : c->timed) {
        float x = 0.f;
        HIPCHK(c, hipEventElapsedTime(&x, t.a, t.b));
        if (t.kind >= 0 && t.kind < RASP_KERNEL_COUNT) {
            if (ms) ms[t.kind] += x;
            if (launches) launches[t.kind] += 1;
        }
        c->ev_pool.push_back(t.a);
        c->ev_pool.push_back(t.b);
    }
    c->timed.clear();
    return RASP_OK;
}

// knobs the autotuner chooses, in the order of its `chosen` array
constexpr int kTuneKnobs = 9;

// a knob moves away from the current setting only for a trial at least 3%
// faster: timings of near-equal settings differ by noise from run to run
constexpr double kTuneMargin = 0.97;

int rasp_autotune(rasp_ctx *c, rasp_batch h, uint64_t budget, uint64_t max_vms, int64_t *chosen,
                  double *best_ms)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    Batch *b = find(c, h);
    if (!b) return fail(c, RASP_E_STATE, "unknown batch handle %llu", (unsigned long long)h);
    // a lazily loaded batch stays lazy: every trial rebuilds c0 of the prefix
    // from the caller's descriptor arrays, as the real run will
    const bool lazy = b->dev.fresh != 0;
    hipStream_t st = c->stream;
    const uint64_t K = (max_vms == 0 || max_vms > b->N) ? b->N : max_vms;
    const uint32_t bud = static_cast<uint32_t>(std::min<uint64_t>(budget, 0x7fffffffull));
    // ends of the prefix's word ranges
    uint64_t mo, to, yo;
    uint32_t nn, el, ss;
    HIPCHK(c, hipMemcpyAsync(&mo, b->dev.mem_off + K - 1, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(&to, b->dev.t_off + K - 1, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(&yo, b->dev.y_off + K - 1, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(&nn, b->dev.n + K - 1, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(&el, b->dev.ell + K - 1, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(&ss, b->dev.s + K - 1, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    const uint64_t m_end = mo + ((nn + 3ull) & ~3ull), t_end = to + el, y_end = yo + ss;
    // snapshot (restore source) and trial batch, both K machines; a lazy
    // batch needs no snapshot (its c0 is rebuilt from the descriptor)
    Batch snap, trial;
    std::vector<Batch *> parts = {&trial};
    if (!lazy) parts.push_back(&snap);
    for (Batch *x : parts) {
        *x = Batch();
        x->N = K;
        x->sum_n_pad = m_end; x->sum_ell = t_end; x->sum_s = y_end;
        x->max_n = b->max_n; x->max_ell = b->max_ell; x->all_pow2 = b->all_pow2;
        x->status_stale = b->status_stale;
        x->tails = b->tails;
        x->wbits = b->wbits;
        if (!arena_alloc(c, meta_bytes(K), &x->meta) || !arena_alloc(c, words_bytes(m_end, t_end, y_end), &x->words)) {
            arena_free(c, &snap.meta); arena_free(c, &snap.words);
            arena_free(c, &trial.meta); arena_free(c, &trial.words);
            return fail(c, RASP_E_NOMEM, "arena cannot hold the autotune snapshot (%llu machines)", (unsigned long long)K);
        }
        carve_meta(at<char>(c, x->meta), K, &x->dev);
        carve_words(at<char>(c, x->words), m_end, t_end, &x->dev);
        x->dev.isa = b->dev.isa;
        x->dev.wshift = b->dev.wshift;
        x->dev.fresh = 0;
        x->dev.prog = b->dev.prog; x->dev.prog_off = b->dev.prog_off;
        x->dev.tape = b->dev.tape; x->dev.tape_off = b->dev.tape_off;
    }
    auto copy_shapes = [&](const DevBatch &src, const DevBatch &dst) -> hipError_t {
        const hipMemcpyKind k = hipMemcpyDeviceToDevice;
        hipError_t e = hipMemcpyAsync(dst.n, src.n, 4 * K, k, st);
        if (!e) e = hipMemcpyAsync(dst.ell, src.ell, 4 * K, k, st);
        if (!e) e = hipMemcpyAsync(dst.s, src.s, 4 * K, k, st);
        if (!e) e = hipMemcpyAsync(dst.mem_off, src.mem_off, 8 * K, k, st);
        if (!e) e = hipMemcpyAsync(dst.t_off, src.t_off, 8 * K, k, st);
        if (!e) e = hipMemcpyAsync(dst.y_off, src.y_off, 8 * K, k, st);
        return e;
    };
    auto copy_batch = [&](const DevBatch &src, const DevBatch &dst) -> hipError_t {
        const hipMemcpyKind k = hipMemcpyDeviceToDevice;
        hipError_t e = hipMemcpyAsync(dst.i, src.i, 4 * K, k, st);
        if (!e) e = hipMemcpyAsync(dst.a, src.a, 4 * K, k, st);
        if (!e) e = hipMemcpyAsync(dst.u0, src.u0, 4 * K, k, st);
        if (!e) e = hipMemcpyAsync(dst.y0, src.y0, 4 * K, k, st);
        if (!e) e = hipMemcpyAsync(dst.steps, src.steps, 8 * K, k, st);
        if (!e) e = hipMemcpyAsync(dst.status, src.status, K, k, st);
        if (!e) e = copy_shapes(src, dst);
        if (!e) e = hipMemcpyAsync(dst.hw, src.hw, 4 * K, k, st);
        if (!e) e = hipMemcpyAsync(dst.M, src.M, 4 * m_end, k, st);
        if (!e && t_end) e = hipMemcpyAsync(dst.T, src.T, 4 * t_end, k, st);
        if (!e && y_end) e = hipMemcpyAsync(dst.Y, src.Y, 4 * y_end, k, st);
        return e;
    };
    auto release = [&]() {
        (void)hipStreamSynchronize(st);
        arena_free(c, &snap.meta); arena_free(c, &snap.words);
        arena_free(c, &trial.meta); arena_free(c, &trial.words);
    };
    hipError_t e = lazy ? copy_shapes(b->dev, trial.dev) : copy_batch(b->dev, snap.dev);
    if (e) { release(); return fail(c, RASP_E_DEVICE, "autotune snapshot: %s", hipGetErrorString(e)); }
    const int64_t saved[] = {c->schedule, c->lds_words, c->first_pass, c->epoch, c->waves_per_cu,
                             c->first_pass_kind, c->hot_cells, c->profile_steps, c->misfit_waves,
                             c->graph, c->profile};
    c->graph = 0;
    c->profile = 0;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    // one trial: the best of up to three runs from the snapshot while a run
    // takes under 20 ms (short runs are the noisy ones), else one run
    auto trial_ms = [&](double *ms) -> int {
        double best_run = 1e30;
        for (int rep = 0; rep < 3; ++rep) {
            if (lazy) {
                trial.dev.fresh = 1;
            } else {
                hipError_t x = copy_batch(snap.dev, trial.dev);
                if (x) return fail(c, RASP_E_DEVICE, "autotune restore: %s", hipGetErrorString(x));
                trial.status_stale = snap.status_stale;
                trial.tails = snap.tails;
            }
            Batch *tb = &trial;
            HIPCHK(c, hipEventRecord(e0, st));
            int r2 = run_batches(c, &tb, &bud, 1);
            if (r2) return r2;
            HIPCHK(c, hipEventRecord(e1, st));
            HIPCHK(c, hipEventSynchronize(e1));
            float f = 0.f;
            HIPCHK(c, hipEventElapsedTime(&f, e0, e1));
            best_run = std::min(best_run, static_cast<double>(f));
            if (f >= 20.f) break;
        }
        *ms = best_run;
        return RASP_OK;
    };
    // candidate values; one knob at a time from the current setting
    const int64_t full = std::max<int64_t>(4, (static_cast<int64_t>(b->max_n) + 3) & ~int64_t(3));
    std::vector<int64_t> lds_c = {0, 32, 64, 128, 256};
    if (full <= 1024 && std::find(lds_c.begin(), lds_c.end(), full) == lds_c.end()) lds_c.push_back(full);
    // and the largest split (low words in LDS, the rest in HBM) that keeps
    // k waves of a compute unit resident: programs that touch only their low
    // cells then run from LDS at a higher occupancy, and memories far larger
    // than any slot keep their hottest low words in LDS at the occupancy
    // that hides the latency of the rest.
    for (int64_t k : {3, 4, 6, 8, 10, 12, 14, 16}) {
        int64_t Pk = (static_cast<int64_t>(c->lds_bytes) / (k * kWave * 4) - 4) & ~int64_t(3);
        if (Pk > 0 && Pk < b->max_n && std::find(lds_c.begin(), lds_c.end(), Pk) == lds_c.end()) lds_c.push_back(Pk);
    }
    const std::vector<int64_t> fp_c = {0, 16, 64, 256}, ep_c = {16, 64, 256, 1024}, wv_c = {8, 16, 32},
                               fk_c = {0, 1};
    int64_t cur[kTuneKnobs] = {RASP_SCHED_PERSISTENT,
                               c->lds_words < 0 ? static_cast<int64_t>(lds_words_for(c, b->max_n, b->max_ell)) : c->lds_words,
                               c->first_pass, c->epoch, c->waves_per_cu, c->first_pass_kind, 0, c->profile_steps,
                               c->misfit_waves};
    auto apply = [&](const int64_t *o) {
        c->schedule = o[0]; c->lds_words = o[1]; c->first_pass = o[2]; c->epoch = o[3]; c->waves_per_cu = o[4];
        c->first_pass_kind = o[5]; c->hot_cells = o[6]; c->profile_steps = o[7]; c->misfit_waves = o[8];
    };
    // one coordinate search (LDS words, first-pass length, epoch, waves per
    // CU) for each first-pass kind, from the same start; the kinds interact
    // with every other knob, so they are not searched one after the other
    int64_t start[kTuneKnobs];
    for (int q = 0; q < kTuneKnobs; ++q) start[q] = cur[q];
    const std::vector<int64_t> *lists[5] = {nullptr, &lds_c, &fp_c, &ep_c, &wv_c};
    double best = 1e30;
    bool warm = false;
    for (int64_t kind : fk_c) {
        if (rc) break;
        int64_t kc[kTuneKnobs];
        for (int q = 0; q < kTuneKnobs; ++q) kc[q] = start[q];
        kc[5] = kind;
        double kbest = 1e30;
        apply(kc);
        if (!warm) { rc = trial_ms(&kbest); warm = true; }     // warm-up run
        if (!rc) rc = trial_ms(&kbest);
        for (int knob = 1; knob <= 4 && !rc; ++knob) {
            for (int64_t val : *lists[knob]) {
                if (val == kc[knob]) continue;
                // the LDS first pass needs whole memories in their slots;
                // with a smaller slot it is the plain first pass, timed already
                if (knob == 1 && kind == 1 && val < static_cast<int64_t>(b->max_n)) continue;
                if (knob == 1 && val > 0 &&
                    static_cast<uint64_t>(kWave) * slot_words(static_cast<uint32_t>(val), b->max_n, b->max_ell) * 4 >
                        static_cast<uint64_t>(c->lds_bytes)) continue;
                int64_t o[kTuneKnobs];
                for (int q = 0; q < kTuneKnobs; ++q) o[q] = kc[q];
                o[knob] = val;
                apply(o);
                double ms = 0;
                if ((rc = trial_ms(&ms))) break;
                if (ms < kbest * kTuneMargin) { kbest = ms; kc[knob] = val; }
            }
        }
        if (!rc && kbest < best * kTuneMargin) {
            best = kbest;
            for (int q = 0; q < kTuneKnobs; ++q) cur[q] = kc[q];
        }
    }
    // hot-cell tables (memories of at most kHotMaxN words, a budget beyond
    // the profiled first pass): slots per machine and the misfits' waves per
    // CU on a grid, then the profile length for the best of them; each
    // against the best setting so far
    if (!rc && b->max_n <= kHotMaxN && bud > 2048) {
        int64_t hb[kTuneKnobs];
        double hbest = 1e30;
        for (int64_t S : {16, 32}) {
            for (int64_t mw : {6, 8, 12}) {
                int64_t o[kTuneKnobs];
                for (int q = 0; q < kTuneKnobs; ++q) o[q] = cur[q];
                o[0] = RASP_SCHED_PERSISTENT; o[2] = 576; o[5] = 0; o[6] = S; o[7] = 512; o[8] = mw;
                o[4] = 16;
                apply(o);
                double ms = 0;
                if ((rc = trial_ms(&ms))) break;
                if (ms < hbest * kTuneMargin) { hbest = ms; for (int q = 0; q < kTuneKnobs; ++q) hb[q] = o[q]; }
            }
            if (rc) break;
        }
        for (int64_t prof : {256, 1024}) {
            if (rc || hbest >= 1e30) break;
            int64_t o[kTuneKnobs];
            for (int q = 0; q < kTuneKnobs; ++q) o[q] = hb[q];
            o[7] = prof; o[2] = prof + 64;
            apply(o);
            double ms = 0;
            if ((rc = trial_ms(&ms))) break;
            if (ms < hbest * kTuneMargin) { hbest = ms; for (int q = 0; q < kTuneKnobs; ++q) hb[q] = o[q]; }
        }
        if (!rc && hbest < best * kTuneMargin) {
            best = hbest;
            for (int q = 0; q < kTuneKnobs; ++q) cur[q] = hb[q];
        }
    }
    if (!rc) {                              // the plain schedule as a whole
        int64_t o[kTuneKnobs];
        for (int q = 0; q < kTuneKnobs; ++q) o[q] = cur[q];
        o[0] = RASP_SCHED_PLAIN;
        o[6] = 0;
        apply(o);
        double ms = 0;
        rc = trial_ms(&ms);
        if (!rc && ms < best * kTuneMargin) { best = ms; cur[0] = RASP_SCHED_PLAIN; cur[6] = 0; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    release();
    c->graph = saved[9];
    c->profile = saved[10];
    if (rc) {
        apply(saved);
        return rc;
    }
    apply(cur);
    if (chosen) for (int q = 0; q < kTuneKnobs; ++q) chosen[q] = cur[q];
    if (best_ms) *best_ms = best;
    return RASP_OK;
}

int rasp_device_info(rasp_ctx *c, int *cus, int *lds_bytes, int *wave_size)
{
    if (!c) return RASP_E_INVAL;
    if (cus) *cus = c->cus;
    if (lds_bytes) *lds_bytes = c->lds_bytes;
    if (wave_size) *wave_size = c->wave;
    return RASP_OK;
}

}  // extern "C"
