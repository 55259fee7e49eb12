// rasp_kernels.hip -- gfx950 kernels of librasp.
//
// The step loop advances one RASP machine per lane.  A machine's configuration
// <i, a, M, u, y> (Sec. 1.1; word RASP of Sec. 2.1) lives in struct-of-arrays
// scalars (i, a, u0, y0, steps, status) plus per-machine word slices of three
// arenas: memory M (program stored at M[0..2m), Sec. 2), tape T, output Y.
//
// One transition (Sec. 2.1 case table; classic set of Sec. 1.1 plus JMP):
//   fetch   o = M[i mod n], j = M[(i+1) mod n]      (circular addressing)
//   decode  one-hot choice of the case (the guarded sum of Sec. 2.1, taken as
//           predicates rather than branches); the machine is at a fixed point
//           (F) when no case moves it: unknown opcode, READ with u0 >= l, or a
//           taken jump whose target equals i
//   execute LOAD a <- j; ADD/SUB/MUL a <- a (+,-,*) M[j mod n]; STORE
//           M[j mod n] <- a; READ M[j mod n] <- T[u0], u0++; PRINT (if y0 < s)
//           Y[y0] <- M[j mod n], y0++; jumps i <- j; otherwise i <- i + 2;
//           all word arithmetic wraps mod 2^w (w = 32, or a narrower word
//           held sign-extended in 32 bits).
// `mod n` is the Euclidean remainder of the signed word (result in [0, n)).
// The position p = i mod n is carried along with i so that the usual
// sequential advance costs an add and a compare instead of a division.

#include "rasp_internal.h"

#include <type_traits>

namespace rasp {

// ---------------------------------------------------------------------------
// circular addressing
// ---------------------------------------------------------------------------

// Euclidean remainder of a signed word by n (1 <= n <= 2^30); the common case
// of an in-range word costs one compare.
__device__ __forceinline__ uint32_t cmod(int32_t v, uint32_t n)
{
    if (static_cast<uint32_t>(v) < n) return static_cast<uint32_t>(v);
    if ((n & (n - 1u)) == 0u) return static_cast<uint32_t>(v) & (n - 1u);
    const int32_t r = v % static_cast<int32_t>(n);
    return static_cast<uint32_t>(r < 0 ? r + static_cast<int32_t>(n) : r);
}

// the w-bit word of x (ws = 32 - w): low w bits, sign-extended
__device__ __forceinline__ int32_t sext(uint32_t x, uint32_t ws)
{
    return static_cast<int32_t>(x << ws) >> ws;
}

// position of the operand word (i + 1) mod n, given p = i mod n; imax is the
// largest w-bit word, where i + 1 wraps to the smallest
__device__ __forceinline__ uint32_t operand_pos(int32_t i, uint32_t p, uint32_t n, int32_t imax)
{
    const uint32_t q = p + 1u;
    uint32_t r = q == n ? 0u : q;
    if (i == imax) r = cmod(-imax - 1, n);
    return r;
}

// position of i + 2 (wrapping mod 2^w) given p = i mod n
__device__ __forceinline__ uint32_t advance_pos(int32_t i, uint32_t p, uint32_t n, int32_t imax,
                                                uint32_t ws)
{
    uint32_t q = p + 2u;
    if (q >= n) q -= n;
    if (q >= n) q -= n;                                     // n == 1
    if (i > imax - 2) q = cmod(sext(static_cast<uint32_t>(i) + 2u, ws), n);
    return q;
}

// ---------------------------------------------------------------------------
// memory accessors.  kLds: every word of the machine is in its LDS slot, so
// the data word is read unconditionally and a store that does not happen is
// redirected to the slot's spare word (no branch).  Otherwise reads and
// stores that would touch HBM are predicated; a split slot first tests, once
// per transition for the whole wave, whether any lane touches HBM at all.
// step() does one transition's memory traffic in program order.
// ---------------------------------------------------------------------------

extern __shared__ int32_t rasp_lds[];

// whether any active lane of the wave has x set (the lane mask of x, ANDed
// with exec, tested in scalar registers)
__device__ __forceinline__ bool any_lane(bool x)
{
    return __builtin_amdgcn_ballot_w64(x) != 0;
}

// pointers known to address global memory: loads and stores compile to
// global_* instructions instead of flat_* ones (which also wait on LDS)
typedef __attribute__((address_space(1))) int32_t gi32;
typedef __attribute__((address_space(1))) uint64_t gu64;
__device__ __forceinline__ gi32 *gptr(int32_t *p) { return (gi32 *)p; }
__device__ __forceinline__ const gi32 *gptr(const int32_t *p) { return (const gi32 *)p; }

// The next instruction's two words from HBM: one 8-byte load of the cell
// holding word np (memory slices are padded to a multiple of 4 words, so the
// cell of the last word of an odd-sized memory is in bounds), and a second
// load only for a lane whose operand is not the cell's second word.
// Scattered loads cost the vector memory pipeline a request per lane.
__device__ __forceinline__ void fetch_pair(const gi32 *M, uint32_t np, uint32_t nq, int32_t &o, int32_t &j)
{
    const uint64_t e = *reinterpret_cast<const gu64 *>(M + (np & ~1u));
    const int32_t e0 = static_cast<int32_t>(static_cast<uint32_t>(e)), e1 = static_cast<int32_t>(e >> 32);
    const bool odd = (np & 1u) != 0u, two = odd | (nq != np + 1u);
    int32_t j2 = 0;
    if (two) j2 = M[nq];
    o = odd ? e1 : e0;
    j = two ? j2 : e1;
}

struct GlobalMem {                       // every word in HBM
    static constexpr bool kLds = false;
    static constexpr bool kColdIO = false;
    gi32 *M;
    __device__ __forceinline__ int32_t ld(uint32_t k) const { return M[k]; }
    __device__ __forceinline__ int32_t ld_data(uint32_t k, bool need) const
    {
        int32_t v = 0;
        if (need) v = M[k];
        return v;
    }
    __device__ __forceinline__ void st(uint32_t k, int32_t v, bool en) const { if (en) M[k] = v; }
    // one transition's memory traffic in program order: the current
    // instruction's store, its data word, then the next instruction's words
    __device__ __forceinline__ void step(uint32_t jj, int32_t w, bool st_en, bool need, uint32_t np,
                                         uint32_t nq, int32_t &d, int32_t &o, int32_t &j) const
    {
        st(jj, w, st_en);
        d = ld_data(jj, need);
        fetch_pair(M, np, nq, o, j);
    }
};

// round up to a multiple of 4 words
__device__ __forceinline__ uint32_t up4(uint32_t x) { return (x + 3u) & ~3u; }


// bcast of a lane's value to the wave (defined with the pack kernel below)
__device__ __forceinline__ uint32_t bcast(uint32_t x, uint32_t L);
__device__ __forceinline__ uint64_t bcast64(uint64_t x, uint32_t L);

// The lanes with f set store their zero tails [hw, top), the wave's active
// lanes together on one machine at a time (a word a lane: this sits inside
// step loops, where a wider store would hold more registers), and set
// hw = top.  Every active lane takes part.
__device__ __forceinline__ void store_tails(bool f, gi32 *M, uint32_t &hw, uint32_t top)
{
    uint64_t m = __builtin_amdgcn_ballot_w64(f);
    if (m == 0) return;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t act = __builtin_amdgcn_ballot_w64(true);
    const uint32_t rank = __popcll(act & ((1ull << lane) - 1ull)), cnt = __popcll(act);
    do {
        const uint32_t L = static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(m)) - 1);
        m &= m - 1ull;
        gi32 *const ML = reinterpret_cast<gi32 *>(bcast64(reinterpret_cast<uint64_t>(M), L));
        const uint32_t h = bcast(hw, L), t = bcast(top, L);
        for (uint32_t x = h + rank; x < t; x += cnt) ML[x] = 0;
    } while (m);
    if (f) hw = top;
}

// every word in HBM, c0's zero tail not yet stored: words at or above hw read
// as zero; a store at k >= hw first stores zeros in words [hw, k] (up to a
// multiple of 4), which become the new hw
struct TailMem {
    static constexpr bool kLds = false;
    static constexpr bool kColdIO = false;
    gi32 *M;
    mutable uint32_t hw;
    __device__ __forceinline__ int32_t ld(uint32_t k) const
    {
        int32_t v = 0;
        if (k < hw) v = M[k];
        return v;
    }
    __device__ __forceinline__ int32_t ld_data(uint32_t k, bool need) const
    {
        int32_t v = 0;
        if (need & (k < hw)) v = M[k];
        return v;
    }
    __device__ __forceinline__ void st(uint32_t k, int32_t v, bool en) const
    {
        const bool f = en & (k >= hw);
        if (__builtin_expect(any_lane(f), 0)) store_tails(f, M, hw, up4(k + 1u));
        if (en) M[k] = v;
    }
    __device__ __forceinline__ void step(uint32_t jj, int32_t w, bool st_en, bool need, uint32_t np,
                                         uint32_t nq, int32_t &d, int32_t &o, int32_t &j) const
    {
        st(jj, w, st_en);
        d = ld_data(jj, need);
        // as fetch_pair; hw is a multiple of 4, so a cell lies wholly below
        // it or wholly above
        const uint32_t c0 = np & ~1u;
        uint64_t e = 0;
        if (c0 < hw) e = *reinterpret_cast<const gu64 *>(M + c0);
        const int32_t e0 = static_cast<int32_t>(static_cast<uint32_t>(e)), e1 = static_cast<int32_t>(e >> 32);
        const bool odd = (np & 1u) != 0u;
        o = odd ? e1 : e0;
        j = e1;
        if (odd | (nq != np + 1u)) j = ld(nq);
    }
};

// LDS slots are interleaved across the lanes of a wave: word k of lane l's
// slot is LDS word wave_base + 64 k + l, so the bank a lane touches depends on
// its lane alone and the 64 lanes of a wave never conflict, whatever
// positions they read (lanes running similar programs in step would collide
// in lane-contiguous slots).  `base` below is wave_base + l; word k is at
// base + (k << 6).
constexpr uint32_t kSlotShift = 6;       // log2 of the distance between a slot's consecutive words

struct LdsMem {                          // whole memory in the lane's LDS slot (n <= P)
    static constexpr bool kLds = true;
    static constexpr bool kColdIO = false;
    uint32_t base;                       // LDS word index of the machine's word 0
    uint32_t spare;                      // index of the slot's spare word
    __device__ __forceinline__ int32_t ld(uint32_t k) const { return rasp_lds[base + (k << kSlotShift)]; }
    __device__ __forceinline__ int32_t ld_data(uint32_t k, bool) const { return ld(k); }
    __device__ __forceinline__ void st(uint32_t k, int32_t v, bool en) const
    {
        rasp_lds[en ? base + (k << kSlotShift) : spare] = v;
    }
    __device__ __forceinline__ void step(uint32_t jj, int32_t w, bool st_en, bool need, uint32_t np,
                                         uint32_t nq, int32_t &d, int32_t &o, int32_t &j) const
    {
        st(jj, w, st_en);
        d = ld_data(jj, need);
        o = ld(np);
        j = ld(nq);
    }
};

struct SplitMem {                        // words [0, P) in LDS, the rest in HBM
    static constexpr bool kLds = false;
    // split slots serve memories larger than LDS holds whole, typically
    // array programs whose reads and prints come in bursts at the start and
    // end: the step loop tests once per transition, for the whole wave,
    // whether any lane reads the tape, appends an output word, touches a
    // word at or above P or needs the general positions, and lays all of
    // that out of line
    static constexpr bool kColdIO = true;
    uint32_t base, P;                    // slot word k < P at base + (k << 6), the spare at k = P
    gi32 *M;
    __device__ __forceinline__ int32_t ld(uint32_t k) const
    {
        int32_t v;
        if (k < P) v = rasp_lds[base + (k << kSlotShift)]; else v = M[k];
        return v;
    }
    __device__ __forceinline__ int32_t ld_data(uint32_t k, bool need) const
    {
        int32_t v = 0;
        if (k < P) v = rasp_lds[base + (k << kSlotShift)]; else if (need) v = M[k];
        return v;
    }
    __device__ __forceinline__ void st(uint32_t k, int32_t v, bool en) const
    {
        if (en) { if (k < P) rasp_lds[base + (k << kSlotShift)] = v; else M[k] = v; }
    }
    // each access picks LDS or HBM per lane
    __device__ __forceinline__ void step(uint32_t jj, int32_t w, bool st_en, bool need, uint32_t np,
                                         uint32_t nq, int32_t &d, int32_t &o, int32_t &j) const
    {
        st(jj, w, st_en);
        d = ld_data(jj, need);
        o = ld(np);
        j = ld(nq);
    }
    // every access of every lane below P, and the next operand at np + 1
    // (no wrap): straight LDS accesses, the next instruction's two words in
    // one read.  jx is the data position of a lane that stores or reads its
    // data word, else 0; the spare word after the P memory words takes the
    // stores of lanes that do not store.
    __device__ __forceinline__ void step_near(uint32_t jx, int32_t w, bool st_en, uint32_t np,
                                              int32_t &d, int32_t &o, int32_t &j) const
    {
        int32_t *const pd = &rasp_lds[base + (jx << kSlotShift)];
        *(st_en ? pd : &rasp_lds[base + (P << kSlotShift)]) = w;
        d = *pd;
        const int32_t *const pn = &rasp_lds[base + (np << kSlotShift)];
        o = pn[0];
        j = pn[1u << kSlotShift];
    }
};

// Hot-cell slot of cell x (words 2x, 2x + 1) for multiplier c: bits
// [16, 16 + log2 S) of x * c (cells are below 2^10, c at most 2^16, so a
// 24-bit multiply is exact); c = 2^16 places consecutive cells in
// consecutive slots
__device__ __forceinline__ uint32_t hot_slot(uint32_t x, uint32_t c, uint32_t mask)
{
    return (__umul24(x, c) >> 16) & mask;
}

// the multiplier tried `k`-th when a profiled machine's cells are placed
__device__ __forceinline__ uint32_t hot_mult(uint32_t k)
{
    return k == 0 ? 65536u : (((k * 0x9E3779B1u) >> 16) | 1u);
}
constexpr uint32_t kHotCandidates = 64;

// every word in HBM, and every cell an access touches marked in the lane's
// profile bitmap (LDS, bit x of the bitmap = cell x; word k of a thread's
// bitmap at bm + k * stride): the fetched cell, and the data cell when the
// transition stores or reads its data word
struct ProfMem {
    static constexpr bool kLds = false;
    static constexpr bool kColdIO = false;
    gi32 *M;
    uint32_t bm, stride;
    __device__ __forceinline__ void mark(uint32_t k) const
    {
        const uint32_t x = k >> 1;
        atomicOr(reinterpret_cast<uint32_t *>(&rasp_lds[bm + (x >> 5) * stride]), 1u << (x & 31u));
    }
    __device__ __forceinline__ int32_t ld(uint32_t k) const { return M[k]; }
    __device__ __forceinline__ void step(uint32_t jj, int32_t w, bool st_en, bool need, uint32_t np,
                                         uint32_t nq, int32_t &d, int32_t &o, int32_t &j) const
    {
        mark(np);
        mark(nq);
        if (st_en | need) mark(jj);
        if (st_en) M[jj] = w;
        d = 0;
        if (need) d = M[jj];
        fetch_pair(M, np, nq, o, j);
    }
};

// A machine's hot cells in its lane's LDS table, every other word in HBM.
// Slot s of lane l: its two words at word wb + 128 s (wb = wave base + 2 l),
// its cell tag (uint16, 0xffff: empty) at halfword tb + 64 s (tb = tag
// base + l): the bank a lane reads depends on its lane, not on the slot it
// picks (the 64 lanes' two-word reads cover 128 consecutive words).  The LDS
// copy of a tagged cell is the machine's word; HBM holds it again only after
// the write-back.  The table starts with the machine's profiled cells; a
// cell missed later whose slot is empty joins it.
struct HotMem {
    static constexpr bool kLds = false;
    static constexpr bool kColdIO = false;
    uint32_t wb, tb, c, mask;
    gi32 *M;
    __device__ __forceinline__ uint32_t slot(uint32_t x) const { return hot_slot(x, c, mask); }
    __device__ __forceinline__ uint32_t tag(uint32_t s) const
    {
        return reinterpret_cast<const uint16_t *>(rasp_lds)[tb + 64u * s];
    }
    __device__ __forceinline__ int2 pair(uint32_t s) const
    {
        return *reinterpret_cast<const int2 *>(&rasp_lds[wb + 128u * s]);
    }
    __device__ __forceinline__ void put(uint32_t s, uint32_t half, int32_t v) const
    {
        rasp_lds[wb + 128u * s + half] = v;
    }
    // LDS word index of word `half` of slot s
    __device__ __forceinline__ uint32_t word(uint32_t s, uint32_t half) const { return wb + 128u * s + half; }
    __device__ __forceinline__ int32_t ld(uint32_t k) const
    {
        const uint32_t x = k >> 1, s = slot(x);
        int32_t v;
        if (tag(s) == x) v = rasp_lds[wb + 128u * s + (k & 1u)]; else v = M[k];
        return v;
    }
    __device__ __forceinline__ int32_t ld_data(uint32_t k, bool need) const
    {
        const uint32_t x = k >> 1, s = slot(x);
        int32_t v = 0;
        if (tag(s) == x) v = rasp_lds[wb + 128u * s + (k & 1u)]; else if (need) v = M[k];
        return v;
    }
    __device__ __forceinline__ void st(uint32_t k, int32_t v, bool en) const
    {
        const uint32_t x = k >> 1, s = slot(x);
        if (en) { if (tag(s) == x) put(s, k & 1u, v); else M[k] = v; }
    }
    // each access looks its cell up on its own (general positions, a
    // misaligned fetch, an operand that wraps, or cells not in the table)
    __device__ __forceinline__ void step(uint32_t jj, int32_t w, bool st_en, bool need, uint32_t np,
                                         uint32_t nq, int32_t &d, int32_t &o, int32_t &j) const
    {
        st(jj, w, st_en);
        d = ld_data(jj, need);
        o = ld(np);
        j = ld(nq);
    }
};

// input tape: in HBM, or staged in the lane's LDS slot
struct TapeG {
    static constexpr bool kLds = false;
    const gi32 *T;
    __device__ __forceinline__ int32_t ld(uint32_t k) const { return T[k]; }
};

struct TapeL {                           // tape word k at base + (k << 6) (interleaved slot)
    static constexpr bool kLds = true;
    uint32_t base;
    __device__ __forceinline__ int32_t ld(uint32_t k) const { return rasp_lds[base + (k << kSlotShift)]; }
};

// output words, appended in HBM
struct OutG {
    gi32 *Y;
    __device__ __forceinline__ void st(uint32_t k, int32_t v, bool en) const { if (en) Y[k] = v; }
};

// ---------------------------------------------------------------------------
// the step loop
// ---------------------------------------------------------------------------

struct Regs {
    int32_t i, a;
    uint32_t p;          // i mod n
    uint32_t u0, y0;
    uint32_t n, ell, s;
};

// the fixed-point predicate of the current configuration (F of Sec. 1.1/2.1):
// unknown opcode, READ with the tape used up, or a taken jump onto itself
template <int ISA>
__device__ __forceinline__ bool stuck(uint32_t op, int32_t j, int32_t a, int32_t i, uint32_t u0, uint32_t ell)
{
    bool taken, valid;
    if (ISA == 1) {
        taken = (op == 8u) | ((op == 5u) & (a > 0));
        valid = (op - 1u) < 8u;
    } else {
        taken = (op == 5u) & (a != 0);
        valid = (op - 1u) < 7u;
    }
    return !valid | ((op == 6u) & (u0 >= ell)) | (taken & (j == i));
}

// Advance one machine by at most `limit` transitions.  Returns the number
// applied; `halted` says whether the machine now sits on a fixed point.
// (The plain kernel and the persistent kernel's slot memories run this loop,
// each lane leaving it on its own; memory wholly in HBM and hot-cell tables
// run the lockstep loop below.)
//
// Software-pipelined: the words of the next instruction are loaded together
// with the data word of the current one (after the current store, so that a
// program that rewrites its next instruction sees the new word), leaving one
// memory round trip per transition; the loop has a single exit.
// POW2 (n a power of two): v mod n = v & (n-1) for every int32 v, and
// (i + k) mod n = (p + k) mod n across the int32 wrap, so positions need no
// division and no special case.  Otherwise the common case -- operand word in
// [0, n), i not within 4 of INT32_MAX, n >= 2 -- is straight-line code and
// the general positions are computed out of line, behind one wave-uniform
// branch that is not taken while no lane needs them (a split slot folds that
// test into its one test for all uncommon work, and there a lane needs them
// only when it uses its data position or jumps).
// WM: words narrower than 32 bits (ws = 32 - w; POW2 then also needs n <= 2^w).
// A tape staged in LDS is read one step ahead: the word at u0 is loaded with
// the next instruction's words, so a READ costs no extra round trip.
template <int ISA, bool POW2, bool WM, class Mem, class Tape, class Out>
__device__ __forceinline__ uint32_t run_machine(const Mem &mem, const Tape &tape, Regs &r,
                                                const Out &out,
                                                uint32_t limit, bool &halted,
                                                uint32_t ws)
{
    const uint32_t n = r.n, nm = r.n - 1u, ell = r.ell, s = r.s;
    const int32_t imax = WM ? static_cast<int32_t>(0x7fffffffu >> ws) : INT32_MAX;
    uint32_t p = r.p, u0 = r.u0, y0 = r.y0;
    int32_t i = r.i, a = r.a;
    int32_t o = mem.ld(p);
    int32_t j = mem.ld(POW2 ? ((p + 1u) & nm) : operand_pos(i, p, n, imax));
    int32_t tv = Tape::kLds ? tape.ld(u0) : 0;          // u0 <= l: the region has l + 1 words
    // split slot: a lane's step is uncommon when its largest position in use,
    // np + 1 included, reaches min(n, P) (a word in HBM, a next operand that
    // wraps to word 0, or an operand outside [0, n) that needs the general
    // positions) or when i is within 4 of the largest word (every step when
    // n < 2)
    uint32_t lim = 0u;
    int32_t ilim = 0;
    if constexpr (Mem::kColdIO) {
        lim = min(n, mem.P);
        ilim = n < 2u ? INT32_MIN : imax - 3;
    }
    uint32_t left = limit;
    for (;;) {
        const uint32_t op = static_cast<uint32_t>(o);
        const bool is_rd = op == 6u;
        bool taken, valid;
        if (ISA == 1) {                  // classic: JPOS (a > 0), JMP
            taken = (op == 8u) | ((op == 5u) & (a > 0));
            valid = (op - 1u) < 8u;
        } else {                         // word: BNZ (a != 0)
            taken = (op == 5u) & (a != 0);
            valid = (op - 1u) < 7u;
        }
        const bool rd_ok = is_rd & (u0 < ell);
        const bool fixed = !valid | (is_rd & !rd_ok) | (taken & (j == i));
        if (fixed | (left == 0u)) break;

        const bool st_en = (op == 4u) | rd_ok;
        const bool need = (op == 2u) | (op == 3u) | (op == 7u);
        const bool app = (op == 7u) & (y0 < s);

        // positions: data word jj = j mod n, next instruction np, its operand nq
        uint32_t jj, seq, np, nq;
        bool rare = false;
        const uint32_t i2 = static_cast<uint32_t>(i) + 2u;
        const int32_t ni = taken ? j : (WM ? sext(i2, ws) : static_cast<int32_t>(i2));
        if (POW2) {
            jj = static_cast<uint32_t>(j) & nm;
            seq = (p + 2u) & nm;
            np = taken ? jj : seq;
            nq = (np + 1u) & nm;
        } else {
            jj = static_cast<uint32_t>(j);
            seq = p + 2u;
            seq = seq >= n ? seq - n : seq;
            np = taken ? jj : seq;
            nq = np + 1u;
            nq = nq == n ? 0u : nq;
            // jj = j only for j in [0, n); with w < 32 a jump target j < n can
            // also be the largest word, whose operand position i + 1 wraps.
            // (A split slot tests its lanes below, with its uncommon work.)
            if constexpr (!Mem::kColdIO) {
                rare = (static_cast<uint32_t>(j) >= n) | (i >= imax - 3) | (n < 2u);
                if (WM) rare |= j >= imax - 3;
            }
        }
        // the general positions, for the lanes that need them (every lane
        // computes them: the caller branches on a wave-uniform test)
        auto general_positions = [&]() {
            const uint32_t jj2 = cmod(j, n);
            const uint32_t seq2 = advance_pos(i, p, n, imax, WM ? ws : 0u);
            const uint32_t np2 = taken ? jj2 : seq2;
            const uint32_t nq2 = operand_pos(ni, np2, n, imax);
            jj = rare ? jj2 : jj;
            np = rare ? np2 : np;
            nq = rare ? nq2 : nq;
        };

        int32_t w = a;
        const int32_t jcur = j;
        int32_t d;
        if constexpr (Mem::kColdIO) {
            // one wave-uniform test for everything uncommon: general
            // positions, a tape read, an output word, a word at or above P,
            // an operand that wraps to word 0.  jx is the data position of a
            // lane that uses it, else 0.  For n >= 2 the larger of jx and np
            // reaches n exactly when j is outside [0, n) and the lane uses jj
            // or jumps to j; np + 1 reaches min(n, P) when the next operand
            // wraps (np = n - 1) or lies at or above P.
            const uint32_t jx = (st_en | need) ? jj : 0u;
            const uint32_t m = max(jx, np);
            const bool j_top = WM && !POW2 && taken && (j >= imax - 3);
            bool cold = app | (max(m, np + 1u) >= lim) | j_top;
            if (!POW2) cold |= i >= ilim;
            if (!Tape::kLds) cold |= rd_ok;
            if (__builtin_expect(any_lane(cold), 0)) {
                if (!POW2) {
                    rare = (m >= n) | (i >= ilim) | j_top;
                    if (any_lane(rare)) general_positions();
                }
                if (Tape::kLds) w = rd_ok ? tv : a;
                else if (rd_ok) w = tape.ld(u0);
                mem.step(jj, w, st_en, need, np, nq, d, o, j);
                out.st(y0, d, app);
            } else {
                if (Tape::kLds) w = rd_ok ? tv : a;
                mem.step_near(jx, w, st_en, np, d, o, j);
            }
        } else {
            if (!POW2 && __builtin_expect(any_lane(rare), 0)) general_positions();
            if (Tape::kLds) w = rd_ok ? tv : a;                // loaded one step ahead
            else if (rd_ok) w = tape.ld(u0);
            mem.step(jj, w, st_en, need, np, nq, d, o, j);
        }
        // the stored word's register is not reused while the store may still
        // read it: a reuse before the next instruction's loads would wait for
        // the store to complete, a second memory round trip
        __asm__ volatile("" : : "v"(w));
        u0 += rd_ok ? 1u : 0u;
        if (Tape::kLds) tv = tape.ld(u0);

        const uint32_t ua = static_cast<uint32_t>(a), ud = static_cast<uint32_t>(d);
        uint32_t na = op == 3u ? (ISA == 1 ? ua - ud : ua * ud) : ua;
        na = op == 2u ? ua + ud : na;
        if (WM) na = static_cast<uint32_t>(sext(na, ws));
        na = op == 1u ? static_cast<uint32_t>(jcur) : na;
        a = static_cast<int32_t>(na);
        if constexpr (!Mem::kColdIO) out.st(y0, d, app);
        y0 += app ? 1u : 0u;
        i = ni;
        p = np;
        --left;
    }
    halted = stuck<ISA>(static_cast<uint32_t>(o), j, a, i, u0, ell);
    r.i = i; r.a = a; r.p = p; r.u0 = u0; r.y0 = y0;
    return limit - left;
}

// the accumulator after opcode op: LOAD takes the operand j, ADD/SUB (MUL in
// the word set) combine a with the data word d, wrapping at w bits
template <int ISA, bool WM>
__device__ __forceinline__ int32_t accumulate(uint32_t op, int32_t a, int32_t d, int32_t j, uint32_t ws)
{
    const uint32_t ua = static_cast<uint32_t>(a), ud = static_cast<uint32_t>(d);
    uint32_t na = op == 3u ? (ISA == 1 ? ua - ud : ua * ud) : ua;
    na = op == 2u ? ua + ud : na;
    if (WM) na = static_cast<uint32_t>(sext(na, ws));
    na = op == 1u ? static_cast<uint32_t>(j) : na;
    return static_cast<int32_t>(na);
}

// The lockstep step loop, for a machine's memory in a hot-cell table
// (HotMem) or wholly in HBM (GlobalMem).  The active lanes of the wave take
// their transitions together, at most L of them (L wave-uniform, counted in a
// scalar register).  A lane's transition is common when
//   * its opcode is LOAD, ADD, SUB/MUL, STORE, the conditional jump, JMP
//     (classic set) or PRINT with the output full -- not HALT, READ, an
//     unknown opcode or an append;
//   * it is not a jump onto its own instruction (i' = i);
//   * (n not a power of two) neither i nor a jump target is within 4 of the
//     largest word (where i + 2 or the next operand's position i' + 1 wraps);
//   * (hot-cell table) the next instruction's cell and, for ADD, SUB/MUL and
//     STORE, the data cell are in the table (their tags match), and the next
//     instruction sits at an even position whose operand follows it without
//     wrapping.
// An operand outside [0, n) that a lane uses as its data position or jump
// target is reduced to its Euclidean remainder first (one wave-uniform test;
// a multiply-high by a per-machine reciprocal, no division).
// The inner loop takes common transitions while every lane has one: the
// straight step (table: LDS reads, HBM: the store or data load and the next
// instruction's cell in one 8-byte load), with no test for a fixed point
// (none is common) and no per-lane loop exit.  At a transition that is not
// common for some lane, the outer loop tests every lane for a fixed point
// exactly (stopping there if any lane sits on one) and takes that one
// transition with general positions and the memory's general accesses, as
// the general step loop does.  Returns the transitions taken, the same for
// every active lane; `halted` says whether the lane now sits on a fixed point.
template <int ISA, bool POW2, bool WM, class Mem, class Tape>
__device__ __forceinline__ uint32_t run_lockstep(const Mem &mem, const Tape &tape, const OutG &out, Regs &r,
                                                 uint32_t L, bool &halted, uint32_t ws)
{
    constexpr bool kTable = std::is_same<Mem, HotMem>::value;
    constexpr bool kHbm = std::is_same<Mem, GlobalMem>::value;
    // bit k: opcode k is common (opcodes above 31 are taken as 31); a memory
    // of fewer than two words has no common transition
    constexpr uint32_t kCommon = ISA == 1 ? 0x1beu : 0xbeu;
    const uint32_t n = r.n, nm = r.n - 1u, ell = r.ell, s = r.s;
    const int32_t imax = WM ? static_cast<int32_t>(0x7fffffffu >> ws) : INT32_MAX;
    // Euclidean remainders by n (not a power of two, n >= 2): see below
    uint32_t rinv = 0, big = 0;
    if (!POW2 && n >= 2u) {
        rinv = 0xffffffffu / n;
        big = (0x80000000u / n + (0x80000000u % n != 0u)) * n;
    }
    uint32_t p = r.p, u0 = r.u0, y0 = r.y0;
    int32_t i = r.i, a = r.a;
    const uint32_t q0 = POW2 ? ((p + 1u) & nm) : operand_pos(i, p, n, imax);
    static_assert(kTable || kHbm, "a hot-cell table or HBM");
    int32_t o, j;
    if constexpr (kHbm) {
        fetch_pair(mem.M, p, q0, o, j);
    } else {
        o = mem.ld(p);
        j = mem.ld(q0);
    }
    uint32_t k = 0;
    for (;;) {
        // PRINT is common while the output is full
        const uint32_t coldops = n < 2u ? ~0u : (~kCommon | (y0 < s ? 0x80u : 0u));
        for (; k < L; ++k) {
            const uint32_t op = static_cast<uint32_t>(o);
            bool taken;
            if (ISA == 1) taken = (op == 8u) | ((op == 5u) & (a > 0));
            else taken = (op == 5u) & (a != 0);
            const uint32_t i2 = static_cast<uint32_t>(i) + 2u;
            const int32_t ni = taken ? j : (WM ? sext(i2, ws) : static_cast<int32_t>(i2));
            const bool uses = (op - 2u) < 3u;                // ADD, SUB/MUL, STORE
            // j mod n: an operand outside [0, n) that a lane uses as its data
            // position or jump target takes its Euclidean remainder (one
            // wave-uniform test; the others' operands are left as they are)
            uint32_t jm = static_cast<uint32_t>(j);
            if (POW2) {
                jm &= nm;
            } else if (__builtin_expect(any_lane((jm >= n) & (uses | taken)), 0)) {
                // a negative word is moved up by big (a multiple of n, at
                // least 2^31) into [0, 2^32); rinv = floor((2^32 - 1) / n)
                // gives the quotient of the unsigned word less at most one
                const uint32_t u = static_cast<uint32_t>(j) + (j < 0 ? big : 0u);
                const uint32_t rr = u - __umulhi(u, rinv) * n;
                jm = rr >= n ? rr - n : rr;
            }
            // the next instruction's position, and the data position of a
            // lane that uses its data word (else the next instruction's again)
            uint32_t np;
            if (POW2) {
                np = taken ? jm : ((p + 2u) & nm);
            } else {
                const uint32_t q = p + 2u;
                np = taken ? jm : min(q, q - n);
            }
            const uint32_t np1 = np + 1u;
            const uint32_t opc = min(op, 31u);
            const uint32_t jx = uses ? jm : np;
            const int32_t jcur = j;
            if constexpr (kTable) {
                const uint32_t cf = np >> 1, cd = jx >> 1;
                const uint32_t sf = mem.slot(cf), sd = mem.slot(cd);
                const uint32_t dwi = mem.word(sd, jx & 1u);
                const int2 ef = mem.pair(sf);
                const int32_t dv = rasp_lds[dwi];
                const uint32_t tf = mem.tag(sf), td = mem.tag(sd);
                // the four reads issue together (one LDS round trip a step):
                // the slot reads are not left behind the test of the tags
                __builtin_amdgcn_sched_barrier(0);
                // each condition's lane mask, ORed in scalar registers
                const uint32_t bad = (tf ^ cf) | (td ^ cd) | (np & 1u) | ((coldops >> opc) & 1u);
                uint64_t cold = __builtin_amdgcn_ballot_w64(bad != 0u) | __builtin_amdgcn_ballot_w64(ni == i);
                if (!POW2) {
                    cold |= __builtin_amdgcn_ballot_w64(np1 == n) | __builtin_amdgcn_ballot_w64(i >= imax - 3);
                    cold |= __builtin_amdgcn_ballot_w64(taken & (j >= imax - 3));
                }
                if (__builtin_expect(cold != 0, 0)) break;
                // every cell hit: a store into the next instruction's words is
                // seen by its fetch (equal positions are the same LDS word)
                const bool st = op == 4u;
                if (st) rasp_lds[dwi] = a;
                o = (st & (jx == np)) ? a : ef.x;
                j = (st & (jx == np1)) ? a : ef.y;
                a = accumulate<ISA, WM>(op, a, dv, jcur, ws);
            } else {
                uint64_t cold = __builtin_amdgcn_ballot_w64(((coldops >> opc) & 1u) != 0u) |
                                __builtin_amdgcn_ballot_w64(ni == i);
                if (!POW2) {
                    cold |= __builtin_amdgcn_ballot_w64(i >= imax - 3);
                    cold |= __builtin_amdgcn_ballot_w64(taken & (j >= imax - 3));
                }
                if (__builtin_expect(cold != 0, 0)) break;
                const uint32_t nq = POW2 ? (np1 & nm) : (np1 == n ? 0u : np1);
                // program order: the store, the data word, the next
                // instruction's words (a store into them is seen by the fetch)
                if (op == 4u) mem.M[jx] = a;
                int32_t d = 0;
                if ((op - 2u) < 2u) d = mem.M[jx];           // ADD, SUB/MUL
                fetch_pair(mem.M, np, nq, o, j);
                a = accumulate<ISA, WM>(op, a, d, jcur, ws);
            }
            i = ni;
            p = np;
        }
        if (k == L) break;
        // a transition that is not common for some lane
        const uint32_t op = static_cast<uint32_t>(o);
        bool taken, valid;
        if (ISA == 1) {
            taken = (op == 8u) | ((op == 5u) & (a > 0));
            valid = (op - 1u) < 8u;
        } else {
            taken = (op == 5u) & (a != 0);
            valid = (op - 1u) < 7u;
        }
        const bool is_rd = op == 6u;
        const bool rd_ok = is_rd & (u0 < ell);
        if (any_lane(!valid | (is_rd & !rd_ok) | (taken & (j == i)))) break;
        const bool st_en = (op == 4u) | rd_ok;
        const bool need = (op == 2u) | (op == 3u) | (op == 7u);
        const bool app = (op == 7u) & (y0 < s);
        const uint32_t i2 = static_cast<uint32_t>(i) + 2u;
        const int32_t ni = taken ? j : (WM ? sext(i2, ws) : static_cast<int32_t>(i2));
        uint32_t jj, np, nq;
        if (POW2) {
            jj = static_cast<uint32_t>(j) & nm;
            np = taken ? jj : ((p + 2u) & nm);
            nq = (np + 1u) & nm;
        } else {
            // as in the general loop: the common positions, and the general
            // ones for a lane that needs them
            jj = static_cast<uint32_t>(j);
            uint32_t q = p + 2u;
            q = q >= n ? q - n : q;
            np = taken ? jj : q;
            nq = np + 1u;
            nq = nq == n ? 0u : nq;
            bool rare = ((static_cast<uint32_t>(j) >= n) & (st_en | need | taken)) | (i >= imax - 3) | (n < 2u);
            if (WM) rare |= taken & (j >= imax - 3);
            if (any_lane(rare)) {
                const uint32_t jj2 = cmod(j, n);
                const uint32_t np2 = taken ? jj2 : advance_pos(i, p, n, imax, WM ? ws : 0u);
                const uint32_t nq2 = operand_pos(ni, np2, n, imax);
                jj = rare ? jj2 : jj;
                np = rare ? np2 : np;
                nq = rare ? nq2 : nq;
            }
        }
        int32_t w = a, d;
        if (rd_ok) w = tape.ld(u0);
        const int32_t jcur = j;
        mem.step(jj, w, st_en, need, np, nq, d, o, j);
        __asm__ volatile("" : : "v"(w));                  // as in the general loop
        if constexpr (kTable) {
            // a cell missed here whose slot is empty enters the table (its
            // two words from HBM, which holds every cell outside the table,
            // this transition's store included): the next instruction's
            // cell, else the data cell of a lane that used it
            const uint32_t xf = np >> 1, xd = jj >> 1;
            const uint32_t sf = mem.slot(xf), sd = mem.slot(xd);
            const bool ef = mem.tag(sf) == 0xffffu;
            const bool ed = (st_en | need) & (xd != xf) & (sd != sf) & (mem.tag(sd) == 0xffffu);
            if (__builtin_expect(any_lane(ef | ed), 0)) {
                const uint32_t x = ef ? xf : xd, sl = ef ? sf : sd;
                if (ef | ed) {
                    const uint64_t e = *reinterpret_cast<const gu64 *>(mem.M + 2u * x);
                    mem.put(sl, 0u, static_cast<int32_t>(static_cast<uint32_t>(e)));
                    mem.put(sl, 1u, static_cast<int32_t>(e >> 32));
                    reinterpret_cast<uint16_t *>(rasp_lds)[mem.tb + 64u * sl] = static_cast<uint16_t>(x);
                }
            }
        }
        out.st(y0, d, app);
        u0 += rd_ok ? 1u : 0u;
        y0 += app ? 1u : 0u;
        a = accumulate<ISA, WM>(op, a, d, jcur, ws);
        i = ni;
        p = np;
        ++k;
    }
    halted = stuck<ISA>(static_cast<uint32_t>(o), j, a, i, u0, ell);
    r.i = i; r.a = a; r.p = p; r.u0 = u0; r.y0 = y0;
    return k;
}

__device__ __forceinline__ int batch_of(const BatchTable *tab, uint64_t g)
{
    int lo = 0, hi = static_cast<int>(tab->count) - 1;
    while (lo < hi) {                    // last k with start[k] <= g
        const int mid = (lo + hi + 1) >> 1;
        if (tab->start[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// K1: pack c0 (Sec. 2.1): M = P 0^(n-2m), T = x 0^(l-|x|), Y = 0^s, scalars 0.
// Only the program words of M are stored (rounded up to 16 bytes); hw marks
// where the zero tail begins, and the step loops read it as zeros.
// One wave per 64 consecutive machines: the scalars and shapes are read and
// written coalesced (lane = machine); then the wave walks its 64 machines and
// copies each memory slice with 16-byte accesses (64 lanes x 4 words).
// status is written RUNNING here; the host marks it stale and the first run
// (or a probe) computes whether c0 is already a fixed point.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t bcast(uint32_t x, uint32_t L)
{
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), static_cast<int>(L)));
}

__device__ __forceinline__ uint64_t bcast64(uint64_t x, uint32_t L)
{
    return (static_cast<uint64_t>(bcast(static_cast<uint32_t>(x >> 32), L)) << 32) |
           bcast(static_cast<uint32_t>(x), L);
}

constexpr int kPackGroup = 4;            // machines whose loads are in flight together

__global__ __launch_bounds__(256) void k_pack(DevBatch b, const int32_t *__restrict__ prog,
                                              const uint64_t *__restrict__ prog_off,
                                              const int32_t *__restrict__ tape,
                                              const uint64_t *__restrict__ tape_off)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t wave = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) / kWave;
    for (uint64_t g = wave * kWave; g < b.N; g += nwaves * kWave) {
        const uint64_t v = g + lane;
        uint64_t p0 = 0, t0 = 0, mo = 0, to = 0, yo = 0;
        uint32_t plen = 0, tlen = 0, n = 0, ell = 0, s = 0;
        if (v < b.N) {
            p0 = prog_off[v];
            plen = static_cast<uint32_t>(prog_off[v + 1] - p0);
            t0 = tape_off[v];
            tlen = static_cast<uint32_t>(tape_off[v + 1] - t0);
            n = b.n[v]; ell = b.ell[v]; s = b.s[v];
            mo = b.mem_off[v]; to = b.t_off[v]; yo = b.y_off[v];
            b.i[v] = 0; b.a[v] = 0; b.u0[v] = 0; b.y0[v] = 0; b.steps[v] = 0; b.status[v] = 0;
            b.hw[v] = min(up4(plen), up4(n));
        }
        const uint32_t cnt = static_cast<uint32_t>(b.N - g < kWave ? b.N - g : kWave);
        // Every machine of the wave one row wide (n <= 256 words, l and s <=
        // 64, program 16-byte aligned and a multiple of 4 words): the loads of
        // kPackGroup machines go out together -- each at an address clamped
        // into its program or tape, the words past the end replaced by zeros
        // afterwards -- so a group costs one memory round trip instead of one
        // per machine.
        const bool row = v >= b.N || (n <= 4u * kWave && ell <= kWave && s <= kWave &&
                                      (p0 & 3u) == 0 && (plen & 3u) == 0);
        if (__ballot(!row) == 0) {
            const uint32_t k = 4u * lane;
            for (uint32_t L0 = 0; L0 < cnt; L0 += kPackGroup) {
                int4 x[kPackGroup];
                int32_t y[kPackGroup];
#pragma unroll
                for (int u = 0; u < kPackGroup; ++u) {
                    const uint32_t L = L0 + u < cnt ? L0 + u : cnt - 1;
                    const uint64_t P0 = bcast64(p0, L), T0 = bcast64(t0, L);
                    const uint32_t PL = bcast(plen, L), TL = bcast(tlen, L);
                    x[u] = int4{0, 0, 0, 0};
                    y[u] = 0;
                    if (PL > 0) x[u] = *reinterpret_cast<const int4 *>(prog + P0 + (k < PL ? k : PL - 4u));
                    if (TL > 0) y[u] = tape[T0 + (lane < TL ? lane : TL - 1u)];
                }
#pragma unroll
                for (int u = 0; u < kPackGroup; ++u) {
                    const uint32_t L = L0 + u;
                    if (L >= cnt) break;
                    const uint64_t MO = bcast64(mo, L), TO = bcast64(to, L), YO = bcast64(yo, L);
                    const uint32_t PL = bcast(plen, L), TL = bcast(tlen, L);
                    const uint32_t NN = bcast(n, L), EL = bcast(ell, L), SS = bcast(s, L);
                    if (k < PL && k < NN) *reinterpret_cast<int4 *>(b.M + MO + k) = x[u];   // slices are padded to 4 words
                    if (lane < EL) b.T[TO + lane] = lane < TL ? y[u] : 0;
                    if (lane < SS) b.Y[YO + lane] = 0;
                }
            }
            continue;
        }
        for (uint32_t L = 0; L < cnt; ++L) {
            const uint64_t P0 = bcast64(p0, L), MO = bcast64(mo, L);
            const uint32_t PL = bcast(plen, L), NN = bcast(n, L);
            const int32_t *src = prog + P0;
            int32_t *M = b.M + MO;
            const bool aligned = (P0 & 3u) == 0;
            const uint32_t HW = min(up4(PL), up4(NN));
            for (uint32_t k = 4 * lane; k < HW; k += 4 * kWave) {
                int4 w;
                if (aligned && k + 4 <= PL) {
                    w = *reinterpret_cast<const int4 *>(src + k);
                } else {
                    w.x = k < PL ? src[k] : 0;
                    w.y = k + 1 < PL ? src[k + 1] : 0;
                    w.z = k + 2 < PL ? src[k + 2] : 0;
                    w.w = k + 3 < PL ? src[k + 3] : 0;
                }
                *reinterpret_cast<int4 *>(M + k) = w;      // slices are padded to 4 words
            }
            const uint64_t T0 = bcast64(t0, L), TO = bcast64(to, L), YO = bcast64(yo, L);
            const uint32_t TL = bcast(tlen, L), EL = bcast(ell, L), SS = bcast(s, L);
            for (uint32_t k = lane; k < EL; k += kWave) b.T[TO + k] = k < TL ? tape[T0 + k] : 0;
            for (uint32_t k = lane; k < SS; k += kWave) b.Y[YO + k] = 0;
        }
    }
}

hipError_t launch_pack(DevBatch b, const int32_t *prog, const uint64_t *prog_off,
                       const int32_t *tape, const uint64_t *tape_off, hipStream_t st)
{
    uint64_t blocks = (b.N + 255) / 256;                   // 4 waves x 64 machines
    if (blocks > 65536) blocks = 65536;
    k_pack<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st>>>(b, prog, prog_off, tape, tape_off);
    return hipGetLastError();
}

// status of every machine = is its current configuration a fixed point
template <int ISA>
__global__ __launch_bounds__(256) void k_probe(DevBatch b)
{
    const uint64_t v = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= b.N) return;
    Regs r;
    r.n = b.n[v]; r.ell = b.ell[v]; r.s = b.s[v];
    r.i = b.i[v]; r.a = b.a[v]; r.u0 = b.u0[v]; r.y0 = b.y0[v];
    r.p = cmod(r.i, r.n);
    const TailMem g{gptr(b.M + b.mem_off[v]), b.hw[v]};
    TapeG tg{gptr(b.T + b.t_off[v])};
    bool halted;
    run_machine<ISA, false, true>(g, tg, r, OutG{gptr(b.Y + b.y_off[v])}, 0u, halted, b.wshift);
    b.status[v] = halted ? 1 : 0;
}

hipError_t launch_probe(DevBatch b, hipStream_t st)
{
    const unsigned blocks = static_cast<unsigned>((b.N + 255) / 256);
    if (b.isa == 1) k_probe<1><<<blocks, 256, 0, st>>>(b);
    else k_probe<0><<<blocks, 256, 0, st>>>(b);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K2: plain step loop, one machine per lane, memory in HBM, no compaction.
// Every lane runs its machine for at most `cap` transitions.  With cap below
// the batch budget, machines still running are appended (wave-aggregated
// atomic) to the survivor list for the persistent kernel.
// PROF (a hot-cell first pass): the last hot.R transitions mark the cells
// they touch in the thread's LDS bitmap; a survivor then looks for a
// multiplier that gives each of its cells a slot of its own among hot.S
// (the first of kHotCandidates that does), and is listed as a fit (count
// q->survivors) with that multiplier and its cells, or on the misfit list
// (count q->misfits).
// ---------------------------------------------------------------------------

// wave-aggregated append of the lanes with `mine` set to a list: one atomic
// per wave; returns the lane's rank-th entry index
__device__ __forceinline__ uint64_t wave_append(bool mine, unsigned long long *counter, uint32_t lane)
{
    const uint64_t mask = __ballot(mine);
    unsigned long long base = 0;
    if (mask) {
        const int leader = __ffsll(static_cast<unsigned long long>(mask)) - 1;
        if (lane == static_cast<uint32_t>(leader))
            base = atomicAdd(counter, static_cast<unsigned long long>(__popcll(mask)));
        base = __shfl(base, leader);
    }
    return base + __popcll(mask & ((1ull << lane) - 1ull));
}

// whether the survivor's profiled cells (bitmap words bm + k * stride,
// k < bw) fit a table: at most hot.S cells and a multiplier c_out that
// places each in a slot of its own
__device__ __forceinline__ bool hot_place(uint32_t bm, uint32_t stride, const HotArgs &hot, uint32_t &c_out)
{
    const uint32_t mask = hot.S - 1u;
    uint32_t h = 0;
    for (uint32_t k = 0; k < hot.bw; ++k) h += __popc(static_cast<uint32_t>(rasp_lds[bm + k * stride]));
    c_out = 65536u;
    if (h > hot.S) return false;
    for (uint32_t cand = 0; cand < kHotCandidates; ++cand) {
        const uint32_t c = hot_mult(cand);
        uint64_t occ = 0;
        bool ok = true;
        for (uint32_t k = 0; k < hot.bw && ok; ++k) {
            uint32_t w = static_cast<uint32_t>(rasp_lds[bm + k * stride]);
            while (w != 0u && ok) {
                const uint32_t x = 32u * k + static_cast<uint32_t>(__builtin_ctz(w));
                w &= w - 1u;
                const uint64_t bit = 1ull << hot_slot(x, c, mask);
                ok = (occ & bit) == 0;
                occ |= bit;
            }
        }
        if (ok) {
            c_out = c;
            return true;
        }
    }
    return false;
}

// write fit p's table: the multiplier and, per slot, its cell or 0xffff
__device__ __forceinline__ void hot_write(uint32_t bm, uint32_t stride, const HotArgs &hot, uint64_t p,
                                          uint32_t c)
{
    const uint32_t mask = hot.S - 1u;
    uint16_t *tg = hot.tags + p * hot.S;
    uint64_t occ = 0;
    for (uint32_t k = 0; k < hot.bw; ++k) {
        uint32_t w = static_cast<uint32_t>(rasp_lds[bm + k * stride]);
        while (w != 0u) {
            const uint32_t x = 32u * k + static_cast<uint32_t>(__builtin_ctz(w));
            w &= w - 1u;
            const uint32_t sl = hot_slot(x, c, mask);
            if (((occ >> sl) & 1ull) == 0) {
                occ |= 1ull << sl;
                tg[sl] = static_cast<uint16_t>(x);
            }
        }
    }
    for (uint32_t sl = 0; sl < hot.S; ++sl)
        if (((occ >> sl) & 1ull) == 0) tg[sl] = 0xffffu;
    hot.mult[p] = c;
}

template <int ISA, bool POW2, bool PACK, bool PROF>
__global__ __launch_bounds__(256) void k_plain(const BatchTable *__restrict__ tab, uint64_t total,
                                               uint32_t cap, uint32_t wm, uint32_t *__restrict__ surv,
                                               QueueState *__restrict__ q, HotArgs hot)
{
    const uint64_t g = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    bool survive = false;
    int k = 0;
    uint64_t v = 0;
    // the zero tail of a machine handed to a later launch of this run is
    // stored after the step loop (those launches read and write whole
    // memories), the wave's lanes together
    bool tail_f = false, tail_v = false;
    uint32_t tail_hw = 0;
    if (g < total) {
        k = batch_of(tab, g);
        v = g - tab->start[k];
    }
    const DevBatch &b = tab->b[k];
    const bool fresh = PACK && g < total && b.fresh;
    if (PACK) {
        // build c0 (Sec. 2.1) of this wave's fresh machines first: each
        // machine's memory slice written by the whole wave, 16 bytes a lane
        uint64_t p0 = 0, t0 = 0;
        uint32_t plen = 0, tlen = 0, n = 0, ell = 0, s = 0;
        const int32_t *src = nullptr, *tsrc = nullptr;
        int32_t *Md = nullptr, *Td = nullptr, *Yd = nullptr;
        if (fresh) {
            p0 = b.prog_off[v];
            plen = static_cast<uint32_t>(b.prog_off[v + 1] - p0);
            t0 = b.tape_off[v];
            tlen = static_cast<uint32_t>(b.tape_off[v + 1] - t0);
            n = b.n[v]; ell = b.ell[v]; s = b.s[v];
            src = b.prog + p0; tsrc = b.tape + t0;
            Md = b.M + b.mem_off[v]; Td = b.T + b.t_off[v]; Yd = b.Y + b.y_off[v];
        }
        uint64_t fm = __ballot(fresh);
        while (fm) {
            const uint32_t L = static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(fm)) - 1);
            fm &= fm - 1;
            const int32_t *S = reinterpret_cast<const int32_t *>(bcast64(reinterpret_cast<uint64_t>(src), L));
            int32_t *D = reinterpret_cast<int32_t *>(bcast64(reinterpret_cast<uint64_t>(Md), L));
            const uint32_t PL = bcast(plen, L), NN = bcast(n, L);
            const bool al = (bcast64(p0, L) & 3u) == 0;
            // the program words; the zero tail stays unstored (hw)
            const uint32_t HW = min(up4(PL), up4(NN));
            for (uint32_t kk = 4 * lane; kk < HW; kk += 4 * kWave) {
                int4 w;
                if (al && kk + 4 <= PL) {
                    w = *reinterpret_cast<const int4 *>(S + kk);
                } else {
                    w.x = kk < PL ? S[kk] : 0;
                    w.y = kk + 1 < PL ? S[kk + 1] : 0;
                    w.z = kk + 2 < PL ? S[kk + 2] : 0;
                    w.w = kk + 3 < PL ? S[kk + 3] : 0;
                }
                *reinterpret_cast<int4 *>(D + kk) = w;
            }
            const int32_t *TS = reinterpret_cast<const int32_t *>(bcast64(reinterpret_cast<uint64_t>(tsrc), L));
            int32_t *TD = reinterpret_cast<int32_t *>(bcast64(reinterpret_cast<uint64_t>(Td), L));
            int32_t *YD = reinterpret_cast<int32_t *>(bcast64(reinterpret_cast<uint64_t>(Yd), L));
            const uint32_t TL = bcast(tlen, L), EL = bcast(ell, L), SS = bcast(s, L);
            for (uint32_t e = lane; e < EL; e += kWave) TD[e] = e < TL ? TS[e] : 0;
            for (uint32_t e = lane; e < SS; e += kWave) YD[e] = 0;
        }
        if (fresh) b.hw[v] = min(up4(plen), up4(n));
        // the wave's own stores must be visible to its lanes' loads below
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
    if (g < total) {
        const uint32_t budget = tab->budget[k];
        if ((fresh || b.status[v] == 0) && budget > 0) {
            Regs r;
            r.n = b.n[v]; r.ell = b.ell[v]; r.s = b.s[v];
            if (fresh) {
                r.i = 0; r.a = 0; r.u0 = 0; r.y0 = 0;
            } else {
                r.i = b.i[v]; r.a = b.a[v]; r.u0 = b.u0[v]; r.y0 = b.y0[v];
            }
            r.p = cmod(r.i, r.n);
            const uint32_t limit = cap < budget ? cap : budget;
            // the memory with its zero tail possibly unstored (hw)
            const uint32_t hw0 = fresh ? min(up4(static_cast<uint32_t>(b.prog_off[v + 1] - b.prog_off[v])), up4(r.n))
                                       : b.hw[v];
            TailMem m{gptr(b.M + b.mem_off[v]), hw0};
            TapeG tg{gptr(b.T + b.t_off[v])};
            bool halted;
            const OutG og{gptr(b.Y + b.y_off[v])};
            uint32_t t;
            uint32_t hw;
            if constexpr (PROF) {
                // the last min(R, limit) transitions are profiled
                for (uint32_t kk = 0; kk < hot.bw; ++kk) rasp_lds[threadIdx.x + kk * blockDim.x] = 0;
                const uint32_t R = hot.R < limit ? hot.R : limit;
                t = wm ? run_machine<ISA, POW2, true>(m, tg, r, og, limit - R, halted, b.wshift)
                       : run_machine<ISA, POW2, false>(m, tg, r, og, limit - R, halted, 0u);
                hw = m.hw;
                // the profiled transitions read whole memories: the machines
                // that reach them store their tails first
                const bool prof = !halted && t == limit - R;
                const uint32_t top = up4(r.n);
                store_tails(prof && hw < top, gptr(b.M + b.mem_off[v]), hw, top);
                if (prof) {
                    const ProfMem pm{gptr(b.M + b.mem_off[v]), threadIdx.x, blockDim.x};
                    t += wm ? run_machine<ISA, POW2, true>(pm, tg, r, og, R, halted, b.wshift)
                            : run_machine<ISA, POW2, false>(pm, tg, r, og, R, halted, 0u);
                }
            } else {
                t = wm ? run_machine<ISA, POW2, true>(m, tg, r, og, limit, halted, b.wshift)
                       : run_machine<ISA, POW2, false>(m, tg, r, og, limit, halted, 0u);
                hw = m.hw;
            }
            tail_f = !halted && t == limit && limit < budget && hw < up4(b.n[v]);
            tail_hw = hw;
            tail_v = true;
            if (t || fresh) {
                b.i[v] = r.i; b.a[v] = r.a; b.u0[v] = r.u0; b.y0[v] = r.y0;
                b.steps[v] = fresh ? t : b.steps[v] + t;
            }
            if (halted || fresh) b.status[v] = halted ? 1 : 0;
            survive = !halted && t == limit && limit < budget;
        } else if (fresh) {
            // budget 0: c0 only
            b.i[v] = 0; b.a[v] = 0; b.u0[v] = 0; b.y0[v] = 0; b.steps[v] = 0; b.status[v] = 0;
        }
    }
    {
        gi32 *const tM = gptr(tail_f ? b.M + b.mem_off[v] : b.M);
        store_tails(tail_f, tM, tail_hw, tail_f ? up4(b.n[v]) : 0u);
    }
    if (tail_v) b.hw[v] = tail_hw;
    if (PROF && surv != nullptr) {
        uint32_t c = 65536u;
        const bool fit = survive && hot_place(threadIdx.x, blockDim.x, hot, c);
        const uint64_t pf = wave_append(fit, &q->survivors, lane);
        const uint64_t pm = wave_append(survive && !fit, &q->misfits, lane);
        if (fit) {
            surv[pf] = static_cast<uint32_t>(g);
            hot_write(threadIdx.x, blockDim.x, hot, pf, c);
        } else if (survive) {
            hot.mis[pm] = static_cast<uint32_t>(g);
        }
    } else if (surv != nullptr) {
        const uint64_t mask = __ballot(survive);
        if (mask) {
            const int leader = __ffsll(static_cast<unsigned long long>(mask)) - 1;
            unsigned long long base = 0;
            if (lane == static_cast<uint32_t>(leader))
                base = atomicAdd(&q->survivors, static_cast<unsigned long long>(__popcll(mask)));
            base = __shfl(base, leader);
            if (survive) {
                const uint32_t rank = __popcll(mask & ((1ull << lane) - 1ull));
                surv[base + rank] = static_cast<uint32_t>(g);
            }
        }
    }
}

template <int ISA, bool POW2>
static void plain_go(bool pack, unsigned blocks, hipStream_t st, const BatchTable *tab, uint64_t total,
                     uint32_t cap, uint32_t wm, uint32_t *surv, QueueState *q, const HotArgs *hot)
{
    if (hot) {
        const size_t shmem = static_cast<size_t>(hot->bw) * 256u * sizeof(int32_t);
        if (pack) k_plain<ISA, POW2, true, true><<<blocks, 256, shmem, st>>>(tab, total, cap, wm, surv, q, *hot);
        else k_plain<ISA, POW2, false, true><<<blocks, 256, shmem, st>>>(tab, total, cap, wm, surv, q, *hot);
        return;
    }
    const HotArgs none{};
    if (pack) k_plain<ISA, POW2, true, false><<<blocks, 256, 0, st>>>(tab, total, cap, wm, surv, q, none);
    else k_plain<ISA, POW2, false, false><<<blocks, 256, 0, st>>>(tab, total, cap, wm, surv, q, none);
}

hipError_t launch_plain(const BatchTable *tab, uint64_t total, uint32_t cap, uint32_t isa,
                        bool pow2, bool pack, bool wm, uint32_t *surv, QueueState *q, hipStream_t st,
                        const HotArgs *hot)
{
    const unsigned blocks = static_cast<unsigned>((total + 255) / 256);
    const uint32_t w = wm ? 1u : 0u;
    if (isa == 1) {
        if (pow2) plain_go<1, true>(pack, blocks, st, tab, total, cap, w, surv, q, hot);
        else plain_go<1, false>(pack, blocks, st, tab, total, cap, w, surv, q, hot);
    } else {
        if (pow2) plain_go<0, true>(pack, blocks, st, tab, total, cap, w, surv, q, hot);
        else plain_go<0, false>(pack, blocks, st, tab, total, cap, w, surv, q, hot);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K3: persistent step loop.  Resident waves pull work items from a device
// queue (one agent-scope atomic per wave refill), run each lane's machine for
// at most `epoch` transitions between refill points, write back machines
// that halted or spent their budget, and refill exactly those lanes (wave
// ballot + popcount prefix ranks).
// MODE 0: memory in HBM.  MODE 1: each live machine's whole memory is staged
// in its lane's LDS slot of P words (every n <= P).  MODE 2: words [0, P) in
// LDS, the rest in HBM.  Slots are interleaved across the wave's lanes (word
// k of lane l at wave_base + 64 k + l).  Each lane stages and writes back its own machine: one direct load
// (or 16-byte store) moves a word (four words) of every lane that has one to
// move; only machines that stored into LDS (or are new) are written back.
// Work item k is machine work[k] of the launch (or machine k when work is
// null); machines have already applied `already` transitions this run.
// With surv non-null the launch is a first pass: a machine runs at most `cap`
// transitions, and one still running after them is written back and appended
// to surv (its index in the launch) for a later launch.
// Slot words past the memory: word P takes the stores that do not happen;
// from P + 4 on (TLDS, MODE 1 only) the tape, TL words.
// ---------------------------------------------------------------------------

// four words as one 16-byte access; global and LDS views of it
typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) v4i gv4i;
// direct global-to-LDS load: lane l's 4 bytes from g land at LDS word row +
// l; row is the same for every lane of the wave
typedef __attribute__((address_space(1))) void gv;
typedef __attribute__((address_space(3))) void lv;
__device__ __forceinline__ void dma4(const int32_t *g, uint32_t row)
{
    __builtin_amdgcn_global_load_lds((const gv *)g, (lv *)&rasp_lds[row], 4, 0, 0);
}

// the largest (smallest) x over the lanes of the wave, in a scalar register;
// every lane of the wave takes part
__device__ __forceinline__ uint32_t wave_max(uint32_t x)
{
    for (int o = kWave / 2; o > 0; o >>= 1) x = max(x, static_cast<uint32_t>(__shfl_xor(static_cast<int>(x), o)));
    return static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(x)));
}
__device__ __forceinline__ uint32_t wave_min(uint32_t x)
{
    for (int o = kWave / 2; o > 0; o >>= 1) x = min(x, static_cast<uint32_t>(__shfl_xor(static_cast<int>(x), o)));
    return static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(x)));
}

// ONE: the launch holds a single batch, so every lane's batch is tab->b[0]
// and its fields are wave-uniform (scalar loads, kept across refills); a
// refill then waits on one round of per-machine loads
template <int ISA, int MODE, bool POW2, bool TLDS, bool ONE>
__device__ __forceinline__ void persistent_body(const BatchTable *__restrict__ tab, uint64_t total,
                                                const uint32_t *__restrict__ work, uint32_t already,
                                                uint32_t epoch, uint32_t P, uint32_t TL, uint32_t wm,
                                                uint32_t cap, uint32_t *__restrict__ surv,
                                                QueueState *__restrict__ q, uint32_t which)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wib = threadIdx.x / kWave;
    const uint32_t TB = P + 4u;                            // tape offset in a slot
    const uint32_t SP = P + 4u + (TLDS ? TL : 0u);         // slot: memory, spares, tape
    const uint32_t wave_base = wib * kWave * SP;           // LDS word index of the wave's slots
    const uint32_t slot = wave_base + lane;                 // this lane's slot word 0 (word k at + 64 k)
    // the survivor (or misfit) count written by the first pass, and the
    // list's claim counter
    if (work != nullptr) total = which ? q->misfits : q->survivors;
    unsigned long long *const head = which ? &q->head_m : &q->head;

    bool has = false, exhausted = false, fresh = false, cut = false;
    Regs r{};
    int32_t *M = nullptr;
    int32_t *T = nullptr;
    int32_t *Y = nullptr;
    uint32_t done = 0, limit = 0, ws = 0, gid = 0;
    const DevBatch *bp = nullptr;
    uint64_t v = 0;
    // memory in HBM: the lanes step in lockstep, a run stopping when any of
    // them reaches a fixed point or its budget; idle lanes are refilled once
    // an epoch (transitions since the last refill, wave-uniform) or when no
    // lane runs.  Slots: each lane runs up to an epoch on its own, and the
    // wave refills after every run.
    uint32_t spent = 0;

    for (;;) {
        // ---- refill idle lanes from the queue ----
        const uint64_t idle = __ballot(!has);
        bool claimed = false;
        bool due = true;
        if (MODE == 0) {
            due = spent >= epoch || idle == ~0ull;
            if (due) spent = 0;
        }
        if (due && idle != 0 && !exhausted) {
            const int leader = __ffsll(static_cast<unsigned long long>(idle)) - 1;
            const uint32_t cnt = __popcll(idle);
            unsigned long long base = 0;
            if (lane == static_cast<uint32_t>(leader))
                base = __hip_atomic_fetch_add(head, static_cast<unsigned long long>(cnt),
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            base = __shfl(base, leader);
            if (base + cnt >= total) exhausted = true;
            if (!has) {
                const uint64_t item = base + __popcll(idle & ((1ull << lane) - 1ull));
                if (item < total) {
                    const uint64_t g = work ? static_cast<uint64_t>(work[item]) : item;
                    const int k = ONE ? 0 : batch_of(tab, g);
                    bp = &tab->b[k];
                    v = ONE ? g : g - tab->start[k];
                    const uint32_t budget = tab->budget[k];
                    fresh = bp->fresh != 0;
                    if ((fresh || bp->status[v] == 0) && budget > already) {
                        r.n = bp->n[v]; r.ell = bp->ell[v]; r.s = bp->s[v];
                        if (fresh) {
                            r.i = 0; r.a = 0; r.u0 = 0; r.y0 = 0;
                        } else {
                            r.i = bp->i[v]; r.a = bp->a[v]; r.u0 = bp->u0[v]; r.y0 = bp->y0[v];
                        }
                        r.p = cmod(r.i, r.n);
                        ws = bp->wshift;
                        M = bp->M + bp->mem_off[v];
                        T = bp->T + bp->t_off[v];
                        Y = bp->Y + bp->y_off[v];
                        gid = static_cast<uint32_t>(g);
                        done = 0;
                        limit = budget - already;
                        cut = cap < limit;
                        if (cut) limit = cap;
                        has = true;
                        claimed = true;
                    }
                }
            }
        }
        if (__ballot(has) == 0) {
            if (exhausted) break;
            continue;
        }
        // ---- stage the claimed machines' low memory words into their slots ----
        // Each claiming lane moves its own machine with direct global-to-LDS
        // loads: one instruction moves word k of every claiming lane's source
        // to LDS word wave_base + 64 k + lane, its slot word k.  The zeros of
        // c0 are stored first (issued after a direct load they would wait for
        // it), every load is issued before a single wait, so a refill pays
        // about one memory latency.
        if (MODE != 0) {
            // what each claiming lane's copy reads: the packed program (c0 of a
            // new machine, Sec. 2.1: program words, then zeros) or its memory
            const int32_t *src = nullptr, *tsrc = nullptr;
            uint32_t n4 = 0, cnt = 0, tlen = 0, tn = 0, el = 0;
            if (claimed) {
                cnt = r.n < P ? r.n : P;
                if (fresh) {
                    const uint64_t p0 = bp->prog_off[v], t0 = bp->tape_off[v];
                    src = bp->prog + p0;
                    const uint32_t srclen = static_cast<uint32_t>(bp->prog_off[v + 1] - p0);
                    n4 = srclen < cnt ? srclen : cnt;           // words copied from the source
                    tsrc = bp->tape + t0;
                    tlen = static_cast<uint32_t>(bp->tape_off[v + 1] - t0);
                } else {
                    src = M;
                    n4 = cnt;
                    tsrc = T;
                    tlen = r.ell;
                }
                if (TLDS) { el = r.ell; tn = tlen < el ? tlen : el; }
            }
            const uint64_t claimed_mask = __ballot(claimed);
            if (claimed_mask) {
                const uint32_t zlo = wave_min(claimed ? n4 : 0xffffffffu), zhi = wave_max(cnt);
                for (uint32_t k = zlo; k < zhi; ++k)
                    if (k >= n4 && k < cnt) rasp_lds[slot + (k << kSlotShift)] = 0;
                if (TLDS) {
                    const uint32_t tlo = wave_min(claimed ? tn : 0xffffffffu), thi = wave_max(el);
                    for (uint32_t e = tlo; e < thi; ++e)
                        if (e >= tn && e < el) rasp_lds[slot + ((TB + e) << kSlotShift)] = 0;
                }
                const uint32_t kmax = wave_max(n4);
                for (uint32_t k = 0; k < kmax; ++k)
                    if (k < n4) dma4(src + k, wave_base + (k << kSlotShift));
                if (TLDS) {
                    const uint32_t tmax = wave_max(tn);
                    for (uint32_t e = 0; e < tmax; ++e)
                        if (e < tn) dma4(tsrc + e, wave_base + ((TB + e) << kSlotShift));
                }
                __builtin_amdgcn_s_waitcnt(0);                  // the direct loads have landed
            }
            // a new machine's tape and output in HBM: x 0^(l-|x|) and 0^s
            uint64_t fm = __ballot(claimed && fresh);
            while (fm) {
                const uint32_t L = static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(fm)) - 1);
                fm &= fm - 1ull;
                const uint32_t EL = bcast(r.ell, L), TN = bcast(tlen, L), SS = bcast(r.s, L);
                gi32 *TD = gptr(reinterpret_cast<int32_t *>(bcast64(reinterpret_cast<uint64_t>(T), L)));
                gi32 *YD = gptr(reinterpret_cast<int32_t *>(bcast64(reinterpret_cast<uint64_t>(Y), L)));
                const gi32 *TS = gptr(reinterpret_cast<const int32_t *>(bcast64(reinterpret_cast<uint64_t>(tsrc), L)));
                for (uint32_t e = lane; e < EL; e += kWave) TD[e] = e < TN ? TS[e] : 0;
                for (uint32_t e = lane; e < SS; e += kWave) YD[e] = 0;
            }
        }
        // ---- run ----
        bool finish = false, survive = false;
        const uint32_t L = MODE == 0 ? wave_min(has ? min(limit - done, epoch - spent) : ~0u) : 0u;
        uint32_t t = 0;
        if (has) {
            uint32_t lim = limit - done;
            if (lim > epoch) lim = epoch;
            bool halted;
            // wm is uniform: one of the two loop bodies runs
#define RASP_RUN(mm, tp, ou)                                                                    \
    (wm ? run_machine<ISA, POW2, true>(mm, tp, r, ou, lim, halted, ws)                         \
        : run_machine<ISA, POW2, false>(mm, tp, r, ou, lim, halted, 0u))
            if (MODE == 1) {
                LdsMem mm{slot, slot + (P << kSlotShift)};
                if (TLDS) {
                    TapeL tl{slot + (TB << kSlotShift)};
                    OutG og{gptr(Y)};
                    t = RASP_RUN(mm, tl, og);
                } else {
                    TapeG tg{gptr(T)};
                    OutG og{gptr(Y)};
                    t = RASP_RUN(mm, tg, og);
                }
            } else if (MODE == 2) {
                SplitMem mm{slot, P, gptr(M)};
                TapeG tg{gptr(T)};
                OutG og{gptr(Y)};
                t = RASP_RUN(mm, tg, og);
            } else {
                GlobalMem mm{gptr(M)};
                TapeG tg{gptr(T)};
                OutG og{gptr(Y)};
                t = wm ? run_lockstep<ISA, POW2, true>(mm, tg, og, r, L, halted, ws)
                       : run_lockstep<ISA, POW2, false>(mm, tg, og, r, L, halted, 0u);
            }
#undef RASP_RUN
            done += t;
            if (halted || done == limit) {
                if (done || fresh) {
                    bp->i[v] = r.i; bp->a[v] = r.a; bp->u0[v] = r.u0; bp->y0[v] = r.y0;
                    bp->steps[v] = fresh ? done : bp->steps[v] + done;
                }
                if (halted || fresh) bp->status[v] = halted ? 1 : 0;
                finish = true;
                survive = cut && !halted;
            }
        }
        if (MODE == 0) spent += wave_max(t);
        // ---- write back the slots of finished machines ----
        // a machine that ran a step (or is new) may have stored: each such
        // lane writes its own slot back, four words (16 bytes) at a time
        // (memory slices are 16-byte aligned)
        if (MODE != 0) {
            const bool back = finish && (done > 0 || fresh);
            const uint32_t cnt = back ? (r.n < P ? r.n : P) : 0u;
            // a new machine (every memory fits, MODE 1) leaves its whole memory stored
            if (back && fresh) bp->hw[v] = up4(r.n);
            const uint32_t kmax = wave_max(cnt);
            if (kmax) {
                gi32 *const MD = gptr(M);
#pragma unroll 2
                for (uint32_t k0 = 0; k0 < kmax; k0 += 4u) {
                    if (k0 < cnt) {
                        const int32_t *const ps = &rasp_lds[slot + (k0 << kSlotShift)];
                        const v4i w{ps[0], ps[1u << kSlotShift], ps[2u << kSlotShift], ps[3u << kSlotShift]};
                        if (k0 + 4u <= cnt) {
                            *reinterpret_cast<gv4i *>(MD + k0) = w;
                        } else {
                            MD[k0] = w[0];
                            if (k0 + 1u < cnt) MD[k0 + 1u] = w[1];
                            if (k0 + 2u < cnt) MD[k0 + 2u] = w[2];
                        }
                    }
                }
            }
        }
        // ---- first pass: append the machines still running to the survivor list ----
        if (surv != nullptr) {
            const uint64_t sm = __ballot(survive);
            if (sm) {
                const int leader = __ffsll(static_cast<unsigned long long>(sm)) - 1;
                unsigned long long base = 0;
                if (lane == static_cast<uint32_t>(leader))
                    base = atomicAdd(&q->survivors, static_cast<unsigned long long>(__popcll(sm)));
                base = __shfl(base, leader);
                if (survive) surv[base + __popcll(sm & ((1ull << lane) - 1ull))] = gid;
            }
        }
        if (finish) has = false;
    }
}

template <int ISA, int MODE, bool POW2, bool TLDS>
__global__ __launch_bounds__(256) void k_persistent(const BatchTable *__restrict__ tab,
                                                    uint64_t total,
                                                    const uint32_t *__restrict__ work,
                                                    uint32_t already, uint32_t epoch,
                                                    uint32_t P, uint32_t TL, uint32_t wm,
                                                    uint32_t cap, uint32_t *__restrict__ surv,
                                                    QueueState *__restrict__ q, uint32_t which)
{
    if (tab->count == 1)
        persistent_body<ISA, MODE, POW2, TLDS, true>(tab, total, work, already, epoch, P, TL, wm, cap, surv, q, which);
    else
        persistent_body<ISA, MODE, POW2, TLDS, false>(tab, total, work, already, epoch, P, TL, wm, cap, surv, q, which);
}

// ---------------------------------------------------------------------------
// K3 over the fits of a hot-cell first pass.  A claimed machine's table is
// filled from its cell list and its memory; a finished machine's tagged
// cells are written back.  Both are done by the whole wave, 64 / S machines
// per instruction (lane k serves slot k mod S of the (k / S)-th machine of
// the pass).
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t shfl64(uint64_t x, uint32_t src)
{
    const uint32_t lo = static_cast<uint32_t>(__shfl(static_cast<int>(static_cast<uint32_t>(x)), static_cast<int>(src)));
    const uint32_t hi = static_cast<uint32_t>(__shfl(static_cast<int>(static_cast<uint32_t>(x >> 32)), static_cast<int>(src)));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// the lane of the (lane / S)-th member of this pass among the set bits of
// *mask (consumed), or 64 when the pass has fewer members
__device__ __forceinline__ uint32_t hot_member(uint64_t &mask, uint32_t lane, uint32_t S)
{
    uint32_t mine = kWave;
    for (uint32_t i = 0; i < kWave / S && mask != 0; ++i) {
        const uint32_t L = static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(mask)) - 1);
        mask &= mask - 1ull;
        if (lane / S == i) mine = L;
    }
    return mine;
}

template <int ISA, bool POW2, bool ONE>
__device__ __forceinline__ void persistent_hot_body(const BatchTable *__restrict__ tab,
                                                    const uint32_t *__restrict__ work, uint32_t already,
                                                    uint32_t epoch, uint32_t wm, const HotArgs hot,
                                                    QueueState *__restrict__ q)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wib = threadIdx.x / kWave;
    const uint32_t S = hot.S, mask = hot.S - 1u;
    const uint32_t wave_base = wib * kWave * hot_slot_words(S);   // slot words, then tags
    const uint32_t tag_base = 2u * (wave_base + 2u * kWave * S);  // in halfwords
    uint16_t *const ltags = reinterpret_cast<uint16_t *>(rasp_lds);
    const uint64_t total = q->survivors;

    bool has = false, exhausted = false;
    Regs r{};
    int32_t *M = nullptr;
    int32_t *T = nullptr;
    int32_t *Y = nullptr;
    uint32_t done = 0, limit = 0, ws = 0, c = 65536u;
    uint64_t pos = 0, v = 0;
    const DevBatch *bp = nullptr;
    uint32_t spent = 0;                  // transitions since the last refill (wave-uniform)

    for (;;) {
        // ---- refill idle lanes from the queue, once an epoch (a lane that
        // finishes earlier waits for the epoch's end) or when no lane runs ----
        const uint64_t idle = __ballot(!has);
        bool claimed = false;
        const bool due = spent >= epoch || idle == ~0ull;
        if (due) spent = 0;
        if (due && idle != 0 && !exhausted) {
            const int leader = __ffsll(static_cast<unsigned long long>(idle)) - 1;
            const uint32_t cnt = __popcll(idle);
            unsigned long long base = 0;
            if (lane == static_cast<uint32_t>(leader))
                base = __hip_atomic_fetch_add(&q->head, static_cast<unsigned long long>(cnt),
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            base = __shfl(base, leader);
            if (base + cnt >= total) exhausted = true;
            if (!has) {
                const uint64_t item = base + __popcll(idle & ((1ull << lane) - 1ull));
                if (item < total) {
                    pos = item;
                    const uint64_t g = work[pos];
                    const int k = ONE ? 0 : batch_of(tab, g);
                    bp = &tab->b[k];
                    v = ONE ? g : g - tab->start[k];
                    const uint32_t budget = tab->budget[k];
                    if (bp->status[v] == 0 && budget > already) {
                        r.n = bp->n[v]; r.ell = bp->ell[v]; r.s = bp->s[v];
                        r.i = bp->i[v]; r.a = bp->a[v]; r.u0 = bp->u0[v]; r.y0 = bp->y0[v];
                        r.p = cmod(r.i, r.n);
                        ws = bp->wshift;
                        M = bp->M + bp->mem_off[v];
                        T = bp->T + bp->t_off[v];
                        Y = bp->Y + bp->y_off[v];
                        c = hot.mult[pos];
                        done = 0;
                        limit = budget - already;
                        has = true;
                        claimed = true;
                    }
                }
            }
        }
        if (__ballot(has) == 0) {
            if (exhausted) break;
            continue;
        }
        // ---- fill the claimed machines' tables ----
        uint64_t cm = __ballot(claimed);
        while (cm != 0) {
            const uint32_t L = hot_member(cm, lane, S);
            const uint32_t src = L & (kWave - 1u);
            const uint64_t pL = shfl64(pos, src);
            const int32_t *ML = reinterpret_cast<const int32_t *>(shfl64(reinterpret_cast<uint64_t>(M), src));
            const uint32_t sl = lane & mask;
            if (L < kWave) {
                const uint32_t x = hot.tags[pL * S + sl];
                int2 wv = int2{0, 0};
                if (x != 0xffffu) wv = *reinterpret_cast<const int2 *>(ML + 2u * x);
                *reinterpret_cast<int2 *>(&rasp_lds[wave_base + 2u * (kWave * sl + L)]) = wv;
                ltags[tag_base + kWave * sl + L] = static_cast<uint16_t>(x);
            }
        }
        // the wave's table writes before its lanes' reads
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        // ---- run: the lanes step together until one of them reaches a
        // fixed point or its budget, or the epoch ends ----
        const uint32_t L = wave_min(has ? min(limit - done, epoch - spent) : ~0u);
        bool finish = false;
        uint32_t t = 0;
        if (has) {
            bool halted;
            const HotMem mm{wave_base + 2u * lane, tag_base + lane, c, mask, gptr(M)};
            const TapeG tg{gptr(T)};
            const OutG og{gptr(Y)};
            t = wm ? run_lockstep<ISA, POW2, true>(mm, tg, og, r, L, halted, ws)
                   : run_lockstep<ISA, POW2, false>(mm, tg, og, r, L, halted, 0u);
            done += t;
            if (halted || done == limit) {
                if (done) {
                    bp->i[v] = r.i; bp->a[v] = r.a; bp->u0[v] = r.u0; bp->y0[v] = r.y0;
                    bp->steps[v] += done;
                }
                if (halted) bp->status[v] = 1;
                finish = true;
            }
        }
        spent += wave_max(t);
        // ---- write the finished machines' cells back ----
        uint64_t fm = __ballot(finish);
        while (fm != 0) {
            const uint32_t L = hot_member(fm, lane, S);
            const uint32_t src = L & (kWave - 1u);
            int32_t *ML = reinterpret_cast<int32_t *>(shfl64(reinterpret_cast<uint64_t>(M), src));
            const uint32_t sl = lane & mask;
            if (L < kWave) {
                const uint32_t x = ltags[tag_base + kWave * sl + L];
                if (x != 0xffffu)
                    *reinterpret_cast<int2 *>(ML + 2u * x) =
                        *reinterpret_cast<const int2 *>(&rasp_lds[wave_base + 2u * (kWave * sl + L)]);
            }
        }
        if (finish) has = false;
    }
}

template <int ISA, bool POW2>
__global__ __launch_bounds__(256) void k_persistent_hot(const BatchTable *__restrict__ tab,
                                                        const uint32_t *__restrict__ work, uint32_t already,
                                                        uint32_t epoch, uint32_t wm, HotArgs hot,
                                                        QueueState *__restrict__ q)
{
    if (tab->count == 1) persistent_hot_body<ISA, POW2, true>(tab, work, already, epoch, wm, hot, q);
    else persistent_hot_body<ISA, POW2, false>(tab, work, already, epoch, wm, hot, q);
}

hipError_t launch_persistent_hot(const BatchTable *tab, const uint32_t *work, uint32_t already, uint32_t isa,
                                 bool pow2, bool wmb, uint32_t epoch, const HotArgs &hot,
                                 uint32_t waves_per_block, uint32_t blocks, QueueState *q, hipStream_t st)
{
    const dim3 grid(blocks), block(waves_per_block * kWave);
    const size_t shmem = static_cast<size_t>(waves_per_block) * kWave * hot_slot_words(hot.S) * sizeof(int32_t);
    const uint32_t wm = wmb ? 1u : 0u;
    if (isa == 1) {
        if (pow2) k_persistent_hot<1, true><<<grid, block, shmem, st>>>(tab, work, already, epoch, wm, hot, q);
        else k_persistent_hot<1, false><<<grid, block, shmem, st>>>(tab, work, already, epoch, wm, hot, q);
    } else {
        if (pow2) k_persistent_hot<0, true><<<grid, block, shmem, st>>>(tab, work, already, epoch, wm, hot, q);
        else k_persistent_hot<0, false><<<grid, block, shmem, st>>>(tab, work, already, epoch, wm, hot, q);
    }
    return hipGetLastError();
}

template <int ISA, int MODE, bool POW2, bool TLDS>
static hipError_t launch_k3(dim3 grid, dim3 block, size_t shmem, hipStream_t st, const BatchTable *tab,
                            uint64_t total, const uint32_t *work, uint32_t already, uint32_t epoch,
                            uint32_t P, uint32_t TL, uint32_t wm, uint32_t cap, uint32_t *surv, QueueState *q,
                            uint32_t which)
{
    k_persistent<ISA, MODE, POW2, TLDS><<<grid, block, shmem, st>>>(tab, total, work, already, epoch, P, TL,
                                                                    wm, cap, surv, q, which);
    return hipGetLastError();
}

template <int ISA, int MODE, bool POW2, bool TLDS>
static void lds_attr()
{
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_persistent<ISA, MODE, POW2, TLDS>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

// Allow the persistent kernels the whole LDS of a compute unit; called once
// per context, outside any stream capture.
void init_kernel_attributes()
{
    lds_attr<0, 1, false, false>(); lds_attr<0, 1, true, false>();
    lds_attr<0, 1, false, true>(); lds_attr<0, 1, true, true>();
    lds_attr<0, 2, false, false>(); lds_attr<0, 2, true, false>();
    lds_attr<1, 1, false, false>(); lds_attr<1, 1, true, false>();
    lds_attr<1, 1, false, true>(); lds_attr<1, 1, true, true>();
    lds_attr<1, 2, false, false>(); lds_attr<1, 2, true, false>();
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_persistent_hot<0, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_persistent_hot<0, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_persistent_hot<1, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_persistent_hot<1, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();
}

template <int ISA, int MODE, bool TLDS>
static hipError_t launch_k3_p(bool pow2, dim3 grid, dim3 block, size_t shmem, hipStream_t st,
                              const BatchTable *tab, uint64_t total, const uint32_t *work,
                              uint32_t already, uint32_t epoch, uint32_t P, uint32_t TL,
                              uint32_t wm, uint32_t cap, uint32_t *surv, QueueState *q, uint32_t which)
{
    return pow2 ? launch_k3<ISA, MODE, true, TLDS>(grid, block, shmem, st, tab, total, work, already, epoch, P, TL, wm, cap, surv, q, which)
                : launch_k3<ISA, MODE, false, TLDS>(grid, block, shmem, st, tab, total, work, already, epoch, P, TL, wm, cap, surv, q, which);
}

// the tape is staged in LDS when every memory fits its slot and every tape
// is at most kTapeLdsMax words; the region holds l + 1 words (the step loop
// reads word u0 <= l unconditionally), rounded up to 16 bytes
uint32_t slot_words(uint32_t lds_words, uint32_t max_n, uint32_t max_ell)
{
    if (lds_words == 0) return 0;
    const bool tl = max_n <= lds_words && max_ell <= kTapeLdsMax;
    return lds_words + 4u + (tl ? (max_ell + 1u + 3u) & ~3u : 0u);
}

hipError_t launch_persistent(const BatchTable *tab, uint64_t total, const uint32_t *work,
                             uint32_t already, uint32_t isa, bool pow2, bool wmb, uint32_t epoch,
                             uint32_t lds_words, uint32_t max_n, uint32_t max_ell,
                             uint32_t waves_per_block, uint32_t blocks, uint32_t cap, uint32_t *surv,
                             QueueState *q, hipStream_t st, bool misfits)
{
    const uint32_t wm = wmb ? 1u : 0u;
    const uint32_t which = misfits ? 1u : 0u;
    const dim3 grid(blocks), block(waves_per_block * kWave);
    const int mode = lds_words == 0 ? 0 : (max_n <= lds_words ? 1 : 2);
    const uint32_t P = mode == 0 ? 0u : lds_words;
    const uint32_t SPw = slot_words(P, max_n, max_ell);
    const uint32_t TL = (mode == 1 && SPw > P + 4u) ? SPw - P - 4u : 0u;
    const size_t shmem = mode == 0 ? 0 : static_cast<size_t>(waves_per_block) * kWave * SPw * sizeof(int32_t);
    if (isa == 1) {
        if (mode == 1 && TL) return launch_k3_p<1, 1, true>(pow2, grid, block, shmem, st, tab, total, work, already, epoch, P, TL, wm, cap, surv, q, which);
        if (mode == 1) return launch_k3_p<1, 1, false>(pow2, grid, block, shmem, st, tab, total, work, already, epoch, P, 0u, wm, cap, surv, q, which);
        if (mode == 2) return launch_k3_p<1, 2, false>(pow2, grid, block, shmem, st, tab, total, work, already, epoch, P, 0u, wm, cap, surv, q, which);
        return launch_k3_p<1, 0, false>(pow2, grid, block, shmem, st, tab, total, work, already, epoch, P, 0u, wm, cap, surv, q, which);
    }
    if (mode == 1 && TL) return launch_k3_p<0, 1, true>(pow2, grid, block, shmem, st, tab, total, work, already, epoch, P, TL, wm, cap, surv, q, which);
    if (mode == 1) return launch_k3_p<0, 1, false>(pow2, grid, block, shmem, st, tab, total, work, already, epoch, P, 0u, wm, cap, surv, q, which);
    if (mode == 2) return launch_k3_p<0, 2, false>(pow2, grid, block, shmem, st, tab, total, work, already, epoch, P, 0u, wm, cap, surv, q, which);
    return launch_k3_p<0, 0, false>(pow2, grid, block, shmem, st, tab, total, work, already, epoch, P, 0u, wm, cap, surv, q, which);
}

__global__ void k_zero_queue(QueueState *q, uint32_t head_only)
{
    if (threadIdx.x == 0) {
        q->head = 0;
        q->head_m = 0;
        if (!head_only) { q->survivors = 0; q->retired = 0; q->pad = 0; q->misfits = 0; }
    }
}

hipError_t launch_zero_queue(QueueState *q, hipStream_t st)
{
    k_zero_queue<<<1, 64, 0, st>>>(q, 0u);
    return hipGetLastError();
}

hipError_t launch_reset_head(QueueState *q, hipStream_t st)
{
    k_zero_queue<<<1, 64, 0, st>>>(q, 1u);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K4: FNV-1a-64 digest of each machine's memory (little-endian bytes),
// one lane per machine, 16-byte loads (memory slices are 16-byte aligned).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_digest(DevBatch b, uint64_t *__restrict__ out)
{
    const uint64_t v = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= b.N) return;
    const uint32_t n = b.n[v], hw = b.hw[v];
    const int32_t *M = b.M + b.mem_off[v];
    uint64_t h = 0xcbf29ce484222325ull;
    const uint64_t prime = 0x100000001b3ull;
    uint32_t k = 0;
    for (; k + 4 <= n; k += 4) {
        const int4 w = k < hw ? *reinterpret_cast<const int4 *>(M + k) : int4{0, 0, 0, 0};
        const uint32_t ws[4] = {static_cast<uint32_t>(w.x), static_cast<uint32_t>(w.y),
                                static_cast<uint32_t>(w.z), static_cast<uint32_t>(w.w)};
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int byte = 0; byte < 4; ++byte) { h ^= (ws[e] >> (8 * byte)) & 0xffu; h *= prime; }
    }
    for (; k < n; ++k) {
        const uint32_t x = k < hw ? static_cast<uint32_t>(M[k]) : 0u;
#pragma unroll
        for (int byte = 0; byte < 4; ++byte) { h ^= (x >> (8 * byte)) & 0xffu; h *= prime; }
    }
    out[v] = h;
}

hipError_t launch_digest(DevBatch b, uint64_t *out, hipStream_t st)
{
    k_digest<<<static_cast<unsigned>((b.N + 255) / 256), 256, 0, st>>>(b, out);
    return hipGetLastError();
}

// per-batch count of machines not at a fixed point
// every machine's zero tail stored (zero_fill) or declared stored (its
// memory was written whole by other means): hw = n rounded up to 4
__global__ __launch_bounds__(256) void k_tails(DevBatch b, uint32_t zero_fill)
{
    const uint64_t v = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool in = v < b.N;
    const uint32_t top = in ? up4(b.n[v]) : 0u;
    uint32_t hw = in ? b.hw[v] : 0u;
    if (zero_fill) store_tails(in && hw < top, gptr(b.M + (in ? b.mem_off[v] : 0)), hw, top);
    if (in) b.hw[v] = top;
}

hipError_t launch_tails(DevBatch b, bool zero_fill, hipStream_t st)
{
    if (b.N == 0) return hipSuccess;
    k_tails<<<static_cast<unsigned>((b.N + 255) / 256), 256, 0, st>>>(b, zero_fill ? 1u : 0u);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_running(const BatchTable *__restrict__ tab, uint64_t total,
                                                 unsigned long long *__restrict__ counts)
{
    const uint64_t g = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    int k = 0;
    bool run = false;
    if (g < total) {
        k = batch_of(tab, g);
        run = tab->b[k].status[g - tab->start[k]] == 0;
    }
    // lanes of a wave may span two batches: aggregate per batch of the leader
    uint64_t rem = __ballot(g < total);
    while (rem) {
        const int leader = __ffsll(static_cast<unsigned long long>(rem)) - 1;
        const int kl = __shfl(k, leader);
        const uint64_t mine = __ballot(g < total && k == kl);
        const uint64_t cnt = __popcll(__ballot(g < total && k == kl && run));
        if ((threadIdx.x & (kWave - 1)) == static_cast<uint32_t>(leader) && cnt)
            atomicAdd(&counts[kl], static_cast<unsigned long long>(cnt));
        rem &= ~mine;
    }
}

hipError_t launch_running(const BatchTable *tab, uint64_t total, unsigned long long *counts,
                          hipStream_t st)
{
    k_running<<<static_cast<unsigned>((total + 255) / 256), 256, 0, st>>>(tab, total, counts);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_steps_sum(DevBatch b, unsigned long long *out)
{
    const uint64_t v = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    unsigned long long x = v < b.N ? b.steps[v] : 0ull;
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_down(x, off);
    if ((threadIdx.x & (kWave - 1)) == 0 && x) atomicAdd(out, x);
}

hipError_t launch_steps_sum(DevBatch b, unsigned long long *out, hipStream_t st)
{
    k_steps_sum<<<static_cast<unsigned>((b.N + 255) / 256), 256, 0, st>>>(b, out);
    return hipGetLastError();
}

// per-machine scalars into caller device buffers (any pointer may be null):
// one launch instead of one copy per field
__global__ __launch_bounds__(256) void k_fetch_scalars(DevBatch b, uint8_t *status, uint64_t *steps, int32_t *i,
                                                       int32_t *a, uint32_t *u0, uint32_t *y0)
{
    const uint64_t v = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= b.N) return;
    if (status) status[v] = b.status[v];
    if (steps) steps[v] = b.steps[v];
    if (i) i[v] = b.i[v];
    if (a) a[v] = b.a[v];
    if (u0) u0[v] = b.u0[v];
    if (y0) y0[v] = b.y0[v];
}

hipError_t launch_fetch_scalars(DevBatch b, uint8_t *status, uint64_t *steps, int32_t *i, int32_t *a,
                                uint32_t *u0, uint32_t *y0, hipStream_t st)
{
    k_fetch_scalars<<<static_cast<unsigned>((b.N + 255) / 256), 256, 0, st>>>(b, status, steps, i, a, u0, y0);
    return hipGetLastError();
}

// checks of a loaded state: u0 <= l, y0 <= s, and i, a w-bit words
__global__ __launch_bounds__(256) void k_check_state(DevBatch b, uint32_t *err)
{
    const uint64_t v = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= b.N) return;
    if (b.u0[v] > b.ell[v] || b.y0[v] > b.s[v]) atomicOr(err, kErrStateRange);
    const int32_t i = b.i[v], a = b.a[v];
    if (sext(static_cast<uint32_t>(i), b.wshift) != i || sext(static_cast<uint32_t>(a), b.wshift) != a)
        atomicOr(err, kErrWordRange);
}

// every word a w-bit value: one flag per block, one atomic per offending block
__global__ __launch_bounds__(256) void k_check_words(const int32_t *__restrict__ w, uint64_t count,
                                                     uint32_t ws, uint32_t *err)
{
    bool bad = false;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t k = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < count; k += stride) {
        const int32_t x = w[k];
        bad |= sext(static_cast<uint32_t>(x), ws) != x;
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(err, kErrWordRange);
}

// the same over words [off[0], off[N]) of a packed array (offsets in device memory)
__global__ __launch_bounds__(256) void k_check_words_off(const int32_t *__restrict__ w,
                                                         const uint64_t *__restrict__ off, uint64_t N,
                                                         uint32_t ws, uint32_t *err)
{
    const uint64_t lo = off[0], hi = off[N];
    bool bad = false;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t k = lo + static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < hi; k += stride) {
        const int32_t x = w[k];
        bad |= sext(static_cast<uint32_t>(x), ws) != x;
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(err, kErrWordRange);
}

hipError_t launch_check_words_off(const int32_t *w, const uint64_t *off, uint64_t N, uint32_t wshift,
                                  uint32_t *err, hipStream_t st)
{
    if (wshift == 0) return hipSuccess;
    k_check_words_off<<<2048, 256, 0, st>>>(w, off, N, wshift, err);
    return hipGetLastError();
}

hipError_t launch_check_words(const int32_t *w, uint64_t count, uint32_t wshift, uint32_t *err,
                              hipStream_t st)
{
    if (count == 0 || wshift == 0) return hipSuccess;
    uint64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_check_words<<<static_cast<unsigned>(blocks), 256, 0, st>>>(w, count, wshift, err);
    return hipGetLastError();
}

hipError_t launch_check_state(DevBatch b, uint32_t *err, hipStream_t st)
{
    k_check_state<<<static_cast<unsigned>((b.N + 255) / 256), 256, 0, st>>>(b, err);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exclusive scan (u32 or u64 in, u64 out): 1024 items per block
// ---------------------------------------------------------------------------

constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;
constexpr uint64_t kScanTile = kScanBlock * kScanItems;

uint64_t scan_scratch_words(uint64_t N) { return (N + kScanTile - 1) / kScanTile + 1; }

template <class T>
__device__ __forceinline__ uint64_t block_exclusive(uint64_t x, uint64_t *tmp, uint64_t &total)
{
    // inclusive scan inside each wave, then across the block's waves
    const uint32_t lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint64_t incl = x;
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t y = __shfl_up(incl, off);
        if (lane >= static_cast<uint32_t>(off)) incl += y;
    }
    if (lane == kWave - 1) tmp[w] = incl;
    __syncthreads();
    uint64_t before = 0;
    total = 0;
    for (int k = 0; k < kScanBlock / kWave; ++k) {
        if (k < static_cast<int>(w)) before += tmp[k];
        total += tmp[k];
    }
    __syncthreads();
    return before + incl - x;
}

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(const T *__restrict__ in, uint64_t N,
                                                           uint64_t *__restrict__ sums)
{
    __shared__ uint64_t tmp[kScanBlock / kWave];
    const uint64_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint64_t x = 0;
    for (int e = 0; e < kScanItems; ++e)
        if (base + e < N) x += static_cast<uint64_t>(in[base + e]);
    uint64_t total;
    block_exclusive<T>(x, tmp, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_sums(uint64_t *sums, uint64_t nb, uint64_t *total_out)
{
    __shared__ uint64_t tmp[kScanBlock / kWave];
    uint64_t carry = 0;
    for (uint64_t b0 = 0; b0 < nb; b0 += kScanBlock) {
        const uint64_t idx = b0 + threadIdx.x;
        const uint64_t x = idx < nb ? sums[idx] : 0;
        uint64_t total;
        const uint64_t ex = block_exclusive<uint64_t>(x, tmp, total);
        if (idx < nb) sums[idx] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const T *__restrict__ in, uint64_t N,
                                                           const uint64_t *__restrict__ sums,
                                                           uint64_t *__restrict__ out)
{
    __shared__ uint64_t tmp[kScanBlock / kWave];
    const uint64_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint64_t vals[kScanItems];
    uint64_t x = 0;
    for (int e = 0; e < kScanItems; ++e) {
        vals[e] = base + e < N ? static_cast<uint64_t>(in[base + e]) : 0;
        x += vals[e];
    }
    uint64_t total;
    uint64_t run = sums[blockIdx.x] + block_exclusive<T>(x, tmp, total);
    for (int e = 0; e < kScanItems; ++e) {
        if (base + e < N) out[base + e] = run;
        run += vals[e];
    }
}

template <class T>
static hipError_t scan_impl(const T *in, uint64_t *out, uint64_t N, uint64_t *sums,
                            uint64_t *total, hipStream_t st)
{
    const uint64_t nb = (N + kScanTile - 1) / kScanTile;
    if (nb == 0) return hipSuccess;
    k_scan_tiles<T><<<static_cast<unsigned>(nb), kScanBlock, 0, st>>>(in, N, sums);
    k_scan_sums<<<1, kScanBlock, 0, st>>>(sums, nb, total);
    k_scan_apply<T><<<static_cast<unsigned>(nb), kScanBlock, 0, st>>>(in, N, sums, out);
    return hipGetLastError();
}

hipError_t launch_scan_u64(const uint64_t *in, uint64_t *out, uint64_t N, uint64_t *sums,
                           uint64_t *total, hipStream_t st)
{
    return scan_impl<uint64_t>(in, out, N, sums, total, st);
}

hipError_t launch_scan_u32(const uint32_t *in, uint64_t *out, uint64_t N, uint64_t *sums,
                           uint64_t *total, hipStream_t st)
{
    return scan_impl<uint32_t>(in, out, N, sums, total, st);
}

// ---------------------------------------------------------------------------
// Batch layout from a device descriptor in three launches: per tile of
// kScanTile machines the shapes, checks, column sums (padded n, l, s, n) and
// maxima; one block scanning the four columns of tile sums; per tile the
// exclusive offsets of the padded memory, tape and output slices.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kScanBlock) void k_layout_tiles(
    const uint64_t *__restrict__ prog_off, const uint64_t *__restrict__ tape_off,
    const uint32_t *__restrict__ mem_words, uint32_t def_mem, const uint32_t *__restrict__ tape_cap,
    const uint32_t *__restrict__ out_cap, uint32_t def_out, uint64_t N, uint32_t *__restrict__ n_out,
    uint32_t *__restrict__ ell_out, uint32_t *__restrict__ s_out, uint64_t *__restrict__ sums, uint64_t nb,
    uint32_t *__restrict__ err, uint32_t *__restrict__ mx)
{
    __shared__ uint64_t part[4][kScanBlock / kWave];
    __shared__ uint32_t pmax[3][kScanBlock / kWave];
    const uint64_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint64_t x[4] = {0, 0, 0, 0};
    uint32_t e = 0, maxn = 0, np2 = 0, maxl = 0;
    for (int it = 0; it < kScanItems; ++it) {
        const uint64_t v = base + it;
        if (v >= N) break;
        const uint64_t p0 = prog_off[v], p1 = prog_off[v + 1];
        const uint64_t t0 = tape_off[v], t1 = tape_off[v + 1];
        if (p1 < p0 || t1 < t0) e |= kErrOffsets;
        const uint64_t plen = p1 >= p0 ? p1 - p0 : 0;
        const uint64_t tlen = t1 >= t0 ? t1 - t0 : 0;
        const uint32_t n = mem_words ? mem_words[v] : def_mem;
        const uint64_t ell = tape_cap ? static_cast<uint64_t>(tape_cap[v]) : tlen;
        const uint32_t s = out_cap ? out_cap[v] : def_out;
        if (n == 0 || n > kMaxMemWords) e |= kErrMemSize;
        if (plen > n) e |= kErrProgTooLong;
        if (tlen > ell || ell > 0x7fffffffull) e |= kErrTapeTooLong;
        if (s > 0x7fffffffu) e |= kErrMemSize;
        n_out[v] = n;
        ell_out[v] = static_cast<uint32_t>(ell);
        s_out[v] = s;
        x[0] += (static_cast<uint64_t>(n) + 3ull) & ~3ull;
        x[1] += ell;
        x[2] += s;
        x[3] += n;
        maxn = max(maxn, n);
        np2 |= (n & (n - 1u)) ? 1u : 0u;
        maxl = max(maxl, static_cast<uint32_t>(ell < 0xffffffffull ? ell : 0xffffffffull));
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        for (int c = 0; c < 4; ++c) x[c] += __shfl_xor(x[c], off);
        maxn = max(maxn, static_cast<uint32_t>(__shfl_xor(static_cast<int>(maxn), off)));
        maxl = max(maxl, static_cast<uint32_t>(__shfl_xor(static_cast<int>(maxl), off)));
        np2 |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(np2), off));
        e |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(e), off));
    }
    const uint32_t w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        for (int c = 0; c < 4; ++c) part[c][w] = x[c];
        pmax[0][w] = maxn; pmax[1][w] = np2 | (e << 1); pmax[2][w] = maxl;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        uint64_t t = 0;
        for (int k = 0; k < kScanBlock / kWave; ++k) t += part[threadIdx.x][k];
        sums[threadIdx.x * nb + blockIdx.x] = t;
    }
    if (threadIdx.x == 0) {
        uint32_t m0 = 0, f = 0, m2 = 0;
        for (int k = 0; k < kScanBlock / kWave; ++k) { m0 = max(m0, pmax[0][k]); f |= pmax[1][k]; m2 = max(m2, pmax[2][k]); }
        atomicMax(mx, m0);
        if (f & 1u) atomicOr(mx + 1, 1u);
        atomicMax(mx + 2, m2);
        if (f >> 1) atomicOr(err, f >> 1);
    }
}

// exclusive scan of the four columns of tile sums (in place); totals out
__global__ __launch_bounds__(kScanBlock) void k_layout_sums(uint64_t *sums, uint64_t nb, uint64_t *totals)
{
    __shared__ uint64_t tmp[kScanBlock / kWave];
    for (int c = 0; c < 4; ++c) {
        uint64_t *col = sums + c * nb;
        uint64_t carry = 0;
        for (uint64_t b0 = 0; b0 < nb; b0 += kScanBlock) {
            const uint64_t idx = b0 + threadIdx.x;
            const uint64_t x = idx < nb ? col[idx] : 0;
            uint64_t total;
            const uint64_t ex = block_exclusive<uint64_t>(x, tmp, total);
            if (idx < nb) col[idx] = carry + ex;
            carry += total;
        }
        if (threadIdx.x == 0) totals[c] = carry;
    }
}

__global__ __launch_bounds__(kScanBlock) void k_layout_apply(
    const uint32_t *__restrict__ n, const uint32_t *__restrict__ ell, const uint32_t *__restrict__ s,
    uint64_t N, const uint64_t *__restrict__ sums, uint64_t nb, uint64_t *__restrict__ mem_off,
    uint64_t *__restrict__ t_off, uint64_t *__restrict__ y_off)
{
    __shared__ uint64_t tmp[kScanBlock / kWave];
    const uint64_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint64_t vn[kScanItems], vl[kScanItems], vs[kScanItems];
    uint64_t xn = 0, xl = 0, xs = 0;
    for (int it = 0; it < kScanItems; ++it) {
        const bool in = base + it < N;
        vn[it] = in ? (static_cast<uint64_t>(n[base + it]) + 3ull) & ~3ull : 0;
        vl[it] = in ? ell[base + it] : 0;
        vs[it] = in ? s[base + it] : 0;
        xn += vn[it]; xl += vl[it]; xs += vs[it];
    }
    uint64_t total;
    uint64_t rn = sums[blockIdx.x] + block_exclusive<uint64_t>(xn, tmp, total);
    uint64_t rl = sums[nb + blockIdx.x] + block_exclusive<uint64_t>(xl, tmp, total);
    uint64_t rs = sums[2 * nb + blockIdx.x] + block_exclusive<uint64_t>(xs, tmp, total);
    for (int it = 0; it < kScanItems; ++it) {
        if (base + it < N) { mem_off[base + it] = rn; t_off[base + it] = rl; y_off[base + it] = rs; }
        rn += vn[it]; rl += vl[it]; rs += vs[it];
    }
}

uint64_t layout_scratch_words(uint64_t N) { return 4 * ((N + kScanTile - 1) / kScanTile) + 4; }

hipError_t launch_layout(const uint64_t *prog_off, const uint64_t *tape_off, const uint32_t *mem_words,
                         uint32_t def_mem, const uint32_t *tape_cap, const uint32_t *out_cap, uint32_t def_out,
                         uint64_t N, DevBatch b, uint64_t *sums, uint64_t *totals, uint32_t *err, uint32_t *mx,
                         hipStream_t st)
{
    const uint64_t nb = (N + kScanTile - 1) / kScanTile;
    k_layout_tiles<<<static_cast<unsigned>(nb), kScanBlock, 0, st>>>(prog_off, tape_off, mem_words, def_mem,
                                                                     tape_cap, out_cap, def_out, N, b.n, b.ell,
                                                                     b.s, sums, nb, err, mx);
    k_layout_sums<<<1, kScanBlock, 0, st>>>(sums, nb, totals);
    k_layout_apply<<<static_cast<unsigned>(nb), kScanBlock, 0, st>>>(b.n, b.ell, b.s, N, sums, nb, b.mem_off,
                                                                     b.t_off, b.y_off);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ragged copies between the padded memory arena and dense machine-major arrays
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_copy_ragged(const int32_t *__restrict__ src,
                                                     const uint64_t *__restrict__ src_off,
                                                     const uint32_t *__restrict__ len, uint64_t N,
                                                     int32_t *__restrict__ dst,
                                                     const uint64_t *__restrict__ dst_off)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t wave = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
    const uint64_t nwaves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) / kWave;
    for (uint64_t v = wave; v < N; v += nwaves) {
        const uint32_t n = len[v];
        const int32_t *s = src + src_off[v];
        int32_t *d = dst + dst_off[v];
        for (uint32_t k = lane; k < n; k += kWave) d[k] = s[k];
    }
}

static hipError_t copy_ragged(const int32_t *src, const uint64_t *src_off, const uint32_t *len,
                              uint64_t N, int32_t *dst, const uint64_t *dst_off, hipStream_t st)
{
    uint64_t blocks = (N + 3) / 4;
    if (blocks > 65536 * 4) blocks = 65536 * 4;
    if (blocks == 0) return hipSuccess;
    k_copy_ragged<<<static_cast<unsigned>(blocks), 256, 0, st>>>(src, src_off, len, N, dst, dst_off);
    return hipGetLastError();
}

hipError_t launch_gather_words(const int32_t *src, const uint64_t *off, const uint32_t *len,
                               uint64_t N, int32_t *dst, const uint64_t *dst_off, hipStream_t st)
{
    return copy_ragged(src, off, len, N, dst, dst_off, st);
}

hipError_t launch_scatter_words(const int32_t *src, const uint64_t *src_off, const uint32_t *len,
                                uint64_t N, int32_t *dst, const uint64_t *dst_off, hipStream_t st)
{
    return copy_ragged(src, src_off, len, N, dst, dst_off, st);
}

}  // namespace rasp
