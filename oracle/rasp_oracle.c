/*
 * rasp_oracle.c -- plain serial CPU oracle for the RASP step loop.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  No product code path calls
 * it, and it shares no source, header, table or helper with the GPU library.
 *
 * What it computes, for every machine independently (Sec. 2: the lifted map
 * Phi acts coordinatewise on d machines, each with static memory):
 *   Phi^B(c): the configuration reached after B applications of the one-step
 *   transition, a fixed point mapping to itself; the number of applications
 *   that changed the configuration (the halting number tau_h of Sec. 3, capped
 *   at B); and whether the final configuration is a fixed point (the halting
 *   set F of Sec. 1.1 and Sec. 2.1).
 *
 * A configuration of the word RASP (Sec. 2.1) is the flat word vector
 *     c = [ i, a, M_0 .. M_{n-1}, u_0, u_1 .. u_l, y_0, y_1 .. y_s ]
 * of length n + l + s + 4, which is the paper's C_w = W^(n+l+s+4).  u_0 is the
 * tape pointer and u_1..u_l the tape words; y_0 is the output count and
 * y_1..y_s the output words.
 *
 * Word arithmetic (Sec. 2.1): a word is w bits, held here sign-extended in an
 * int64_t; + and * wrap mod 2^w.  w is 32 everywhere outside the tests; the
 * tests also run w = 29 (the busy-beaver step counts of App. B come out only at
 * that width).
 *
 * Two instruction sets share the paper's numbering:
 *   WORD    (Sec. 2.1): 1 LOD, 2 ADD, 3 MUL, 4 STO, 5 BNZ, 6 RD, 7 PRI.
 *   CLASSIC (Sec. 1.1 plus JMP of Sec. 2.2): 1 LOD, 2 ADD, 3 SUB, 4 STO,
 *            5 BPA (jump if a > 0), 6 RD, 7 PRI, 8 JMP.
 * Every other opcode value falls in the "otherwise" case and is a fixed point
 * (HLT of Sec. 2.2 is the pair 0 0).
 *
 * Readings taken where the paper is silent or loose:
 *   - memory is addressed circularly, index = Euclidean remainder of the
 *     signed word by n, for fetch and for data (Sec. 2.1 fetch rule);
 *   - LOD is immediate (a <- j) in both sets (Sec. 1.1 and Sec. 2.1 tables);
 *   - RD reads tape word u_{u0+1} and advances u0; it is enabled only while
 *     u0 < l, otherwise the machine is stuck (Sec. 2.1 guard);
 *   - PRI appends only while y0 < s, else it is a no-op that still advances i
 *     (Sec. 2.1 y :: z);
 *   - a taken jump is a fixed point exactly when j equals i as a word;
 *   - the classic set reuses the word-RASP bounds (finite n, l, s) so that
 *     both sets run on the same finite configuration space.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define OR_ISA_WORD 0
#define OR_ISA_CLASSIC 1
#define OR_RUNNING 0
#define OR_HALTED 1

/* ---- word arithmetic (Sec. 2.1) ------------------------------------------ */

/* reduce v to w bits and sign-extend: the word that v names mod 2^w */
static int64_t wred(int64_t v, int w)
{
    uint64_t mask = (w >= 64) ? ~0ull : ((1ull << w) - 1ull);
    uint64_t x = (uint64_t)v & mask;
    uint64_t sign = 1ull << (w - 1);
    return (int64_t)(x ^ sign) - (int64_t)sign;
}

/* circular index: Euclidean remainder of a signed word by n (n >= 1) */
static uint32_t cidx(int64_t v, uint32_t n)
{
    int64_t r = v % (int64_t)n;
    if (r < 0) r += (int64_t)n;
    return (uint32_t)r;
}

/* ---- the definitional form: Phi_w on a whole configuration vector -------- */

/*
 * or_step_full: d <- Phi_w(c) for one machine, both flat vectors as described
 * at the top of this file.  Every case of the Sec. 1.1 / Sec. 2.1 table is
 * written out; the result is a complete new configuration (c is not touched).
 * Used by the tests on tiny machines, where a fixed point is detected by
 * comparing the whole vector with its successor.
 */
void or_step_full(int isa, int w, uint32_t n, uint32_t l, uint32_t s,
                  const int64_t *c, int64_t *d)
{
    const uint64_t len = (uint64_t)n + l + s + 4;
    const int64_t i = c[0], a = c[1];
    const int64_t *M = c + 2;
    const int64_t u0 = c[2 + n];
    const int64_t *u = c + 2 + n;           /* u[0] = u0, u[1..l] = tape */
    const int64_t y0 = c[3 + n + l];
    int64_t *dM = d + 2;
    int64_t *du = d + 2 + n;
    int64_t *dy = d + 3 + n + l;            /* dy[0] = y0, dy[1..s] = words */
    memcpy(d, c, len * sizeof(int64_t));

    const int64_t o = M[cidx(i, n)];
    const int64_t j = M[cidx(wred(i + 1, w), n)];
    const int64_t next = wred(i + 2, w);

    if (isa == OR_ISA_WORD) {
        switch (o) {
        case 1: d[0] = next; d[1] = j; return;                              /* LOD */
        case 2: d[0] = next; d[1] = wred(a + M[cidx(j, n)], w); return;     /* ADD */
        case 3: d[0] = next; d[1] = wred(a * M[cidx(j, n)], w); return;     /* MUL */
        case 4: d[0] = next; dM[cidx(j, n)] = a; return;                    /* STO */
        case 5: d[0] = (a != 0) ? j : next; return;                         /* BNZ */
        case 6:                                                             /* RD  */
            if (u0 < (int64_t)l) {
                d[0] = next;
                dM[cidx(j, n)] = u[u0 + 1];
                du[0] = u0 + 1;
            }
            return;
        case 7:                                                             /* PRI */
            d[0] = next;
            if (y0 < (int64_t)s) { dy[y0 + 1] = M[cidx(j, n)]; dy[0] = y0 + 1; }
            return;
        default: return;                                                    /* otherwise */
        }
    } else {
        switch (o) {
        case 1: d[0] = next; d[1] = j; return;                              /* LOD */
        case 2: d[0] = next; d[1] = wred(a + M[cidx(j, n)], w); return;     /* ADD */
        case 3: d[0] = next; d[1] = wred(a - M[cidx(j, n)], w); return;     /* SUB */
        case 4: d[0] = next; dM[cidx(j, n)] = a; return;                    /* STO */
        case 5: d[0] = (a > 0) ? j : next; return;                          /* BPA */
        case 6:                                                             /* RD  */
            if (u0 < (int64_t)l) {
                d[0] = next;
                dM[cidx(j, n)] = u[u0 + 1];
                du[0] = u0 + 1;
            }
            return;
        case 7:                                                             /* PRI */
            d[0] = next;
            if (y0 < (int64_t)s) { dy[y0 + 1] = M[cidx(j, n)]; dy[0] = y0 + 1; }
            return;
        case 8: d[0] = j; return;                                           /* JMP */
        default: return;                                                    /* otherwise */
        }
    }
}

/* ---- the interpreter: Phi^B in place, one machine at a time -------------- */

/*
 * One machine's state, held in place.  M, T, Y are that machine's slices of
 * the batch arrays; the successor is computed as the handful of coordinates
 * the transition may change, and the machine is at a fixed point exactly when
 * every one of them equals its current value (F = { c : c -> c }).
 */
typedef struct {
    int64_t i, a;
    int32_t *M; uint32_t n;
    const int32_t *T; uint32_t l; int64_t u0;
    int32_t *Y; uint32_t s; int64_t y0;
} vm_t;

/* Advance one machine by at most `budget` transitions.  Returns the number of
 * transitions applied; *halted says whether the final configuration is a fixed
 * point. */
static uint64_t run_one(int isa, int w, vm_t *v, uint64_t budget, int *halted,
                        uint64_t *hist)
{
    uint64_t t = 0;
    for (;;) {
        const int64_t i = v->i, a = v->a;
        const int64_t o = v->M[cidx(i, v->n)];
        const int64_t j = v->M[cidx(wred(i + 1, w), v->n)];
        const int64_t next = wred(i + 2, w);

        /* successor coordinates, defaulting to "unchanged" */
        int64_t ni = i, na = a, nu0 = v->u0, ny0 = v->y0;
        int mw = 0; uint32_t maddr = 0; int64_t mval = 0;   /* memory write  */
        int yw = 0; uint32_t yidx = 0; int64_t yval = 0;    /* output write  */

        int kind = (int)o;                 /* map both sets onto one switch */
        if (o < 1 || o > 8 || (isa == OR_ISA_WORD && o == 8)) kind = 0;
        switch (kind) {
        case 1: ni = next; na = j; break;
        case 2: ni = next; na = wred(a + v->M[cidx(j, v->n)], w); break;
        case 3:
            ni = next;
            if (isa == OR_ISA_WORD) na = wred(a * v->M[cidx(j, v->n)], w);
            else                    na = wred(a - v->M[cidx(j, v->n)], w);
            break;
        case 4: ni = next; mw = 1; maddr = cidx(j, v->n); mval = a; break;
        case 5:
            if (isa == OR_ISA_WORD) ni = (a != 0) ? j : next;
            else                    ni = (a > 0) ? j : next;
            break;
        case 6:
            if (v->u0 < (int64_t)v->l) {
                ni = next; mw = 1; maddr = cidx(j, v->n);
                mval = v->T[v->u0]; nu0 = v->u0 + 1;
            }
            break;
        case 7:
            ni = next;
            if (v->y0 < (int64_t)v->s) {
                yw = 1; yidx = (uint32_t)v->y0; yval = v->M[cidx(j, v->n)];
                ny0 = v->y0 + 1;
            }
            break;
        case 8: ni = j; break;
        default: break;
        }

        const int fixed = (ni == i) && (na == a) && (nu0 == v->u0) &&
                          (ny0 == v->y0) &&
                          (!mw || v->M[maddr] == mval) &&
                          (!yw || v->Y[yidx] == yval);
        if (fixed) { *halted = 1; return t; }
        if (t == budget) { *halted = 0; return t; }

        v->i = ni; v->a = na; v->u0 = nu0; v->y0 = ny0;
        if (mw) v->M[maddr] = (int32_t)mval;
        if (yw) v->Y[yidx] = (int32_t)yval;
        if (hist) {                      /* retired opcode, and appended outputs */
            hist[kind] += 1;
            hist[9] += (uint64_t)yw;
        }
        ++t;
    }
}

/* ---- batch entry points --------------------------------------------------- */

/*
 * or_c0: write the initial configuration c0(P, x) of Sec. 2.1 for N machines:
 *   i = 0, a = 0, M = P 0^(n-2m), tape = x 0^(l-|x|), u0 = 0, y = 0^(s+1),
 *   steps = 0.  P is stored in memory (Sec. 2: each machine stores its program
 *   in memory).  prog words of machine v are prog[prog_off[v] .. prog_off[v+1]),
 *   its tape words tape[tape_off[v] .. tape_off[v+1]).  mem/T/Y are the output
 *   arenas addressed by mem_off/t_off/y_off.  Words are reduced to w bits.
 *   Returns 0, or -1 if some machine violates 2m <= n or |x| <= l.
 */
int or_c0(int w, uint64_t N,
          const int32_t *prog, const uint64_t *prog_off,
          const int32_t *tape, const uint64_t *tape_off,
          const uint32_t *n, const uint32_t *l, const uint32_t *s,
          const uint64_t *mem_off, const uint64_t *t_off, const uint64_t *y_off,
          int32_t *ri, int32_t *ra, uint32_t *ru0, uint32_t *ry0,
          uint64_t *steps, uint8_t *status,
          int32_t *mem, int32_t *T, int32_t *Y)
{
    for (uint64_t v = 0; v < N; ++v) {
        const uint64_t pm = prog_off[v + 1] - prog_off[v];
        const uint64_t tx = tape_off[v + 1] - tape_off[v];
        if (pm > n[v] || tx > l[v]) return -1;
        for (uint64_t k = 0; k < n[v]; ++k)
            mem[mem_off[v] + k] = (k < pm) ? (int32_t)wred(prog[prog_off[v] + k], w) : 0;
        for (uint64_t k = 0; k < l[v]; ++k)
            T[t_off[v] + k] = (k < tx) ? (int32_t)wred(tape[tape_off[v] + k], w) : 0;
        for (uint64_t k = 0; k < s[v]; ++k) Y[y_off[v] + k] = 0;
        ri[v] = 0; ra[v] = 0; ru0[v] = 0; ry0[v] = 0; steps[v] = 0; status[v] = OR_RUNNING;
    }
    return 0;
}

typedef struct {
    int isa, w; uint64_t N, budget; int stride, first;
    uint64_t hist[16]; int count;
    int32_t *ri, *ra; uint32_t *ru0, *ry0; uint64_t *steps; uint8_t *status;
    int32_t *mem; const uint64_t *mem_off; const uint32_t *n;
    const int32_t *T; const uint64_t *t_off; const uint32_t *l;
    int32_t *Y; const uint64_t *y_off; const uint32_t *s;
} job_t;

static void *advance_stripe(void *arg)
{
    job_t *jb = (job_t *)arg;
    for (uint64_t v = (uint64_t)jb->first; v < jb->N; v += (uint64_t)jb->stride) {
        vm_t m;
        m.i = wred(jb->ri[v], jb->w); m.a = wred(jb->ra[v], jb->w);
        m.M = jb->mem + jb->mem_off[v]; m.n = jb->n[v];
        m.T = jb->T + jb->t_off[v]; m.l = jb->l[v]; m.u0 = jb->ru0[v];
        m.Y = jb->Y + jb->y_off[v]; m.s = jb->s[v]; m.y0 = jb->ry0[v];
        int halted = 0;
        uint64_t t = run_one(jb->isa, jb->w, &m, jb->budget, &halted,
                             jb->count ? jb->hist : NULL);
        jb->ri[v] = (int32_t)m.i; jb->ra[v] = (int32_t)m.a;
        jb->ru0[v] = (uint32_t)m.u0; jb->ry0[v] = (uint32_t)m.y0;
        jb->steps[v] += t;
        jb->status[v] = halted ? OR_HALTED : OR_RUNNING;
    }
    return NULL;
}

/*
 * or_advance: advance N machines, each by at most `budget` more transitions,
 * in place.  Machines are independent; with threads > 1 machine v goes to host
 * thread v mod threads (the static round-robin striping of Sec. 2.3), which
 * changes nothing in the result.  steps[] accumulates; status[] is recomputed
 * as "final configuration is a fixed point".  Every machine must satisfy
 * u0 <= l and y0 <= s.  Returns 0, or -1 on bad arguments.
 */
int or_advance_mix(int isa, int w, uint64_t N, uint64_t budget, int threads,
                   int32_t *ri, int32_t *ra, uint32_t *ru0, uint32_t *ry0,
                   uint64_t *steps, uint8_t *status,
                   int32_t *mem, const uint64_t *mem_off, const uint32_t *n,
                   const int32_t *T, const uint64_t *t_off, const uint32_t *l,
                   int32_t *Y, const uint64_t *y_off, const uint32_t *s,
                   uint64_t *mix);

int or_advance(int isa, int w, uint64_t N, uint64_t budget, int threads,
               int32_t *ri, int32_t *ra, uint32_t *ru0, uint32_t *ry0,
               uint64_t *steps, uint8_t *status,
               int32_t *mem, const uint64_t *mem_off, const uint32_t *n,
               const int32_t *T, const uint64_t *t_off, const uint32_t *l,
               int32_t *Y, const uint64_t *y_off, const uint32_t *s)
{
    return or_advance_mix(isa, w, N, budget, threads, ri, ra, ru0, ry0, steps, status,
                          mem, mem_off, n, T, t_off, l, Y, y_off, s, NULL);
}

/*
 * or_advance_mix: or_advance that also adds, into mix[16] (when not NULL), the
 * number of retired transitions per opcode (mix[1..8]; the stuck kinds never
 * retire) and in mix[9] the number of PRINTs that appended an output word.
 */
int or_advance_mix(int isa, int w, uint64_t N, uint64_t budget, int threads,
                   int32_t *ri, int32_t *ra, uint32_t *ru0, uint32_t *ry0,
                   uint64_t *steps, uint8_t *status,
                   int32_t *mem, const uint64_t *mem_off, const uint32_t *n,
                   const int32_t *T, const uint64_t *t_off, const uint32_t *l,
                   int32_t *Y, const uint64_t *y_off, const uint32_t *s,
                   uint64_t *mix)
{
    if (w < 2 || w > 32 || (isa != OR_ISA_WORD && isa != OR_ISA_CLASSIC)) return -1;
    for (uint64_t v = 0; v < N; ++v)
        if (n[v] == 0 || ru0[v] > l[v] || ry0[v] > s[v]) return -1;
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > N && N > 0) threads = (int)N;
    job_t *jobs = (job_t *)calloc((size_t)threads, sizeof(job_t));
    pthread_t *tids = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    if (!jobs || !tids) { free(jobs); free(tids); return -1; }
    for (int t = 0; t < threads; ++t) {
        job_t *jb = &jobs[t];
        jb->isa = isa; jb->w = w; jb->N = N; jb->budget = budget;
        jb->stride = threads; jb->first = t; jb->count = (mix != NULL);
        jb->ri = ri; jb->ra = ra; jb->ru0 = ru0; jb->ry0 = ry0;
        jb->steps = steps; jb->status = status;
        jb->mem = mem; jb->mem_off = mem_off; jb->n = n;
        jb->T = T; jb->t_off = t_off; jb->l = l;
        jb->Y = Y; jb->y_off = y_off; jb->s = s;
    }
    /* calloc zeroed every jobs[t].hist; run_one counts only when asked */
    if (threads == 1) {
        advance_stripe(&jobs[0]);
    } else {
        int started = 0;
        for (int t = 0; t < threads; ++t) {
            if (pthread_create(&tids[t], NULL, advance_stripe, &jobs[t]) != 0) break;
            ++started;
        }
        for (int t = 0; t < started; ++t) pthread_join(tids[t], NULL);
        for (int t = started; t < threads; ++t) advance_stripe(&jobs[t]);
    }
    if (mix)
        for (int t = 0; t < threads; ++t)
            for (int k = 0; k < 16; ++k) mix[k] += jobs[t].hist[k];
    free(jobs); free(tids);
    return 0;
}

/*
 * or_fnv1a64: FNV-1a 64-bit hash (offset basis 0xcbf29ce484222325, prime
 * 0x100000001b3, as published by Fowler, Noll and Vo) of n words taken as
 * little-endian bytes.  Used to compare large memories without moving them.
 */
uint64_t or_fnv1a64(const int32_t *words, uint64_t n)
{
    uint64_t h = 0xcbf29ce484222325ull;
    for (uint64_t k = 0; k < n; ++k) {
        uint32_t x = (uint32_t)words[k];
        for (int b = 0; b < 4; ++b) {
            h ^= (x >> (8 * b)) & 0xffu;
            h *= 0x100000001b3ull;
        }
    }
    return h;
}

void or_digest_batch(uint64_t N, const int32_t *mem, const uint64_t *mem_off,
                     const uint32_t *n, uint64_t *out)
{
    for (uint64_t v = 0; v < N; ++v) out[v] = or_fnv1a64(mem + mem_off[v], n[v]);
}
