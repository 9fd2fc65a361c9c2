/*
 * CPU oracle for exact multiple pattern matching.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or
 * call this file; it exists so that tests and the benchmark's CPU baseline can
 * check the GPU path against an independent, plainly written implementation.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Problem (paper, Section 1, Definition): given a text T = t_0..t_{n-1} and d
 * patterns p^0..p^{d-1}, all of length m, report every pair (i, r) with
 * 0 <= i < n-m+1 such that t_{i+j} = p^r_j for every 0 <= j < m. (The printed
 * condition reads "t_i = p^r_j"; the index i+j is the only reading under which
 * the definition describes an occurrence.)
 *
 * Every routine emits pairs in ascending (position, pattern id) order and can
 * be restricted to the start positions [lo, hi), which is how the paper splits
 * a text between workers (Section 4.2.1 and the chunk-assignment equation of
 * Section 4.4: each worker reads m-1 characters past its own range).
 *
 * Four implementations:
 *   orc_bf   - the definition, position by position and pattern by pattern.
 *   orc_win  - the definition at scale: every length-m window is looked up in
 *              the sorted list of patterns (binary search). Exact.
 *   orc_ac_* - Aho-Corasick as the paper states it (Section 3.1, Algorithms
 *              1-3): goto function over all 256 byte values with creation-order
 *              state numbers, supply function built in breadth-first order,
 *              search with the supply while-loop.
 *   orc_wm_* - Wu-Manber as the paper states it (Section 3.2, Algorithms 4-5):
 *              SHIFT/HASH/PREFIX tables over B-character blocks with the
 *              shift-and-add hash over byte values (B = 3, B' = 2, bitshift = 2
 *              in the paper's experiments; all three are parameters here), and
 *              direct verification with memcmp.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Output sink: stores pairs while there is room, always counts.            */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t *pos;
    uint32_t *id;
    uint64_t cap;
    uint64_t count;
} sink_t;

static void emit(sink_t *s, uint64_t pos, uint32_t id)
{
    if (s->count < s->cap) {
        s->pos[s->count] = (uint32_t)pos;
        s->id[s->count] = id;
    }
    s->count++;
}

static uint64_t min_u64(uint64_t a, uint64_t b) { return a < b ? a : b; }

/* ------------------------------------------------------------------------ */
/* orc_bf: the definition, literally (Section 1).                           */
/* ------------------------------------------------------------------------ */
uint64_t orc_bf(const uint8_t *T, uint64_t n, const uint8_t *P, uint32_t d,
                uint32_t m, uint64_t lo, uint64_t hi, uint32_t *pos,
                uint32_t *id, uint64_t cap)
{
    sink_t s = {pos, id, cap, 0};
    if (m == 0 || n < m)
        return 0;
    uint64_t last = n - m + 1; /* 0 <= i < n - m + 1 */
    hi = min_u64(hi, last);
    for (uint64_t i = lo; i < hi; i++) {
        for (uint32_t r = 0; r < d; r++) {
            int all = 1;
            for (uint32_t j = 0; j < m; j++) {
                if (T[i + j] != P[(uint64_t)r * m + j]) {
                    all = 0;
                    break;
                }
            }
            if (all)
                emit(&s, i, r);
        }
    }
    return s.count;
}

/* ------------------------------------------------------------------------ */
/* orc_win: every window looked up in the sorted pattern list.              */
/* ------------------------------------------------------------------------ */
typedef struct {
    const uint8_t *P;
    uint32_t m;
    uint32_t d;
    uint32_t *order; /* pattern ids sorted by (bytes, id) */
} win_t;

static const uint8_t *g_sort_P;
static uint32_t g_sort_m;

static int cmp_ids(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    int c = memcmp(g_sort_P + (uint64_t)x * g_sort_m, g_sort_P + (uint64_t)y * g_sort_m, g_sort_m);
    if (c)
        return c;
    return (x > y) - (x < y);
}

void *orc_win_build(const uint8_t *P, uint32_t d, uint32_t m)
{
    win_t *w = (win_t *)calloc(1, sizeof(win_t));
    uint8_t *copy = (uint8_t *)malloc((uint64_t)d * m + 1);
    memcpy(copy, P, (uint64_t)d * m);
    w->P = copy;
    w->m = m;
    w->d = d;
    w->order = (uint32_t *)malloc(sizeof(uint32_t) * (d ? d : 1));
    for (uint32_t r = 0; r < d; r++)
        w->order[r] = r;
    g_sort_P = copy; /* qsort has no context argument; build is single-threaded */
    g_sort_m = m;
    qsort(w->order, d, sizeof(uint32_t), cmp_ids);
    return w;
}

void orc_win_free(void *h)
{
    win_t *w = (win_t *)h;
    if (!w)
        return;
    free((void *)w->P);
    free(w->order);
    free(w);
}

/* Thread-safe (read-only on the built structure). */
uint64_t orc_win_scan(const void *h, const uint8_t *T, uint64_t n, uint64_t lo,
                      uint64_t hi, uint32_t *pos, uint32_t *id, uint64_t cap)
{
    const win_t *w = (const win_t *)h;
    sink_t s = {pos, id, cap, 0};
    uint32_t m = w->m;
    if (m == 0 || n < m || w->d == 0)
        return 0;
    hi = min_u64(hi, n - m + 1);
    for (uint64_t i = lo; i < hi; i++) {
        const uint8_t *win = T + i;
        /* first sorted entry whose pattern is >= the window */
        uint32_t a = 0, b = w->d;
        while (a < b) {
            uint32_t mid = a + (b - a) / 2;
            if (memcmp(w->P + (uint64_t)w->order[mid] * m, win, m) < 0)
                a = mid + 1;
            else
                b = mid;
        }
        while (a < w->d && memcmp(w->P + (uint64_t)w->order[a] * m, win, m) == 0) {
            emit(&s, i, w->order[a]);
            a++;
        }
    }
    return s.count;
}

/* ------------------------------------------------------------------------ */
/* orc_ac: Aho-Corasick, Section 3.1, Algorithms 1-3.                       */
/* ------------------------------------------------------------------------ */
#define AC_FAIL (-1)

typedef struct {
    uint32_t m, d;
    uint64_t nstates, capstates;
    int32_t *g;        /* goto: nstates x 256, AC_FAIL where undefined */
    int32_t *supply;   /* supply (failure) link per state */
    uint32_t *depth;   /* |L(q)| */
    uint32_t **out;    /* Output(q): pattern ids, ascending */
    uint32_t *nout;
    uint32_t *capout;
} ac_t;

static uint64_t ac_new_state(ac_t *a, uint32_t depth)
{
    if (a->nstates == a->capstates) {
        uint64_t nc = a->capstates ? a->capstates * 2 : 64;
        a->g = (int32_t *)realloc(a->g, nc * 256 * sizeof(int32_t));
        a->supply = (int32_t *)realloc(a->supply, nc * sizeof(int32_t));
        a->depth = (uint32_t *)realloc(a->depth, nc * sizeof(uint32_t));
        a->out = (uint32_t **)realloc(a->out, nc * sizeof(uint32_t *));
        a->nout = (uint32_t *)realloc(a->nout, nc * sizeof(uint32_t));
        a->capout = (uint32_t *)realloc(a->capout, nc * sizeof(uint32_t));
        a->capstates = nc;
    }
    uint64_t q = a->nstates++;
    for (int c = 0; c < 256; c++) /* for all alpha: g(q, alpha) := fail */
        a->g[q * 256 + c] = AC_FAIL;
    a->supply[q] = AC_FAIL;
    a->depth[q] = depth;
    a->out[q] = NULL;
    a->nout[q] = 0;
    a->capout[q] = 0;
    return q;
}

static void ac_add_output(ac_t *a, uint64_t q, uint32_t r)
{
    if (a->nout[q] == a->capout[q]) {
        uint32_t nc = a->capout[q] ? a->capout[q] * 2 : 2;
        a->out[q] = (uint32_t *)realloc(a->out[q], nc * sizeof(uint32_t));
        a->capout[q] = nc;
    }
    a->out[q][a->nout[q]++] = r;
}

void *orc_ac_build(const uint8_t *P, uint32_t d, uint32_t m)
{
    ac_t *a = (ac_t *)calloc(1, sizeof(ac_t));
    a->m = m;
    a->d = d;
    ac_new_state(a, 0); /* q0 */

    /* Algorithm 1: goto function. Patterns are inserted in id order; states
     * are numbered in creation order. */
    for (uint32_t i = 0; i < d; i++) {
        const uint8_t *p = P + (uint64_t)i * m;
        uint32_t j = 0;
        int64_t state = 0;
        while (j < m && a->g[state * 256 + p[j]] != AC_FAIL) {
            state = a->g[state * 256 + p[j]];
            j++;
        }
        for (uint32_t l = j; l < m; l++) {
            uint64_t q = ac_new_state(a, l + 1);
            a->g[state * 256 + p[l]] = (int32_t)q;
            state = (int64_t)q;
        }
        /* Output(state) gains p^i. When the pattern was already in the trie
         * (a duplicate) the loop above creates nothing and the terminal is
         * the state the walk ended in. */
        ac_add_output(a, (uint64_t)state, i);
    }

    /* Algorithm 2: supply function. Root transitions that fail become root
     * self-loops; the root's children get the root as supply. */
    uint64_t S = a->nstates;
    uint32_t *queue = (uint32_t *)malloc(sizeof(uint32_t) * (S ? S : 1));
    uint64_t qh = 0, qt = 0;
    for (int c = 0; c < 256; c++) {
        int32_t s = a->g[c];
        if (s == AC_FAIL) {
            a->g[c] = 0;
        } else {
            a->supply[s] = 0;
            queue[qt++] = (uint32_t)s;
        }
    }
    a->supply[0] = 0;
    /* States in breadth-first ("transversal") order, so a state's supply is
     * known before its children are visited. */
    while (qh < qt) {
        uint32_t cur = queue[qh++];
        for (int c = 0; c < 256; c++) {
            int32_t s = a->g[(uint64_t)cur * 256 + c];
            if (s == AC_FAIL)
                continue;
            int32_t state = a->supply[cur];
            while (a->g[(uint64_t)state * 256 + c] == AC_FAIL)
                state = a->supply[state];
            a->supply[s] = a->g[(uint64_t)state * 256 + c];
            queue[qt++] = (uint32_t)s;
        }
    }
    free(queue);
    return a;
}

void orc_ac_free(void *h)
{
    ac_t *a = (ac_t *)h;
    if (!a)
        return;
    for (uint64_t q = 0; q < a->nstates; q++)
        free(a->out[q]);
    free(a->g);
    free(a->supply);
    free(a->depth);
    free(a->out);
    free(a->nout);
    free(a->capout);
    free(a);
}

uint64_t orc_ac_nstates(const void *h) { return ((const ac_t *)h)->nstates; }

/* g(q, c) as built (after Algorithm 2 the root has self-loops). */
int32_t orc_ac_goto(const void *h, uint64_t q, uint32_t c)
{
    const ac_t *a = (const ac_t *)h;
    return a->g[q * 256 + (c & 255)];
}

int32_t orc_ac_supply(const void *h, uint64_t q) { return ((const ac_t *)h)->supply[q]; }
uint32_t orc_ac_depth(const void *h, uint64_t q) { return ((const ac_t *)h)->depth[q]; }
uint32_t orc_ac_nout(const void *h, uint64_t q) { return ((const ac_t *)h)->nout[q]; }
uint32_t orc_ac_out(const void *h, uint64_t q, uint32_t k) { return ((const ac_t *)h)->out[q][k]; }

/* Algorithm 3 over the start positions [lo, hi): the walk begins in q0 at lo
 * and reads up to m-1 characters past hi (the overlap of Section 4.2.1). At a
 * state with non-empty Output the match is reported at i-m+1. Thread-safe. */
uint64_t orc_ac_scan(const void *h, const uint8_t *T, uint64_t n, uint64_t lo,
                     uint64_t hi, uint32_t *pos, uint32_t *id, uint64_t cap)
{
    const ac_t *a = (const ac_t *)h;
    sink_t s = {pos, id, cap, 0};
    uint32_t m = a->m;
    if (m == 0 || n < m)
        return 0;
    hi = min_u64(hi, n - m + 1);
    if (lo >= hi)
        return 0;
    uint64_t stop = min_u64(hi + m - 1, n);
    int64_t state = 0;
    for (uint64_t i = lo; i < stop; i++) {
        int32_t next;
        while ((next = a->g[state * 256 + T[i]]) == AC_FAIL)
            state = a->supply[state];
        state = next;
        if (a->nout[state] != 0) {
            for (uint32_t k = 0; k < a->nout[state]; k++)
                emit(&s, i - m + 1, a->out[state][k]);
        }
    }
    return s.count;
}

/* The state after each character (for checking the longest-suffix
 * characterisation of Section 3.1). states[i - lo] for i in [lo, hi). */
void orc_ac_trace(const void *h, const uint8_t *T, uint64_t lo, uint64_t hi, int32_t *states)
{
    const ac_t *a = (const ac_t *)h;
    int64_t state = 0;
    for (uint64_t i = lo; i < hi; i++) {
        int32_t next;
        while ((next = a->g[state * 256 + T[i]]) == AC_FAIL)
            state = a->supply[state];
        state = next;
        states[i - lo] = (int32_t)state;
    }
}

/* ------------------------------------------------------------------------ */
/* orc_wm: Wu-Manber, Section 3.2, Algorithms 4-5.                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t m, d, B, Bp, bitshift;
    uint64_t tsize;      /* SHIFT/HASH table size: sum_{i<B} 256 * (2^bitshift)^i */
    uint8_t *P;          /* copy of the patterns */
    uint32_t *SHIFT;
    uint32_t **HASH;     /* ascending pattern ids per suffix hash */
    uint32_t *nhash;
    uint32_t *caphash;
    uint64_t *PREFIX;    /* h2 of each pattern's first B' characters */
} wm_t;

/* Shift-and-add hash: shift left by bitshift, add the byte value. */
static uint64_t wm_hash(const uint8_t *c, uint32_t len, uint32_t bitshift)
{
    uint64_t h = 0;
    for (uint32_t k = 0; k < len; k++)
        h = (h << bitshift) + c[k];
    return h;
}

uint64_t orc_wm_table_size(uint32_t B, uint32_t bitshift)
{
    uint64_t t = 0, p = 1;
    for (uint32_t i = 0; i < B; i++) {
        t += 256 * p;
        p <<= bitshift;
    }
    return t;
}

/* Returns NULL when m < B or m < B' (SHIFT starts at m-B+1, Algorithm 4). */
void *orc_wm_build(const uint8_t *P, uint32_t d, uint32_t m, uint32_t B,
                   uint32_t Bp, uint32_t bitshift)
{
    if (B == 0 || Bp == 0 || m < B || m < Bp || bitshift > 8 || B > 6 || Bp > 6)
        return NULL;
    wm_t *w = (wm_t *)calloc(1, sizeof(wm_t));
    w->m = m;
    w->d = d;
    w->B = B;
    w->Bp = Bp;
    w->bitshift = bitshift;
    w->tsize = orc_wm_table_size(B, bitshift);
    w->P = (uint8_t *)malloc((uint64_t)d * m + 1);
    memcpy(w->P, P, (uint64_t)d * m);
    w->SHIFT = (uint32_t *)malloc(sizeof(uint32_t) * w->tsize);
    w->HASH = (uint32_t **)calloc(w->tsize, sizeof(uint32_t *));
    w->nhash = (uint32_t *)calloc(w->tsize, sizeof(uint32_t));
    w->caphash = (uint32_t *)calloc(w->tsize, sizeof(uint32_t));
    w->PREFIX = (uint64_t *)calloc(d ? d : 1, sizeof(uint64_t));

    /* Algorithm 4 */
    for (uint64_t h = 0; h < w->tsize; h++)
        w->SHIFT[h] = m - B + 1;
    for (uint32_t i = 0; i < d; i++) {
        const uint8_t *p = w->P + (uint64_t)i * m;
        for (uint32_t q = m; q >= B; q--) {
            /* the B characters ending at p_{q-1}: p_{q-B} .. p_{q-1} */
            uint64_t h = wm_hash(p + q - B, B, bitshift);
            uint32_t shiftlen = m - q;
            if (shiftlen < w->SHIFT[h])
                w->SHIFT[h] = shiftlen;
            if (shiftlen == 0) {
                if (w->nhash[h] == w->caphash[h]) {
                    uint32_t nc = w->caphash[h] ? w->caphash[h] * 2 : 2;
                    w->HASH[h] = (uint32_t *)realloc(w->HASH[h], nc * sizeof(uint32_t));
                    w->caphash[h] = nc;
                }
                w->HASH[h][w->nhash[h]++] = i;
                w->PREFIX[i] = wm_hash(p, Bp, bitshift);
            }
            if (q == B)
                break; /* unsigned loop guard */
        }
    }
    return w;
}

void orc_wm_free(void *h)
{
    wm_t *w = (wm_t *)h;
    if (!w)
        return;
    for (uint64_t t = 0; t < w->tsize; t++)
        free(w->HASH[t]);
    free(w->HASH);
    free(w->nhash);
    free(w->caphash);
    free(w->SHIFT);
    free(w->PREFIX);
    free(w->P);
    free(w);
}

uint64_t orc_wm_tsize(const void *h) { return ((const wm_t *)h)->tsize; }
uint32_t orc_wm_shift(const void *h, uint64_t t) { return ((const wm_t *)h)->SHIFT[t]; }
uint32_t orc_wm_nhash(const void *h, uint64_t t) { return ((const wm_t *)h)->nhash[t]; }
uint32_t orc_wm_hash_entry(const void *h, uint64_t t, uint32_t k) { return ((const wm_t *)h)->HASH[t][k]; }
uint64_t orc_wm_prefix(const void *h, uint32_t r) { return ((const wm_t *)h)->PREFIX[r]; }

/* Algorithm 5 over the start positions [lo, hi): window ends run from
 * lo+m-1 while the window start is below hi and the end is inside the text.
 * Thread-safe. */
uint64_t orc_wm_scan(const void *h, const uint8_t *T, uint64_t n, uint64_t lo,
                     uint64_t hi, uint32_t *pos, uint32_t *id, uint64_t cap)
{
    const wm_t *w = (const wm_t *)h;
    sink_t s = {pos, id, cap, 0};
    uint32_t m = w->m, B = w->B, Bp = w->Bp;
    if (n < m)
        return 0;
    hi = min_u64(hi, n - m + 1);
    if (lo >= hi)
        return 0;
    uint64_t end = hi + m - 1; /* exclusive bound on the window end; <= n */
    uint64_t i = lo + m - 1;
    while (i < end) {
        /* the B-character suffix of the window: t_{i-B+1} .. t_i */
        uint64_t hv = wm_hash(T + i - B + 1, B, w->bitshift);
        uint32_t sh = w->SHIFT[hv];
        if (sh > 0) {
            i += sh;
        } else {
            uint64_t start = i - m + 1;
            uint64_t hp = wm_hash(T + start, Bp, w->bitshift);
            for (uint32_t k = 0; k < w->nhash[hv]; k++) {
                uint32_t r = w->HASH[hv][k];
                if (w->PREFIX[r] == hp && memcmp(w->P + (uint64_t)r * m, T + start, m) == 0)
                    emit(&s, start, r);
            }
            i += 1;
        }
    }
    return s.count;
}
