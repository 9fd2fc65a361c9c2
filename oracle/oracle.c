/*
 * CPU oracle for exact multiple pattern matching.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or
 * call this file; it exists so that tests and the benchmark's CPU baseline can
 * check the GPU path against an independent, plainly written implementation.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Problem (paper, Section 1, Definition): given a text T = t_0..t_{n-1} and d
 * patterns p^0..p^{d-1}, report every pair (i, r) such that pattern r occurs
 * at i: t_{i+j} = p^r_j for every 0 <= j < |p^r| (the printed condition reads
 * "t_i = p^r_j"; the index i+j is the only reading under which it describes an
 * occurrence). The paper gives every pattern the same length m; the routines
 * below also take patterns of different lengths (pattern r is the byte range
 * [off[r], off[r+1]) of one array), with the equal-length entry points as the
 * special case off[r] = r * m. A start i needs i + |p^r| <= n.
 *
 * Every routine emits pairs in ascending (position, pattern id) order and can
 * be restricted to the starting positions [lo, hi), which is how the paper
 * splits a text between workers (Section 4.2.1 and the chunk-assignment
 * equation of Section 4.4: each worker reads up to (longest length - 1)
 * characters past its own range).
 *
 * Four implementations:
 *   orc_bf   - the definition, position by position and pattern by pattern.
 *   orc_win  - the definition at scale: for every starting position and every
 *              pattern length, the window is looked up in that length's sorted
 *              list of patterns (binary search). Exact.
 *   orc_ac_* - Aho-Corasick (Section 3.1, Algorithms 1-3): a goto function
 *              over all 256 byte values whose states are numbered in the
 *              order they are created while the patterns are inserted in id
 *              order; supply links found in breadth-first order from the
 *              longest-suffix rule of Section 3.1; the search follows supply
 *              links whenever a transition fails. With patterns of several
 *              lengths a state must also report the patterns that end at the
 *              states of its supply chain (a pattern can be a suffix of a
 *              longer path), so each state's output set is merged with its
 *              supply state's (the merge the paper's Algorithm 2 has no need
 *              for when all lengths are equal).
 *   orc_wm_* - Wu-Manber (Section 3.2, Algorithms 4-5): SHIFT/HASH/PREFIX
 *              over B-character blocks with the shift-and-add hash over byte
 *              values (B = 3, B' = 2, bitshift = 2 in the paper's experiments;
 *              all three are parameters here) and direct verification with
 *              memcmp. The window has the shortest pattern length, and the
 *              tables are built from every pattern's first (shortest length)
 *              characters; verification compares whole patterns.
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

/* A pattern set: pattern r is bytes[off[r] .. off[r+1]). */
typedef struct {
    uint8_t *bytes;
    uint64_t *off;
    uint32_t d;
    uint32_t shortest, longest;
} pset_t;

static uint32_t plen(const pset_t *ps, uint32_t r) { return (uint32_t)(ps->off[r + 1] - ps->off[r]); }
static const uint8_t *pat(const pset_t *ps, uint32_t r) { return ps->bytes + ps->off[r]; }

/* Copy a pattern set; returns 0 if a pattern is empty. */
static int pset_init(pset_t *ps, const uint8_t *P, const uint64_t *off, uint32_t d)
{
    uint64_t total = d ? off[d] : 0;
    ps->bytes = (uint8_t *)malloc(total + 1);
    ps->off = (uint64_t *)malloc(sizeof(uint64_t) * ((uint64_t)d + 1));
    if (total)
        memcpy(ps->bytes, P, total);
    ps->off[0] = 0;
    ps->d = d;
    ps->shortest = d ? 0xffffffffu : 0;
    ps->longest = 0;
    for (uint32_t r = 0; r < d; r++) {
        ps->off[r + 1] = off[r + 1] - off[0];
        uint32_t len = plen(ps, r);
        if (len == 0)
            return 0;
        if (len < ps->shortest)
            ps->shortest = len;
        if (len > ps->longest)
            ps->longest = len;
    }
    return 1;
}

static void pset_free(pset_t *ps)
{
    free(ps->bytes);
    free(ps->off);
}

/* Offsets of d patterns of length m each. */
static uint64_t *equal_offsets(uint32_t d, uint32_t m)
{
    uint64_t *off = (uint64_t *)malloc(sizeof(uint64_t) * ((uint64_t)d + 1));
    for (uint32_t r = 0; r <= d; r++)
        off[r] = (uint64_t)r * m;
    return off;
}

/* Pair order: ascending start, then id. */
typedef struct {
    uint64_t start;
    uint32_t id;
} hit_t;

static int cmp_hit(const void *a, const void *b)
{
    const hit_t *x = (const hit_t *)a, *y = (const hit_t *)b;
    if (x->start != y->start)
        return x->start < y->start ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* ------------------------------------------------------------------------ */
/* orc_bf: the definition, literally (Section 1).                           */
/* ------------------------------------------------------------------------ */
uint64_t orc_bf_v(const uint8_t *T, uint64_t n, const uint8_t *P, const uint64_t *off, uint32_t d,
                  uint64_t lo, uint64_t hi, uint32_t *pos, uint32_t *id, uint64_t cap)
{
    sink_t s = {pos, id, cap, 0};
    hi = min_u64(hi, n);
    for (uint64_t i = lo; i < hi; i++) {
        for (uint32_t r = 0; r < d; r++) {
            uint64_t len = off[r + 1] - off[r];
            if (len == 0 || i + len > n)
                continue;
            int all = 1;
            for (uint64_t j = 0; j < len; j++) {
                if (T[i + j] != P[off[r] + j]) {
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

uint64_t orc_bf(const uint8_t *T, uint64_t n, const uint8_t *P, uint32_t d, uint32_t m,
                uint64_t lo, uint64_t hi, uint32_t *pos, uint32_t *id, uint64_t cap)
{
    if (m == 0)
        return 0;
    uint64_t *off = equal_offsets(d, m);
    uint64_t c = orc_bf_v(T, n, P, off, d, lo, hi, pos, id, cap);
    free(off);
    return c;
}

/* ------------------------------------------------------------------------ */
/* orc_win: every window looked up in its length's sorted pattern list.     */
/* ------------------------------------------------------------------------ */
typedef struct {
    pset_t ps;
    uint32_t nlen;        /* distinct pattern lengths, ascending */
    uint32_t *lens;
    uint32_t **order;     /* per length: its pattern ids sorted by (bytes, id) */
    uint32_t *count;      /* per length: number of patterns */
} win_t;

static const pset_t *g_sort_ps; /* qsort has no context argument; builds are single-threaded */

static int cmp_ids(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    uint32_t len = plen(g_sort_ps, x); /* equal lengths within one list */
    int c = memcmp(pat(g_sort_ps, x), pat(g_sort_ps, y), len);
    if (c)
        return c;
    return (x > y) - (x < y);
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

void *orc_win_build_v(const uint8_t *P, const uint64_t *off, uint32_t d)
{
    win_t *w = (win_t *)calloc(1, sizeof(win_t));
    if (!pset_init(&w->ps, P, off, d)) {
        pset_free(&w->ps);
        free(w);
        return NULL;
    }
    /* distinct lengths */
    uint32_t *all = (uint32_t *)malloc(sizeof(uint32_t) * (d ? d : 1));
    for (uint32_t r = 0; r < d; r++)
        all[r] = plen(&w->ps, r);
    qsort(all, d, sizeof(uint32_t), cmp_u32);
    w->lens = (uint32_t *)malloc(sizeof(uint32_t) * (d ? d : 1));
    for (uint32_t r = 0; r < d; r++)
        if (r == 0 || all[r] != all[r - 1])
            w->lens[w->nlen++] = all[r];
    free(all);
    w->order = (uint32_t **)calloc(w->nlen ? w->nlen : 1, sizeof(uint32_t *));
    w->count = (uint32_t *)calloc(w->nlen ? w->nlen : 1, sizeof(uint32_t));
    for (uint32_t k = 0; k < w->nlen; k++) {
        w->order[k] = (uint32_t *)malloc(sizeof(uint32_t) * d);
        for (uint32_t r = 0; r < d; r++)
            if (plen(&w->ps, r) == w->lens[k])
                w->order[k][w->count[k]++] = r;
        g_sort_ps = &w->ps;
        qsort(w->order[k], w->count[k], sizeof(uint32_t), cmp_ids);
    }
    return w;
}

void *orc_win_build(const uint8_t *P, uint32_t d, uint32_t m)
{
    if (m == 0)
        return NULL;
    uint64_t *off = equal_offsets(d, m);
    void *w = orc_win_build_v(P, off, d);
    free(off);
    return w;
}

void orc_win_free(void *h)
{
    win_t *w = (win_t *)h;
    if (!w)
        return;
    for (uint32_t k = 0; k < w->nlen; k++)
        free(w->order[k]);
    free(w->order);
    free(w->count);
    free(w->lens);
    pset_free(&w->ps);
    free(w);
}

/* Thread-safe (read-only on the built structure). */
uint64_t orc_win_scan(const void *h, const uint8_t *T, uint64_t n, uint64_t lo,
                      uint64_t hi, uint32_t *pos, uint32_t *id, uint64_t cap)
{
    const win_t *w = (const win_t *)h;
    sink_t s = {pos, id, cap, 0};
    uint32_t ids_cap = 64, nids;
    uint32_t *ids = (uint32_t *)malloc(sizeof(uint32_t) * ids_cap);
    hi = min_u64(hi, n);
    for (uint64_t i = lo; i < hi; i++) {
        nids = 0;
        for (uint32_t k = 0; k < w->nlen; k++) {
            uint32_t len = w->lens[k];
            if (i + len > n)
                break;
            const uint8_t *win = T + i;
            const uint32_t *ord = w->order[k];
            /* first sorted entry whose pattern is >= the window */
            uint32_t a = 0, b = w->count[k];
            while (a < b) {
                uint32_t mid = a + (b - a) / 2;
                if (memcmp(pat(&w->ps, ord[mid]), win, len) < 0)
                    a = mid + 1;
                else
                    b = mid;
            }
            for (; a < w->count[k] && memcmp(pat(&w->ps, ord[a]), win, len) == 0; a++) {
                if (nids == ids_cap) {
                    ids_cap *= 2;
                    ids = (uint32_t *)realloc(ids, sizeof(uint32_t) * ids_cap);
                }
                ids[nids++] = ord[a];
            }
        }
        if (w->nlen > 1)
            qsort(ids, nids, sizeof(uint32_t), cmp_u32);
        for (uint32_t k = 0; k < nids; k++)
            emit(&s, i, ids[k]);
    }
    free(ids);
    return s.count;
}

/* ------------------------------------------------------------------------ */
/* orc_ac: Aho-Corasick, Section 3.1, Algorithms 1-3.                       */
/* ------------------------------------------------------------------------ */
#define AC_FAIL (-1)

typedef struct {
    uint32_t *v;
    uint32_t n, cap;
} idlist_t;

static void idlist_add(idlist_t *l, uint32_t r)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 2;
        l->v = (uint32_t *)realloc(l->v, sizeof(uint32_t) * l->cap);
    }
    l->v[l->n++] = r;
}

typedef struct {
    pset_t ps;
    uint64_t nstates, capstates;
    int32_t *g;         /* goto: nstates x 256, AC_FAIL where undefined */
    int32_t *supply;    /* supply (failure) state of each state */
    uint32_t *depth;    /* |L(q)| */
    idlist_t *own;      /* patterns whose path ends at q, ascending */
    idlist_t *out;      /* own(q) and the output of Supply(q): every pattern
                           that is a suffix of L(q), ascending */
} ac_t;

static uint64_t ac_add_state(ac_t *a, uint32_t depth)
{
    if (a->nstates == a->capstates) {
        uint64_t c = a->capstates ? 2 * a->capstates : 64;
        a->g = (int32_t *)realloc(a->g, c * 256 * sizeof(int32_t));
        a->supply = (int32_t *)realloc(a->supply, c * sizeof(int32_t));
        a->depth = (uint32_t *)realloc(a->depth, c * sizeof(uint32_t));
        a->own = (idlist_t *)realloc(a->own, c * sizeof(idlist_t));
        a->out = (idlist_t *)realloc(a->out, c * sizeof(idlist_t));
        a->capstates = c;
    }
    uint64_t q = a->nstates++;
    for (int c = 0; c < 256; c++)
        a->g[q * 256 + c] = AC_FAIL; /* no transitions yet */
    a->supply[q] = AC_FAIL;
    a->depth[q] = depth;
    memset(&a->own[q], 0, sizeof(idlist_t));
    memset(&a->out[q], 0, sizeof(idlist_t));
    return q;
}

/* Union of two ascending id lists, ascending. */
static void merge_into(idlist_t *dst, const idlist_t *x, const idlist_t *y)
{
    uint32_t i = 0, j = 0;
    while (i < x->n || j < y->n) {
        if (j == y->n || (i < x->n && x->v[i] < y->v[j]))
            idlist_add(dst, x->v[i++]);
        else if (i == x->n || y->v[j] < x->v[i])
            idlist_add(dst, y->v[j++]);
        else {
            idlist_add(dst, x->v[i++]);
            j++;
        }
    }
}

void *orc_ac_build_v(const uint8_t *P, const uint64_t *off, uint32_t d)
{
    ac_t *a = (ac_t *)calloc(1, sizeof(ac_t));
    if (!pset_init(&a->ps, P, off, d)) {
        pset_free(&a->ps);
        free(a);
        return NULL;
    }
    ac_add_state(a, 0); /* the initial state q0 */

    /* Goto function (Algorithm 1): each pattern, in id order, follows the
     * existing path of its longest prefix already in the trie and then adds
     * one new state per remaining character; the state where it ends gains
     * the pattern in its output set (also when the pattern added no state:
     * a duplicate, or a prefix of an earlier pattern). */
    for (uint32_t r = 0; r < d; r++) {
        const uint8_t *p = pat(&a->ps, r);
        uint32_t len = plen(&a->ps, r);
        uint64_t q = 0;
        for (uint32_t j = 0; j < len; j++) {
            int32_t next = a->g[q * 256 + p[j]];
            if (next == AC_FAIL) {
                next = (int32_t)ac_add_state(a, j + 1);
                a->g[q * 256 + p[j]] = next;
            }
            q = (uint64_t)next;
        }
        idlist_add(&a->own[q], r);
    }

    /* Supply function (Algorithm 2). At the root, characters without a
     * transition loop back to the root, and every child of the root has the
     * root as supply state. Deeper states are visited breadth first, so the
     * supply state of a state's parent is known when the state is reached:
     * the supply state of g(parent, c) is g(f, c) for the first state f on
     * the parent's supply chain that has a transition by c (the root always
     * has one). Output sets are merged along the same order. */
    uint64_t S = a->nstates;
    uint32_t *bfs = (uint32_t *)malloc(sizeof(uint32_t) * S);
    uint64_t head = 0, tail = 0;
    a->supply[0] = 0; /* the root's output set stays empty: no pattern is empty */
    for (int c = 0; c < 256; c++) {
        int32_t child = a->g[c];
        if (child == AC_FAIL) {
            a->g[c] = 0;
        } else {
            a->supply[child] = 0;
            bfs[tail++] = (uint32_t)child;
        }
    }
    while (head < tail) {
        uint32_t q = bfs[head++];
        /* q's supply state was set when q was queued: finish its output */
        merge_into(&a->out[q], &a->own[q], &a->out[a->supply[q]]);
        for (int c = 0; c < 256; c++) {
            int32_t child = a->g[(uint64_t)q * 256 + c];
            if (child == AC_FAIL)
                continue;
            int32_t f = a->supply[q];
            while (a->g[(uint64_t)f * 256 + c] == AC_FAIL)
                f = a->supply[f];
            a->supply[child] = a->g[(uint64_t)f * 256 + c];
            bfs[tail++] = (uint32_t)child;
        }
    }
    free(bfs);
    return a;
}

void *orc_ac_build(const uint8_t *P, uint32_t d, uint32_t m)
{
    if (m == 0)
        return NULL;
    uint64_t *off = equal_offsets(d, m);
    void *a = orc_ac_build_v(P, off, d);
    free(off);
    return a;
}

void orc_ac_free(void *h)
{
    ac_t *a = (ac_t *)h;
    if (!a)
        return;
    for (uint64_t q = 0; q < a->nstates; q++) {
        free(a->own[q].v);
        free(a->out[q].v);
    }
    free(a->g);
    free(a->supply);
    free(a->depth);
    free(a->own);
    free(a->out);
    pset_free(&a->ps);
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
/* Patterns whose own path ends at q. */
uint32_t orc_ac_nout(const void *h, uint64_t q) { return ((const ac_t *)h)->own[q].n; }
uint32_t orc_ac_out(const void *h, uint64_t q, uint32_t k) { return ((const ac_t *)h)->own[q].v[k]; }
/* Merged output set of q (every pattern that is a suffix of L(q)). */
uint32_t orc_ac_nout_all(const void *h, uint64_t q) { return ((const ac_t *)h)->out[q].n; }
uint32_t orc_ac_out_all(const void *h, uint64_t q, uint32_t k) { return ((const ac_t *)h)->out[q].v[k]; }

/* One character of the search (Algorithm 3): follow supply links while the
 * goto function fails, then take the transition. */
static int64_t ac_step(const ac_t *a, int64_t q, uint8_t c)
{
    while (a->g[q * 256 + c] == AC_FAIL)
        q = a->supply[q];
    return a->g[q * 256 + c];
}

/* Algorithm 3 over the start positions [lo, hi): the walk begins in q0 at lo
 * and reads up to (longest length - 1) characters past hi (the overlap of
 * Section 4.2.1). After character e, every pattern r in the state's merged
 * output set ends at e and starts at e - |p^r| + 1; starts inside [lo, hi)
 * are reported. Reports come in order of their end; they are sorted by
 * (start, id) before being emitted. Thread-safe. */
uint64_t orc_ac_scan(const void *h, const uint8_t *T, uint64_t n, uint64_t lo,
                     uint64_t hi, uint32_t *pos, uint32_t *id, uint64_t cap)
{
    const ac_t *a = (const ac_t *)h;
    sink_t s = {pos, id, cap, 0};
    hi = min_u64(hi, n);
    if (lo >= hi || a->ps.d == 0)
        return 0;
    uint64_t stop = min_u64(hi + a->ps.longest - 1, n);
    uint64_t nh = 0, caph = 1024;
    hit_t *hits = (hit_t *)malloc(sizeof(hit_t) * caph);
    int64_t q = 0;
    for (uint64_t e = lo; e < stop; e++) {
        q = ac_step(a, q, T[e]);
        const idlist_t *o = &a->out[q];
        for (uint32_t k = 0; k < o->n; k++) {
            uint32_t r = o->v[k];
            uint64_t start = e + 1 - plen(&a->ps, r);
            if (start < hi) {  /* start >= lo: the walk began at lo */
                if (nh == caph) {
                    caph *= 2;
                    hits = (hit_t *)realloc(hits, sizeof(hit_t) * caph);
                }
                hits[nh].start = start;
                hits[nh].id = r;
                nh++;
            }
        }
    }
    if (a->ps.shortest != a->ps.longest)
        qsort(hits, nh, sizeof(hit_t), cmp_hit);
    for (uint64_t k = 0; k < nh; k++)
        emit(&s, hits[k].start, hits[k].id);
    free(hits);
    return s.count;
}

/* The state after each character (for checking the longest-suffix
 * characterisation of Section 3.1). states[i - lo] for i in [lo, hi). */
void orc_ac_trace(const void *h, const uint8_t *T, uint64_t lo, uint64_t hi, int32_t *states)
{
    const ac_t *a = (const ac_t *)h;
    int64_t q = 0;
    for (uint64_t i = lo; i < hi; i++) {
        q = ac_step(a, q, T[i]);
        states[i - lo] = (int32_t)q;
    }
}

/* ------------------------------------------------------------------------ */
/* orc_wm: Wu-Manber, Section 3.2, Algorithms 4-5.                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    pset_t ps;
    uint32_t w;          /* window length: the shortest pattern length */
    uint32_t B, Bp, bitshift;
    uint64_t tsize;      /* SHIFT/HASH table size: sum_{i<B} 256 * (2^bitshift)^i */
    uint32_t *SHIFT;
    idlist_t *HASH;      /* per block hash: ascending pattern ids */
    uint64_t *PREFIX;    /* h2 of each pattern's first B' characters */
} wm_t;

/* Shift-and-add hash over byte values: shift left by bitshift, add the byte. */
static uint64_t shift_add(const uint8_t *c, uint32_t len, uint32_t bitshift)
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

/* Returns NULL when the shortest pattern is shorter than B or B' (SHIFT
 * starts at w - B + 1 >= 1, Algorithm 4). */
void *orc_wm_build_v(const uint8_t *P, const uint64_t *off, uint32_t d, uint32_t B, uint32_t Bp,
                     uint32_t bitshift)
{
    if (B == 0 || Bp == 0 || bitshift > 8 || B > 6 || Bp > 6)
        return NULL;
    wm_t *t = (wm_t *)calloc(1, sizeof(wm_t));
    if (!pset_init(&t->ps, P, off, d) || (d && (t->ps.shortest < B || t->ps.shortest < Bp))) {
        pset_free(&t->ps);
        free(t);
        return NULL;
    }
    const uint32_t w = t->ps.shortest;
    t->w = w;
    t->B = B;
    t->Bp = Bp;
    t->bitshift = bitshift;
    t->tsize = orc_wm_table_size(B, bitshift);
    t->SHIFT = (uint32_t *)malloc(sizeof(uint32_t) * t->tsize);
    t->HASH = (idlist_t *)calloc(t->tsize, sizeof(idlist_t));
    t->PREFIX = (uint64_t *)calloc(d ? d : 1, sizeof(uint64_t));

    /* SHIFT (Algorithm 4): a block that occurs in no pattern's first w
     * characters allows the largest shift, w - B + 1; otherwise the shift is
     * the distance from the block's rightmost occurrence, over all patterns,
     * to the end of those w characters. */
    for (uint64_t hv = 0; hv < t->tsize; hv++)
        t->SHIFT[hv] = w - B + 1;
    for (uint32_t r = 0; r < d; r++) {
        const uint8_t *p = pat(&t->ps, r);
        for (uint32_t end = B; end <= w; end++) { /* block p[end-B .. end) */
            uint64_t hv = shift_add(p + end - B, B, bitshift);
            if (w - end < t->SHIFT[hv])
                t->SHIFT[hv] = w - end;
        }
        /* HASH lists every pattern under the hash of its block that ends the
         * window (ids ascending); PREFIX keeps the hash of its first B'. */
        idlist_add(&t->HASH[shift_add(p + w - B, B, bitshift)], r);
        t->PREFIX[r] = shift_add(p, Bp, bitshift);
    }
    return t;
}

void *orc_wm_build(const uint8_t *P, uint32_t d, uint32_t m, uint32_t B, uint32_t Bp,
                   uint32_t bitshift)
{
    if (m == 0)
        return NULL;
    uint64_t *off = equal_offsets(d, m);
    void *t = orc_wm_build_v(P, off, d, B, Bp, bitshift);
    free(off);
    return t;
}

void orc_wm_free(void *h)
{
    wm_t *t = (wm_t *)h;
    if (!t)
        return;
    for (uint64_t hv = 0; hv < t->tsize; hv++)
        free(t->HASH[hv].v);
    free(t->HASH);
    free(t->SHIFT);
    free(t->PREFIX);
    pset_free(&t->ps);
    free(t);
}

uint64_t orc_wm_tsize(const void *h) { return ((const wm_t *)h)->tsize; }
uint32_t orc_wm_shift(const void *h, uint64_t hv) { return ((const wm_t *)h)->SHIFT[hv]; }
uint32_t orc_wm_nhash(const void *h, uint64_t hv) { return ((const wm_t *)h)->HASH[hv].n; }
uint32_t orc_wm_hash_entry(const void *h, uint64_t hv, uint32_t k) { return ((const wm_t *)h)->HASH[hv].v[k]; }
uint64_t orc_wm_prefix(const void *h, uint32_t r) { return ((const wm_t *)h)->PREFIX[r]; }

/* Algorithm 5 over the start positions [lo, hi): the window of w characters
 * starts at lo; the block of B characters that ends it (t_{e-B+1} .. t_e for
 * the window end e) selects SHIFT; a positive shift moves the window right
 * by that much, a zero shift checks the HASH list of the block (ids
 * ascending) against the window: PREFIX first, then the whole pattern with
 * memcmp where it fits in the text; then the window moves by one. Windows
 * start in increasing order, so the pairs come out sorted. Thread-safe. */
uint64_t orc_wm_scan(const void *h, const uint8_t *T, uint64_t n, uint64_t lo,
                     uint64_t hi, uint32_t *pos, uint32_t *id, uint64_t cap)
{
    const wm_t *t = (const wm_t *)h;
    sink_t s = {pos, id, cap, 0};
    const uint32_t w = t->w;
    if (t->ps.d == 0 || n < w)
        return 0;
    hi = min_u64(hi, n - w + 1);
    uint64_t start = lo;
    while (start < hi) {
        uint64_t e = start + w - 1; /* the window's last character */
        uint64_t hv = shift_add(T + e + 1 - t->B, t->B, t->bitshift);
        uint32_t sh = t->SHIFT[hv];
        if (sh > 0) {
            start += sh;
            continue;
        }
        uint64_t hp = shift_add(T + start, t->Bp, t->bitshift);
        const idlist_t *cand = &t->HASH[hv];
        for (uint32_t k = 0; k < cand->n; k++) {
            uint32_t r = cand->v[k];
            uint32_t len = plen(&t->ps, r);
            if (t->PREFIX[r] == hp && start + len <= n && memcmp(pat(&t->ps, r), T + start, len) == 0)
                emit(&s, start, r);
        }
        start += 1;
    }
    return s.count;
}
