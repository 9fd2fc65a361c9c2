// Host side of the library: index builders, device-image packing and the
// C-ABI entry points declared in include/mpm.h.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <numeric>
#include <tuple>
#include <vector>

#include "mpm_internal.h"

namespace mpm {

static thread_local std::string g_err;

void set_error(const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

mpm_status fail(mpm_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

static uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// Distinct pattern strings
// ---------------------------------------------------------------------------
// Number the distinct strings by their number of ids (ascending), each
// group in ascending string order: strings u < n_single stand for exactly
// one id, and within a group of strings with c ids the id list of u starts
// at group_off + (u - group_start) * c, so the scan counts and finds a
// string's ids without reading the CSR offsets.
static mpm_status number_by_count(mpm_index *ix)
{
    const uint32_t m = ix->m;
    auto str_begin = [&](uint32_t u) -> uint64_t { return ix->var ? ix->upoff[u] : (uint64_t)u * m; };
    auto str_end = [&](uint32_t u) -> uint64_t { return ix->var ? ix->upoff[u + 1] : (uint64_t)(u + 1) * m; };
    std::vector<uint32_t> perm(ix->du);
    std::iota(perm.begin(), perm.end(), 0u);
    std::stable_sort(perm.begin(), perm.end(), [&](uint32_t a, uint32_t b) {
        return ix->uoff[a + 1] - ix->uoff[a] < ix->uoff[b + 1] - ix->uoff[b];
    });
    ix->n_single = 0;
    while (ix->n_single < ix->du &&
           ix->uoff[perm[ix->n_single] + 1] - ix->uoff[perm[ix->n_single]] == 1)
        ix->n_single++;
    if (ix->n_single < ix->du) {
        std::vector<uint32_t> uoff2(1, 0), uids2, upoff2(1, 0);
        std::vector<uint8_t> upats2;
        uids2.reserve(ix->uids.size());
        upats2.reserve(ix->upats.size());
        for (uint32_t u : perm) {
            for (uint32_t j = ix->uoff[u]; j < ix->uoff[u + 1]; j++)
                uids2.push_back(ix->uids[j]);
            uoff2.push_back((uint32_t)uids2.size());
            upats2.insert(upats2.end(), ix->upats.begin() + str_begin(u), ix->upats.begin() + str_end(u));
            upoff2.push_back((uint32_t)upats2.size());
        }
        ix->uoff.swap(uoff2);
        ix->uids.swap(uids2);
        ix->upats.swap(upats2);
        if (ix->var)
            ix->upoff.swap(upoff2);
    }
    // groups of strings sharing an id count above one
    ix->grp_u0.clear();
    ix->grp_cnt.clear();
    ix->grp_off.clear();
    for (uint32_t u = ix->n_single; u < ix->du; u++) {
        const uint32_t c = ix->uoff[u + 1] - ix->uoff[u];
        if (ix->grp_cnt.empty() || ix->grp_cnt.back() != c) {
            ix->grp_u0.push_back(u);
            ix->grp_cnt.push_back(c);
            ix->grp_off.push_back(ix->uoff[u]);
        }
    }
    return MPM_OK;
}

// The Definition reports every pattern id, so equal patterns are kept as one
// string with an ascending id list (the output set of a terminal state in
// Algorithm 1 holds every pattern that ends there).
static mpm_status dedup(const uint8_t *P, uint32_t d, uint32_t m, mpm_index *ix)
{
    std::vector<uint32_t> order(d);
    std::iota(order.begin(), order.end(), 0u);
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        int c = memcmp(P + (uint64_t)a * m, P + (uint64_t)b * m, m);
        return c != 0 ? c < 0 : a < b;
    });
    ix->uoff.clear();
    ix->uids.resize(d);
    ix->upats.clear();
    ix->max_dup = 0;
    uint32_t run = 0;
    for (uint32_t k = 0; k < d; k++) {
        const uint8_t *p = P + (uint64_t)order[k] * m;
        bool fresh = k == 0 || memcmp(p, P + (uint64_t)order[k - 1] * m, m) != 0;
        if (fresh) {
            if (k)
                ix->max_dup = std::max(ix->max_dup, run);
            run = 0;
            ix->uoff.push_back(k);
            ix->upats.insert(ix->upats.end(), p, p + m);
        }
        ix->uids[k] = order[k];
        run++;
    }
    ix->max_dup = std::max(ix->max_dup, run);
    ix->uoff.push_back(d);
    ix->du = (uint32_t)(ix->uoff.size() - 1);
    return number_by_count(ix);
}

// Patterns of different lengths (pattern r is P[off[r] .. off[r + 1])): the
// Definition read with a length per pattern. Wherever a distinct string
// occurs, so does every pattern that is a prefix of it, so each distinct
// string keeps the ascending ids of all of them; a scan reports, per start,
// only the longest distinct string found there. In sorted order a string's
// prefixes in the set are the chain kept on a stack, and its list is its
// longest proper prefix's list merged with its own ids.
static mpm_status dedup_var(const uint8_t *P, const uint64_t *off, uint32_t d, mpm_index *ix)
{
    auto len = [&](uint32_t r) { return off[r + 1] - off[r]; };
    auto cmp = [&](uint32_t a, uint32_t b) -> int {
        const uint64_t la = len(a), lb = len(b);
        const int c = memcmp(P + off[a], P + off[b], std::min(la, lb));
        if (c)
            return c;
        return la < lb ? -1 : la > lb ? 1 : 0;  // a proper prefix sorts first
    };
    std::vector<uint32_t> order(d);
    std::iota(order.begin(), order.end(), 0u);
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        const int c = cmp(a, b);
        return c != 0 ? c < 0 : a < b;
    });
    // distinct strings and their own ids
    std::vector<uint32_t> own_off, own_ids(d);
    ix->upats.clear();
    ix->upoff.assign(1, 0);
    for (uint32_t k = 0; k < d; k++) {
        const uint32_t r = order[k];
        if (k == 0 || cmp(r, order[k - 1]) != 0) {
            own_off.push_back(k);
            if (ix->upats.size() + len(r) >= (1ull << 32))
                return fail(MPM_ETOOBIG, "build: distinct pattern bytes exceed 4 GiB");
            ix->upats.insert(ix->upats.end(), P + off[r], P + off[r + 1]);
            ix->upoff.push_back((uint32_t)ix->upats.size());
        }
        own_ids[k] = r;
    }
    own_off.push_back(d);
    ix->du = (uint32_t)(own_off.size() - 1);
    auto is_prefix = [&](uint32_t v, uint32_t u) {  // distinct string v a prefix of u
        const uint32_t lv = ix->upoff[v + 1] - ix->upoff[v], lu = ix->upoff[u + 1] - ix->upoff[u];
        return lv <= lu && memcmp(ix->upats.data() + ix->upoff[v], ix->upats.data() + ix->upoff[u], lv) == 0;
    };
    ix->uoff.assign(1, 0);
    ix->uids.clear();
    ix->max_dup = 0;
    std::vector<uint32_t> chain;
    for (uint32_t u = 0; u < ix->du; u++) {
        while (!chain.empty() && !is_prefix(chain.back(), u))
            chain.pop_back();
        const uint32_t *ob = own_ids.data() + own_off[u], *oe = own_ids.data() + own_off[u + 1];
        std::sort(own_ids.begin() + own_off[u], own_ids.begin() + own_off[u + 1]);
        const uint64_t base = ix->uids.size();
        if (chain.empty()) {
            ix->uids.insert(ix->uids.end(), ob, oe);
        } else {
            const uint32_t v = chain.back();
            const uint64_t pb = ix->uoff[v], pe = ix->uoff[v + 1];
            if (base + (pe - pb) + (oe - ob) >= (1ull << 31))
                return fail(MPM_ETOOBIG, "build: id lists of prefix patterns exceed 2^31 entries");
            ix->uids.resize(base + (pe - pb) + (oe - ob));
            // the prefix's list lives in uids too: merge from a copy
            std::vector<uint32_t> pre(ix->uids.begin() + pb, ix->uids.begin() + pe);
            std::merge(pre.begin(), pre.end(), ob, oe, ix->uids.begin() + base);
        }
        ix->uoff.push_back((uint32_t)ix->uids.size());
        ix->max_dup = std::max<uint32_t>(ix->max_dup, (uint32_t)(ix->uids.size() - base));
        chain.push_back(u);
    }
    return number_by_count(ix);
}

template <typename T>
static uint64_t put(std::vector<uint8_t> &img, const T *src, uint64_t count)
{
    uint64_t off = align_up(img.size(), 256);
    uint64_t bytes = count * sizeof(T);
    img.resize(align_up(off + bytes, 16), 0);
    if (bytes)
        memcpy(img.data() + off, src, bytes);
    return off;
}

// ---------------------------------------------------------------------------
// Aho-Corasick: trie (Algorithm 1), supply links in breadth-first order
// (Algorithm 2), flattened transition table.
// ---------------------------------------------------------------------------
static mpm_status build_ac_tables(mpm_index *ix)
{
    const uint32_t m = ix->m, du = ix->du;
    // Symbol classes: the distinct bytes of the patterns, ascending.
    bool present[256] = {false};
    for (uint8_t b : ix->upats)
        present[b] = true;
    uint32_t C = 0;
    memset(ix->cls, 0, sizeof ix->cls);
    for (int b = 0; b < 256; b++)
        if (present[b]) {
            ix->class_bytes[C] = (uint8_t)b;
            ix->cls[b] = (uint16_t)(C + 1);
            C++;
        }
    ix->n_classes = C;
    const uint32_t cp = C + 1;

    uint64_t max_nodes = (uint64_t)m * du + 1;
    if (max_nodes > (1ull << 31))
        return fail(MPM_ETOOBIG, "build_ac: up to %llu states exceed 2^31",
                    (unsigned long long)max_nodes);

    // Trie over the distinct strings in ascending order; nodes numbered in
    // creation order (Algorithm 1).
    std::vector<int32_t> child;
    std::vector<uint32_t> depth;
    std::vector<uint32_t> term(du);  // the depth-m state of each distinct string
    child.reserve(std::min<uint64_t>(max_nodes, 1u << 22) * C);
    child.assign(C, -1);
    depth.push_back(0);
    for (uint32_t u = 0; u < du; u++) {
        const uint8_t *p = ix->upats.data() + (uint64_t)u * m;
        int64_t q = 0;
        for (uint32_t j = 0; j < m; j++) {
            uint32_t c = ix->cls[p[j]] - 1;
            int32_t nx = child[q * C + c];
            if (nx < 0) {
                nx = (int32_t)depth.size();
                child[q * C + c] = nx;
                child.resize(child.size() + C, -1);
                depth.push_back(j + 1);
            }
            q = nx;
        }
        term[u] = (uint32_t)q;
    }
    const uint64_t S = depth.size();

    // Breadth-first order; children visited in ascending byte order, so each
    // depth level is in lexicographic order of the state labels.
    std::vector<uint32_t> order;
    order.reserve(S);
    order.push_back(0);
    for (uint64_t h = 0; h < order.size(); h++) {
        uint32_t v = order[h];
        for (uint32_t c = 0; c < C; c++) {
            int32_t w = child[(uint64_t)v * C + c];
            if (w >= 0)
                order.push_back((uint32_t)w);
        }
    }
    // The deepest level comes last in breadth-first order; number it in the
    // order of the distinct strings, so that state first_term + u is string u.
    for (uint32_t u = 0; u < du; u++)
        order[S - du + u] = term[u];
    std::vector<uint32_t> newid(S);
    for (uint64_t k = 0; k < S; k++)
        newid[order[k]] = (uint32_t)k;

    // Supply (failure) links in breadth-first order (Algorithm 2): the supply
    // state of w = g(v, c) is g(f, c) for the first f on v's supply chain
    // that has a c-transition, else the root.
    std::vector<uint32_t> supply(S, 0);
    for (uint64_t h = 0; h < S; h++) {
        uint32_t v = order[h];
        for (uint32_t c = 0; c < C; c++) {
            int32_t w = child[(uint64_t)v * C + c];
            if (w < 0)
                continue;
            if (v == 0) {
                supply[w] = 0;
                continue;
            }
            uint32_t f = supply[v];
            while (f != 0 && child[(uint64_t)f * C + c] < 0)
                f = supply[f];
            int32_t g = child[(uint64_t)f * C + c];
            supply[w] = g >= 0 ? (uint32_t)g : 0;
        }
    }

    // Flatten: delta(v, c) = g(v, c) if defined, else delta(supply(v), c),
    // and the root's undefined transitions stay at the root. Supply states
    // are shallower, so breadth-first order has them complete already.
    std::vector<uint32_t> delta(S * C);
    for (uint64_t h = 0; h < S; h++) {
        uint32_t v = order[h];
        for (uint32_t c = 0; c < C; c++) {
            int32_t w = child[(uint64_t)v * C + c];
            if (w >= 0)
                delta[(uint64_t)v * C + c] = (uint32_t)w;
            else
                delta[(uint64_t)v * C + c] = v == 0 ? 0 : delta[(uint64_t)supply[v] * C + c];
        }
    }

    // Table in breadth-first numbering with the "other byte" column 0.
    ix->n_states = S;
    ix->dfa.assign(S * cp, 0);
    for (uint64_t k = 0; k < S; k++) {
        uint32_t v = order[k];
        for (uint32_t c = 0; c < C; c++)
            ix->dfa[k * cp + 1 + c] = newid[delta[(uint64_t)v * C + c]];
    }
    // The deepest level holds exactly the distinct strings, in order.
    uint64_t first_term = S - du;
    for (uint64_t k = 0; k < S; k++) {
        bool term = depth[order[k]] == m;
        if (term != (k >= first_term))
            return fail(MPM_EINVAL, "build_ac: internal error (terminal block)");
    }
    ix->state_bytes = S <= 65535 ? 2 : 4;
    if (S * cp * ix->state_bytes >= (1ull << 32))
        return fail(MPM_ETOOBIG, "build_ac: table of %llu states x %u columns exceeds 4 GiB",
                    (unsigned long long)S, cp);

    // Device image: table, class map, distinct-string CSR.
    ix->image.clear();
    if (ix->state_bytes == 2) {
        std::vector<uint16_t> t16(ix->dfa.begin(), ix->dfa.end());
        ix->off_a = put(ix->image, t16.data(), t16.size());
    } else {
        ix->off_a = put(ix->image, ix->dfa.data(), ix->dfa.size());
    }
    ix->table_bytes = align_up(S * cp * ix->state_bytes, 16);
    // Column byte offsets per byte value, and the table-free class codes.
    uint16_t cls_off[256];
    for (int b = 0; b < 256; b++)
        cls_off[b] = (uint16_t)(ix->cls[b] * ix->state_bytes);
    ix->off_b = put(ix->image, cls_off, 256);
    ix->swar_ok = 0;
    if (C <= 7 && ix->state_bytes * C <= 255) {
        for (uint32_t sh = 0; sh < 6 && !ix->swar_ok; sh++) {
            int owner[8];
            for (int k = 0; k < 8; k++)
                owner[k] = -1;
            bool ok = true;
            for (uint32_t c = 0; c < C && ok; c++) {
                int code = (ix->class_bytes[c] >> sh) & 7;
                if (owner[code] >= 0)
                    ok = false;
                owner[code] = (int)c;
            }
            if (!ok)
                continue;
            ix->swar_ok = 1;
            ix->swar_shift = sh;
            for (int k = 0; k < 8; k++) {
                if (owner[k] >= 0) {
                    ix->perm_byte[k] = ix->class_bytes[owner[k]];
                    ix->perm_col[k] = (uint8_t)((owner[k] + 1) * ix->state_bytes);
                } else {
                    // A code of no pattern byte goes to column 0 whatever the
                    // byte; its expected byte only decides whether the kernel
                    // can skip the exact per-byte test, so pick a likely
                    // separator byte with this code when there is one.
                    static const uint8_t likely[] = {'\n', 'N', '\r', ' ', 'n', '>', '\t', '-', 0};
                    ix->perm_byte[k] = (uint8_t)(((k + 1) & 7) << sh);  // has another code
                    for (uint8_t b : likely)
                        if (((b >> sh) & 7) == (uint32_t)k && !present[b]) {
                            ix->perm_byte[k] = b;
                            break;
                        }
                    ix->perm_col[k] = 0;
                }
            }
        }
    }
    ix->off_c = put(ix->image, ix->uoff.data(), ix->uoff.size());
    ix->off_d = put(ix->image, ix->uids.data(), ix->uids.size());
    if (ix->keep_goto) {
        // Goto rows in the table's numbering and columns: a missing
        // transition is all ones, except at the root, where it stays at the
        // root (column 0, bytes of no pattern, included); then the supply
        // link of every state.
        const uint32_t fail_id = ix->state_bytes == 2 ? 0xffffu : 0xffffffffu;
        std::vector<uint32_t> go(S * cp), sup(S);
        for (uint64_t k = 0; k < S; k++) {
            const uint32_t v = order[k];
            go[k * cp] = v == 0 ? 0u : fail_id;
            for (uint32_t c = 0; c < C; c++) {
                const int32_t w = child[(uint64_t)v * C + c];
                go[k * cp + 1 + c] = w >= 0 ? newid[w] : (v == 0 ? 0u : fail_id);
            }
            sup[k] = newid[supply[v]];
        }
        if (ix->state_bytes == 2) {
            std::vector<uint16_t> g16(go.begin(), go.end()), s16(sup.begin(), sup.end());
            ix->off_go = put(ix->image, g16.data(), g16.size());
            ix->sup_off = put(ix->image, s16.data(), s16.size()) - ix->off_go;
        } else {
            ix->off_go = put(ix->image, go.data(), go.size());
            ix->sup_off = put(ix->image, sup.data(), sup.size()) - ix->off_go;
        }
        ix->go_bytes = align_up(ix->image.size() - ix->off_go, 16);
    }
    ix->image.resize(align_up(ix->image.size(), 256), 0);
    return MPM_OK;
}

// ---------------------------------------------------------------------------
// Wu-Manber tables (Algorithm 4) over 2-bit character codes.
// ---------------------------------------------------------------------------
static inline uint32_t wm_code(uint8_t c, uint32_t sh) { return (c >> sh) & 3u; }

static inline uint32_t wm_block_hash(const uint8_t *p, uint32_t B, uint32_t sh)
{
    uint32_t h = 0;
    for (uint32_t k = 0; k < B; k++)
        h |= wm_code(p[k], sh) << (2 * k);
    return h;
}

// The first m bytes of every distinct string, m bytes each: the strings
// themselves for one length, their window prefixes for several.
static const uint8_t *wm_windows(const mpm_index *ix)
{
    return ix->var ? ix->wpats.data() : ix->upats.data();
}

static void wm_tables(const mpm_index *ix, uint32_t B, uint32_t sh, std::vector<uint8_t> &shift,
                      std::vector<uint32_t> &bcount)
{
    const uint32_t m = ix->m;
    const uint32_t H = 1u << (2 * B);
    shift.assign(H, (uint8_t)(m - B + 1));
    bcount.assign(H, 0);
    const uint8_t *win = wm_windows(ix);
    for (uint32_t u = 0; u < ix->du; u++) {
        const uint8_t *p = win + (uint64_t)u * m;
        for (uint32_t q = B; q <= m; q++) {
            // the block p_{q-B} .. p_{q-1}, m - q characters from the end
            uint32_t h = wm_block_hash(p + q - B, B, sh);
            uint8_t s = (uint8_t)(m - q);
            if (s < shift[h])
                shift[h] = s;
            if (q == m)
                bcount[h]++;
        }
    }
}

static double wm_cost(const std::vector<uint8_t> &shift, const std::vector<uint32_t> &bcount,
                      uint32_t /*B*/)
{
    // Expected work per text byte for uniformly random block codes: windows
    // visited per byte (1 / mean advance) times work per window. The scan
    // reads each block hash out of a register history, so a window costs the
    // same for every B; a zero shift adds the bucket walk.
    double adv = 0, work = 0;
    const double H = (double)shift.size();
    for (size_t h = 0; h < shift.size(); h++) {
        adv += shift[h] ? shift[h] : 1;
        work += 1.0 + (shift[h] == 0 ? 1.0 + 0.5 * bcount[h] : 0.0);
    }
    adv /= H;
    work /= H;
    return work / adv;
}

static mpm_status build_wm_tables(mpm_index *ix, uint32_t B_req)
{
    const uint32_t m = ix->m;
    // Character code shift: the one under which two random pattern
    // characters collide least often (sum over codes of the squared share of
    // pattern characters with that code), so frequent bytes get codes of
    // their own.
    double freq[256] = {0};
    const uint8_t *win = wm_windows(ix);
    for (uint64_t k = 0; k < (uint64_t)ix->du * m; k++)
        freq[win[k]] += 1.0;
    uint32_t best_sh = 0;
    double best_c = 1e300;
    for (uint32_t sh = 0; sh < 6; sh++) {
        double mass[4] = {0, 0, 0, 0};
        for (int b = 0; b < 256; b++)
            mass[wm_code((uint8_t)b, sh)] += freq[b];
        const double c = mass[0] * mass[0] + mass[1] * mass[1] + mass[2] * mass[2] + mass[3] * mass[3];
        if (c < best_c * (1 - 1e-12)) {
            best_c = c;
            best_sh = sh;
        }
    }
    ix->code_shift = best_sh;
    // Zero-shift hashes carry a 15-bit bucket number, so B = 8 is used only
    // when fewer than 2^15 distinct strings exist.
    const uint32_t Bmax = std::min<uint32_t>(std::min<uint32_t>(m, 8), ix->du < 32768 ? 8 : 7);
    if (B_req > Bmax)
        return fail(MPM_EUNSUPPORTED, "mpm_build_wm: B=%u exceeds %u for m=%u, %u strings", B_req,
                    Bmax, m, ix->du);
    std::vector<uint8_t> shift;
    std::vector<uint32_t> bcount;
    uint32_t B = B_req;
    if (B == 0) {
        double best = 1e300;
        for (uint32_t b = 1; b <= Bmax; b++) {
            wm_tables(ix, b, best_sh, shift, bcount);
            double c = wm_cost(shift, bcount, b);
            if (c < best * 0.999) {
                best = c;
                B = b;
            }
        }
    }
    ix->B = B;
    wm_tables(ix, B, best_sh, shift, bcount);
    const uint32_t H = 1u << (2 * B);
    ix->shift = shift;
    // Buckets: one per zero-shift hash, in hash order; entries are the
    // distinct strings (ascending) whose last block hashes there.
    std::vector<uint32_t> bucket_of(H, 0xffffffffu);
    uint32_t nb = 0;
    for (uint32_t h = 0; h < H; h++)
        if (shift[h] == 0)
            bucket_of[h] = nb++;
    ix->shift16.assign(H, 0);
    for (uint32_t h = 0; h < H; h++)
        ix->shift16[h] = shift[h] ? (uint16_t)shift[h] : (uint16_t)(0x8000u | bucket_of[h]);
    ix->boff.assign(nb + 1, 0);
    for (uint32_t h = 0; h < H; h++)
        if (shift[h] == 0)
            ix->boff[bucket_of[h] + 1] = bcount[h];
    for (uint32_t b = 0; b < nb; b++)
        ix->boff[b + 1] += ix->boff[b];
    // Filter key: codes of the characters just before the last block, first
    // character in the low bits. The scan reads block and key from a 32-
    // character history in which a window ends at most 16 characters before
    // its end, so B + key_len <= 17.
    const uint32_t kl = std::min<uint32_t>(std::min<uint32_t>(16, m - B), 17 - B);
    ix->key_len = kl;
    ix->bu.assign(ix->du, 0);
    ix->bkey.assign(ix->du, 0);
    std::vector<uint32_t> fillp(ix->boff.begin(), ix->boff.end() - 1);
    // Ascending ranks within a bucket; for several lengths, longer strings
    // first, so that the first string found at a window is the longest one
    // starting there.
    std::vector<uint32_t> fill_order(ix->du);
    std::iota(fill_order.begin(), fill_order.end(), 0u);
    if (ix->var)
        std::stable_sort(fill_order.begin(), fill_order.end(), [&](uint32_t a, uint32_t b) {
            return ix->upoff[a + 1] - ix->upoff[a] > ix->upoff[b + 1] - ix->upoff[b];
        });
    for (uint32_t u : fill_order) {
        const uint8_t *p = win + (uint64_t)u * m;
        uint32_t h = wm_block_hash(p + m - B, B, best_sh);
        uint32_t slot = fillp[bucket_of[h]]++;
        ix->bu[slot] = u;
        ix->bkey[slot] = kl ? wm_block_hash(p + m - B - kl, kl, best_sh) : 0;
    }
    double sum = 0;
    uint32_t zeros = 0;
    for (uint8_t sv : shift) {
        sum += sv;
        zeros += sv == 0;
    }
    ix->mean_shift = sum / H;
    ix->zero_shift = zeros;
    ix->n_buckets = nb;

    // Device image: SHIFT (u16) | bucket offsets | keys | ranks, then the
    // distinct strings and the id CSR. The first four are what the window
    // loop reads and what LDS placement copies.
    ix->image.clear();
    ix->off_a = put(ix->image, ix->shift16.data(), ix->shift16.size());
    ix->off_b = put(ix->image, ix->boff.data(), ix->boff.size());
    ix->off_c = put(ix->image, ix->bkey.data(), ix->bkey.size());
    ix->off_d = put(ix->image, ix->bu.data(), ix->bu.size());
    ix->table_bytes = align_up(ix->off_d + 4 * ix->bu.size(), 16);  // contiguous from off_a = 0
    ix->off_e = put(ix->image, ix->upats.data(), ix->upats.size());
    ix->off_f = put(ix->image, ix->uoff.data(), ix->uoff.size());
    ix->off_g = put(ix->image, ix->uids.data(), ix->uids.size());
    if (ix->var)
        ix->off_h = put(ix->image, ix->upoff.data(), ix->upoff.size());
    ix->image.resize(align_up(ix->image.size(), 256), 0);
    return MPM_OK;
}

static mpm_status build_common(const uint8_t *P, uint32_t d, uint32_t m, mpm_index **out,
                               const char *who)
{
    if (!out)
        return fail(MPM_EINVAL, "%s: out is NULL", who);
    *out = nullptr;
    if (!P)
        return fail(MPM_EINVAL, "%s: patterns is NULL", who);
    if (d == 0)
        return fail(MPM_EINVAL, "%s: d must be positive", who);
    if (m == 0)
        return fail(MPM_EINVAL, "%s: m must be positive", who);
    if ((uint64_t)d * m > (1ull << 34))
        return fail(MPM_ETOOBIG, "%s: pattern bytes exceed 16 GiB", who);
    return MPM_OK;
}

}  // namespace mpm

using namespace mpm;

extern "C" {

const char *mpm_last_error(void) { return g_err.c_str(); }
const char *mpm_version(void) { return "mpm 1.0 (gfx950)"; }

mpm_status mpm_build_ac(const uint8_t *patterns, uint32_t d, uint32_t m, const mpm_opts *opts,
                        mpm_index **out)
{
    mpm_status st = build_common(patterns, d, m, out, "mpm_build_ac");
    if (st)
        return st;
    try {
        mpm_index *ix = new mpm_index();
        ix->algo = MPM_ALGO_AC;
        ix->keep_goto = opts && opts->ac_goto ? 1u : 0u;
        ix->m = m;
        ix->d = d;
        dedup(patterns, d, m, ix);
        st = build_ac_tables(ix);
        if (st) {
            delete ix;
            return st;
        }
        *out = ix;
        g_err.clear();
        return MPM_OK;
    } catch (const std::bad_alloc &) {
        return fail(MPM_ENOMEM, "mpm_build_ac: out of host memory");
    }
}

mpm_status mpm_build_wm(const uint8_t *patterns, uint32_t d, uint32_t m, const mpm_opts *opts,
                        mpm_index **out)
{
    mpm_status st = build_common(patterns, d, m, out, "mpm_build_wm");
    if (st)
        return st;
    uint32_t B = opts ? opts->wm_block : 0;
    if (B != 0 && (B > m || B > 8))
        return fail(MPM_EUNSUPPORTED, "mpm_build_wm: B=%u needs 1 <= B <= min(m=%u, 8)", B, m);
    try {
        mpm_index *ix = new mpm_index();
        ix->algo = MPM_ALGO_WM;
        ix->m = m;
        ix->d = d;
        dedup(patterns, d, m, ix);
        st = build_wm_tables(ix, B);
        if (st) {
            delete ix;
            return st;
        }
        *out = ix;
        g_err.clear();
        return MPM_OK;
    } catch (const std::bad_alloc &) {
        return fail(MPM_ENOMEM, "mpm_build_wm: out of host memory");
    }
}

// Sets of different lengths: checks, and the lengths (0: offsets invalid).
static mpm_status var_args(const uint8_t *bytes, const uint64_t *off, uint32_t d, mpm_index **out,
                           uint32_t *m_min, uint32_t *m_max, const char *who)
{
    if (!out)
        return fail(MPM_EINVAL, "%s: out is NULL", who);
    *out = nullptr;
    if (!bytes || !off)
        return fail(MPM_EINVAL, "%s: patterns or offsets is NULL", who);
    if (d == 0)
        return fail(MPM_EINVAL, "%s: d must be positive", who);
    uint64_t lo = ~0ull, hi = 0;
    for (uint32_t r = 0; r < d; r++) {
        if (off[r + 1] <= off[r])
            return fail(MPM_EINVAL, "%s: pattern %u is empty or its offsets descend", who, r);
        lo = std::min(lo, off[r + 1] - off[r]);
        hi = std::max(hi, off[r + 1] - off[r]);
    }
    if (off[d] - off[0] > (1ull << 34))
        return fail(MPM_ETOOBIG, "%s: pattern bytes exceed 16 GiB", who);
    if (hi >= (1ull << 31))
        return fail(MPM_ETOOBIG, "%s: a pattern of %llu bytes", who, (unsigned long long)hi);
    *m_min = (uint32_t)lo;
    *m_max = (uint32_t)hi;
    return MPM_OK;
}

mpm_status mpm_build_ac_var(const uint8_t *patterns, const uint64_t *offsets, uint32_t d,
                            const mpm_opts *opts, mpm_index **out)
{
    uint32_t lo = 0, hi = 0;
    mpm_status st = var_args(patterns, offsets, d, out, &lo, &hi, "mpm_build_ac_var");
    if (st)
        return st;
    if (lo == hi)  // one length: rows are contiguous
        return mpm_build_ac(patterns + offsets[0], d, lo, opts, out);
    if (opts && opts->ac_goto)
        return fail(MPM_EUNSUPPORTED, "mpm_build_ac_var: the supply-link walk needs one length");
    try {
        mpm_index *ix = new mpm_index();
        ix->algo = MPM_ALGO_AC;
        ix->var = 1;
        ix->m = lo;
        ix->m_max = hi;
        ix->d = d;
        st = dedup_var(patterns, offsets, d, ix);
        if (!st)
            st = build_ac_rev_tables(ix);
        if (st) {
            delete ix;
            return st;
        }
        *out = ix;
        g_err.clear();
        return MPM_OK;
    } catch (const std::bad_alloc &) {
        return fail(MPM_ENOMEM, "mpm_build_ac_var: out of host memory");
    }
}

mpm_status mpm_build_wm_var(const uint8_t *patterns, const uint64_t *offsets, uint32_t d,
                            const mpm_opts *opts, mpm_index **out)
{
    uint32_t lo = 0, hi = 0;
    mpm_status st = var_args(patterns, offsets, d, out, &lo, &hi, "mpm_build_wm_var");
    if (st)
        return st;
    if (lo == hi)
        return mpm_build_wm(patterns + offsets[0], d, lo, opts, out);
    const uint32_t B = opts ? opts->wm_block : 0;
    if (B != 0 && (B > lo || B > 8))
        return fail(MPM_EUNSUPPORTED, "mpm_build_wm_var: B=%u needs 1 <= B <= min(shortest "
                    "length %u, 8)", B, lo);
    try {
        mpm_index *ix = new mpm_index();
        ix->algo = MPM_ALGO_WM;
        ix->var = 1;
        ix->m = lo;
        ix->m_max = hi;
        ix->d = d;
        st = dedup_var(patterns, offsets, d, ix);
        if (!st) {
            ix->wpats.resize((uint64_t)ix->du * lo);
            for (uint32_t u = 0; u < ix->du; u++)
                memcpy(ix->wpats.data() + (uint64_t)u * lo, ix->upats.data() + ix->upoff[u], lo);
            st = build_wm_tables(ix, B);
        }
        if (st) {
            delete ix;
            return st;
        }
        *out = ix;
        g_err.clear();
        return MPM_OK;
    } catch (const std::bad_alloc &) {
        return fail(MPM_ENOMEM, "mpm_build_wm_var: out of host memory");
    }
}

void mpm_free(mpm_index *idx) { delete idx; }

uint64_t mpm_device_bytes(const mpm_index *idx) { return idx ? idx->image.size() : 0; }

mpm_status mpm_upload(mpm_index *idx, void *d_buf, uint64_t bytes, void *stream)
{
    if (!idx || !d_buf)
        return fail(MPM_EINVAL, "mpm_upload: null argument");
    if (((uintptr_t)d_buf) & 255)
        return fail(MPM_EINVAL, "mpm_upload: device buffer must be 256-byte aligned");
    if (bytes < idx->image.size())
        return fail(MPM_ENOMEM, "mpm_upload: buffer of %llu bytes, need %llu",
                    (unsigned long long)bytes, (unsigned long long)idx->image.size());
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(d_buf, idx->image.data(), idx->image.size(),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail(MPM_EHIP, "mpm_upload: %s", hipGetErrorString(e));
    idx->d_image = (const uint8_t *)d_buf;
    g_err.clear();
    return MPM_OK;
}

mpm_status mpm_index_info(const mpm_index *idx, mpm_info *o)
{
    if (!idx || !o)
        return fail(MPM_EINVAL, "mpm_index_info: null argument");
    memset(o, 0, sizeof *o);
    o->algo = idx->algo;
    o->m = idx->m;
    o->d = idx->d;
    o->d_unique = idx->du;
    o->max_dup = idx->max_dup;
    o->n_classes = idx->n_classes;
    o->n_states = idx->n_states;
    o->state_bytes = idx->state_bytes;
    o->wm_block = idx->B;
    o->wm_code_shift = idx->code_shift;
    o->wm_zero_shift = idx->zero_shift;
    o->wm_mean_shift = idx->mean_shift;
    o->table_bytes = idx->table_bytes;
    o->device_bytes = idx->image.size();
    o->m_max = idx->var ? idx->m_max : idx->m;
    return MPM_OK;
}

mpm_status mpm_export_ac(const mpm_index *idx, uint32_t *table, uint8_t *classes)
{
    if (!idx || idx->algo != MPM_ALGO_AC)
        return fail(MPM_EINVAL, "mpm_export_ac: not an Aho-Corasick index");
    if (table)
        memcpy(table, idx->dfa.data(), idx->dfa.size() * sizeof(uint32_t));
    if (classes)
        memcpy(classes, idx->class_bytes, idx->n_classes);
    return MPM_OK;
}

mpm_status mpm_export_wm_shift(const mpm_index *idx, uint8_t *shift)
{
    if (!idx || idx->algo != MPM_ALGO_WM || !shift)
        return fail(MPM_EINVAL, "mpm_export_wm_shift: not a Wu-Manber index");
    memcpy(shift, idx->shift.data(), idx->shift.size());
    return MPM_OK;
}

mpm_status mpm_export_unique(const mpm_index *idx, uint32_t *uoff, uint32_t *ids)
{
    if (!idx)
        return fail(MPM_EINVAL, "mpm_export_unique: null index");
    if (uoff)
        memcpy(uoff, idx->uoff.data(), idx->uoff.size() * sizeof(uint32_t));
    if (ids)
        memcpy(ids, idx->uids.data(), idx->uids.size() * sizeof(uint32_t));
    return MPM_OK;
}

// ---------------------------------------------------------------------------
// Single-text scan
// ---------------------------------------------------------------------------

static uint64_t n_starts(uint64_t n, uint32_t m) { return n >= m ? n - m + 1 : 0; }

}  // extern "C"

// Bounds of the kernels' counters: a lane counts its ids in 32 bits and a
// wave's prefix sum over its 64 lanes stays in 32 bits (at most
// 64 * lane_bytes * max_dup ids); a look-back status word carries a text's
// inclusive count in ST_VAL_BITS bits (at most ns * max_dup ids).
static mpm_status check_counts(const mpm_index *ix, uint64_t ns, uint32_t lane_bytes,
                               const char *who)
{
    const uint64_t md = ix->max_dup ? ix->max_dup : 1;
    if (64ull * lane_bytes * md >= (1ull << 32))
        return fail(MPM_EUNSUPPORTED, "%s: %u copies of one pattern overflow a wave's 32-bit "
                    "count at %u starting positions per lane", who, ix->max_dup, lane_bytes);
    if (ns * md >= (1ull << ST_VAL_BITS))
        return fail(MPM_ETOOBIG, "%s: %llu starting positions x %u copies of one pattern "
                    "exceed the %u-bit count of a text", who, (unsigned long long)ns, ix->max_dup,
                    (unsigned)ST_VAL_BITS);
    return MPM_OK;
}

extern "C" {

}  // extern "C"

namespace mpm {
// Workspace of a single-text scan: the header and one status word per chunk
// (the minimum), then the staging area, which holds every occurrence a lane
// can have (one distinct string per starting position) when the workspace
// has room for it (the full size); a smaller staging area only means that
// lanes with more occurrences than it holds walk their range again.
mpm_status workspace_sizes(const mpm_index *idx, uint64_t n, const mpm_variant *v,
                           uint64_t *min_bytes, uint64_t *full_bytes, const char *who)
{
    if (!idx)
        return fail(MPM_EINVAL, "%s: null index", who);
    LaunchCfg cfg;
    mpm_status st = resolve_variant(idx, v, 0, &cfg);
    if (st)
        return st;
    const uint64_t tb = tile_bytes(cfg);
    const uint64_t nt = (n_starts(n, idx->m) + tb - 1) / tb;
    *min_bytes = WS_HEADER_BYTES + 8 * nt;
    *full_bytes = *min_bytes;
    if (full_bytes != min_bytes && nt && !cfg.dense) {  // dense output stages nothing
        st = resolve_variant(idx, v, nt, &cfg);
        if (st)
            return st;
        *full_bytes = align_up(*min_bytes, 256) + (uint64_t)cfg.grid * tb * sizeof(mpm_match);
    }
    return MPM_OK;
}
}  // namespace mpm

extern "C" {

mpm_status mpm_workspace_bytes(const mpm_index *idx, uint64_t n, const mpm_variant *v,
                               uint64_t *bytes)
{
    if (!idx || !bytes)
        return fail(MPM_EINVAL, "mpm_workspace_bytes: null argument");
    uint64_t lo = 0;
    return workspace_sizes(idx, n, v, &lo, bytes, "mpm_workspace_bytes");
}

}  // extern "C"

namespace mpm {
// mpm_scan on a given workspace; `who` names the entry point in errors.
mpm_status scan_with_workspace(const mpm_index *idx, const uint8_t *d_text, uint64_t n,
                               mpm_match *d_out, uint64_t capacity, void *d_work,
                               uint64_t work_bytes, uint64_t *d_total, const mpm_variant *v,
                               void *stream, const char *who)
{
    if (!idx || !d_total || !d_work)
        return fail(MPM_EINVAL, "%s: null index, workspace or total", who);
    if (n >= (1ull << 32))
        return fail(MPM_ETOOBIG, "%s: n = %llu needs 32-bit positions", who,
                    (unsigned long long)n);
    if (capacity && !d_out)
        return fail(MPM_EINVAL, "%s: d_out is NULL with capacity > 0", who);
    if (n && !d_text)
        return fail(MPM_EINVAL, "%s: d_text is NULL", who);
    if (((uintptr_t)d_work) & 7)
        return fail(MPM_EINVAL, "%s: workspace must be 8-byte aligned", who);
    LaunchCfg cfg;
    uint64_t ns = n_starts(n, idx->m);
    mpm_status st = resolve_variant(idx, v, 0, &cfg);
    if (st)
        return st;
    uint64_t tb = tile_bytes(cfg);
    uint64_t nt = (ns + tb - 1) / tb;
    st = check_counts(idx, ns, cfg.lane_bytes, who);
    if (st)
        return st;
    if (!idx->d_image)
        return fail(MPM_ESTATE, "%s: index not uploaded (call mpm_upload)", who);
    if (work_bytes < WS_HEADER_BYTES + 8 * nt)
        return fail(MPM_ENOMEM, "%s: workspace of %llu bytes, need %llu", who,
                    (unsigned long long)work_bytes, (unsigned long long)(WS_HEADER_BYTES + 8 * nt));
    if (nt == 0)
        return launch_zero_totals(nullptr, 0, d_total, stream);
    st = resolve_variant(idx, v, nt, &cfg, true);
    if (st)
        return st;
    ScanDev sd;
    memset(&sd, 0, sizeof sd);
    // staging: as many slots per virtual lane as the workspace holds, at most
    // one per starting position of the lane
    // (none for dense output, or for a counting call with no output at all)
    const uint64_t stage_off = align_up(WS_HEADER_BYTES + 8 * nt, 256);
    if (work_bytes > stage_off && capacity && !cfg.dense) {
        const uint64_t per_slot = (uint64_t)cfg.grid * cfg.block_threads * cfg.ilp * sizeof(mpm_match);
        const uint64_t slots = std::min<uint64_t>(cfg.lane_bytes, (work_bytes - stage_off) / per_slot);
        if (slots) {
            sd.stage = (mpm_match *)((uint8_t *)d_work + stage_off);
            sd.stage_cap = (uint32_t)slots;
        }
    }
    if (cfg.csr_lds) {
        sd.csr_uoff_words = csr_uoff_words(idx);
        sd.csr_uids_words = csr_uids_words(idx);
        sd.csr_uoff_lds = cfg.csr_lds;
        sd.csr_uids_lds = cfg.csr_lds + 4 * sd.csr_uoff_words;
    }
    sd.single = TextDesc{d_text, n, d_out, capacity, d_total, 0, nt};
    sd.multi = nullptr;
    sd.ntexts = 1;
    sd.lane_bytes = cfg.lane_bytes;
    sd.ntiles = nt;
    sd.hdr = (uint32_t *)d_work;
    sd.status = (uint64_t *)((uint8_t *)d_work + WS_HEADER_BYTES);
    sd.mark_lds = cfg.mark_lds;
    return launch_scan(idx, cfg, sd, stream);
}
}  // namespace mpm

extern "C" {

mpm_status mpm_scan(const mpm_index *idx, const uint8_t *d_text, uint64_t n, mpm_match *d_out,
                    uint64_t capacity, void *d_work, uint64_t work_bytes, uint64_t *d_total,
                    const mpm_variant *v, void *stream)
{
    return scan_with_workspace(idx, d_text, n, d_out, capacity, d_work, work_bytes, d_total, v,
                               stream, "mpm_scan");
}

mpm_status mpm_scan_sync(const mpm_index *idx, const uint8_t *d_text, uint64_t n, mpm_match *d_out,
                         uint64_t capacity, void *d_work, uint64_t work_bytes, uint64_t *d_total,
                         const mpm_variant *v, void *stream, uint64_t *total)
{
    if (!total)
        return fail(MPM_EINVAL, "mpm_scan_sync: total is NULL");
    mpm_status st = mpm_scan(idx, d_text, n, d_out, capacity, d_work, work_bytes, d_total, v, stream);
    if (st)
        return st;
    hipStream_t s = (hipStream_t)stream;
    uint32_t hdr[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(total, d_total, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hdr, d_work, sizeof hdr, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail(MPM_EHIP, "mpm_scan_sync: %s", hipGetErrorString(e));
    if (hdr[WS_ERR]) {
        (void)hipMemsetAsync((uint8_t *)d_work + 4 * WS_ERR, 0, 4, s);
        (void)hipStreamSynchronize(s);
        if (hdr[WS_ERR] & WS_ERR_LDS_LAYOUT)
            return fail(MPM_ESTATE, "mpm_scan_sync: kernel LDS layout check failed");
        return fail(MPM_ESTATE, "mpm_scan_sync: device look-back did not complete");
    }
    if (*total > capacity)
        return fail(MPM_EOVERFLOW, "mpm_scan_sync: %llu matches, capacity %llu",
                    (unsigned long long)*total, (unsigned long long)capacity);
    g_err.clear();
    return MPM_OK;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
}  // extern "C"

// Launch key of a batch request: walker kind, block size and LDS class. Each
// launch runs one kernel (one walker kind); its LDS size is the largest its
// texts need, so texts with small tables are kept apart from texts whose
// tables limit a CU to one or two workgroups.
static uint32_t launch_key(uint32_t kind, const LaunchCfg &c)
{
    const uint32_t lds = c.lds_bytes;
    const uint32_t lds_class = lds <= 8192 ? 0 : lds <= 32768 ? 1 : lds <= 65536 ? 2 : 3;
    return (kind & 0xffu) << 16 | (c.block_threads & 0x3fffu) << 2 | lds_class;
}

struct mpm_batch {
    // One persistent launch per block size; its texts ordered by index and
    // walker kind so that LDS tables are reused across consecutive chunks.
    struct Group {
        uint32_t kind = 0;  // walker kind of the launch (BK_*)
        uint32_t W = 0;
        uint32_t grid_req = 0;
        uint32_t grid = 0;
        uint32_t lds = 0;
        std::vector<BatchText> texts;
        std::vector<BatchIndex> idx;
        uint64_t ntiles = 0;
        uint64_t text_off = 0, idx_off = 0, work_off = 0, stage_off = 0;
    };
    std::vector<mpm_request> reqs;
    std::vector<Group> groups;
    std::vector<uint64_t *> zero_totals;   // requests with no starting position
    uint64_t zero_off = 0;
    uint64_t bytes = 0;
    uint8_t *d_buf = nullptr;
    bool serial = false;       // launches one after another (timed requests)
    float us_per_tick = 0.f;   // wall-clock tick length
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // Side streams (default priority) so that the plan's launches run as
    // parallel branches: each launch's tail overlaps the others' work.
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> done;
    hipEvent_t fork = nullptr;
};

extern "C" {

mpm_status mpm_batch_plan(const mpm_request *reqs, uint32_t count, mpm_batch **out)
{
    if (!out || (!reqs && count))
        return fail(MPM_EINVAL, "mpm_batch_plan: null argument");
    *out = nullptr;
    try {
        mpm_batch *b = new mpm_batch();
        b->reqs.assign(reqs, reqs + count);
        struct Item {
            uint32_t req;
            const mpm_index *ix;
            LaunchCfg cfg;
            uint32_t kind;
            float hint;
            float group_hint;
        };
        std::map<uint32_t, std::vector<Item>> byw;
        for (uint32_t k = 0; k < count; k++) {
            const mpm_request &r = reqs[k];
            if (!r.idx || !r.d_total || (r.n && !r.d_text) || (r.capacity && !r.d_out)) {
                delete b;
                return fail(MPM_EINVAL, "mpm_batch_plan: request %u has a null pointer", k);
            }
            if (!r.idx->d_image) {
                delete b;
                return fail(MPM_ESTATE, "mpm_batch_plan: request %u: index not uploaded", k);
            }
            if (r.idx->var) {
                delete b;
                return fail(MPM_EUNSUPPORTED, "mpm_batch_plan: request %u: sets of different "
                            "lengths run in single-text scans only", k);
            }
            if (r.n >= (1ull << 32)) {
                delete b;
                return fail(MPM_ETOOBIG, "mpm_batch_plan: request %u: n >= 2^32", k);
            }
            if (n_starts(r.n, r.idx->m) == 0) {
                b->zero_totals.push_back(r.d_total);
                continue;
            }
            mpm_variant v = r.variant;
            // batched walkers run one range per lane and write per lane
            v.flags &= ~(MPM_VARIANT_ILP2 | MPM_VARIANT_DENSE | MPM_VARIANT_TEXT_BYTES | MPM_VARIANT_TEXT_LDS);
            Item it;
            it.req = k;
            it.ix = r.idx;
            it.hint = r.cost_hint > 0.f ? r.cost_hint : 0.f;
            it.group_hint = 0.f;
            mpm_status st = resolve_variant(r.idx, &v, 0, &it.cfg);
            if (!st && it.cfg.supply)
                st = fail(MPM_EUNSUPPORTED, "mpm_batch_plan: the supply-link walk runs in "
                          "single-text scans only");
            if (st) {
                delete b;
                return st;
            }
            st = check_counts(r.idx, n_starts(r.n, r.idx->m), it.cfg.lane_bytes, "mpm_batch_plan");
            if (st) {
                delete b;
                return st;
            }
            it.kind = batch_kind(r.idx, it.cfg);
            const uint32_t key = launch_key(it.kind, it.cfg);
            byw[key].push_back(it);
            if (r.variant.grid)
                byw[key].back().cfg.grid = r.variant.grid;
        }
        for (auto &kv : byw) {
            std::vector<Item> &items = kv.second;
            // Longest expected chunks first, by (index, kind) group so that
            // consecutive chunks keep sharing their LDS tables.
            std::map<std::pair<const mpm_index *, uint32_t>, float> ghint;
            for (const Item &it : items) {
                float &g = ghint[std::make_pair(it.ix, it.kind)];
                g = std::max(g, it.hint);
            }
            for (Item &it : items)
                it.group_hint = ghint[std::make_pair(it.ix, it.kind)];
            std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) {
                if (x.group_hint != y.group_hint)
                    return x.group_hint > y.group_hint;
                if (x.ix != y.ix)
                    return (uintptr_t)x.ix < (uintptr_t)y.ix;
                if (x.kind != y.kind)
                    return x.kind < y.kind;
                return x.hint > y.hint;
            });
            mpm_batch::Group g;
            g.kind = items.front().kind;
            g.W = items.front().cfg.block_threads;
            std::map<const mpm_index *, uint32_t> slot;
            for (const Item &it : items) {
                const mpm_request &r = reqs[it.req];
                auto f = slot.find(it.ix);
                uint32_t si;
                if (f == slot.end()) {
                    si = (uint32_t)g.idx.size();
                    slot[it.ix] = si;
                    BatchIndex bi;
                    memset(&bi, 0, sizeof bi);
                    if (it.ix->algo == MPM_ALGO_AC)
                        bi.ac = ac_dev(it.ix);
                    else
                        bi.wm = wm_dev(it.ix);
                    g.idx.push_back(bi);
                } else {
                    si = f->second;
                }
                if (it.cfg.grid)
                    g.grid_req = std::max(g.grid_req, it.cfg.grid);
                const uint64_t tb = (uint64_t)it.cfg.lane_bytes * it.cfg.block_threads;
                const uint64_t nt = (n_starts(r.n, it.ix->m) + tb - 1) / tb;
                BatchText bt;
                memset(&bt, 0, sizeof bt);
                bt.td = TextDesc{r.d_text, r.n, r.d_out, r.capacity, r.d_total, g.ntiles, nt};
                bt.index = si;
                bt.kind = it.kind;
                bt.lane_bytes = it.cfg.lane_bytes;
                bt.cost = r.d_cost;
                if (r.d_cost)
                    b->serial = true;
                g.texts.push_back(bt);
                g.ntiles += nt;
                g.lds = std::max(g.lds, it.cfg.lds_bytes);
            }
            b->groups.push_back(std::move(g));
        }
        uint64_t off = 0;
        for (auto &g : b->groups) {
            g.grid = batch_grid(g.kind, g.W, g.lds, g.ntiles, g.grid_req);
            g.text_off = off;
            off = align_up(off + g.texts.size() * sizeof(BatchText), 256);
            g.idx_off = off;
            off = align_up(off + g.idx.size() * sizeof(BatchIndex), 256);
            g.work_off = off;
            off = align_up(off + WS_HEADER_BYTES + 8 * g.ntiles, 256);
            g.stage_off = off;
            off = align_up(off + (uint64_t)g.grid * g.W * BATCH_STAGE_CAP * sizeof(mpm_match), 256);
        }
        b->zero_off = off;
        off = align_up(off + 8 * b->zero_totals.size() + 8, 256);
        b->bytes = off;
        if (b->serial) {
            int dev = 0, khz = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
                khz <= 0) {
                delete b;
                return fail(MPM_EHIP, "mpm_batch_plan: wall-clock rate unavailable");
            }
            b->us_per_tick = 1000.f / (float)khz;
        }
        *out = b;
        g_err.clear();
        return MPM_OK;
    } catch (const std::bad_alloc &) {
        return fail(MPM_ENOMEM, "mpm_batch_plan: out of host memory");
    }
}

uint64_t mpm_batch_device_bytes(const mpm_batch *b) { return b ? b->bytes : 0; }

uint32_t mpm_batch_groups(const mpm_batch *b) { return b ? (uint32_t)b->groups.size() : 0; }

mpm_status mpm_batch_launch_key(const mpm_index *idx, const mpm_variant *variant, uint32_t *key)
{
    if (!idx || !key)
        return fail(MPM_EINVAL, "mpm_batch_launch_key: null argument");
    if (idx->var)
        return fail(MPM_EUNSUPPORTED, "mpm_batch_launch_key: sets of different lengths run in "
                    "single-text scans only");
    mpm_variant v = variant ? *variant : mpm_variant{0, 0, 0, 0, 0};
    v.flags &= ~(MPM_VARIANT_ILP2 | MPM_VARIANT_DENSE | MPM_VARIANT_TEXT_BYTES | MPM_VARIANT_TEXT_LDS);
    LaunchCfg cfg;
    mpm_status st = resolve_variant(idx, &v, 0, &cfg);
    if (st)
        return st;
    if (cfg.supply)
        return fail(MPM_EUNSUPPORTED, "mpm_batch_launch_key: the supply-link walk runs in "
                    "single-text scans only");
    *key = launch_key(batch_kind(idx, cfg), cfg);
    g_err.clear();
    return MPM_OK;
}

mpm_status mpm_batch_upload(mpm_batch *b, void *d_buf, uint64_t bytes, void *stream)
{
    if (!b || !d_buf)
        return fail(MPM_EINVAL, "mpm_batch_upload: null argument");
    if (((uintptr_t)d_buf) & 255)
        return fail(MPM_EINVAL, "mpm_batch_upload: buffer must be 256-byte aligned");
    if (bytes < b->bytes)
        return fail(MPM_ENOMEM, "mpm_batch_upload: buffer too small");
    std::vector<uint8_t> host(b->bytes, 0);
    for (const auto &g : b->groups) {
        memcpy(host.data() + g.text_off, g.texts.data(), g.texts.size() * sizeof(BatchText));
        memcpy(host.data() + g.idx_off, g.idx.data(), g.idx.size() * sizeof(BatchIndex));
    }
    memcpy(host.data() + b->zero_off, b->zero_totals.data(), 8 * b->zero_totals.size());
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(d_buf, host.data(), b->bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail(MPM_EHIP, "mpm_batch_upload: %s", hipGetErrorString(e));
    b->d_buf = (uint8_t *)d_buf;
    return MPM_OK;
}

static mpm_status ensure_side_streams(mpm_batch *b)
{
    const size_t need = b->groups.size() > 1 ? b->groups.size() : 0;
    while (b->side.size() < need) {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return fail(MPM_EHIP, "mpm_batch: side stream creation failed");
        b->side.push_back(s);
        b->done.push_back(e);
    }
    if (need && !b->fork &&
        hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
        return fail(MPM_EHIP, "mpm_batch: event creation failed");
    return MPM_OK;
}

mpm_status mpm_batch_run(const mpm_batch *cb, void *stream)
{
    mpm_batch *b = const_cast<mpm_batch *>(cb);
    if (!b || !b->d_buf)
        return fail(MPM_ESTATE, "mpm_batch_run: plan not uploaded");
    mpm_status st0 = ensure_side_streams(b);
    if (st0)
        return st0;
    if (!b->zero_totals.empty()) {
        mpm_status st = launch_zero_totals((uint64_t *const *)(b->d_buf + b->zero_off),
                                           (uint32_t)b->zero_totals.size(), nullptr, stream);
        if (st)
            return st;
    }
    const bool fan = b->groups.size() > 1 && !b->serial;
    hipStream_t main_s = (hipStream_t)stream;
    if (fan && hipEventRecord(b->fork, main_s) != hipSuccess)
        return fail(MPM_EHIP, "mpm_batch_run: fork event failed");
    for (size_t gi = 0; gi < b->groups.size(); gi++) {
        const auto &g = b->groups[gi];
        void *ls = stream;
        if (fan) {
            if (hipStreamWaitEvent(b->side[gi], b->fork, 0) != hipSuccess)
                return fail(MPM_EHIP, "mpm_batch_run: stream wait failed");
            ls = b->side[gi];
        }
        BatchDev bd;
        memset(&bd, 0, sizeof bd);
        bd.texts = (const BatchText *)(b->d_buf + g.text_off);
        bd.idx = (const BatchIndex *)(b->d_buf + g.idx_off);
        bd.ntexts = (uint32_t)g.texts.size();
        bd.ntiles = g.ntiles;
        bd.hdr = (uint32_t *)(b->d_buf + g.work_off);
        bd.status = (uint64_t *)(b->d_buf + g.work_off + WS_HEADER_BYTES);
        bd.stage = (mpm_match *)(b->d_buf + g.stage_off);
        bd.stage_cap = BATCH_STAGE_CAP;
        bd.us_per_tick = b->us_per_tick;
        mpm_status st = launch_batch(bd, g.kind, g.W, g.grid, g.lds, ls);
        if (st)
            return st;
        if (fan && (hipEventRecord(b->done[gi], (hipStream_t)ls) != hipSuccess ||
                    hipStreamWaitEvent(main_s, b->done[gi], 0) != hipSuccess))
            return fail(MPM_EHIP, "mpm_batch_run: join failed");
    }
    return MPM_OK;
}

mpm_status mpm_batch_capture(mpm_batch *b, void *stream)
{
    if (!b || !b->d_buf)
        return fail(MPM_ESTATE, "mpm_batch_capture: plan not uploaded");
    hipStream_t s = (hipStream_t)stream;
    mpm_status st0 = ensure_side_streams(b);
    if (st0)
        return st0;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return fail(MPM_EHIP, "mpm_batch_capture: begin: %s", hipGetErrorString(e));
    mpm_status st = mpm_batch_run(b, stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (st) {
        if (g)
            (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess)
        return fail(MPM_EHIP, "mpm_batch_capture: end: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(MPM_EHIP, "mpm_batch_capture: instantiate: %s", hipGetErrorString(e));
    }
    b->graph = g;
    return MPM_OK;
}

mpm_status mpm_batch_replay(const mpm_batch *b, void *stream)
{
    if (!b || !b->exec)
        return fail(MPM_ESTATE, "mpm_batch_replay: no captured graph");
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    if (e != hipSuccess)
        return fail(MPM_EHIP, "mpm_batch_replay: %s", hipGetErrorString(e));
    return MPM_OK;
}

// ---------------------------------------------------------------------------
// Autotuning support
// ---------------------------------------------------------------------------
static mpm_status tune_layout(const mpm_index *idx, uint64_t n, uint32_t copies,
                              const mpm_variant *v, LaunchCfg *cfg, uint64_t *nt_copy,
                              uint64_t *idx_off, uint64_t *work_off, uint64_t *stage_off,
                              uint32_t *grid, uint64_t *bytes)
{
    if (!idx || copies == 0)
        return fail(MPM_EINVAL, "mpm_tune: null index or zero copies");
    if (idx->var)
        return fail(MPM_EUNSUPPORTED, "mpm_tune: sets of different lengths run in single-text "
                    "scans only");
    mpm_variant w = v ? *v : mpm_variant{0, 0, 0, 0, 0};
    w.flags &= ~(MPM_VARIANT_ILP2 | MPM_VARIANT_DENSE | MPM_VARIANT_TEXT_BYTES | MPM_VARIANT_TEXT_LDS);
    mpm_status st = resolve_variant(idx, &w, 0, cfg);
    if (st)
        return st;
    if (cfg->supply)
        return fail(MPM_EUNSUPPORTED, "mpm_tune: the supply-link walk runs in single-text scans only");
    const uint64_t tb = (uint64_t)cfg->lane_bytes * cfg->block_threads;
    *nt_copy = (n_starts(n, idx->m) + tb - 1) / tb;
    *idx_off = align_up((uint64_t)copies * sizeof(BatchText), 256);
    *work_off = align_up(*idx_off + sizeof(BatchIndex), 256);
    *stage_off = align_up(*work_off + WS_HEADER_BYTES + 8 * (*nt_copy) * copies, 256);
    *grid = *nt_copy ? batch_grid(batch_kind(idx, *cfg), cfg->block_threads, cfg->lds_bytes,
                                  *nt_copy * copies, v ? v->grid : 0)
                     : 1;
    *bytes = *stage_off + (uint64_t)(*grid) * cfg->block_threads * BATCH_STAGE_CAP *
                              sizeof(mpm_match);
    return MPM_OK;
}

uint64_t mpm_tune_work_bytes(const mpm_index *idx, uint64_t n, uint32_t copies,
                             const mpm_variant *v)
{
    LaunchCfg cfg;
    uint64_t nt, io, wo, so, bytes;
    uint32_t grid;
    if (tune_layout(idx, n, copies, v, &cfg, &nt, &io, &wo, &so, &grid, &bytes))
        return 0;
    return bytes;
}

mpm_status mpm_tune_time(const mpm_index *idx, const uint8_t *d_text, uint64_t n, uint32_t copies,
                         const mpm_variant *v, mpm_match *d_out, uint64_t capacity, uint64_t *d_total,
                         void *d_work, uint64_t work_bytes, uint32_t reps, void *stream,
                         float *ms_out)
{
    if (!idx || !d_text || !d_total || !d_work || !ms_out || (capacity && !d_out) || reps == 0)
        return fail(MPM_EINVAL, "mpm_tune_time: null argument");
    if (!idx->d_image)
        return fail(MPM_ESTATE, "mpm_tune_time: index not uploaded");
    if (n >= (1ull << 32))
        return fail(MPM_ETOOBIG, "mpm_tune_time: n >= 2^32");
    if (((uintptr_t)d_work) & 255)
        return fail(MPM_EINVAL, "mpm_tune_time: workspace must be 256-byte aligned");
    LaunchCfg cfg;
    uint64_t nt, io, wo, so, bytes;
    uint32_t grid;
    mpm_status st = tune_layout(idx, n, copies, v, &cfg, &nt, &io, &wo, &so, &grid, &bytes);
    if (st)
        return st;
    if (work_bytes < bytes)
        return fail(MPM_ENOMEM, "mpm_tune_time: workspace of %llu bytes, need %llu",
                    (unsigned long long)work_bytes, (unsigned long long)bytes);
    st = check_counts(idx, n_starts(n, idx->m), cfg.lane_bytes, "mpm_tune_time");
    if (st)
        return st;
    if (nt == 0) {
        *ms_out = 0.f;
        return MPM_OK;
    }
    try {
        std::vector<uint8_t> host(wo + WS_HEADER_BYTES, 0);
        BatchText *bt = (BatchText *)host.data();
        for (uint32_t k = 0; k < copies; k++) {
            // every copy writes the same region: identical values, one total
            bt[k].td = TextDesc{d_text, n, d_out, capacity, d_total, (uint64_t)k * nt, nt};
            bt[k].index = 0;
            bt[k].kind = batch_kind(idx, cfg);
            bt[k].lane_bytes = cfg.lane_bytes;
            bt[k].cost = nullptr;
        }
        BatchIndex *bi = (BatchIndex *)(host.data() + io);
        if (idx->algo == MPM_ALGO_AC)
            bi->ac = ac_dev(idx);
        else
            bi->wm = wm_dev(idx);
        hipStream_t s = (hipStream_t)stream;
        hipError_t e = hipMemcpyAsync(d_work, host.data(), host.size(), hipMemcpyHostToDevice, s);
        if (e != hipSuccess)
            return fail(MPM_EHIP, "mpm_tune_time: upload: %s", hipGetErrorString(e));
        const uint64_t ntiles = nt * copies;
        BatchDev bd;
        memset(&bd, 0, sizeof bd);
        bd.texts = (const BatchText *)d_work;
        bd.idx = (const BatchIndex *)((uint8_t *)d_work + io);
        bd.ntexts = copies;
        bd.ntiles = ntiles;
        bd.hdr = (uint32_t *)((uint8_t *)d_work + wo);
        bd.status = (uint64_t *)((uint8_t *)d_work + wo + WS_HEADER_BYTES);
        bd.stage = (mpm_match *)((uint8_t *)d_work + so);
        bd.stage_cap = BATCH_STAGE_CAP;
        const uint32_t kind = batch_kind(idx, cfg);
        hipEvent_t a, z;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&z) != hipSuccess)
            return fail(MPM_EHIP, "mpm_tune_time: event creation failed");
        // warm-up, then `reps` launches between two events: the mean launch
        st = launch_batch(bd, kind, cfg.block_threads, grid, cfg.lds_bytes, stream);
        (void)hipEventRecord(a, s);
        for (uint32_t r = 0; r < reps && st == MPM_OK; r++)
            st = launch_batch(bd, kind, cfg.block_threads, grid, cfg.lds_bytes, stream);
        (void)hipEventRecord(z, s);
        float ms = 0.f;
        if (st == MPM_OK && hipEventSynchronize(z) == hipSuccess)
            (void)hipEventElapsedTime(&ms, a, z);
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(z);
        if (st)
            return st;
        *ms_out = ms / (float)reps;
        return MPM_OK;
    } catch (const std::bad_alloc &) {
        return fail(MPM_ENOMEM, "mpm_tune_time: out of host memory");
    }
}

void mpm_batch_free(mpm_batch *b)
{
    if (!b)
        return;
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    for (hipEvent_t e : b->done)
        (void)hipEventDestroy(e);
    for (hipStream_t s : b->side)
        (void)hipStreamDestroy(s);
    if (b->fork)
        (void)hipEventDestroy(b->fork);
    delete b;
}

}  // extern "C"
