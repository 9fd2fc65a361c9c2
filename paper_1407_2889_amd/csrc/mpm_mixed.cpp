// Aho-Corasick for pattern sets of different lengths: the automaton of the
// reversed patterns, flattened, for a scan that reads each lane's range from
// its end to its start.
//
// Reading the text backwards, the state after character j is the longest
// string that starts at j and ends some pattern (its reverse is a prefix of a
// reversed pattern). Merged along supply links (Section 3.1: a state reports
// every pattern that is a suffix of its label, so the output sets of the
// supply chain are added, Algorithm 2's update for sets whose lengths
// differ), the state's output set is exactly the set of patterns that occur
// at j: those that are prefixes of the longest string that starts at j and
// is a pattern. The scan therefore meets every start once, with all of its
// patterns together, and reports it as one distinct string (the longest)
// whose id list holds the ids of all of them; reading backwards, the starts
// come in descending order.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "mpm_internal.h"

namespace mpm {

static uint64_t align_up_m(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

template <typename T>
static uint64_t put_m(std::vector<uint8_t> &img, const T *src, uint64_t count)
{
    uint64_t off = align_up_m(img.size(), 256);
    uint64_t bytes = count * sizeof(T);
    img.resize(align_up_m(off + bytes, 16), 0);
    if (bytes)
        memcpy(img.data() + off, src, bytes);
    return off;
}

// Builds the flattened table of the reversed distinct strings of ix (upats,
// upoff, with their id lists already in uoff/uids): rows in breadth-first
// order with the states that report a string last, term_u[t] the string
// reported by state first_term + t.
mpm_status build_ac_rev_tables(mpm_index *ix)
{
    const uint32_t du = ix->du;
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
    const uint64_t max_nodes = (uint64_t)ix->upats.size() + 1;
    if (max_nodes > (1ull << 31))
        return fail(MPM_ETOOBIG, "build_ac: up to %llu states exceed 2^31",
                    (unsigned long long)max_nodes);

    // Trie of the reversed strings; own[q] = the string whose reverse ends at q.
    std::vector<int32_t> child(C, -1);
    std::vector<uint32_t> depth(1, 0);
    std::vector<int32_t> own(1, -1);
    for (uint32_t u = 0; u < du; u++) {
        const uint8_t *p = ix->upats.data() + ix->upoff[u];
        const uint32_t len = (uint32_t)(ix->upoff[u + 1] - ix->upoff[u]);
        int64_t q = 0;
        for (uint32_t j = 0; j < len; j++) {
            const uint32_t c = ix->cls[p[len - 1 - j]] - 1u;
            int32_t nx = child[q * C + c];
            if (nx < 0) {
                nx = (int32_t)depth.size();
                child[q * C + c] = nx;
                child.resize(child.size() + C, -1);
                depth.push_back(j + 1);
                own.push_back(-1);
            }
            q = nx;
        }
        own[q] = (int32_t)u;
    }
    const uint64_t S = depth.size();

    // Breadth-first order; supply links; the reported string of each state:
    // its own, else its supply state's (the longest reversed pattern that is
    // a suffix of the state's label).
    std::vector<uint32_t> bfs;
    bfs.reserve(S);
    bfs.push_back(0);
    for (uint64_t h = 0; h < bfs.size(); h++)
        for (uint32_t c = 0; c < C; c++) {
            const int32_t w = child[(uint64_t)bfs[h] * C + c];
            if (w >= 0)
                bfs.push_back((uint32_t)w);
        }
    std::vector<uint32_t> supply(S, 0);
    std::vector<int32_t> rep(S, -1);
    std::vector<uint32_t> delta(S * C);
    for (uint64_t h = 0; h < S; h++) {
        const uint32_t v = bfs[h];
        rep[v] = own[v] >= 0 ? own[v] : (v == 0 ? -1 : rep[supply[v]]);
        for (uint32_t c = 0; c < C; c++) {
            const int32_t w = child[(uint64_t)v * C + c];
            if (w >= 0) {
                if (v != 0) {
                    uint32_t f = supply[v];
                    while (f != 0 && child[(uint64_t)f * C + c] < 0)
                        f = supply[f];
                    const int32_t g = child[(uint64_t)f * C + c];
                    supply[w] = g >= 0 ? (uint32_t)g : 0;
                }
                delta[(uint64_t)v * C + c] = (uint32_t)w;
            } else {
                delta[(uint64_t)v * C + c] = v == 0 ? 0 : delta[(uint64_t)supply[v] * C + c];
            }
        }
    }

    // Numbering: non-reporting states in breadth-first order, then the
    // reporting ones in breadth-first order.
    std::vector<uint32_t> order;
    order.reserve(S);
    for (uint32_t v : bfs)
        if (rep[v] < 0)
            order.push_back(v);
    const uint64_t first_term = order.size();
    for (uint32_t v : bfs)
        if (rep[v] >= 0)
            order.push_back(v);
    std::vector<uint32_t> newid(S);
    for (uint64_t k = 0; k < S; k++)
        newid[order[k]] = (uint32_t)k;
    ix->n_states = S;
    ix->first_term = first_term;
    ix->term_u.resize(S - first_term);
    for (uint64_t k = first_term; k < S; k++)
        ix->term_u[k - first_term] = (uint32_t)rep[order[k]];
    ix->dfa.assign(S * cp, 0);
    for (uint64_t k = 0; k < S; k++)
        for (uint32_t c = 0; c < C; c++)
            ix->dfa[k * cp + 1 + c] = newid[delta[(uint64_t)order[k] * C + c]];
    ix->state_bytes = S <= 65535 ? 2 : 4;
    if (S * cp * ix->state_bytes >= (1ull << 32))
        return fail(MPM_ETOOBIG, "build_ac: table of %llu states x %u columns exceeds 4 GiB",
                    (unsigned long long)S, cp);

    // Device image: table, column offsets per byte, id CSR, reported strings.
    ix->image.clear();
    if (ix->state_bytes == 2) {
        std::vector<uint16_t> t16(ix->dfa.begin(), ix->dfa.end());
        ix->off_a = put_m(ix->image, t16.data(), t16.size());
    } else {
        ix->off_a = put_m(ix->image, ix->dfa.data(), ix->dfa.size());
    }
    ix->table_bytes = align_up_m(S * cp * ix->state_bytes, 16);
    uint16_t cls_off[256];
    for (int b = 0; b < 256; b++)
        cls_off[b] = (uint16_t)(ix->cls[b] * ix->state_bytes);
    ix->off_b = put_m(ix->image, cls_off, 256);
    ix->swar_ok = 0;  // the reverse walk reads bytes through the class map
    ix->off_c = put_m(ix->image, ix->uoff.data(), ix->uoff.size());
    ix->off_d = put_m(ix->image, ix->uids.data(), ix->uids.size());
    ix->off_e = put_m(ix->image, ix->term_u.data(), ix->term_u.size());
    ix->image.resize(align_up_m(ix->image.size(), 256), 0);
    return MPM_OK;
}

}  // namespace mpm
