// Internal declarations shared by the host builders (mpm_host.cpp) and the
// scan kernels (mpm_scan.hip). Not part of the public interface.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mpm.h"

namespace mpm {

// ---------------------------------------------------------------------------
// Kernel-argument descriptors (passed by value)
// ---------------------------------------------------------------------------

// Bytes at the start of a scan kernel's LDS before the matching tables: the
// per-workgroup header (with the id groups below) and the byte-class map.
static const uint32_t LDS_FIXED_BYTES = 1536;

// Distinct strings numbered by their id count: strings below n_single have
// one id (at CSR slot u); then groups k < n of strings sharing a count: group
// k holds strings [u0[k], u0[k + 1]) with cnt[k] ids each, the first one's
// ids from CSR slot off[k]. Strings from u0[n] on (past the groups kept
// here) read the CSR offsets.
static const int ID_GROUPS = 8;
struct IdGroups {
    uint32_t n;
    uint32_t u0[ID_GROUPS + 1];
    uint32_t cnt[ID_GROUPS];
    uint32_t off[ID_GROUPS];
};

// Dense Aho-Corasick table. Row s holds `cp` entries: column 0 is the class of
// bytes that occur in no pattern (always leads to the root), columns 1..cp-1
// the pattern bytes in ascending order. States are numbered breadth-first, so
// the depth-m states (one per distinct pattern string, in ascending string
// order) are the last `n_unique` rows: state s is terminal iff
// s >= first_term, and then u = s - first_term is the string's rank.
struct AcDev {
    const void *dfa;        // uint16 or uint32 entries
    const uint8_t *cls;     // 256 uint16 entries: byte offset of the column within a row
    const uint32_t *uoff;   // n_unique + 1: CSR offsets into uids
    const uint32_t *uids;   // d: ascending pattern ids per distinct string
    uint32_t n_states;
    uint32_t first_term;
    uint32_t cp;            // columns per row
    uint32_t m;
    uint32_t dfa_bytes;     // bytes of the table (multiple of 16)
    uint32_t dupfree;       // every distinct string has exactly one id
    uint32_t n_single;      // distinct strings below this have one id each
    IdGroups grp;           // id count groups of the other strings
    uint32_t hot_states;    // hot placement: rows [0, hot_states) in LDS
    uint32_t hot_bytes;     // bytes of those rows (multiple of 16)
    // Goto rows (same numbering and columns as the table, all-ones for a
    // missing transition) followed by the supply link of every state, for
    // the supply-link walk; go_bytes = 0 when the index has none.
    const void *go;
    uint32_t go_bytes;      // goto rows and supply links (multiple of 16)
    uint32_t sup_off;       // byte offset of the supply links within go
    // Byte classes without a lookup table, usable when the pattern bytes
    // have distinct 3-bit codes (b >> swar_shift) & 7: perm_byte selects, per
    // code, the only byte with that code that is a pattern byte (or a byte
    // whose code differs, for unused codes); perm_col gives its column's byte
    // offset (0 for unused codes). Bytes that are not their code's pattern
    // byte take column 0.
    uint32_t swar_ok;
    uint32_t swar_shift;
    uint32_t perm_byte_lo, perm_byte_hi, perm_col_lo, perm_col_hi;
    // Sets of different lengths: the table is the automaton of the reversed
    // strings, walked from a range's end to its start; a state s >=
    // first_term reports string term_u[s - first_term] (null for one length).
    const uint32_t *term_u;
    uint32_t m_max;         // longest string (m: the shortest)
};

// Wu-Manber tables. Characters map to 2-bit codes (c >> code_shift) & 3; a
// string of k characters hashes to sum_j code(c_j) << 2j (first character
// in the low bits). SHIFT is stored per block hash as a uint16: the shift
// when positive, else 0x8000 | bucket. Bucket b lists, in ascending order,
// the distinct strings whose last block hashes to that value
// (bu[boff[b] .. boff[b+1])), each with a filter key: the hash of the
// key_len characters just before its last block.
struct WmDev {
    const uint8_t *tables;  // shift16 | boff | bkey | bu, contiguous (table_bytes)
    uint32_t off_boff, off_bkey, off_bu;  // byte offsets inside `tables`
    const uint8_t *pats;    // distinct strings, n_unique * m bytes, ascending
    const uint32_t *uoff;
    const uint32_t *uids;
    uint32_t B;
    uint32_t code_shift;
    uint32_t m;
    uint32_t key_len;
    uint32_t table_bytes;
    uint32_t dupfree;
    uint32_t n_single;
    uint32_t shift_bytes;   // bytes of SHIFT at the start of `tables` (multiple of 16)
    IdGroups grp;
    // Sets of different lengths (var != 0): m is the shortest length, the
    // window; string u is pats[upoff[u] .. upoff[u + 1]) and buckets list
    // longer strings first. Null for one length.
    const uint32_t *upoff;
    uint32_t var;
};

// One text of a launch. Tiles of a launch are numbered globally; a text
// owns tiles [tile_begin, tile_begin + ntiles).
struct TextDesc {
    const uint8_t *text;
    uint64_t n;
    mpm_match *out;
    uint64_t cap;
    uint64_t *total;
    uint64_t tile_begin;
    uint64_t ntiles;
};

// Workspace header words (uint32): ticket counter, finished-workgroup
// counter, launch epoch, device error flag. Followed (at byte 64) by one
// uint64 look-back status word per tile, then (256-byte aligned) by the
// staging area: per workgroup, `stage_cap` slots for each of its virtual
// lanes, slot j of virtual lane v at (j * lanes + v), one (position, string)
// pair each. A lane keeps its first occurrences in registers, stages the next
// stage_cap ones there, and walks its range again only past those.
enum { WS_TICKET = 0, WS_DONE = 1, WS_EPOCH = 2, WS_ERR = 3 };
// Device error flag bits.
enum { WS_ERR_LOOKBACK = 1u, WS_ERR_LDS_LAYOUT = 2u };
static const uint64_t WS_HEADER_BYTES = 64;

struct ScanDev {
    TextDesc single;          // used when ntexts == 1
    const TextDesc *multi;    // device array when ntexts > 1
    uint32_t ntexts;
    uint32_t lane_bytes;
    uint64_t ntiles;
    uint32_t *hdr;
    uint64_t *status;
    // The distinct-string -> id CSR copied to LDS at these byte offsets
    // (0: read from global memory), with its word counts.
    uint32_t csr_uoff_lds, csr_uids_lds;
    uint32_t csr_uoff_words, csr_uids_words;
    mpm_match *stage;     // staging area (null when stage_cap is 0)
    uint32_t stage_cap;   // staged occurrences per virtual lane
    uint32_t mark_lds;    // dense output: LDS byte offset of the position marks
};

// Batched launches: one descriptor per text (in queue order) and one per
// index. kind selects the walker; BK_SWAR marks AC byte classes computed in
// registers.
enum {
    BK_AC16_LDS = 0,
    BK_AC16_GLB = 1,
    BK_AC32_GLB = 2,
    BK_WM_LDS = 3,
    BK_WM_GLB = 4,
    BK_AC16_HOT = 5,
    BK_WM_HOT = 6,
    BK_AC32_HOT = 7,
    BK_WALK_MASK = 0x7f,
    BK_SWAR = 0x80
};

struct BatchIndex {
    AcDev ac;
    WmDev wm;
};

struct BatchText {
    TextDesc td;
    uint32_t index;       // into the launch's BatchIndex array
    uint32_t kind;        // BK_*
    uint32_t lane_bytes;
    uint32_t pad;
    float *cost;          // per-request time share and longest chunk (null: not timed)
};

struct BatchDev {
    const BatchText *texts;
    const BatchIndex *idx;
    uint32_t ntexts;
    uint32_t pad;
    uint64_t ntiles;
    uint32_t *hdr;
    uint64_t *status;
    mpm_match *stage;     // staging area (null when stage_cap is 0)
    uint32_t stage_cap;   // staged occurrences per lane
    float us_per_tick;    // microseconds per wall-clock tick (timed requests)
};

// Staged occurrences per lane: single-text scans stage a lane's whole range
// when the workspace allows; batched launches (many workspaces at once)
// stage at most this many.
static const uint32_t BATCH_STAGE_CAP = 16;

// Look-back status word: [63:38] epoch, [37:36] flag, [35:0] value.
static const uint64_t ST_VAL_BITS = 36;
static const uint64_t ST_VAL_MASK = (1ull << ST_VAL_BITS) - 1;
static const uint32_t ST_EPOCH_MASK = (1u << 26) - 1;

}  // namespace mpm

// ---------------------------------------------------------------------------
// Host-side index
// ---------------------------------------------------------------------------
struct mpm_index {
    uint32_t algo = 0;
    uint32_t m = 0, d = 0, du = 0, max_dup = 0;
    uint32_t n_single = 0;              // distinct strings 0..n_single-1 have one id each
    std::vector<uint32_t> uoff, uids;   // distinct strings -> ids
    // Strings from n_single on come in groups sharing an id count: group k
    // starts at string grp_u0[k], its strings have grp_cnt[k] ids each, and
    // its first string's ids start at grp_off[k].
    std::vector<uint32_t> grp_u0, grp_cnt, grp_off;
    std::vector<uint8_t> upats;         // du * m, ascending strings
    // Sets of different lengths (var): m is the shortest length, m_max the
    // longest; string u is upats[upoff[u] .. upoff[u + 1]) and its id list
    // holds the ids of every pattern that is a prefix of it (those occur
    // wherever it does).
    uint32_t var = 0, m_max = 0;
    std::vector<uint32_t> upoff;
    std::vector<uint8_t> wpats;         // Wu-Manber: first m bytes of every string

    // Aho-Corasick
    uint32_t n_classes = 0;
    uint8_t class_bytes[256] = {0};
    uint16_t cls[256] = {0};         // byte -> 1 + class (0: in no pattern); up to 256 classes
    uint32_t swar_ok = 0, swar_shift = 0;
    uint8_t perm_byte[8] = {0}, perm_col[8] = {0};
    uint64_t n_states = 0;
    uint32_t state_bytes = 0;
    std::vector<uint32_t> dfa;          // n_states * (1 + n_classes)
    uint64_t first_term = 0;            // var: states from here on report a string
    std::vector<uint32_t> term_u;       // var: the string each reporting state reports

    // Wu-Manber
    uint32_t B = 0, code_shift = 0, zero_shift = 0, n_buckets = 0, key_len = 0;
    double mean_shift = 0;
    std::vector<uint8_t> shift;       // SHIFT per block hash
    std::vector<uint16_t> shift16;    // SHIFT, or 0x8000 | bucket when zero
    std::vector<uint32_t> boff, bu, bkey;

    // Device image: host copy, offsets, and the caller-owned device buffer.
    std::vector<uint8_t> image;
    uint64_t off_a = 0, off_b = 0, off_c = 0, off_d = 0, off_e = 0, off_f = 0, off_g = 0, off_h = 0;
    // Aho-Corasick goto rows and supply links (kept when asked for)
    uint32_t keep_goto = 0;
    uint64_t off_go = 0, go_bytes = 0, sup_off = 0;
    uint64_t table_bytes = 0;
    const uint8_t *d_image = nullptr;
};

namespace mpm {
void set_error(const char *fmt, ...);
mpm_status fail(mpm_status st, const char *fmt, ...);

// Launch the scan kernels (mpm_scan.hip).
struct LaunchCfg {
    uint32_t lane_bytes;
    uint32_t block_threads;
    uint32_t placement;   // resolved: LDS or GLOBAL
    uint32_t grid;        // resolved workgroup count
    uint32_t lds_bytes;   // dynamic LDS per workgroup
    bool swar;            // AC: byte classes computed in registers
    bool supply;          // AC: goto function and supply links at run time
    uint32_t ilp;         // virtual lanes per thread (1 or 2)
    uint32_t csr_lds;     // LDS byte offset of the id CSR (0: global memory)
    bool dense;           // dense output (position marks in LDS)
    uint32_t mark_lds;    // LDS byte offset of the marks (dense)
    uint32_t text_mode;   // 0: line streaming; 1: bytes from global; 2: text staged in LDS
    uint32_t text_lds;    // text_mode 2: LDS byte offset of the staged text
};
// LDS bytes of the dense output's position marks (1024 lanes x 16 positions).
static const uint32_t DENSE_MARK_BYTES = 1024 * 16 * 4;
// csr_in_lds: single-text scans may copy the id CSR to LDS (batched launches
// keep it in global memory).
mpm_status resolve_variant(const mpm_index *idx, const mpm_variant *v, uint64_t ntiles_hint,
                           LaunchCfg *cfg, bool csr_in_lds = false);
// Words of the id CSR arrays: uoff (d_unique + 1) and ids (d), each padded
// to 16 bytes.
uint32_t csr_uoff_words(const mpm_index *idx);
uint32_t csr_uids_words(const mpm_index *idx);
uint64_t tile_bytes(const LaunchCfg &cfg);
mpm_status launch_scan(const mpm_index *idx, const LaunchCfg &cfg, const ScanDev &sd,
                       void *stream);
mpm_status launch_zero_totals(uint64_t *const *d_totals_dev, uint32_t count, uint64_t *single,
                              void *stream);
// reserve: LDS bytes the launch keeps beside the tables (the hot part of an
// Aho-Corasick table shrinks by as much).
AcDev ac_dev(const mpm_index *ix, uint32_t reserve = 0);
WmDev wm_dev(const mpm_index *ix);
// Sets of different lengths (mpm_mixed.cpp, mpm_scan_var.hip).
mpm_status build_ac_rev_tables(mpm_index *ix);
const void *var_kernel(const mpm_index *ix, const LaunchCfg &c);
mpm_status var_launch(const mpm_index *ix, const LaunchCfg &c, const ScanDev &sd, void *stream);
// Text-access ladder variants (mpm_scan_ladder.hip).
const void *ladder_kernel(const mpm_index *ix, const LaunchCfg &c);
mpm_status ladder_launch(const mpm_index *ix, const LaunchCfg &c, const ScanDev &sd, void *stream);
uint32_t batch_kind(const mpm_index *ix, const LaunchCfg &c);
// Batched launches run one kernel per walker kind (BK_*, with BK_SWAR).
uint32_t batch_grid(uint32_t kind, uint32_t W, uint32_t lds_bytes, uint64_t ntiles,
                    uint32_t grid_req);
mpm_status launch_batch(const BatchDev &bd, uint32_t kind, uint32_t W, uint32_t grid, uint32_t lds,
                        void *stream);
}  // namespace mpm
