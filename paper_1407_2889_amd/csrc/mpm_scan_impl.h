// Scan kernels for gfx950 (CDNA4, wave64).
//
// Decomposition (the paper's data-parallel strategy, Section 4.2.1, recast
// for CDNA): the starting positions of a text are cut into chunks of
// block_threads * lane_bytes positions. A persistent grid of workgroups takes
// chunks in ascending order from an atomic ticket counter. Inside a chunk,
// lane k owns lane_bytes consecutive starting positions and reads m - 1 bytes
// beyond them (the overlap of Section 4.2.1), so every occurrence is found by
// exactly one lane: the lane whose range holds its start.
//
// Each chunk runs three phases:
//   A. every lane walks its range, counts the pattern ids it must report and
//      keeps its first few occurrences in registers;
//   B. a workgroup prefix sum orders the lanes' counts, and a decoupled
//      look-back over the previous chunks' published counts gives the chunk's
//      offset in the text's output, so the global list comes out sorted with
//      no sort pass (the paper sums per-thread counts on the host, Section 6,
//      GPU-U stage; here the sum becomes the output offset);
//   C. lanes write their (position, id) pairs at their offsets; a lane with
//      more occurrences than its registers hold walks its range again.
//
// Walkers:
//   AC - one dependent lookup per byte in the dense table (Section 3.1, array
//        form of the goto function with supply transitions precomputed); the
//        table sits in LDS when it fits, else its first (shallow) rows do and
//        the rest is read through the caches, else all of it is read through
//        the caches. Each lane streams its text as whole 128-byte lines of
//        16-byte loads, the next line in flight while the current one is
//        walked (the paper stages text in shared memory, Section 4.2.2; on
//        this hardware a lane's own whole-line loads move full cache lines and
//        LDS is left to the table).
//   WM - each lane runs the Wu-Manber window loop (Section 3.2, Algorithm 5)
//        over its window ends on a history of 2-bit character codes held in
//        registers, with SHIFT in LDS (or read through the caches), and
//        verifies candidate windows against the bucket (HASH), a filter key
//        (PREFIX) and the pattern bytes.
#pragma once
#include <hip/hip_runtime.h>

#include <string.h>

#include <type_traits>

#include "mpm_internal.h"

namespace mpm {

// Address-space qualified pointers: LDS tables must be read with ds_read and
// global data with global_load (a generic pointer would give flat loads).
#define LDS_AS __attribute__((address_space(3)))
#define GLB_AS __attribute__((address_space(1)))
template <typename T> using lds_cptr = const LDS_AS T *;
template <typename T> using glb_cptr = const GLB_AS T *;
template <bool InLds, typename T> struct TabPtr { using type = glb_cptr<T>; };
// Table placements of the walkers: global memory, wholly in LDS, or the hot
// part in LDS and the rest in global memory.
enum { PL_GLB = 0, PL_LDS = 1, PL_HOT = 2 };
typedef uint32_t v4u __attribute__((ext_vector_type(4)));  // 16-byte load/store unit
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));  // two 16-bit states
template <typename T> struct TabPtr<true, T> { using type = lds_cptr<T>; };

static const int K_SLOTS = 2;  // occurrences a lane keeps in registers (more are staged)

// Dynamic LDS layout. The scan kernels declare no static LDS, so their
// dynamic allocation starts at LDS address 0 (checked at kernel start) and
// every region sits at a constant address: table reads then need no base
// register, the constant goes into the ds_read offset field.
static const uint32_t LDS_HDR_OFF = 0;     // LdsHdr: per-workgroup scalars
static const uint32_t LDS_CLS_OFF = 1024;  // AC: column byte offset per byte value
static const uint32_t LDS_TAB_OFF = 1536;  // matching tables (LDS placement)
static_assert(LDS_TAB_OFF == LDS_FIXED_BYTES, "LDS layout and its host-side size disagree");

template <typename T>
__device__ __forceinline__ LDS_AS T *lds_at(uint32_t off)
{
    return (LDS_AS T *)(uintptr_t)off;
}

static const int LDS_SCAN_WORDS = 2 * (1024 / 64) + 1;  // chunk_offsets words, at most

struct LdsHdr {
    uint64_t scan[LDS_SCAN_WORDS];
    uint64_t tile;   // chunk ticket of the workgroup's current chunk
    uint32_t epoch;  // launch epoch
    uint32_t pad;
    TextDesc td;     // the current chunk's text (single-index kernel)
    BatchText bt;    // the current chunk's text (batched kernel)
    IdGroups grp;    // id count groups of the current index
};
static_assert(sizeof(LdsHdr) <= LDS_CLS_OFF - LDS_HDR_OFF, "LDS header overflows its region");

// Whether the kernel's dynamic LDS starts at address 0. If not (static LDS
// appeared in the kernel), flag a device error and let every workgroup return
// before taking a ticket, so the workspace stays clean.
__device__ __forceinline__ bool lds_layout_ok(uint8_t *smem, uint32_t *hdr)
{
    if ((uint32_t)(uintptr_t)(LDS_AS uint8_t *)smem == 0u)
        return true;
    if (threadIdx.x == 0)
        atomicOr(&hdr[WS_ERR], WS_ERR_LDS_LAYOUT);
    return false;
}

// A uniform value kept in a VGPR (v_perm takes at most one SGPR operand, so
// its table words are held in VGPRs once instead of being copied per use).
__device__ __forceinline__ uint32_t in_vgpr(uint32_t x)
{
    uint32_t r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
    return r;
}
static const uint32_t SPIN_LIMIT = 1u << 24;

// The same value, hidden from the optimizer. A walk repeated to report its
// occurrences starts from an opaque copy of its first state: otherwise the
// compiler proves that it retraces the first walk and keeps that walk's states
// (one per byte) for it instead, which costs far more registers than the
// rare second walk costs time.
__device__ __forceinline__ uint32_t opaque(uint32_t x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// ---------------------------------------------------------------------------
// Look-back status words
// ---------------------------------------------------------------------------
// A status word carries its flag and its value together, so no other memory
// is published through it: relaxed device-coherent atomics suffice. (Acquire
// or release at device scope would write back or invalidate the L2 of every
// chunk's XCD, which costs far more than the scan of a chunk.)
__device__ __forceinline__ uint64_t ld_status(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_status(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t make_status(uint32_t epoch, uint32_t flag, uint64_t val)
{
    return ((uint64_t)(epoch & ST_EPOCH_MASK) << 38) | ((uint64_t)flag << ST_VAL_BITS) |
           (val & ST_VAL_MASK);
}

// Publish this chunk's count and return the sum of all earlier chunks of the
// same text (decoupled look-back). flag 1: this chunk's count only; flag 2:
// inclusive prefix. Run by the 64 lanes of wave 0: each probe reads the 64
// preceding status words at once and stops at the nearest inclusive one.
// Chunks before the text's first chunk count as an inclusive zero.
__device__ __forceinline__ uint64_t look_back(uint64_t *status, uint64_t g, uint64_t first_g, uint64_t agg,
                              uint32_t epoch, uint32_t *err)
{
    const int lane = threadIdx.x & 63;
    if (g == first_g) {
        if (lane == 0)
            st_status(&status[g], make_status(epoch, 2, agg));
        return 0;
    }
    if (lane == 0)
        st_status(&status[g], make_status(epoch, 1, agg));
    const uint64_t tag = epoch & ST_EPOCH_MASK;
    uint64_t excl = 0;
    int64_t top = (int64_t)g - 1;  // status index probed by lane 0
    uint32_t spins = 0;
    while (true) {
        const int64_t j = top - lane;
        uint32_t fl = 2;
        uint64_t val = 0;
        if (j >= (int64_t)first_g) {
            const uint64_t v = ld_status(&status[j]);
            fl = ((v >> 38) == tag) ? ((uint32_t)(v >> ST_VAL_BITS) & 3u) : 0u;
            val = v & ST_VAL_MASK;
        }
        const uint64_t ready = __ballot(fl != 0);
        const uint64_t incl = __ballot(fl == 2);
        const int k = incl ? __ffsll((long long)incl) - 1 : 64;      // nearest inclusive lane
        const uint64_t need = k >= 63 ? ~0ull : ((2ull << k) - 1);   // lanes 0..k
        if ((ready & need) != need) {
            if (++spins > SPIN_LIMIT) {  // never expected; keeps every wave finite
                if (lane == 0)
                    atomicOr(err, (uint32_t)WS_ERR_LOOKBACK);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        uint64_t x = lane <= k ? val : 0;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
            x += __shfl_xor(x, o, 64);
        excl += x;
        if (k < 64)
            break;
        top -= 64;
    }
    if (lane == 0)
        st_status(&status[g], make_status(epoch, 2, excl + agg));
    return excl;
}

// Exclusive prefix sum of c over the lanes of a wave, and the wave's total,
// one bit plane at a time: each plane is a ballot whose lanes below this one
// are counted by mbcnt. As many planes as the largest c has bits (one when
// every c is 0 or 1), each a few ALU instructions, where a shuffle scan
// waits out six LDS-crossbar round trips.
__device__ __forceinline__ uint32_t wave_excl_sum(uint32_t c, uint32_t &total)
{
    uint32_t pre = 0, tot = 0;
#pragma unroll 1
    for (uint32_t b = 0; b < 32; ++b) {
        const uint64_t bal = __ballot((c >> b) & 1u);
        const uint32_t below =
            __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        pre += below << b;
        tot += (uint32_t)__popcll(bal) << b;
        if (b == 31 || __ballot((c >> (b + 1)) != 0u) == 0)
            break;
    }
    total = tot;
    return pre;
}

// Offsets of a chunk's virtual lanes in the text's output. A chunk holds
// I * W virtual lanes in text order; lane t runs virtual lanes t, t + W, ...
// cnt[v] is the number of pairs of this lane's v-th virtual lane; ob[v]
// receives its first output index. s_scan holds I * (W / 64) + 1 words.
template <int W, int I>
__device__ __forceinline__ void chunk_offsets(const uint32_t (&cnt)[I], uint64_t (&ob)[I],
                                              uint64_t *s_scan, uint64_t *status, uint64_t g,
                                              uint64_t first_g, bool last, uint64_t *total,
                                              uint32_t epoch, uint32_t *err)
{
    constexpr int NW = W / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x[I], tot[I];  // exclusive prefix within the wave, wave total
#pragma unroll
    for (int v = 0; v < I; ++v)
        x[v] = wave_excl_sum(cnt[v], tot[v]);
    if (lane == 0) {
#pragma unroll
        for (int v = 0; v < I; ++v)
            s_scan[v * NW + wave] = tot[v];
    }
    __syncthreads();
    if (wave == 0) {
        uint64_t run = 0;
        for (int w = 0; w < I * NW; ++w)
            run += s_scan[w];
        const uint64_t excl = look_back(status, g, first_g, run, epoch, err);
        if (lane == 0) {
            uint64_t r = 0;
            for (int w = 0; w < I * NW; ++w) {
                const uint64_t t = s_scan[w];
                s_scan[w] = r;
                r += t;
            }
            s_scan[I * NW] = excl;
            if (last)
                *total = excl + run;
        }
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < I; ++v)
        ob[v] = s_scan[I * NW] + s_scan[v * NW + wave] + x[v];
}

typedef uint32_t v2u __attribute__((ext_vector_type(2)));

// The distinct-string -> id CSR (uoff, ids), read from LDS when the launch
// copied it there (nonzero byte offsets) and from global memory otherwise.
struct IdMap {
    glb_cptr<uint32_t> uoff, uids;
    uint32_t lds_uoff, lds_uids;
    uint32_t dupfree;
    uint32_t n_single;  // strings below this have one id: no CSR read to count

    __device__ __forceinline__ uint32_t off(uint32_t u) const
    {
        return lds_uoff ? lds_at<const uint32_t>(lds_uoff)[u] : uoff[u];
    }
    __device__ __forceinline__ uint32_t id(uint32_t j) const
    {
        return lds_uids ? lds_at<const uint32_t>(lds_uids)[j] : uids[j];
    }
    // CSR slots [b, e) of the ids of distinct string u: for strings in an id
    // count group (the LDS header's copy of the index's groups) by
    // arithmetic, otherwise from the CSR offsets.
    __device__ __forceinline__ void span(uint32_t u, uint32_t &b, uint32_t &e) const
    {
        if (u < n_single) {
            b = u;
            e = u + 1;
            return;
        }
        const LDS_AS IdGroups *g = lds_at<const IdGroups>(LDS_HDR_OFF + offsetof(LdsHdr, grp));
        if (u < g->u0[g->n]) {
            // groups ascend and u0[n] bounds u: the scan stops at a group
            uint32_t k = 0;
#pragma unroll 1
            while (u >= g->u0[k + 1])
                ++k;
            const uint32_t c = g->cnt[k];
            b = g->off[k] + (u - g->u0[k]) * c;
            e = b + c;
            return;
        }
        b = off(u);
        e = off(u + 1);
    }
    // ids reported for one occurrence of distinct string u
    __device__ __forceinline__ uint32_t count(uint32_t u) const
    {
        uint32_t b, e;
        span(u, b, e);
        return e - b;
    }
};

// Copy an index's id count groups into the LDS header (no barrier).
__device__ __forceinline__ void load_groups(const IdGroups &src)
{
    constexpr int NW = (int)(sizeof(IdGroups) / 4);
    LDS_AS uint32_t *d = lds_at<uint32_t>(LDS_HDR_OFF + offsetof(LdsHdr, grp));
    const uint32_t *s = (const uint32_t *)&src;
    if (threadIdx.x < (uint32_t)NW)
        d[threadIdx.x] = s[threadIdx.x];
}

__device__ __forceinline__ void write_ids(mpm_match *out_, uint64_t cap, uint64_t &ob, uint32_t pos,
                                          uint32_t u, const IdMap &im)
{
    GLB_AS v2u *out = (GLB_AS v2u *)out_;
    if (u < im.n_single) {  // one id, at CSR slot u (single-id strings come first)
        if (ob < cap)
            out[ob] = v2u{pos, im.id(u)};
        ++ob;
        return;
    }
    uint32_t b, e;
    im.span(u, b, e);
    for (uint32_t j = b; j < e; ++j) {
        if (ob < cap)
            out[ob] = v2u{pos, im.id(j)};
        ++ob;
    }
}

// Cooperative global -> LDS copy (bytes multiple of 16, both 16-aligned).
template <int W>
__device__ __forceinline__ void copy_to_lds(uint32_t dst, const uint8_t *src, uint32_t bytes)
{
    glb_cptr<v4u> s = (glb_cptr<v4u>)src;
    LDS_AS v4u *d = lds_at<v4u>(dst);
    const uint32_t n = bytes / 16;
    uint32_t k = threadIdx.x;
    // four loads in flight per thread before their stores
    for (; k + 3 * W < n; k += 4 * W) {
        const v4u a = s[k], b = s[k + W], c = s[k + 2 * W], e = s[k + 3 * W];
        d[k] = a;
        d[k + W] = b;
        d[k + 2 * W] = c;
        d[k + 3 * W] = e;
    }
    for (; k < n; k += W)
        d[k] = s[k];
}

// Stream bytes [p, end) of a text through registers: single bytes up to a
// 16-byte boundary, 16-byte pieces up to a 128-byte (cache line) boundary,
// then whole lines (eight 16-byte loads issued together, the next line's
// loads issued before the current one is consumed), then 16-byte pieces, then
// bytes. Reading whole lines matters: with a thousand lanes per CU streaming
// separate ranges, a line read in two halves is often evicted from L2 between
// them and fetched from HBM twice. one(byte, pos) and sixteen(v4u, pos)
// consume in text order.
// prep(v4u) turns 16 loaded bytes into whatever the consumer keeps (the bytes
// themselves, or something smaller); it runs on a whole line as soon as the
// line is consumed, so only the prepared form stays live next to the
// in-flight loads of the following line.
template <class F1, class FP, class FU>
__device__ __forceinline__ void stream_text(glb_cptr<uint8_t> text, uint64_t p, uint64_t end,
                                            F1 &&one, FP &&prep, FU &&use)
{
    while (p < end && (((uintptr_t)(text + p)) & 15u)) {
        one((uint32_t)text[p], p);
        ++p;
    }
    while (p + 16 <= end && (((uintptr_t)(text + p)) & 127u)) {
        use(prep(*(glb_cptr<v4u>)(text + p)), p);
        p += 16;
    }
    if (p + 128 <= end) {
        v4u c[8];
        {
            glb_cptr<v4u> q = (glb_cptr<v4u>)(text + p);
#pragma unroll
            for (int j = 0; j < 8; ++j)
                c[j] = q[j];
        }
        while (true) {
            decltype(prep(c[0])) t[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                t[j] = prep(c[j]);
            const bool more = p + 256 <= end;
            glb_cptr<v4u> nq = (glb_cptr<v4u>)(text + (more ? p + 128 : p));
            v4u nx[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                nx[j] = nq[j];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                use(t[j], p + 16 * j);
            p += 128;
            if (!more)
                break;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                c[j] = nx[j];
        }
    }
    while (p + 16 <= end) {
        use(prep(*(glb_cptr<v4u>)(text + p)), p);
        p += 16;
    }
    while (p < end) {
        one((uint32_t)text[p], p);
        ++p;
    }
}

template <class F1, class F16>
__device__ __forceinline__ void stream_text(glb_cptr<uint8_t> text, uint64_t p, uint64_t end,
                                            F1 &&one, F16 &&sixteen)
{
    stream_text(text, p, end, one, [](const v4u c) { return c; }, sixteen);
}

// ---------------------------------------------------------------------------
// Aho-Corasick walker
// ---------------------------------------------------------------------------
// Column byte offsets of four text bytes at once (Swar variant): 3-bit codes
// pick each byte's expected pattern byte and column through v_perm; a SWAR
// zero-byte test sends every byte that is not its code's pattern byte to
// column 0 (the root).
__device__ __forceinline__ uint32_t swar_cols(uint32_t w, uint32_t sh, uint32_t pb_lo,
                                              uint32_t pb_hi, uint32_t pc_lo, uint32_t pc_hi)
{
    const uint32_t code = (w >> sh) & 0x07070707u;
    const uint32_t expect = __builtin_amdgcn_perm(pb_hi, pb_lo, code);
    const uint32_t col = __builtin_amdgcn_perm(pc_hi, pc_lo, code);
    const uint32_t x = w ^ expect;
    const uint32_t nz = (((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;  // bit 7: byte != 0
    return col & ~(nz | (nz - (nz >> 7)));  // 0xFF in every byte != 0
}

template <typename St, int P, bool Swar, int Ilp>
struct AcWalk {
    using Dev = AcDev;
    static constexpr int ILP = Ilp;
    static constexpr bool DESC = false;  // reports starts in ascending order
    static constexpr bool STAGE = false;  // reads text through registers
    static constexpr bool InLds = P == PL_LDS;
    // PL_HOT: states below hot (the first rows in breadth-first order, where
    // a walk over text spends nearly all its steps) are read from LDS, the
    // others from global memory.
    static constexpr bool Hot = P == PL_HOT;
    typename TabPtr<InLds, uint8_t>::type dfab;  // table, addressed in bytes
    lds_cptr<uint16_t> cls;                      // column byte offset per byte value
    uint32_t rowb, first_term, m, sh, pb_lo, pb_hi, pc_lo, pc_hi, hot;

    // Copy what this walker reads from LDS (no barrier).
    template <int W>
    __device__ __forceinline__ static void load(const AcDev &a)
    {
        copy_to_lds<W>(LDS_CLS_OFF, a.cls, 512);
        if (InLds)
            copy_to_lds<W>(LDS_TAB_OFF, (const uint8_t *)a.dfa, a.dfa_bytes);
        if (Hot)
            copy_to_lds<W>(LDS_TAB_OFF, (const uint8_t *)a.dfa, a.hot_bytes);
    }

    __device__ __forceinline__ void bind(const AcDev &a)
    {
        rowb = a.cp * (uint32_t)sizeof(St);
        first_term = a.first_term;
        m = a.m;
        sh = a.swar_shift;
        pb_hi = a.perm_byte_hi;
        pc_hi = a.perm_col_hi;
        if (Swar) {
            pb_lo = in_vgpr(a.perm_byte_lo);
            pc_lo = in_vgpr(a.perm_col_lo);
        } else {
            pb_lo = a.perm_byte_lo;
            pc_lo = a.perm_col_lo;
        }
        cls = lds_at<const uint16_t>(LDS_CLS_OFF);
        if constexpr (InLds)
            dfab = lds_at<const uint8_t>(LDS_TAB_OFF);
        else
            dfab = (glb_cptr<uint8_t>)a.dfa;
        hot = a.hot_states;
    }

    template <int W>
    __device__ __forceinline__ void setup(const AcDev &a, uint32_t /*unused*/)
    {
        load<W>(a);
        bind(a);
        __syncthreads();
    }

    // One transition: row s, column at byte offset coloff.
    __device__ __forceinline__ uint32_t next(uint32_t s, uint32_t coloff) const
    {
        const uint32_t off = sizeof(St) == 2 ? __umul24(s, rowb) + coloff : s * rowb + coloff;
        if constexpr (Hot) {
            if (s < hot)
                return *(lds_cptr<St>)(lds_at<const uint8_t>(LDS_TAB_OFF) + off);
        }
        return *(typename TabPtr<InLds, St>::type)(dfab + off);
    }

    // Byte-offset columns of the 16 bytes of c. Swar: when every byte is its
    // code's expected byte (the usual case: the expected byte of a code is
    // its pattern byte, or for codes of no pattern byte a likely separator),
    // the columns are one v_perm per word; otherwise the exact per-byte test
    // sends unexpected bytes to column 0.
    __device__ __forceinline__ void cols16(const v4u c, uint32_t (&cw)[4]) const
    {
        if (Swar) {
            const uint32_t k0 = (c.x >> sh) & 0x07070707u, k1 = (c.y >> sh) & 0x07070707u;
            const uint32_t k2 = (c.z >> sh) & 0x07070707u, k3 = (c.w >> sh) & 0x07070707u;
            const uint32_t miss = (c.x ^ __builtin_amdgcn_perm(pb_hi, pb_lo, k0)) |
                                  (c.y ^ __builtin_amdgcn_perm(pb_hi, pb_lo, k1)) |
                                  (c.z ^ __builtin_amdgcn_perm(pb_hi, pb_lo, k2)) |
                                  (c.w ^ __builtin_amdgcn_perm(pb_hi, pb_lo, k3));
            if (__builtin_expect(miss != 0, 0)) {
                cw[0] = swar_cols(c.x, sh, pb_lo, pb_hi, pc_lo, pc_hi);
                cw[1] = swar_cols(c.y, sh, pb_lo, pb_hi, pc_lo, pc_hi);
                cw[2] = swar_cols(c.z, sh, pb_lo, pb_hi, pc_lo, pc_hi);
                cw[3] = swar_cols(c.w, sh, pb_lo, pb_hi, pc_lo, pc_hi);
            } else {
                cw[0] = __builtin_amdgcn_perm(pc_hi, pc_lo, k0);
                cw[1] = __builtin_amdgcn_perm(pc_hi, pc_lo, k1);
                cw[2] = __builtin_amdgcn_perm(pc_hi, pc_lo, k2);
                cw[3] = __builtin_amdgcn_perm(pc_hi, pc_lo, k3);
            }
        } else {
            cw[0] = c.x;
            cw[1] = c.y;
            cw[2] = c.z;
            cw[3] = c.w;
        }
    }

    __device__ __forceinline__ uint32_t col_of(const uint32_t (&cw)[4], int k) const
    {
        const uint32_t byte = (cw[k >> 2] >> (8 * (k & 3))) & 0xffu;
        return Swar ? byte : (uint32_t)cls[byte];
    }

    template <class F>
    __device__ __forceinline__ void report16(const uint32_t (&st)[16], uint32_t mx, uint64_t q,
                                             F &cb) const
    {
        if (mx >= first_term) {
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (st[k] >= first_term)
                    cb(q + k + 1 - m, st[k] - first_term);
        }
    }

    // Continue a walk in state s over bytes [p, end); cb(start, u) for every
    // terminal state reached (start = index of the byte - m + 1).
    template <class F>
    __device__ __forceinline__ void walk_from(uint32_t &s, glb_cptr<uint8_t> text, uint64_t p,
                                              uint64_t end, F &cb) const
    {
        stream_text(
            text, p, end,
            [&](uint32_t b, uint64_t q) {
                s = next(s, cls[b]);
                if (s >= first_term)
                    cb(q + 1 - m, s - first_term);
            },
            [&](const v4u c, uint64_t q) {
                uint32_t cw[4];
                cols16(c, cw);
                uint32_t st[16];
                uint32_t mx = 0;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    s = next(s, col_of(cw, k));
                    st[k] = s;
                    mx = max(mx, s);
                }
                report16(st, mx, q, cb);
            });
    }

    template <class F>
    __device__ __forceinline__ void walk(glb_cptr<uint8_t> text, uint64_t p, uint64_t end,
                                         F &cb) const
    {
        uint32_t s = 0;
        walk_from(s, text, p, end, cb);
    }

    // Steps of one 16-byte piece whose column words are cw, from state s:
    // returns the largest state reached (a terminal state shows as a value
    // >= first_term), s is left at the state after the piece.
    __device__ __forceinline__ uint32_t steps16(uint32_t &s, const uint32_t (&cw)[4]) const
    {
        uint32_t mx = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            s = next(s, col_of(cw, k));
            mx = max(mx, s);
        }
        return mx;
    }

    // The first cnt bytes of a piece again from state s, reporting every
    // terminal state (q = text position of the piece's first byte). Runs only
    // for pieces that reached a terminal state.
    template <class F>
    __device__ __forceinline__ void report_piece(uint32_t s, const uint32_t (&cw)[4], uint32_t cnt,
                                                 uint64_t q, F &cb) const
    {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if ((uint32_t)k < cnt) {
                s = next(s, col_of(cw, k));
                if (s >= first_term)
                    cb(q + k + 1 - m, s - first_term);
            }
        }
    }

    // Column byte offset of byte k of a piece packed as two words of
    // nibbles: word k >> 3, bytes 0-3 of the word's half in the low nibbles,
    // bytes 4-7 in the high nibbles.
    __device__ __forceinline__ static uint32_t col_nib(uint32_t p0, uint32_t p1, int k)
    {
        const uint32_t w = k < 8 ? p0 : p1;
        const int kk = k & 7;
        return (w >> (8 * (kk & 3) + 4 * (kk >> 2))) & 15u;
    }

    // Steps of a packed piece from state s (as steps16).
    __device__ __forceinline__ uint32_t steps_nib(uint32_t &s, uint32_t p0, uint32_t p1) const
    {
        uint32_t mx = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            s = next(s, col_nib(p0, p1, k));
            mx = max(mx, s);
        }
        return mx;
    }

    // The first cnt bytes of a packed piece from state s (left at the state
    // after them), reporting every terminal state (q = text position of the
    // piece's first byte).
    template <class F>
    __device__ __forceinline__ void report_nib(uint32_t &s, uint32_t p0, uint32_t p1, uint32_t cnt,
                                               uint64_t q, F &cb) const
    {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if ((uint32_t)k < cnt) {
                s = next(s, col_nib(p0, p1, k));
                if (s >= first_term)
                    cb(q + k + 1 - m, s - first_term);
            }
        }
    }

    // I walks in lockstep over whole 128-byte lines (I independent lookup
    // chains per lane). Walk c covers bytes [p[c], e[c]); every p[c] is
    // 128-byte aligned in memory. Each walk keeps two lines: the one being
    // walked, its 128 column offsets packed as nibbles (16 registers), and
    // the next one in flight as raw bytes (32 registers), requested as a
    // whole line with eight back-to-back 16-byte loads: lines whose pieces
    // are requested far apart are evicted from L2 between requests and
    // fetched from HBM again. With one walk, the first bytes past the common
    // lines (the m - 1 overlap into the next lane's range, which that lane
    // reads at its start) are loaded with the first line, from the same
    // cache line fill, instead of by a second fetch at the end.
    // cb(c, start, u) reports an occurrence found by walk c.
    template <int I, class F>
    __device__ __forceinline__ void walk_lines(glb_cptr<uint8_t> text, uint64_t n,
                                               const uint64_t (&p)[I], const uint64_t (&e)[I],
                                               F &cb) const
    {
        static_assert(Swar && sizeof(St) == 2, "walk_lines packs 4-bit column offsets");
        constexpr int NT = I == 1 ? 2 : 0;  // tail pieces loaded up front
        uint64_t common = e[0] - p[0];
#pragma unroll
        for (int c = 1; c < I; ++c)
            common = min(common, e[c] - p[c]);
        const uint32_t nl = (uint32_t)(common >> 7);
        uint32_t s[I];
        v4u raw[I][8];
        uint32_t cur[I][16];
        v4u tail[I][NT > 0 ? NT : 1];
        auto pack = [&](int c) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                uint32_t cw[4];
                cols16(raw[c][j], cw);
                cur[c][2 * j] = cw[0] | (cw[1] << 4);
                cur[c][2 * j + 1] = cw[2] | (cw[3] << 4);
            }
        };
        auto fetch = [&](int c, uint32_t l) {
            glb_cptr<v4u> q = (glb_cptr<v4u>)(text + p[c] + ((uint64_t)l << 7));
#pragma unroll
            for (int j = 0; j < 8; ++j)
                raw[c][j] = q[j];
        };
#pragma unroll
        for (int c = 0; c < I; ++c) {
            s[c] = 0;
            fetch(c, 0);
            const uint64_t t0 = p[c] + ((uint64_t)nl << 7);
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const uint64_t tq = t0 + 16 * j;
                tail[c][j] = (tq < e[c] && tq + 16 <= n) ? *(glb_cptr<v4u>)(text + tq) : v4u{0, 0, 0, 0};
            }
        }
        // One walk double-buffers: the next line is in flight while the
        // current one is walked. Several walks fetch their next lines only
        // once the current ones are done and wait for them (the other waves
        // of the CU cover the wait): the registers of a second line per walk
        // would not fit.
        constexpr bool DB = I == 1;
#pragma unroll
        for (int c = 0; c < I; ++c) {
            pack(c);
            if (DB)
                fetch(c, nl > 1 ? 1 : 0);
        }
        for (uint32_t l = 0; l < nl; ++l) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if constexpr (I == 1) {
                    // The piece's 16 states, packed in pairs of 16 bits (the
                    // table has fewer than 2^16 states), with their running
                    // maximum per half: a piece that reached a terminal state
                    // is reported from these, without walking it again
                    // (which would cost the whole wave a second chain of
                    // lookups whenever any of its lanes had a hit).
                    u16x2 pk[8];
                    u16x2 mxp = {0, 0};
                    uint32_t prev = 0;
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        s[0] = next(s[0], col_nib(cur[0][2 * j], cur[0][2 * j + 1], k));
                        if (k & 1) {
                            // low halves of both states (they are below 2^16)
                            pk[k >> 1] = __builtin_bit_cast(
                                u16x2, __builtin_amdgcn_perm(s[0], prev, 0x05040100u));
                            mxp = __builtin_elementwise_max(mxp, pk[k >> 1]);
                        } else {
                            prev = s[0];
                        }
                    }
                    if ((uint32_t)max(mxp.x, mxp.y) >= first_term) {
                        const uint64_t q = p[0] + ((uint64_t)l << 7) + 16 * j;
#pragma unroll
                        for (int k = 0; k < 16; ++k) {
                            const uint32_t st = (k & 1) ? pk[k >> 1].y : pk[k >> 1].x;
                            if (st >= first_term)
                                cb(0, q + k + 1 - m, st - first_term);
                        }
                    }
                } else {
                    uint32_t s0[I], mx[I];
#pragma unroll
                    for (int c = 0; c < I; ++c) {
                        s0[c] = s[c];
                        mx[c] = 0;
                    }
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
#pragma unroll
                        for (int c = 0; c < I; ++c) {
                            s[c] = next(s[c], col_nib(cur[c][2 * j], cur[c][2 * j + 1], k));
                            mx[c] = max(mx[c], s[c]);
                        }
                    }
#pragma unroll
                    for (int c = 0; c < I; ++c) {
                        if (mx[c] >= first_term) {
                            auto one = [&](uint64_t st, uint32_t u) { cb(c, st, u); };
                            uint32_t st = opaque(s0[c]);
                            report_nib(st, cur[c][2 * j], cur[c][2 * j + 1], 16,
                                       p[c] + ((uint64_t)l << 7) + 16 * j, one);
                        }
                    }
                }
            }
            if (l + 1 < nl) {
                if (DB) {
                    // the next line into the packed buffer, the one after it
                    // (the last line again at the end) into flight
                    const uint32_t l2 = l + 2 < nl ? l + 2 : nl - 1;
#pragma unroll
                    for (int c = 0; c < I; ++c) {
                        pack(c);
                        fetch(c, l2);
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < I; ++c)
                        fetch(c, l + 1);
#pragma unroll
                    for (int c = 0; c < I; ++c)
                        pack(c);
                }
            }
        }
        // the tail: preloaded pieces, then whatever lies beyond them
#pragma unroll
        for (int c = 0; c < I; ++c) {
            auto one = [&](uint64_t st, uint32_t u) { cb(c, st, u); };
            uint64_t q = p[c] + ((uint64_t)nl << 7);
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                if (q < e[c] && q + 16 <= n) {
                    uint32_t cw[4];
                    cols16(tail[c][j], cw);
                    const uint32_t cnt = (uint32_t)min((uint64_t)16, e[c] - q);
                    const uint32_t s0 = s[c];
                    if (cnt == 16) {
                        if (steps16(s[c], cw) >= first_term)
                            report_piece(opaque(s0), cw, 16, q, one);
                    } else {
                        report_piece(s0, cw, cnt, q, one);
                    }
                    q += cnt;
                }
            }
            if (q < e[c])
                walk_rest(s[c], text, q, e[c], one);
        }
    }

    // Bytes [p, end) from state s, without the line ring: 16-byte pieces
    // where they are aligned, single bytes elsewhere. Used for the rare
    // remainders of walk_lines and for second walks of a range.
    template <class F>
    __device__ __forceinline__ void walk_rest(uint32_t &s, glb_cptr<uint8_t> text, uint64_t p,
                                              uint64_t end, F &cb) const
    {
        while (p < end) {
            if ((((uintptr_t)(text + p)) & 15u) == 0 && p + 16 <= end) {
                uint32_t cw[4];
                cols16(*(glb_cptr<v4u>)(text + p), cw);
                const uint32_t s0 = s;
                if (steps16(s, cw) >= first_term)
                    report_piece(opaque(s0), cw, 16, p, cb);
                p += 16;
            } else {
                s = next(s, Swar ? byte_col((uint32_t)text[p]) : (uint32_t)cls[text[p]]);
                if (s >= first_term)
                    cb(p + 1 - m, s - first_term);
                ++p;
            }
        }
    }

    // Column byte offset of one byte (Swar: the code's column when the byte
    // is the code's expected byte, else column 0).
    __device__ __forceinline__ uint32_t byte_col(uint32_t b) const
    {
        const uint32_t code = (b >> sh) & 7u;
        const uint32_t ex = __builtin_amdgcn_perm(pb_hi, pb_lo, code) & 0xffu;
        const uint32_t col = __builtin_amdgcn_perm(pc_hi, pc_lo, code) & 0xffu;
        return ex == b ? col : 0u;
    }

    // The range of a lane again (the write pass of a lane with more
    // occurrences than it kept). One chain per lane: the same line walk as
    // the first pass (texts with many occurrences send most lanes through
    // here). Two chains per lane: the plain walk, which keeps this copy small.
    template <class F>
    __device__ __forceinline__ void lane_again(glb_cptr<uint8_t> text, uint64_t n, uint64_t base,
                                               uint32_t lo, uint32_t hi, F &&cb) const
    {
        if constexpr (Ilp == 1) {
            lane(text, n, base, lo, hi, cb);
        } else {
            if (lo >= hi)
                return;
            uint64_t end = base + hi + m - 1;
            if (end > n)
                end = n;
            uint32_t s = 0;
            walk_rest(s, text, base + lo, end, cb);
        }
    }

    // Whether walk c's start is where walk_lines can take it.
    __device__ __forceinline__ static bool line_aligned(glb_cptr<uint8_t> text, uint64_t p)
    {
        return (((uintptr_t)(text + p)) & 127u) == 0;
    }

    // Lane range: starts [lo, hi) relative to the chunk at text offset base.
    template <class F>
    __device__ __forceinline__ void lane(glb_cptr<uint8_t> text, uint64_t n, uint64_t base,
                                         uint32_t lo, uint32_t hi, F &&cb) const
    {
        if (lo >= hi)
            return;
        uint64_t end = base + hi + m - 1;
        if (end > n)
            end = n;
        if constexpr (Swar && Ilp == 1 && sizeof(St) == 2) {
            if (line_aligned(text, base + lo) && end - (base + lo) >= 128) {
                const uint64_t pp[1] = {base + lo}, ee[1] = {end};
                auto one = [&](int, uint64_t st, uint32_t u) { cb(st, u); };
                walk_lines<1>(text, n, pp, ee, one);
                return;
            }
        }
        walk(text, base + lo, end, cb);
    }

    // One lane of dense output (16 starts): its 16 + m - 1 bytes as two or
    // three 16-byte pieces requested together, then walked from registers,
    // instead of a piece followed by single-byte loads that each wait out a
    // round trip. Other ranges (the last lanes of a text, misaligned text,
    // m > 33) take the piece-or-byte walk, which (unlike the line walk of
    // long ranges) keeps few registers live: the dense kernel then fits its
    // registers without spilling.
    static constexpr bool LANE16 = true;
    template <class F>
    __device__ __forceinline__ void lane16(glb_cptr<uint8_t> text, uint64_t n, uint64_t base,
                                           uint32_t lo, uint32_t hi, F &&cb) const
    {
        const uint64_t p = base + lo;
        const uint32_t np = m <= 17 ? 2u : 3u;  // pieces holding 16 + m - 1 bytes
        if (hi - lo != 16 || m > 33 || p + 16 * np > n || (((uintptr_t)(text + p)) & 15u)) {
            if (lo >= hi)
                return;
            uint64_t end = base + hi + m - 1;
            if (end > n)
                end = n;
            uint32_t s = 0;
            walk_rest(s, text, p, end, cb);
            return;
        }
        glb_cptr<v4u> q = (glb_cptr<v4u>)(text + p);
        const v4u r0 = q[0], r1 = q[1];
        const v4u r2 = np == 3 ? q[2] : r1;
        uint32_t c0[4], c1[4], c2[4];
        cols16(r0, c0);
        cols16(r1, c1);
        cols16(r2, c2);
        const int steps = 15 + (int)m;
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < 48; ++k) {
            if (k < steps) {
                const uint32_t col = k < 16 ? col_of(c0, k) : k < 32 ? col_of(c1, k - 16)
                                                                     : col_of(c2, k - 32);
                s = next(s, col);
                if (s >= first_term)
                    cb(p + k + 1 - m, s - first_term);
            }
        }
    }

    // Two lane ranges of the same chunk walked in lockstep (text 16-byte
    // aligned), or one after the other.
    template <class FA, class FB>
    __device__ __forceinline__ void lane2(glb_cptr<uint8_t> text, uint64_t n, uint64_t base,
                                          uint32_t lo0, uint32_t hi0, uint32_t lo1, uint32_t hi1,
                                          FA &&cba, FB &&cbb) const
    {
        if (lo1 >= hi1) {
            lane_again(text, n, base, lo0, hi0, cba);
            return;
        }
        uint64_t ea = base + hi0 + m - 1, eb = base + hi1 + m - 1;
        if (ea > n)
            ea = n;
        if (eb > n)
            eb = n;
        if constexpr (Swar && sizeof(St) == 2) {
            if (line_aligned(text, base + lo0) && line_aligned(text, base + lo1) &&
                ea - (base + lo0) >= 128 && eb - (base + lo1) >= 128) {
                const uint64_t pp[2] = {base + lo0, base + lo1}, ee[2] = {ea, eb};
                auto two = [&](int c, uint64_t st, uint32_t u) {
                    if (c == 0)
                        cba(st, u);
                    else
                        cbb(st, u);
                };
                walk_lines<2>(text, n, pp, ee, two);
                return;
            }
        }
        // misaligned text, short ranges or no register columns: one walk
        // after the other, compact code
        uint32_t sa = 0, sb = 0;
        walk_rest(sa, text, base + lo0, ea, cba);
        walk_rest(sb, text, base + lo1, eb, cbb);
    }
};

// ---------------------------------------------------------------------------
// Aho-Corasick with the goto function and supply links at run time
// ---------------------------------------------------------------------------
// The search of Algorithm 3 as the paper's kernels run it (Section 4.2): a
// transition the goto function lacks follows supply links until a state has
// one (the root has one for every byte), one byte at a time. It gives the
// flattened walk's result and is kept to measure what flattening buys. The
// goto rows use the flattened table's numbering and byte-offset columns; a
// missing transition is all ones. Supply strictly lowers the depth, so a
// byte follows at most m links: the loop is bounded by m as well.
template <typename St, int P>
struct AcSupplyWalk {
    using Dev = AcDev;
    static constexpr int ILP = 1;
    static constexpr bool DESC = false;
    static constexpr bool STAGE = false;  // reads text through registers
    static constexpr bool InLds = P == PL_LDS;
    static constexpr uint32_t FAIL = sizeof(St) == 2 ? 0xffffu : 0xffffffffu;
    typename TabPtr<InLds, uint8_t>::type gob;  // goto rows, addressed in bytes
    typename TabPtr<InLds, St>::type sup;       // supply link per state
    lds_cptr<uint16_t> cls;                     // column byte offset per byte value
    uint32_t rowb, first_term, m;

    template <int W>
    __device__ __forceinline__ static void load(const AcDev &a)
    {
        copy_to_lds<W>(LDS_CLS_OFF, a.cls, 512);
        if (InLds)
            copy_to_lds<W>(LDS_TAB_OFF, (const uint8_t *)a.go, a.go_bytes);
    }

    __device__ __forceinline__ void bind(const AcDev &a)
    {
        rowb = a.cp * (uint32_t)sizeof(St);
        first_term = a.first_term;
        m = a.m;
        cls = lds_at<const uint16_t>(LDS_CLS_OFF);
        if constexpr (InLds)
            gob = lds_at<const uint8_t>(LDS_TAB_OFF);
        else
            gob = (glb_cptr<uint8_t>)a.go;
        sup = (typename TabPtr<InLds, St>::type)(gob + a.sup_off);
    }

    template <int W>
    __device__ __forceinline__ void setup(const AcDev &a, uint32_t /*unused*/)
    {
        load<W>(a);
        bind(a);
        __syncthreads();
    }

    __device__ __forceinline__ uint32_t go(uint32_t s, uint32_t coloff) const
    {
        return *(typename TabPtr<InLds, St>::type)(gob + s * rowb + coloff);
    }

    // One byte: goto, else supply links until a goto exists.
    __device__ __forceinline__ uint32_t step(uint32_t s, uint32_t coloff) const
    {
        uint32_t t = go(s, coloff);
        for (uint32_t k = 0; t == FAIL && k < m; ++k) {
            s = sup[s];
            t = go(s, coloff);
        }
        return t == FAIL ? 0u : t;
    }

    template <class F>
    __device__ __forceinline__ void lane(glb_cptr<uint8_t> text, uint64_t n, uint64_t base,
                                         uint32_t lo, uint32_t hi, F &&cb) const
    {
        if (lo >= hi)
            return;
        uint64_t end = base + hi + m - 1;
        if (end > n)
            end = n;
        uint32_t s = 0;
        auto one = [&](uint32_t b, uint64_t q) {
            s = step(s, cls[b]);
            if (s >= first_term)
                cb(q + 1 - m, s - first_term);
        };
        stream_text(text, base + lo, end, one, [&](const v4u c, uint64_t q) {
            const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
            for (int j = 0; j < 16; ++j)
                one((w[j >> 2] >> (8 * (j & 3))) & 0xffu, q + j);
        });
    }

    template <class F>
    __device__ __forceinline__ void lane_again(glb_cptr<uint8_t> text, uint64_t n, uint64_t base,
                                               uint32_t lo, uint32_t hi, F &&cb) const
    {
        lane(text, n, base, lo, hi, cb);
    }
};

// ---------------------------------------------------------------------------
// Aho-Corasick over the reversed strings (sets of different lengths)
// ---------------------------------------------------------------------------
// Bytes [a, e) of a text from e - 1 down to a: single bytes down to a 16-byte
// boundary, 16-byte pieces down to a 128-byte boundary, whole 128-byte lines
// (eight 16-byte loads issued together, the next lower line's loads issued
// before the current one is consumed: a line read piece by piece is often
// evicted from L2 between its pieces), then 16-byte pieces and single bytes.
// one(byte, pos) and sixteen(v4u, pos of its first byte) consume; a piece's
// bytes are taken from its last to its first.
template <class F1, class F16>
__device__ __forceinline__ void rstream_text(glb_cptr<uint8_t> text, uint64_t a, uint64_t e,
                                             F1 &&one, F16 &&sixteen)
{
    uint64_t p = e;
    while (p > a && (((uintptr_t)(text + p)) & 15u)) {
        --p;
        one((uint32_t)text[p], p);
    }
    while (p >= a + 16 && (((uintptr_t)(text + p)) & 127u)) {
        p -= 16;
        sixteen(*(glb_cptr<v4u>)(text + p), p);
    }
    if (p >= a + 128) {
        v4u c[8];
        {
            glb_cptr<v4u> q = (glb_cptr<v4u>)(text + p - 128);
#pragma unroll
            for (int j = 0; j < 8; ++j)
                c[j] = q[j];
        }
        while (true) {
            const bool more = p >= a + 256;
            glb_cptr<v4u> nq = (glb_cptr<v4u>)(text + (more ? p - 256 : p - 128));
            v4u nx[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                nx[j] = nq[j];
            p -= 128;
#pragma unroll
            for (int j = 7; j >= 0; --j)
                sixteen(c[j], p + 16 * j);
            if (!more)
                break;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                c[j] = nx[j];
        }
    }
    while (p >= a + 16) {
        p -= 16;
        sixteen(*(glb_cptr<v4u>)(text + p), p);
    }
    while (p > a) {
        --p;
        one((uint32_t)text[p], p);
    }
}

// A lane walks its range backwards with the automaton of the reversed
// strings. After the byte at q, the state's label is the longest string
// that starts at q and ends some string of the set; the state reports a
// string exactly when one starts at q, namely the longest one, whose id list
// holds every pattern that is a prefix of it (Section 3.1's output sets,
// merged along the supply links of the reversed automaton). The state at q
// depends on the bytes [q, q + m_max) only, so a lane starts m_max - 1 bytes
// past its range. Starts are reported in descending order.
template <typename St, int P>
struct AcRevWalk {
    using Dev = AcDev;
    static constexpr int ILP = 1;
    static constexpr bool DESC = true;
    static constexpr bool STAGE = false;  // reads text through registers
    static constexpr bool InLds = P == PL_LDS;
    // PL_HOT: the first rows (breadth-first, the short labels a walk spends
    // most steps in) from LDS, the others from global memory.
    static constexpr bool Hot = P == PL_HOT;
    typename TabPtr<InLds, uint8_t>::type dfab;  // table, addressed in bytes
    lds_cptr<uint16_t> cls;                      // column byte offset per byte value
    glb_cptr<uint32_t> term;                     // string of each reporting state
    uint32_t rowb, first_term, mx, hot;

    template <int W>
    __device__ __forceinline__ static void load(const AcDev &a)
    {
        copy_to_lds<W>(LDS_CLS_OFF, a.cls, 512);
        if (InLds)
            copy_to_lds<W>(LDS_TAB_OFF, (const uint8_t *)a.dfa, a.dfa_bytes);
        if (Hot)
            copy_to_lds<W>(LDS_TAB_OFF, (const uint8_t *)a.dfa, a.hot_bytes);
    }

    __device__ __forceinline__ void bind(const AcDev &a)
    {
        rowb = a.cp * (uint32_t)sizeof(St);
        first_term = a.first_term;
        mx = a.m_max;
        cls = lds_at<const uint16_t>(LDS_CLS_OFF);
        if constexpr (InLds)
            dfab = lds_at<const uint8_t>(LDS_TAB_OFF);
        else
            dfab = (glb_cptr<uint8_t>)a.dfa;
        term = (glb_cptr<uint32_t>)a.term_u;
        hot = a.hot_states;
    }

    template <int W>
    __device__ __forceinline__ void setup(const AcDev &a, uint32_t /*unused*/)
    {
        load<W>(a);
        bind(a);
        __syncthreads();
    }

    __device__ __forceinline__ uint32_t next(uint32_t s, uint32_t coloff) const
    {
        const uint32_t off = sizeof(St) == 2 ? __umul24(s, rowb) + coloff : s * rowb + coloff;
        if constexpr (Hot) {
            if (s < hot)
                return *(lds_cptr<St>)(lds_at<const uint8_t>(LDS_TAB_OFF) + off);
        }
        return *(typename TabPtr<InLds, St>::type)(dfab + off);
    }

    // Starts [base + lo, base + hi), from the last to the first.
    template <class F>
    __device__ __forceinline__ void lane(glb_cptr<uint8_t> text, uint64_t n, uint64_t base,
                                         uint32_t lo, uint32_t hi, F &&cb) const
    {
        if (lo >= hi)
            return;
        const uint64_t a = base + lo, b = base + hi;
        uint64_t e = b + mx - 1;
        if (e > n)
            e = n;
        uint32_t s = 0;
        auto one = [&](uint32_t byte, uint64_t q) {
            s = next(s, cls[byte]);
            if (s >= first_term && q < b)
                cb(q, term[s - first_term]);
        };
        rstream_text(text, a, e, one, [&](const v4u c, uint64_t q) {
            const uint32_t w[4] = {c.x, c.y, c.z, c.w};
            uint32_t st[16];
            uint32_t mxs = 0;
#pragma unroll
            for (int j = 15; j >= 0; --j) {
                s = next(s, cls[(w[j >> 2] >> (8 * (j & 3))) & 0xffu]);
                st[j] = s;
                mxs = max(mxs, s);
            }
            if (mxs >= first_term) {
#pragma unroll
                for (int j = 15; j >= 0; --j)
                    if (st[j] >= first_term && q + j < b)
                        cb(q + j, term[st[j] - first_term]);
            }
        });
    }

    template <class F>
    __device__ __forceinline__ void lane_again(glb_cptr<uint8_t> text, uint64_t n, uint64_t base,
                                               uint32_t lo, uint32_t hi, F &&cb) const
    {
        lane(text, n, base, lo, hi, cb);
    }
};

// ---------------------------------------------------------------------------
// Aho-Corasick with the text read a byte at a time (the kernel ladder)
// ---------------------------------------------------------------------------
// TM 1: every lane loads its bytes one at a time from global memory. TM 2:
// the workgroup copies its chunk's text (and the m - 1 bytes after it) into
// LDS with coalesced 16-byte loads before the walk (stage), and lanes read
// their bytes from there. Byte q of the chunk starting at base sits at LDS
// offset tl + sh + (q - base), sh being the text address's offset within 16
// bytes, so the copy's 16-byte pieces land on 16-byte LDS boundaries. The
// byte -> column map is the LDS table (no register byte classes).
template <typename St, int P, int TM>
struct AcTextWalk {
    using Dev = AcDev;
    static constexpr int ILP = 1;
    static constexpr bool DESC = false;
    static constexpr bool STAGE = TM == 2;
    static constexpr bool InLds = P == PL_LDS;
    typename TabPtr<InLds, uint8_t>::type dfab;
    lds_cptr<uint16_t> cls;
    uint32_t rowb, first_term, m, tl;

    template <int W>
    __device__ __forceinline__ void setup(const AcDev &a, uint32_t text_lds)
    {
        copy_to_lds<W>(LDS_CLS_OFF, a.cls, 512);
        if (InLds)
            copy_to_lds<W>(LDS_TAB_OFF, (const uint8_t *)a.dfa, a.dfa_bytes);
        rowb = a.cp * (uint32_t)sizeof(St);
        first_term = a.first_term;
        m = a.m;
        cls = lds_at<const uint16_t>(LDS_CLS_OFF);
        if constexpr (InLds)
            dfab = lds_at<const uint8_t>(LDS_TAB_OFF);
        else
            dfab = (glb_cptr<uint8_t>)a.dfa;
        tl = text_lds;
        __syncthreads();
    }

    __device__ __forceinline__ uint32_t next(uint32_t s, uint32_t coloff) const
    {
        const uint32_t off = sizeof(St) == 2 ? __umul24(s, rowb) + coloff : s * rowb + coloff;
        return *(typename TabPtr<InLds, St>::type)(dfab + off);
    }

    // Copy text [base, base + bytes) into LDS (TM 2; no barrier).
    template <int W>
    __device__ __forceinline__ void stage(glb_cptr<uint8_t> text, uint64_t base, uint64_t bytes) const
    {
        const uint32_t sh = (uint32_t)((uintptr_t)(text + base) & 15u);
        LDS_AS uint8_t *d = lds_at<uint8_t>(tl);
        const uint64_t head = min((uint64_t)((16u - sh) & 15u), bytes);
        if (threadIdx.x < head)
            d[sh + threadIdx.x] = text[base + threadIdx.x];
        const uint64_t nw = (bytes - head) / 16;
        glb_cptr<v4u> src = (glb_cptr<v4u>)(text + base + head);
        LDS_AS v4u *dst = (LDS_AS v4u *)(d + sh + head);
        for (uint64_t k = threadIdx.x; k < nw; k += W)
            dst[k] = src[k];
        for (uint64_t k = head + nw * 16 + threadIdx.x; k < bytes; k += W)
            d[sh + k] = text[base + k];
    }

    template <class F>
    __device__ __forceinline__ void lane(glb_cptr<uint8_t> text, uint64_t n, uint64_t base,
                                         uint32_t lo, uint32_t hi, F &&cb) const
    {
        if (lo >= hi)
            return;
        uint64_t end = base + hi + m - 1;
        if (end > n)
            end = n;
        uint32_t s = 0;
        if constexpr (TM == 2) {
            lds_cptr<uint8_t> d =
                lds_at<const uint8_t>(tl + (uint32_t)((uintptr_t)(text + base) & 15u));
            for (uint32_t q = lo; q < (uint32_t)(end - base); ++q) {
                s = next(s, cls[d[q]]);
                if (s >= first_term)
                    cb(base + q + 1 - m, s - first_term);
            }
        } else {
            for (uint64_t q = base + lo; q < end; ++q) {
                s = next(s, cls[text[q]]);
                if (s >= first_term)
                    cb(q + 1 - m, s - first_term);
            }
        }
    }

    template <class F>
    __device__ __forceinline__ void lane_again(glb_cptr<uint8_t> text, uint64_t n, uint64_t base,
                                               uint32_t lo, uint32_t hi, F &&cb) const
    {
        lane(text, n, base, lo, hi, cb);
    }
};

// ---------------------------------------------------------------------------
// Wu-Manber walker
// ---------------------------------------------------------------------------
static const int WM_QUEUE = 4;  // filtered candidates kept before exact checks

// 2-bit codes of four bytes, first byte in the low bits.
__device__ __forceinline__ uint32_t codes4(uint32_t w, uint32_t sh)
{
    uint32_t x = (w >> sh) & 0x03030303u;
    x = (x | (x >> 6)) & 0x000F000Fu;
    return (x | (x >> 12)) & 0xFFu;
}

// Var: strings of different lengths (the window is the shortest length; a
// bucket lists longer strings first and the first one that matches a window
// is the one reported there, its id list covering the shorter matches).
template <int P, bool Var = false>
struct WmWalk {
    using Dev = WmDev;
    static constexpr int ILP = 1;
    static constexpr bool DESC = false;
    static constexpr bool STAGE = false;  // reads text through registers
    static constexpr bool LANE16 = false;  // dense lanes walk with lane()
    static constexpr bool InLds = P == PL_LDS;
    // PL_HOT: SHIFT (read for every window) in LDS, the buckets (read only
    // for windows with a zero shift) in global memory.
    static constexpr bool Hot = P == PL_HOT;
    typename TabPtr<InLds || Hot, uint16_t>::type sh16;
    typename TabPtr<InLds, uint32_t>::type boff, bkey, bu;
    glb_cptr<uint8_t> pats;
    glb_cptr<uint32_t> upoff;  // Var: string u is pats[upoff[u] .. upoff[u + 1])
    uint32_t m, B, csh, kl, hmask, kmask;

    // Copy what this walker reads from LDS (no barrier).
    template <int W>
    __device__ __forceinline__ static void load(const WmDev &a)
    {
        if (InLds)
            copy_to_lds<W>(LDS_TAB_OFF, a.tables, a.table_bytes);
        if (Hot)
            copy_to_lds<W>(LDS_TAB_OFF, a.tables, a.shift_bytes);
    }

    __device__ __forceinline__ void bind(const WmDev &a)
    {
        m = a.m;
        B = a.B;
        csh = a.code_shift;
        kl = a.key_len;
        hmask = (1u << (2 * B)) - 1u;
        kmask = kl >= 16 ? 0xffffffffu : ((1u << (2 * kl)) - 1u);
        typename TabPtr<InLds, uint8_t>::type base;
        if constexpr (InLds)
            base = lds_at<const uint8_t>(LDS_TAB_OFF);
        else
            base = (glb_cptr<uint8_t>)a.tables;
        if constexpr (Hot)
            sh16 = lds_at<const uint16_t>(LDS_TAB_OFF);
        else
            sh16 = (typename TabPtr<InLds, uint16_t>::type)base;
        boff = (typename TabPtr<InLds, uint32_t>::type)(base + a.off_boff);
        bkey = (typename TabPtr<InLds, uint32_t>::type)(base + a.off_bkey);
        bu = (typename TabPtr<InLds, uint32_t>::type)(base + a.off_bu);
        pats = (glb_cptr<uint8_t>)a.pats;
        upoff = (glb_cptr<uint32_t>)a.upoff;
    }

    template <int W>
    __device__ __forceinline__ void setup(const WmDev &a, uint32_t /*unused*/)
    {
        load<W>(a);
        bind(a);
        __syncthreads();
    }

    // Window loop (Algorithm 5) over one lane's range, the text streamed
    // through registers as 2-bit character codes. The history holds the
    // codes of the last 32 characters read (positions [e-32, e), position q
    // at bit 2(q-e+32) of {h1:h0}). Every window end nx < e is examined: the
    // hash of its last B characters picks SHIFT; a zero shift sends the
    // window to its bucket, where the filter key (codes of the key_len
    // characters before the block) must equal the candidate's before the
    // window is compared byte by byte with the pattern. Window ends are never
    // more than 16 characters behind e (every append adds at most 16 and all
    // earlier windows are done), and the builder keeps B + key_len <= 17, so
    // block and key both lie in the history: each is one 64-bit shift.
    template <class F>
    __device__ __forceinline__ void lane(glb_cptr<uint8_t> text, uint64_t n, uint64_t base,
                                         uint32_t lo, uint32_t hi, F &&cb) const
    {
        if (lo >= hi)
            return;
        // Texts are shorter than 2^32 bytes: positions fit in 32 bits.
        const uint32_t p = (uint32_t)(base + lo);
        uint64_t end64 = base + hi + m - 1;
        if (end64 > n)
            end64 = n;
        const uint32_t end = (uint32_t)end64;
        uint32_t nx = p + m - 1;
        uint32_t e = p;
        uint64_t h = 0;
        uint32_t qn = 0;
        uint32_t qp[WM_QUEUE];  // window ends
        uint32_t qu[WM_QUEUE];
#pragma unroll
        for (int k = 0; k < WM_QUEUE; ++k) {
            qp[k] = 0;
            qu[k] = 0;
        }
        // Exact check of the queued candidates, eight bytes of window and
        // pattern per step with no early exit, so a step's loads are in
        // flight together.
        // Var: window end of the last report (a window reports one string).
        uint32_t done = 0xffffffffu;
        auto flush = [&]() {
#pragma unroll
            for (int k = 0; k < WM_QUEUE; ++k) {
                if ((uint32_t)k < qn) {
                    const uint64_t st = (uint64_t)qp[k] + 1 - m;
                    if constexpr (Var) {
                        const uint32_t po = upoff[qu[k]];
                        const uint32_t len = upoff[qu[k] + 1] - po;
                        // strings running past the text's end do not occur
                        if (qp[k] != done && st + len <= n) {
                            glb_cptr<uint8_t> pp = pats + po;
                            uint32_t diff = 0;
                            for (uint32_t j = 0; j < len; j += 8) {
#pragma unroll
                                for (uint32_t t = 0; t < 8; ++t)
                                    if (j + t < len)
                                        diff |= (uint32_t)(pp[j + t] ^ text[st + j + t]);
                            }
                            if (diff == 0) {
                                cb(st, qu[k]);
                                done = qp[k];
                            }
                        }
                    } else {
                        glb_cptr<uint8_t> pp = pats + (uint64_t)qu[k] * m;
                        uint32_t diff = 0;
                        for (uint32_t j = 0; j < m; j += 8) {
#pragma unroll
                            for (uint32_t t = 0; t < 8; ++t)
                                if (j + t < m)
                                    diff |= (uint32_t)(pp[j + t] ^ text[st + j + t]);
                        }
                        if (diff == 0)
                            cb(st, qu[k]);
                    }
                }
            }
            qn = 0;
        };
        // block bit (minus one, for the byte offset of a u16 entry) and key
        // bit of the window ending at nx: c2 + 2 (nx - e) and that + 1 - 2 kl
        const uint32_t c2 = 65u - 2u * B;
        const uint32_t hmask2 = hmask << 1;
        const uint32_t kdrop = 2u * kl - 1u;
        auto windows = [&]() {
            while (nx < e) {
                const uint32_t o2 = c2 + 2u * (nx - e);
                const uint32_t hb = (uint32_t)(h >> o2) & hmask2;
                const uint32_t sv = *(typename TabPtr<InLds || Hot, uint16_t>::type)(
                    (typename TabPtr<InLds || Hot, uint8_t>::type)sh16 + hb);
                if (sv & 0x8000u) {
                    const uint32_t b = sv & 0x7fffu;
                    const uint32_t key = kl ? ((uint32_t)(h >> (o2 - kdrop)) & kmask) : 0u;
                    const uint32_t je = boff[b + 1];
                    for (uint32_t j = boff[b]; j < je; ++j) {
                        if (bkey[j] == key) {
                            if (qn == (uint32_t)WM_QUEUE)
                                flush();
#pragma unroll
                            for (int k = 0; k < WM_QUEUE; ++k)
                                if (qn == (uint32_t)k) {
                                    qp[k] = nx;
                                    qu[k] = bu[j];
                                }
                            ++qn;
                        }
                    }
                    nx += 1;
                } else {
                    nx += sv;
                }
            }
        };
        stream_text(
            text, p, end,
            [&](uint32_t b, uint64_t) {
                h = (h >> 2) | ((uint64_t)((b >> csh) & 3u) << 62);
                e += 1;
                windows();
            },
            [&](const v4u c) {
                return codes4(c.x, csh) | (codes4(c.y, csh) << 8) | (codes4(c.z, csh) << 16) |
                       (codes4(c.w, csh) << 24);
            },
            [&](uint32_t codes, uint64_t) {
                h = (h >> 32) | ((uint64_t)codes << 32);
                e += 16;
                windows();
            });
        flush();
    }

    template <class F>
    __device__ __forceinline__ void lane_again(glb_cptr<uint8_t> text, uint64_t n, uint64_t base,
                                               uint32_t lo, uint32_t hi, F &&cb) const
    {
        lane(text, n, base, lo, hi, cb);
    }
};

// ---------------------------------------------------------------------------
// Persistent chunk driver
// ---------------------------------------------------------------------------
// One chunk (phases A-C). The chunk is chunk g of its text; base is its
// first starting position, `starts` how many starting positions it holds.
// Staging area of one workgroup: slot j of virtual lane v at j * lanes + v
// (slots of neighbouring lanes are neighbours, so lanes that stage or read
// their j-th occurrence together touch one contiguous run).
struct Stage {
    GLB_AS v2u *base;  // this workgroup's area (null: no staging)
    uint32_t cap;      // slots per virtual lane
    uint32_t lanes;    // virtual lanes of the workgroup
};

template <class Walk, int W>
__device__ __forceinline__ void process_chunk(const Walk &wk, glb_cptr<uint8_t> text, uint64_t n,
                                              mpm_match *out, uint64_t cap, uint64_t *total,
                                              uint64_t first_g, uint64_t nt, uint64_t g,
                                              uint32_t L, uint32_t m, uint32_t epoch,
                                              const IdMap &im, uint32_t *hdr, uint64_t *status,
                                              uint64_t *s_scan, const Stage &stg)
{
    constexpr int I = Walk::ILP;
    constexpr int KS = K_SLOTS;  // occurrences kept per virtual lane
    const uint32_t scap = stg.base ? stg.cap : 0u;
    const uint64_t chunk = (uint64_t)W * L * I;
    const uint64_t lt = g - first_g;
    const uint64_t ns = n - m + 1;
    const uint64_t base = lt * chunk;
    const uint64_t starts = (ns - base) < chunk ? (ns - base) : chunk;

    if constexpr (Walk::STAGE) {  // the chunk's text (and m - 1 bytes) into LDS
        const uint64_t bytes = (starts + m - 1) < (n - base) ? (starts + m - 1) : (n - base);
        wk.template stage<W>(text, base, bytes);
        __syncthreads();
    }

    // Virtual lane v of this thread owns starts [lo[v], hi[v]) of the chunk.
    uint32_t lo[I], hi[I];
#pragma unroll
    for (int v = 0; v < I; ++v) {
        const uint32_t l0 = (threadIdx.x + v * W) * L;
        lo[v] = l0 < starts ? l0 : (uint32_t)starts;
        hi[v] = (l0 + L) < starts ? (l0 + L) : (uint32_t)starts;
    }

    // Phase A: count, keep the first occurrences in registers, stage the
    // next ones in the workspace.
    uint32_t nu[I], nid[I];
    uint32_t so[I][KS], su[I][KS];
#pragma unroll
    for (int v = 0; v < I; ++v) {
        nu[v] = 0;
        nid[v] = 0;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            so[v][k] = 0;
            su[v][k] = 0;
        }
    }
    auto rec = [&](int v, uint64_t start, uint32_t u) {
        if (nu[v] < (uint32_t)KS) {
#pragma unroll
            for (int k = 0; k < KS; ++k)
                if (nu[v] == (uint32_t)k) {
                    so[v][k] = (uint32_t)start;
                    su[v][k] = u;
                }
        } else if (nu[v] - (uint32_t)KS < scap) {
            stg.base[(uint64_t)(nu[v] - KS) * stg.lanes + threadIdx.x + v * W] =
                v2u{(uint32_t)start, u};
        }
        ++nu[v];
        nid[v] += im.count(u);
    };
    auto rec0 = [&](uint64_t start, uint32_t u) { rec(0, start, u); };
    if constexpr (I == 1) {
        wk.lane(text, n, base, lo[0], hi[0], rec0);
    } else {
        auto rec1 = [&](uint64_t start, uint32_t u) { rec(I - 1, start, u); };
        wk.lane2(text, n, base, lo[0], hi[0], lo[I - 1], hi[I - 1], rec0, rec1);
    }

    // Phase B: offsets.
    const bool last = lt + 1 == nt;
    uint64_t ob[I];
    chunk_offsets<W, I>(nid, ob, s_scan, status, g, first_g, last, total, epoch, &hdr[WS_ERR]);

    // Phase C: ordered writes.
#pragma unroll
    for (int v = 0; v < I; ++v) {
        // nothing to write: no occurrences, or all of them past the capacity
        // (a counting call with capacity 0 walks each range once)
        if (nu[v] == 0 || ob[v] >= cap)
            continue;
        if constexpr (Walk::DESC) {
            // Occurrences come from the range's last start down: each one's
            // ids go just below the previous one's, from the lane's end.
            uint64_t o = ob[v] + nid[v];
            auto put = [&](uint32_t pos, uint32_t u) {
                o -= im.count(u);
                uint64_t w = o;
                write_ids(out, cap, w, pos, u, im);
            };
#pragma unroll
            for (int k = 0; k < KS; ++k)
                if ((uint32_t)k < nu[v])
                    put(so[v][k], su[v][k]);
            if (nu[v] > (uint32_t)KS) {
                const uint32_t ns_ = min(nu[v] - (uint32_t)KS, scap);
                for (uint32_t j = 0; j < ns_; ++j) {
                    const v2u e = stg.base[(uint64_t)j * stg.lanes + threadIdx.x + v * W];
                    put(e.x, e.y);
                }
            }
            if (nu[v] > (uint32_t)KS + scap && o > ob[v]) {
                // the rest start below the last kept or staged one
                const uint32_t last =
                    scap ? stg.base[(uint64_t)(scap - 1) * stg.lanes + threadIdx.x + v * W].x
                         : so[v][KS - 1];
                wk.lane_again(text, n, base, lo[v], (uint32_t)((uint64_t)last - base),
                              [&](uint64_t start, uint32_t u) { put((uint32_t)start, u); });
            }
            continue;
        }
        uint64_t o = ob[v];
#pragma unroll
        for (int k = 0; k < KS; ++k)
            if ((uint32_t)k < nu[v])
                write_ids(out, cap, o, so[v][k], su[v][k], im);
        if (nu[v] > (uint32_t)KS) {
            const uint32_t ns_ = min(nu[v] - (uint32_t)KS, scap);
            for (uint32_t j = 0; j < ns_ && o < cap; ++j) {
                const v2u e = stg.base[(uint64_t)j * stg.lanes + threadIdx.x + v * W];
                write_ids(out, cap, o, e.x, e.y, im);
            }
        }
        if (nu[v] > (uint32_t)KS + scap && o < cap) {
            // The rest start after the last kept or staged one (one distinct
            // string per start): walk again from there, from the root / an
            // empty window.
            const uint32_t last =
                scap ? stg.base[(uint64_t)(scap - 1) * stg.lanes + threadIdx.x + v * W].x
                     : so[v][KS - 1];
            const uint32_t lo2 = (uint32_t)((uint64_t)last + 1 - base);
            wk.lane_again(text, n, base, lo2, hi[v], [&](uint64_t start, uint32_t u) {
                write_ids(out, cap, o, (uint32_t)start, u, im);
            });
        }
    }
}

// Dense output: each lane owns DENSE_LANE starting positions and marks, per
// position, the distinct string that starts there (or none) in an LDS array
// laid out in position order; after the chunk's offsets are known, every wave
// sweeps its 64 * DENSE_LANE positions in rounds of 64 consecutive ones, a
// prefix sum over the round gives each position its output slot, and the
// wave writes the round's pairs to consecutive slots. Lists with many
// occurrences per position are written in whole cache lines by few
// instructions, instead of every lane appending to its own output range.
static const uint32_t DENSE_LANE = 16;
static const uint32_t MARK_NONE = 0xffffffffu;

template <class Walk, int W>
__device__ __forceinline__ void process_chunk_dense(const Walk &wk, glb_cptr<uint8_t> text,
                                                    uint64_t n, mpm_match *out_, uint64_t cap,
                                                    uint64_t *total, uint64_t first_g, uint64_t nt,
                                                    uint64_t g, uint32_t m, uint32_t epoch,
                                                    const IdMap &im, uint32_t *hdr,
                                                    uint64_t *status, uint64_t *s_scan,
                                                    uint32_t mark_lds)
{
    static_assert(Walk::ILP == 1, "dense output runs one range per lane");
    constexpr uint32_t DL = DENSE_LANE;
    const uint64_t chunk = (uint64_t)W * DL;
    const uint64_t lt = g - first_g;
    const uint64_t ns = n - m + 1;
    const uint64_t base = lt * chunk;
    const uint64_t starts = (ns - base) < chunk ? (ns - base) : chunk;
    const uint32_t l0 = threadIdx.x * DL;
    const uint32_t lo = l0 < starts ? l0 : (uint32_t)starts;
    const uint32_t hi = (l0 + DL) < starts ? (l0 + DL) : (uint32_t)starts;
    LDS_AS uint32_t *mk = lds_at<uint32_t>(mark_lds);

    // Phase A: marks and the lane's count of ids. The wave clears its own
    // 64 * DL marks, 64 consecutive ones per store (bank-conflict free);
    // its LDS operations complete in program order, so each lane's marks
    // below land after the clearing.
    const uint32_t wmk = (threadIdx.x & ~63u) * DL;
#pragma unroll
    for (uint32_t j = 0; j < DL; ++j)
        mk[wmk + j * 64 + (threadIdx.x & 63u)] = MARK_NONE;
    __builtin_amdgcn_wave_barrier();
    uint32_t nid[1] = {0};
    auto mark = [&](uint64_t start, uint32_t u) {
        mk[(uint32_t)(start - base)] = u;
        nid[0] += im.count(u);
    };
    if constexpr (Walk::LANE16)
        wk.lane16(text, n, base, lo, hi, mark);
    else
        wk.lane(text, n, base, lo, hi, mark);

    // Phase B: offsets (its barriers also publish the marks to the wave).
    const bool last = lt + 1 == nt;
    uint64_t ob[1];
    chunk_offsets<W, 1>(nid, ob, s_scan, status, g, first_g, last, total, epoch, &hdr[WS_ERR]);

    // Phase C: the wave's positions in order, 64 at a time.
    const int lane = threadIdx.x & 63;
    const uint32_t wpos = threadIdx.x & ~63u;  // first lane of the wave
    uint64_t o = ob[0];
    o = ((uint64_t)__shfl((uint32_t)(o >> 32), 0, 64) << 32) | __shfl((uint32_t)o, 0, 64);
    GLB_AS v2u *out = (GLB_AS v2u *)out_;
#pragma unroll 1
    for (uint32_t r = 0; r < DL && o < cap; ++r) {
        const uint32_t p = wpos * DL + r * 64 + lane;  // chunk-relative start
        const uint32_t u = mk[p];
        uint32_t b = 0, e = 0;
        if (u != MARK_NONE)
            im.span(u, b, e);
        const uint32_t c = e - b;
        uint32_t round;
        const uint32_t pre = wave_excl_sum(c, round);
        uint64_t q = o + pre;
        const uint32_t pos = (uint32_t)(base + p);
        for (uint32_t j = b; j < e && q < cap; ++j, ++q)
            out[q] = v2u{pos, im.id(j)};
        o += round;
    }
}

// Take a ticket (thread 0), returning it through LDS; the caller syncs.
__device__ __forceinline__ uint64_t take_ticket(uint32_t *hdr)
{
    return atomicAdd(&hdr[WS_TICKET], 1u);
}

// Last workgroup to finish resets the ticket and done counters and moves the
// epoch on, so the next launch on this workspace starts clean.
__device__ __forceinline__ void finish_launch(uint32_t *hdr, uint32_t epoch)
{
    if (threadIdx.x == 0) {
        const uint32_t dn = atomicAdd(&hdr[WS_DONE], 1u);
        if (dn == gridDim.x - 1) {
            __hip_atomic_store(&hdr[WS_TICKET], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&hdr[WS_DONE], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&hdr[WS_EPOCH], epoch + 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <class Walk, int W, bool Dense = false>
__global__ __launch_bounds__(W) void scan_kernel(typename Walk::Dev a, ScanDev sd,
                                                 const uint32_t *uoff_, const uint32_t *uids_,
                                                 uint32_t dupfree, uint32_t unused)
{
    extern __shared__ __align__(16) uint8_t smem[];
    static_assert(Walk::ILP * (W / 64) + 1 <= LDS_SCAN_WORDS, "scan words");
    if (!lds_layout_ok(smem, sd.hdr))
        return;
    LdsHdr *const H = (LdsHdr *)lds_at<LdsHdr>(LDS_HDR_OFF);
    TextDesc &s_td = H->td;
    uint64_t &s_tile = H->tile;
    uint32_t &s_epoch = H->epoch;
    uint64_t *const s_scan = H->scan;

    // Launch constants as plain values (no by-reference use of the argument
    // structs, which would place them in private memory).
    const uint32_t ntexts = sd.ntexts;
    const uint64_t ntiles = sd.ntiles;
    const uint32_t L = sd.lane_bytes;
    uint32_t *const hdr = sd.hdr;
    uint64_t *const status = sd.status;
    const TextDesc *const multi = sd.multi;
    IdMap im;
    im.uoff = (glb_cptr<uint32_t>)uoff_;
    im.uids = (glb_cptr<uint32_t>)uids_;
    im.lds_uoff = sd.csr_uoff_lds;
    im.lds_uids = sd.csr_uids_lds;
    im.dupfree = dupfree;
    im.n_single = a.n_single;
    const uint32_t m = a.m;
    if (im.lds_uoff) {  // the id CSR into LDS (synchronised by the setup below)
        copy_to_lds<W>(im.lds_uoff, (const uint8_t *)uoff_, 4 * sd.csr_uoff_words);
        copy_to_lds<W>(im.lds_uids, (const uint8_t *)uids_, 4 * sd.csr_uids_words);
    }

    Stage stg;
    stg.cap = sd.stage_cap;
    stg.lanes = Walk::ILP * W;
    stg.base = sd.stage ? (GLB_AS v2u *)sd.stage + (uint64_t)blockIdx.x * stg.cap * stg.lanes
                        : nullptr;

    load_groups(a.grp);  // synchronised by the setup below
    Walk wk;
    wk.template setup<W>(a, unused);
    if (threadIdx.x == 0)
        s_epoch = __hip_atomic_load(&hdr[WS_EPOCH], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    while (true) {
        if (threadIdx.x == 0) {
            const uint64_t t = take_ticket(hdr);
            s_tile = t;
            if (t < ntiles) {
                if (ntexts == 1) {
                    s_td = sd.single;
                } else {  // the text whose chunk range holds t
                    uint32_t lo = 0, hi = ntexts;
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (multi[mid].tile_begin <= t)
                            lo = mid;
                        else
                            hi = mid;
                    }
                    s_td = multi[lo];
                }
            }
        }
        __syncthreads();
        const uint64_t g = s_tile;
        if (g >= ntiles)
            break;
        if constexpr (Dense)
            process_chunk_dense<Walk, W>(wk, (glb_cptr<uint8_t>)s_td.text, s_td.n, s_td.out,
                                         s_td.cap, s_td.total, s_td.tile_begin, s_td.ntiles, g, m,
                                         s_epoch, im, hdr, status, s_scan, sd.mark_lds);
        else
            process_chunk<Walk, W>(wk, (glb_cptr<uint8_t>)s_td.text, s_td.n, s_td.out, s_td.cap,
                                   s_td.total, s_td.tile_begin, s_td.ntiles, g, L, m, s_epoch, im,
                                   hdr, status, s_scan, stg);
        __syncthreads();
    }
    finish_launch(hdr, s_epoch);
}

// ---------------------------------------------------------------------------
// Batched persistent kernel: many texts, each scanned with its own index and
// walker kind, in one launch. Texts are ordered by index in the queue, so a
// workgroup reloads its LDS tables only when the index of its next chunk
// differs from the one it holds.
// ---------------------------------------------------------------------------
template <class Walk, int W, class Dev>
__device__ __forceinline__ void batch_chunk(const Dev &dev, glb_cptr<uint8_t> text,
                                            uint64_t n, mpm_match *out, uint64_t cap,
                                            uint64_t *total, uint64_t first_g, uint64_t nt,
                                            uint64_t g, uint32_t L, uint32_t epoch, uint32_t *hdr,
                                            uint64_t *status, uint64_t *s_scan, const Stage &stg)
{
    Walk wk;
    wk.bind(dev);
    IdMap im;
    im.uoff = (glb_cptr<uint32_t>)dev.uoff;
    im.uids = (glb_cptr<uint32_t>)dev.uids;
    im.lds_uoff = 0;
    im.lds_uids = 0;
    im.dupfree = dev.dupfree;
    im.n_single = dev.n_single;
    process_chunk<Walk, W>(wk, text, n, out, cap, total, first_g, nt, g, L, dev.m, epoch, im,
                           hdr, status, s_scan, stg);
}

template <class Walk>
__device__ __forceinline__ const typename Walk::Dev &dev_of(const BatchIndex &bi)
{
    if constexpr (std::is_same<typename Walk::Dev, AcDev>::value)
        return bi.ac;
    else
        return bi.wm;
}

// One launch serves one walker kind (algorithm, table placement, byte-class
// method); a batch's texts are split into launches by kind and block size.
template <class Walk, int W>
__global__ __launch_bounds__(W) void batch_kernel(BatchDev bd)
{
    extern __shared__ __align__(16) uint8_t smem[];
    static_assert(W / 64 + 1 <= LDS_SCAN_WORDS, "scan words");
    if (!lds_layout_ok(smem, bd.hdr))
        return;
    LdsHdr *const H = (LdsHdr *)lds_at<LdsHdr>(LDS_HDR_OFF);
    BatchText &s_bt = H->bt;
    uint64_t &s_tile = H->tile;
    uint32_t &s_epoch = H->epoch;
    uint64_t *const s_scan = H->scan;

    const uint32_t ntexts = bd.ntexts;
    const uint64_t ntiles = bd.ntiles;
    uint32_t *const hdr = bd.hdr;
    uint64_t *const status = bd.status;
    const BatchText *const texts = bd.texts;
    Stage stg;
    stg.cap = bd.stage_cap;
    stg.lanes = W;
    stg.base = bd.stage ? (GLB_AS v2u *)bd.stage + (uint64_t)blockIdx.x * stg.cap * stg.lanes
                        : nullptr;
    if (threadIdx.x == 0)
        s_epoch = __hip_atomic_load(&hdr[WS_EPOCH], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t loaded = 0xffffffffu;  // index whose tables LDS holds (uniform)

    while (true) {
        if (threadIdx.x == 0) {
            const uint64_t t = take_ticket(hdr);
            s_tile = t;
            if (t < ntiles) {
                uint32_t lo = 0, hi = ntexts;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (texts[mid].td.tile_begin <= t)
                        lo = mid;
                    else
                        hi = mid;
                }
                s_bt = texts[lo];
            }
        }
        __syncthreads();
        const uint64_t g = s_tile;
        if (g >= ntiles)
            break;
        uint64_t t0 = 0;
        if (threadIdx.x == 0)
            t0 = wall_clock64();
        const uint32_t ix = s_bt.index;
        const auto &dev = dev_of<Walk>(bd.idx[ix]);
        if (ix != loaded) {
            Walk::template load<W>(dev);
            load_groups(dev.grp);
            __syncthreads();
            loaded = ix;
        }
        batch_chunk<Walk, W>(dev, (glb_cptr<uint8_t>)s_bt.td.text, s_bt.td.n, s_bt.td.out,
                             s_bt.td.cap, s_bt.td.total, s_bt.td.tile_begin, s_bt.td.ntiles, g,
                             s_bt.lane_bytes, s_epoch, hdr, status, s_scan, stg);
        __syncthreads();
        // a timed request: its share of the launch and its longest chunk
        // (s_bt holds this chunk's text until thread 0 takes the next ticket)
        if (threadIdx.x == 0 && s_bt.cost) {
            const float us = (float)(wall_clock64() - t0) * bd.us_per_tick;
            atomicAdd(&s_bt.cost[0], us / (float)gridDim.x);
            atomicMax((uint32_t *)&s_bt.cost[1], __float_as_uint(us));  // order of >= 0 floats
        }
    }
    finish_launch(hdr, s_epoch);
}

template <class Walk>
static const void *batch_pick_w(uint32_t W)
{
    switch (W) {
    case 256: return (const void *)batch_kernel<Walk, 256>;
    case 512: return (const void *)batch_kernel<Walk, 512>;
    case 1024: return (const void *)batch_kernel<Walk, 1024>;
    }
    return nullptr;
}

template <class Walk>
static hipError_t batch_launch_w(const BatchDev &bd, uint32_t W, uint32_t grid, uint32_t lds,
                                 hipStream_t s)
{
    switch (W) {
    case 256: hipLaunchKernelGGL((batch_kernel<Walk, 256>), dim3(grid), dim3(256), lds, s, bd); break;
    case 512: hipLaunchKernelGGL((batch_kernel<Walk, 512>), dim3(grid), dim3(512), lds, s, bd); break;
    default: hipLaunchKernelGGL((batch_kernel<Walk, 1024>), dim3(grid), dim3(1024), lds, s, bd); break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launch helper shared by the per-family translation units
// ---------------------------------------------------------------------------
template <class Walk>
static const void *pick_w(uint32_t W)
{
    switch (W) {
    case 256: return (const void *)scan_kernel<Walk, 256>;
    case 512: return (const void *)scan_kernel<Walk, 512>;
    case 1024: return (const void *)scan_kernel<Walk, 1024>;
    }
    return nullptr;
}

template <class Walk>
static hipError_t launch_w(const typename Walk::Dev &a, const LaunchCfg &c, const ScanDev &sd,
                           const uint32_t *uoff, const uint32_t *uids, uint32_t dupfree,
                           uint32_t tl, hipStream_t s)
{
    const dim3 grid(c.grid), block(c.block_threads);
    switch (c.block_threads) {
    case 256:
        hipLaunchKernelGGL((scan_kernel<Walk, 256>), grid, block, c.lds_bytes, s, a, sd, uoff, uids,
                           dupfree, tl);
        break;
    case 512:
        hipLaunchKernelGGL((scan_kernel<Walk, 512>), grid, block, c.lds_bytes, s, a, sd, uoff, uids,
                           dupfree, tl);
        break;
    default:
        hipLaunchKernelGGL((scan_kernel<Walk, 1024>), grid, block, c.lds_bytes, s, a, sd, uoff,
                           uids, dupfree, tl);
        break;
    }
    return hipGetLastError();
}

// The dense-output kernel of a walker (1024 threads per workgroup).
template <class Walk>
static const void *pick_dense()
{
    return (const void *)scan_kernel<Walk, 1024, true>;
}

template <class Walk>
static hipError_t launch_dense(const typename Walk::Dev &a, const LaunchCfg &c, const ScanDev &sd,
                               const uint32_t *uoff, const uint32_t *uids, uint32_t dupfree,
                               hipStream_t s)
{
    hipLaunchKernelGGL((scan_kernel<Walk, 1024, true>), dim3(c.grid), dim3(1024), c.lds_bytes, s, a,
                       sd, uoff, uids, dupfree, 0u);
    return hipGetLastError();
}

// Kernel families, one translation unit each.
template <int P> const void *batch_kernel_ac16(bool swar, uint32_t W);
template <int P>
hipError_t batch_launch_ac16(const BatchDev &bd, bool swar, uint32_t W, uint32_t grid, uint32_t lds,
                             hipStream_t s);
// One translation unit per placement, each defining its specialisation.
#define MPM_BATCH_AC16_TU(P)                                                                      \
    template <>                                                                                   \
    const void *batch_kernel_ac16<P>(bool swar, uint32_t W)                                       \
    {                                                                                             \
        return swar ? batch_pick_w<AcWalk<uint16_t, P, true, 1>>(W)                               \
                    : batch_pick_w<AcWalk<uint16_t, P, false, 1>>(W);                             \
    }                                                                                             \
    template <>                                                                                   \
    hipError_t batch_launch_ac16<P>(const BatchDev &bd, bool swar, uint32_t W, uint32_t grid,     \
                                    uint32_t lds, hipStream_t s)                                  \
    {                                                                                             \
        return swar ? batch_launch_w<AcWalk<uint16_t, P, true, 1>>(bd, W, grid, lds, s)           \
                    : batch_launch_w<AcWalk<uint16_t, P, false, 1>>(bd, W, grid, lds, s);         \
    }
const void *batch_kernel_other(uint32_t kind, uint32_t W);
hipError_t batch_launch_other(const BatchDev &bd, uint32_t kind, uint32_t W, uint32_t grid,
                              uint32_t lds, hipStream_t s);
const void *wm_kernel(const LaunchCfg &c);
hipError_t wm_launch(const WmDev &a, const LaunchCfg &c, const ScanDev &sd, hipStream_t s);

}  // namespace mpm
