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
//        table sits in LDS when it fits, otherwise it is read through L2.
//        Text bytes are read by each lane with 16-byte loads, one 64-byte
//        block ahead of use.
//   WM - the chunk's text is staged in LDS with 16-byte coalesced loads
//        (Section 4.2.2, collective reads into shared memory); each lane then
//        runs the Wu-Manber window loop (Section 3.2, Algorithm 5) over its
//        window ends with SHIFT in LDS or L2, and verifies candidate windows
//        against HASH/PREFIX and the pattern bytes.
#include <hip/hip_runtime.h>

#include <string.h>

#include <mutex>

#include "mpm_internal.h"

namespace mpm {

// Address-space qualified pointers: LDS tables must be read with ds_read and
// global data with global_load (a generic pointer would give flat loads).
#define LDS_AS __attribute__((address_space(3)))
#define GLB_AS __attribute__((address_space(1)))
template <typename T> using lds_cptr = const LDS_AS T *;
template <typename T> using glb_cptr = const GLB_AS T *;
template <bool InLds, typename T> struct TabPtr { using type = glb_cptr<T>; };
typedef uint32_t v4u __attribute__((ext_vector_type(4)));  // 16-byte load/store unit
template <typename T> struct TabPtr<true, T> { using type = lds_cptr<T>; };

static const int K_SLOTS = 4;  // occurrences a lane keeps in registers
static const uint32_t SPIN_LIMIT = 1u << 24;

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
                    atomicOr(err, 1u);
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

// Lane-ordered exclusive offsets within the chunk plus the chunk offset.
template <int W>
__device__ __forceinline__ uint64_t chunk_offsets(uint32_t cnt, uint64_t *s_scan, uint64_t *status,
                                                  uint64_t g, uint64_t first_g, bool last,
                                                  uint64_t *total, uint32_t epoch, uint32_t *err)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o)
            x += y;
    }
    if (lane == 63)
        s_scan[wave] = x;
    __syncthreads();
    if (wave == 0) {
        uint64_t run = 0;
#pragma unroll
        for (int w = 0; w < W / 64; ++w)
            run += s_scan[w];
        uint64_t excl = look_back(status, g, first_g, run, epoch, err);
        if (lane == 0) {
            uint64_t r = 0;
            for (int w = 0; w < W / 64; ++w) {
                uint64_t t = s_scan[w];
                s_scan[w] = r;
                r += t;
            }
            s_scan[W / 64] = excl;
            if (last)
                *total = excl + run;
        }
    }
    __syncthreads();
    return s_scan[W / 64] + s_scan[wave] + (x - cnt);
}

// Write the ids of distinct string u at position pos, advancing ob.
typedef uint32_t v2u __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void write_ids(mpm_match *out_, uint64_t cap, uint64_t &ob, uint32_t pos,
                                          uint32_t u, const GLB_AS uint32_t *uoff,
                                          const GLB_AS uint32_t *uids, uint32_t dupfree)
{
    GLB_AS v2u *out = (GLB_AS v2u *)out_;
    if (dupfree) {
        if (ob < cap)
            out[ob] = v2u{pos, uids[u]};
        ++ob;
        return;
    }
    const uint32_t b = uoff[u], e = uoff[u + 1];
    for (uint32_t j = b; j < e; ++j) {
        if (ob < cap)
            out[ob] = v2u{pos, uids[j]};
        ++ob;
    }
}

// Cooperative global -> LDS copy (bytes multiple of 16, both 16-aligned).
template <int W>
__device__ __forceinline__ void copy_to_lds(uint8_t *dst, const uint8_t *src, uint32_t bytes)
{
    glb_cptr<v4u> s = (glb_cptr<v4u>)src;
    LDS_AS v4u *d = (LDS_AS v4u *)dst;
    for (uint32_t k = threadIdx.x; k < bytes / 16; k += W)
        d[k] = s[k];
}

// Stream bytes [p, end) of a text through registers: single bytes up to a
// 16-byte boundary, then 64-byte blocks (the next block's loads are issued
// before the current one is consumed), then 16-byte pieces, then bytes.
// one(byte, pos) and sixteen(v4u, pos) consume in text order.
template <class F1, class F16>
__device__ __forceinline__ void stream_text(glb_cptr<uint8_t> text, uint64_t p, uint64_t end,
                                            F1 &&one, F16 &&sixteen)
{
    while (p < end && (((uintptr_t)(text + p)) & 15u)) {
        one((uint32_t)text[p], p);
        ++p;
    }
    if (p + 64 <= end) {
        glb_cptr<v4u> q = (glb_cptr<v4u>)(text + p);
        v4u c0 = q[0], c1 = q[1], c2 = q[2], c3 = q[3];
        while (true) {
            const bool more = p + 128 <= end;
            glb_cptr<v4u> nq = (glb_cptr<v4u>)(text + (more ? p + 64 : p));
            const v4u n0 = nq[0], n1 = nq[1], n2 = nq[2], n3 = nq[3];
            sixteen(c0, p);
            sixteen(c1, p + 16);
            sixteen(c2, p + 32);
            sixteen(c3, p + 48);
            p += 64;
            if (!more)
                break;
            c0 = n0;
            c1 = n1;
            c2 = n2;
            c3 = n3;
        }
    }
    while (p + 16 <= end) {
        sixteen(*(glb_cptr<v4u>)(text + p), p);
        p += 16;
    }
    while (p < end) {
        one((uint32_t)text[p], p);
        ++p;
    }
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
    return col & ~((nz >> 7) * 0xFFu);
}

template <typename St, bool InLds, bool Swar>
struct AcWalk {
    using Dev = AcDev;
    typename TabPtr<InLds, uint8_t>::type dfab;  // table, addressed in bytes
    lds_cptr<uint16_t> cls;                      // column byte offset per byte value
    uint32_t rowb, first_term, m, sh, pb_lo, pb_hi, pc_lo, pc_hi;

    template <int W>
    __device__ __forceinline__ void setup(const AcDev &a, uint8_t *smem, uint32_t /*unused*/)
    {
        rowb = a.cp * (uint32_t)sizeof(St);
        first_term = a.first_term;
        m = a.m;
        sh = a.swar_shift;
        pb_lo = a.perm_byte_lo;
        pb_hi = a.perm_byte_hi;
        pc_lo = a.perm_col_lo;
        pc_hi = a.perm_col_hi;
        copy_to_lds<W>(smem, a.cls, 512);
        cls = (lds_cptr<uint16_t>)smem;
        if (InLds) {
            copy_to_lds<W>(smem + 512, (const uint8_t *)a.dfa, a.dfa_bytes);
            dfab = (typename TabPtr<InLds, uint8_t>::type)(smem + 512);
        } else {
            dfab = (typename TabPtr<InLds, uint8_t>::type)a.dfa;
        }
        __syncthreads();
    }

    // One transition: row s, column at byte offset coloff.
    __device__ __forceinline__ uint32_t next(uint32_t s, uint32_t coloff) const
    {
        const uint32_t off = sizeof(St) == 2 ? __umul24(s, rowb) + coloff : s * rowb + coloff;
        return *(typename TabPtr<InLds, St>::type)(dfab + off);
    }

    // Walk bytes [p, end) from the root; cb(start, u) for every terminal
    // state reached (start = index of the byte - m + 1).
    template <class F>
    __device__ __forceinline__ void walk(glb_cptr<uint8_t> text, uint64_t p, uint64_t end,
                                         F &cb) const
    {
        uint32_t s = 0;
        stream_text(
            text, p, end,
            [&](uint32_t b, uint64_t q) {
                s = next(s, cls[b]);
                if (s >= first_term)
                    cb(q + 1 - m, s - first_term);
            },
            [&](const v4u c, uint64_t q) {
                uint32_t cw[4];
                if (Swar) {
                    cw[0] = swar_cols(c.x, sh, pb_lo, pb_hi, pc_lo, pc_hi);
                    cw[1] = swar_cols(c.y, sh, pb_lo, pb_hi, pc_lo, pc_hi);
                    cw[2] = swar_cols(c.z, sh, pb_lo, pb_hi, pc_lo, pc_hi);
                    cw[3] = swar_cols(c.w, sh, pb_lo, pb_hi, pc_lo, pc_hi);
                }
                uint32_t st[16];
                uint32_t mx = 0;
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    uint32_t col;
                    if (Swar) {
                        col = (cw[k >> 2] >> (8 * (k & 3))) & 0xffu;
                    } else {
                        const uint32_t w = k < 4 ? c.x : k < 8 ? c.y : k < 12 ? c.z : c.w;
                        col = cls[(w >> (8 * (k & 3))) & 0xffu];
                    }
                    s = next(s, col);
                    st[k] = s;
                    mx = max(mx, s);
                }
                if (mx >= first_term) {
#pragma unroll
                    for (int k = 0; k < 16; ++k)
                        if (st[k] >= first_term)
                            cb(q + k + 1 - m, st[k] - first_term);
                }
            });
    }

    // Lane range: starts [lo, hi) relative to the chunk at text offset base.
    template <class F>
    __device__ __forceinline__ void lane(glb_cptr<uint8_t> text, uint64_t n, uint64_t base,
                                         uint32_t lo, uint32_t hi, F &&cb) const
    {
        uint64_t end = base + hi + m - 1;
        if (end > n)
            end = n;
        walk(text, base + lo, end, cb);
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

template <bool InLds>
struct WmWalk {
    using Dev = WmDev;
    typename TabPtr<InLds, uint16_t>::type sh16;
    typename TabPtr<InLds, uint32_t>::type boff, bkey, bu;
    glb_cptr<uint8_t> pats;
    uint32_t m, B, csh, kl, hmask, kmask;

    template <int W>
    __device__ __forceinline__ void setup(const WmDev &a, uint8_t *smem, uint32_t /*unused*/)
    {
        m = a.m;
        B = a.B;
        csh = a.code_shift;
        kl = a.key_len;
        hmask = (1u << (2 * B)) - 1u;
        kmask = kl >= 16 ? 0xffffffffu : ((1u << (2 * kl)) - 1u);
        const uint8_t *base = a.tables;
        if (InLds) {
            copy_to_lds<W>(smem, a.tables, a.table_bytes);
            base = smem;
        }
        sh16 = (typename TabPtr<InLds, uint16_t>::type)base;
        boff = (typename TabPtr<InLds, uint32_t>::type)(base + a.off_boff);
        bkey = (typename TabPtr<InLds, uint32_t>::type)(base + a.off_bkey);
        bu = (typename TabPtr<InLds, uint32_t>::type)(base + a.off_bu);
        pats = (glb_cptr<uint8_t>)a.pats;
        __syncthreads();
    }

    // 32 bits of the 96-bit history {h2:h1:h0} from bit o (o <= 64).
    __device__ __forceinline__ static uint32_t bits(uint32_t h0, uint32_t h1, uint32_t h2, uint32_t o)
    {
        const uint32_t q = o >> 5;
        const uint32_t lo = q == 0 ? h0 : (q == 1 ? h1 : h2);
        const uint32_t hi = q == 0 ? h1 : h2;
        return __builtin_amdgcn_alignbit(hi, lo, o & 31u);
    }

    // Window loop (Algorithm 5) over one lane's range, the text streamed
    // through registers. The history keeps the 2-bit codes of the last 48
    // characters read (positions [e-48, e), position q at bit 2(q-e+48)).
    // Every window end nx < e is examined: the hash of its last B
    // characters picks SHIFT; a zero shift sends the window to its bucket,
    // where the filter key (codes of the key_len characters before the block)
    // must equal the candidate's before the window is compared byte by byte
    // with the pattern.
    template <class F>
    __device__ __forceinline__ void lane(glb_cptr<uint8_t> text, uint64_t n, uint64_t base,
                                         uint32_t lo, uint32_t hi, F &&cb) const
    {
        const uint64_t p = base + lo;
        uint64_t end = base + hi + m - 1;
        if (end > n)
            end = n;
        uint64_t nx = p + m - 1;
        uint64_t e = p;
        uint32_t h0 = 0, h1 = 0, h2 = 0;
        uint32_t qn = 0;
        uint64_t qp[WM_QUEUE];
        uint32_t qu[WM_QUEUE];
#pragma unroll
        for (int k = 0; k < WM_QUEUE; ++k) {
            qp[k] = 0;
            qu[k] = 0;
        }
        auto flush = [&]() {
#pragma unroll
            for (int k = 0; k < WM_QUEUE; ++k) {
                if ((uint32_t)k < qn) {
                    const uint64_t st = qp[k] + 1 - m;
                    glb_cptr<uint8_t> pp = pats + (uint64_t)qu[k] * m;
                    bool ok = true;
                    for (uint32_t j = 0; j < m; ++j)
                        if (pp[j] != text[st + j]) {
                            ok = false;
                            break;
                        }
                    if (ok)
                        cb(st, qu[k]);
                }
            }
            qn = 0;
        };
        auto windows = [&]() {
            while (nx < e) {
                const uint32_t o = 2u * (uint32_t)(nx + 49 - e - B);
                const uint32_t h = bits(h0, h1, h2, o) & hmask;
                const uint32_t sv = sh16[h];
                if (sv & 0x8000u) {
                    const uint32_t b = sv & 0x7fffu;
                    const uint32_t key = kl ? (bits(h0, h1, h2, o - 2u * kl) & kmask) : 0u;
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
                h0 = (h0 >> 2) | (h1 << 30);
                h1 = (h1 >> 2) | (h2 << 30);
                h2 = (h2 >> 2) | (((b >> csh) & 3u) << 30);
                e += 1;
                windows();
            },
            [&](const v4u c, uint64_t) {
                h0 = h1;
                h1 = h2;
                h2 = codes4(c.x, csh) | (codes4(c.y, csh) << 8) | (codes4(c.z, csh) << 16) |
                     (codes4(c.w, csh) << 24);
                e += 16;
                windows();
            });
        flush();
    }
};

// ---------------------------------------------------------------------------
// Persistent chunk driver
// ---------------------------------------------------------------------------
template <class Walk, int W>
__global__ __launch_bounds__(W) void scan_kernel(typename Walk::Dev a, ScanDev sd,
                                                 const uint32_t *uoff_, const uint32_t *uids_,
                                                 uint32_t dupfree, uint32_t unused)
{
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ TextDesc s_td;
    __shared__ uint64_t s_tile;
    __shared__ uint32_t s_epoch;
    __shared__ uint64_t s_scan[W / 64 + 1];

    // Launch constants as plain values (no by-reference use of the argument
    // structs, which would place them in private memory).
    const uint32_t ntexts = sd.ntexts;
    const uint64_t ntiles = sd.ntiles;
    const uint32_t L = sd.lane_bytes;
    uint32_t *const hdr = sd.hdr;
    uint64_t *const status = sd.status;
    const TextDesc *const multi = sd.multi;
    glb_cptr<uint32_t> uoff = (glb_cptr<uint32_t>)uoff_;
    glb_cptr<uint32_t> uids = (glb_cptr<uint32_t>)uids_;
    const uint32_t m = a.m;
    const uint64_t chunk = (uint64_t)W * L;

    Walk wk;
    wk.template setup<W>(a, smem, unused);
    if (threadIdx.x == 0)
        s_epoch = __hip_atomic_load(&hdr[WS_EPOCH], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    while (true) {
        if (threadIdx.x == 0) {
            const uint64_t t = atomicAdd(&hdr[WS_TICKET], 1u);
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
        glb_cptr<uint8_t> text = (glb_cptr<uint8_t>)s_td.text;
        const uint64_t n = s_td.n;
        mpm_match *const out = s_td.out;
        const uint64_t cap = s_td.cap;
        uint64_t *const total = s_td.total;
        const uint64_t first_g = s_td.tile_begin;
        const uint64_t nt = s_td.ntiles;
        const uint32_t epoch = s_epoch;
        const uint64_t lt = g - first_g;
        const uint64_t ns = n - m + 1;
        const uint64_t base = lt * chunk;
        const uint64_t starts = (ns - base) < chunk ? (ns - base) : chunk;

        const uint32_t lo0 = threadIdx.x * L;
        const uint32_t lo = lo0 < starts ? lo0 : (uint32_t)starts;
        const uint32_t hi = (lo0 + L) < starts ? (lo0 + L) : (uint32_t)starts;

        // Phase A: count and keep the first occurrences.
        uint32_t nu = 0, nid = 0;
        uint32_t so[K_SLOTS], su[K_SLOTS];
#pragma unroll
        for (int k = 0; k < K_SLOTS; ++k) {
            so[k] = 0;
            su[k] = 0;
        }
        if (lo < hi) {
            wk.lane(text, n, base, lo, hi, [&](uint64_t start, uint32_t u) {
#pragma unroll
                for (int k = 0; k < K_SLOTS; ++k)
                    if (nu == (uint32_t)k) {
                        so[k] = (uint32_t)start;
                        su[k] = u;
                    }
                ++nu;
                nid += dupfree ? 1u : (uoff[u + 1] - uoff[u]);
            });
        }

        // Phase B: offsets.
        const bool last = lt + 1 == nt;
        uint64_t ob = chunk_offsets<W>(nid, s_scan, status, g, first_g, last, total, epoch,
                                       &hdr[WS_ERR]);

        // Phase C: ordered writes.
        if (nu != 0) {
            if (nu <= (uint32_t)K_SLOTS) {
#pragma unroll
                for (int k = 0; k < K_SLOTS; ++k)
                    if ((uint32_t)k < nu)
                        write_ids(out, cap, ob, so[k], su[k], uoff, uids, dupfree);
            } else {
                wk.lane(text, n, base, lo, hi, [&](uint64_t start, uint32_t u) {
                    write_ids(out, cap, ob, (uint32_t)start, u, uoff, uids, dupfree);
                });
            }
        }
        __syncthreads();
    }

    if (threadIdx.x == 0) {
        const uint32_t dn = atomicAdd(&hdr[WS_DONE], 1u);
        if (dn == gridDim.x - 1) {
            __hip_atomic_store(&hdr[WS_TICKET], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&hdr[WS_DONE], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&hdr[WS_EPOCH], s_epoch + 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__global__ void zero_totals_kernel(uint64_t *const *ptrs, uint32_t count, uint64_t *single)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (single) {
        if (i == 0)
            *single = 0;
        return;
    }
    if (i < count)
        *ptrs[i] = 0;
}

// ---------------------------------------------------------------------------
// Host: variant resolution and launch
// ---------------------------------------------------------------------------
struct DeviceLimits {
    int cus = 0;
    int max_lds = 0;
};

static DeviceLimits limits()
{
    static std::mutex mu;
    static DeviceLimits cache[64];
    static bool have[64] = {false};
    int dev = 0;
    hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(mu);
    if (dev < 0 || dev >= 64)
        dev = 0;
    if (!have[dev]) {
        DeviceLimits L;
        hipDeviceGetAttribute(&L.cus, hipDeviceAttributeMultiprocessorCount, dev);
        hipDeviceGetAttribute(&L.max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (L.cus <= 0)
            L.cus = 256;
        if (L.max_lds <= 0)
            L.max_lds = 65536;
        cache[dev] = L;
        have[dev] = true;
    }
    return cache[dev];
}

static AcDev ac_dev(const mpm_index *ix)
{
    AcDev a;
    a.dfa = ix->d_image + ix->off_a;
    a.cls = ix->d_image + ix->off_b;
    a.uoff = (const uint32_t *)(ix->d_image + ix->off_c);
    a.uids = (const uint32_t *)(ix->d_image + ix->off_d);
    a.n_states = (uint32_t)ix->n_states;
    a.first_term = (uint32_t)(ix->n_states - ix->du);
    a.cp = ix->n_classes + 1;
    a.m = ix->m;
    a.dfa_bytes = (uint32_t)ix->table_bytes;
    a.dupfree = ix->max_dup == 1;
    a.swar_ok = ix->swar_ok;
    a.swar_shift = ix->swar_shift;
    uint32_t w[4];
    memcpy(&w[0], ix->perm_byte, 4);
    memcpy(&w[1], ix->perm_byte + 4, 4);
    memcpy(&w[2], ix->perm_col, 4);
    memcpy(&w[3], ix->perm_col + 4, 4);
    a.perm_byte_lo = w[0];
    a.perm_byte_hi = w[1];
    a.perm_col_lo = w[2];
    a.perm_col_hi = w[3];
    return a;
}

static WmDev wm_dev(const mpm_index *ix)
{
    WmDev a;
    a.tables = ix->d_image + ix->off_a;
    a.off_boff = (uint32_t)(ix->off_b - ix->off_a);
    a.off_bkey = (uint32_t)(ix->off_c - ix->off_a);
    a.off_bu = (uint32_t)(ix->off_d - ix->off_a);
    a.pats = ix->d_image + ix->off_e;
    a.uoff = (const uint32_t *)(ix->d_image + ix->off_f);
    a.uids = (const uint32_t *)(ix->d_image + ix->off_g);
    a.B = ix->B;
    a.code_shift = ix->code_shift;
    a.m = ix->m;
    a.key_len = ix->key_len;
    a.table_bytes = (uint32_t)ix->table_bytes;
    a.dupfree = ix->max_dup == 1;
    return a;
}

// Kernel pointer for a resolved configuration.
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

static const void *kernel_for(const mpm_index *ix, const LaunchCfg &c)
{
    const bool lds = c.placement == MPM_PLACE_LDS;
    if (ix->algo == MPM_ALGO_AC) {
        const bool sw = c.swar;
        if (ix->state_bytes == 2) {
            if (lds)
                return sw ? pick_w<AcWalk<uint16_t, true, true>>(c.block_threads)
                          : pick_w<AcWalk<uint16_t, true, false>>(c.block_threads);
            return sw ? pick_w<AcWalk<uint16_t, false, true>>(c.block_threads)
                      : pick_w<AcWalk<uint16_t, false, false>>(c.block_threads);
        }
        if (lds)
            return sw ? pick_w<AcWalk<uint32_t, true, true>>(c.block_threads)
                      : pick_w<AcWalk<uint32_t, true, false>>(c.block_threads);
        return sw ? pick_w<AcWalk<uint32_t, false, true>>(c.block_threads)
                  : pick_w<AcWalk<uint32_t, false, false>>(c.block_threads);
    }
    return lds ? pick_w<WmWalk<true>>(c.block_threads) : pick_w<WmWalk<false>>(c.block_threads);
}

static const uint32_t STATIC_LDS_RESERVE = 512;

uint64_t tile_bytes(const LaunchCfg &cfg) { return (uint64_t)cfg.lane_bytes * cfg.block_threads; }

mpm_status resolve_variant(const mpm_index *ix, const mpm_variant *v, uint64_t ntiles,
                           LaunchCfg *cfg)
{
    mpm_variant d = {0, 0, 0, 0, 0};
    if (v)
        d = *v;
    uint32_t L = d.lane_bytes ? d.lane_bytes : 64;
    uint32_t W = d.block_threads ? d.block_threads : 256;
    if (L % 16 || L < 16 || L > 4096)
        return fail(MPM_EINVAL, "variant: lane_bytes=%u must be a multiple of 16 in 16..4096", L);
    if (W != 256 && W != 512 && W != 1024)
        return fail(MPM_EINVAL, "variant: block_threads=%u must be 256, 512 or 1024", W);
    if (d.placement > MPM_PLACE_GLOBAL)
        return fail(MPM_EINVAL, "variant: unknown placement %u", d.placement);
    const DeviceLimits lim = limits();
    const uint32_t fixed = ix->algo == MPM_ALGO_AC ? 512u : 0u;  // AC byte-class map
    const uint64_t table_lds = fixed + ix->table_bytes;
    const bool fits = table_lds + STATIC_LDS_RESERVE <= (uint64_t)lim.max_lds;
    uint32_t place = d.placement;
    if (place == MPM_PLACE_AUTO)
        place = fits ? MPM_PLACE_LDS : MPM_PLACE_GLOBAL;
    if (place == MPM_PLACE_LDS && !fits)
        return fail(MPM_EUNSUPPORTED, "variant: tables of %llu bytes do not fit in LDS",
                    (unsigned long long)ix->table_bytes);
    cfg->lane_bytes = L;
    cfg->block_threads = W;
    cfg->placement = place;
    cfg->swar = ix->algo == MPM_ALGO_AC && ix->swar_ok && !(d.flags & MPM_VARIANT_NO_SWAR);
    cfg->lds_bytes = fixed + (place == MPM_PLACE_LDS ? (uint32_t)ix->table_bytes : 0u);
    cfg->grid = 0;
    if (ntiles) {
        const void *k = kernel_for(ix, *cfg);
        if (cfg->lds_bytes > 65536)
            hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cfg->lds_bytes);
        int nb = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, (int)W, cfg->lds_bytes);
        if (e != hipSuccess || nb <= 0)
            nb = 1;
        uint64_t grid = (uint64_t)nb * lim.cus;
        if (d.grid)
            grid = d.grid;
        if (grid > ntiles)
            grid = ntiles;
        if (grid < 1)
            grid = 1;
        cfg->grid = (uint32_t)grid;
    }
    return MPM_OK;
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

mpm_status launch_scan(const mpm_index *ix, const LaunchCfg &c, const ScanDev &sd, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const bool lds = c.placement == MPM_PLACE_LDS;
    hipError_t e;
    if (c.lds_bytes > 65536)
        hipFuncSetAttribute(kernel_for(ix, c), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)c.lds_bytes);
    if (ix->algo == MPM_ALGO_AC) {
        AcDev a = ac_dev(ix);
        const bool sw = c.swar;
#define MPM_AC(ST, LD, SW) launch_w<AcWalk<ST, LD, SW>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s)
        if (ix->state_bytes == 2)
            e = lds ? (sw ? MPM_AC(uint16_t, true, true) : MPM_AC(uint16_t, true, false))
                    : (sw ? MPM_AC(uint16_t, false, true) : MPM_AC(uint16_t, false, false));
        else
            e = lds ? (sw ? MPM_AC(uint32_t, true, true) : MPM_AC(uint32_t, true, false))
                    : (sw ? MPM_AC(uint32_t, false, true) : MPM_AC(uint32_t, false, false));
#undef MPM_AC
    } else {
        WmDev a = wm_dev(ix);
        e = lds ? launch_w<WmWalk<true>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s)
                : launch_w<WmWalk<false>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
    }
    if (e != hipSuccess)
        return fail(MPM_EHIP, "scan launch: %s", hipGetErrorString(e));
    return MPM_OK;
}

mpm_status launch_zero_totals(uint64_t *const *d_totals_dev, uint32_t count, uint64_t *single,
                              void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    uint32_t blocks = single ? 1 : (count + 255) / 256;
    if (blocks == 0)
        return MPM_OK;
    hipLaunchKernelGGL(zero_totals_kernel, dim3(blocks), dim3(256), 0, s, d_totals_dev, count, single);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(MPM_EHIP, "zero-total launch: %s", hipGetErrorString(e));
    return MPM_OK;
}

}  // namespace mpm
