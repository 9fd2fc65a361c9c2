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

#include <mutex>

#include "mpm_internal.h"

namespace mpm {

static const int K_SLOTS = 4;  // occurrences a lane keeps in registers
static const uint32_t SPIN_LIMIT = 1u << 24;

// ---------------------------------------------------------------------------
// Look-back status words
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t ld_acquire(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_release(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t make_status(uint32_t epoch, uint32_t flag, uint64_t val)
{
    return ((uint64_t)(epoch & ST_EPOCH_MASK) << 38) | ((uint64_t)flag << ST_VAL_BITS) |
           (val & ST_VAL_MASK);
}

// Publish this chunk's count and find the sum of all earlier chunks of the
// same text. flag 1: count of this chunk only; flag 2: inclusive prefix.
__device__ uint64_t look_back(uint64_t *status, uint64_t g, uint64_t agg, bool first,
                              uint32_t epoch, uint32_t *err)
{
    if (first) {
        st_release(&status[g], make_status(epoch, 2, agg));
        return 0;
    }
    st_release(&status[g], make_status(epoch, 1, agg));
    uint64_t excl = 0;
    uint64_t j = g - 1;
    uint32_t spins = 0;
    const uint64_t tag = epoch & ST_EPOCH_MASK;
    while (true) {
        uint64_t v = ld_acquire(&status[j]);
        uint32_t fl = (uint32_t)(v >> ST_VAL_BITS) & 3u;
        if ((v >> 38) != tag || fl == 0) {
            if (++spins > SPIN_LIMIT) {  // never expected; keeps every wave finite
                atomicOr(err, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        excl += v & ST_VAL_MASK;
        if (fl == 2)
            break;
        --j;
    }
    st_release(&status[g], make_status(epoch, 2, excl + agg));
    return excl;
}

// Lane-ordered exclusive offsets within the chunk plus the chunk offset.
template <int W>
__device__ __forceinline__ uint64_t chunk_offsets(uint32_t cnt, uint64_t *s_scan, uint64_t *status,
                                                  uint64_t g, bool first, bool last,
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
    if (threadIdx.x == 0) {
        uint64_t run = 0;
#pragma unroll
        for (int w = 0; w < W / 64; ++w) {
            uint64_t t = s_scan[w];
            s_scan[w] = run;
            run += t;
        }
        uint64_t excl = look_back(status, g, run, first, epoch, err);
        s_scan[W / 64] = excl;
        if (last)
            *total = excl + run;
    }
    __syncthreads();
    return s_scan[W / 64] + s_scan[wave] + (x - cnt);
}

// Write the ids of distinct string u at position pos, advancing ob.
__device__ __forceinline__ void write_ids(mpm_match *__restrict__ out, uint64_t cap, uint64_t &ob,
                                          uint32_t pos, uint32_t u, const uint32_t *__restrict__ uoff,
                                          const uint32_t *__restrict__ uids, uint32_t dupfree)
{
    if (dupfree) {
        if (ob < cap)
            *(uint2 *)&out[ob] = make_uint2(pos, uids[u]);
        ++ob;
        return;
    }
    const uint32_t b = uoff[u], e = uoff[u + 1];
    for (uint32_t j = b; j < e; ++j) {
        if (ob < cap)
            *(uint2 *)&out[ob] = make_uint2(pos, uids[j]);
        ++ob;
    }
}

// Cooperative global -> LDS copy (bytes multiple of 16, both 16-aligned).
template <int W>
__device__ __forceinline__ void copy_to_lds(uint8_t *dst, const uint8_t *src, uint32_t bytes)
{
    const uint4 *s = (const uint4 *)src;
    uint4 *d = (uint4 *)dst;
    for (uint32_t k = threadIdx.x; k < bytes / 16; k += W)
        d[k] = s[k];
}

// ---------------------------------------------------------------------------
// Aho-Corasick walker
// ---------------------------------------------------------------------------
template <typename St, bool LDS>
struct AcWalk {
    using Dev = AcDev;
    const St *dfa;
    const uint8_t *cls;
    uint32_t cp, first_term, m;

    static uint32_t lds_bytes(const AcDev &a, uint32_t /*W*/, uint32_t /*L*/)
    {
        return 256 + (LDS ? a.dfa_bytes : 0);
    }

    template <int W>
    __device__ void setup(const AcDev &a, uint8_t *smem, uint32_t /*text_lds_bytes*/)
    {
        cp = a.cp;
        first_term = a.first_term;
        m = a.m;
        copy_to_lds<W>(smem, a.cls, 256);
        cls = smem;
        if (LDS) {
            copy_to_lds<W>(smem + 256, (const uint8_t *)a.dfa, a.dfa_bytes);
            dfa = (const St *)(smem + 256);
        } else {
            dfa = (const St *)a.dfa;
        }
        __syncthreads();
    }

    template <int W>
    __device__ void begin_chunk(const TextDesc &, uint64_t, uint64_t) {}

    template <class F>
    __device__ __forceinline__ void chunk16(uint32_t &s, const uint4 c, uint64_t p, F &cb) const
    {
        uint32_t st[16];
        uint32_t mx = 0;
        const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            uint32_t b = (w[k >> 2] >> (8 * (k & 3))) & 0xffu;
            s = dfa[s * cp + cls[b]];
            st[k] = s;
            mx = max(mx, s);
        }
        if (mx >= first_term) {
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (st[k] >= first_term)
                    cb(p + k + 1 - m, st[k] - first_term);
        }
    }

    // Walk bytes [p, end) of the text from the root; cb(start, u) for every
    // terminal state reached (start = index of the byte - m + 1).
    template <class F>
    __device__ __forceinline__ void walk(const uint8_t *__restrict__ text, uint64_t p, uint64_t end,
                                         F &&cb) const
    {
        uint32_t s = 0;
        while (p < end && (((uintptr_t)(text + p)) & 15u)) {
            s = dfa[s * cp + cls[text[p]]];
            if (s >= first_term)
                cb(p + 1 - m, s - first_term);
            ++p;
        }
        if (p + 64 <= end) {
            const uint4 *q = (const uint4 *)(text + p);
            uint4 c0 = q[0], c1 = q[1], c2 = q[2], c3 = q[3];
            while (true) {
                const bool more = p + 128 <= end;
                const uint4 *nq = (const uint4 *)(text + (more ? p + 64 : p));
                uint4 n0 = nq[0], n1 = nq[1], n2 = nq[2], n3 = nq[3];
                chunk16(s, c0, p, cb);
                chunk16(s, c1, p + 16, cb);
                chunk16(s, c2, p + 32, cb);
                chunk16(s, c3, p + 48, cb);
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
            uint4 c = *(const uint4 *)(text + p);
            chunk16(s, c, p, cb);
            p += 16;
        }
        while (p < end) {
            s = dfa[s * cp + cls[text[p]]];
            if (s >= first_term)
                cb(p + 1 - m, s - first_term);
            ++p;
        }
    }

    // Lane range: starts [lo, hi) relative to the chunk at text offset base.
    template <class F>
    __device__ __forceinline__ void lane(const TextDesc &td, uint64_t base, uint32_t lo, uint32_t hi,
                                         F &&cb) const
    {
        uint64_t p = base + lo;
        uint64_t end = base + hi + m - 1;
        if (end > td.n)
            end = td.n;
        walk(td.text, p, end, cb);
    }
};

// ---------------------------------------------------------------------------
// Wu-Manber walker
// ---------------------------------------------------------------------------
template <bool LDS>
struct WmWalk {
    using Dev = WmDev;
    const uint8_t *shift;
    uint8_t *tb;  // chunk text in LDS
    const uint32_t *boff, *bu, *prefix;
    const uint8_t *pats;
    uint32_t m, B, sh;

    static uint32_t lds_bytes(const WmDev &a, uint32_t W, uint32_t L)
    {
        uint32_t text = (W * L + 64 + 15) & ~15u;
        return text + (LDS ? a.shift_bytes : 0);
    }

    // LDS: the chunk's text first, then SHIFT when it is placed in LDS.
    template <int W>
    __device__ void setup(const WmDev &a, uint8_t *smem, uint32_t text_bytes)
    {
        m = a.m;
        B = a.B;
        sh = a.code_shift;
        boff = a.boff;
        bu = a.bu;
        prefix = a.prefix;
        pats = a.pats;
        tb = smem;
        shift = a.shift;
        if (LDS) {
            copy_to_lds<W>(smem + text_bytes, a.shift, a.shift_bytes);
            shift = smem + text_bytes;
        }
        __syncthreads();
    }

    // Stage the chunk's bytes [base, base + starts + m - 1) into LDS.
    template <int W>
    __device__ void begin_chunk(const TextDesc &td, uint64_t base, uint64_t starts)
    {
        uint64_t len = starts + m - 1;
        if (base + len > td.n)
            len = td.n - base;
        const uint8_t *src = td.text + base;
        const uint32_t L32 = (uint32_t)len;
        if ((((uintptr_t)src) & 15u) == 0) {
            const uint32_t nv = L32 / 16;
            for (uint32_t k = threadIdx.x; k < nv; k += W)
                ((uint4 *)tb)[k] = ((const uint4 *)src)[k];
            for (uint32_t k = nv * 16 + threadIdx.x; k < L32; k += W)
                tb[k] = src[k];
        } else {
            for (uint32_t k = threadIdx.x; k < L32; k += W)
                tb[k] = src[k];
        }
        __syncthreads();
    }

    template <class F>
    __device__ __forceinline__ void verify(uint32_t i, uint32_t h, uint64_t base, F &cb) const
    {
        const uint32_t ws = i + 1 - m;
        const uint32_t pk = m < 4 ? m : 4;
        uint32_t key = 0;
        for (uint32_t k = 0; k < pk; ++k)
            key |= (uint32_t)tb[ws + k] << (8 * k);
        const uint32_t e = boff[h + 1];
        for (uint32_t j = boff[h]; j < e; ++j) {
            const uint32_t u = bu[j];
            if (prefix[u] != key)
                continue;
            const uint8_t *pp = pats + (uint64_t)u * m;
            bool ok = true;
            for (uint32_t k = pk; k < m; ++k)
                if (pp[k] != tb[ws + k]) {
                    ok = false;
                    break;
                }
            if (ok) {  // distinct strings of equal length: at most one matches
                cb(base + ws, u);
                break;
            }
        }
    }

    template <class F>
    __device__ __forceinline__ void lane(const TextDesc &, uint64_t base, uint32_t lo, uint32_t hi,
                                         F &&cb) const
    {
        uint32_t i = lo + m - 1;
        const uint32_t iend = hi + m - 1;
        while (i < iend) {
            uint32_t h = 0;
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k)
                if (k < B)
                    h |= (((uint32_t)tb[i + 1 - B + k] >> sh) & 3u) << (2 * k);
            const uint32_t s = shift[h];
            if (s == 0) {
                verify(i, h, base, cb);
                i += 1;
            } else {
                i += s;
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Persistent chunk driver
// ---------------------------------------------------------------------------
template <class Walk, int W>
__device__ __forceinline__ void find_text(const ScanDev &sd, uint64_t g, TextDesc &td)
{
    if (sd.ntexts == 1) {
        td = sd.single;
        return;
    }
    uint32_t lo = 0, hi = sd.ntexts;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (sd.multi[mid].tile_begin <= g)
            lo = mid;
        else
            hi = mid;
    }
    td = sd.multi[lo];
}

template <class Walk, int W>
__global__ __launch_bounds__(W) void scan_kernel(typename Walk::Dev a, ScanDev sd,
                                                 const uint32_t *uoff, const uint32_t *uids,
                                                 uint32_t dupfree, uint32_t text_lds_bytes)
{
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ TextDesc s_td;
    __shared__ uint64_t s_tile;
    __shared__ uint32_t s_epoch;
    __shared__ uint64_t s_scan[W / 64 + 1];

    Walk wk;
    wk.template setup<W>(a, smem, text_lds_bytes);
    if (threadIdx.x == 0)
        s_epoch = __hip_atomic_load(&sd.hdr[WS_EPOCH], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    const uint32_t L = sd.lane_bytes;
    const uint64_t chunk = (uint64_t)W * L;
    const uint32_t m = a.m;

    while (true) {
        if (threadIdx.x == 0) {
            uint64_t t = atomicAdd(&sd.hdr[WS_TICKET], 1u);
            s_tile = t;
            if (t < sd.ntiles)
                find_text<Walk, W>(sd, t, s_td);
        }
        __syncthreads();
        const uint64_t g = s_tile;
        if (g >= sd.ntiles)
            break;
        const TextDesc td = s_td;
        const uint32_t epoch = s_epoch;
        const uint64_t lt = g - td.tile_begin;
        const uint64_t ns = td.n - m + 1;
        const uint64_t base = lt * chunk;
        const uint64_t starts = (ns - base) < chunk ? (ns - base) : chunk;

        wk.template begin_chunk<W>(td, base, starts);

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
            wk.lane(td, base, lo, hi, [&](uint64_t start, uint32_t u) {
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
        const bool first = lt == 0;
        const bool last = lt + 1 == td.ntiles;
        uint64_t ob = chunk_offsets<W>(nid, s_scan, sd.status, g, first, last, td.total, epoch,
                                       &sd.hdr[WS_ERR]);

        // Phase C: ordered writes.
        if (nu != 0) {
            if (nu <= (uint32_t)K_SLOTS) {
#pragma unroll
                for (int k = 0; k < K_SLOTS; ++k)
                    if ((uint32_t)k < nu)
                        write_ids(td.out, td.cap, ob, so[k], su[k], uoff, uids, dupfree);
            } else {
                wk.lane(td, base, lo, hi, [&](uint64_t start, uint32_t u) {
                    write_ids(td.out, td.cap, ob, (uint32_t)start, u, uoff, uids, dupfree);
                });
            }
        }
        __syncthreads();
    }

    if (threadIdx.x == 0) {
        uint32_t dn = atomicAdd(&sd.hdr[WS_DONE], 1u);
        if (dn == gridDim.x - 1) {
            __hip_atomic_store(&sd.hdr[WS_TICKET], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&sd.hdr[WS_DONE], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&sd.hdr[WS_EPOCH], s_epoch + 1u, __ATOMIC_RELEASE,
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
    return a;
}

static WmDev wm_dev(const mpm_index *ix)
{
    WmDev a;
    a.shift = ix->d_image + ix->off_a;
    a.boff = (const uint32_t *)(ix->d_image + ix->off_b);
    a.bu = (const uint32_t *)(ix->d_image + ix->off_c);
    a.prefix = (const uint32_t *)(ix->d_image + ix->off_d);
    a.pats = ix->d_image + ix->off_e;
    a.uoff = (const uint32_t *)(ix->d_image + ix->off_f);
    a.uids = (const uint32_t *)(ix->d_image + ix->off_g);
    a.B = ix->B;
    a.code_shift = ix->code_shift;
    a.m = ix->m;
    a.shift_bytes = (uint32_t)ix->table_bytes;
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
        if (ix->state_bytes == 2)
            return lds ? pick_w<AcWalk<uint16_t, true>>(c.block_threads)
                       : pick_w<AcWalk<uint16_t, false>>(c.block_threads);
        return lds ? pick_w<AcWalk<uint32_t, true>>(c.block_threads)
                   : pick_w<AcWalk<uint32_t, false>>(c.block_threads);
    }
    return lds ? pick_w<WmWalk<true>>(c.block_threads) : pick_w<WmWalk<false>>(c.block_threads);
}

static uint32_t text_lds(const mpm_index *ix, uint32_t W, uint32_t L)
{
    if (ix->algo != MPM_ALGO_WM)
        return 0;
    return (W * L + 64 + 15) & ~15u;
}

static const uint32_t STATIC_LDS_RESERVE = 512;

uint64_t tile_bytes(const LaunchCfg &cfg) { return (uint64_t)cfg.lane_bytes * cfg.block_threads; }

mpm_status resolve_variant(const mpm_index *ix, const mpm_variant *v, uint64_t ntiles,
                           LaunchCfg *cfg)
{
    mpm_variant d = {0, 0, 0, 0};
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
    const uint32_t tl = text_lds(ix, W, L);
    if (tl + STATIC_LDS_RESERVE + 256 > (uint32_t)lim.max_lds)
        return fail(MPM_EINVAL, "variant: chunk of %u bytes does not fit in LDS", W * L);
    const uint64_t table_lds = (ix->algo == MPM_ALGO_AC ? 256 : 0) + ix->table_bytes;
    const bool fits = tl + table_lds + STATIC_LDS_RESERVE <= (uint64_t)lim.max_lds;
    uint32_t place = d.placement;
    if (place == MPM_PLACE_AUTO)
        place = fits ? MPM_PLACE_LDS : MPM_PLACE_GLOBAL;
    if (place == MPM_PLACE_LDS && !fits)
        return fail(MPM_EUNSUPPORTED, "variant: tables of %llu bytes do not fit in LDS",
                    (unsigned long long)ix->table_bytes);
    cfg->lane_bytes = L;
    cfg->block_threads = W;
    cfg->placement = place;
    cfg->lds_bytes = (ix->algo == MPM_ALGO_AC ? 256u : tl) +
                     (place == MPM_PLACE_LDS ? (uint32_t)ix->table_bytes : 0u);
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
        if (ix->state_bytes == 2)
            e = lds ? launch_w<AcWalk<uint16_t, true>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s)
                    : launch_w<AcWalk<uint16_t, false>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
        else
            e = lds ? launch_w<AcWalk<uint32_t, true>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s)
                    : launch_w<AcWalk<uint32_t, false>>(a, c, sd, a.uoff, a.uids, a.dupfree, 0, s);
    } else {
        WmDev a = wm_dev(ix);
        uint32_t tl = text_lds(ix, c.block_threads, c.lane_bytes);
        e = lds ? launch_w<WmWalk<true>>(a, c, sd, a.uoff, a.uids, a.dupfree, tl, s)
                : launch_w<WmWalk<false>>(a, c, sd, a.uoff, a.uids, a.dupfree, tl, s);
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
