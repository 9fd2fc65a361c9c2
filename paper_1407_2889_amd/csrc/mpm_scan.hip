// Scan launch configuration (host side): variant resolution, occupancy,
// kernel selection and the launches. The kernels live in mpm_scan_impl.h and
// are instantiated in mpm_scan_ac16.hip, mpm_scan_ac32.hip and mpm_scan_wm.hip.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "mpm_scan_impl.h"

namespace mpm {

const void *ac16_lds_kernel(const LaunchCfg &c);
const void *ac16_glb_kernel(const LaunchCfg &c);
const void *ac16_hot_kernel(const LaunchCfg &c);
hipError_t ac16_hot_launch(const AcDev &a, const LaunchCfg &c, const ScanDev &sd, hipStream_t s);
const void *ac32_glb_kernel(const LaunchCfg &c);
const void *ac32_hot_kernel(const LaunchCfg &c);
hipError_t ac32_hot_launch(const AcDev &a, const LaunchCfg &c, const ScanDev &sd, hipStream_t s);
const void *ac_supply_kernel(uint32_t state_bytes, const LaunchCfg &c);
hipError_t ac_supply_launch(uint32_t state_bytes, const AcDev &a, const LaunchCfg &c,
                            const ScanDev &sd, hipStream_t s);
hipError_t ac16_lds_launch(const AcDev &a, const LaunchCfg &c, const ScanDev &sd, hipStream_t s);
hipError_t ac16_glb_launch(const AcDev &a, const LaunchCfg &c, const ScanDev &sd, hipStream_t s);
hipError_t ac32_glb_launch(const AcDev &a, const LaunchCfg &c, const ScanDev &sd, hipStream_t s);

// Streaming read of a buffer with coalesced 16-byte loads; the folded value
// is written only if it equals an impossible sentinel, so the reads cannot be
// optimised away and the kernel writes nothing in practice.
__global__ void read_probe_kernel(const v4u *__restrict__ p, uint64_t n16, uint32_t sentinel,
                                  uint32_t *sink)
{
    uint32_t acc = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
        const v4u v = ((glb_cptr<v4u>)p)[i];
        acc += v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == sentinel)
        sink[0] = acc;
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
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(mu);
    if (dev < 0 || dev >= 64)
        dev = 0;
    if (!have[dev]) {
        DeviceLimits L;
        (void)hipDeviceGetAttribute(&L.cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipDeviceGetAttribute(&L.max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (L.cus <= 0)
            L.cus = 256;
        if (L.max_lds <= 0)
            L.max_lds = 160 * 1024;  // gfx950's LDS per workgroup (host-only callers)
        cache[dev] = L;
        have[dev] = true;
    }
    return cache[dev];
}

static IdGroups id_groups(const mpm_index *ix)
{
    IdGroups g;
    memset(&g, 0, sizeof g);
    g.n = (uint32_t)std::min<size_t>(ix->grp_u0.size(), ID_GROUPS);
    for (uint32_t k = 0; k < g.n; k++) {
        g.u0[k] = ix->grp_u0[k];
        g.cnt[k] = ix->grp_cnt[k];
        g.off[k] = ix->grp_off[k];
    }
    g.u0[g.n] = g.n < ix->grp_u0.size() ? ix->grp_u0[g.n] : ix->du;
    return g;
}

AcDev ac_dev(const mpm_index *ix, uint32_t reserve)
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
    a.n_single = ix->n_single;
    a.grp = id_groups(ix);
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
    // hot placement: as many whole rows as the LDS holds beside the fixed
    // regions (16-byte multiple)
    const uint64_t budget = ((uint64_t)limits().max_lds - LDS_FIXED_BYTES - reserve) & ~15ull;
    const uint64_t hb = std::min<uint64_t>(budget, ix->table_bytes);
    a.hot_bytes = (uint32_t)hb;
    a.go = ix->keep_goto ? (const void *)(ix->d_image + ix->off_go) : nullptr;
    a.go_bytes = (uint32_t)ix->go_bytes;
    a.sup_off = (uint32_t)ix->sup_off;
    a.hot_states = (uint32_t)(hb / ((uint64_t)a.cp * ix->state_bytes));
    a.term_u = ix->var ? (const uint32_t *)(ix->d_image + ix->off_e) : nullptr;
    a.m_max = ix->var ? ix->m_max : ix->m;
    if (ix->var)
        a.first_term = (uint32_t)ix->first_term;
    return a;
}

WmDev wm_dev(const mpm_index *ix)
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
    a.n_single = ix->n_single;
    a.grp = id_groups(ix);
    a.shift_bytes = (uint32_t)(((uint64_t)ix->shift16.size() * 2 + 15) / 16 * 16);
    a.upoff = ix->var ? (const uint32_t *)(ix->d_image + ix->off_h) : nullptr;
    a.var = ix->var;
    return a;
}

// Whether an index can run with the hot part of its tables in LDS.
static bool has_hot(const mpm_index *ix)
{
    return ix->algo == MPM_ALGO_WM || ix->algo == MPM_ALGO_AC;
}

// LDS bytes of the hot part (reserve: bytes the launch keeps beside it).
static uint64_t hot_lds_bytes(const mpm_index *ix, uint32_t reserve)
{
    if (ix->algo == MPM_ALGO_AC)
        return ac_dev(ix, reserve).hot_bytes;
    return ((uint64_t)ix->shift16.size() * 2 + 15) / 16 * 16;
}

static const void *kernel_for(const mpm_index *ix, const LaunchCfg &c)
{
    if (ix->var)
        return var_kernel(ix, c);
    if (c.text_mode)
        return ladder_kernel(ix, c);
    if (ix->algo == MPM_ALGO_AC && c.supply)
        return ac_supply_kernel(ix->state_bytes, c);
    if (ix->algo == MPM_ALGO_AC) {
        if (ix->state_bytes == 4)  // tables of 2^16 states or more never fit whole in LDS
            return c.placement == MPM_PLACE_HOT ? ac32_hot_kernel(c) : ac32_glb_kernel(c);
        if (c.placement == MPM_PLACE_HOT)
            return ac16_hot_kernel(c);
        return c.placement == MPM_PLACE_LDS ? ac16_lds_kernel(c) : ac16_glb_kernel(c);
    }
    return wm_kernel(c);
}

uint64_t tile_bytes(const LaunchCfg &cfg)
{
    return (uint64_t)cfg.lane_bytes * cfg.block_threads * cfg.ilp;
}

uint32_t csr_uoff_words(const mpm_index *ix) { return (ix->du + 1 + 3) / 4 * 4; }
uint32_t csr_uids_words(const mpm_index *ix) { return ((uint32_t)ix->uids.size() + 3) / 4 * 4; }

mpm_status resolve_variant(const mpm_index *ix, const mpm_variant *v, uint64_t ntiles,
                           LaunchCfg *cfg, bool csr_in_lds)
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
    if (d.placement > MPM_PLACE_HOT)
        return fail(MPM_EINVAL, "variant: unknown placement %u", d.placement);
    if (d.flags & ~(MPM_VARIANT_NO_SWAR | MPM_VARIANT_ILP2 | MPM_VARIANT_SUPPLY | MPM_VARIANT_DENSE |
                    MPM_VARIANT_TEXT_BYTES | MPM_VARIANT_TEXT_LDS))
        return fail(MPM_EINVAL, "variant: unknown flags 0x%x", d.flags);
    const uint32_t text_flags = d.flags & (MPM_VARIANT_TEXT_BYTES | MPM_VARIANT_TEXT_LDS);
    if (text_flags) {
        if (text_flags == (MPM_VARIANT_TEXT_BYTES | MPM_VARIANT_TEXT_LDS) ||
            (d.flags & (MPM_VARIANT_ILP2 | MPM_VARIANT_SUPPLY | MPM_VARIANT_DENSE)) ||
            d.placement == MPM_PLACE_HOT)
            return fail(MPM_EUNSUPPORTED, "variant: the text-access variants are one alone, one "
                        "chain per lane, tables in LDS or global memory");
        if (ix->algo != MPM_ALGO_AC || ix->var || ix->state_bytes != 2)
            return fail(MPM_EUNSUPPORTED, "variant: the text-access variants run Aho-Corasick "
                        "with 16-bit entries and one pattern length");
    }
    const bool dense = (d.flags & MPM_VARIANT_DENSE) != 0;
    if (dense && (d.flags & (MPM_VARIANT_ILP2 | MPM_VARIANT_SUPPLY)))
        return fail(MPM_EUNSUPPORTED, "variant: dense output runs the flattened walk, one range "
                    "per lane");
    if (ix->var && (d.flags & (MPM_VARIANT_ILP2 | MPM_VARIANT_SUPPLY | MPM_VARIANT_DENSE)))
        return fail(MPM_EUNSUPPORTED, "variant: sets of different lengths run one range per lane "
                    "with the flattened walk and per-lane output");
    if (dense && d.block_threads && d.block_threads != 1024)
        return fail(MPM_EINVAL, "variant: dense output needs block_threads 1024");
    if (dense) {
        L = 16;  // DENSE_LANE starting positions per lane
        W = 1024;
    }
    const bool supply = ix->algo == MPM_ALGO_AC && (d.flags & MPM_VARIANT_SUPPLY);
    if (supply && !ix->keep_goto)
        return fail(MPM_EUNSUPPORTED, "variant: the supply-link walk needs an index built with "
                    "ac_goto set");
    if (supply && (d.flags & MPM_VARIANT_ILP2))
        return fail(MPM_EUNSUPPORTED, "variant: the supply-link walk has one chain per lane");
    const DeviceLimits lim = limits();
    // dynamic LDS: the kernels' fixed header and byte-class regions, then the
    // tables when they are placed in LDS
    const uint32_t fixed = LDS_FIXED_BYTES;
    // LDS kept beside the tables: the dense marks, or the staged text
    const uint32_t stage_bytes =
        (text_flags & MPM_VARIANT_TEXT_LDS)
            ? (uint32_t)(((uint64_t)L * W + ix->m + 47) / 16 * 16)
            : 0u;
    const uint32_t reserve = dense ? DENSE_MARK_BYTES : stage_bytes;
    const uint64_t table_lds = fixed + reserve + (supply ? ix->go_bytes : ix->table_bytes);
    const bool fits = table_lds <= (uint64_t)lim.max_lds;
    const bool ilp2 = ix->algo == MPM_ALGO_AC && (d.flags & MPM_VARIANT_ILP2);
    if (fixed + reserve > (uint64_t)lim.max_lds)
        return fail(MPM_EUNSUPPORTED, "variant: %u bytes of staged text exceed LDS", reserve);
    const bool hot_ok = has_hot(ix) && !ilp2 && !supply && !text_flags &&
                        fixed + reserve + hot_lds_bytes(ix, reserve) <= (uint64_t)lim.max_lds;
    uint32_t place = d.placement;
    if (place == MPM_PLACE_AUTO)
        place = fits ? MPM_PLACE_LDS : (hot_ok ? MPM_PLACE_HOT : MPM_PLACE_GLOBAL);
    if (place == MPM_PLACE_LDS && !fits)
        return fail(MPM_EUNSUPPORTED, "variant: tables of %llu bytes do not fit in LDS",
                    (unsigned long long)ix->table_bytes);
    if (place == MPM_PLACE_HOT && !hot_ok)
        return fail(MPM_EUNSUPPORTED, "variant: this index (or the two-chain variant) has no "
                    "hot placement");
    cfg->lane_bytes = L;
    cfg->block_threads = W;
    cfg->placement = place;
    cfg->supply = supply;
    cfg->swar = ix->algo == MPM_ALGO_AC && ix->swar_ok && !(d.flags & MPM_VARIANT_NO_SWAR) &&
                !supply && !text_flags;
    cfg->text_mode = (text_flags & MPM_VARIANT_TEXT_BYTES) ? 1u : (text_flags ? 2u : 0u);
    cfg->ilp = (ix->algo == MPM_ALGO_AC && (d.flags & MPM_VARIANT_ILP2)) ? 2 : 1;
    cfg->lds_bytes = fixed + (place == MPM_PLACE_LDS   ? (uint32_t)(supply ? ix->go_bytes
                                                                           : ix->table_bytes)
                              : place == MPM_PLACE_HOT ? (uint32_t)hot_lds_bytes(ix, reserve)
                                                       : 0u);
    cfg->dense = dense;
    cfg->mark_lds = dense ? cfg->lds_bytes : 0u;
    cfg->text_lds = stage_bytes ? cfg->lds_bytes : 0u;
    cfg->lds_bytes += reserve;
    cfg->csr_lds = 0;
    if (csr_in_lds) {
        // Every reported occurrence reads the id CSR (the ids of its string,
        // and their count when strings repeat): served from LDS when it fits
        // without costing a workgroup slot per CU.
        const uint64_t csr = 4ull * (csr_uoff_words(ix) + csr_uids_words(ix));
        const uint64_t with = cfg->lds_bytes + csr;
        if (with <= (uint64_t)lim.max_lds &&
            (uint64_t)lim.max_lds / with == (uint64_t)lim.max_lds / cfg->lds_bytes) {
            cfg->csr_lds = cfg->lds_bytes;
            cfg->lds_bytes = (uint32_t)with;
        }
    }
    cfg->grid = 0;
    if (ntiles) {
        const void *k = kernel_for(ix, *cfg);
        if (cfg->lds_bytes > 65536)
            (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cfg->lds_bytes);
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

mpm_status launch_scan(const mpm_index *ix, const LaunchCfg &c, const ScanDev &sd, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (c.lds_bytes > 65536)
        (void)hipFuncSetAttribute(kernel_for(ix, c), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)c.lds_bytes);
    if (ix->var)
        return var_launch(ix, c, sd, stream);
    if (c.text_mode)
        return ladder_launch(ix, c, sd, stream);
    if (ix->algo == MPM_ALGO_AC && c.supply) {
        e = ac_supply_launch(ix->state_bytes, ac_dev(ix), c, sd, s);
    } else if (ix->algo == MPM_ALGO_AC) {
        const AcDev a = ac_dev(ix, c.dense ? DENSE_MARK_BYTES : 0u);
        if (ix->state_bytes == 4)
            e = c.placement == MPM_PLACE_HOT ? ac32_hot_launch(a, c, sd, s) : ac32_glb_launch(a, c, sd, s);
        else if (c.placement == MPM_PLACE_HOT)
            e = ac16_hot_launch(a, c, sd, s);
        else
            e = c.placement == MPM_PLACE_LDS ? ac16_lds_launch(a, c, sd, s) : ac16_glb_launch(a, c, sd, s);
    } else {
        e = wm_launch(wm_dev(ix), c, sd, s);
    }
    if (e != hipSuccess)
        return fail(MPM_EHIP, "scan launch: %s", hipGetErrorString(e));
    return MPM_OK;
}

uint32_t batch_kind(const mpm_index *ix, const LaunchCfg &c)
{
    uint32_t k;
    if (ix->algo == MPM_ALGO_AC)
        k = ix->state_bytes == 4 ? (c.placement == MPM_PLACE_HOT ? BK_AC32_HOT : BK_AC32_GLB)
            : c.placement == MPM_PLACE_LDS     ? BK_AC16_LDS
            : c.placement == MPM_PLACE_HOT     ? BK_AC16_HOT
                                               : BK_AC16_GLB;
    else
        k = c.placement == MPM_PLACE_LDS   ? BK_WM_LDS
            : c.placement == MPM_PLACE_HOT ? BK_WM_HOT
                                           : BK_WM_GLB;
    return k | (c.swar ? (uint32_t)BK_SWAR : 0u);
}

static const void *batch_kernel_ptr(uint32_t kind, uint32_t W)
{
    const bool swar = (kind & BK_SWAR) != 0;
    switch (kind & BK_WALK_MASK) {
    case BK_AC16_LDS: return batch_kernel_ac16<PL_LDS>(swar, W);
    case BK_AC16_GLB: return batch_kernel_ac16<PL_GLB>(swar, W);
    case BK_AC16_HOT: return batch_kernel_ac16<PL_HOT>(swar, W);
    }
    return batch_kernel_other(kind, W);
}

uint32_t batch_grid(uint32_t kind, uint32_t W, uint32_t lds_bytes, uint64_t ntiles,
                    uint32_t grid_req)
{
    const DeviceLimits lim = limits();
    const void *k = batch_kernel_ptr(kind, W);
    if (lds_bytes > 65536)
        (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, (int)W, lds_bytes);
    if (e != hipSuccess || nb <= 0)
        nb = 1;
    uint64_t grid = grid_req ? grid_req : (uint64_t)nb * lim.cus;
    if (grid > ntiles)
        grid = ntiles;
    return (uint32_t)(grid < 1 ? 1 : grid);
}

mpm_status launch_batch(const BatchDev &bd, uint32_t kind, uint32_t W, uint32_t grid, uint32_t lds,
                        void *stream)
{
    if (lds > 65536)
        (void)hipFuncSetAttribute(batch_kernel_ptr(kind, W), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
    hipError_t e;
    const bool swar = (kind & BK_SWAR) != 0;
    hipStream_t s = (hipStream_t)stream;
    switch (kind & BK_WALK_MASK) {
    case BK_AC16_LDS: e = batch_launch_ac16<PL_LDS>(bd, swar, W, grid, lds, s); break;
    case BK_AC16_GLB: e = batch_launch_ac16<PL_GLB>(bd, swar, W, grid, lds, s); break;
    case BK_AC16_HOT: e = batch_launch_ac16<PL_HOT>(bd, swar, W, grid, lds, s); break;
    default: e = batch_launch_other(bd, kind, W, grid, lds, s); break;
    }
    if (e != hipSuccess)
        return fail(MPM_EHIP, "batch launch: %s", hipGetErrorString(e));
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

extern "C" mpm_status mpm_read_probe(const uint8_t *d_buf, uint64_t bytes, uint32_t *d_sink,
                                     void *stream)
{
    using namespace mpm;
    if (!d_buf || !d_sink || (((uintptr_t)d_buf) & 15u))
        return fail(MPM_EINVAL, "mpm_read_probe: null or unaligned buffer");
    const DeviceLimits lim = limits();
    const uint64_t n16 = bytes / 16;
    hipLaunchKernelGGL(read_probe_kernel, dim3(lim.cus * 8), dim3(256), 0, (hipStream_t)stream,
                       (const v4u *)d_buf, n16, 0xA5C3E1F7u, d_sink);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(MPM_EHIP, "mpm_read_probe: %s", hipGetErrorString(e));
    return MPM_OK;
}
