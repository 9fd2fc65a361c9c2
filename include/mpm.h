/*
 * mpm.h - exact multiple pattern matching on AMD Instinct MI355X (gfx950).
 *
 * The problem (Kouzinopoulos, Assael, Pyrgiotis, Margaritis, "A Hybrid
 * Parallel Implementation of the Aho-Corasick and Wu-Manber Algorithms Using
 * NVIDIA CUDA and MPI", Section 1, Definition): given a text T of n bytes and
 * d patterns of equal length m, report every pair (i, r) such that the m bytes
 * of T starting at i equal pattern r. Two index kinds solve it:
 *
 *   - Aho-Corasick (Section 3.1, Algorithms 1-3): the goto/supply automaton,
 *     flattened into a dense transition table (Section 3.1, the array
 *     representation that precomputes every supply transition).
 *   - Wu-Manber (Section 3.2, Algorithms 4-5): SHIFT/HASH/PREFIX tables over
 *     B-character blocks with direct verification.
 *
 * Results are bit-identical whichever index or launch variant is used: the
 * list of (position, pattern id) pairs in ascending (position, id) order,
 * every id of a duplicated pattern included.
 *
 * Conventions
 *   - Host pointers are plain CPU memory; "device" pointers are HIP device
 *     memory of the current device. Streams are hipStream_t passed as void*
 *     (NULL = the default stream).
 *   - Every call returns an mpm_status; nothing is thrown across this
 *     boundary. On failure mpm_last_error() describes the cause (thread-local
 *     string, valid until the next call on the same thread).
 *   - Device memory is supplied by the caller (the index image, the
 *     workspace, the outputs); the library allocates device memory only for
 *     batch plans' small descriptor tables when asked to (see mpm_batch_*).
 *   - Positions are uint32: texts must be shorter than 2^32 bytes.
 */
#ifndef MPM_H
#define MPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mpm_status;
#define MPM_OK 0
#define MPM_EINVAL (-1)        /* bad argument (null pointer, d == 0, m == 0, bad variant) */
#define MPM_EOVERFLOW (-2)     /* more matches than the output capacity */
#define MPM_ENOMEM (-3)        /* host allocation failed or a caller buffer is too small */
#define MPM_EHIP (-4)          /* a HIP runtime call failed */
#define MPM_ETOOBIG (-5)       /* text of 2^32 bytes or more, or tables beyond the encodable size */
#define MPM_EUNSUPPORTED (-6)  /* valid request this index cannot serve (e.g. Wu-Manber with m < B) */
#define MPM_ESTATE (-7)        /* index not uploaded, or the device reported a failed look-back */

typedef struct mpm_index mpm_index;

/* One occurrence: pattern `id` (0-based, its row in the pattern array) starts
 * at byte `pos` of the text (Section 1: the i of the Definition; Algorithm 3
 * reports it as i - m + 1 from the end of the window). */
typedef struct {
    uint32_t pos;
    uint32_t id;
} mpm_match;

#define MPM_ALGO_AC 1
#define MPM_ALGO_WM 2

/* Build options. Zero-initialise and set what you need; NULL means defaults. */
typedef struct {
    /* Wu-Manber block length B in characters (Section 3.2). 0 lets the
     * builder choose the B that minimises the expected work per text byte for
     * uniformly random text over the patterns' alphabet. Must satisfy
     * 1 <= B <= min(m, 8). Ignored by mpm_build_ac. */
    uint32_t wm_block;
    /* Aho-Corasick: nonzero also keeps the goto function and the supply
     * links (Algorithms 1-2) in the device image, for scans with
     * MPM_VARIANT_SUPPLY. Ignored by mpm_build_wm. */
    uint32_t ac_goto;
    uint32_t reserved[6];
} mpm_opts;

#define MPM_PLACE_AUTO 0    /* LDS when the tables fit beside the scan's own LDS use, else
                               MPM_PLACE_HOT when the index has a hot part, else global */
#define MPM_PLACE_LDS 1     /* matching tables copied into LDS once per workgroup */
#define MPM_PLACE_GLOBAL 2  /* matching tables read through the L2/L1 caches */
#define MPM_PLACE_HOT 3     /* the part of the tables read on nearly every step in LDS, the
                               rest through the caches: Aho-Corasick keeps its first rows
                               in breadth-first order (the shallow states a walk over text
                               visits), Wu-Manber keeps SHIFT and leaves the buckets
                               global. EUNSUPPORTED with MPM_VARIANT_ILP2 */

/* Launch variant of a scan. Zero fields take defaults. The text is split
 * into chunks of lane_bytes * block_threads starting positions; each lane owns
 * lane_bytes consecutive starting positions and reads m - 1 bytes past them
 * (Section 4.2.1: sub-chunks with an m - 1 character overlap). */
typedef struct {
    uint32_t lane_bytes;     /* multiple of 16, 16..4096 (default 64 for AC, 64 for WM) */
    uint32_t block_threads;  /* 256, 512 or 1024 (default 256) */
    uint32_t placement;      /* MPM_PLACE_* */
    uint32_t grid;           /* workgroups launched; 0 = enough to fill the device */
    uint32_t flags;          /* MPM_VARIANT_* bits */
} mpm_variant;

/* Aho-Corasick normally maps text bytes to table columns in registers when
 * the pattern bytes have distinct 3-bit codes; this flag forces the byte ->
 * column lookup table in LDS instead. */
#define MPM_VARIANT_NO_SWAR 1u
/* Aho-Corasick: each thread walks two lane ranges of its chunk in lockstep
 * (two independent table-lookup chains); a chunk then holds
 * 2 * lane_bytes * block_threads starting positions. */
#define MPM_VARIANT_ILP2 2u
/* Aho-Corasick: walk the goto function and follow supply links after a
 * failed transition (the search of Algorithm 3 as the paper's kernels run
 * it, Section 4.2) instead of the flattened table: the same result, kept to
 * measure what the flattening buys. Needs an index built with ac_goto set;
 * one chain per lane; placement LDS (when goto rows and supply links fit) or
 * GLOBAL; single-text scans only (a batch plan refuses it). */
#define MPM_VARIANT_SUPPLY 4u
/* Dense output, for texts with many occurrences per position (short
 * patterns against large sets): each lane owns 16 starting positions
 * (lane_bytes is ignored) and marks, per position, the pattern string that
 * starts there in an LDS array kept in position order; whole waves then write
 * the pairs of 64 consecutive positions at a time to consecutive output
 * slots, instead of every lane appending to its own output range (which,
 * with many occurrences, leaves cache lines half written when they are
 * evicted). Needs block_threads 1024; the marks take 64 KiB of LDS beside the
 * tables (an Aho-Corasick hot part shrinks by as much; tables that then no
 * longer fit are read through the caches). Single-text scans; a batch plan
 * ignores the flag. EUNSUPPORTED with MPM_VARIANT_ILP2 or
 * MPM_VARIANT_SUPPLY. */
#define MPM_VARIANT_DENSE 8u
/* Text access of the paper's kernel ladder (Section 4.2.2), kept to measure
 * what line streaming buys; Aho-Corasick with 16-bit table entries, fixed
 * pattern length, placement LDS or GLOBAL, the byte -> column table in LDS,
 * single-text scans only (a batch plan ignores them). TEXT_BYTES: every
 * lane reads its bytes one at a time from global memory (the unoptimised
 * kernel's reads). TEXT_LDS: the workgroup first copies its chunk's text
 * (and the m - 1 bytes after it) into LDS with coalesced 16-byte loads, then
 * every lane walks its bytes from LDS (the staged-text kernel); needs
 * lane_bytes * block_threads + m + 47 bytes of LDS beside the tables.
 * EUNSUPPORTED together, or with ILP2, SUPPLY, DENSE or the hot placement. */
#define MPM_VARIANT_TEXT_BYTES 16u
#define MPM_VARIANT_TEXT_LDS 32u

/* Facts about a built index. */
typedef struct {
    uint32_t algo;           /* MPM_ALGO_AC or MPM_ALGO_WM */
    uint32_t m;              /* pattern length (the shortest, for several) */
    uint32_t d;              /* number of patterns */
    uint32_t d_unique;       /* distinct pattern strings */
    uint32_t max_dup;        /* most ids sharing one string */
    uint32_t n_classes;      /* AC: distinct pattern bytes (symbol classes) */
    uint64_t n_states;       /* AC: automaton states (trie nodes) */
    uint32_t state_bytes;    /* AC: 2 (uint16 entries) or 4 (uint32) */
    uint32_t wm_block;       /* WM: chosen B */
    uint32_t wm_code_shift;  /* WM: block characters hash as (byte >> shift) & 3 */
    uint32_t wm_zero_shift;  /* WM: SHIFT entries equal to zero */
    double wm_mean_shift;    /* WM: mean SHIFT over all block hashes */
    uint64_t table_bytes;    /* bytes of the matching tables read by the scan loop */
    uint64_t device_bytes;   /* size of the device image (mpm_device_bytes) */
    uint32_t m_max;          /* longest pattern (m when all lengths are equal) */
} mpm_info;

/* ---------------------------------------------------------------------- */
/* Building                                                                */
/* ---------------------------------------------------------------------- */

/* Aho-Corasick index (Section 3.1, Algorithm 1 for the goto function,
 * Algorithm 2 for the supply function, flattened so that every transition
 * the supply function would simulate is precomputed).
 *   patterns: host, d rows of m bytes, row-major; any byte values. Copied.
 *   out:      receives the index; release with mpm_free.
 * Errors: EINVAL (null pointer, d == 0, m == 0), ETOOBIG (more than 2^31
 * automaton states), ENOMEM. Host-only: touches no GPU. */
mpm_status mpm_build_ac(const uint8_t *patterns, uint32_t d, uint32_t m,
                        const mpm_opts *opts, mpm_index **out);

/* Wu-Manber index (Section 3.2, Algorithm 4: SHIFT initialised to m - B + 1
 * and lowered to the distance of each block's rightmost occurrence from the
 * pattern end; HASH lists the patterns per suffix-block hash in ascending
 * order; PREFIX holds each pattern's leading bytes). Blocks hash 2 bits per
 * character. Arguments and errors as mpm_build_ac, plus EUNSUPPORTED when
 * opts->wm_block is outside 1..min(m, 8). Host-only. */
mpm_status mpm_build_wm(const uint8_t *patterns, uint32_t d, uint32_t m,
                        const mpm_opts *opts, mpm_index **out);

/* Indexes over patterns of different lengths (the Definition of Section 1
 * read with a length per pattern: (i, r) is reported when the |p^r| bytes at
 * i equal p^r). A scan reports, per starting position, the ids of every
 * pattern that occurs there, ascending, positions ascending, exactly as for
 * one length; starting positions run over 0 .. n - (shortest length).
 *   patterns: host bytes; pattern r is patterns[offsets[r] .. offsets[r + 1]).
 *   offsets:  host, d + 1 ascending entries (every pattern non-empty).
 * Wherever a distinct string occurs, so does every pattern that is a prefix
 * of it: each distinct string's id list (mpm_export_unique) holds the ids of
 * all of them, and a scan finds the longest string at each start.
 * Aho-Corasick builds the automaton of the reversed strings, each state's
 * output set merged with its supply state's (Section 3.1, Algorithm 2); a
 * lane walks its range from the end, m_max - 1 bytes past it. Wu-Manber
 * takes the shortest length as its window m and builds SHIFT, HASH and
 * PREFIX from every pattern's first m bytes (Section 3.2); a bucket lists
 * longer strings first and the first whole match at a window is reported.
 * When all lengths are equal these return the index of mpm_build_ac /
 * mpm_build_wm. Indexes of several lengths run in single-text scans
 * (mpm_scan, mpm_scan_sync, mpm_scan_noalloc) with one range per lane and
 * per-lane output: MPM_VARIANT_ILP2, _SUPPLY and _DENSE, batches, tuning and
 * mpm_scan_host give EUNSUPPORTED, as does opts->ac_goto.
 * Errors: EINVAL (null pointer, d == 0, an empty pattern or descending
 * offsets), ETOOBIG (more than 2^31 automaton states, 4 GiB of distinct
 * pattern bytes or 2^31 id-list entries), EUNSUPPORTED (wm_block outside
 * 1..min(shortest length, 8)), ENOMEM. Host-only. */
mpm_status mpm_build_ac_var(const uint8_t *patterns, const uint64_t *offsets, uint32_t d,
                            const mpm_opts *opts, mpm_index **out);
mpm_status mpm_build_wm_var(const uint8_t *patterns, const uint64_t *offsets, uint32_t d,
                            const mpm_opts *opts, mpm_index **out);

/* Release an index (host memory only; the caller owns the device image).
 * NULL is accepted. */
void mpm_free(mpm_index *idx);

/* Size in bytes of the index's device image. */
uint64_t mpm_device_bytes(const mpm_index *idx);

/* Copy the index's tables into caller-owned device memory d_buf (at least
 * mpm_device_bytes bytes, 256-byte aligned) on `stream`, then wait for the
 * copy. The index keeps d_buf (not a copy): the caller keeps it alive and
 * unchanged while the index is used for scans.
 * Errors: EINVAL, ENOMEM (bytes too small), EHIP. */
mpm_status mpm_upload(mpm_index *idx, void *d_buf, uint64_t bytes, void *stream);

/* Describe an index. Errors: EINVAL. */
mpm_status mpm_index_info(const mpm_index *idx, mpm_info *out);

/* ---------------------------------------------------------------------- */
/* Scanning one text                                                       */
/* ---------------------------------------------------------------------- */

/* Workspace needed by mpm_scan for a text of n bytes under variant v (NULL =
 * default). Errors: EINVAL. */
mpm_status mpm_workspace_bytes(const mpm_index *idx, uint64_t n, const mpm_variant *v,
                               uint64_t *bytes);

/* Find every occurrence of every pattern in d_text (Section 1, Definition).
 * Enqueued on `stream`; returns without waiting.
 *   d_text:   device, n bytes, any alignment. n < m is legal (no matches).
 *   d_out:    device, room for `capacity` pairs; may be NULL iff capacity == 0.
 *             Receives the first min(total, capacity) pairs of the sorted list.
 *   d_work:   device workspace of at least mpm_workspace_bytes bytes, 8-byte
 *             aligned, zero-filled before its first use; the scan leaves it
 *             ready for the next scan. Scans that overlap in time must not
 *             share a workspace.
 *   d_total:  device uint64; receives the full number of pairs (may exceed
 *             capacity; the caller compares).
 *   v:        launch variant; NULL = defaults.
 * Errors: EINVAL, ETOOBIG (n >= 2^32), ESTATE (index not uploaded), ENOMEM
 * (workspace too small), EHIP (launch failed). Device-side errors (a
 * look-back that never completes) set a flag read by mpm_scan_sync. */
mpm_status mpm_scan(const mpm_index *idx, const uint8_t *d_text, uint64_t n,
                    mpm_match *d_out, uint64_t capacity, void *d_work, uint64_t work_bytes,
                    uint64_t *d_total, const mpm_variant *v, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): mpm_scan
 * without a caller workspace. The scan's workspace (counters, launch epoch and
 * one look-back status word per chunk) lives in a static device array of
 * MPM_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs on
 * until the process ends; the first call on a device zero-fills it on
 * `stream`, and every launch leaves its counters at zero for the next one.
 * The call allocates nothing (no hipMalloc, no allocating library routine).
 * The caller still passes the text, the output and the device total, with the
 * meaning of mpm_scan; enqueued on `stream`, no wait.
 * All calls on one device share its scratch: calls that overlap in time on one
 * device (two streams, two threads) race and give wrong results; serialise
 * them (one stream, or events).
 * Errors: those of mpm_scan, and ENOMEM when the scan needs more than
 * MPM_NOALLOC_SCRATCH_BYTES of workspace (mpm_workspace_bytes > the limit:
 * more than (MPM_NOALLOC_SCRATCH_BYTES - 64) / 8 chunks of lane_bytes x
 * block_threads starting positions), checked before anything is enqueued. A
 * device-side look-back failure (never expected) is not reported here: use
 * mpm_scan_sync for that check. */
#define MPM_NOALLOC_SCRATCH_BYTES (1u << 20)
mpm_status mpm_scan_noalloc(const mpm_index *idx, const uint8_t *d_text, uint64_t n,
                            mpm_match *d_out, uint64_t capacity, uint64_t *d_total,
                            const mpm_variant *v, void *stream);

/* mpm_scan followed by a wait on `stream` and a read of the total into
 * *total (host). Returns EOVERFLOW when *total > capacity (the first
 * `capacity` pairs are valid), ESTATE when the device flagged a failure.
 * d_total is device scratch for one uint64 as in mpm_scan. */
mpm_status mpm_scan_sync(const mpm_index *idx, const uint8_t *d_text, uint64_t n,
                         mpm_match *d_out, uint64_t capacity, void *d_work, uint64_t work_bytes,
                         uint64_t *d_total, const mpm_variant *v, void *stream,
                         uint64_t *total);

/* Scan a text that stays in host memory (Section 5: the texts exceeded device
 * memory and the kernels read them from host memory). The text is cut into
 * chunks of `chunk` starting positions; each chunk and the m - 1 bytes after
 * it are copied into one half of d_stage on a copy stream the call creates
 * (default priority) while the previous chunk is scanned on `stream`. Waits
 * for completion; the result is that of mpm_scan_sync on the whole text.
 *   h_text:      host, n bytes. Pinned memory (hipHostMalloc) lets the copies
 *                overlap the scans; pageable memory works, serialized.
 *   d_stage:     device staging buffer of stage_bytes >= 2 * (c + m - 1)
 *                bytes, c = min(chunk, n - m + 1) (one half suffices when the
 *                text is a single chunk).
 *   chunk:       starting positions per chunk, >= 1.
 *   d_out, capacity, v: as mpm_scan; positions are offsets into h_text.
 *   d_work:      workspace of mpm_workspace_bytes(idx, c + m - 1, v) bytes.
 *   d_total:     device uint64 scratch.
 *   total:       host; receives the full number of pairs.
 * Errors: EINVAL, ETOOBIG, ENOMEM (staging or workspace too small), EHIP,
 * ESTATE, and EOVERFLOW as mpm_scan_sync (the first `capacity` pairs valid). */
mpm_status mpm_scan_host(const mpm_index *idx, const uint8_t *h_text, uint64_t n,
                         uint8_t *d_stage, uint64_t stage_bytes, uint64_t chunk,
                         mpm_match *d_out, uint64_t capacity, void *d_work, uint64_t work_bytes,
                         uint64_t *d_total, const mpm_variant *v, void *stream,
                         uint64_t *total);

/* Per-pattern occurrence counts of a match list: d_counts[r] = number of
 * pairs in d_pairs whose id is r (Section 4.2: the per-thread counts, each
 * terminal adding the number of patterns it stands for, summed per pattern;
 * their sum is the list's length). One pass over the list, enqueued on
 * `stream`, no wait.
 *   d_pairs:  device, M pairs as written by mpm_scan (8-byte aligned); may be
 *             NULL iff M == 0. Pairs whose id is not below d are not counted.
 *   d_counts: device uint32[d], caller-owned; overwritten (zeroed first).
 * Errors: EINVAL (d == 0, null or unaligned pointers), EHIP. */
mpm_status mpm_count_ids(const mpm_match *d_pairs, uint64_t M, uint32_t d, uint32_t *d_counts,
                         void *stream);

/* ---------------------------------------------------------------------- */
/* Scanning many texts in one replayable launch                            */
/* ---------------------------------------------------------------------- */

/* One request of a batch: one text scanned with one index under one variant.
 * Output semantics per request are those of mpm_scan. */
typedef struct {
    const mpm_index *idx;
    const uint8_t *d_text;
    uint64_t n;
    mpm_match *d_out;
    uint64_t capacity;
    uint64_t *d_total;
    mpm_variant variant;
    /* Expected time of one of this request's chunks (any unit, 0 = unknown).
     * Within a launch, requests sharing an index form a group; groups whose
     * chunks take longest are queued first, so that long chunks do not end
     * up as the launch's tail. Does not affect results. */
    float cost_hint;
    /* Device float[2] or NULL (autotuning; does not affect results). When
     * set, every run of the batch adds to d_cost[0], for each chunk of this
     * request, the wall-clock time a workgroup spent on it divided by the
     * number of workgroups of its launch (the request's share of a launch
     * that has the device to itself), and raises d_cost[1] to the longest
     * such chunk time, both in microseconds (the caller zeroes them). A plan
     * with such a request runs its launches one after another. */
    float *d_cost;
} mpm_request;

typedef struct mpm_batch mpm_batch;

/* Plan a batch: requests sharing (index, variant) are grouped into one
 * persistent launch whose workgroups take chunks of all the group's texts
 * from a shared ticket counter, each text keeping its own ordered output.
 * The plan copies the request array. Host-only.
 * Errors: EINVAL, ETOOBIG, ENOMEM. */
mpm_status mpm_batch_plan(const mpm_request *reqs, uint32_t count, mpm_batch **out);

/* Device bytes the plan needs (descriptor tables + workspace), and the upload
 * of the descriptors into caller memory d_buf (256-byte aligned; zero-filled
 * by the caller before first use). */
uint64_t mpm_batch_device_bytes(const mpm_batch *b);
mpm_status mpm_batch_upload(mpm_batch *b, void *d_buf, uint64_t bytes, void *stream);

/* Enqueue every group launch of the plan on `stream` (no wait). */
mpm_status mpm_batch_run(const mpm_batch *b, void *stream);

/* Capture the plan's launches into a HIP graph once, then replay it with
 * mpm_batch_replay (a single graph launch per batch). */
mpm_status mpm_batch_capture(mpm_batch *b, void *stream);
mpm_status mpm_batch_replay(const mpm_batch *b, void *stream);

/* Number of group launches in the plan. */
uint32_t mpm_batch_groups(const mpm_batch *b);

/* The launch a request with this index and variant joins in a plan: two
 * requests share a launch exactly when their keys are equal (walker kind,
 * block size, LDS class). Lets a caller predict a plan's launches while it
 * chooses variants; the value has no other meaning. Host-only.
 * Errors: EINVAL, EUNSUPPORTED (as mpm_batch_plan). */
mpm_status mpm_batch_launch_key(const mpm_index *idx, const mpm_variant *variant, uint32_t *key);

void mpm_batch_free(mpm_batch *b);

/* ---------------------------------------------------------------------- */
/* Autotuning                                                              */
/* ---------------------------------------------------------------------- */

/* Time one request under one variant as it runs inside a batched launch:
 * the text is queued `copies` times in a single batched launch (every copy
 * writes the same output region and total, with identical values), the
 * launch runs once to warm up and then `reps` times back to back, and *ms_out
 * receives the mean launch time in milliseconds (divide by copies for the
 * per-request cost).
 * Not a step of the paper's method: it feeds the exhaustive autotuner that
 * picks each request's variant. d_work: device, 256-byte aligned, at least
 * mpm_tune_work_bytes; its contents are overwritten. Waits for the launches.
 * Errors: EINVAL, ESTATE, ETOOBIG, ENOMEM, EHIP. */
mpm_status mpm_tune_time(const mpm_index *idx, const uint8_t *d_text, uint64_t n, uint32_t copies,
                         const mpm_variant *v, mpm_match *d_out, uint64_t capacity, uint64_t *d_total,
                         void *d_work, uint64_t work_bytes, uint32_t reps, void *stream,
                         float *ms_out);

/* Workspace bytes for mpm_tune_time (0 on invalid arguments). */
uint64_t mpm_tune_work_bytes(const mpm_index *idx, uint64_t n, uint32_t copies,
                             const mpm_variant *v);

/* ---------------------------------------------------------------------- */
/* Learned variant selector                                                */
/* ---------------------------------------------------------------------- */

/* A dense network predicts each scan variant's log-throughput from a
 * request's features (7 -> 64 -> 64 -> 64 -> 24, ReLU on the hidden layers);
 * it is trained on the autotuner's timings with these FP32 kernels. Not part
 * of the paper's method: it chooses among launch variants that all return
 * the same matches. Parameter vector (float, device): W1[7][64] b1[64]
 * W2[64][64] b2[64] W3[64][64] b3[64] W4[64][24] b4[24], row-major, layer
 * computing Z = A_prev W + b. All calls enqueue on `stream` and return. */
#define MPM_MLP_IN 7
#define MPM_MLP_HIDDEN 64
#define MPM_MLP_OUT 24
#define MPM_MLP_PARAMS 10392

/* Floats of the activation buffer a forward pass of `batch` rows keeps. */
uint64_t mpm_mlp_act_floats(uint32_t batch);

/* d_x: batch x 7 features; d_act: mpm_mlp_act_floats(batch) floats
 * (written, kept for the backward pass); d_y: batch x 24 outputs. */
mpm_status mpm_mlp_forward(const float *d_theta, const float *d_x, uint32_t batch, float *d_act,
                           float *d_y, void *stream);

/* Masked mean squared error of d_y against d_t under d_mask (all batch x
 * 24): *d_loss (device float, may be NULL) = sum M (Y-T)^2 / sum M, and
 * d_dy = 2 M (Y-T) / sum M. */
mpm_status mpm_mlp_loss_grad(const float *d_y, const float *d_t, const float *d_mask, uint32_t batch,
                             float *d_dy, float *d_loss, void *stream);

/* Gradient of the loss w.r.t. all parameters into d_grad (10,392 floats),
 * given the forward pass's d_act and d_dy. d_tmp: 2 * batch * 64 floats. */
mpm_status mpm_mlp_backward(const float *d_theta, const float *d_x, const float *d_act,
                            const float *d_dy, uint32_t batch, float *d_grad, float *d_tmp,
                            void *stream);

/* One Adam step (t >= 1) on n parameters with moments d_m, d_v. */
mpm_status mpm_mlp_adam(float *d_theta, const float *d_grad, float *d_m, float *d_v, uint32_t n,
                        uint32_t t, float lr, float b1, float b2, float eps, void *stream);

/* ---------------------------------------------------------------------- */
/* Inspection (host-only; used by tests)                                   */
/* ---------------------------------------------------------------------- */

/* Copy the dense Aho-Corasick table. Rows are states in breadth-first order
 * (root 0; the d_unique depth-m states last, state n_states - d_unique + u
 * being distinct string u of mpm_export_unique; for several lengths, the
 * automaton of the reversed strings, states that report a string last);
 * columns are 1 + n_classes:
 * column 0 (bytes in no pattern)
 * leads to the root, column c to the state after the c-th smallest pattern
 * byte. classes receives the n_classes bytes (may be NULL).
 * table: n_states * (1 + n_classes) uint32 entries (may be NULL).
 * Errors: EINVAL (not an AC index). */
mpm_status mpm_export_ac(const mpm_index *idx, uint32_t *table, uint8_t *classes);

/* Copy the Wu-Manber SHIFT table (4^B uint8 entries). Errors: EINVAL. */
mpm_status mpm_export_wm_shift(const mpm_index *idx, uint8_t *shift);

/* Copy the unique-string index: uoff (d_unique + 1 entries) and ids
 * (uoff[d_unique] entries: d for one length) so that ids[uoff[u] .. uoff[u+1])
 * are the ascending pattern ids reported where distinct pattern string u is
 * found (its copies, and for several lengths every pattern that is a prefix
 * of it). Distinct strings are numbered by how many ids they stand for (one
 * first, then two, and so on), each group in ascending string order. Either
 * pointer may be NULL. Errors: EINVAL. */
mpm_status mpm_export_unique(const mpm_index *idx, uint32_t *uoff, uint32_t *ids);

/* ---------------------------------------------------------------------- */
/* Measurement                                                             */
/* ---------------------------------------------------------------------- */

/* Read `bytes` of device memory d_buf (16-byte aligned) once with coalesced
 * 16-byte loads (enqueued on `stream`, no wait). Not part of the matching
 * method: it measures the streaming-read ceiling of the device against which
 * the scans' text throughput is compared, and gives hardware counters a
 * kernel of known traffic. d_sink: device uint32, written only in the
 * (practically impossible) event that the folded data equals a fixed
 * sentinel. Errors: EINVAL, EHIP. */
mpm_status mpm_read_probe(const uint8_t *d_buf, uint64_t bytes, uint32_t *d_sink, void *stream);

/* Read `bytes` of d_buf (128-byte aligned) in the scans' text access
 * pattern, without their table walk: 1024-thread workgroups, each lane
 * reading its own lane_bytes range (a multiple of 128) as whole 128-byte
 * lines with the next line in flight, lanes' ranges side by side, one chunk
 * of 1024 ranges per workgroup; `bytes` a multiple of 1024 * lane_bytes.
 * Measurement only, as mpm_read_probe. Errors: EINVAL, EHIP. */
mpm_status mpm_read_probe_lanes(const uint8_t *d_buf, uint64_t bytes, uint32_t lane_bytes,
                                uint32_t *d_sink, void *stream);

/* Last error message of this thread ("" if none). */
const char *mpm_last_error(void);

/* Library version string. */
const char *mpm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MPM_H */
