/*
 * mi355sort.h -- C ABI of the MI355X (gfx950) sort library.
 *
 * The library computes the result of the paper's "scatter / sort / merge"
 * method (El-Nashar, IJDPS 2(3) 2011, Section 3.2, Figure 1): a list of n keys
 * is split into p contiguous parts, every part is sorted, and the sorted parts
 * are merged into one ordered list.  Every call produces the STABLE ASCENDING
 * order: keys in the key type's natural order (signed for MS_KEY_I32, unsigned
 * otherwise), equal keys in their original order, optional 32-bit values
 * travelling with their keys.  All arithmetic is integer, so results are
 * exact and deterministic.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers are DEVICE pointers (hipMalloc / torch CUDA tensors) unless the
 *    comment says (host).  The caller owns every buffer.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls only enqueue work on that stream and return; results are ready
 *    when the stream is synchronised.  Nothing is allocated inside a call:
 *    scratch space is the caller's workspace `ws` of `ws_bytes` bytes, whose
 *    size ms_workspace_size() reports.  The workspace content on entry does
 *    not matter and is undefined afterwards; two calls in flight at once must
 *    not share a workspace.
 *  - Keys are 4 bytes (MS_KEY_I32, MS_KEY_U32) or 8 bytes (MS_KEY_U64), values
 *    are uint32_t.  Arrays are dense, element i at byte offset i * size.
 *    Device pointers must be aligned to their element size.
 *  - Segment / run offsets are a device array of uint64_t with count+1
 *    entries: off[0] = 0, non-decreasing, off[count] = n_total.  The host
 *    never reads them; an offsets array that breaks these rules gives an
 *    unspecified order inside [0, n_total) but no access outside it... as
 *    long as every off[i] <= n_total.
 *  - Errors are return codes; nothing throws across the ABI.  On a non-OK
 *    return nothing was enqueued, and ms_last_error() (per host thread) holds
 *    a message.  Device-side faults surface at the next synchronisation, as
 *    HIP reports them.
 */
#ifndef MI355SORT_H
#define MI355SORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ms_status {
    MS_OK = 0,
    MS_EINVAL = 1,  /* bad argument: NULL pointer with n > 0, short workspace, ... */
    MS_ENOMEM = 2,  /* reserved: the library itself never allocates device memory */
    MS_EDEVICE = 3, /* a HIP call or kernel launch failed */
    MS_ENOTSUP = 4  /* unknown key type, or a size beyond what the build supports */
} ms_status;

/* Key types.  Section 3.2 never states the key type; Figure 2's swap
 * temporary is an int, so signed 32-bit keys are the baseline. */
typedef enum ms_key_type { MS_KEY_I32 = 0, MS_KEY_U32 = 1, MS_KEY_U64 = 2 } ms_key_type;

typedef enum ms_op {
    MS_OP_SORT_KEYS = 0,
    MS_OP_SORT_PAIRS = 1,
    MS_OP_SORT_SEGMENTED = 2,
    MS_OP_MERGE_RUNS = 3,
    MS_OP_MERGE_SPLIT = 4,
    MS_OP_SORT_STEP = 5
} ms_op;

/*
 * Workspace bytes a call of `op` needs (written to *bytes, a host pointer).
 * n_total is the number of keys; num_segments the number of segments or runs
 * (ignored for the whole-list sorts); has_values selects the key/value form.
 * The figure depends only on the arguments, never on the data, so a serving
 * layer can admit work by exact bytes (and, for MS_OP_SORT_SEGMENTED, on
 * whether MS_TUNE_SEG_PASSES is 2 at the time of the query: see
 * ms_tune_set).  Returns MS_EINVAL for a NULL `bytes`,
 * MS_ENOTSUP for an unknown key type or op.
 */
ms_status ms_workspace_size(ms_op op, ms_key_type kt, int has_values, uint64_t n_total,
                            uint64_t num_segments, size_t *bytes);

/*
 * Sort n keys (the whole list: Figure 1 with p = 1).  keys_out may equal
 * keys_in (in-place); otherwise the two must not overlap.  n = 0 is a no-op.
 * Errors: MS_EINVAL (NULL pointer with n > 0, workspace smaller than
 * ms_workspace_size(MS_OP_SORT_KEYS, ...)), MS_ENOTSUP (unknown key type).
 */
ms_status sort_keys(const void *keys_in, void *keys_out, uint64_t n, ms_key_type kt, void *ws,
                    size_t ws_bytes, void *stream);

/*
 * Sort n (key, value) pairs by key, stably (Figure 1 with p = 1, the items
 * carrying a payload): the list of Section 3.2 is put in ascending key order,
 * a value moves with its key and equal keys keep their input order (the
 * order a left-first merge in Figure 3's merge sort keeps).  In-place is
 * allowed when keys_out == keys_in AND vals_out == vals_in.  Errors as for
 * sort_keys, plus MS_EINVAL when only one of keys and values is in place.
 */
ms_status sort_pairs(const void *keys_in, const uint32_t *vals_in, void *keys_out, uint32_t *vals_out,
                     uint64_t n, ms_key_type kt, void *ws, size_t ws_bytes, void *stream);

/*
 * The scatter phase of Figure 1 (the master computes s = n/p and hands out
 * contiguous sub-lists): writes the p + 1 boundaries of p contiguous parts of
 * a list of n items to offsets_out, a device array of num_parts + 1 uint64_t
 * owned by the caller: part i = [floor(i*n/p), floor((i+1)*n/p)), exactly
 * (the product i*n is formed in 128 bits), so parts differ in size by at most
 * one when p does not divide n and are s = n/p each when it does.  The
 * result is the offsets argument of sort_segmented and merge_runs for the
 * paper's method.  One small launch on `stream`; no key moves.  Errors:
 * MS_EINVAL for num_parts = 0 or UINT64_MAX, or a NULL offsets_out.
 */
ms_status part_offsets(uint64_t n, uint64_t num_parts, uint64_t *offsets_out, void *stream);

/*
 * The sorting phase of Figure 1 for many lists at once: each
 * segment [seg_offsets[s], seg_offsets[s+1]) of the input is sorted on its
 * own (no item crosses a segment boundary; empty segments are allowed).
 * vals_in / vals_out may both be NULL for a key-only sort.  In-place is
 * allowed under the same rule as sort_pairs.  Several segments averaging more
 * than 8,192 keys are sorted by whole-device digit passes over all of them
 * (unless MS_TUNE_SEG_PASSES is 0; with MS_TUNE_SEG_PASSES = 2 from 1,024 keys
 * on average), other calls by three small planning launches and one launch
 * of a persistent kernel whose workgroups each take whole segments; the
 * result is the same.
 * The persistent kernel counts a segment's keys in 32 bits: on that path
 * every segment must hold fewer than 2^32 keys (a longer one is left in an
 * unspecified order, with no access outside it).  num_segments = 0 requires
 * n_total = 0.  Errors: MS_EINVAL for NULL pointers with n_total > 0, a NULL
 * offsets array with num_segments > 0, num_segments = 0 with n_total > 0, a
 * short workspace, or only one of vals_in / vals_out given.
 */
ms_status sort_segmented(const void *keys_in, const uint32_t *vals_in, void *keys_out,
                         uint32_t *vals_out, const uint64_t *seg_offsets, uint64_t num_segments,
                         uint64_t n_total, ms_key_type kt, void *ws, size_t ws_bytes, void *stream);

/*
 * The merge phase (Figure 1 merge loop; Section 3.2.2 master merge): num_runs
 * adjacent runs [run_offsets[r], run_offsets[r+1]), each already sorted
 * ascending, are combined into one sorted list.  On equal keys the item from
 * the earlier run comes first, so the result is the stable sort of the
 * concatenation whichever merge schedule is used.  keys_out must not overlap
 * keys_in (nor vals_out vals_in).  Runs that are not sorted give an
 * unspecified order (never an out-of-bounds access).  Errors as for
 * sort_segmented; num_runs = 0 is MS_EINVAL.
 */
ms_status merge_runs(const void *keys_in, const uint32_t *vals_in, void *keys_out, uint32_t *vals_out,
                     const uint64_t *run_offsets, uint64_t num_runs, uint64_t n_total,
                     ms_key_type kt, void *ws, size_t ws_bytes, void *stream);

/*
 * The merge phase by Figure 1's own schedule, odd/even transposition
 * merge-split: the input holds num_parts sorted parts of n_total / num_parts
 * keys each (part i = [i*s, (i+1)*s)); in phase k = 0 .. num_parts-1 the
 * parts (0,1), (2,3), ... (k even) or (1,2), (3,4), ... (k odd) are merged
 * pairwise (the lower part's item first on equal keys) and split by count,
 * the lower part keeping the first s items; an unpaired part is copied.
 * After num_parts phases the list is sorted, with the same result as
 * merge_runs over the same parts (the stable sort of the concatenation), at
 * num_parts passes over the data instead of ceil(log2(num_parts)).
 * keys_out must not overlap keys_in (nor vals_out vals_in).  Errors:
 * MS_EINVAL for NULL pointers with n_total > 0, num_parts = 0, num_parts
 * not dividing n_total (count-preserving exchanges cannot carry items across
 * unequal parts), aliasing, only one of vals_in / vals_out, or a workspace
 * below ms_workspace_size(MS_OP_MERGE_SPLIT, kt, has_values, n_total,
 * num_parts); MS_ENOTSUP for an unknown key type.
 */
ms_status merge_split(const void *keys_in, const uint32_t *vals_in, void *keys_out, uint32_t *vals_out,
                      uint64_t n_total, uint64_t num_parts, ms_key_type kt, void *ws, size_t ws_bytes,
                      void *stream);

/*
 * Continuous batching of sort requests (the serving form of the method: each
 * request is a whole list of Section 3.2 sorted on its own).  A request of
 * n keys is sorted over the phases ms_step_plan reports: 1 phase when n fits
 * one LDS tile (8,192 keys of 4 bytes, 4,096 of 8 bytes: sorted whole), else
 * 1 + P phases (P = key bytes): phase 0 reads the keys once for the P 8-bit
 * digit histograms, phase 1 + p is digit pass p (stable counting scatter by
 * decoupled look-back over the request's tiles).  One sort_step call is one
 * step: every request it names runs ITS OWN current phase, so requests at
 * different phases share the launch; a serving loop admits new requests at
 * phase 0 at any step boundary and drops a request after its last phase.
 * After a request's last phase (stream order) keys_out / vals_out hold its
 * stable ascending sort (equal keys in input order).
 */
#define MS_STEP_MAX_REQUESTS 1024

typedef struct ms_step_request {
    const void *keys_in;       /* the request's n keys (device) */
    const uint32_t *vals_in;   /* its n values, or NULL for a key-only request */
    void *keys_out;            /* its result (device); must not overlap keys_in or work */
    uint32_t *vals_out;        /* NULL exactly when vals_in is NULL */
    void *work;                /* per-request state (device), ms_step_plan's work_bytes,
                                  owned by the caller, left alone between the request's
                                  steps; no initialisation needed; NULL if 0 bytes */
    uint64_t n;                /* keys, at most 2^30 - 1 */
    uint32_t phase;            /* the phase to run in this step, 0 .. phases - 1 */
    uint32_t reserved;         /* 0 */
} ms_step_request;

/*
 * Phases (host *phases) and per-request work bytes (host *work_bytes) of a
 * request of n keys of type kt, with or without values.  n = 0: 0 phases.
 * Errors: MS_EINVAL for NULL outputs, MS_ENOTSUP for an unknown key type or
 * n >= 2^30.
 */
ms_status ms_step_plan(ms_key_type kt, int has_values, uint64_t n, uint32_t *phases, size_t *work_bytes);

/*
 * One step: `reqs` is a DEVICE array of num_reqs descriptors (at most
 * MS_STEP_MAX_REQUESTS; each request at most once), all of key type kt and
 * all with values (has_values = 1) or all without.  ws is the step's control
 * block, ms_workspace_size(MS_OP_SORT_STEP, ...) bytes, content irrelevant on
 * entry; two steps in flight at once must not share it.  Two launches on
 * `stream` (clear the control block, then one persistent kernel over the
 * tiles of every request).  A request's phases must run in order, one per
 * step, on one stream (or otherwise ordered); a descriptor whose phase is
 * out of range is skipped.  Phases run out of order give an unspecified
 * order inside the request's buffers, never an access outside them.
 * Errors: MS_EINVAL for num_reqs > MS_STEP_MAX_REQUESTS, NULL reqs with
 * num_reqs > 0, or a short ws; MS_ENOTSUP for an unknown key type.
 */
ms_status sort_step(const ms_step_request *reqs, uint64_t num_reqs, ms_key_type kt, int has_values, void *ws,
                    size_t ws_bytes, void *stream);

/*
 * Achievable HBM bandwidth, measured with this library's own streaming
 * kernels (16-byte coalesced accesses, 2,048 workgroups): kind 0 reads
 * `bytes` of src (dst receives one 32-bit word per workgroup: at least 8 KiB),
 * 1 writes `bytes` of dst, 2 copies src to dst; 3, 4, 5 the same with
 * non-temporal (streaming) accesses.  bytes must be a multiple of 16.  Not
 * part of the sort; used to read the sort kernels' rates against the
 * practical ceiling.  Errors: MS_EINVAL for an unknown kind, a size not a
 * multiple of 16, or NULL pointers.
 */
ms_status ms_hbm_probe(int kind, const void *src, void *dst, size_t bytes, void *stream);

/*
 * sort_keys for callers that cannot allocate device memory: code under HIP
 * graph capture, serving loops that must not allocate, harnesses that forbid
 * hipMalloc.  Same result and same kernels as sort_keys, but the workspace is
 * a fixed 64 MiB array in the library's own device memory (one per GPU,
 * held until the process ends) instead of a caller's buffer; nothing is
 * allocated by the call.  Size limit: n whose sort_keys workspace fits in
 * 64 MiB, i.e. at most 14,910,784 keys for MS_KEY_I32 / MS_KEY_U32 and
 * 7,892,992 for MS_KEY_U64; beyond that MS_EINVAL with a message.  Every
 * call on one GPU shares that GPU's array: calls that overlap in time on
 * the same GPU (other streams, other host threads) race and give undefined
 * results; calls ordered on one stream are fine.  keys_out may equal
 * keys_in.  Errors otherwise as for sort_keys.
 */
ms_status sort_keys_noalloc(const void *keys_in, void *keys_out, uint64_t n, ms_key_type kt, void *stream);

/* Text describing the last non-OK status returned on this host thread
 * ("" if none).  The pointer stays valid until the thread's next call. */
const char *ms_last_error(void);

/*
 * Launch tuning (used by the autotuner).  Values apply to calls enqueued
 * after the change, process-wide; they never change results, only speed.
 *   MS_TUNE_PASS_THREADS  workgroup size of the whole-list digit pass: 256,
 *                         512 or 1024 threads of 16 keys each (tiles of
 *                         4,096 / 8,192 / 16,384 keys).  Default 1024.
 *                         1024 applies to 32-bit keys without values; other
 *                         sorts use 512 when 1024 is set.
 *   MS_TUNE_SEG_BLOCKS    persistent workgroups of sort_segmented (1 .. 65536;
 *                         0 = the default, 1024).
 *   MS_TUNE_HIST_BLOCKS   workgroups of the digit-histogram read of sort_keys /
 *                         sort_pairs (1 .. 65536; 0 = the default, one per
 *                         compute unit).
 *   MS_TUNE_SMALL_SORT    longest segment of sort_segmented ordered by a
 *                         comparison network (a bitonic network over one
 *                         wave, ties ordered by input position, so still the
 *                         stable sort) instead of radix passes: 64 (the
 *                         default) or 0 (radix passes for every segment).
 *   MS_TUNE_SEG_PASS_THREADS  workgroup size of sort_segmented's whole-device
 *                         digit passes (segments averaging more than 8,192
 *                         keys): 512 or 1024 threads of 16 keys each (tiles
 *                         of 8,192 / 16,384 keys).  Default 512.  1024
 *                         applies to 32-bit keys without values; other
 *                         sorts use 512.
 *   MS_TUNE_SEG_PASSES    1 (the default): sort_segmented runs whole-device
 *                         digit passes when the segments average more than
 *                         8,192 keys, one launch per phase; 2: the same
 *                         phases, for segments averaging more than 1,024
 *                         keys (those averaging at most 8,192 only with a
 *                         workspace sized while this value was 2, else they
 *                         take the persistent kernel: their per-segment
 *                         counters need up to 8 bytes per key), as one
 *                         persistent launch (a work queue of
 *                         (phase, tile) items in 8 queues of consecutive
 *                         segments, one per XCD, a queue's items of phase f
 *                         starting once its phase f - 1 is done), after the
 *                         planning launches (lists of 2^30 keys and more add
 *                         a second launch that returns at entry unless a
 *                         segment has 2^30 keys or more); 0: every
 *                         sort_segmented call is one launch of the
 *                         persistent kernel, whose workgroups each take
 *                         whole segments.
 * ms_tune_set returns MS_EINVAL for an unknown parameter or value;
 * ms_tune_get returns the current value (0 for an unknown parameter).
 */
typedef enum ms_tune_param {
    MS_TUNE_PASS_THREADS = 0,
    MS_TUNE_SEG_BLOCKS = 1,
    MS_TUNE_HIST_BLOCKS = 2,
    MS_TUNE_SMALL_SORT = 3,
    MS_TUNE_SEG_PASS_THREADS = 4,
    MS_TUNE_SEG_PASSES = 5,
    MS_TUNE_COUNT = 6
} ms_tune_param;

ms_status ms_tune_set(ms_tune_param param, int64_t value);
int64_t ms_tune_get(ms_tune_param param);

/*
 * Kernel timing (instrumentation for benchmarks).  While enabled, every
 * kernel the library enqueues is bracketed by HIP events on its own stream;
 * ms_timing_read() synchronises on those events and returns, per kernel name,
 * the launch count and the summed duration.  names_out receives up to
 * max_entries NUL-terminated names of at most 63 characters (host array of
 * max_entries * 64 chars), count_out and ms_out the matching figures (host
 * arrays).  Returns the number of distinct kernels seen (which may exceed
 * max_entries).  ms_timing_enable(0) stops recording; ms_timing_reset()
 * clears what was recorded.  Not for use while other threads call the
 * library.
 */
ms_status ms_timing_enable(int on);
ms_status ms_timing_reset(void);
int ms_timing_read(char *names_out, uint64_t *count_out, double *ms_out, int max_entries);

#ifdef __cplusplus
}
#endif

#endif /* MI355SORT_H */
