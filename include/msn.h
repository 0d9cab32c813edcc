/*
 * msn.h — C ABI of libmsn: a GPU merge sort whose base cases are fixed
 * sorting networks, for AMD Instinct MI355X (gfx950).
 *
 * Method: Aly, Jensen, ElAarag, "Improving Merge Sort and Quick Sort
 * Performance by Utilizing AlphaDev's Sorting Networks as Base Cases",
 * ACMSE 2025 (arXiv 2503.05934), Sec. 3, Algorithm 1: a merge sort that
 * hands every subarray whose size matches a configured network size to that
 * network instead of recursing further; Table 3 lists the network sets, and
 * the 6-to-8 set is the paper's recommended one.  The problem each call
 * solves is Algorithm 1's: rearrange an array into ascending order.  Here the
 * recursion runs bottom-up: each GPU lane first applies one network to a
 * fixed group of keys (8 keys for the 6-to-8 set, 4 for 3-to-5), and merges
 * follow.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Data pointers (keys, values, offsets, permutations, workspace) are device
 *    memory owned by the caller.  The library never allocates, frees or
 *    synchronises and never reads device data on the host; all work is
 *    enqueued on `stream` (a hipStream_t; NULL = the default stream) and the
 *    call returns without waiting.  This makes every call safe to record into
 *    a HIP graph.
 *  - Keys are 32-bit: MSN_U32 (unsigned), MSN_I32 (two's complement) or
 *    MSN_F32 (IEEE binary32).  Order is ascending.  For MSN_F32, -0.0 and
 *    +0.0 compare equal, every NaN sorts after +inf and all NaNs compare
 *    equal; outputs are bit copies of inputs, so -0.0 and NaN payloads
 *    survive.  Because distinct float bit patterns can compare equal, float
 *    keys are always sorted stably.
 *  - Pairs (and float keys) are sorted stably: equal keys keep their input
 *    order.
 *  - In-place operation is allowed when an output pointer equals the
 *    corresponding input pointer; any other overlap is an error.
 *  - Sizes: n and every segment hold at most 2^31 - 1 elements.
 *  - Pointers must be 4-byte aligned; 16-byte alignment enables wider loads.
 *  - Calls may come from several host threads and for several devices (the
 *    device of `stream`, or the current one): the library's host-side caches
 *    (kernel attributes, resident grid sizes, scratch addresses) are kept per
 *    device and guarded by locks.
 *
 * Return codes: 0 = success; < 0 = argument error found on the host before
 * anything is enqueued (see MSN_ERR_*); > 0 = the hipError_t of a failed
 * launch.  msn_status_string() names each code.
 */
#ifndef MSN_H
#define MSN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* key types */
#define MSN_U32 0
#define MSN_I32 1
#define MSN_F32 2

/* Base-case network sets (Table 3).  Each lane sorts groups of 8 or 4 keys:
   with the 8- or 4-key network when the set holds that size, else with two
   member networks and one merge (5 + 3 keys, or 3 + 1).  A subarray of at
   most one group (a short segment, a quick sort leaf) takes the network of
   its own size when the set holds it.  Every set yields the same sorted
   bits; only the work per key differs.
       code              set          group of  group sorted by          short subarrays
       MSN_LEAF_6TO8     {6,7,8}      8 keys    8-key network            up to 8 keys
       MSN_LEAF_3TO5     {3,4,5}      4 keys    4-key network            up to 4 keys
       MSN_LEAF_POW2     {4,8}        8 keys    8-key network            up to 8 keys
       MSN_LEAF_EVEN     {4,6,8}      8 keys    8-key network            up to 8 keys
       MSN_LEAF_ODD      {3,5,7}      8 keys    5- and 3-key networks    up to 8 keys
       MSN_LEAF_3        {3}          4 keys    3-key network + 1 key    up to 4 keys
       MSN_LEAF_3TO4     {3,4}        4 keys    4-key network            up to 4 keys
       MSN_LEAF_3TO8     {3..8}       8 keys    8-key network            up to 8 keys
       MSN_LEAF_VARSORT3 {2,3}        4 keys    3-key network + 1 key    up to 3 keys
       MSN_LEAF_VARSORT4 {2,3,4}      4 keys    4-key network            up to 4 keys
       MSN_LEAF_VARSORT5 {2..5}       8 keys    5- and 3-key networks    up to 5 keys
   ("short subarrays": the default seg_lane_max of msn_segmented_sort.) */
#define MSN_LEAF_6TO8 0
#define MSN_LEAF_3TO5 1
/* no network at all: merges from runs of one key, the classical merge sort
   the paper measures against (its empty network set); flat sorts only
   (msn_segmented_sort returns MSN_ERR_UNSUPPORTED), tiles as for 6-to-8 */
#define MSN_LEAF_NONE 2
#define MSN_LEAF_POW2 3
#define MSN_LEAF_EVEN 4
#define MSN_LEAF_ODD 5
#define MSN_LEAF_3 6
#define MSN_LEAF_3TO4 7
#define MSN_LEAF_3TO8 8
#define MSN_LEAF_VARSORT3 9
#define MSN_LEAF_VARSORT4 10
#define MSN_LEAF_VARSORT5 11

/* status codes */
#define MSN_OK 0
#define MSN_ERR_NULL (-1)        /* required pointer is NULL                  */
#define MSN_ERR_SIZE (-2)        /* size/offset/overlap out of range          */
#define MSN_ERR_DTYPE (-3)       /* unknown key type                          */
#define MSN_ERR_CONFIG (-4)      /* unknown leaf set, flag or tuning value    */
#define MSN_ERR_WORKSPACE (-5)   /* workspace missing or too small            */
#define MSN_ERR_UNSUPPORTED (-6) /* valid request this build cannot serve     */

/* flags for msn_segmented_sort */
#define MSN_ARGSORT 1u     /* vals_in must be NULL; vals_out receives segment-local indices */
#define MSN_DEBUG_CHECK 2u /* after sorting, check every segment's keys on the device      */

/* Bits of the segmented sort's status word (msn_segmented_status_offset).
 * The first three describe invalid offsets; they are checked on every call,
 * with or without MSN_DEBUG_CHECK. */
#define MSN_SEG_BAD_FIRST 1u  /* offsets[0] != 0                                  */
#define MSN_SEG_BAD_ORDER 2u  /* some offsets[s + 1] < offsets[s]                 */
#define MSN_SEG_BAD_LAST 4u   /* an entry above n_total, or the last != n_total   */
#define MSN_SEG_BAD_RESULT 8u /* MSN_DEBUG_CHECK found a segment out of order     */

/*
 * Optional tuning.  Pass NULL for the defaults.  A zero field means "default".
 * Every accepted setting yields the same bits; only speed differs.
 *   merge_tile      outputs per workgroup in a global merge pass:
 *                   2048, 4096 or 8192 (default 8192).
 *   seg_lane_max    segments of at most this many keys are sorted by one lane
 *                   with one network: 0 .. the group size (8 or 4; default:
 *                   the leaf set's short-subarray limit above).
 *   seg_wave_max    segments up to this length are sorted by one wavefront:
 *                   up to 128 x leaf size (default 128 x leaf size).
 *   seg_block_max   segments up to this length are sorted by one workgroup
 *                   in LDS: up to 1024 x leaf size (default 1024 x leaf).
 *   seg_grid        workgroups of the persistent segmented kernel
 *                   (default: enough to fill every compute unit).
 *   block_tile      run length after the first sweep of msn_sort_keys /
 *                   msn_sort_pairs: 1024, 2048 or 4096 x leaf size (default
 *                   2048 x leaf size).  Only integer keys-only sorts use runs
 *                   above 1024 x leaf size; other sorts accept the value and
 *                   keep 1024 x leaf size.
 *   merge_ways      fan-in of the global merge passes: 2 or 4 (default 4).
 *                   Four-way passes serve integer keys, with or without
 *                   values; float keys always merge pairs of runs.
 *   merge4_kpt      keys per thread of the four-way merge kernel: 16 (512
 *                   threads per tile) or 32 (256 threads); default 16.
 *   quick_rounds    partition rounds of msn_quick_sort_keys, 1..96; a
 *                   subarray still longer than one block-sort tile in the
 *                   last round is merge-sorted by one workgroup (default
 *                   2 ceil(log2(n / tile)) + 8, capped at 96).
 */
typedef struct {
    int32_t merge_tile;
    int32_t seg_lane_max;
    int32_t seg_wave_max;
    int32_t seg_block_max;
    int32_t seg_grid;
    int32_t block_tile;
    int32_t merge_ways;
    int32_t merge4_kpt;
    int32_t quick_rounds;
} msn_tuning;

/*
 * Bytes of workspace msn_sort_keys (pairs = 0) or msn_sort_pairs (pairs = 1)
 * needs for n keys.  Writes *bytes; returns a status code.
 * msn_sort_workspace_bytes is the same function under its earlier name.
 */
int msn_sort_keys_workspace_bytes(int64_t n, int dtype, int pairs, size_t* bytes);
int msn_sort_workspace_bytes(int64_t n, int dtype, int pairs, size_t* bytes);

/*
 * Sorts n keys ascending: keys_out = sorted(keys_in).
 *   keys_in, keys_out  device arrays of n 32-bit keys (may be equal).
 *   leaf               MSN_LEAF_* base-case network set.
 *   ws, ws_bytes       device workspace of at least
 *                      msn_sort_workspace_bytes(n, dtype, 0) bytes.
 * Paper: Sec. 3, Algorithm 1 applied to the whole array.
 */
int msn_sort_keys(const void* keys_in, void* keys_out, int64_t n, int dtype, int leaf,
                  const msn_tuning* tuning, void* ws, size_t ws_bytes, void* stream);

/* Largest n msn_sort_keys_noalloc accepts (2^22 keys). */
#define MSN_NOALLOC_MAX_KEYS 4194304

/*
 * msn_sort_keys with no workspace argument and no allocation, for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  The workspace is a fixed
 * array inside the library's code object (about 16.2 MiB, the keys-only
 * workspace of MSN_NOALLOC_MAX_KEYS keys); each device the library runs on
 * holds its own copy until the process ends.  Its device address is looked
 * up on the first call for each device (the device of `stream`, or the
 * current device for the null stream).
 *   keys_in, keys_out, dtype, leaf, tuning, stream: as msn_sort_keys.
 *   n  0 .. MSN_NOALLOC_MAX_KEYS; larger n returns MSN_ERR_SIZE before
 *      anything is enqueued.
 * The call never allocates or frees device memory and never synchronises.
 * Every call on one device shares that device's array, and nothing in it
 * needs clearing between calls (each call writes what it later reads).
 * Calls that may overlap in time on one device -- on different streams, or
 * from different threads -- race on the array and give undefined results;
 * calls in order on one stream are safe.
 */
int msn_sort_keys_noalloc(const void* keys_in, void* keys_out, int64_t n, int dtype, int leaf,
                          const msn_tuning* tuning, void* stream);

/*
 * Bytes of workspace msn_quick_sort_keys needs for n keys (integer dtypes;
 * MSN_F32 returns MSN_ERR_UNSUPPORTED).
 */
int msn_quick_sort_workspace_bytes(int64_t n, int dtype, size_t* bytes);

/*
 * Sorts n integer keys ascending by quick sort with network base cases:
 * keys_out = sorted(keys_in), the same bits as msn_sort_keys.
 *   keys_in, keys_out  device arrays of n MSN_U32 or MSN_I32 keys (may be
 *                      equal); MSN_F32 returns MSN_ERR_UNSUPPORTED, because
 *                      the partition is not stable and float keys that
 *                      compare equal must keep their order.
 *   leaf               MSN_LEAF_6TO8 / MSN_LEAF_3TO5: subarrays of at most
 *                      8 (4) keys take one network, subarrays of at most one
 *                      block-sort tile (8192 / 4096 keys) the block sort;
 *                      MSN_LEAF_NONE: the same without any network.
 *   tuning             NULL, or quick_rounds (other fields are ignored).
 *   ws, ws_bytes       at least msn_quick_sort_workspace_bytes(n, dtype).
 * The pivot of every subarray is the median of its first, middle and last
 * keys; each partition round is one launch, and the number of launches
 * depends only on n and the tuning.
 * Paper: Sec. 3, Algorithm 2 (MedianOfThree, HoarePartition, network base
 * cases).
 */
int msn_quick_sort_keys(const void* keys_in, void* keys_out, int64_t n, int dtype, int leaf,
                        const msn_tuning* tuning, void* ws, size_t ws_bytes, void* stream);

/*
 * Stable key-value sort of n pairs: the keys as msn_sort_keys, and
 * vals_out[i] = vals_in[p(i)] where p(i) is the input position of the i-th
 * output key; equal keys keep input order.  vals_in == NULL asks for an
 * argsort: vals_out[i] = p(i).
 *   vals_in, vals_out  device arrays of n uint32 (vals_out required).
 *   ws, ws_bytes       at least msn_sort_workspace_bytes(n, dtype, 1) bytes.
 * Paper: Sec. 3, Algorithm 1; stability is this library's reading (the
 * paper sorts bare keys).
 */
int msn_sort_pairs(const void* keys_in, const uint32_t* vals_in, void* keys_out,
                   uint32_t* vals_out, int64_t n, int dtype, int leaf,
                   const msn_tuning* tuning, void* ws, size_t ws_bytes, void* stream);

/*
 * Bytes of workspace msn_segmented_sort needs.
 */
int msn_segmented_sort_workspace_bytes(int64_t n_total, int64_t num_segments, int dtype,
                                       int pairs, size_t* bytes);

/*
 * Sorts each segment independently.  Segment s covers positions
 * [offsets[s], offsets[s+1]) of the key (and value) arrays.  The work is a
 * fixed sequence of launches that never reads the offsets on the host: a
 * clearing kernel, a binning kernel that also validates the offsets, a
 * tile-sort launch for segments of a few tiles, one persistent launch for
 * the rest (work queue), and up to three pairs of tile-merge launches.
 *   offsets        device uint32 array of num_segments + 1 entries, starting
 *                  at 0, non-decreasing, ending at n_total.  The binning
 *                  kernel checks these rules on every call; if one fails, the
 *                  status word (msn_segmented_status_offset) gets the
 *                  MSN_SEG_BAD_* bits, every later kernel returns at entry
 *                  and the outputs are left unwritten: no access goes outside
 *                  the arrays.  NULL means equal rows: n_total must be a
 *                  multiple of num_segments and every segment has
 *                  n_total / num_segments keys.
 *   vals_in/out    as msn_sort_pairs, per segment; both NULL sorts keys only.
 *                  With flags & MSN_ARGSORT, vals_in must be NULL and
 *                  vals_out[i] receives the index, local to its segment, of
 *                  the input element that lands at i.
 *   Empty segments are allowed.  Pairs and float keys are stable.
 * Paper: Algorithm 1 applied to every segment; segments of at most 8 keys
 * take one network, the role of the variable-size networks of Table 3.
 */
int msn_segmented_sort(const void* keys_in, const uint32_t* vals_in, void* keys_out,
                       uint32_t* vals_out, const uint32_t* offsets, int64_t num_segments,
                       int64_t n_total, int dtype, int leaf, unsigned flags,
                       const msn_tuning* tuning, void* ws, size_t ws_bytes, void* stream);

/*
 * Byte offset, inside the workspace of a msn_segmented_sort call with these
 * sizes, of its uint32 status word: 0 when the offsets were valid (and, with
 * MSN_DEBUG_CHECK, every segment came out in order), else MSN_SEG_BAD_* bits.
 * The call writes it on the device in stream order; the caller reads it after
 * the call's work has completed (the library itself never reads it back).
 * Problem statement: Algorithm 1 sorts one array given by its bounds; each
 * CSR segment is such an array, which the rules above make well-formed.
 */
int msn_segmented_status_offset(int64_t n_total, int64_t num_segments, int pairs,
                                size_t* offset);

/*
 * Backward of a row-wise sort y[r][i] = x[r][perm[r][i]]:
 * grad_in[r][perm[r][i]] = grad_out[r][i].  No arithmetic, so the result is
 * exact.
 *   grad_out, grad_in  device fp32 [rows x cols], row-major (must not overlap).
 *   perm               device int32 [rows x cols]; each row must be a
 *                      permutation of 0..cols-1 (as msn_segmented_sort's
 *                      MSN_ARGSORT output is).  Entries outside [0, cols) are
 *                      skipped, never written out of bounds.
 * Not in the paper (it has no gradients); a sort's derivative routes each
 * output gradient to the input the value came from.
 */
int msn_sort_backward(const float* grad_out, const int32_t* perm, float* grad_in,
                      int64_t rows, int64_t cols, void* stream);

/*
 * Merge-path split (diagnostics): out[i] = how many elements of a are among
 * the first diags[i] outputs of the stable merge of the sorted arrays a (la
 * keys) and b (lb keys), a first on equal keys -- the co-rank search (Green,
 * McColl, Bader 2012) by which the merge passes split their outputs, run on
 * the device.  A diagonal outside [0, la + lb] gives -1.  Device arrays;
 * out must not overlap a, b or diags (unless out == diags).
 * Paper: Algorithm 1's Merge.
 */
int msn_merge_path_split(const void* a, int64_t la, const void* b, int64_t lb,
                         const int32_t* diags, int32_t* out, int64_t count, int dtype,
                         void* stream);

/*
 * Copies n 32-bit words, dst[i] = src[i] (diagnostics): the library's own
 * streaming kernel, 16-byte loads and stores when both pointers are 16-byte
 * aligned, which measures the HBM rate a sweep can reach on this device next
 * to the sorts.  src and dst must not overlap.  Kernel kind "copy_words".
 */
int msn_copy_words(const void* src, void* dst, int64_t n, void* stream);

/*
 * Kernel timing (diagnostics, for benchmarks and profiling).  While enabled,
 * the library brackets each kernel it launches with two hipEvents recorded on
 * the launching stream (no synchronisation).  msn_timing_read waits for the
 * recorded events and reports, per kernel kind, the number of launches, the
 * elements they processed and the summed event time.  Not thread-safe; events
 * are host-allocated by msn_timing_enable and freed by msn_timing_disable.
 * Launches beyond max_launches are not timed.  Do not enable while capturing
 * a HIP graph.
 */
typedef struct {
    char kind[24];      /* "block_sort", "partition", "merge", "seg_init", ... */
    int64_t launches;
    int64_t elements;   /* keys (or rows x cols) processed, summed */
    double total_ms;
} msn_kernel_stats;

int msn_timing_enable(int max_launches);
int msn_timing_read(msn_kernel_stats* out, int capacity, int* count);
int msn_timing_disable(void);

/* Human-readable name of a status code. */
const char* msn_status_string(int status);

/* Library version, major * 10000 + minor * 100 + patch. */
int msn_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MSN_H */
