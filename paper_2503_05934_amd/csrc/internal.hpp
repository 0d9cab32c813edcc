// Host-side declarations shared by the C ABI (api.cpp) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "msn.h"

namespace msn {

constexpr int kWave = 64;
constexpr int kBlockThreads = 512;   // block sort: 8 wavefronts x 16 keys per lane
constexpr int kMergeThreads = 256;   // global merge pass

enum KeyType : int { kU32 = 0, kI32 = 1, kF32 = 2 };

// How a lane sorts one group of its keys (the leaf set's network family):
// no network (merges from single keys), the group-sized network, or two
// member networks and a merge (sets without a member of the group's size).
constexpr int kNetNone = 0;
constexpr int kNetPlain = 1;
constexpr int kNetSplit = 2;

// Values travelling with the keys.
enum ValMode : int {
    kNoVals = 0,  // keys only
    kVals = 1,    // caller's uint32 payload
    kArg = 2,     // payload = index (argsort); generated, never read
};

struct SortArgs {
    const uint32_t* kin;
    const uint32_t* vin;  // kVals only
    uint32_t* kout;
    uint32_t* vout;       // kVals / kArg
    int64_t n;
    int dtype;
    int leaf_k;           // keys per lane in the base case: 8 or 4
    int vmode;
    int merge_tile;       // 2048, 4096 or 8192
    int block_tile;       // first-sweep run length: 1024K, 2048K or 4096K
    int merge_ways;       // 2 or 4 (four-way passes: integer keys)
    int merge4_kpt;       // keys per thread of the four-way merge: 16 or 32
    void* ws;
    size_t ws_bytes;
    hipStream_t stream;
    int nets = 1;         // network family: 0 none (the classical merge sort, tiles of
                          // leaf_k = 8), 1 the leaf_k-key network, 2 two member
                          // networks and a merge (sets without a leaf_k-key member)
};

struct SegArgs {
    const uint32_t* kin;
    const uint32_t* vin;
    uint32_t* kout;
    uint32_t* vout;
    const uint32_t* offsets;  // NULL = equal rows
    int64_t num_segments;
    int64_t n_total;
    int dtype;
    int leaf_k;
    int vmode;                // kArg = segment-local argsort
    int lane_max, wave_max, block_max, grid;
    void* ws;
    size_t ws_bytes;
    hipStream_t stream;
    int debug_check = 0;      // MSN_DEBUG_CHECK: verify every segment after sorting
    int net = 1;              // network family of the leaves (kNetPlain / kNetSplit)
    uint32_t set_mask = ~0u;  // network sizes of the leaf set (bit k = size k)
};

constexpr size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

constexpr int kMinMergeTile = 2048;
// Chunk size of the key samples every sweep of a flat sort leaves behind
// (first and last key of each chunk); merge-path splits search them first.
constexpr int kSampleChunk = 256;

struct Samples {
    uint32_t* first;  // first key of chunk c (position c * kSampleChunk)
    uint32_t* last;   // last key of chunk c (position c * kSampleChunk + kSampleChunk - 1)
    int64_t base;     // global position of the tile being written
};
constexpr int kDefaultMergeTile = 8192;
constexpr int kDefaultBlockTileMult = 2048;  // first-sweep run = 2048 x leaf size

// Four-way passes: samples merged per group of four runs cut output tiles at
// every kM4SamplesPerTile-th sample.
constexpr int kM4SamplesPerTile = 27;

// Upper bound on the tile boundaries of any four-way pass (runs of at least
// 4096 keys): chunks / kM4SamplesPerTile + 2 per group + slack.
constexpr size_t m4_max_bounds(int64_t n) {
    const size_t chunks = (size_t)((n + kSampleChunk - 1) / kSampleChunk);
    return chunks / kM4SamplesPerTile + (size_t)(n / 8192) + 8;
}

// Workspace of the four-way passes: the boundary table (four splits per
// tile boundary).
constexpr size_t m4_ws_bytes(int64_t n) { return align_up(m4_max_bounds(n) * 16, 256); }

// Workspace of the flat sort: ping-pong keys (+ values), one merge-path split
// per merge tile, the two chunk-sample arrays, the four-way passes' boundary
// table, and the presorted-input flag.
constexpr size_t sort_ws_bytes(int64_t n, bool vals) {
    const size_t nk = align_up((size_t)n * 4, 256);
    const size_t nv = vals ? nk : 0;
    const size_t tiles = (size_t)((n + kMinMergeTile - 1) / kMinMergeTile) + 1;
    const size_t chunks = (size_t)((n + kSampleChunk - 1) / kSampleChunk);
    return nk + nv + align_up(tiles * 4, 256) + 2 * align_up(chunks * 4, 256) + m4_ws_bytes(n) +
           256;
}

size_t seg_ws_bytes(int64_t n_total, int64_t num_segments, bool vals);
// Byte offset of the segmented sort's status word inside its workspace.
size_t seg_status_offset(int64_t n_total, int64_t num_segments, bool vals);

// Raises a kernel's dynamic-LDS limit to `bytes` (needed beyond 64 KiB); done
// once per kernel and device (thread-safe).  Returns a hipError_t value.
int set_dynamic_lds(const void* kernel, size_t bytes);
// Workgroups of `threads` threads with `lds` bytes of dynamic LDS that fill
// every compute unit of the current device with `kernel` (its occupancy
// times the compute units); cached per kernel, device and shape
// (thread-safe).  Returns a hipError_t value.
int resident_grid(const void* kernel, int threads, size_t lds, int* out);

// Brackets one kernel launch with hipEvents when timing is enabled
// (msn_timing_enable); a no-op otherwise.
class LaunchTimer {
   public:
    LaunchTimer(const char* kind, int64_t elements, hipStream_t stream);
    ~LaunchTimer();
    LaunchTimer(const LaunchTimer&) = delete;
    LaunchTimer& operator=(const LaunchTimer&) = delete;

   private:
    int slot_;
    hipStream_t stream_;
};

int launch_sort(const SortArgs& a);
int launch_copy(const uint32_t* src, uint32_t* dst, int64_t n, hipStream_t stream);

// Keys accepted by msn_sort_keys_noalloc, and the bytes of its device-resident
// scratch (the flat keys-only workspace at that size).
constexpr int64_t kNoAllocMaxKeys = MSN_NOALLOC_MAX_KEYS;
constexpr size_t kNoAllocScratchBytes = sort_ws_bytes(kNoAllocMaxKeys, false);
// Address of this library's scratch array on the device that `stream`
// belongs to (the current device for the null stream), looked up once per
// device; *bytes receives its size.  Returns a hipError_t value.
int noalloc_scratch(hipStream_t stream, void** ptr, size_t* bytes);
int launch_segmented(const SegArgs& a);
int launch_merge_path_split(const uint32_t* a, int64_t la, const uint32_t* b, int64_t lb,
                            const int32_t* diags, int32_t* out, int64_t count, int dtype,
                            hipStream_t stream);

struct QuickArgs {
    const uint32_t* kin;
    uint32_t* kout;
    int64_t n;
    int dtype;       // kU32 or kI32
    int leaf_k;      // keys of the leaf network: 8 or 4
    int nets;        // network family as in SortArgs (0: the classical quick sort)
    uint32_t set_mask;  // network sizes of the leaf set (bit k = size k)
    int rounds;      // partition rounds (0 = quick_rounds(n, leaf tile))
    void* ws;
    size_t ws_bytes;
    hipStream_t stream;
};
// Rounds (launches of the round kernel) of a quick sort of n keys whose
// leaves hold up to leaf_max keys, by default.
constexpr int kQuickMaxRounds = 96;
int quick_rounds(int64_t n, int64_t leaf_max);
// Workspace of the quick sort: the partition buffer and three item lists.
size_t quick_ws_bytes(int64_t n);
int launch_quick(const QuickArgs& a);
int launch_backward(const float* grad_out, const int32_t* perm, float* grad_in, int64_t rows,
                    int64_t cols, hipStream_t stream);

}  // namespace msn
