// Batched (segmented) sort: many independent arrays of uneven length in a
// fixed sequence of launches that never reads the offsets on the host (so a
// graph can capture it).  Algorithm 1 of the paper (Sec. 3) is applied to
// every segment; the work unit is chosen by segment length:
//   lane   (<= lane_max keys, at most one leaf): one lane, one network with
//          padding -- the role of the paper's variable-size networks
//          (Table 3, VarSort);
//   wave   (<= wave_max): one wavefront, networks + bitonic merges;
//   block  (<= block_max): one workgroup, network + bitonic + LDS merges;
//   tiled  (up to kSegTiledMax block-sort tiles): every run is a work item
//          of its own (k_seg_tile_sort: keys-only runs are two tiles long,
//          sorted by the flat sort's 1024-thread block sort; stable runs are
//          one tile), then merge passes over all such segments at once, one
//          workgroup per output tile: keys-only segments of two runs take one
//          binary pass (k_seg_tile_part, then k_seg_tile_merge) and those of
//          three or four runs one four-way pass (k_seg_m4_bounds, then
//          k_seg_merge4); stable segments take up to three binary passes;
//          tiles already in order are copied rather than sorted or merged;
//   big    (longer): one workgroup sorts the segment's tiles in turn and then
//          merges them pass by pass through global memory.
// k_seg_bin sorts segment ids into per-class lists, the tiles of tiled
// segments into a tile list (and those of segments that take binary passes
// into a merge list), and the four-way segments into a list of their own;
// the persistent k_segmented pulls the lane, wave,
// block and big work items (big segments first) from one atomic counter
// until the lists are exhausted.  No workgroup ever waits for another, so any
// grid size terminates.
#include <algorithm>

#include "merge4.hpp"
#include "seg_tasks.hpp"

namespace msn {

enum SegClass : int {
    kCLane = 0,
    kCWave = 1,
    kCBlock = 2,
    kCTiled = 3,  // its tiles go to the tile list
    kCBig = 4,    // longer than kSegTiledMax tiles
    kNumClasses = 5
};
// The class lists, then the list of four-way segments (keys-only tiled
// segments of three or four runs).
constexpr int kList4 = kNumClasses;
constexpr int kNumLists = kNumClasses + 1;

// Work queues of the tile sort: one per XCD (workgroups are dispatched to
// the eight XCDs in turn), each head on a 128-byte line of its own.
constexpr int kSegQueues = 8;

struct SegState {
    uint32_t count[8];
    uint32_t head;
    uint32_t tiles;   // entries of the tile list
    uint32_t status;  // MSN_SEG_BAD_* bits found in this call (0 = offsets valid)
    uint32_t tiles4;  // entries of the four-way tile list
    uint32_t mtiles;  // entries of the merge list (tiles of segments with binary passes)
    uint32_t pad[3];
    uint32_t queue[kSegQueues][32];  // tile-sort queue heads (word 0 of each line)
};

// Segments of up to this many block-sort tiles take the tiled path (at most
// three merge passes from one-tile runs, two from keys-only two-tile runs).
constexpr int kSegTiledMax = 8;

// Tile list bound: a tiled segment of len keys has ceil(len / tile) tiles,
// tile >= 4096 keys (3-to-5 leaves).
inline size_t seg_max_tiles(int64_t n_total, int64_t num_segments) {
    return (size_t)(n_total / 4096) + (size_t)num_segments + 1;
}

// Four-way tiles: a four-way segment has runs of at most kSeg4MaxChunks
// chunks of kSampleChunk keys, so at most kSeg4MaxTiles tiles of
// kM4SamplesPerTile samples; each tile is one self-contained record.
constexpr int kSeg4MaxChunks = 64;
constexpr int kSeg4MaxTiles =
    (4 * kSeg4MaxChunks + kM4SamplesPerTile - 1) / kM4SamplesPerTile;
struct Seg4Tile {
    uint32_t off;    // the segment's first key
    int32_t lo[4];   // first key of run r's slice, from the run's start
    int32_t c[4];    // keys of run r's slice
    uint32_t pad[7];
};
static_assert(sizeof(Seg4Tile) == 64, "one record per 64 bytes");
// A four-way segment holds more than two runs of at least 8192 keys.
inline size_t seg_max_tiles4(int64_t n_total, int64_t num_segments) {
    const int64_t segs = std::min<int64_t>(num_segments, n_total / 16385 + 1);
    return (size_t)segs * kSeg4MaxTiles;
}

// Workspace: ping-pong keys (and values), the lists, the state block, the
// tile list (segment, tile) of every tiled segment, the merge list (the
// entries of the segments that take binary merge passes) with one
// merge-path split per entry, and the four-way tile records.
size_t seg_ws_bytes(int64_t n_total, int64_t num_segments, bool vals) {
    const size_t nk = align_up((size_t)n_total * 4, 256);
    const size_t lists = align_up((size_t)num_segments * 4 * kNumLists, 256);
    const size_t mt = seg_max_tiles(n_total, num_segments);
    return nk + (vals ? nk : 0) + lists + align_up(sizeof(SegState), 256) +
           2 * align_up(mt * 8, 256) + align_up(mt * 4, 256) +
           align_up(seg_max_tiles4(n_total, num_segments) * sizeof(Seg4Tile), 256);
}

// Merge passes of a segment of `tiles` block-sort tiles: ceil(log2(tiles)).
__host__ __device__ inline int seg_passes(uint32_t tiles) {
    int p = 0;
    while ((1u << p) < tiles) ++p;
    return p;
}

// Global passes a tiled segment of len keys takes after its runs of `run`
// keys are sorted: binary merge passes, except that a keys-only (FOUR)
// segment of three or four runs takes one four-way pass instead of two.
template <bool FOUR>
__host__ __device__ inline int seg_global_passes(uint32_t len, int run) {
    const int p = seg_passes((len + run - 1) / run);
    return (FOUR && p == 2) ? 1 : p;
}

// Runs the tile sort leaves in a tiled segment: keys-only tiles take the
// flat sort's 1024-thread shape (runs of two list tiles, one merge pass
// fewer); stable tiles keep the list tile.
template <int DT, int K, bool STABLE>
struct SegRun {
    static constexpr int kShape = STABLE ? 0 : 1;
    using Tr = TileTraits<DT, K, STABLE, kShape>;
    static constexpr int kRun = Tr::kTile;
    static constexpr int kListTile = TileTraits<DT, K, STABLE>::kTile;
    static_assert(kRun % kListTile == 0, "runs are whole list tiles");
};

__device__ __forceinline__ void seg_bounds(const uint32_t* offsets, uint32_t s, uint32_t uni_len,
                                           uint32_t& off, uint32_t& len) {
    if (offsets) {
        off = offsets[s];
        len = offsets[s + 1] - off;
    } else {
        off = s * uni_len;
        len = uni_len;
    }
}

// Zeroes the class counters and the work-queue head (a kernel, not a memset,
// so that graph replays reset it reliably).
__global__ void k_seg_init(SegState* st) {
    for (uint32_t i = threadIdx.x; i < sizeof(SegState) / 4; i += blockDim.x)
        reinterpret_cast<uint32_t*>(st)[i] = 0u;
}

// Classes (and tiles) are counted per workgroup in LDS first, so each
// workgroup makes one global atomic per class instead of one per segment (a
// few global counters shared by every segment would serialise).
// The same pass validates the offsets: offsets[0] == 0, no entry below its
// predecessor, and the last equal to n_total (equivalently every entry within
// n_total).  A segment whose own pair of offsets breaks a rule is not binned,
// and the status word records which rule broke; every later kernel of the
// call returns at entry when it is set, so a bad array never leads to an
// access outside the key, value, list or tile arrays.  Valid offsets cannot
// overflow the tile list; the bound check on it covers the invalid case
// (where the binned segments may overlap) until the status word stops the
// call.
__global__ __launch_bounds__(256) void k_seg_bin(const uint32_t* __restrict__ offsets,
                                                 int64_t num_segments, int64_t n_total,
                                                 uint32_t uni_len, int lane_max, int wave_max,
                                                 int block_max, uint32_t tile, uint32_t merge_min,
                                                 uint32_t four_min, SegState* st,
                                                 uint32_t* __restrict__ lists,
                                                 uint2* __restrict__ tiles,
                                                 uint2* __restrict__ mtiles, uint32_t max_tiles) {
    // the class counts, the tile count, the four-way segment count, the
    // merge-list count
    __shared__ uint32_t cnt[kNumClasses + 3], base[kNumClasses + 3];
    __shared__ uint32_t bad;
    const int tid = threadIdx.x;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + tid;
    if (tid <= kNumClasses + 2) cnt[tid] = 0u;
    if (tid == 0) bad = 0u;
    __syncthreads();
    int cls = -1;
    uint32_t pos = 0, nt = 0, tpos = 0, fpos = 0, mpos = 0;
    bool four = false, merged = false;
    if (s < num_segments) {
        uint32_t off, len;
        uint32_t err = 0u;
        if (offsets) {
            const uint32_t a = offsets[s], b = offsets[s + 1];
            if (s == 0 && a != 0u) err |= MSN_SEG_BAD_FIRST;
            if (b < a) err |= MSN_SEG_BAD_ORDER;
            if ((int64_t)b > n_total || (s == num_segments - 1 && (int64_t)b != n_total))
                err |= MSN_SEG_BAD_LAST;
            off = a;
            len = b - a;
        } else {
            off = (uint32_t)s * uni_len;
            len = uni_len;
        }
        if (err) {
            atomicOr(&bad, err);
        } else {
            if (len <= (uint32_t)lane_max) cls = kCLane;
            else if (len <= (uint32_t)wave_max) cls = kCWave;
            else if (len <= (uint32_t)block_max) cls = kCBlock;
            else if (len <= (uint32_t)kSegTiledMax * tile) cls = kCTiled;
            else cls = kCBig;
            if (cls == kCTiled) {
                nt = (len + tile - 1) / tile;
                tpos = atomicAdd(&cnt[kNumClasses], nt);
                four = four_min != 0u && len > four_min;
                if (four) fpos = atomicAdd(&cnt[kNumClasses + 1], 1u);
                merged = !four && len > merge_min;
                if (merged) mpos = atomicAdd(&cnt[kNumClasses + 2], nt);
            } else {
                pos = atomicAdd(&cnt[cls], 1u);
            }
        }
        (void)off;
    }
    __syncthreads();
    if (tid < kNumClasses && cnt[tid] != 0u) base[tid] = atomicAdd(&st->count[tid], cnt[tid]);
    if (tid == kNumClasses && cnt[tid] != 0u) base[tid] = atomicAdd(&st->tiles, cnt[tid]);
    if (tid == kNumClasses + 1 && cnt[tid] != 0u)
        base[tid] = atomicAdd(&st->count[kList4], cnt[tid]);
    if (tid == kNumClasses + 2 && cnt[tid] != 0u) base[tid] = atomicAdd(&st->mtiles, cnt[tid]);
    if (tid == kNumClasses + 3 && bad != 0u) atomicOr(&st->status, bad);
    __syncthreads();
    if (cls == kCTiled) {
        for (uint32_t c = 0; c < nt; ++c) {
            const uint32_t e = base[kNumClasses] + tpos + c;
            if (e < max_tiles) tiles[e] = make_uint2((uint32_t)s, c);
            const uint32_t m = base[kNumClasses + 2] + mpos + c;
            if (merged && m < max_tiles) mtiles[m] = make_uint2((uint32_t)s, c);
        }
        if (four) lists[(int64_t)kList4 * num_segments + base[kNumClasses + 1] + fpos] = (uint32_t)s;
    } else if (cls >= 0) {
        lists[(int64_t)cls * num_segments + base[cls] + pos] = (uint32_t)s;
    }
}

// MSN_DEBUG_CHECK: after the sort, one wavefront per segment checks that the
// segment's keys are in order and records MSN_SEG_BAD_RESULT otherwise (a
// fault of the library, not of the caller).
template <int DT>
__global__ __launch_bounds__(256) void k_seg_verify(const uint32_t* __restrict__ kout,
                                                    const uint32_t* __restrict__ offsets,
                                                    int64_t num_segments, uint32_t uni_len,
                                                    SegState* st) {
    if (st->status) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    int bad = 0;
    for (int64_t s = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
         s < num_segments; s += waves) {
        const uint32_t off = offsets ? offsets[s] : (uint32_t)s * uni_len;
        const uint32_t len = offsets ? offsets[s + 1] - off : uni_len;
        for (uint32_t i = 1 + (uint32_t)lane; i < len; i += kWave)
            bad |= (int)(ord_key<DT>(kout[off + i]) < ord_key<DT>(kout[off + i - 1]));
    }
    if (bad) atomicOr(&st->status, (uint32_t)MSN_SEG_BAD_RESULT);
}

// Register budgets by occupancy: keys-only kernels are held to 84 VGPRs so
// that three workgroups fit a compute unit, stable ones to 128 for two (what
// their LDS allows).  Both spill some registers (a few bytes keys-only, up to
// a few hundred bytes for the 8-key stable tiles), and both are faster for
// it: 4 % on the 100,000-segment workload, 25 % on the fp32 row argsort,
// where one workgroup per compute unit could not hide its LDS latency.
template <int DT, int K, bool STABLE, int VM, int NET>
__global__ __launch_bounds__(kBlockThreads, STABLE ? 4 : 6) void k_segmented(
    const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, uint32_t* wk,
    uint32_t* wv, const uint32_t* __restrict__ offsets, int64_t num_segments, uint32_t uni_len,
    SegState* st, const uint32_t* __restrict__ lists, uint32_t set_mask) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_item;
    const int tid = threadIdx.x;
    if (st->status) return;

    const uint32_t n_lane = st->count[kCLane];
    const uint32_t n_wave = st->count[kCWave];
    const uint32_t n_block = st->count[kCBlock];
    const uint32_t n_big = st->count[kCBig];
    constexpr uint32_t kWavesPerBlock = kBlockThreads / kWave;
    const uint32_t wave_items = (n_wave + kWavesPerBlock - 1) / kWavesPerBlock;
    const uint32_t lane_items = (n_lane + kBlockThreads - 1) / kBlockThreads;
    // queue order: big segments, block, wave items, lane items (the tiles of
    // tiled segments have a launch of their own)
    const uint32_t e0 = n_big;
    const uint32_t e2 = e0 + n_block;
    const uint32_t e3 = e2 + wave_items;
    const uint32_t e4 = e3 + lane_items;
    const uint32_t* L = lists;
    const int64_t S = num_segments;

    for (;;) {
        if (tid == 0) s_item = atomicAdd(&st->head, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= e4) break;
        if (item < e0) {
            uint32_t off, len;
            seg_bounds(offsets, L[kCBig * S + item], uni_len, off, len);
            big_task<DT, K, STABLE, VM, NET>(kin, vin, kout, vout, wk, wv, off, (int)len, smem);
        } else if (item < e2) {
            uint32_t off, len;
            seg_bounds(offsets, L[kCBlock * S + (item - e0)], uni_len, off, len);
            bool done = false;
            if constexpr (!STABLE)
                done = copy_if_in_order<DT, keys_per_lane<K>()>(kin + off, kout + off, (int)len,
                                                                smem);
            if (!__builtin_amdgcn_readfirstlane(done))
                block_sort_tile<DT, K, STABLE, VM, 0, false, false, NET>(
                    kin + off, VM == kVals ? vin + off : nullptr,
                                                   kout + off,
                                                   VM != kNoVals ? vout + off : nullptr, (int)len,
                                                   0u, smem);
        } else if (item < e3) {
            const uint32_t w = (uint32_t)tid / kWave;
            const uint32_t idx = (item - e2) * kWavesPerBlock + w;
            if (idx < n_wave) {
                uint32_t off, len;
                seg_bounds(offsets, L[kCWave * S + idx], uni_len, off, len);
                uint32_t* wst = reinterpret_cast<uint32_t*>(smem) +
                                (size_t)w * 2 * kWave * keys_per_lane<K>();
                wave_task<DT, K, STABLE, VM, NET>(kin, vin, kout, vout, off, (int)len, wst);
            }
        } else {
            const uint32_t idx = (item - e3) * kBlockThreads + (uint32_t)tid;
            if (idx < n_lane) {
                uint32_t off, len;
                seg_bounds(offsets, L[kCLane * S + idx], uni_len, off, len);
                lane_task<DT, K, STABLE, VM, NET>(kin, vin, kout, vout, off, (int)len,
                                                  set_mask);
            }
        }
    }
}

// --------------------------------------------------- equal stable rows ---
// Equal rows of at most one tile sorted stably (float keys, pairs,
// argsorts; the differentiable row sort): one 1024-thread workgroup per row
// with one leaf group of K keys per lane (tile shape 3), rows taken in turn.
// Against the persistent kernel's 512 threads x 2K keys this halves the
// registers a lane holds and doubles the wavefronts per SIMD, which keeps the
// VALU busier through the 64-bit composite exchanges.
template <int DT, int K, int VM, int NET>
__global__ __launch_bounds__((TileTraits<DT, K, true, 3>::kThreads),
                             (TileTraits<DT, K, true, 3>::kWavesPerSimd))
void k_seg_rows(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                int64_t rows, uint32_t len, const SegState* st) {
    using Tr = TileTraits<DT, K, true, 3>;
    __shared__ __align__(16) unsigned char smem[Tr::kLdsBytes];
    if (st->status) return;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int64_t off = r * (int64_t)len;
        block_sort_tile<DT, K, true, VM, 3, false, false, NET>(
            kin + off, VM == kVals ? vin + off : nullptr, kout + off,
            VM != kNoVals ? vout + off : nullptr, (int)len, 0u, smem);
        __syncthreads();  // the next row reuses the LDS
    }
}

// ---------------------------------------------- sorts, tiled path ---
// The runs of the tiled segments, sorted by the flat sort's block sort (for
// keys-only runs its 1024-thread shape, 32 outputs per thread in its LDS
// levels, its own register budget), each run written where its segment's
// first merge pass reads it (the output itself for one run).  A resident
// grid takes slots of two list entries from kSegQueues queues (slot k from
// queue k % kSegQueues; workgroup b draws from queue b % kSegQueues, the
// queue of its XCD); the entry of a run's first list tile sorts the run.
// Runs cost from a copy (already in order) to a whole block sort, so
// workgroups draw slots as they finish; each draws its next slot before
// sorting the current one, so the atomic's latency hides behind the loads.
template <int DT, int K, bool STABLE, int VM, int NET>
__global__ __launch_bounds__((SegRun<DT, K, STABLE>::Tr::kThreads),
                             (SegRun<DT, K, STABLE>::Tr::kWavesPerSimd))
void k_seg_tile_sort(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                     uint32_t* wk, uint32_t* wv, const uint32_t* __restrict__ offsets,
                     uint32_t uni_len, const SegState* st, const uint2* __restrict__ tiles) {
    using R = SegRun<DT, K, STABLE>;
    using Tr = typename R::Tr;
    __shared__ __align__(16) unsigned char smem[Tr::kLdsBytes];
    constexpr int kRun = R::kRun;
    constexpr uint32_t kPer = R::kRun / R::kListTile;  // list tiles per run
    __shared__ uint32_t s_next;
    if (st->status) return;
    const uint32_t n = st->tiles;
    const uint32_t q = blockIdx.x % kSegQueues;
    uint32_t* head = const_cast<uint32_t*>(&st->queue[q][0]);
    if (threadIdx.x == 0) s_next = atomicAdd(head, 1u);
    __syncthreads();
    uint32_t slot = s_next * kSegQueues + q;
    __syncthreads();  // s_next is written again at the end of the first round
    while (2 * (uint64_t)slot < n) {
        // the next slot, drawn now and published at the end of this one
        uint32_t next = 0;
        if (threadIdx.x == 0) next = atomicAdd(head, 1u);
        for (uint32_t e = 2 * slot; e < 2 * slot + 2 && e < n; ++e) {
            const uint2 tc = tiles[e];
            if (tc.y % kPer != 0) continue;  // uniform: not a run's first list tile
            uint32_t off, len;
            seg_bounds(offsets, tc.x, uni_len, off, len);
            const int passes = seg_global_passes<!STABLE>(len, kRun);
            const uint32_t first = tc.y * (uint32_t)R::kListTile;
            const int nv = min(kRun, (int)(len - first));
            uint32_t* kd = ((passes & 1) ? wk : kout) + off + first;
            uint32_t* vd = VM != kNoVals ? ((passes & 1) ? wv : vout) + off + first : nullptr;
            const uint32_t* ks = kin + off + first;
            const uint32_t* vs = VM == kVals ? vin + off + first : nullptr;
            bool done = false;
            if constexpr (!STABLE) done = copy_if_in_order<DT, Tr::kKPL>(ks, kd, nv, smem);
            if (!__builtin_amdgcn_readfirstlane(done))
                block_sort_tile<DT, K, STABLE, VM, R::kShape, true, false, NET>(
                    ks, vs, kd, vd, nv, first, smem);
            __syncthreads();  // the next run reuses the LDS
        }
        if (threadIdx.x == 0) s_next = next;
        __syncthreads();
        slot = s_next * kSegQueues + q;
        __syncthreads();  // s_next is written again in the next round
    }
}

// ---------------------------------------------- merge passes, tiled path ---
// Pass p of every tiled segment that has more than p passes: runs of
// run << p become runs of run << (p + 1), one output tile (a list tile) per
// list entry.
// The data alternate between the output and the workspace so that the last
// pass of each segment lands in the output.

struct SegTilePass {
    const uint32_t* ks;  // keys before the pass (segment-relative after + off)
    const uint32_t* vs;
    uint32_t* kd;        // keys after the pass
    uint32_t* vd;
    uint32_t off, len;
    int base, la, lb, d0, d1;  // merge of [base, base+la) and [base+la, base+la+lb)
};

// Geometry of list entry (seg, c) in pass p (runs of `run` keys after the
// tile sort, output tiles of `tile` keys); false when the segment has no
// binary pass p (FOUR: keys-only, whose segments of three or four runs take
// the four-way pass instead).
template <bool VALS, bool FOUR>
__device__ __forceinline__ bool seg_tile_pass(uint2 tc, int p, int tile, int run,
                                              const uint32_t* offsets, uint32_t uni_len,
                                              uint32_t* kout, uint32_t* vout, uint32_t* wk,
                                              uint32_t* wv, SegTilePass& g) {
    seg_bounds(offsets, tc.x, uni_len, g.off, g.len);
    const int passes = seg_passes((g.len + run - 1) / run);
    if (passes <= p || (FOUR && passes == 2)) return false;
    const bool src_ws = ((passes - p) & 1) != 0;  // before pass p the data sit in wk
    g.ks = (src_ws ? wk : kout) + g.off;
    g.kd = (src_ws ? kout : wk) + g.off;
    g.vs = VALS ? (src_ws ? wv : vout) + g.off : nullptr;
    g.vd = VALS ? (src_ws ? vout : wv) + g.off : nullptr;
    const int L = run << p;
    const int len = (int)g.len;
    const int g0 = (int)tc.y * tile;
    g.base = g0 & ~(2 * L - 1);
    g.la = min(L, len - g.base);
    g.lb = min(L, len - g.base - g.la);
    g.d0 = g0 - g.base;
    g.d1 = min(g.d0 + tile, g.la + g.lb);
    return true;
}

// Merge-path split of every list entry's first output (one thread each).
template <int DT, bool VALS>
__global__ __launch_bounds__(256) void k_seg_tile_part(
    uint32_t* kout, uint32_t* vout, uint32_t* wk, uint32_t* wv,
    const uint32_t* __restrict__ offsets, uint32_t uni_len, const SegState* st,
    const uint2* __restrict__ tiles, int32_t* __restrict__ part, int tile, int run, int p) {
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (st->status || e >= st->mtiles) return;
    SegTilePass g;
    if (!seg_tile_pass<VALS, !VALS && DT != kF32>(tiles[e], p, tile, run, offsets, uni_len, kout,
                                                   vout, wk, wv, g))
        return;
    part[e] = corank_global<DT>(g.ks + g.base, g.la, g.ks + g.base + g.la, g.lb, g.d0);
}

// The output tiles of pass p, workgroups taking list entries in turn.  The
// integer kernels are held to three workgroups per compute unit (84 VGPRs,
// which they fit without spilling); the float ones would spill.
template <int DT, bool VALS, int KPT>
__global__ __launch_bounds__(kBlockThreads, DT == kF32 ? 1 : 6) void k_seg_tile_merge(
    uint32_t* kout, uint32_t* vout, uint32_t* wk, uint32_t* wv,
    const uint32_t* __restrict__ offsets, uint32_t uni_len, const SegState* st,
    const uint2* __restrict__ tiles, const int32_t* __restrict__ part, int run, int p) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int kTile = KPT * kBlockThreads;
    uint32_t* sk = reinterpret_cast<uint32_t*>(smem);
    uint32_t* sv = sk + seg_merge_words(kTile);
    if (st->status) return;
    const uint32_t n = st->mtiles;
    for (uint32_t e = blockIdx.x; e < n; e += gridDim.x) {
        SegTilePass g;
        if (!seg_tile_pass<VALS, !VALS && DT != kF32>(tiles[e], p, kTile, run, offsets, uni_len,
                                                       kout, vout, wk, wv, g))
            continue;
        const int i0 = part[e];
        const int i1 = g.d1 == g.la + g.lb ? g.la : part[e + 1];
        seg_merge_tile<DT, VALS, KPT>(g.ks, g.vs, g.kd, g.vd, g.base, g.la, g.d0, g.d1, i0, i1,
                                      sk, sv);
    }
}

// ------------------------------------------ four-way pass, tiled path ---
// A keys-only tiled segment of three or four runs merges them in one pass,
// with the tiles and the tile merge of the flat sort's four-way passes.  One
// workgroup per segment of the four-way list: the first key of every
// kSampleChunk-key chunk of every run is staged in LDS (run r at r * CL, CL
// = run / kSampleChunk chunks) and ranked in the segment's order (key, run,
// position) against the other runs' samples; every kM4SamplesPerTile-th
// sample in that order is a tile boundary, whose splits in the other runs
// are refined inside one chunk.  The segment then appends one record per
// tile to the four-way tile list.
template <int DT>
__global__ __launch_bounds__(256) void k_seg_m4_bounds(const uint32_t* __restrict__ src,
                                                       const uint32_t* __restrict__ offsets,
                                                       uint32_t uni_len, int64_t num_segments,
                                                       SegState* st,
                                                       const uint32_t* __restrict__ lists,
                                                       Seg4Tile* __restrict__ tiles4, int run,
                                                       int lg_cl) {
    __shared__ uint32_t smp_g[1 + 4 * kSeg4MaxChunks];  // a guard word, then the samples
    __shared__ int32_t rows[(kSeg4MaxTiles + 1) * 4];
    __shared__ M4Cut cuts[kSeg4MaxTiles];
    __shared__ int ncut;
    __shared__ uint32_t s_base;
    uint32_t* smp = smp_g + 1;
    const int tid = threadIdx.x;
    const int CL = 1 << lg_cl;
    if (st->status) return;
    const uint32_t n4 = st->count[kList4];
    const uint32_t* list4 = lists + (int64_t)kList4 * num_segments;
    for (uint32_t g = blockIdx.x; g < n4; g += gridDim.x) {
        uint32_t off, len;
        seg_bounds(offsets, list4[g], uni_len, off, len);
        const uint32_t* gin = src + off;
        int64_t rl[4], rs[4];
        int total = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t rem = (int64_t)len - (int64_t)k * run;
            rl[k] = rem <= 0 ? 0 : (rem < run ? rem : run);
            rs[k] = m4_ceil_div(rl[k], kSampleChunk);
            total += (int)rs[k];
        }
        const int tiles = (total + kM4SamplesPerTile - 1) / kM4SamplesPerTile;
        if (tid == 0) ncut = 0;
        if (tid < 4 * CL) {
            const int r = tid >> lg_cl, i = tid & (CL - 1);
            if (i < m4_sel(rs, r)) smp[tid] = ord_key<DT>(gin[(int64_t)r * run + (int64_t)i * kSampleChunk]);
        }
        __syncthreads();
        if (tid < 4 * CL) {
            const int r = tid >> lg_cl;
            const int64_t ic = tid & (CL - 1);
            if (ic < m4_sel(rs, r)) {
                const uint32_t ov = smp[tid];
                const int o[3] = {r == 0 ? 1 : 0, r <= 1 ? 2 : 1, r <= 2 ? 3 : 2};  // other runs
                const uint32_t* sa[3] = {smp + o[0] * CL, smp + o[1] * CL, smp + o[2] * CL};
                const int ma[3] = {(int)m4_sel(rs, o[0]), (int)m4_sel(rs, o[1]),
                                   (int)m4_sel(rs, o[2])};
                int cj[3];
                m4_lds_count3(sa, ma, o, ov, r, lg_cl, cj);
                const int64_t rank = ic + cj[0] + cj[1] + cj[2];
                if (rank == 0) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        rows[k] = 0;
                        rows[tiles * 4 + k] = (int32_t)rl[k];
                    }
                } else if (rank % kM4SamplesPerTile == 0) {
                    M4Cut c;
                    c.g = 0;
                    c.ic = ic;
                    c.rank = rank;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        c.cnt[k] = k == r ? ic : k == o[0] ? cj[0] : k == o[1] ? cj[1] : cj[2];
                    c.ov = ov;
                    c.r = r;
                    cuts[atomicAdd(&ncut, 1)] = c;  // at most tiles - 1 cuts
                }
            }
        }
        __syncthreads();
        // each (cut, run) pair by one thread: keys of run k before the cut
        {
            const int e = tid >> 2, k = tid & 3;
            if (e < ncut) {
                const M4Cut& c = cuts[e];
                const int64_t split =
                    k == c.r ? c.ic * kSampleChunk
                             : m4_key_count<DT>(gin + (int64_t)k * run, m4_sel(rl, k),
                                                m4_sel(c.cnt, k), c.ov, k, c.r);
                rows[(c.rank / kM4SamplesPerTile) * 4 + k] = (int32_t)split;
            }
        }
        if (tid == 0) s_base = atomicAdd(&st->tiles4, (uint32_t)tiles);
        __syncthreads();
        if (tid < tiles) {
            Seg4Tile t;
            t.off = off;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                t.lo[k] = rows[tid * 4 + k];
                t.c[k] = rows[(tid + 1) * 4 + k] - rows[tid * 4 + k];
            }
#pragma unroll
            for (int k = 0; k < 7; ++k) t.pad[k] = 0u;
            tiles4[s_base + tid] = t;
        }
        __syncthreads();  // the LDS is reused for the next segment
    }
}

// The four-way tiles, workgroups taking records in turn: slices of the
// runs in src (where the tile sort left them), merged into dst.
template <int DT, int THREADS, int KPT>
__global__ __launch_bounds__(THREADS, 8) void k_seg_merge4(const uint32_t* __restrict__ src,
                                                        uint32_t* __restrict__ dst,
                                                        const SegState* st,
                                                        const Seg4Tile* __restrict__ tiles4,
                                                        int run) {
    __shared__ __align__(16) uint32_t lds[m4_lds_words(THREADS)];
    if (st->status) return;
    const uint32_t n = st->tiles4;
    for (uint32_t e = blockIdx.x; e < n; e += gridDim.x) {
        const Seg4Tile t = tiles4[e];
        int lo[4], c[4];
        int64_t ostart = t.off;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            lo[k] = t.lo[k];
            c[k] = t.c[k];
            ostart += lo[k];
        }
        m4_merge_tile<DT, THREADS, KPT, false>(src + t.off, run, lo, c, dst, ostart, nullptr,
                                               nullptr, lds);
        __syncthreads();  // the LDS is reused for the next tile
    }
}

// ------------------------------------------------- merge-path diagnostic ---
// out[i] = number of elements of A among the first diags[i] outputs of the
// stable merge of A and B (A first on equal keys), by the co-rank search the
// merge passes use.  One thread per diagonal.
template <int DT>
__global__ __launch_bounds__(256) void k_merge_path_split(const uint32_t* __restrict__ a, int la,
                                                          const uint32_t* __restrict__ b, int lb,
                                                          const int32_t* __restrict__ diags,
                                                          int32_t* __restrict__ out, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int d = diags[i];
    out[i] = (d < 0 || d > la + lb) ? -1 : corank_global<DT>(a, la, b, lb, d);
}

int launch_merge_path_split(const uint32_t* a, int64_t la, const uint32_t* b, int64_t lb,
                            const int32_t* diags, int32_t* out, int64_t count, int dtype,
                            hipStream_t stream) {
    if (count == 0) return 0;
    const unsigned grid = (unsigned)((count + 255) / 256);
    switch (dtype) {
        case kU32:
            hipLaunchKernelGGL(k_merge_path_split<kU32>, dim3(grid), dim3(256), 0, stream, a,
                               (int)la, b, (int)lb, diags, out, (int)count);
            break;
        case kI32:
            hipLaunchKernelGGL(k_merge_path_split<kI32>, dim3(grid), dim3(256), 0, stream, a,
                               (int)la, b, (int)lb, diags, out, (int)count);
            break;
        default:
            hipLaunchKernelGGL(k_merge_path_split<kF32>, dim3(grid), dim3(256), 0, stream, a,
                               (int)la, b, (int)lb, diags, out, (int)count);
            break;
    }
    return (int)hipGetLastError();
}

// ------------------------------------------------------------------ host ---
namespace {

template <typename Kern>
int fill_grid(Kern kern, int threads, size_t lds, int* out) {
    return resident_grid(reinterpret_cast<const void*>(kern), threads, lds, out);
}

struct SegWs {
    uint32_t *wk, *wv, *lists;
    SegState* st;
    uint2* tiles;
    uint2* mtiles;
    int32_t* part;
    Seg4Tile* tiles4;
    size_t max_tiles;
    size_t max_segs4;  // bound on the four-way segments
};

template <int DT, int K, bool STABLE, int VM, int NET>
int launch_seg_kernel(const SegArgs& a, const SegWs& w, uint32_t uni_len) {
    using Tr = SegTraits<DT, K, STABLE, VM>;
    constexpr bool kVals = VM != kNoVals;
    constexpr int kTile = TileTraits<DT, K, STABLE>::kTile;
    constexpr int kKpt = kTile / kBlockThreads;
    constexpr int kRun = SegRun<DT, K, STABLE>::kRun;
    auto kern = &k_segmented<DT, K, STABLE, VM, NET>;
    if (int rc = set_dynamic_lds(reinterpret_cast<const void*>(kern), Tr::kLds)) return rc;
    int grid = a.grid;
    if (grid <= 0) {
        if (int rc = fill_grid(kern, kBlockThreads, Tr::kLds, &grid)) return rc;
    }
    // equal-length segments: the host knows their class and pass count
    // binary passes, and whether any segment takes the four-way pass
    // (keys-only segments of three or four runs: seg_global_passes)
    bool any_tiled = true;
    int npass = seg_passes((uint32_t)(kSegTiledMax * kTile / kRun));
    if (!STABLE) npass = std::min(npass, 1);
    bool any4 = !STABLE;
    if (!a.offsets) {
        const int64_t len = uni_len;
        any_tiled = len > a.block_max && len <= (int64_t)kSegTiledMax * kTile;
        const int p = any_tiled ? seg_passes((uint32_t)((len + kRun - 1) / kRun)) : 0;
        any4 = !STABLE && p == 2;
        npass = any4 ? 0 : p;
    }
    // equal stable rows of one workgroup-sized tile: the row kernel
    if constexpr (STABLE) {
        constexpr int kRowTile = TileTraits<DT, K, true, 3>::kTile;
        if (!a.offsets && uni_len > (uint32_t)a.wave_max && uni_len <= (uint32_t)a.block_max &&
            uni_len <= (uint32_t)kRowTile) {
            auto rkern = &k_seg_rows<DT, K, VM, NET>;
            int rgrid = 0;
            if (int rc = fill_grid(rkern, TileTraits<DT, K, true, 3>::kThreads, 0, &rgrid))
                return rc;
            {
                LaunchTimer timer("seg_rows", a.n_total, a.stream);
                hipLaunchKernelGGL(rkern, dim3(rgrid), dim3(TileTraits<DT, K, true, 3>::kThreads),
                                   0, a.stream, a.kin, a.vin, a.kout, a.vout, a.num_segments,
                                   uni_len, w.st);
            }
            return (int)hipGetLastError();
        }
    }
    if (any_tiled) {
        auto skern = &k_seg_tile_sort<DT, K, STABLE, VM, NET>;
        constexpr int kSortThreads = SegRun<DT, K, STABLE>::Tr::kThreads;
        int sgrid = 0;
        if (int rc = fill_grid(skern, kSortThreads, 0, &sgrid)) return rc;
        // a resident grid, a multiple of the queue count
        sgrid = std::max(kSegQueues, sgrid - sgrid % kSegQueues);
        LaunchTimer timer("seg_tile_sort", a.n_total, a.stream);
        hipLaunchKernelGGL(skern, dim3(sgrid), dim3(kSortThreads), 0, a.stream, a.kin, a.vin,
                           a.kout, a.vout, w.wk, w.wv, a.offsets, uni_len, w.st, w.tiles);
    }
    if (int rc = (int)hipGetLastError()) return rc;
    {
        LaunchTimer timer("segmented", a.n_total, a.stream);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlockThreads), Tr::kLds, a.stream, a.kin,
                           a.vin, a.kout, a.vout, w.wk, w.wv, a.offsets, a.num_segments, uni_len,
                           w.st, w.lists, a.set_mask);
    }
    if (int rc = (int)hipGetLastError()) return rc;
    // merge passes of the tiled segments (none of them when the list is empty)
    auto mkern = &k_seg_tile_merge<DT, kVals, kKpt>;
    const size_t mlds = (size_t)seg_merge_words(kTile) * 4 * (kVals ? 2 : 1);
    if (int rc = set_dynamic_lds(reinterpret_cast<const void*>(mkern), mlds)) return rc;
    int mgrid = 0;
    if (int rc = fill_grid(mkern, kBlockThreads, mlds, &mgrid)) return rc;
    const unsigned pgrid = (unsigned)((w.max_tiles + 255) / 256);
    for (int p = 0; p < npass; ++p) {
        {
            LaunchTimer timer("seg_tile_part", a.n_total, a.stream);
            hipLaunchKernelGGL((k_seg_tile_part<DT, kVals>), dim3(pgrid), dim3(256), 0, a.stream,
                               a.kout, a.vout, w.wk, w.wv, a.offsets, uni_len, w.st, w.mtiles,
                               w.part, kTile, kRun, p);
        }
        if (int rc = (int)hipGetLastError()) return rc;
        {
            LaunchTimer timer("seg_tile_merge", a.n_total, a.stream);
            hipLaunchKernelGGL(mkern, dim3(mgrid), dim3(kBlockThreads), mlds, a.stream, a.kout,
                               a.vout, w.wk, w.wv, a.offsets, uni_len, w.st, w.mtiles, w.part,
                               kRun, p);
        }
        if (int rc = (int)hipGetLastError()) return rc;
    }
    if constexpr (!STABLE) {
        if (any4) {
            static_assert(kRun / kSampleChunk <= kSeg4MaxChunks, "four-way runs fit the samples");
            const int lg_cl = ilog2(kRun / kSampleChunk);
            const unsigned bgrid = (unsigned)std::max<size_t>(
                1, std::min<size_t>(w.max_segs4, 4096));
            {
                LaunchTimer timer("seg_m4_bounds", a.n_total, a.stream);
                hipLaunchKernelGGL(k_seg_m4_bounds<DT>, dim3(bgrid), dim3(256), 0, a.stream, w.wk,
                                   a.offsets, uni_len, a.num_segments, w.st, w.lists, w.tiles4,
                                   kRun, lg_cl);
            }
            if (int rc = (int)hipGetLastError()) return rc;
            auto m4kern = &k_seg_merge4<DT, 512, 16>;
            int m4grid = 0;
            if (int rc = fill_grid(m4kern, 512, 0, &m4grid)) return rc;
            {
                LaunchTimer timer("seg_merge4", a.n_total, a.stream);
                hipLaunchKernelGGL(m4kern, dim3(m4grid), dim3(512), 0, a.stream, w.wk, a.kout,
                                   w.st, w.tiles4, kRun);
            }
            if (int rc = (int)hipGetLastError()) return rc;
        }
    }
    return 0;
}

template <int DT, int K, int NET>
int dispatch_seg_net(const SegArgs& a, const SegWs& w, uint32_t uni_len) {
    if (a.vmode == kVals) return launch_seg_kernel<DT, K, true, kVals, NET>(a, w, uni_len);
    if (a.vmode == kArg) return launch_seg_kernel<DT, K, true, kArg, NET>(a, w, uni_len);
    if constexpr (DT == kF32)
        return launch_seg_kernel<DT, K, true, kNoVals, NET>(a, w, uni_len);
    else
        return launch_seg_kernel<DT, K, false, kNoVals, NET>(a, w, uni_len);
}

template <int DT, int K>
int dispatch_seg(const SegArgs& a, const SegWs& w, uint32_t uni_len) {
    return a.net == kNetSplit ? dispatch_seg_net<DT, K, kNetSplit>(a, w, uni_len)
                              : dispatch_seg_net<DT, K, kNetPlain>(a, w, uni_len);
}

}  // namespace

int launch_segmented(const SegArgs& a) {
    if (a.num_segments == 0 || a.n_total == 0) return 0;
    const bool vals = a.vmode != kNoVals;
    uint8_t* ws = static_cast<uint8_t*>(a.ws);
    const size_t nk = align_up((size_t)a.n_total * 4, 256);
    const size_t nl = align_up((size_t)a.num_segments * 4 * kNumLists, 256);
    SegWs w;
    w.max_tiles = seg_max_tiles(a.n_total, a.num_segments);
    w.max_segs4 = seg_max_tiles4(a.n_total, a.num_segments) / kSeg4MaxTiles;
    w.wk = reinterpret_cast<uint32_t*>(ws);
    w.wv = vals ? reinterpret_cast<uint32_t*>(ws + nk) : nullptr;
    uint8_t* q = ws + nk + (vals ? nk : 0);
    w.lists = reinterpret_cast<uint32_t*>(q);
    q += nl;
    w.st = reinterpret_cast<SegState*>(q);
    q += align_up(sizeof(SegState), 256);
    w.tiles = reinterpret_cast<uint2*>(q);
    q += align_up(w.max_tiles * 8, 256);
    w.mtiles = reinterpret_cast<uint2*>(q);
    q += align_up(w.max_tiles * 8, 256);
    w.part = reinterpret_cast<int32_t*>(q);
    q += align_up(w.max_tiles * 4, 256);
    w.tiles4 = reinterpret_cast<Seg4Tile*>(q);
    const uint32_t uni_len = a.offsets ? 0u : (uint32_t)(a.n_total / a.num_segments);
    const uint32_t tile = 1024u * (uint32_t)a.leaf_k;  // the block-sort tile of every segmented kernel
    // keys-only sorts (integer keys, no payload) sort runs of two tiles and
    // merge segments of more than two runs four ways
    const bool stable = a.vmode != kNoVals || a.dtype == kF32;
    const uint32_t merge_min = stable ? tile : 2u * tile;  // one run of the tile sort
    const uint32_t four_min = stable ? 0u : 4u * tile;

    {
        LaunchTimer timer("seg_init", 1, a.stream);
        hipLaunchKernelGGL(k_seg_init, dim3(1), dim3(256), 0, a.stream, w.st);
    }
    if (int rc = (int)hipGetLastError()) return rc;
    {
        LaunchTimer timer("seg_bin", a.num_segments, a.stream);
        hipLaunchKernelGGL(k_seg_bin, dim3((unsigned)((a.num_segments + 255) / 256)), dim3(256),
                           0, a.stream, a.offsets, a.num_segments, a.n_total, uni_len,
                           a.lane_max, a.wave_max, a.block_max, tile, merge_min, four_min, w.st,
                           w.lists, w.tiles, w.mtiles, (uint32_t)w.max_tiles);
    }
    if (int rc = (int)hipGetLastError()) return rc;
    int rc = 0;
    switch (a.dtype) {
        case kU32:
            rc = a.leaf_k == 8 ? dispatch_seg<kU32, 8>(a, w, uni_len)
                               : dispatch_seg<kU32, 4>(a, w, uni_len);
            break;
        case kI32:
            rc = a.leaf_k == 8 ? dispatch_seg<kI32, 8>(a, w, uni_len)
                               : dispatch_seg<kI32, 4>(a, w, uni_len);
            break;
        default:
            rc = a.leaf_k == 8 ? dispatch_seg<kF32, 8>(a, w, uni_len)
                               : dispatch_seg<kF32, 4>(a, w, uni_len);
            break;
    }
    if (rc || !a.debug_check) return rc;
    const unsigned vgrid = (unsigned)std::min<int64_t>((a.num_segments + 3) / 4, 4096);
    {
        LaunchTimer timer("seg_verify", a.n_total, a.stream);
        switch (a.dtype) {
            case kU32:
                hipLaunchKernelGGL(k_seg_verify<kU32>, dim3(vgrid), dim3(256), 0, a.stream, a.kout,
                                   a.offsets, a.num_segments, uni_len, w.st);
                break;
            case kI32:
                hipLaunchKernelGGL(k_seg_verify<kI32>, dim3(vgrid), dim3(256), 0, a.stream, a.kout,
                                   a.offsets, a.num_segments, uni_len, w.st);
                break;
            default:
                hipLaunchKernelGGL(k_seg_verify<kF32>, dim3(vgrid), dim3(256), 0, a.stream, a.kout,
                                   a.offsets, a.num_segments, uni_len, w.st);
                break;
        }
    }
    return (int)hipGetLastError();
}

size_t seg_status_offset(int64_t n_total, int64_t num_segments, bool vals) {
    const size_t nk = align_up((size_t)n_total * 4, 256);
    const size_t nl = align_up((size_t)num_segments * 4 * kNumLists, 256);
    return nk + (vals ? nk : 0) + nl + offsetof(SegState, status);
}

}  // namespace msn
