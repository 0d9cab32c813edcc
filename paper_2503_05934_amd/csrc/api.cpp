// C ABI of libmsn (declared in include/msn.h): argument validation on the
// host, then the kernel launches of sort.hip, segmented.hip, backward.hip.
// Every check runs before anything is enqueued, so a rejected call never
// touches the GPU.
#include <string.h>

#include <initializer_list>
#include <map>
#include <tuple>
#include <utility>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace msn {

int set_dynamic_lds(const void* kernel, size_t bytes) {
    int dev = 0;
    if (int rc = (int)hipGetDevice(&dev)) return rc;
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, size_t> done;  // (kernel, device)
    std::lock_guard<std::mutex> lock(mu);
    auto it = done.find({kernel, dev});
    if (it != done.end() && it->second >= bytes) return 0;
    const int rc =
        (int)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (rc == 0) done[{kernel, dev}] = bytes;
    return rc;
}

int resident_grid(const void* kernel, int threads, size_t lds, int* out) {
    int dev = 0;
    if (int rc = (int)hipGetDevice(&dev)) return rc;
    using Key = std::tuple<const void*, int, int, size_t>;  // kernel, device, threads, LDS
    static std::mutex mu;
    static std::map<Key, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    const Key key{kernel, dev, threads, lds};
    auto it = cache.find(key);
    if (it == cache.end()) {
        int cus = 0, per_cu = 0;
        if (int rc = (int)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev))
            return rc;
        if (int rc = (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads,
                                                                       lds))
            return rc;
        it = cache.emplace(key, cus * (per_cu > 0 ? per_cu : 1)).first;
    }
    *out = it->second;
    return 0;
}

namespace {

struct TimedLaunch {
    const char* kind;
    int64_t elements;
    int ev0;
    int ev1;
};

struct TimingState {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> events;
    std::vector<TimedLaunch> launches;
    size_t next = 0;
};

TimingState& timing() {
    static TimingState t;
    return t;
}

}  // namespace

LaunchTimer::LaunchTimer(const char* kind, int64_t elements, hipStream_t stream)
    : slot_(-1), stream_(stream) {
    TimingState& t = timing();
    std::lock_guard<std::mutex> lock(t.mu);
    if (!t.on || t.next + 2 > t.events.size()) return;
    slot_ = (int)t.launches.size();
    t.launches.push_back({kind, elements, (int)t.next, (int)t.next + 1});
    t.next += 2;
    (void)hipEventRecord(t.events[t.launches[slot_].ev0], stream_);
}

LaunchTimer::~LaunchTimer() {
    if (slot_ < 0) return;
    TimingState& t = timing();
    std::lock_guard<std::mutex> lock(t.mu);
    (void)hipEventRecord(t.events[t.launches[slot_].ev1], stream_);
}

}  // namespace msn

namespace {

constexpr int64_t kMaxN = 0x7fffffffLL;

bool valid_dtype(int d) { return d == MSN_U32 || d == MSN_I32 || d == MSN_F32; }
// A network set of Table 3 on the GPU: the keys of a lane's group, how the
// group is sorted (msn::kNet*), the set's network sizes (bit k = size k) and
// the longest subarray one lane sorts by default in the batched sort.
struct LeafSet {
    int group;
    int net;
    uint32_t sizes;
    int lane_max;
};

constexpr uint32_t bits(std::initializer_list<int> l) {
    uint32_t m = 0;
    for (int x : l) m |= 1u << x;
    return m;
}

// Returns false for an unknown code.  The network-free sort keeps the 6-to-8
// tile shapes.
bool leaf_set(int leaf, LeafSet* out) {
    using msn::kNetNone;
    using msn::kNetPlain;
    using msn::kNetSplit;
    switch (leaf) {
        case MSN_LEAF_6TO8: *out = {8, kNetPlain, bits({6, 7, 8}), 8}; return true;
        case MSN_LEAF_3TO5: *out = {4, kNetPlain, bits({3, 4, 5}), 4}; return true;
        case MSN_LEAF_NONE: *out = {8, kNetNone, 0u, 0}; return true;
        case MSN_LEAF_POW2: *out = {8, kNetPlain, bits({4, 8}), 8}; return true;
        case MSN_LEAF_EVEN: *out = {8, kNetPlain, bits({4, 6, 8}), 8}; return true;
        case MSN_LEAF_ODD: *out = {8, kNetSplit, bits({3, 5, 7}), 8}; return true;
        case MSN_LEAF_3: *out = {4, kNetSplit, bits({3}), 4}; return true;
        case MSN_LEAF_3TO4: *out = {4, kNetPlain, bits({3, 4}), 4}; return true;
        case MSN_LEAF_3TO8: *out = {8, kNetPlain, bits({3, 4, 5, 6, 7, 8}), 8}; return true;
        case MSN_LEAF_VARSORT3: *out = {4, kNetSplit, bits({2, 3}), 3}; return true;
        case MSN_LEAF_VARSORT4: *out = {4, kNetPlain, bits({2, 3, 4}), 4}; return true;
        case MSN_LEAF_VARSORT5: *out = {8, kNetSplit, bits({2, 3, 4, 5}), 5}; return true;
        default: return false;
    }
}

int leaf_keys(int leaf) {
    LeafSet ls;
    return leaf_set(leaf, &ls) ? ls.group : 0;
}

bool misaligned(const void* p) { return p && ((uintptr_t)p & 3u) != 0; }

// Two ranges of n words either coincide (in-place) or do not overlap.
bool bad_overlap(const void* a, const void* b, int64_t n) {
    if (!a || !b || a == b) return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b, len = (uintptr_t)n * 4;
    return x < y + len && y < x + len;
}

// Ranges of na and nb words that share any word (equal starts included):
// the pairs that must stay apart even for in-place calls (a key array and a
// value array, the offsets and an output).
bool ranges_overlap(const void* a, int64_t na, const void* b, int64_t nb) {
    if (!a || !b || na <= 0 || nb <= 0) return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + (uintptr_t)nb * 4 && y < x + (uintptr_t)na * 4;
}
bool any_overlap(const void* a, const void* b, int64_t n) { return ranges_overlap(a, n, b, n); }

int merge_tile_of(const msn_tuning* t, int* out) {
    int mt = t && t->merge_tile ? t->merge_tile : msn::kDefaultMergeTile;
    if (mt != 2048 && mt != 4096 && mt != 8192) return MSN_ERR_CONFIG;
    *out = mt;
    return MSN_OK;
}

// Merge fan-in of the global passes: 2 or 4 (default 4).
int merge_ways_of(const msn_tuning* t, int* out) {
    const int w = t && t->merge_ways ? t->merge_ways : 4;
    if (w != 2 && w != 4) return MSN_ERR_CONFIG;
    *out = w;
    return MSN_OK;
}

// Keys per thread of the four-way merge kernel: 16 or 32 (default 16).
int merge4_kpt_of(const msn_tuning* t, int* out) {
    const int v = t && t->merge4_kpt ? t->merge4_kpt : 16;
    if (v != 16 && v != 32) return MSN_ERR_CONFIG;
    *out = v;
    return MSN_OK;
}

// First-sweep run length: 1024, 2048 or 4096 x the leaf size (default 2048 K).
int block_tile_of(const msn_tuning* t, int k, int* out) {
    int bt = t && t->block_tile ? t->block_tile : msn::kDefaultBlockTileMult * k;
    if (bt != 1024 * k && bt != 2048 * k && bt != 4096 * k) return MSN_ERR_CONFIG;
    *out = bt;
    return MSN_OK;
}

int sort_common(const void* keys_in, const uint32_t* vals_in, void* keys_out, uint32_t* vals_out,
                int64_t n, int dtype, int leaf, const msn_tuning* tuning, void* ws,
                size_t ws_bytes, void* stream, bool pairs) {
    if (!valid_dtype(dtype)) return MSN_ERR_DTYPE;
    const int k = leaf_keys(leaf);
    if (!k) return MSN_ERR_CONFIG;
    int mt = 0, bt = 0, mw = 0, m4k = 0;
    if (int rc = merge_tile_of(tuning, &mt)) return rc;
    if (int rc = merge4_kpt_of(tuning, &m4k)) return rc;
    if (int rc = block_tile_of(tuning, k, &bt)) return rc;
    if (int rc = merge_ways_of(tuning, &mw)) return rc;
    if (n < 0 || n > kMaxN) return MSN_ERR_SIZE;
    if (n == 0) return MSN_OK;
    if (!keys_in || !keys_out) return MSN_ERR_NULL;
    if (pairs && !vals_out) return MSN_ERR_NULL;
    if (misaligned(keys_in) || misaligned(keys_out) || misaligned(vals_in) || misaligned(vals_out) ||
        misaligned(ws))
        return MSN_ERR_UNSUPPORTED;
    if (bad_overlap(keys_in, keys_out, n) || bad_overlap(vals_in, vals_out, n) ||
        (pairs && (bad_overlap(keys_out, vals_out, n) || keys_out == (void*)vals_out)) ||
        any_overlap(keys_in, vals_out, n) || any_overlap(vals_in, keys_out, n))
        return MSN_ERR_SIZE;
    const int vmode = !pairs ? msn::kNoVals : vals_in ? msn::kVals : msn::kArg;
    const size_t need = msn::sort_ws_bytes(n, vmode != msn::kNoVals);
    if (!ws || ws_bytes < need) return MSN_ERR_WORKSPACE;
    msn::SortArgs a{static_cast<const uint32_t*>(keys_in), vals_in,
                    static_cast<uint32_t*>(keys_out), vals_out, n, dtype, k, vmode, mt, bt, mw, m4k, ws,
                    ws_bytes, static_cast<hipStream_t>(stream)};
    LeafSet ls;
    leaf_set(leaf, &ls);
    a.nets = ls.net;
    return msn::launch_sort(a);
}

}  // namespace

extern "C" {

int msn_version(void) { return 10000; }

int msn_timing_enable(int max_launches) {
    if (max_launches <= 0 || max_launches > (1 << 20)) return MSN_ERR_SIZE;
    msn::TimingState& t = msn::timing();
    std::lock_guard<std::mutex> lock(t.mu);
    for (hipEvent_t e : t.events) (void)hipEventDestroy(e);
    t.events.assign((size_t)max_launches * 2, nullptr);
    for (auto& e : t.events)
        if (int rc = (int)hipEventCreate(&e)) {
            t.events.clear();
            t.on = false;
            return rc;
        }
    t.launches.clear();
    t.next = 0;
    t.on = true;
    return MSN_OK;
}

int msn_timing_read(msn_kernel_stats* out, int capacity, int* count) {
    if (!count || (capacity > 0 && !out)) return MSN_ERR_NULL;
    msn::TimingState& t = msn::timing();
    std::lock_guard<std::mutex> lock(t.mu);
    std::map<std::string, msn_kernel_stats> acc;
    for (const auto& l : t.launches) {
        if (int rc = (int)hipEventSynchronize(t.events[l.ev1])) return rc;
        float ms = 0.f;
        if (int rc = (int)hipEventElapsedTime(&ms, t.events[l.ev0], t.events[l.ev1])) return rc;
        msn_kernel_stats& k = acc[l.kind];
        strncpy(k.kind, l.kind, sizeof k.kind - 1);
        k.launches += 1;
        k.elements += l.elements;
        k.total_ms += ms;
    }
    int i = 0;
    for (const auto& kv : acc) {
        if (i < capacity) out[i] = kv.second;
        ++i;
    }
    *count = i;
    return MSN_OK;
}

int msn_timing_disable(void) {
    msn::TimingState& t = msn::timing();
    std::lock_guard<std::mutex> lock(t.mu);
    for (hipEvent_t e : t.events) (void)hipEventDestroy(e);
    t.events.clear();
    t.launches.clear();
    t.next = 0;
    t.on = false;
    return MSN_OK;
}

const char* msn_status_string(int status) {
    switch (status) {
        case MSN_OK: return "ok";
        case MSN_ERR_NULL: return "required pointer is NULL";
        case MSN_ERR_SIZE: return "size, offset or overlap out of range";
        case MSN_ERR_DTYPE: return "unknown key type";
        case MSN_ERR_CONFIG: return "unknown leaf set, flag or tuning value";
        case MSN_ERR_WORKSPACE: return "workspace missing or too small";
        case MSN_ERR_UNSUPPORTED: return "request not supported (alignment)";
        default: return status > 0 ? "HIP launch error" : "unknown status";
    }
}

int msn_sort_keys_workspace_bytes(int64_t n, int dtype, int pairs, size_t* bytes) {
    if (!bytes) return MSN_ERR_NULL;
    if (!valid_dtype(dtype)) return MSN_ERR_DTYPE;
    if (n < 0 || n > kMaxN) return MSN_ERR_SIZE;
    *bytes = msn::sort_ws_bytes(n, pairs != 0);
    return MSN_OK;
}

int msn_sort_workspace_bytes(int64_t n, int dtype, int pairs, size_t* bytes) {
    return msn_sort_keys_workspace_bytes(n, dtype, pairs, bytes);
}

int msn_sort_keys(const void* keys_in, void* keys_out, int64_t n, int dtype, int leaf,
                  const msn_tuning* tuning, void* ws, size_t ws_bytes, void* stream) {
    return sort_common(keys_in, nullptr, keys_out, nullptr, n, dtype, leaf, tuning, ws, ws_bytes,
                       stream, false);
}

int msn_sort_keys_noalloc(const void* keys_in, void* keys_out, int64_t n, int dtype, int leaf,
                          const msn_tuning* tuning, void* stream) {
    if (n < 0 || n > msn::kNoAllocMaxKeys) return MSN_ERR_SIZE;
    if (n == 0) return sort_common(keys_in, nullptr, keys_out, nullptr, 0, dtype, leaf, tuning,
                                   nullptr, 0, stream, false);
    void* ws = nullptr;
    size_t ws_bytes = 0;
    if (int rc = msn::noalloc_scratch(static_cast<hipStream_t>(stream), &ws, &ws_bytes))
        return rc;
    return sort_common(keys_in, nullptr, keys_out, nullptr, n, dtype, leaf, tuning, ws, ws_bytes,
                       stream, false);
}

int msn_sort_pairs(const void* keys_in, const uint32_t* vals_in, void* keys_out,
                   uint32_t* vals_out, int64_t n, int dtype, int leaf, const msn_tuning* tuning,
                   void* ws, size_t ws_bytes, void* stream) {
    return sort_common(keys_in, vals_in, keys_out, vals_out, n, dtype, leaf, tuning, ws, ws_bytes,
                       stream, true);
}

int msn_quick_sort_workspace_bytes(int64_t n, int dtype, size_t* bytes) {
    if (!bytes) return MSN_ERR_NULL;
    if (!valid_dtype(dtype)) return MSN_ERR_DTYPE;
    if (dtype == MSN_F32) return MSN_ERR_UNSUPPORTED;
    if (n < 0 || n > kMaxN) return MSN_ERR_SIZE;
    *bytes = msn::quick_ws_bytes(n);
    return MSN_OK;
}

int msn_quick_sort_keys(const void* keys_in, void* keys_out, int64_t n, int dtype, int leaf,
                        const msn_tuning* tuning, void* ws, size_t ws_bytes, void* stream) {
    if (!valid_dtype(dtype)) return MSN_ERR_DTYPE;
    if (dtype == MSN_F32) return MSN_ERR_UNSUPPORTED;  // the partition is not stable
    const int k = leaf_keys(leaf);
    if (!k) return MSN_ERR_CONFIG;
    const int rounds = tuning ? tuning->quick_rounds : 0;
    if (rounds < 0 || rounds > msn::kQuickMaxRounds) return MSN_ERR_CONFIG;
    if (n < 0 || n > kMaxN) return MSN_ERR_SIZE;
    if (n == 0) return MSN_OK;
    if (!keys_in || !keys_out) return MSN_ERR_NULL;
    if (misaligned(keys_in) || misaligned(keys_out) || misaligned(ws)) return MSN_ERR_UNSUPPORTED;
    if (bad_overlap(keys_in, keys_out, n)) return MSN_ERR_SIZE;
    const size_t need = msn::quick_ws_bytes(n);
    if (!ws || ws_bytes < need) return MSN_ERR_WORKSPACE;
    LeafSet ls;
    leaf_set(leaf, &ls);
    msn::QuickArgs a{static_cast<const uint32_t*>(keys_in), static_cast<uint32_t*>(keys_out), n,
                     dtype, k, ls.net, ls.sizes, rounds, ws, ws_bytes,
                     static_cast<hipStream_t>(stream)};
    return msn::launch_quick(a);
}

int msn_segmented_sort_workspace_bytes(int64_t n_total, int64_t num_segments, int dtype,
                                       int pairs, size_t* bytes) {
    if (!bytes) return MSN_ERR_NULL;
    if (!valid_dtype(dtype)) return MSN_ERR_DTYPE;
    if (n_total < 0 || n_total > kMaxN || num_segments < 0 || num_segments > kMaxN)
        return MSN_ERR_SIZE;
    *bytes = msn::seg_ws_bytes(n_total, num_segments, pairs != 0);
    return MSN_OK;
}

int msn_segmented_sort(const void* keys_in, const uint32_t* vals_in, void* keys_out,
                       uint32_t* vals_out, const uint32_t* offsets, int64_t num_segments,
                       int64_t n_total, int dtype, int leaf, unsigned flags,
                       const msn_tuning* tuning, void* ws, size_t ws_bytes, void* stream) {
    if (!valid_dtype(dtype)) return MSN_ERR_DTYPE;
    const int k = leaf_keys(leaf);
    if (!k) return MSN_ERR_CONFIG;
    if (leaf == MSN_LEAF_NONE) return MSN_ERR_UNSUPPORTED;  // flat sorts only
    if (flags & ~(MSN_ARGSORT | MSN_DEBUG_CHECK)) return MSN_ERR_CONFIG;
    const bool argsort = (flags & MSN_ARGSORT) != 0;
    if (argsort && vals_in) return MSN_ERR_CONFIG;
    if (!argsort && !vals_in && vals_out) return MSN_ERR_CONFIG;
    if ((argsort || vals_in) && !vals_out) return MSN_ERR_NULL;
    if (n_total < 0 || n_total > kMaxN || num_segments < 0 || num_segments > kMaxN)
        return MSN_ERR_SIZE;
    if (num_segments == 0) return n_total == 0 ? MSN_OK : MSN_ERR_SIZE;
    if (!offsets && n_total % num_segments != 0) return MSN_ERR_SIZE;

    LeafSet ls;
    leaf_set(leaf, &ls);
    const int tile = 2 * k * msn::kBlockThreads;    // 2k keys per lane in a workgroup
    const int wave_tile = 2 * k * msn::kWave;
    int lane_max = ls.lane_max, wave_max = wave_tile, block_max = tile, grid = 0;
    if (tuning) {
        if (tuning->seg_lane_max) lane_max = tuning->seg_lane_max;
        if (tuning->seg_wave_max) wave_max = tuning->seg_wave_max;
        if (tuning->seg_block_max) block_max = tuning->seg_block_max;
        grid = tuning->seg_grid;
        if (lane_max < 0 || lane_max > k || wave_max < lane_max || wave_max > wave_tile ||
            block_max < wave_max || block_max > tile || grid < 0)
            return MSN_ERR_CONFIG;
    }
    if (n_total == 0) return MSN_OK;
    if (!keys_in || !keys_out) return MSN_ERR_NULL;
    if (misaligned(keys_in) || misaligned(keys_out) || misaligned(vals_in) || misaligned(vals_out) ||
        misaligned(ws) || misaligned(offsets))
        return MSN_ERR_UNSUPPORTED;
    if (bad_overlap(keys_in, keys_out, n_total) || bad_overlap(vals_in, vals_out, n_total) ||
        (vals_out && (bad_overlap(keys_out, vals_out, n_total) || keys_out == (void*)vals_out)) ||
        any_overlap(keys_in, vals_out, n_total) || any_overlap(vals_in, keys_out, n_total) ||
        ranges_overlap(offsets, num_segments + 1, keys_out, n_total) ||
        ranges_overlap(offsets, num_segments + 1, vals_out, n_total))
        return MSN_ERR_SIZE;
    const int vmode = argsort ? msn::kArg : vals_in ? msn::kVals : msn::kNoVals;
    const size_t need = msn::seg_ws_bytes(n_total, num_segments, vmode != msn::kNoVals);
    if (!ws || ws_bytes < need) return MSN_ERR_WORKSPACE;
    msn::SegArgs a{static_cast<const uint32_t*>(keys_in),
                   vals_in,
                   static_cast<uint32_t*>(keys_out),
                   vals_out,
                   offsets,
                   num_segments,
                   n_total,
                   dtype,
                   k,
                   vmode,
                   lane_max,
                   wave_max,
                   block_max,
                   grid,
                   ws,
                   ws_bytes,
                   static_cast<hipStream_t>(stream)};
    a.debug_check = (flags & MSN_DEBUG_CHECK) != 0;
    a.net = ls.net;
    a.set_mask = ls.sizes;
    return msn::launch_segmented(a);
}

int msn_segmented_status_offset(int64_t n_total, int64_t num_segments, int pairs,
                                size_t* offset) {
    if (!offset) return MSN_ERR_NULL;
    if (n_total < 0 || n_total > kMaxN || num_segments < 0 || num_segments > kMaxN)
        return MSN_ERR_SIZE;
    *offset = msn::seg_status_offset(n_total, num_segments, pairs != 0);
    return MSN_OK;
}

int msn_merge_path_split(const void* a, int64_t la, const void* b, int64_t lb,
                         const int32_t* diags, int32_t* out, int64_t count, int dtype,
                         void* stream) {
    if (!valid_dtype(dtype)) return MSN_ERR_DTYPE;
    if (la < 0 || lb < 0 || la + lb > kMaxN || count < 0 || count > kMaxN) return MSN_ERR_SIZE;
    if (count == 0) return MSN_OK;
    if ((la > 0 && !a) || (lb > 0 && !b) || !diags || !out) return MSN_ERR_NULL;
    if (misaligned(a) || misaligned(b) || misaligned(diags) || misaligned(out))
        return MSN_ERR_UNSUPPORTED;
    if (ranges_overlap(out, count, a, la) || ranges_overlap(out, count, b, lb) ||
        ranges_overlap(out, count, diags, count) && out != diags)
        return MSN_ERR_SIZE;
    return msn::launch_merge_path_split(static_cast<const uint32_t*>(a), la,
                                        static_cast<const uint32_t*>(b), lb, diags, out, count,
                                        dtype, static_cast<hipStream_t>(stream));
}

int msn_copy_words(const void* src, void* dst, int64_t n, void* stream) {
    if (n < 0) return MSN_ERR_SIZE;
    if (n == 0) return MSN_OK;
    if (!src || !dst) return MSN_ERR_NULL;
    if (misaligned(src) || misaligned(dst)) return MSN_ERR_UNSUPPORTED;
    if (any_overlap(src, dst, n)) return MSN_ERR_SIZE;
    return msn::launch_copy(static_cast<const uint32_t*>(src), static_cast<uint32_t*>(dst), n,
                            static_cast<hipStream_t>(stream));
}

int msn_sort_backward(const float* grad_out, const int32_t* perm, float* grad_in, int64_t rows,
                      int64_t cols, void* stream) {
    if (rows < 0 || cols < 0 || cols > kMaxN || (cols > 0 && rows > kMaxN / cols))
        return MSN_ERR_SIZE;
    if (rows == 0 || cols == 0) return MSN_OK;
    if (!grad_out || !perm || !grad_in) return MSN_ERR_NULL;
    if (misaligned(grad_out) || misaligned(perm) || misaligned(grad_in))
        return MSN_ERR_UNSUPPORTED;
    if (bad_overlap(grad_out, grad_in, rows * cols) || (const void*)grad_out == (void*)grad_in)
        return MSN_ERR_SIZE;
    return msn::launch_backward(grad_out, perm, grad_in, rows, cols,
                                static_cast<hipStream_t>(stream));
}

}  // extern "C"
