// Quick sort with sorting-network base cases (paper Sec. 3, Algorithm 2):
// a subarray whose size is a leaf size goes to a network; otherwise its pivot
// is the median of its first, middle and last keys, the subarray is
// partitioned around it and both sides are sorted the same way.
//
// On the GPU the recursion runs level by level.  Round r works through two
// lists of subarrays ("items") of the whole array in one launch (the first
// workgroups take the partition list, the others the leaf list) and builds
// the lists of round r + 1:
//   partition list:
//     partition item (longer than one block-sort tile): cut into claim
//       tiles, one workgroup each: 8192-key chunks once the round's items
//       are down to about a quarter of kQOnePassMax keys, 65,536-key
//       super-tiles in the rounds before (the host picks the size per
//       round).  A tile
//       counts its keys below and above the item's pivot, claims room for
//       them with one 64-bit atomic on the item (smaller keys fill the
//       subarray from its left end, larger keys from its right end),
//       compacts them in LDS and writes them to the other buffer; a
//       super-tile counts all its chunks first and reads them again to
//       scatter them.  The tile that finishes the item last appends the
//       item's children: the smaller side, the larger side, and the keys
//       equal to the pivot, which are already in their final place (a
//       three-way split; the paper splits in two, which for equal keys only
//       moves them to one side or the other);
//     fill item: the keys equal to a pivot, written to the output;
//   leaf list:
//     leaf item (at most one block-sort tile): sorted by one workgroup into
//       the output -- a subarray of at most K keys by one lane with one
//       K-key network, a longer one by the block sort (K-key networks in
//       every lane, then merges), an already ordered one copied as it stands;
//     big item: only in the last round, when a subarray is still longer than
//       one tile (inputs that defeat the median of three): one workgroup
//       merge-sorts it through global memory.
// Partitions alternate between the workspace and the output array, both at
// the item's own positions, so finished subarrays are never moved again.
// The early rounds of large sorts claim per super-tile rather than per
// chunk: the claims queue behind each other on their item, and the first
// round of a 2^28-key array would otherwise make 65,536 of them on one
// address.  Once the items are short enough to be many, claims spread over
// their addresses and each chunk is read once.  No launch reads
// anything on the host.  Integer keys only: the partition is not stable, and
// float keys that compare equal (-0 and +0, NaNs) must keep their input
// order.
#include <algorithm>
#include <cstdio>

#include "seg_tasks.hpp"

namespace msn {

enum QKind : uint32_t { kQPart = 0, kQLeaf = 1, kQFill = 2, kQBig = 3 };

// One item of a list.  `claimed` holds the keys placed so far: those below
// the pivot in its low word, those above it in its high word.
struct QItem {
    uint32_t start, len, kind;
    uint32_t pivot;  // fill items: the key bits to write
    uint32_t tile0;  // partition lists: the item's first super-tile in its round
    uint32_t done;   // partition items: super-tiles finished
    unsigned long long claimed;
};
static_assert(sizeof(QItem) == 32, "item layout");

// List header: items << 32 | super-tiles, advanced by one atomic per append,
// so items' first super-tiles grow with their index.
struct QList {
    unsigned long long packed;
    uint32_t status;  // set if an append found the list full
    uint32_t pad[61];
};
static_assert(sizeof(QList) == 256, "list header");

constexpr int kQKeysPerThread = 16;
constexpr int kQChunk = kQKeysPerThread * kBlockThreads;  // 8192 keys per pass step
constexpr int kQChunks = 8;
constexpr int kQSuper = kQChunk * kQChunks;  // keys per claim of a large sort: 65,536
// Sorts of at most this many keys, and the rounds of larger ones whose items
// hold about a quarter as many keys or fewer (n / 2^round, for
// median-of-three splits), claim room per 8192-key chunk and read their keys
// once; earlier rounds claim per super-tile, counting and scattering in two
// reads.  Claims are device-scope atomics that queue behind each other on
// their item: the first round of a 2^28-key sort in chunks makes 65,536 of
// them (claims and completions) on one item, about 3 ms, against about
// 0.6 ms of traffic.
constexpr int64_t kQOnePassMax = 1ll << 23;

__device__ __forceinline__ QItem* q_items(QList* l) { return reinterpret_cast<QItem*>(l + 1); }

// Work units of an item: claim tiles of claim_keys keys for partitions,
// super-tiles for fills.
__device__ __forceinline__ uint32_t q_tiles(uint32_t kind, uint32_t len, uint32_t claim_keys) {
    const uint32_t t = kind == kQPart ? claim_keys : (uint32_t)kQSuper;
    return (len + t - 1) / t;
}

// Appends an item (one thread).
__device__ __forceinline__ void q_append(QList* l, uint32_t cap, uint32_t start, uint32_t len,
                                         uint32_t kind, uint32_t pivot, uint32_t claim_keys) {
    const unsigned long long tiles =
        (kind == kQPart || kind == kQFill) ? q_tiles(kind, len, claim_keys) : 1u;
    const unsigned long long old = atomicAdd(&l->packed, (1ull << 32) | tiles);
    const uint32_t idx = (uint32_t)(old >> 32);
    if (idx >= cap) {  // cannot happen: a list holds three children per partition
        atomicOr(&l->status, 1u);
        return;
    }
    QItem it;
    it.start = start;
    it.len = len;
    it.kind = kind;
    it.pivot = pivot;
    it.tile0 = (uint32_t)old;
    it.done = 0u;
    it.claimed = 0ull;
    q_items(l)[idx] = it;
}

// The item holding super-tile t: the largest i < count with
// items[i].tile0 <= t.  One wavefront probes 64 items per step.
__device__ __forceinline__ uint32_t q_find(const QItem* items, uint32_t count, uint32_t t) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    uint32_t lo = 0, hi = count;
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + kWave - 1) / kWave;
        const uint32_t idx = lo + lane * step;
        const bool pred = idx < hi && items[idx].tile0 <= t;
        const unsigned long long b = __ballot(pred);
        const uint32_t last = 63u - (uint32_t)__clzll(b);
        lo += last * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

// Sum of x over the workgroup's threads, two values at once.  sw: 2 *
// kBlockThreads / kWave words of LDS.  Ends with a barrier.
__device__ __forceinline__ void q_sum2(uint32_t& x, uint32_t& y, uint32_t* sw) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        x += __shfl_xor(x, d, kWave);
        y += __shfl_xor(y, d, kWave);
    }
    constexpr int kW = kBlockThreads / kWave;
    if (lane == 0) {
        sw[w] = x;
        sw[kW + w] = y;
    }
    __syncthreads();
    x = 0;
    y = 0;
#pragma unroll
    for (int i = 0; i < kW; ++i) {
        x += sw[i];
        y += sw[kW + i];
    }
    __syncthreads();
}

// Exclusive prefix sum over the workgroup's threads; *total gets the sum.
// sw: kBlockThreads / kWave words of LDS.
__device__ __forceinline__ uint32_t q_scan(uint32_t v, uint32_t* sw, uint32_t* total) {
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, kWave);
        x += lane >= d ? y : 0u;
    }
    if (lane == kWave - 1) sw[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kBlockThreads / kWave; ++i) {
        const uint32_t s = sw[i];
        before += i < w ? s : 0u;
        all += s;
    }
    *total = all;
    return before + x - v;
}

// Thread tid's keys of one chunk (positions first .. first + 15 of src).
__device__ __forceinline__ void q_load(const uint32_t* src, int first, int nv,
                                       uint32_t (&x)[kQKeysPerThread]) {
    if (first + kQKeysPerThread <= nv) {
#pragma unroll
        for (int q = 0; q < kQKeysPerThread / 4; ++q) {
            const uint4 w = ld4(src + first + 4 * q);
            x[4 * q + 0] = w.x;
            x[4 * q + 1] = w.y;
            x[4 * q + 2] = w.z;
            x[4 * q + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kQKeysPerThread; ++j) x[j] = first + j < nv ? src[first + j] : 0u;
    }
}

struct QPartRound {
    const uint32_t* cur;  // where this round's items are
    uint32_t* other;      // where partitions write
    uint32_t* out;        // the output array
    QList* lin;           // this round's partition list
    QList* lout_p;        // next round's partition list
    QList* lout_l;        // next round's leaf list
    QList* clr_p;         // the lists two rounds ahead: emptied here
    QList* clr_l;
    uint32_t cap;         // items per list
    uint32_t leaf_max;    // longest leaf item
    int final_next;       // the next round is the last: long children become big items
    uint32_t next_claim_keys;  // keys per claim tile of the next round: kQChunk or kQSuper
};

// Appends one side of a finished partition to the list its length calls for.
__device__ __forceinline__ void q_child(const QPartRound& r, uint32_t start, uint32_t len) {
    if (len == 0) return;
    if (len <= r.leaf_max) q_append(r.lout_l, r.cap, start, len, kQLeaf, 0u, r.next_claim_keys);
    else if (r.final_next) q_append(r.lout_l, r.cap, start, len, kQBig, 0u, r.next_claim_keys);
    else q_append(r.lout_p, r.cap, start, len, kQPart, 0u, r.next_claim_keys);
}

// One claim tile of partition item `it` (index sub of its claim tiles of CK
// keys: kQChunk, read once, or kQSuper, counted and then read again).  The
// claim size is a template parameter so that each kernel holds the registers
// of its own path only.
template <int DT, int CK>
__device__ void q_partition(const QPartRound& r, QItem* itp, const QItem& it, uint32_t sub,
                            uint32_t* smem) {
    const int tid = threadIdx.x;
    const uint32_t* src = r.cur + it.start;
    // median of the first, middle and last keys (Algorithm 2's MedianOfThree)
    const uint32_t ka = ord_key<DT>(src[0]);
    const uint32_t kb = ord_key<DT>(src[(it.len - 1) / 2]);
    const uint32_t kc = ord_key<DT>(src[it.len - 1]);
    const uint32_t p = max(min(ka, kb), min(max(ka, kb), kc));

    constexpr int ck = CK;
    const int s0 = (int)sub * ck;
    const int ns = min(ck, (int)it.len - s0);
    const int first = tid * kQKeysPerThread;
    uint32_t* sw = smem + kQChunk;
    __shared__ unsigned long long s_base;

    if constexpr (ck == kQChunk) {
        // one chunk per claim: read once, count, claim, compact, write
        uint32_t x[kQKeysPerThread];
        q_load(src + s0, first, ns, x);
        uint32_t l = 0, g = 0;
#pragma unroll
        for (int j = 0; j < kQKeysPerThread; ++j) {
            const bool live = first + j < ns;
            const uint32_t o = ord_key<DT>(x[j]);
            l += (live && o < p) ? 1u : 0u;
            g += (live && o > p) ? 1u : 0u;
        }
        uint32_t tot = 0;
        const uint32_t pre = q_scan(l | (g << 16), sw, &tot);
        const uint32_t TL = tot & 0xffffu, TG = tot >> 16;
        if (tid == 0)
            s_base = atomicAdd(&itp->claimed,
                               (unsigned long long)TL | ((unsigned long long)TG << 32));
        uint32_t pl = pre & 0xffffu, pg = TL + (pre >> 16);
#pragma unroll
        for (int j = 0; j < kQKeysPerThread; ++j) {
            const bool live = first + j < ns;
            const uint32_t o = ord_key<DT>(x[j]);
            if (live && o < p) smem[pl++] = x[j];
            if (live && o > p) smem[pg++] = x[j];
        }
        __syncthreads();
        const uint32_t base_l = (uint32_t)s_base, base_g = (uint32_t)(s_base >> 32);
        uint32_t* dl = r.other + it.start + base_l;
        uint32_t* dg = r.other + it.start + it.len - base_g - TG - TL;
        for (uint32_t e = tid; e < TL + TG; e += kBlockThreads) {
            if (e < TL) dl[e] = smem[e];
            else dg[e] = smem[e];
        }
        __syncthreads();  // the LDS and the scan words are reused
    } else {
        // a super-tile per claim: count, claim, then read again and scatter;
        // the first two chunks, the ones longest out of the caches by the
        // scatter, stay in registers from the count to the scatter
        const int nch = (ns + kQChunk - 1) / kQChunk;
        // pass 1: count
        uint32_t cl = 0, cg = 0;
        uint32_t x0[kQKeysPerThread], x1[kQKeysPerThread];  // chunks 0 and 1
        for (int c = 0; c < nch; ++c) {
            uint32_t x[kQKeysPerThread];
            const int nv = min(kQChunk, ns - c * kQChunk);
            q_load(src + s0 + c * kQChunk, first, nv, x);
#pragma unroll
            for (int j = 0; j < kQKeysPerThread; ++j) {
                const bool live = first + j < nv;
                const uint32_t o = ord_key<DT>(x[j]);
                cl += (live && o < p) ? 1u : 0u;
                cg += (live && o > p) ? 1u : 0u;
            }
            if (c == 0) {
#pragma unroll
                for (int j = 0; j < kQKeysPerThread; ++j) x0[j] = x[j];
            } else if (c == 1) {
#pragma unroll
                for (int j = 0; j < kQKeysPerThread; ++j) x1[j] = x[j];
            }
        }
        q_sum2(cl, cg, sw);
        if (tid == 0)
            s_base = atomicAdd(&itp->claimed,
                               (unsigned long long)cl | ((unsigned long long)cg << 32));
        __syncthreads();
        uint32_t run_l = (uint32_t)s_base;           // smaller keys placed before this chunk
        uint32_t run_g = (uint32_t)(s_base >> 32);   // larger keys placed after it

        // pass 2: compact and write each chunk; the two held chunks, then the
        // others read again
        auto scatter = [&](const uint32_t (&x)[kQKeysPerThread], int nv) {
            uint32_t l = 0, g = 0;
#pragma unroll
            for (int j = 0; j < kQKeysPerThread; ++j) {
                const bool live = first + j < nv;
                const uint32_t o = ord_key<DT>(x[j]);
                l += (live && o < p) ? 1u : 0u;
                g += (live && o > p) ? 1u : 0u;
            }
            // chunk counts stay below 2^16: one scan carries both
            uint32_t tot = 0;
            const uint32_t pre = q_scan(l | (g << 16), sw, &tot);
            const uint32_t TL = tot & 0xffffu, TG = tot >> 16;
            // stage: smaller keys at [0, TL), larger keys at [TL, TL + TG)
            uint32_t pl = pre & 0xffffu, pg = TL + (pre >> 16);
#pragma unroll
            for (int j = 0; j < kQKeysPerThread; ++j) {
                const bool live = first + j < nv;
                const uint32_t o = ord_key<DT>(x[j]);
                if (live && o < p) smem[pl++] = x[j];
                if (live && o > p) smem[pg++] = x[j];
            }
            __syncthreads();
            uint32_t* dl = r.other + it.start + run_l;
            // dg[TL + j] is larger key j: they end where the previous chunk's began
            uint32_t* dg = r.other + it.start + it.len - run_g - TG - TL;
            for (uint32_t e = tid; e < TL + TG; e += kBlockThreads) {
                if (e < TL) dl[e] = smem[e];
                else dg[e] = smem[e];
            }
            run_l += TL;
            run_g += TG;
            __syncthreads();  // the LDS and the scan words are reused
        };
        scatter(x0, min(kQChunk, ns));
        if (nch >= 2) scatter(x1, min(kQChunk, ns - kQChunk));
        for (int c = 2; c < nch; ++c) {
            uint32_t x[kQKeysPerThread];
            const int nv = min(kQChunk, ns - c * kQChunk);
            q_load(src + s0 + c * kQChunk, first, nv, x);
            scatter(x, nv);
        }
    }
    if (tid == 0) {
        // No fence: the children are read by later launches only, and a
        // device-scope release here would write back the L2 for every
        // claim tile.  This tile's claim returned before this increment.
        if (atomicAdd(&itp->done, 1u) + 1u == q_tiles(kQPart, it.len, (uint32_t)CK)) {
            // every tile has claimed its room: the totals are final
            const unsigned long long c = atomicAdd(&itp->claimed, 0ull);
            const uint32_t nl = (uint32_t)c, ng = (uint32_t)(c >> 32);
            const uint32_t ne = it.len - nl - ng;
            q_child(r, it.start, nl);
            q_child(r, it.start + it.len - ng, ng);
            if (ne)
                q_append(r.lout_p, r.cap, it.start + nl, ne, kQFill, unord_key<DT>(p),
                         r.next_claim_keys);
        }
    }
}

// LDS words of the partition work: one chunk and the scan's per-wave words.
constexpr int kQPartWords = kQChunk + 2 * kBlockThreads / kWave;

// Partition and fill items.  Workgroup b of nb takes a contiguous range of
// the round's claim tiles, so it looks its first item up once and then steps
// through the list.
template <int DT, int CK>
__device__ __forceinline__ void q_part_work(const QPartRound& r, uint32_t b, uint32_t nb,
                                            uint32_t* smem) {
    __shared__ uint32_t s_item;
    const int tid = threadIdx.x;
    if (b == 0 && tid == 0) {
        r.clr_p->packed = 0ull;
        r.clr_l->packed = 0ull;
    }
    const unsigned long long pk = r.lin->packed;
    const uint32_t count = (uint32_t)(pk >> 32);
    const uint32_t tiles = (uint32_t)pk;
    if (count > r.cap) return;  // an append was dropped (status set); never index past the list
    const uint32_t per = (tiles + nb - 1) / nb;
    const uint32_t t0 = b * per;
    const uint32_t t1 = min(tiles, t0 + per);
    if (t0 >= t1) return;
    QItem* items = q_items(r.lin);
    if (tid < kWave) {
        const uint32_t i = q_find(items, count, t0);
        if (tid == 0) s_item = i;
    }
    __syncthreads();
    uint32_t i = s_item;
    for (uint32_t t = t0; t < t1; ++t) {
        while (i + 1 < count && items[i + 1].tile0 <= t) ++i;
        const QItem it = items[i];
        const uint32_t sub = t - it.tile0;
        if (it.kind == kQPart) {
            q_partition<DT, CK>(r, items + i, it, sub, smem);
        } else {  // fill
            const uint32_t f0 = sub * kQSuper;
            const uint32_t nf = min((uint32_t)kQSuper, it.len - f0);
            uint32_t* d = r.out + it.start + f0;
            for (uint32_t e = 4 * tid; e < nf; e += 4 * kBlockThreads) {
                if (e + 4 <= nf) {
                    st4(d + e, it.pivot, it.pivot, it.pivot, it.pivot);
                } else {
                    for (uint32_t k = e; k < nf; ++k) d[k] = it.pivot;
                }
            }
        }
    }
}

struct QLeafRound {
    const uint32_t* cur;  // where this round's items are
    uint32_t* out;        // the output array
    uint32_t* wk;         // the workspace buffer (scratch of big items)
    QList* lin;           // this round's leaf list
    uint32_t cap;
    uint32_t set_mask;    // network sizes of the leaf set
};

// Leaf and big items, one workgroup each (workgroup b of nb).
template <int DT, int K, int NETS>
__device__ __forceinline__ void q_leaf_work(const QLeafRound& r, uint32_t b, uint32_t nb,
                                            unsigned char* smem) {
    const int tid = threadIdx.x;
    const uint32_t count = min((uint32_t)(r.lin->packed >> 32), r.cap);
    const QItem* items = q_items(r.lin);
    for (uint32_t i = b; i < count; i += nb) {
        const QItem it = items[i];
        if (it.kind == kQLeaf) {
            constexpr int KPL = TileTraits<DT, K, false>::kKPL;
            if (NETS != kNetNone && it.len <= (uint32_t)K) {
                if (tid == 0)
                    lane_task<DT, K, false, kNoVals, NETS == kNetNone ? kNetPlain : NETS>(
                        r.cur, nullptr, r.out, nullptr, it.start, (int)it.len, r.set_mask);
            } else {
                const bool done = copy_if_in_order<DT, KPL>(r.cur + it.start, r.out + it.start,
                                                            (int)it.len, smem);
                if (!__builtin_amdgcn_readfirstlane(done))
                    block_sort_tile<DT, K, false, kNoVals, 0, NETS != kNetNone, false, NETS>(
                        r.cur + it.start, nullptr, r.out + it.start, nullptr, (int)it.len, 0u,
                        smem);
            }
        } else {
            big_task<DT, K, false, kNoVals, NETS>(r.cur, nullptr, r.out, nullptr, r.wk, nullptr,
                                                  it.start, (int)it.len, smem);
        }
        __syncthreads();  // the LDS is reused
    }
}

template <int DT, int K, int NETS>
__global__ __launch_bounds__(kBlockThreads, 4) void k_qs_leaf(QLeafRound r) {
    extern __shared__ __align__(16) unsigned char smem[];
    q_leaf_work<DT, K, NETS>(r, blockIdx.x, gridDim.x, smem);
}

// One whole round: the first pb workgroups partition (claim tiles of CK
// keys), the others sort the round's leaves.  The two are independent (the
// round's leaves came from the previous round's partitions, and the
// partitions write other positions and other lists), so one launch serves
// both: the leaves overlap the partitions, and a sort of short rounds makes
// half the launches.  (Two launches per round: 10,000 keys 79.5 against
// 56.9 us, 2^28 keys 17.3 against 16.1 ms.)
template <int DT, int K, int NETS, int CK>
__global__ __launch_bounds__(kBlockThreads, 4) void k_qs_round(QPartRound rp, QLeafRound rl,
                                                               uint32_t pb) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (blockIdx.x < pb)
        q_part_work<DT, CK>(rp, blockIdx.x, pb, reinterpret_cast<uint32_t*>(smem));
    else
        q_leaf_work<DT, K, NETS>(rl, blockIdx.x - pb, gridDim.x - pb, smem);
}

// Round 0's lists: the whole array as one item (a partition item, or a leaf
// or big item when it is short or there is one round); the rest empty.
__global__ void k_qs_init(QList* p0, QList* p1, QList* p2, QList* l0, QList* l1, QList* l2,
                          uint32_t n, uint32_t leaf_max, int only_round, uint32_t claim_keys) {
    if (threadIdx.x != 0) return;
    QList* all[6] = {p0, p1, p2, l0, l1, l2};
    for (QList* l : all) {
        l->packed = 0ull;
        l->status = 0u;
    }
    if (n <= leaf_max) q_append(l0, 1u, 0u, n, kQLeaf, 0u, claim_keys);
    else if (only_round) q_append(l0, 1u, 0u, n, kQBig, 0u, claim_keys);
    else q_append(p0, 1u, 0u, n, kQPart, 0u, claim_keys);
}

// ------------------------------------------------------------------ host ---
namespace {

// Items a list can hold: three children for each partition item of the
// round before, whose subarrays are disjoint and longer than 4096 keys (the
// shortest leaf limit).
size_t q_cap(int64_t n) { return 3 * (size_t)(n / 4097) + 3; }
size_t q_list_bytes(int64_t n) { return align_up(sizeof(QList) + q_cap(n) * sizeof(QItem), 256); }

template <int DT, int K, int NETS>
constexpr size_t q_leaf_lds() {
    return SegTraits<DT, K, false, kNoVals>::kLds;
}

// Timing kinds "qs_round_00" ..: one per round index ("qs_leaf_00" for a
// sort of one round).
struct QRoundKinds {
    char round[kQuickMaxRounds][16];
    char leaf[kQuickMaxRounds][16];
    QRoundKinds() {
        for (int i = 0; i < kQuickMaxRounds; ++i) {
            snprintf(round[i], sizeof round[i], "qs_round_%02d", i);
            snprintf(leaf[i], sizeof leaf[i], "qs_leaf_%02d", i);
        }
    }
};
const QRoundKinds& q_kinds() {
    static const QRoundKinds kinds;  // initialised once, thread-safe
    return kinds;
}

template <typename Kern>
int q_grid(Kern kern, size_t lds, int* out) {
    return resident_grid(reinterpret_cast<const void*>(kern), kBlockThreads, lds, out);
}

// Claim size of round r: chunks throughout for sorts of at most kQOnePassMax
// keys; in larger ones super-tiles while the round's items (about n / 2^r
// keys each) are longer than a quarter of that, and in the first two rounds,
// whose one or two items would queue too many chunk claims each.  (Chunks
// from items of about kQOnePassMax or half of it: 2^28 keys 14.3-14.5 and
// 13.8-14.2 ms against 13.6 ms.)
int q_claim_keys(int64_t n, int r) {
    if (n <= kQOnePassMax) return kQChunk;
    return r < 2 || (r < 32 && (n >> r) > kQOnePassMax / 4) ? kQSuper : kQChunk;
}

template <int DT, int K, int NETS>
int q_run(const QuickArgs& a) {
    constexpr uint32_t kLeafMax = TileTraits<DT, K, false>::kTile;
    auto lkern = &k_qs_leaf<DT, K, NETS>;
    auto rchunk = &k_qs_round<DT, K, NETS, kQChunk>;
    auto rsuper = &k_qs_round<DT, K, NETS, kQSuper>;
    const bool any_super = a.n > kQOnePassMax;
    const size_t llds = q_leaf_lds<DT, K, NETS>();
    const size_t rlds = std::max(llds, (size_t)kQPartWords * 4);
    if (int rc = set_dynamic_lds(reinterpret_cast<const void*>(lkern), llds)) return rc;
    if (int rc = set_dynamic_lds(reinterpret_cast<const void*>(rchunk), rlds)) return rc;
    if (any_super)
        if (int rc = set_dynamic_lds(reinterpret_cast<const void*>(rsuper), rlds)) return rc;
    int lgrid = 0, cgrid = 0, sgrid = 0;
    if (int rc = q_grid(lkern, llds, &lgrid)) return rc;
    if (int rc = q_grid(rchunk, rlds, &cgrid)) return rc;
    if (any_super)
        if (int rc = q_grid(rsuper, rlds, &sgrid)) return rc;

    const int rounds =
        a.n <= kLeafMax ? 1 : a.rounds > 0 ? a.rounds : quick_rounds(a.n, kLeafMax);
    uint8_t* ws = static_cast<uint8_t*>(a.ws);
    uint32_t* wk = reinterpret_cast<uint32_t*>(ws);
    uint8_t* lb = ws + align_up((size_t)a.n * 4, 256);
    const size_t lbytes = q_list_bytes(a.n);
    QList* P[3];
    QList* L[3];
    for (int i = 0; i < 3; ++i) {
        P[i] = reinterpret_cast<QList*>(lb + i * lbytes);
        L[i] = reinterpret_cast<QList*>(lb + (3 + i) * lbytes);
    }
    {
        LaunchTimer timer("qs_init", 1, a.stream);
        hipLaunchKernelGGL(k_qs_init, dim3(1), dim3(64), 0, a.stream, P[0], P[1], P[2], L[0],
                           L[1], L[2], (uint32_t)a.n, kLeafMax, rounds == 1 ? 1 : 0,
                           (uint32_t)q_claim_keys(a.n, 0));
    }
    if (int rc = (int)hipGetLastError()) return rc;
    const QRoundKinds& kinds = q_kinds();
    const uint32_t cap = (uint32_t)q_cap(a.n);
    for (int r = 0; r < rounds; ++r) {
        const uint32_t* cur = r == 0 ? a.kin : (r & 1) ? wk : a.kout;
        if (rounds > 1) {
            const int ck = q_claim_keys(a.n, r);
            QPartRound q;
            q.cur = cur;
            q.other = (r & 1) ? a.kout : wk;
            q.out = a.kout;
            q.lin = P[r % 3];
            q.lout_p = P[(r + 1) % 3];
            q.lout_l = L[(r + 1) % 3];
            q.clr_p = P[(r + 2) % 3];
            q.clr_l = L[(r + 2) % 3];
            q.cap = cap;
            q.leaf_max = kLeafMax;
            q.final_next = r + 2 == rounds ? 1 : 0;
            q.next_claim_keys = (uint32_t)q_claim_keys(a.n, r + 1);
            // the round's partitions and leaves in one launch: partition
            // workgroups for the most claim tiles the round can hold (its
            // items are longer than a leaf, so fewer than 2 n / ck tiles),
            // capped at a resident grid, then a resident grid's worth for the
            // leaves
            const int rgrid = ck == kQChunk ? cgrid : sgrid;
            const uint32_t rpart =
                (uint32_t)std::min<int64_t>(std::max<int64_t>(1, (2 * a.n + ck - 1) / ck), rgrid);
            QLeafRound ql{cur, a.kout, wk, L[r % 3], cap, a.set_mask};
            LaunchTimer timer(kinds.round[r], a.n, a.stream);
            if (ck == kQChunk)
                hipLaunchKernelGGL(rchunk, dim3(rpart + (uint32_t)rgrid), dim3(kBlockThreads), rlds,
                                   a.stream, q, ql, rpart);
            else
                hipLaunchKernelGGL(rsuper, dim3(rpart + (uint32_t)rgrid), dim3(kBlockThreads), rlds,
                                   a.stream, q, ql, rpart);
            if (int rc = (int)hipGetLastError()) return rc;
            continue;
        }
        // a sort of one round: its one leaf or big item
        QLeafRound ql{cur, a.kout, wk, L[r % 3], cap, a.set_mask};
        LaunchTimer timer(kinds.leaf[r], a.n, a.stream);
        hipLaunchKernelGGL(lkern, dim3(lgrid), dim3(kBlockThreads), llds, a.stream, ql);
        if (int rc = (int)hipGetLastError()) return rc;
    }
    return 0;
}

template <int DT>
int q_dispatch(const QuickArgs& a) {
    if (a.nets == kNetNone) return q_run<DT, 8, kNetNone>(a);
    if (a.nets == kNetSplit)
        return a.leaf_k == 8 ? q_run<DT, 8, kNetSplit>(a) : q_run<DT, 4, kNetSplit>(a);
    return a.leaf_k == 8 ? q_run<DT, 8, kNetPlain>(a) : q_run<DT, 4, kNetPlain>(a);
}

}  // namespace

int quick_rounds(int64_t n, int64_t leaf_max) {
    if (n <= leaf_max) return 1;
    int lg = 0;
    while ((leaf_max << lg) < n) ++lg;
    return std::min(2 * lg + 8, kQuickMaxRounds);
}

size_t quick_ws_bytes(int64_t n) { return align_up((size_t)n * 4, 256) + 6 * q_list_bytes(n); }

int launch_quick(const QuickArgs& a) {
    if (a.n == 0) return 0;
    return a.dtype == kU32 ? q_dispatch<kU32>(a) : q_dispatch<kI32>(a);
}

}  // namespace msn
