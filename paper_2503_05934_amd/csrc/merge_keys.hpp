// Keys-only global merge pass for integer keys: the kernel that dominates a
// flat sort of uint32 / int32 keys.  Kept in its own file so that its
// source (with device.hpp) identifies the code its profiles were taken on.
#pragma once

#include <algorithm>
#include <type_traits>

#include "device.hpp"

namespace msn {

// Keys-only merge pass for integer keys (uint32 / int32).  Same tiling as
// k_merge, but in LDS each run slice is followed by KPT copies of the
// largest key, so the sequential merge runs without bounds checks: a side
// that is used up offers the maximum, which is taken only when the other
// side's key is the maximum too -- the same value either way.
template <int DT, int KPT>
__global__ __launch_bounds__(kMergeThreads) void k_merge_keys(const uint32_t* __restrict__ kin,
                                                              uint32_t* __restrict__ kout,
                                                              const int32_t* __restrict__ part,
                                                              int64_t n, int64_t L, int vec,
                                                              uint32_t* __restrict__ samp_first,
                                                              uint32_t* __restrict__ samp_last,
                                                              const int* __restrict__ skip) {
    static_assert(DT == kU32 || DT == kI32, "integer keys only");
    if (*skip) return;  // the input is already sorted
    using Key = std::conditional_t<DT == kI32, int32_t, uint32_t>;
    constexpr Key kMax = DT == kI32 ? (Key)0x7fffffff : (Key)0xffffffffu;
    constexpr int MT = KPT * kMergeThreads;
    extern __shared__ __align__(16) unsigned char smem[];
    Key* s = reinterpret_cast<Key*>(smem);

    const int t = blockIdx.x;
    const int64_t g0 = (int64_t)t * MT;
    const int64_t base = g0 & ~(2 * L - 1);
    const int64_t la = (n - base) < L ? (n - base) : L;
    const int64_t rest = n - base - la;
    const int64_t lb = rest < L ? rest : L;
    const int64_t plen = la + lb;
    const int64_t d0 = g0 - base;
    const int64_t d1 = (d0 + MT) < plen ? (d0 + MT) : plen;
    const int64_t i0 = part[t];
    const int64_t i1 = (d1 == plen) ? la : (int64_t)part[t + 1];
    const int na = (int)(i1 - i0);
    const int cnt = (int)(d1 - d0);
    const int nb = cnt - na;
    const int64_t j0 = d0 - i0;
    const int b0 = na + KPT;  // LDS position of B's first key

    {
        // element x of the tile lives at A + x (x < na) or at B + (x - na)
        const uint32_t* pa_src = kin + base + i0;
        const uint32_t* pb_src = kin + base + la + j0 - na;
        constexpr int kDummy = MT + 2 * KPT;  // absorbs the writes of lanes past the tile
        Key r[KPT];
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const int x = min((int)threadIdx.x + q * kMergeThreads, cnt - 1);
            r[q] = (Key)(x < na ? pa_src : pb_src)[x];
        }
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const int x = (int)threadIdx.x + q * kMergeThreads;
            const int pos = x < na ? x : (x < cnt ? x + KPT : kDummy);
            s[lds_idx<Key>(pos)] = r[q];
        }
        if (threadIdx.x < KPT) {
            s[lds_idx<Key>(na + threadIdx.x)] = kMax;
            s[lds_idx<Key>(b0 + nb + threadIdx.x)] = kMax;
        }
    }
    __syncthreads();

    const int d = threadIdx.x * KPT;
    uint32_t o[KPT];
    if (d < cnt) {
        int pa = corank_lds(s, 0, na, b0, nb, d, PlainLess{});
        // pa + pb grows by one per output, so pb = (b0 + d + k) - pa after k outputs
        const int sum0 = b0 + d;
        Key a = s[lds_idx<Key>(pa)];
        Key b = s[lds_idx<Key>(sum0 - pa)];
#pragma unroll
        for (int k = 0; k < KPT; ++k) {
            const bool take_a = !(b < a);
            o[k] = (uint32_t)(take_a ? a : b);
            pa += take_a ? 1 : 0;
            const int p = take_a ? pa : sum0 + k + 1 - pa;
            const Key x = s[(p + (p >> 5))];
            a = take_a ? x : a;
            b = take_a ? b : x;
        }
    }
    // Stage the outputs in LDS (one spare word every 16 keeps the per-thread
    // rows on distinct banks) and write them out as contiguous 16-byte
    // chunks: lane l of a wave stores bytes [16 l, 16 l + 16) of a 1 KiB run.
    uint32_t* st = reinterpret_cast<uint32_t*>(smem);
    __syncthreads();
    if (d < cnt) {
#pragma unroll
        for (int k = 0; k < KPT; ++k) st[(d + k) + ((d + k) >> 4)] = o[k];
    }
    __syncthreads();
    uint32_t* ko = kout + g0;
#pragma unroll
    for (int q = 0; q < KPT / 4; ++q) {
        const int e = 4 * ((int)threadIdx.x + q * kMergeThreads);
        const int pe = e + (e >> 4);
        if (vec && e + 4 <= cnt) {
            *reinterpret_cast<uint4*>(ko + e) = make_uint4(st[pe], st[pe + 1], st[pe + 2], st[pe + 3]);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (e + k < cnt) ko[e + k] = st[pe + k];
        }
    }
    // Chunk samples for the next pass's splits: the tile's first and last key
    // of every chunk, written by the first wavefront as two contiguous runs.
    constexpr int kChunks = MT / kSampleChunk;
    static_assert(2 * kChunks <= kMergeThreads, "one thread per sample");
    const int c = (int)threadIdx.x;
    if (c < kChunks) {
        const int e = c * kSampleChunk;
        if (e < cnt) samp_first[g0 / kSampleChunk + c] = st[e + (e >> 4)];
    } else if (c < 2 * kChunks) {
        const int e = (c - kChunks) * kSampleChunk + kSampleChunk - 1;
        if (e < cnt) samp_last[g0 / kSampleChunk + (c - kChunks)] = st[e + (e >> 4)];
    }
}

}  // namespace msn
