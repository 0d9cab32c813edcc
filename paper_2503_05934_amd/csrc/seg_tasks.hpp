// Work units shared by the batched sort and the quick sort: one lane, one
// wavefront or one workgroup sorting a subarray of a larger array, and one
// workgroup merge-sorting a long subarray through global memory.  Each is
// Algorithm 1 of the paper (Sec. 3) applied to the subarray: networks at the
// leaves, then merges.
#pragma once

#include "block_tile.hpp"

namespace msn {

constexpr int kSegMergeKPT = 16;                               // keys per thread, big merges
constexpr int kSegMergeTile = kSegMergeKPT * kBlockThreads;    // 8192 outputs per step
constexpr int kSegBoundWords = kBlockThreads + 4;

// LDS words of one merge tile of t outputs (keys or values): the tile, the
// two runs' sentinels and a dummy slot, padded.
__host__ __device__ constexpr int seg_merge_words(int t) {
    return lds_words<uint32_t>(t + 2 * (t / kBlockThreads) + 1);
}


// ------------------------------------------------------------ lane tasks ---
// One lane sorts a subarray of len <= K keys with one network: the network
// of size len when the configured set holds it (bit len of set_mask), else
// the family's group procedure on the padded keys.
template <int DT, int K, bool STABLE, int VM, int NET>
__device__ __forceinline__ void lane_task(const uint32_t* kin, const uint32_t* vin,
                                          uint32_t* kout, uint32_t* vout, uint32_t off,
                                          int len, uint32_t set_mask) {
    using T = typename TileTraits<DT, K, STABLE>::T;
    uint32_t raw[K], pv[K];
    T v[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const bool live = j < len;
        raw[j] = live ? kin[off + j] : 0u;
        if constexpr (VM == kVals) pv[j] = live ? vin[off + j] : 0u;
        if constexpr (STABLE)
            v[j] = live ? comp_make(ord_key<DT>(raw[j]), (uint32_t)j) : kCompMax;
        else
            v[j] = live ? ord_key<DT>(raw[j]) : 0xffffffffu;
    }
    lane_networks<T, K, NET>(v, len, set_mask);
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j >= len) break;
        if constexpr (!STABLE) {
            kout[off + j] = unord_key<DT>(v[j]);
        } else {
            const uint32_t tag = comp_pos(v[j]);
            uint32_t key = unord_key<DT>(comp_ord(v[j]));
            uint32_t val = tag;
#pragma unroll
            for (int q = 0; q < K; ++q) {
                if constexpr (DT == kF32) key = (tag == (uint32_t)q) ? raw[q] : key;
                if constexpr (VM == kVals) val = (tag == (uint32_t)q) ? pv[q] : val;
            }
            kout[off + j] = key;
            if constexpr (VM != kNoVals) vout[off + j] = val;
        }
    }
}

// ------------------------------------------------------------ wave tasks ---
// One wavefront sorts one segment of at most 64*KPL keys (KPL = 2K keys per
// lane).  wst: this wave's private LDS staging (2 * 64 * KPL words) for
// position gathers.
template <int DT, int K, bool STABLE, int VM, int NET>
__device__ __forceinline__ void wave_task(const uint32_t* kin, const uint32_t* vin,
                                          uint32_t* kout, uint32_t* vout, uint32_t off, int len,
                                          uint32_t* wst) {
    using T = typename TileTraits<DT, K, STABLE>::T;
    constexpr int KPL = keys_per_lane<K>();
    const int lane = threadIdx.x & (kWave - 1);
    const int first = lane * KPL;
    T v[KPL];
#pragma unroll
    for (int j = 0; j < KPL; ++j) {
        const bool live = first + j < len;
        const uint32_t x = live ? kin[off + first + j] : 0u;
        if constexpr (STABLE)
            v[j] = live ? comp_make(ord_key<DT>(x), (uint32_t)(first + j)) : kCompMax;
        else
            v[j] = live ? ord_key<DT>(x) : 0xffffffffu;
    }
    {
        T lo[K], hi[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            lo[j] = v[j];
            hi[j] = v[K + j];
        }
        leaf_group<T, K, NET>(lo);
        leaf_group<T, K, NET>(hi);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            v[j] = lo[j];
            v[K + j] = hi[j];
        }
    }
    lane_merge_halves<T, KPL>(v);
    wave_merge<T, KPL>(v, lane);
    if constexpr (!STABLE) {
#pragma unroll
        for (int j = 0; j < KPL; ++j)
            if (first + j < len) kout[off + first + j] = unord_key<DT>(v[j]);
    } else {
        constexpr bool kNeedBits = DT == kF32;
        constexpr bool kNeedVals = VM == kVals;
        uint32_t* sbits = wst;
        uint32_t* svals = wst + kWave * KPL;
        if constexpr (kNeedBits || kNeedVals) {
            for (int i = lane; i < len; i += kWave) {
                if constexpr (kNeedBits) sbits[i] = kin[off + i];
                if constexpr (kNeedVals) svals[i] = vin[off + i];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
#pragma unroll
        for (int j = 0; j < KPL; ++j) {
            if (first + j < len) {
                const uint32_t tag = comp_pos(v[j]);
                uint32_t key;
                if constexpr (kNeedBits) key = sbits[tag];
                else key = unord_key<DT>(comp_ord(v[j]));
                kout[off + first + j] = key;
                if constexpr (VM == kVals) vout[off + first + j] = svals[tag];
                if constexpr (VM == kArg) vout[off + first + j] = tag;
            }
        }
    }
}

// ------------------------------------------------------------- big tasks ---
// Stable merge-path split in global memory (same rule as the flat passes).
template <int DT>
__device__ __forceinline__ int corank_global(const uint32_t* A, int la, const uint32_t* B, int lb,
                                             int d) {
    int lo = d > lb ? d - lb : 0;
    int hi = d < la ? d : la;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (!(ord_key<DT>(B[d - 1 - mid]) < ord_key<DT>(A[mid])))
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// One output tile of a merge pass, by one workgroup: outputs [d0, d1) of the
// stable merge of A = ks[base, base + la) and B = ks[base + la, base + la +
// lb) (segment positions), A contributing [i0, i1); they land at kd[base +
// d0 ...].  sk/sv: LDS of seg_merge_words(KPT * kBlockThreads) words each.
template <int DT, bool VALS, int KPT>
__device__ __forceinline__ void seg_merge_tile(const uint32_t* ks, const uint32_t* vs,
                                               uint32_t* kd, uint32_t* vd, int base, int la,
                                               int d0, int d1, int i0, int i1, uint32_t* sk,
                                               uint32_t* sv) {
    const int tid = threadIdx.x;
    const int na = i1 - i0;
    const int cnt = d1 - d0;
    const int nb = cnt - na;
    const int j0 = d0 - i0;
    if constexpr (!VALS && DT != kF32) {
        // integer keys alone: both pieces closed by KPT maxima in LDS (B
        // starts KPT past A's end), so the sequential merge checks no bounds;
        // equal keys may come from either piece, which keys alone cannot show
        using Key = std::conditional_t<DT == kI32, int32_t, uint32_t>;
        constexpr Key kMax = DT == kI32 ? (Key)0x7fffffff : (Key)0xffffffffu;
        constexpr int kDummy = KPT * kBlockThreads + 2 * KPT;
        Key* s = reinterpret_cast<Key*>(sk);
        const int b0 = na + KPT;
        Key r[KPT];
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const int x = min(tid + q * kBlockThreads, cnt - 1);
            r[q] = (Key)ks[x < na ? base + i0 + x : base + la + j0 + (x - na)];
        }
        // A's piece ends at or below the start of B's (runs already in
        // order, as in a presorted array): the merge is the concatenation
        // the loads just read, stored as it stands
        const int pa = max(base + i1 - 1, base);                 // A's last (when na > 0)
        const int pb = min(base + la + j0, base + la + nb + j0 - 1);  // B's first (nb > 0)
        const bool concat = na == 0 || nb == 0 || !((Key)ks[pb] < (Key)ks[pa]);
        if (__builtin_amdgcn_readfirstlane((int)concat)) {
            uint32_t* kr = kd + base + d0;
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                const int x = tid + q * kBlockThreads;
                if (x < cnt) kr[x] = (uint32_t)r[q];
            }
            __syncthreads();  // as the merge path ends: callers reuse the LDS after it
            return;
        }
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const int x = tid + q * kBlockThreads;
            s[lds_idx<Key>(x < na ? x : (x < cnt ? x + KPT : kDummy))] = r[q];
        }
        if (tid < KPT) {
            s[lds_idx<Key>(na + tid)] = kMax;
            s[lds_idx<Key>(b0 + nb + tid)] = kMax;
        }
        __syncthreads();
        const int d = tid * KPT;
        Key o[KPT];
        if (d < cnt) {
            const int i = corank_lds(s, 0, na, b0, nb, d, PlainLess{});
            serial_merge_closed<Key, KPT>(s, i, b0 + d - i, o);
        }
        __syncthreads();
        if (d < cnt) {
#pragma unroll
            for (int k = 0; k < KPT; ++k) {
                const int e = d + k;
                if (e < cnt) sk[e + (e >> 5)] = (uint32_t)o[k];
            }
        }
        __syncthreads();
        uint32_t* kr = kd + base + d0;
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const int e = tid + q * kBlockThreads;
            if (e < cnt) kr[e] = sk[e + (e >> 5)];
        }
        __syncthreads();
        return;
    }
    {
        uint32_t rk[KPT], rv[KPT];
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const int x = min(tid + q * kBlockThreads, cnt - 1);
            const int src = x < na ? base + i0 + x : base + la + j0 + (x - na);
            rk[q] = ks[src];
            if constexpr (VALS) rv[q] = vs[src];
        }
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const int x = tid + q * kBlockThreads;
            if (x < cnt) {
                sk[lds_idx<uint32_t>(x)] = rk[q];
                if constexpr (VALS) sv[lds_idx<uint32_t>(x)] = rv[q];
            }
        }
    }
    __syncthreads();
    const int d = tid * KPT;
    uint32_t o[KPT], ov[KPT];
    if (d < cnt) {
        const int i = corank_lds(sk, 0, na, na, nb, d, OrdLess<DT>{});
        int srcpos[KPT];
        serial_merge<uint32_t, KPT, VALS>(sk, 0, na, na, nb, i, d - i, cnt - 1, o, srcpos,
                                          OrdLess<DT>{});
        if constexpr (VALS) {
#pragma unroll
            for (int k = 0; k < KPT; ++k) ov[k] = sv[lds_idx<uint32_t>(srcpos[k])];
        }
    }
    // stage the outputs (a spare word every 32) and store them as rows of
    // consecutive words, so that every store instruction is coalesced
    __syncthreads();
    if (d < cnt) {
#pragma unroll
        for (int k = 0; k < KPT; ++k) {
            const int e = d + k;
            if (e < cnt) {
                sk[e + (e >> 5)] = o[k];
                if constexpr (VALS) sv[e + (e >> 5)] = ov[k];
            }
        }
    }
    __syncthreads();
    uint32_t* kr = kd + base + d0;
    uint32_t* vr = VALS ? vd + base + d0 : nullptr;
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
        const int e = tid + q * kBlockThreads;
        if (e < cnt) {
            kr[e] = sk[e + (e >> 5)];
            if constexpr (VALS) vr[e] = sv[e + (e >> 5)];
        }
    }
    __syncthreads();
}

// One merge pass over a whole segment by one workgroup: runs of L become
// runs of 2L, kSegMergeTile outputs per step.
template <int DT, bool VALS>
__device__ void wg_merge_pass(const uint32_t* ks, const uint32_t* vs, uint32_t* kd, uint32_t* vd,
                              int len, int L, void* smem) {
    int32_t* sb = reinterpret_cast<int32_t*>(smem);
    uint32_t* sk = reinterpret_cast<uint32_t*>(sb + kSegBoundWords);
    uint32_t* sv = sk + seg_merge_words(kSegMergeTile);
    const int tid = threadIdx.x;
    const int ntiles = (len + kSegMergeTile - 1) / kSegMergeTile;
    for (int t0 = 0; t0 < ntiles; t0 += kBlockThreads) {
        const int nt = min(kBlockThreads, ntiles - t0);
        if (tid <= nt && t0 + tid < ntiles) {
            const int g0 = (t0 + tid) * kSegMergeTile;
            const int base = g0 & ~(2 * L - 1);
            const int la = min(L, len - base);
            const int lb = min(L, len - base - la);
            sb[tid] = corank_global<DT>(ks + base, la, ks + base + la, lb, g0 - base);
        }
        __syncthreads();
        for (int t = t0; t < t0 + nt; ++t) {
            const int g0 = t * kSegMergeTile;
            const int base = g0 & ~(2 * L - 1);
            const int la = min(L, len - base);
            const int lb = min(L, len - base - la);
            const int plen = la + lb;
            const int d0 = g0 - base;
            const int d1 = min(d0 + kSegMergeTile, plen);
            const int i0 = sb[t - t0];
            const int i1 = (d1 == plen) ? la : sb[t + 1 - t0];
            seg_merge_tile<DT, VALS, kSegMergeKPT>(ks, vs, kd, vd, base, la, d0, d1, i0, i1, sk,
                                                   sv);
        }
    }
}

// A keys-only tile that is already in order (a presorted array, or a piece
// of one) is copied as it stands.  Every thread checks its own keys and its
// first key against the previous thread's last (one LDS word per thread),
// and the workgroup agrees through one barrier-or.  Returns whether it
// copied; on false the caller sorts the tile (reading it again, from L2).
// The keys live only here, so the sort that may follow keeps its registers.
template <int DT, int KPL>
__device__ __forceinline__ bool copy_if_in_order(const uint32_t* kin, uint32_t* kout, int nv,
                                              void* smem) {
    uint32_t* edge = reinterpret_cast<uint32_t*>(smem);
    const int tid = threadIdx.x;
    const int first = tid * KPL;
    uint32_t x[KPL];
    if (first + KPL <= nv) {
#pragma unroll
        for (int q = 0; q < KPL / 4; ++q) {
            const uint4 w = ld4(kin + first + 4 * q);
            x[4 * q + 0] = w.x;
            x[4 * q + 1] = w.y;
            x[4 * q + 2] = w.z;
            x[4 * q + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < KPL; ++j) x[j] = (first + j < nv) ? kin[first + j] : 0u;
    }
    int bad = 0;
#pragma unroll
    for (int j = 0; j + 1 < KPL; ++j)
        bad |= (int)((first + j + 1 < nv) & (ord_key<DT>(x[j + 1]) < ord_key<DT>(x[j])));
    if (first < nv) edge[tid] = ord_key<DT>(first + KPL <= nv ? x[KPL - 1] : kin[nv - 1]);
    __syncthreads();
    if (tid > 0 && first < nv) bad |= (int)(ord_key<DT>(x[0]) < edge[tid - 1]);
    // the same for every thread: a uniform branch for the compiler too
    if (__builtin_amdgcn_readfirstlane(__syncthreads_or(bad))) return false;
    if (first + KPL <= nv) {
#pragma unroll
        for (int q = 0; q < KPL / 4; ++q)
            st4(kout + first + 4 * q, x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < KPL; ++j)
            if (first + j < nv) kout[first + j] = x[j];
    }
    return true;
}

// NETS: the network family of the tiles (kNetNone: merges from runs of one
// key).
template <int DT, int K, bool STABLE, int VM, int NETS>
__device__ void big_task(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                         uint32_t* wk, uint32_t* wv, uint32_t off, int len, void* smem) {
    constexpr int kTile = TileTraits<DT, K, STABLE>::kTile;
    const int chunks = (len + kTile - 1) / kTile;
    int passes = 0;
    while ((1 << passes) < chunks) ++passes;
    uint32_t* kb[2] = {kout + off, wk + off};
    uint32_t* vb[2] = {VM != kNoVals ? vout + off : nullptr, VM != kNoVals ? wv + off : nullptr};
    int cur = passes & 1;
    for (int c = 0; c < chunks; ++c) {
        const int nv = min(kTile, len - c * kTile);
        block_sort_tile<DT, K, STABLE, VM, 0, false, false, NETS>(kin + off + c * kTile,
                                           VM == kVals ? vin + off + c * kTile : nullptr,
                                           kb[cur] + c * kTile,
                                           VM != kNoVals ? vb[cur] + c * kTile : nullptr, nv,
                                           (uint32_t)(c * kTile), smem);
        __syncthreads();
    }
    for (int p = 0; p < passes; ++p) {
        const int L = kTile << p;
        wg_merge_pass<DT, VM != kNoVals>(kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], len, L, smem);
        cur ^= 1;
    }
}

// ------------------------------------------------ LDS of the work units ---
template <int DT, int K, bool STABLE, int VM>
struct SegTraits {
    static constexpr size_t kTileLds = TileTraits<DT, K, STABLE>::kLdsBytes;
    // per-wave staging of the position gathers: stable sorts only
    static constexpr size_t kWaveLds =
        STABLE ? (size_t)(kBlockThreads / kWave) * 2 * kWave * keys_per_lane<K>() * 4 : 0;
    static constexpr size_t kMergeLds =
        (size_t)kSegBoundWords * 4 +
        (size_t)seg_merge_words(kSegMergeTile) * 4 * (VM != kNoVals ? 2 : 1);
    static constexpr size_t kLds = kTileLds > kWaveLds
                                       ? (kTileLds > kMergeLds ? kTileLds : kMergeLds)
                                       : (kWaveLds > kMergeLds ? kWaveLds : kMergeLds);
};


}  // namespace msn
