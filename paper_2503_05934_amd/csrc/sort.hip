// Flat (single-array) sort: first sweep = block sort of K*1024-key tiles,
// then global merge-path passes that double the run length until one run
// remains (paper Sec. 3, Algorithm 1, run bottom-up).
#include <algorithm>
#include <mutex>

#include "block_tile.hpp"
#include "merge4.hpp"
#include "merge_keys.hpp"

namespace msn {

// ----------------------------------------------------------- first sweep ---
template <int DT, int K, bool STABLE, int VM, int SHAPE, int NETS>
__global__ __launch_bounds__((TileTraits<DT, K, STABLE, SHAPE>::kThreads),
                             (TileTraits<DT, K, STABLE, SHAPE>::kWavesPerSimd)) void k_block_sort(
    const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, int64_t n,
    uint32_t* samp_first, uint32_t* samp_last, int* sorted_flag) {
    // presumed sorted until k_runs_in_order finds two runs out of order
    if (blockIdx.x == 0 && threadIdx.x == 0) *sorted_flag = 1;
    // static LDS (gfx950 allows up to 160 KiB): its base is a compile-time
    // constant that the padded-slot address math folds away
    __shared__ __align__(16) unsigned char smem[TileTraits<DT, K, STABLE, SHAPE>::kLdsBytes];
    constexpr int kTile = TileTraits<DT, K, STABLE, SHAPE>::kTile;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int nv = (int)((n - base) < kTile ? (n - base) : kTile);
    // network tiles take the wide LDS levels and packed composites
    block_sort_tile<DT, K, STABLE, VM, SHAPE, NETS != kNetNone, NETS != kNetNone, NETS>(kin + base,
                                             VM == kVals ? vin + base : nullptr,
                                             kout + base, VM != kNoVals ? vout + base : nullptr,
                                             nv, (uint32_t)base, smem,
                                             Samples{samp_first, samp_last, base});
}

// Stable integer first sweep in two launches.  Most tiles pack (every key
// below 2^(32 - kPackPosBits), 32-bit composites): k_block_sort_packed sorts
// those with the LDS of the packed path only, so that three workgroups share
// a compute unit instead of the two that the 64-bit path's LDS allows, and
// flags every other tile; k_block_sort_wide then sorts the flagged tiles
// with 64-bit composites, each workgroup scanning 64 flags at a time (when
// every tile packed, it reads the flags and returns).
template <int DT, int K, int VM, int NETS>
__global__ __launch_bounds__(kBlockThreads, 6) void k_block_sort_packed(
    const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout, int64_t n,
    uint32_t* samp_first, uint32_t* samp_last, int* sorted_flag, int* wide_flag) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *sorted_flag = 1;
    __shared__ __align__(16) unsigned char smem[packed_lds_bytes<DT, K>()];
    constexpr int kTile = TileTraits<DT, K, true, 0>::kTile;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int nv = (int)((n - base) < kTile ? (n - base) : kTile);
    const bool sorted = block_sort_tile<DT, K, true, VM, 0, false, kPackOnly, NETS>(
        kin + base, VM == kVals ? vin + base : nullptr, kout + base,
        VM != kNoVals ? vout + base : nullptr, nv, (uint32_t)base, smem,
        Samples{samp_first, samp_last, base});
    if (threadIdx.x == 0) wide_flag[blockIdx.x] = sorted ? 0 : 1;
}

template <int DT, int K, int VM, int NETS>
__global__ __launch_bounds__(kBlockThreads, (TileTraits<DT, K, true, 0>::kWavesPerSimd)) void
k_block_sort_wide(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                  int64_t n, uint32_t* samp_first, uint32_t* samp_last,
                  const int* __restrict__ wide_flag, int64_t tiles) {
    __shared__ __align__(16) unsigned char smem[TileTraits<DT, K, true, 0>::kLdsBytes];
    __shared__ unsigned long long s_mask;
    constexpr int kTile = TileTraits<DT, K, true, 0>::kTile;
    for (int64_t b0 = (int64_t)blockIdx.x * kWave; b0 < tiles; b0 += (int64_t)gridDim.x * kWave) {
        if (threadIdx.x < kWave) {
            const int64_t t = b0 + threadIdx.x;
            const unsigned long long m = __ballot(t < tiles && wide_flag[t] != 0);
            if (threadIdx.x == 0) s_mask = m;
        }
        __syncthreads();
        unsigned long long m = s_mask;
        __syncthreads();  // s_mask is written again for the next 64 flags
        while (m != 0ull) {
            const int j = __builtin_ctzll(m);
            m &= m - 1ull;
            const int64_t base = (b0 + j) * kTile;
            const int nv = (int)((n - base) < kTile ? (n - base) : kTile);
            block_sort_tile<DT, K, true, VM, 0, false, kPackNone, NETS>(
                kin + base, VM == kVals ? vin + base : nullptr, kout + base,
                VM != kNoVals ? vout + base : nullptr, nv, (uint32_t)base, smem,
                Samples{samp_first, samp_last, base});
            __syncthreads();  // the LDS is reused for the next flagged tile
        }
    }
}

// ------------------------------------------------------- merge-path split ---
// For merge tile t of a pass that merges runs of length L: the number of
// elements of the pair's left run among the tile's first output position.
// One binary search per tile (Green, McColl, Bader 2012); stable (left run
// wins ties).  The search first runs over chunk-aligned candidates, reading
// the chunk samples the previous sweep wrote (A's chunk-first keys, B's
// chunk-last keys: a few MiB, cache- and TLB-friendly), which narrows it to
// one chunk; the last steps read the runs themselves.
template <int DT>
__global__ __launch_bounds__(256) void k_partition(const uint32_t* __restrict__ kin,
                                                   const uint32_t* __restrict__ samp_first,
                                                   const uint32_t* __restrict__ samp_last,
                                                   int32_t* __restrict__ part, int64_t n,
                                                   int64_t L, int mt, int ntiles,
                                                   const int* __restrict__ skip) {
    if (*skip) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const int64_t g0 = (int64_t)t * mt;
    const int64_t base = g0 & ~(2 * L - 1);
    const int64_t la = (n - base) < L ? (n - base) : L;
    const int64_t rest = n - base - la;
    const int64_t lb = rest < L ? rest : L;
    const int64_t d = g0 - base;
    const uint32_t* A = kin + base;
    const uint32_t* B = A + la;
    int64_t lo = d > lb ? d - lb : 0;
    int64_t hi = d < la ? d : la;
    if (samp_first && lb > 0 && lo < hi) {
        // base, la (= L), d and every candidate are multiples of the chunk, so
        // A[i] is a chunk's first key and B[d-1-i] a full chunk's last key.
        constexpr int64_t G = kSampleChunk;
        int64_t clo = (lo + G - 1) / G;
        int64_t chi = (hi - 1) / G;
        while (clo <= chi) {
            const int64_t cm = (clo + chi) >> 1;
            const int64_t i = cm * G;
            const uint32_t a = samp_first[(base + i) / G];
            const uint32_t b = samp_last[(base + la + d - i) / G - 1];
            if (!(ord_key<DT>(b) < ord_key<DT>(a))) {
                lo = i + 1;
                clo = cm + 1;
            } else {
                hi = i;
                chi = cm - 1;
            }
        }
    }
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (!(ord_key<DT>(B[d - 1 - mid]) < ord_key<DT>(A[mid])))
            lo = mid + 1;
        else
            hi = mid;
    }
    part[t] = (int32_t)lo;
}

// ------------------------------------------------------ global merge pass ---
// Workgroup t writes outputs [t*MT, (t+1)*MT) of the pass: it copies its
// slices of the two runs (split points from k_partition) into LDS with
// coalesced loads, each thread finds its own split inside the tile by merge
// path and merges KPT outputs sequentially, and the results go out as
// 16-byte stores.  Payloads are gathered from LDS by source position.
template <int DT, int KPT, bool VALS>
__global__ __launch_bounds__(kMergeThreads) void k_merge(const uint32_t* __restrict__ kin,
                                                         const uint32_t* __restrict__ vin,
                                                         uint32_t* __restrict__ kout,
                                                         uint32_t* __restrict__ vout,
                                                         const int32_t* __restrict__ part,
                                                         int64_t n, int64_t L, int vec,
                                                         uint32_t* __restrict__ samp_first,
                                                         uint32_t* __restrict__ samp_last,
                                                         const int* __restrict__ skip) {
    if (*skip) return;
    constexpr int MT = KPT * kMergeThreads;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* sk = reinterpret_cast<uint32_t*>(smem);
    uint32_t* sv = sk + lds_words<uint32_t>(MT);

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

    // Issue every load of the tile before the first LDS write, so each thread
    // has KPT loads in flight (addresses clamped into the tile, always valid).
    {
        uint32_t rk[KPT], rv[KPT];
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const int x = min((int)threadIdx.x + q * kMergeThreads, cnt - 1);
            const int64_t src = x < na ? base + i0 + x : base + la + j0 + (x - na);
            rk[q] = ld1_stream(kin + src);
            if constexpr (VALS) rv[q] = ld1_stream(vin + src);
        }
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const int x = (int)threadIdx.x + q * kMergeThreads;
            if (x < cnt) {
                sk[lds_idx<uint32_t>(x)] = rk[q];
                if constexpr (VALS) sv[lds_idx<uint32_t>(x)] = rv[q];
            }
        }
    }
    __syncthreads();

    const int d = threadIdx.x * KPT;
    uint32_t o[KPT], y[KPT];
    if (d < cnt) {
        const int i = corank_lds(sk, 0, na, na, nb, d, OrdLess<DT>{});
        int src[KPT];
        serial_merge<uint32_t, KPT, VALS>(sk, 0, na, na, nb, i, d - i, cnt - 1, o, src,
                                          OrdLess<DT>{});
        if constexpr (VALS) {
#pragma unroll
            for (int k = 0; k < KPT; ++k) y[k] = sv[lds_idx<uint32_t>(min(src[k], cnt - 1))];
        }
    }
    // Stage outputs in LDS (a spare word every 16) and store them as
    // contiguous 16-byte chunks per lane, keys and payload alike.
    constexpr int kStage = MT + MT / 16;
    uint32_t* stk = reinterpret_cast<uint32_t*>(smem);
    uint32_t* stv = stk + kStage;
    __syncthreads();
    if (d < cnt) {
#pragma unroll
        for (int k = 0; k < KPT; ++k) {
            stk[(d + k) + ((d + k) >> 4)] = o[k];
            if constexpr (VALS) stv[(d + k) + ((d + k) >> 4)] = y[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < KPT / 4; ++q) {
        const int e = 4 * ((int)threadIdx.x + q * kMergeThreads);
        const int pe = e + (e >> 4);
        if (vec && e + 4 <= cnt) {
            st4_stream(kout + g0 + e, stk[pe], stk[pe + 1], stk[pe + 2], stk[pe + 3]);
            if constexpr (VALS)
                st4_stream(vout + g0 + e, stv[pe], stv[pe + 1], stv[pe + 2], stv[pe + 3]);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (e + k < cnt) {
                    kout[g0 + e + k] = stk[pe + k];
                    if constexpr (VALS) vout[g0 + e + k] = stv[pe + k];
                }
        }
    }
    if (!samp_first) return;
    constexpr int kChunks = MT / kSampleChunk;
    const int c = (int)threadIdx.x;
    if (c < kChunks) {
        const int e = c * kSampleChunk;
        if (e < cnt) samp_first[g0 / kSampleChunk + c] = stk[e + (e >> 4)];
    } else if (c < 2 * kChunks) {
        const int e = (c - kChunks) * kSampleChunk + kSampleChunk - 1;
        if (e < cnt) samp_last[g0 / kSampleChunk + (c - kChunks)] = stk[e + (e >> 4)];
    }
}

// ------------------------------------------------------ presorted input ---
// After the first sweep every run is sorted, so the whole array is sorted
// exactly when no run's last key is ordered after the next run's first key
// (ties keep the runs' order, which is the stable order).  Runs are whole
// chunks, so both keys are chunk samples the sweep left behind.  The first
// sweep sets *flag; here one thread per pair of neighbouring runs clears it
// when the pair is out of order (every writer stores 0).  With the flag
// still set the global passes return at entry and the first sweep's result
// is the sorted array (k_copy_if moves it to the output when the sweep
// wrote the workspace).
template <int DT>
__global__ __launch_bounds__(256) void k_runs_in_order(const uint32_t* __restrict__ samp_first,
                                                       const uint32_t* __restrict__ samp_last,
                                                       int64_t runs, int64_t run_chunks,
                                                       int* __restrict__ flag) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r + 1 < runs; r += stride) {
        const uint32_t a = samp_last[(r + 1) * run_chunks - 1];
        const uint32_t b = samp_first[(r + 1) * run_chunks];
        if (ord_key<DT>(b) < ord_key<DT>(a)) *flag = 0;
    }
}

// kd = ks (and vd = vs) when *flag is set; returns at once otherwise.
__global__ __launch_bounds__(512) void k_copy_if(const uint32_t* __restrict__ ks,
                                                 const uint32_t* __restrict__ vs,
                                                 uint32_t* __restrict__ kd,
                                                 uint32_t* __restrict__ vd, int64_t n,
                                                 const int* __restrict__ flag) {
    if (!*flag) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n4 = n / 4;
    for (int64_t i = t0; i < n4; i += stride) {
        const uint4 k = ld4(ks + 4 * i);
        st4(kd + 4 * i, k.x, k.y, k.z, k.w);
        if (vs) {
            const uint4 v = ld4(vs + 4 * i);
            st4(vd + 4 * i, v.x, v.y, v.z, v.w);
        }
    }
    if (t0 < n - 4 * n4) {
        kd[4 * n4 + t0] = ks[4 * n4 + t0];
        if (vs) vd[4 * n4 + t0] = vs[4 * n4 + t0];
    }
}

// ------------------------------------------------------------- plain copy ---
// dst = src, n words: the achievable HBM rate next to the sorts.  One 16-byte
// nontemporal load and store per lane, one workgroup per 4096 words (the
// fastest of the shapes measured: grid-stride loops and several vectors per
// lane reached 4.2-5.8 TB/s, this one 6.5 TB/s on 2 GiB).  The tail of fewer
// than four words is copied word by word.
typedef uint32_t cpy_u4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy_words(const uint32_t* __restrict__ src,
                                                    uint32_t* __restrict__ dst, int64_t n) {
    const int64_t n4 = n / 4;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) {
        const cpy_u4 v = __builtin_nontemporal_load(reinterpret_cast<const cpy_u4*>(src) + i);
        __builtin_nontemporal_store(v, reinterpret_cast<cpy_u4*>(dst) + i);
    }
    if (i < n - 4 * n4) dst[4 * n4 + i] = src[4 * n4 + i];
}

__global__ __launch_bounds__(256) void k_copy_words_unaligned(const uint32_t* __restrict__ src,
                                                              uint32_t* __restrict__ dst,
                                                              int64_t n) {
    const int64_t lanes = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += lanes)
        dst[i] = src[i];
}

int launch_copy(const uint32_t* src, uint32_t* dst, int64_t n, hipStream_t stream) {
    if (n == 0) return 0;
    const bool vec = (((uintptr_t)src | (uintptr_t)dst) & 15u) == 0;
    LaunchTimer timer("copy_words", n, stream);
    if (vec) {
        const int64_t blocks = std::max<int64_t>(1, (n / 4 + 255) / 256);
        hipLaunchKernelGGL(k_copy_words, dim3((unsigned)blocks), dim3(256), 0, stream, src, dst,
                           n);
    } else {
        const unsigned grid =
            (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 1023) / 1024, 65536));
        hipLaunchKernelGGL(k_copy_words_unaligned, dim3(grid), dim3(256), 0, stream, src, dst, n);
    }
    return (int)hipGetLastError();
}

// ------------------------------------------------------------------ host ---
namespace {

template <typename Kern>
int ensure_lds(Kern kern, size_t bytes) {
    return set_dynamic_lds(reinterpret_cast<const void*>(kern), bytes);
}

template <int DT, int K, bool STABLE, int VM, int SHAPE, int NETS>
int launch_block_sort(const SortArgs& a, uint32_t* kdst, uint32_t* vdst,
                      const Samples& sm, int* sorted_flag) {
    using Tr = TileTraits<DT, K, STABLE, SHAPE>;
    auto kern = &k_block_sort<DT, K, STABLE, VM, SHAPE, NETS>;
    const int64_t blocks = (a.n + Tr::kTile - 1) / Tr::kTile;
    {
        LaunchTimer timer("block_sort", a.n, a.stream);
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(Tr::kThreads), 0, a.stream, a.kin,
                           a.vin, kdst, vdst, a.n, sm.first, sm.last, sorted_flag);
    }
    return (int)hipGetLastError();
}

// Tile shape of the first sweep: larger shapes only for integer keys-only
// sorts, chosen by the requested first-run length (block_tile / 1024K).
inline int block_shape(const SortArgs& a) {
    if (a.vmode != kNoVals || a.dtype == kF32) return 0;
    const int ratio = a.block_tile / (1024 * a.leaf_k);
    return ratio >= 4 ? 2 : ratio == 2 ? 1 : 0;
}

// The two-launch stable first sweep (k_block_sort_packed, k_block_sort_wide);
// wide: one flag per tile.
template <int DT, int K, int VM, int NETS>
int launch_block_sort_packed(const SortArgs& a, uint32_t* kdst, uint32_t* vdst,
                             const Samples& sm, int* sorted_flag, int* wide) {
    using Tr = TileTraits<DT, K, true, 0>;
    const int64_t tiles = (a.n + Tr::kTile - 1) / Tr::kTile;
    {
        LaunchTimer timer("block_sort", a.n, a.stream);
        hipLaunchKernelGGL((k_block_sort_packed<DT, K, VM, NETS>), dim3((unsigned)tiles),
                           dim3(kBlockThreads), 0, a.stream, a.kin, a.vin, kdst, vdst, a.n,
                           sm.first, sm.last, sorted_flag, wide);
    }
    if (int rc = (int)hipGetLastError()) return rc;
    auto wkern = &k_block_sort_wide<DT, K, VM, NETS>;
    int grid = 0;
    if (int rc = resident_grid(reinterpret_cast<const void*>(wkern), kBlockThreads, 0, &grid))
        return rc;
    grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, (tiles + kWave - 1) / kWave));
    {
        LaunchTimer timer("block_sort_wide", a.n, a.stream);
        hipLaunchKernelGGL(wkern, dim3((unsigned)grid), dim3(kBlockThreads), 0, a.stream, a.kin,
                           a.vin, kdst, vdst, a.n, sm.first, sm.last, wide, tiles);
    }
    return (int)hipGetLastError();
}

template <int DT, int K, int NETS>
int dispatch_block_sort(const SortArgs& a, uint32_t* kdst, uint32_t* vdst,
                        const Samples& sm, int* fl, int* wide) {
    // stable integer sorts with 8-key groups pack their tiles when they can
    constexpr bool kPacks = DT != kF32 && K == 8 && NETS != kNetNone;
    if (a.vmode == kVals) {
        if constexpr (kPacks)
            return launch_block_sort_packed<DT, K, kVals, NETS>(a, kdst, vdst, sm, fl, wide);
        return launch_block_sort<DT, K, true, kVals, 0, NETS>(a, kdst, vdst, sm, fl);
    }
    if (a.vmode == kArg) {
        if constexpr (kPacks)
            return launch_block_sort_packed<DT, K, kArg, NETS>(a, kdst, vdst, sm, fl, wide);
        return launch_block_sort<DT, K, true, kArg, 0, NETS>(a, kdst, vdst, sm, fl);
    }
    if constexpr (DT == kF32) {
        return launch_block_sort<DT, K, true, kNoVals, 0, NETS>(a, kdst, vdst, sm, fl);
    } else {
        switch (block_shape(a)) {
            case 1: return launch_block_sort<DT, K, false, kNoVals, 1, NETS>(a, kdst, vdst, sm, fl);
            case 2: return launch_block_sort<DT, K, false, kNoVals, 2, NETS>(a, kdst, vdst, sm, fl);
            default:
                return launch_block_sort<DT, K, false, kNoVals, 0, NETS>(a, kdst, vdst, sm, fl);
        }
    }
}

// Run length after the first sweep (the tile of the chosen shape).
inline int first_run_length(const SortArgs& a) {
    const int shape = block_shape(a);
    if (a.leaf_k == 8)
        return shape == 2 ? TileTraits<kU32, 8, false, 2>::kTile
             : shape == 1 ? TileTraits<kU32, 8, false, 1>::kTile
                          : TileTraits<kU32, 8, false, 0>::kTile;
    return shape == 2 ? TileTraits<kU32, 4, false, 2>::kTile
         : shape == 1 ? TileTraits<kU32, 4, false, 1>::kTile
                      : TileTraits<kU32, 4, false, 0>::kTile;
}

template <int DT, int KPT, bool VALS>
int launch_merge(const SortArgs& a, const uint32_t* ks, const uint32_t* vs, uint32_t* kd,
                 uint32_t* vd, int32_t* part, int64_t L, int vec, const Samples& sm,
                 const int* skip) {
    constexpr int MT = KPT * kMergeThreads;
    const int ntiles = (int)((a.n + MT - 1) / MT);
    {
        LaunchTimer timer("partition", ntiles, a.stream);
        hipLaunchKernelGGL(k_partition<DT>, dim3((ntiles + 255) / 256), dim3(256), 0, a.stream,
                           ks, sm.first, sm.last, part, a.n, L, MT, ntiles, skip);
    }
    if (int rc = (int)hipGetLastError()) return rc;
    if constexpr (!VALS && DT != kF32) {
        auto kern = &k_merge_keys<DT, KPT>;
        const size_t lds = (size_t)std::max(lds_words<uint32_t>(MT + 2 * KPT + 1),
                                            MT + MT / 16 + 1) * 4;
        if (int rc = ensure_lds(kern, lds)) return rc;
        LaunchTimer timer("merge", a.n, a.stream);
        hipLaunchKernelGGL(kern, dim3(ntiles), dim3(kMergeThreads), lds, a.stream, ks, kd, part,
                           a.n, L, vec, sm.first, sm.last, skip);
    } else {
        auto kern = &k_merge<DT, KPT, VALS>;
        const size_t lds = (size_t)std::max(lds_words<uint32_t>(MT), MT + MT / 16) * 4 *
                           (VALS ? 2 : 1);
        if (int rc = ensure_lds(kern, lds)) return rc;
        LaunchTimer timer("merge", a.n, a.stream);
        hipLaunchKernelGGL(kern, dim3(ntiles), dim3(kMergeThreads), lds, a.stream, ks, vs, kd, vd,
                           part, a.n, L, vec, sm.first, sm.last, skip);
    }
    return (int)hipGetLastError();
}

template <int DT, bool VALS>
int dispatch_merge(const SortArgs& a, const uint32_t* ks, const uint32_t* vs, uint32_t* kd,
                   uint32_t* vd, int32_t* part, int64_t L, int vec, const Samples& sm,
                   const int* skip) {
    switch (a.merge_tile) {
        case 2048: return launch_merge<DT, 8, VALS>(a, ks, vs, kd, vd, part, L, vec, sm, skip);
        case 8192: return launch_merge<DT, 32, VALS>(a, ks, vs, kd, vd, part, L, vec, sm, skip);
        default: return launch_merge<DT, 16, VALS>(a, ks, vs, kd, vd, part, L, vec, sm, skip);
    }
}

template <int DT, int THREADS, int KPT>
int launch_merge4(const SortArgs& a, const uint32_t* in, uint32_t* out, const M4Geom& g4,
                  const int32_t* bnd, const Samples& sm) {
    {
        LaunchTimer timer("merge4", a.n, a.stream);
        hipLaunchKernelGGL((k_merge4<DT, THREADS, KPT>), dim3((unsigned)m4_tiles(g4)),
                           dim3(THREADS), 0, a.stream, in, out, bnd, g4, sm.first, sm.last);
    }
    return (int)hipGetLastError();
}

// One four-way pass: runs of L in `in` -> runs of 4L in `out` (and their
// values, vin -> vout, when vin is set).  L is a power of two (the
// first-sweep run length times a power of four).
template <int DT>
int run_merge4(const SortArgs& a, const uint32_t* in, uint32_t* out, const uint32_t* vin,
               uint32_t* vout, int64_t L, const Samples& sm, int32_t* bnd, const int* skip) {
    M4Geom g4 = m4_geometry(a.n, L);
    g4.skip = skip;
    const int64_t nck = (a.n + kSampleChunk - 1) / kSampleChunk;
    int lg_cl = 0;
    while ((int64_t)kSampleChunk << lg_cl < L) ++lg_cl;
    if (((int64_t)kSampleChunk << lg_cl) != L) return (int)hipErrorInvalidValue;
    {
        LaunchTimer timer("m4_bounds", nck, a.stream);
        if ((1 << lg_cl) <= kM4SmallRun) {
            hipLaunchKernelGGL(k_m4_bounds_small<DT>,
                               dim3((unsigned)((nck + kM4BoundsBlock - 1) / kM4BoundsBlock)),
                               dim3(256), 0, a.stream, in, sm.first, bnd, g4, lg_cl, nck);
        } else {
            const int64_t bs = std::min<int64_t>(kM4BoundsBlock, (int64_t)1 << lg_cl);
            hipLaunchKernelGGL(k_m4_bounds_large<DT>, dim3((unsigned)((nck + bs - 1) / bs)),
                               dim3(256), 0, a.stream, in, sm.first, bnd, g4, lg_cl, nck);
        }
    }
    if (int rc = (int)hipGetLastError()) return rc;
    if (vin) {
        LaunchTimer timer("merge4_pairs", a.n, a.stream);
        hipLaunchKernelGGL((k_merge4_pairs<DT, 1024, 8>), dim3((unsigned)m4_tiles(g4)),
                           dim3(1024), 0, a.stream, in, vin, out, vout, bnd, g4, sm.first,
                           sm.last);
        return (int)hipGetLastError();
    }
    return a.merge4_kpt == 32 ? launch_merge4<DT, 256, 32>(a, in, out, g4, bnd, sm)
                              : launch_merge4<DT, 512, 16>(a, in, out, g4, bnd, sm);
}

template <int DT>
int run_sort(const SortArgs& a) {
    const int tile = first_run_length(a);
    // Pass plan: four-way passes (integer keys, with or without values)
    // while at least three runs remain, binary passes otherwise.
    bool four = false;
    if constexpr (DT != kF32) four = a.merge_ways == 4;
    int ways[64];
    int passes = 0;
    for (int64_t runs = (a.n + tile - 1) / tile; runs > 1;) {
        const int w = (four && runs >= 3) ? 4 : 2;
        ways[passes++] = w;
        runs = (runs + w - 1) / w;
    }

    const bool vals = a.vmode != kNoVals;
    uint8_t* ws = static_cast<uint8_t*>(a.ws);
    const size_t nk = align_up((size_t)a.n * 4, 256);
    uint32_t* wk = reinterpret_cast<uint32_t*>(ws);
    uint32_t* wv = vals ? reinterpret_cast<uint32_t*>(ws + nk) : nullptr;
    int32_t* part = reinterpret_cast<int32_t*>(ws + nk + (vals ? nk : 0));
    const size_t ntile_max = (size_t)((a.n + kMinMergeTile - 1) / kMinMergeTile) + 1;
    uint8_t* sbase = reinterpret_cast<uint8_t*>(part) + align_up(ntile_max * 4, 256);
    const size_t nchunks = (size_t)((a.n + kSampleChunk - 1) / kSampleChunk);
    const size_t ca = align_up(nchunks * 4, 256);
    Samples sm{reinterpret_cast<uint32_t*>(sbase), reinterpret_cast<uint32_t*>(sbase + ca), 0};
    // boundary table of the four-way passes, then the presorted flag
    int32_t* bnd = reinterpret_cast<int32_t*>(sbase + 2 * ca);
    int* sorted_flag = reinterpret_cast<int*>(sbase + 2 * ca + m4_ws_bytes(a.n));

    // Ping-pong so that the last pass lands in the output.
    uint32_t* kb[2] = {a.kout, wk};
    uint32_t* vb[2] = {a.vout, wv};
    auto aligned = [](const void* p) { return ((uintptr_t)p & 15u) == 0; };
    const int vec = aligned(a.kin) && aligned(a.kout) && aligned(wk) &&
                    (!vals || (aligned(a.vout) && aligned(wv) &&
                               (a.vmode != kVals || aligned(a.vin))));

    int cur = passes & 1;
    int rc = 0;
    // the merge-path split table (one word per 2048 keys) is free during the
    // first sweep: it holds the per-tile flags of the stable packed sweep
    int* wide = part;
    if (a.nets == kNetNone)
        rc = dispatch_block_sort<DT, 8, kNetNone>(a, kb[cur], vb[cur], sm, sorted_flag, wide);
    else if (a.nets == kNetSplit)
        rc = a.leaf_k == 8
                 ? dispatch_block_sort<DT, 8, kNetSplit>(a, kb[cur], vb[cur], sm, sorted_flag, wide)
                 : dispatch_block_sort<DT, 4, kNetSplit>(a, kb[cur], vb[cur], sm, sorted_flag, wide);
    else
        rc = a.leaf_k == 8
                 ? dispatch_block_sort<DT, 8, kNetPlain>(a, kb[cur], vb[cur], sm, sorted_flag, wide)
                 : dispatch_block_sort<DT, 4, kNetPlain>(a, kb[cur], vb[cur], sm, sorted_flag, wide);
    if (rc) return rc;
    if (passes > 0) {
        const int64_t runs = (a.n + tile - 1) / tile;
        {
            LaunchTimer timer("presorted", a.n, a.stream);
            hipLaunchKernelGGL(k_runs_in_order<DT>,
                               dim3((unsigned)std::min<int64_t>((runs + 254) / 256, 512)),
                               dim3(256), 0, a.stream, sm.first, sm.last, runs,
                               (int64_t)(tile / kSampleChunk), sorted_flag);
        }
        if (int e = (int)hipGetLastError()) return e;
        if (cur == 1) {
            LaunchTimer timer("copy", a.n, a.stream);
            hipLaunchKernelGGL(k_copy_if, dim3(512), dim3(512), 0, a.stream, kb[1],
                               vals ? vb[1] : nullptr, kb[0], vals ? vb[0] : nullptr, a.n,
                               sorted_flag);
        }
        if (int e = (int)hipGetLastError()) return e;
    }
    int64_t L = tile;
    for (int p = 0; p < passes; ++p) {
        const int nxt = cur ^ 1;
        if (ways[p] == 4) {
            if constexpr (DT != kF32)
                rc = run_merge4<DT>(a, kb[cur], kb[nxt], vals ? vb[cur] : nullptr,
                                    vals ? vb[nxt] : nullptr, L, sm, bnd, sorted_flag);
        } else {
            rc = vals ? dispatch_merge<DT, true>(a, kb[cur], vb[cur], kb[nxt], vb[nxt], part, L,
                                                 vec, sm, sorted_flag)
                      : dispatch_merge<DT, false>(a, kb[cur], nullptr, kb[nxt], nullptr, part, L,
                                                  vec, sm, sorted_flag);
        }
        if (rc) return rc;
        L *= ways[p];
        cur = nxt;
    }
    return 0;
}

}  // namespace

// ------------------------------------------------ allocation-free scratch ---
// The workspace of msn_sort_keys_noalloc: a fixed array in the code object,
// which every device the library runs on holds until the process ends.  In
// host code `scratch` names a host-side stand-in, never the device array: its
// device address comes from hipGetSymbolAddress, looked up once per device
// with that device current, and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};
}  // namespace

int noalloc_scratch(hipStream_t stream, void** ptr, size_t* bytes) {
    int dev = 0;
    if (int rc = (int)hipGetDevice(&dev)) return rc;
    int sdev = dev;
    if (stream) {
        if (int rc = (int)hipStreamGetDevice(stream, &sdev)) return rc;
    }
    if (sdev < 0 || sdev >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[sdev]) {
        if (sdev != dev) {
            if (int rc = (int)hipSetDevice(sdev)) return rc;
        }
        void* p = nullptr;
        const int rc = (int)hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (sdev != dev) (void)hipSetDevice(dev);
        if (rc) return rc;
        if (!p) return (int)hipErrorInvalidSymbol;
        scratch_ptr[sdev] = p;
    }
    *ptr = scratch_ptr[sdev];
    *bytes = kNoAllocScratchBytes;
    return 0;
}

int launch_sort(const SortArgs& a) {
    if (a.n == 0) return 0;
    switch (a.dtype) {
        case kU32: return run_sort<kU32>(a);
        case kI32: return run_sort<kI32>(a);
        default: return run_sort<kF32>(a);
    }
}

}  // namespace msn
