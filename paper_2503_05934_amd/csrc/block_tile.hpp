// Workgroup-wide sort of one tile of up to 2K * 512 keys (steps a1-a4: key
// map, per-lane networks, wavefront bitonic merge, LDS merge path).  Used by
// the flat sort's first sweep and by the segmented kernel for segments that
// fit one workgroup.
#pragma once

#include <type_traits>

#include "device.hpp"
#include "internal.hpp"

namespace msn {

// Tile shapes of the block sort (SHAPE): 0 = 512 threads x 2K keys per lane
// (the default); 1 = 1024 threads x 2K; 2 = 1024 threads x 4K (32768-key
// runs for the 6-to-8 set, 137 KiB of LDS); 3 = 1024 threads x K (the tile
// of shape 0 spread over twice the threads: one leaf group per lane, half
// the registers, twice the wavefronts per SIMD).  Shapes 1 and 2 serve the
// first sweep of flat integer keys-only sorts, shape 3 the stable sort of
// equal rows of at most one tile.
template <int DT, int K, bool STABLE, int SHAPE = 0>
struct TileTraits {
    using T = std::conditional_t<STABLE, uint64_t, uint32_t>;
    static_assert(SHAPE == 0 || SHAPE == 3 || !STABLE, "large tiles hold 32-bit keys only");
    static constexpr int kThreads = SHAPE == 0 ? kBlockThreads : 2 * kBlockThreads;
    static constexpr int kKPL = SHAPE == 2   ? 2 * keys_per_lane<K>()
                                : SHAPE == 3 ? K
                                             : keys_per_lane<K>();
    static constexpr int kTile = kKPL * kThreads;
    // keys-only tiles of 16 keys per lane can merge in LDS at 32 outputs per
    // thread (block_sort_regs2); LDS is sized for either layout
    static constexpr bool kWideOk = !STABLE && kKPL == 16;
    static constexpr size_t kLdsBytes =
        (size_t)(kWideOk && block_lds_words2<T, kKPL, 2 * kKPL>(kTile) >
                                block_lds_words<T, kKPL>(kTile)
                     ? block_lds_words2<T, kKPL, 2 * kKPL>(kTile)
                     : block_lds_words<T, kKPL>(kTile)) * sizeof(T);
    static_assert(!STABLE || kLdsBytes >= (size_t)2 * kTile * 4, "staging must fit");
    // waves per SIMD that the LDS footprint allows (160 KiB per compute unit,
    // 4 SIMDs, at most 8 waves per SIMD): the register budget the compiler is
    // held to
    static constexpr int kLdsWaves = (int)((163840 / kLdsBytes) * (kThreads / kWave) / 4);
    static constexpr int kWavesPerSimd = kLdsWaves < 1 ? 1 : kLdsWaves > 8 ? 8 : kLdsWaves;
};

// Bits of a tile position in the 32-bit composites of stable tiles whose keys
// all fit the remaining bits.
constexpr int kPackPosBits = 13;

// Sorts kin[0..nv) into kout[0..nv) (nv <= 2K*512).  STABLE sorts
// (key, position) composites; VM selects the payload: vout[i] = vin[p(i)]
// (kVals) or val_base + p(i) (kArg), p(i) = tile position of output i.  Float
// keys are copied bit for bit from the input.  All threads of the workgroup
// must call this (it contains barriers).  Full groups of four keys move as
// 16-byte accesses at any word alignment.  kout may equal kin (and vout vin):
// each position is read and
// written only by its owning thread, or read before a barrier that precedes
// every write.
// Records the chunk samples among a thread's outputs x[0..N) at tile
// positions first.. (global position samp.base + first + j).  N divides the
// chunk and tiles start on chunk boundaries, so only x[0] can open a chunk
// and only x[N-1] can close one.
template <int N>
__device__ __forceinline__ void write_samples(const Samples& samp, int first, int nv,
                                              const uint32_t (&x)[N]) {
    static_assert(kSampleChunk % N == 0, "keys per lane must divide the sample chunk");
    if (!samp.first) return;
    const int64_t p = samp.base + first;
    if ((p & (kSampleChunk - 1)) == 0 && first < nv) samp.first[p / kSampleChunk] = x[0];
    if (((p + N - 1) & (kSampleChunk - 1)) == kSampleChunk - 1 && first + N - 1 < nv)
        samp.last[(p + N - 1) / kSampleChunk] = x[N - 1];
}

// Stable tiles: copies what the outputs gather by tile position into LDS
// (the float bits of the keys, the payloads).  Call between barriers.
template <int DT, int VM, int THREADS>
__device__ __forceinline__ void stage_stable(const uint32_t* kin, const uint32_t* vin, int nv,
                                             uint32_t* sbits, uint32_t* svals) {
    if constexpr (DT == kF32 || VM == kVals) {
        for (int i = threadIdx.x; i < nv; i += THREADS) {
            if constexpr (DT == kF32) sbits[i] = kin[i];
            if constexpr (VM == kVals) svals[i] = vin[i];
        }
    }
}

// Stable tiles: writes N sorted outputs at tile positions first.., output j
// holding ordered key ok[j] from tile position t[j].  Float keys are copied
// bit for bit from the staged input, payloads gathered from the staged values
// (kVals) or generated (kArg: val_base + position).
template <int DT, int VM, int N>
__device__ __forceinline__ void emit_stable(const uint32_t (&t)[N], const uint32_t (&ok)[N],
                                            int first, int nv, const uint32_t* sbits,
                                            const uint32_t* svals, uint32_t* kout,
                                            uint32_t* vout, uint32_t val_base,
                                            const Samples& samp) {
    uint32_t kx[N], vy[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const uint32_t tj = first + j < nv ? t[j] : 0u;
        if constexpr (DT == kF32) kx[j] = sbits[tj];
        else kx[j] = unord_key<DT>(ok[j]);
        if constexpr (VM == kVals) vy[j] = svals[tj];
        else vy[j] = val_base + tj;
    }
    write_samples(samp, first, nv, kx);
    if (first + N <= nv) {
#pragma unroll
        for (int q = 0; q < N / 4; ++q) {
            st4(kout + first + 4 * q, kx[4 * q], kx[4 * q + 1], kx[4 * q + 2], kx[4 * q + 3]);
            if constexpr (VM != kNoVals)
                st4(vout + first + 4 * q, vy[4 * q], vy[4 * q + 1], vy[4 * q + 2],
                    vy[4 * q + 3]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < N; ++j)
            if (first + j < nv) {
                kout[first + j] = kx[j];
                if constexpr (VM != kNoVals) vout[first + j] = vy[j];
            }
    }
}

// WIDE (keys-only tiles of 16 keys per lane): LDS merge levels at 32 outputs
// per thread; fewer co-rank searches for more live registers.
// PACK (stable integer tiles of 16 keys per lane): tiles whose keys all fit
// 32 - kPackPosBits bits sort 32-bit (key, position) composites instead of
// 64-bit ones (a run-time choice per tile); kPackOnly leaves any other tile
// untouched and returns false (its caller then needs only the LDS of the
// packed path, packed_lds_bytes).  Returns true when the tile was sorted.
constexpr int kPackNone = 0, kPackAuto = 1, kPackOnly = 2;

template <int DT, int K, bool STABLE, int VM, int SHAPE = 0, bool WIDE = false,
          int PACK = kPackNone, int NETS = kNetPlain>
__device__ __forceinline__ bool block_sort_tile(const uint32_t* kin, const uint32_t* vin,
                                                uint32_t* kout, uint32_t* vout, int nv,
                                                uint32_t val_base, void* smem,
                                                Samples samp = Samples{nullptr, nullptr, 0}) {
    using Tr = TileTraits<DT, K, STABLE, SHAPE>;
    using T = typename Tr::T;
    static_assert(STABLE || (DT != kF32 && VM == kNoVals), "float keys and pairs sort stably");
    static_assert(PACK != kPackOnly || (STABLE && DT != kF32 && Tr::kKPL == 16 &&
                                        Tr::kTile <= (1 << kPackPosBits)),
                  "pack-only tiles are stable integer tiles of 16 keys per lane");
    static_assert(NETS != kNetNone || (!WIDE && !PACK),
                  "the network-free tile takes the plain paths");
    T* s = reinterpret_cast<T*>(smem);
    const int tid = threadIdx.x;
    constexpr int KPL = Tr::kKPL;
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
    T v[KPL];
#pragma unroll
    for (int j = 0; j < KPL; ++j) {
        if constexpr (STABLE) {
            v[j] = (first + j < nv) ? comp_make(ord_key<DT>(x[j]), (uint32_t)(first + j))
                                    : kCompMax;
        } else {
            v[j] = (first + j < nv) ? ord_key<DT>(x[j]) : 0xffffffffu;
        }
    }

    const int span = span_for(nv, kWave * KPL);
    if constexpr (WIDE && Tr::kWideOk) {
        constexpr int MK = 2 * KPL;
        T o[MK];
        block_sort_regs2<T, K, KPL, MK, NETS>(v, o, s, span, nv);
        const int first2 = tid * MK;
        if (first2 < span) {
            uint32_t y[MK];
#pragma unroll
            for (int j = 0; j < MK; ++j) y[j] = unord_key<DT>(o[j]);
            write_samples(samp, first2, nv, y);
            if (first2 + MK <= nv) {
#pragma unroll
                for (int q = 0; q < MK / 4; ++q)
                    st4(kout + first2 + 4 * q, y[4 * q], y[4 * q + 1], y[4 * q + 2],
                    y[4 * q + 3]);
            } else {
#pragma unroll
                for (int j = 0; j < MK; ++j)
                    if (first2 + j < nv) kout[first2 + j] = y[j];
            }
        }
    } else if constexpr (!STABLE) {
        if constexpr (NETS != kNetNone)
            block_sort_regs<T, K, KPL, NETS>(v, s, span, nv);
        else
            block_merge_only<T, KPL>(v, s, span);
#pragma unroll
        for (int j = 0; j < KPL; ++j) x[j] = unord_key<DT>(v[j]);
        write_samples(samp, first, nv, x);
        if (first + KPL <= nv) {
#pragma unroll
            for (int q = 0; q < KPL / 4; ++q)
                st4(kout + first + 4 * q, x[4 * q], x[4 * q + 1], x[4 * q + 2],
                    x[4 * q + 3]);
        } else {
#pragma unroll
            for (int j = 0; j < KPL; ++j)
                if (first + j < nv) kout[first + j] = x[j];
        }
    } else {
        constexpr bool kNeedBits = DT == kF32;
        uint32_t* sbits = reinterpret_cast<uint32_t*>(smem);
        uint32_t* svals = kNeedBits ? sbits + Tr::kTile : sbits;
        if constexpr (PACK && DT != kF32 && KPL == 16 && Tr::kTile <= (1 << kPackPosBits)) {
            // Every key of the tile below 2^(32 - kPackPosBits): the composite
            // (key, position) fits 32 bits, and the tile takes the keys-only
            // sort (32 outputs per thread in the LDS levels); keys (float
            // bits) and payloads are then gathered by position as below.
            uint32_t orv = 0;
#pragma unroll
            for (int j = 0; j < KPL; ++j) orv |= (first + j < nv) ? ord_key<DT>(x[j]) : 0u;
            if (__syncthreads_or((int)(orv >> (32 - kPackPosBits))) == 0) {
                constexpr int MK = 2 * KPL;
                uint32_t w[KPL], o[MK];
#pragma unroll
                for (int j = 0; j < KPL; ++j)
                    w[j] = (first + j < nv)
                               ? (ord_key<DT>(x[j]) << kPackPosBits) | (uint32_t)(first + j)
                               : 0xffffffffu;
                block_sort_regs2<uint32_t, K, KPL, MK, NETS>(w, o, reinterpret_cast<uint32_t*>(smem),
                                                       span, nv);
                stage_stable<DT, VM, Tr::kThreads>(kin, vin, nv, sbits, svals);
                __syncthreads();
                const int first2 = tid * MK;
                if (first2 < span) {
                    uint32_t t[MK], ok[MK];
#pragma unroll
                    for (int j = 0; j < MK; ++j) {
                        t[j] = o[j] & ((1u << kPackPosBits) - 1u);
                        ok[j] = o[j] >> kPackPosBits;
                    }
                    emit_stable<DT, VM, MK>(t, ok, first2, nv, sbits, svals, kout, vout,
                                            val_base, samp);
                }
                return true;
            }
            if constexpr (PACK == kPackOnly) return false;
        }
        if constexpr (NETS != kNetNone)
            block_sort_regs<T, K, KPL, NETS>(v, s, span, nv);
        else
            block_merge_only<T, KPL>(v, s, span);
        // Stage what must be gathered by position (float bits, payload).
        __syncthreads();
        stage_stable<DT, VM, Tr::kThreads>(kin, vin, nv, sbits, svals);
        __syncthreads();
        uint32_t t[KPL], ok[KPL];
#pragma unroll
        for (int j = 0; j < KPL; ++j) {
            t[j] = comp_pos(v[j]);
            ok[j] = comp_ord(v[j]);
        }
        emit_stable<DT, VM, KPL>(t, ok, first, nv, sbits, svals, kout, vout, val_base, samp);
    }
    return true;
}

// LDS bytes of a stable tile of shape 0 that takes only the packed path:
// the 32-bit composite layout of the wide merge levels, or the staged float
// bits and payloads, whichever is larger.
template <int DT, int K>
constexpr size_t packed_lds_bytes() {
    constexpr int kTile = TileTraits<DT, K, true, 0>::kTile;
    constexpr int KPL = TileTraits<DT, K, true, 0>::kKPL;
    constexpr size_t sort = (size_t)block_lds_words2<uint32_t, KPL, 2 * KPL>(kTile) * 4;
    constexpr size_t stage = (size_t)kTile * 4 * (DT == kF32 ? 2 : 1);
    return sort > stage ? sort : stage;
}

}  // namespace msn
