// Device building blocks of the network-leaf merge sort (gfx950, wave64).
//
// Paper (arXiv 2503.05934), Sec. 3, Algorithm 1: a merge sort that sorts
// small subarrays with fixed sorting networks and merges the rest.  On the GPU
// the recursion is run bottom-up:
//   1. every lane loads K consecutive keys and sorts them with one K-input
//      network held in VGPRs (the base case; K = 8 for the 6-to-8 set of
//      Table 3, K = 4 for 3-to-5);
//   2. a wavefront merges its 64 runs into one run of 64*K keys with bitonic
//      merges over cross-lane exchanges;
//   3. a workgroup merges its wavefront runs in LDS by merge path;
//   4. global passes merge pairs of runs until one run remains.
// Every merge is stable: on equal keys the left run's element goes first, as
// in the paper's Merge.  Networks and bitonic stages are not stable, so when
// stability matters the key travels with its tile position in one 64-bit
// word (a "composite", see comp_make) and ties are broken by position.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace msn {

// ------------------------------------------------------------ key order ---
// Order-preserving map of a key's bits to an unsigned 32-bit word.  uint32 is
// the identity, int32 flips the sign bit.  float32 first replaces -0 by +0
// and every NaN by one quiet NaN (they compare equal), then flips negative
// numbers bitwise and sets the sign bit of the rest, so that unsigned order is
// IEEE order with NaN above +inf.  The largest value a float can map to is
// 0xFFC00000.
template <int DT>
__device__ __forceinline__ uint32_t ord_key(uint32_t b) {
    if constexpr (DT == kU32) {
        return b;
    } else if constexpr (DT == kI32) {
        return b ^ 0x80000000u;
    } else {
        const uint32_t mag = b & 0x7fffffffu;
        b = (mag == 0u) ? 0u : b;
        b = (mag > 0x7f800000u) ? 0x7fc00000u : b;
        return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    }
}

// Inverse of ord_key for the bijective maps (uint32, int32).
template <int DT>
__device__ __forceinline__ uint32_t unord_key(uint32_t o) {
    if constexpr (DT == kI32) return o ^ 0x80000000u;
    return o;
}

// ------------------------------------------------------ 16-byte access ---
// Four consecutive words at any 4-byte-aligned address in one 16-byte load or
// store: gfx950 code objects run with unaligned multi-dword access enabled,
// so a tile that starts at any word of an array still moves 16 bytes per
// lane and instruction.
typedef uint32_t u32x4_w __attribute__((ext_vector_type(4), aligned(4)));
__device__ __forceinline__ uint4 ld4(const uint32_t* p) {
    const u32x4_w r = *reinterpret_cast<const u32x4_w*>(p);
    return make_uint4(r.x, r.y, r.z, r.w);
}
__device__ __forceinline__ void st4(uint32_t* p, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    const u32x4_w w = {a, b, c, d};
    *reinterpret_cast<u32x4_w*>(p) = w;
}

// ------------------------------------------------------ streaming access ---
// Global loads and stores with the nontemporal hint, for the binary merge of
// key-value pairs: each 64-lane load row and 16-byte-per-lane store row there
// covers whole cache lines, every key and value is read once and written once
// per pass, and the hint raises its sustained rate (about 4% per pass on
// 2^28 pairs).  Sweeps whose lanes each read or write a strided 64-byte
// stretch in several instructions lose by it: the line leaves the cache
// between them.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint32_t ld1_stream(const uint32_t* p) {
    return __builtin_nontemporal_load(p);
}
__device__ __forceinline__ void st4_stream(uint32_t* p, uint32_t a, uint32_t b, uint32_t c,
                                           uint32_t d) {
    const u32x4 w = {a, b, c, d};
    __builtin_nontemporal_store(w, reinterpret_cast<u32x4*>(p));
}

// ---------------------------------------------------- stable composites ---
// A stable sort carries each key with its tile position in one 64-bit word,
// the composite 2^52 + ord(key) * 2^20 + position (positions below 2^20),
// stored as the bits of that number as a double: the exponent field of 2^52
// (0x433) on top, ord(key) and the position in the 52 fraction bits.  Every
// composite has that exponent, so the word's unsigned integer order, its
// double order and the order (key, position) agree, and a compare-exchange
// is one v_min_f64 and one v_max_f64 instead of a 64-bit compare and four
// 32-bit selects.  The padding and sentinel composite is +inf (0x7FF0...),
// above every composite in both orders.  No composite is a NaN or a
// denormal, so the double minimum and maximum are exact.
constexpr int kCompPosBits = 20;
constexpr uint64_t kCompBase = 0x4330000000000000ull;  // the bits of 2^52
constexpr uint64_t kCompMax = 0x7FF0000000000000ull;   // the bits of +inf

__device__ __forceinline__ uint64_t comp_make(uint32_t ord, uint32_t pos) {
    return kCompBase | ((uint64_t)ord << kCompPosBits) | pos;
}
__device__ __forceinline__ uint32_t comp_ord(uint64_t c) { return (uint32_t)(c >> kCompPosBits); }
__device__ __forceinline__ uint32_t comp_pos(uint64_t c) {
    return (uint32_t)c & ((1u << kCompPosBits) - 1u);
}

// ------------------------------------------------------ compare-exchange ---
__device__ __forceinline__ uint32_t kmin(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t kmax(uint32_t a, uint32_t b) { return a < b ? b : a; }
// 64-bit words are composites (or kCompMax): minimum and maximum as doubles.
// The library is built without NaN handling (no key is ever a double NaN), so
// the compiler does not canonicalise the operands first.
__device__ __forceinline__ uint64_t kmin(uint64_t a, uint64_t b) {
    return __builtin_bit_cast(
        uint64_t, __builtin_fmin(__builtin_bit_cast(double, a), __builtin_bit_cast(double, b)));
}
__device__ __forceinline__ uint64_t kmax(uint64_t a, uint64_t b) {
    return __builtin_bit_cast(
        uint64_t, __builtin_fmax(__builtin_bit_cast(double, a), __builtin_bit_cast(double, b)));
}

// Half of a compare-exchange between lanes: the lane whose all-ones `upper`
// mask is set keeps the larger of (mine, theirs), the other the smaller.  For
// 32-bit keys that is the median of (mine, theirs, upper): 0 never exceeds
// the smaller and all-ones never falls below the larger, so one v_med3_u32
// replaces a min, a max and a select.
__device__ __forceinline__ uint32_t keep(uint32_t mine, uint32_t theirs, uint32_t upper) {
    return kmax(kmin(mine, theirs), kmin(kmax(mine, theirs), upper));
}
// Half of a compare-exchange between lanes for four 64-bit composites at
// once, where lane bit BIT selects the upper lanes: the lower lanes take the
// double minima and the upper lanes the double maxima, each under its own
// execution mask (eight VALU and four scalar instructions for four keys;
// keep() would take a compare and two selects per key).  The mask is
// restored before the block ends, and the closing s_nop covers the two wait
// states a DPP move that reads a result next needs.
template <int BIT>
__device__ __forceinline__ void keep_lanes4(uint64_t (&v)[4], const uint64_t (&o)[4]) {
    static_assert(BIT >= 0 && BIT < 6, "lane bit");
    constexpr uint64_t kUpper = BIT == 0   ? 0xAAAAAAAAAAAAAAAAull
                                : BIT == 1 ? 0xCCCCCCCCCCCCCCCCull
                                : BIT == 2 ? 0xF0F0F0F0F0F0F0F0ull
                                : BIT == 3 ? 0xFF00FF00FF00FF00ull
                                : BIT == 4 ? 0xFFFF0000FFFF0000ull
                                           : 0xFFFFFFFF00000000ull;
    double r0, r1, r2, r3;
    uint64_t save;
    asm("s_mov_b64 %4, exec\n\t"
        "s_andn2_b64 exec, %4, %13\n\t"
        "v_min_f64 %0, %5, %9\n\t"
        "v_min_f64 %1, %6, %10\n\t"
        "v_min_f64 %2, %7, %11\n\t"
        "v_min_f64 %3, %8, %12\n\t"
        "s_and_b64 exec, %4, %13\n\t"
        "v_max_f64 %0, %5, %9\n\t"
        "v_max_f64 %1, %6, %10\n\t"
        "v_max_f64 %2, %7, %11\n\t"
        "v_max_f64 %3, %8, %12\n\t"
        "s_mov_b64 exec, %4\n\t"
        "s_nop 1"
        : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&s"(save)
        : "v"(__builtin_bit_cast(double, v[0])), "v"(__builtin_bit_cast(double, v[1])),
          "v"(__builtin_bit_cast(double, v[2])), "v"(__builtin_bit_cast(double, v[3])),
          "v"(__builtin_bit_cast(double, o[0])), "v"(__builtin_bit_cast(double, o[1])),
          "v"(__builtin_bit_cast(double, o[2])), "v"(__builtin_bit_cast(double, o[3])),
          "s"(kUpper)
        : "scc");
    v[0] = __builtin_bit_cast(uint64_t, r0);
    v[1] = __builtin_bit_cast(uint64_t, r1);
    v[2] = __builtin_bit_cast(uint64_t, r2);
    v[3] = __builtin_bit_cast(uint64_t, r3);
}

// The same for eight composites under one pair of masks (groups of eight
// keys per lane): half the scalar instructions and wait states per key.
template <int BIT>
__device__ __forceinline__ void keep_lanes8(uint64_t (&v)[8], const uint64_t (&o)[8]) {
    static_assert(BIT >= 0 && BIT < 6, "lane bit");
    constexpr uint64_t kUpper = BIT == 0   ? 0xAAAAAAAAAAAAAAAAull
                                : BIT == 1 ? 0xCCCCCCCCCCCCCCCCull
                                : BIT == 2 ? 0xF0F0F0F0F0F0F0F0ull
                                : BIT == 3 ? 0xFF00FF00FF00FF00ull
                                : BIT == 4 ? 0xFFFF0000FFFF0000ull
                                           : 0xFFFFFFFF00000000ull;
    double r0, r1, r2, r3, r4, r5, r6, r7;
    uint64_t save;
    asm("s_mov_b64 %8, exec\n\t"
        "s_andn2_b64 exec, %8, %25\n\t"
        "v_min_f64 %0, %9, %17\n\t"
        "v_min_f64 %1, %10, %18\n\t"
        "v_min_f64 %2, %11, %19\n\t"
        "v_min_f64 %3, %12, %20\n\t"
        "v_min_f64 %4, %13, %21\n\t"
        "v_min_f64 %5, %14, %22\n\t"
        "v_min_f64 %6, %15, %23\n\t"
        "v_min_f64 %7, %16, %24\n\t"
        "s_and_b64 exec, %8, %25\n\t"
        "v_max_f64 %0, %9, %17\n\t"
        "v_max_f64 %1, %10, %18\n\t"
        "v_max_f64 %2, %11, %19\n\t"
        "v_max_f64 %3, %12, %20\n\t"
        "v_max_f64 %4, %13, %21\n\t"
        "v_max_f64 %5, %14, %22\n\t"
        "v_max_f64 %6, %15, %23\n\t"
        "v_max_f64 %7, %16, %24\n\t"
        "s_mov_b64 exec, %8\n\t"
        "s_nop 1"
        : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(r6),
          "=&v"(r7), "=&s"(save)
        : "v"(__builtin_bit_cast(double, v[0])), "v"(__builtin_bit_cast(double, v[1])),
          "v"(__builtin_bit_cast(double, v[2])), "v"(__builtin_bit_cast(double, v[3])),
          "v"(__builtin_bit_cast(double, v[4])), "v"(__builtin_bit_cast(double, v[5])),
          "v"(__builtin_bit_cast(double, v[6])), "v"(__builtin_bit_cast(double, v[7])),
          "v"(__builtin_bit_cast(double, o[0])), "v"(__builtin_bit_cast(double, o[1])),
          "v"(__builtin_bit_cast(double, o[2])), "v"(__builtin_bit_cast(double, o[3])),
          "v"(__builtin_bit_cast(double, o[4])), "v"(__builtin_bit_cast(double, o[5])),
          "v"(__builtin_bit_cast(double, o[6])), "v"(__builtin_bit_cast(double, o[7])),
          "s"(kUpper)
        : "scc");
    v[0] = __builtin_bit_cast(uint64_t, r0);
    v[1] = __builtin_bit_cast(uint64_t, r1);
    v[2] = __builtin_bit_cast(uint64_t, r2);
    v[3] = __builtin_bit_cast(uint64_t, r3);
    v[4] = __builtin_bit_cast(uint64_t, r4);
    v[5] = __builtin_bit_cast(uint64_t, r5);
    v[6] = __builtin_bit_cast(uint64_t, r6);
    v[7] = __builtin_bit_cast(uint64_t, r7);
}

// keep() on K keys against their partners o[] for the upper lanes of lane
// bit BIT (upper: their all-ones mask).
template <int BIT, int K>
__device__ __forceinline__ void keep_all(uint32_t (&v)[K], const uint32_t (&o)[K],
                                         uint32_t upper) {
#pragma unroll
    for (int j = 0; j < K; ++j) v[j] = keep(v[j], o[j], upper);
}
template <int BIT, int K>
__device__ __forceinline__ void keep_all(uint64_t (&v)[K], const uint64_t (&o)[K], uint32_t) {
    static_assert(K % 4 == 0, "groups of four keys");
    if constexpr (K % 8 == 0) {  // groups of eight
#pragma unroll
        for (int g = 0; g < K; g += 8) {
            uint64_t a[8], b[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                a[j] = v[g + j];
                b[j] = o[g + j];
            }
            keep_lanes8<BIT>(a, b);
#pragma unroll
            for (int j = 0; j < 8; ++j) v[g + j] = a[j];
        }
        return;
    }
#pragma unroll
    for (int g = 0; g < K; g += 4) {
        uint64_t a[4] = {v[g], v[g + 1], v[g + 2], v[g + 3]};
        const uint64_t b[4] = {o[g], o[g + 1], o[g + 2], o[g + 3]};
        keep_lanes4<BIT>(a, b);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[g + j] = a[j];
    }
}

// floor(log2(x)) for x >= 1.
__host__ __device__ constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

// All-ones when bit `bit` of lane is set, else 0.
__device__ __forceinline__ uint32_t lane_bit_mask(int lane, int bit) {
    return 0u - (((uint32_t)lane >> bit) & 1u);
}

template <typename T>
__device__ __forceinline__ void cx(T& a, T& b) {
    const T lo = kmin(a, b);
    const T hi = kmax(a, b);
    a = lo;
    b = hi;
}

// --------------------------------------------------------------- networks ---
// Fixed sorting networks, branch-free min/max in registers.  Both are
// Batcher's odd-even merge sort (Knuth, TAOCP 3, Sec. 5.3.4), written out in
// parallel layers: 8 inputs = 19 comparators in 6 layers, 4 inputs = 5 in 3.
// Fewer live keys (a tail) are handled by padding with the largest value,
// which never moves and so equals the pruned smaller network.
template <typename T>
__device__ __forceinline__ void network8(T (&v)[8]) {
    cx(v[0], v[1]); cx(v[2], v[3]); cx(v[4], v[5]); cx(v[6], v[7]);
    cx(v[0], v[2]); cx(v[1], v[3]); cx(v[4], v[6]); cx(v[5], v[7]);
    cx(v[1], v[2]); cx(v[5], v[6]);
    cx(v[0], v[4]); cx(v[1], v[5]); cx(v[2], v[6]); cx(v[3], v[7]);
    cx(v[2], v[4]); cx(v[3], v[5]);
    cx(v[1], v[2]); cx(v[3], v[4]); cx(v[5], v[6]);
}

template <typename T>
__device__ __forceinline__ void network4(T (&v)[4]) {
    cx(v[0], v[1]); cx(v[2], v[3]);
    cx(v[0], v[2]); cx(v[1], v[3]);
    cx(v[1], v[2]);
}

template <typename T, int K>
__device__ __forceinline__ void leaf_network(T (&v)[K]) {
    static_assert(K == 8 || K == 4, "leaf size");
    if constexpr (K == 8) network8(v); else network4(v);
}

// Largest value of a register key: the padding of short runs and the
// sentinel that closes every LDS run.
template <typename T>
__device__ __forceinline__ constexpr T key_max() {
    return sizeof(T) == 8 ? (T)kCompMax : (T)0xffffffffu;
}

// The N-input network (2 <= N <= K) on v[0..N): the K-input network with
// inputs N..K-1 fixed at the largest value.  Those inputs are compile-time
// constants here, so every comparator that touches them folds away and what
// remains is the pruned N-key network (Batcher's construction restricted to
// N wires).
template <typename T, int K, int N>
__device__ __forceinline__ void pruned_network(T (&v)[K]) {
    static_assert(N >= 1 && N <= K, "network size");
#pragma unroll
    for (int j = N; j < K; ++j) v[j] = key_max<T>();
    leaf_network<T, K>(v);
}

// Network families (kNetNone / kNetPlain / kNetSplit, internal.hpp): how a
// lane sorts one group of K keys.
//   kNetPlain: the K-key network (sets that hold K: 6-to-8, PowerOf2, Even,
//     3-to-8 for K = 8; 3-to-5, 3-to-4, VarSort4 for K = 4);
//   kNetSplit: two member networks and one merge, for sets without a
//     K-key member: K = 8 sorts keys 0..4 with the 5-key network and keys
//     5..7 with the 3-key network (Odd = {3, 5, 7}, VarSort5 = {2..5});
//     K = 4 sorts keys 0..2 with the 3-key network and takes key 3 alone
//     (the set {3}, VarSort3).  The two sorted pieces, the second reversed,
//     form a bitonic sequence that half-cleaners at distances K/2 .. 1 sort.
template <typename T, int K, int NET>
__device__ __forceinline__ void leaf_group(T (&v)[K]) {
    static_assert(NET == kNetPlain || NET == kNetSplit, "network family");
    if constexpr (NET == kNetPlain) {
        leaf_network<T, K>(v);
    } else {
        constexpr int A = K == 8 ? 5 : 3;  // keys of the first piece
        T a[K], b[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            a[j] = j < A ? v[j] : key_max<T>();
            b[j] = j < K - A ? v[A + j] : key_max<T>();
        }
        if constexpr (A > 1) pruned_network<T, K, A>(a);
        if constexpr (K - A > 1) pruned_network<T, K, K - A>(b);
        // ascending first piece, then the second piece descending
#pragma unroll
        for (int j = 0; j < A; ++j) v[j] = a[j];
#pragma unroll
        for (int j = 0; j < K - A; ++j) v[K - 1 - j] = b[j];
#pragma unroll
        for (int d = K / 2; d >= 1; d >>= 1) {
#pragma unroll
            for (int j = 0; j < K; ++j)
                if ((j & d) == 0) cx(v[j], v[j + d]);
        }
    }
}

// A lane's whole subarray of len <= K keys (v[len..K) hold the largest
// value): the network of that size when the configured set holds it (bit
// len of set_mask), else the family's group procedure on the padded keys --
// the role of the paper's variable-size networks (VarSort, Table 3).
template <typename T, int K, int NET>
__device__ __forceinline__ void lane_networks(T (&v)[K], int len, uint32_t set_mask) {
    if (len < K && ((set_mask >> len) & 1u)) {
        switch (len) {
            case 2: pruned_network<T, K, 2>(v); return;
            case 3: pruned_network<T, K, 3>(v); return;
            case 4: if constexpr (K > 4) { pruned_network<T, K, 4>(v); return; } break;
            case 5: if constexpr (K > 5) { pruned_network<T, K, 5>(v); return; } break;
            case 6: if constexpr (K > 6) { pruned_network<T, K, 6>(v); return; } break;
            case 7: if constexpr (K > 7) { pruned_network<T, K, 7>(v); return; } break;
            default: break;
        }
    }
    leaf_group<T, K, NET>(v);
}

// -------------------------------------------------------- lane exchanges ---
// Value of x in lane (lane ^ mask).  Patterns that DPP can express inside a
// row of 16 lanes go through the VALU's data-parallel-primitive moves:
// quad_perm for masks 1, 2, 3, row_ror:8 for 8, row_half_mirror (lane i <-
// 7 - i) for 7 and row_mirror (i <- 15 - i) for 15.  Other masks below 32 use
// ds_swizzle's bit mode (and = 0x1f, xor = mask) inside 32-lane halves, and
// masks of 32 and above use ds_bpermute.  None of them touches LDS memory.
template <int MASK>
__device__ __forceinline__ uint32_t xor_lane(uint32_t x) {
    static_assert(MASK > 0 && MASK < 64, "mask");
    constexpr int kQuadXor1 = 0xb1;   // quad_perm [1,0,3,2]
    constexpr int kQuadXor2 = 0x4e;   // quad_perm [2,3,0,1]
    constexpr int kQuadXor3 = 0x1b;   // quad_perm [3,2,1,0]
    constexpr int kRowRor8 = 0x128;
    constexpr int kRowMirror = 0x140;
    constexpr int kRowHalfMirror = 0x141;
    if constexpr (MASK == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, kQuadXor1, 0xf, 0xf, true);
    } else if constexpr (MASK == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, kQuadXor2, 0xf, 0xf, true);
    } else if constexpr (MASK == 3) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, kQuadXor3, 0xf, 0xf, true);
    } else if constexpr (MASK == 7) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, kRowHalfMirror, 0xf, 0xf, true);
    } else if constexpr (MASK == 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, kRowRor8, 0xf, 0xf, true);
    } else if constexpr (MASK == 15) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, kRowMirror, 0xf, 0xf, true);
    } else if constexpr (MASK < 32) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, (MASK << 10) | 0x1f);
    } else {
        const int src = ((int)(threadIdx.x & 63) ^ MASK) << 2;
        return (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)x);
    }
}

template <int MASK>
__device__ __forceinline__ uint64_t xor_lane(uint64_t x) {
    const uint32_t lo = xor_lane<MASK>((uint32_t)x);
    const uint32_t hi = xor_lane<MASK>((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// ----------------------------------------------------- wavefront merging ---
// Cross-lane half-cleaner at lane distance M, then the next one down.
template <typename T, int K, int M>
__device__ __forceinline__ void wave_cross_stages(T (&v)[K], int lane) {
    if constexpr (M >= 1) {
        const uint32_t upper = lane_bit_mask(lane, ilog2(M));
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int j = 0; j < K; ++j) v[j] = keep(v[j], xor_lane<M>(v[j]), upper);
        } else {
            T o[K];
#pragma unroll
            for (int j = 0; j < K; ++j) o[j] = xor_lane<M>(v[j]);
            keep_all<ilog2(M), K>(v, o, upper);
        }
        wave_cross_stages<T, K, M / 2>(v, lane);
    }
}

// Runs of G lanes (G*K keys, lane-major: key e sits in lane e / K, slot
// e % K) are merged pairwise into runs of 2G lanes by a bitonic merge:
//   flip  : key e of the pair meets key (2GK-1-e): lane l meets lane
//           l ^ (2G-1), slot j meets slot K-1-j; the lower key keeps the min.
//   clean : distance d = GK/2, ..., 1: key e meets e + d; for d >= K that is
//           lane l ^ (d/K) in the same slot, below K it is inside the lane.
template <typename T, int K, int G>
__device__ __forceinline__ void wave_merge_level(T (&v)[K], int lane) {
    {
        T o[K];
#pragma unroll
        for (int j = 0; j < K; ++j) o[j] = xor_lane<2 * G - 1>(v[K - 1 - j]);
        keep_all<ilog2(G), K>(v, o, lane_bit_mask(lane, ilog2(G)));
    }
    // cross-lane half-cleaners, lane distance G/2 ... 1
    wave_cross_stages<T, K, G / 2>(v, lane);
    // in-lane half-cleaners, distance K/2 ... 1
#pragma unroll
    for (int d = K / 2; d >= 1; d >>= 1) {
#pragma unroll
        for (int j = 0; j < K; ++j)
            if ((j & d) == 0) cx(v[j], v[j + d]);
    }
}

// 64 sorted lane runs of K keys -> one sorted run of 64*K keys per wavefront.
template <typename T, int K>
__device__ __forceinline__ void wave_merge(T (&v)[K], int lane) {
    wave_merge_level<T, K, 1>(v, lane);
    wave_merge_level<T, K, 2>(v, lane);
    wave_merge_level<T, K, 4>(v, lane);
    wave_merge_level<T, K, 8>(v, lane);
    wave_merge_level<T, K, 16>(v, lane);
    wave_merge_level<T, K, 32>(v, lane);
}

// --------------------------------------------------------------- LDS maps ---
// Padded LDS index: one spare slot every 32 words (every 16 for 64-bit keys)
// so that the strided accesses of merge path do not pile onto few banks.
template <typename T>
__device__ __forceinline__ int lds_idx(int i) {
    // indices are never negative: unsigned shifts let the compiler fold the
    // scaling into one shift-add
    const unsigned u = (unsigned)i;
    return (int)(sizeof(T) == 8 ? u + (u >> 4) : u + (u >> 5));
}
template <typename T>
__host__ __device__ constexpr int lds_words(int n) {
    return sizeof(T) == 8 ? n + (n >> 4) + 1 : n + (n >> 5) + 1;
}
// Byte offset of padded slot i, sizeof(T) * lds_idx<T>(i), in one shift and
// one shift-add.
template <typename T>
__device__ __forceinline__ uint32_t lds_off(uint32_t i) {
    uint32_t r;
    if constexpr (sizeof(T) == 8)
        asm("v_add_lshl_u32 %0, %1, %2, 3" : "=v"(r) : "v"(i), "v"(i >> 4));
    else
        asm("v_add_lshl_u32 %0, %1, %2, 2" : "=v"(r) : "v"(i), "v"(i >> 5));
    return r;
}
template <typename T>
__device__ __forceinline__ T lds_load(const T* s, uint32_t i) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const unsigned char*>(s) + lds_off<T>(i));
}

// Merge path (Green, McColl, Bader 2012): number of elements of A among the
// first d outputs of the stable merge of A (la keys) and B (lb keys), both
// sorted; A wins ties.  `less` compares two stored keys.
template <typename T, typename Less>
__device__ __forceinline__ int corank_lds(const T* s, int a0, int la, int b0, int lb, int d,
                                          Less less) {
    int lo = d > lb ? d - lb : 0;
    int hi = d < la ? d : la;
    const int kb = b0 + d - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (!less(lds_load(s, (uint32_t)(kb - mid)), lds_load(s, (uint32_t)(a0 + mid))))
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// corank_lds with PlainLess for two runs of L keys each (L a power of two)
// laid out so that LDS words [a0, b0 + L) all belong to the pair: A at a0, B
// at b0 >= a0 + L.  Binary lifting with the steps L, L/2, ..., 1, the same
// for every lane: m is the last position of A known to go before
// B[d-1-m]; a step is taken when its new last position is still inside A's
// share of the diagonal and goes first.  A probe beyond that share stays
// inside the pair's words (at most L past the share on either side) and its
// result is discarded.  Nine VALU instructions per step and no exit test.
template <typename T>
__device__ __forceinline__ int corank_pow2(const T* s, int a0, int b0, int L, int d) {
    const int lo = d > L ? d - L : 0;
    const int hi = d < L ? d : L;
    const uint32_t lim = (uint32_t)(a0 + hi);
    const uint32_t c = (uint32_t)(b0 + d - 1 + a0);  // B[d-1-(t-a0)] sits at c - t
    uint32_t m = (uint32_t)(a0 + lo) - 1u;
    for (int step = L; step > 0; step >>= 1) {
        const uint32_t t = m + (uint32_t)step;
        const T av = lds_load(s, t);
        const T bv = lds_load(s, c - t);
        if (t < lim && !(bv < av)) m = t;
    }
    return (int)(m + 1u) - a0;
}

// Sequential stable merge of N outputs starting at A[i], B[j] (LDS runs
// [a0, a0+la) and [b0, b0+lb)).  One LDS read per output; reads past a run's
// end are clamped to `limit` and their values ignored.  src[k] receives the
// (unpadded) LDS position of output k.
template <typename T, int N, bool SRC, typename Less>
__device__ __forceinline__ void serial_merge(const T* s, int a0, int la, int b0, int lb, int i,
                                             int j, int limit, T (&out)[N], int (&src)[N],
                                             Less less) {
    T a = s[lds_idx<T>(min(a0 + i, limit))];
    T b = s[lds_idx<T>(min(b0 + j, limit))];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const bool take_a = (i < la) && (j >= lb || !less(b, a));
        out[k] = take_a ? a : b;
        if constexpr (SRC) src[k] = take_a ? a0 + i : b0 + j;
        i += take_a ? 1 : 0;
        j += take_a ? 0 : 1;
        const int nxt = take_a ? a0 + i : b0 + j;
        const T x = s[lds_idx<T>(min(nxt, limit))];
        a = take_a ? x : a;
        b = take_a ? b : x;
    }
}

struct PlainLess {
    template <typename T>
    __device__ __forceinline__ bool operator()(T x, T y) const { return x < y; }
};

template <int DT>
struct OrdLess {
    __device__ __forceinline__ bool operator()(uint32_t x, uint32_t y) const {
        return ord_key<DT>(x) < ord_key<DT>(y);
    }
};

// Sequential merge of N outputs from LDS runs that are each followed by at
// least N copies of key_max(): no bounds checks are needed, because a used-up
// run offers the maximum, which is taken only when the other run's key is the
// maximum too (the same value; composite keys never reach it).  pa, pb:
// (unpadded) positions of the next key of each run.  The state is the head x
// of the run that gave the last output (its next key at pc) and the head y of
// the other run (next key at po).  Equal keys may come from either run, which
// yields the values of the stable merge: all a key-only merge keeps
// (composite keys are unique).
template <typename T, int N>
__device__ __forceinline__ void serial_merge_closed(const T* s, int pa, int pb, T (&out)[N]) {
    if constexpr (sizeof(T) == 4) {
        T x = lds_load(s, (uint32_t)pa);
        T y = lds_load(s, (uint32_t)pb);
        uint32_t pc = (uint32_t)pa + 1, po = (uint32_t)pb + 1;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const bool keep = !(y < x);
            out[k] = keep ? x : y;
            const T hi = keep ? y : x;
            const uint32_t p = keep ? pc : po;
            po = keep ? po : pc;
            pc = p + 1;
            x = lds_load(s, p);
            y = hi;
        }
    } else {
        // 64-bit composites (unique, so no ties): the output and the head
        // kept for the next step are the double minimum and maximum, and
        // only the positions follow the comparison
        T x = lds_load(s, (uint32_t)pa);
        T y = lds_load(s, (uint32_t)pb);
        uint32_t pc = (uint32_t)pa + 1, po = (uint32_t)pb + 1;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const bool keep = !(y < x);
            out[k] = kmin(x, y);
            const T hi = kmax(x, y);
            const uint32_t p = keep ? pc : po;
            po = keep ? po : pc;
            pc = p + 1;
            x = lds_load(s, p);
            y = hi;
        }
    }
}

// Adjacent sorted runs of R keys in one lane's v[0..N) -> sorted runs of 2R
// (bitonic: flip each pair of runs, then half-cleaners inside each run).
template <typename T, int N, int R>
__device__ __forceinline__ void lane_merge_runs(T (&v)[N]) {
#pragma unroll
    for (int b = 0; b < N; b += 2 * R) {
#pragma unroll
        for (int j = 0; j < R; ++j) cx(v[b + j], v[b + 2 * R - 1 - j]);
#pragma unroll
        for (int d = R / 2; d >= 1; d >>= 1) {
#pragma unroll
            for (int j = 0; j < 2 * R; ++j)
                if ((j & d) == 0) cx(v[b + j], v[b + j + d]);
        }
    }
}

// Two sorted runs v[0..N/2) and v[N/2..N) in one lane -> one sorted run.
template <typename T, int N>
__device__ __forceinline__ void lane_merge_halves(T (&v)[N]) {
    lane_merge_runs<T, N, N / 2>(v);
}

// Each group of K keys in v[0..N) sorted by the K-key network, then the
// groups merged in-lane into one sorted run of N keys.
template <typename T, int K, int N, int NET = kNetPlain>
__device__ __forceinline__ void lane_sort(T (&v)[N]) {
#pragma unroll
    for (int g = 0; g < N; g += K) {
        T w[K];
#pragma unroll
        for (int j = 0; j < K; ++j) w[j] = v[g + j];
        leaf_group<T, K, NET>(w);
#pragma unroll
        for (int j = 0; j < K; ++j) v[g + j] = w[j];
    }
    if constexpr (N >= 2 * K) lane_merge_runs<T, N, K>(v);
    if constexpr (N >= 4 * K) lane_merge_runs<T, N, 2 * K>(v);
    if constexpr (N >= 8 * K) lane_merge_runs<T, N, 4 * K>(v);
    static_assert(N == K || N == 2 * K || N == 4 * K || N == 8 * K, "keys per lane");
}

// --------------------------------------------------------- block sorting ---
// Keys per lane in the block sort: two base-case groups of K keys.
template <int K>
constexpr int keys_per_lane() { return 2 * K; }

// LDS words block_sort_regs needs for a tile of n keys: the keys, KPL
// sentinels after each of the (at most n / (64*KPL)) runs, and padding.
template <typename T, int KPL>
__host__ __device__ constexpr int block_lds_words(int n) {
    return lds_words<T>(n + (n / (kWave * KPL)) * KPL + KPL);
}

// Sorts the KPL*(threads) keys held as v[] by all threads of a workgroup
// (thread t holds keys t*KPL .. t*KPL+KPL-1 in registers; KPL is a multiple
// of K).  Each lane applies the K-key network to each of its groups and
// merges them; the wavefront merges its 64 lane runs by bitonic exchanges;
// then LDS merge-path levels double the run length up to `span` (a power of
// two, at least 64*KPL): lanes beyond it still take part in barriers but skip
// the work.  Keys from position nv on are padding (the largest value): a
// wavefront holding only padding is sorted already and skips the networks
// and its merge.  On return thread t holds outputs t*KPL .. t*KPL+KPL-1 of
// the sorted span.  s is LDS of block_lds_words<T, KPL>(tile keys) words.
template <typename T, int K, int KPL, int NET = kNetPlain>
__device__ __forceinline__ void block_sort_regs(T (&v)[KPL], T* s, int span, int nv) {
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const bool active = tid * KPL < span;
    if (active && __builtin_amdgcn_readfirstlane((tid - lane) * KPL) < nv) {
        lane_sort<T, K, KPL, NET>(v);
        wave_merge<T, KPL>(v, lane);
    }
    for (int L = kWave * KPL; L < span; L <<= 1) {
        // run r occupies [r*(L+KPL), r*(L+KPL)+L), then KPL sentinels
        const int e = tid * KPL;
        const int run = e / L;
        if (active) {
            const int pos = e + run * KPL;
#pragma unroll
            for (int j = 0; j < KPL; ++j) s[lds_idx<T>(pos + j)] = v[j];
            if ((e % L) == L - KPL) {
#pragma unroll
                for (int j = 0; j < KPL; ++j) s[lds_idx<T>(pos + KPL + j)] = key_max<T>();
            }
        }
        __syncthreads();
        if (active) {
            const int ra = run & ~1;
            const int a0 = ra * (L + KPL);
            const int b0 = a0 + L + KPL;
            const int d = e - ra * L;
            const int i = corank_pow2(s, a0, b0, L, d);
            serial_merge_closed<T, KPL>(s, a0 + i, b0 + d - i, v);
        }
        __syncthreads();
    }
}

// The same contract as block_sort_regs with no network anywhere: the
// classical merge sort the paper measures its network leaves against (its
// empty network set), in the same tile shape.  Each thread first merges its
// KPL keys from runs of one key up to one run of KPL, pairs of runs read
// back from its own LDS window; merge-path levels across threads then double
// the runs up to `span`.  Every merge is sequential and stable, and checks
// the run ends instead of relying on sentinels, so the LDS holds the span
// and nothing more.
template <typename T, int L, int KPL>
__device__ __forceinline__ void merge_in_thread(T (&v)[KPL], T* s, int e) {
    if constexpr (L < KPL) {
        // the window is this thread's own: its earlier reads precede these
        // writes in program order, and no other thread touches it
#pragma unroll
        for (int j = 0; j < KPL; ++j) s[lds_idx<T>(e + j)] = v[j];
#pragma unroll
        for (int p = 0; p < KPL / (2 * L); ++p) {
            T o[2 * L];
            int src[2 * L];
            const int a0 = e + p * 2 * L;
            serial_merge<T, 2 * L, false>(s, a0, L, a0 + L, L, 0, 0, e + KPL - 1, o, src,
                                          PlainLess{});
#pragma unroll
            for (int k = 0; k < 2 * L; ++k) v[p * 2 * L + k] = o[k];
        }
        merge_in_thread<T, 2 * L, KPL>(v, s, e);
    }
}

template <typename T, int KPL>
__device__ __forceinline__ void block_merge_only(T (&v)[KPL], T* s, int span) {
    const int e = (int)threadIdx.x * KPL;
    const bool active = e < span;
    if (active) merge_in_thread<T, 1, KPL>(v, s, e);
    for (int L = KPL; L < span; L <<= 1) {
        __syncthreads();  // the previous level's readers are done with s
        if (active) {
#pragma unroll
            for (int j = 0; j < KPL; ++j) s[lds_idx<T>(e + j)] = v[j];
        }
        __syncthreads();
        if (active) {
            const int a0 = e & ~(2 * L - 1);
            const int d = e - a0;
            const int i = corank_pow2(s, a0, a0 + L, L, d);
            int src[KPL];
            serial_merge<T, KPL, false>(s, a0, L, a0 + L, L, i, d - i, span - 1, v, src,
                                        PlainLess{});
        }
    }
    __syncthreads();  // the caller may reuse s
}

// LDS words block_sort_regs2 needs: as block_lds_words with MK sentinels per run.
template <typename T, int KPL, int MK>
__host__ __device__ constexpr int block_lds_words2(int n) {
    return lds_words<T>(n + (n / (kWave * KPL)) * MK + MK);
}

// As block_sort_regs, with the LDS merge levels run by the first half of the
// threads at MK = 2 KPL outputs each (one co-rank search per MK outputs): on
// return thread t < threads/2 holds outputs t*MK .. t*MK+MK-1 of the sorted
// span in o[].  s is LDS of block_lds_words2<T, KPL, MK>(tile keys) words.
template <typename T, int K, int KPL, int MK, int NET = kNetPlain>
__device__ __forceinline__ void block_sort_regs2(T (&v)[KPL], T (&o)[MK], T* s, int span,
                                                 int nv) {
    static_assert(MK == 2 * KPL, "two lanes' keys per merger");
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    int L = kWave * KPL;  // wavefront runs
    if (tid * KPL < span) {
        if (__builtin_amdgcn_readfirstlane((tid - lane) * KPL) < nv) {
            lane_sort<T, K, KPL, NET>(v);
            wave_merge<T, KPL>(v, lane);
        }
        // run r occupies [r*(L+MK), r*(L+MK)+L), then MK sentinels
        const int e = tid * KPL;
        const int run = e / L;
        const int pos = e + run * MK;
#pragma unroll
        for (int j = 0; j < KPL; ++j) s[lds_idx<T>(pos + j)] = v[j];
        if ((e % L) == L - KPL) {
#pragma unroll
            for (int j = 0; j < MK; ++j) s[lds_idx<T>(pos + KPL + j)] = key_max<T>();
        }
    }
    __syncthreads();
    const int e = tid * MK;
    const bool merger = e < span;
    if (L >= span) {  // one wavefront run: regroup it, MK keys per thread
        if (merger) {
#pragma unroll
            for (int j = 0; j < MK; ++j) o[j] = lds_load(s, (uint32_t)(e + j));
        }
        __syncthreads();
        return;
    }
    for (;;) {
        if (merger) {
            const int run = e / L;
            const int ra = run & ~1;
            const int a0 = ra * (L + MK);
            const int b0 = a0 + L + MK;
            const int d = e - ra * L;
            const int i = corank_pow2(s, a0, b0, L, d);
            serial_merge_closed<T, MK>(s, a0 + i, b0 + d - i, o);
        }
        L <<= 1;
        __syncthreads();
        if (L >= span) break;
        if (merger) {
            const int run = e / L;
            const int pos = e + run * MK;  // a multiple of MK: one padded block
#pragma unroll
            for (int j = 0; j < MK; ++j) s[lds_idx<T>(pos + j)] = o[j];
            if ((e % L) == L - MK) {
#pragma unroll
                for (int j = 0; j < MK; ++j) s[lds_idx<T>(pos + MK + j)] = key_max<T>();
            }
        }
        __syncthreads();
    }
}

// Smallest power of two >= max(n, lo).
__device__ __forceinline__ int span_for(int n, int lo) {
    int s = lo;
    while (s < n) s <<= 1;
    return s;
}

}  // namespace msn
