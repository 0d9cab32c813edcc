// Four-way global merge passes for integer keys-only flat sorts: each pass
// merges groups of four sorted runs of length L into runs of 4L, reading and
// writing every key once -- half the HBM sweeps of binary passes.
//
// Output tiles are cut at sampled splitters rather than at fixed output
// positions, so no tile needs a four-sequence co-rank search:
//   1. the chunk samples of the input (the first key of every 256-key chunk,
//      left by the previous sweep) are runs of L/256 sorted keys; k_m4_bounds
//      ranks every sample in its group's total order (key, run, position) by
//      binary searches of the other runs' samples;
//   2. every kM4SamplesPerTile-th sample in that order is a tile boundary; its
//      thread finds, for each of the four runs, how many of the run's keys
//      precede it (its own run: its position; earlier runs: keys <= it; later
//      runs: keys < it) by a search inside one chunk;
//   3. k_merge4 merges a tile's four slices in LDS, two binary levels, and
//      writes them at the output position the splits imply.
// Between consecutive boundaries a run contributes a contiguous slice that
// holds at most (its samples inside the tile + 1) chunks, so a tile holds at
// most (kM4SamplesPerTile + 4) * 256 - 4 keys.  Runs are stable-merged (lower
// run first on equal keys), which for keys alone only fixes the tie order.
#pragma once

#include <algorithm>
#include <type_traits>

#include "device.hpp"

namespace msn {

constexpr int kM4MaxTile = (kM4SamplesPerTile + 4) * kSampleChunk - 4;
// Word 3 of a raw (unswizzled, stride 0) buffer descriptor on CDNA: 32-bit
// data format; accesses at byte offsets >= num_records are dropped (stores)
// or return zero (loads).
constexpr int kRawBufferWord3 = 0x00020000;
constexpr int kM4Gap = 64;  // slice spacing in LDS (>= KPT sentinels, lane-aligned)
// LDS keys: the slices with their gaps, or X and Y with theirs (Y starts at a
// multiple of 32 at least KPT <= 32 past X), plus a dummy slot.
__host__ __device__ constexpr int m4_buf_keys() { return kM4MaxTile + 4 * kM4Gap + 8; }
// Level 1 needs ceil(nx/KPT) + ceil(ny/KPT) <= kM4MaxTile/KPT + 2 threads.
// LDS words: the padded buffer, or the staged output (a spare word every 16).
__host__ __device__ constexpr int m4_lds_words(int threads, int kpt) {
    return lds_words<uint32_t>(m4_buf_keys()) + 16 > threads * kpt + threads * kpt / 16 + 16
               ? lds_words<uint32_t>(m4_buf_keys()) + 16
               : threads * kpt + threads * kpt / 16 + 16;
}

// Division by a launch-invariant divisor with a multiply-high and shifts
// (Granlund and Montgomery 1994, unsigned case): for 32-bit n and d >= 1,
// q = (t + ((n - t) >> s1)) >> s2 with t = mulhi(n, mul).
struct M4Div {
    uint32_t mul, s1, s2;
};

inline M4Div m4_div(uint32_t d) {
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    const uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
    return {(uint32_t)m, l ? 1u : 0u, l ? l - 1 : 0u};
}

__device__ __forceinline__ uint32_t m4_udiv(uint32_t n, M4Div v) {
    const uint32_t t = __umulhi(n, v.mul);
    return (t + ((n - t) >> v.s1)) >> v.s2;
}

// Geometry of one four-way pass (host-computed, passed by value).
struct M4Geom {
    int64_t n;
    int64_t L;            // input run length (a multiple of the sample chunk)
    int64_t full_groups;  // groups of four full runs
    int tiles_full;       // tiles per full group
    int tiles_tail;       // tiles of the last, partial group (0 if none)
    M4Div by_tiles;       // division by tiles_full
};

__host__ __device__ inline int64_t m4_ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Number of chunk samples of group g (runs shorter than L at the array end).
__host__ __device__ inline int64_t m4_group_samples(const M4Geom& g4, int64_t g) {
    int64_t s = 0;
    for (int r = 0; r < 4; ++r) {
        const int64_t rb = g * 4 * g4.L + r * g4.L;
        const int64_t len = rb >= g4.n ? 0 : (g4.n - rb < g4.L ? g4.n - rb : g4.L);
        s += m4_ceil_div(len, kSampleChunk);
    }
    return s;
}

inline M4Geom m4_geometry(int64_t n, int64_t L) {
    M4Geom g4{n, L, n / (4 * L), 0, 0, {}};
    g4.tiles_full = (int)m4_ceil_div(4 * L / kSampleChunk, kM4SamplesPerTile);
    g4.by_tiles = m4_div((uint32_t)g4.tiles_full);
    if (n - g4.full_groups * 4 * L > 0)
        g4.tiles_tail = (int)m4_ceil_div(m4_group_samples(g4, g4.full_groups), kM4SamplesPerTile);
    return g4;
}

inline int64_t m4_tiles(const M4Geom& g4) {
    return g4.full_groups * g4.tiles_full + g4.tiles_tail;
}

inline int64_t m4_bounds(const M4Geom& g4) {
    return g4.full_groups * (g4.tiles_full + 1) + (g4.tiles_tail ? g4.tiles_tail + 1 : 0);
}

// Boundary table row of tile boundary j of group g.
__device__ __forceinline__ int64_t m4_bound_row(const M4Geom& g4, int64_t g, int64_t j) {
    return g * (g4.tiles_full + 1) + j;
}

// Tile boundaries of one four-way pass, one thread per input chunk sample.
// A sample's rank in its group's total order (key, run, position) is its
// index in its own run plus, for each other run, how many of that run's
// samples precede it (earlier runs win ties).  Samples whose rank is a
// positive multiple of kM4SamplesPerTile are the tile boundaries; their
// thread turns each run's sample count into a key count by a search inside
// one chunk and writes the boundary row: bnd[row * 4 + r] = keys of run r
// before the boundary.  The group's first sample in that order writes the
// group's rows 0 and `tiles`.  Chunks per run: 1 << lg_cl.
template <int DT>
__global__ __launch_bounds__(256) void k_m4_bounds(const uint32_t* __restrict__ in,
                                                   const uint32_t* __restrict__ samp_first,
                                                   int32_t* __restrict__ bnd, M4Geom g4,
                                                   int lg_cl, int64_t nck) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nck) return;
    constexpr int64_t G = kSampleChunk;
    const int64_t g = c >> (lg_cl + 2);
    const int r = (int)((c >> lg_cl) & 3);
    const int64_t ic = c & ((1ll << lg_cl) - 1);
    const int64_t gb = g * 4 * g4.L;
    int64_t len[4], cnt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t rb = gb + k * g4.L;
        len[k] = rb >= g4.n ? 0 : (g4.n - rb < g4.L ? g4.n - rb : g4.L);
    }
    const uint32_t ov = ord_key<DT>(samp_first[c]);
    // samples of run k before this one: a prefix of run k, found by a
    // binary search; the three searches advance in lockstep
    int64_t lo[4], hi[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        lo[k] = 0;
        hi[k] = k == r ? 0 : m4_ceil_div(len[k], G);
    }
    for (int it = 0; it <= lg_cl; ++it) {
        uint32_t x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            x[k] = lo[k] < hi[k] ? samp_first[(gb + k * g4.L) / G + ((lo[k] + hi[k]) >> 1)] : 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (lo[k] < hi[k]) {
                const int64_t mid = (lo[k] + hi[k]) >> 1;
                const uint32_t ox = ord_key<DT>(x[k]);
                if (k < r ? ox <= ov : ox < ov) lo[k] = mid + 1; else hi[k] = mid;
            }
        }
    }
    int64_t rank = ic;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        cnt[k] = k == r ? ic : lo[k];
        if (k != r) rank += lo[k];
    }
    const int64_t tiles = g < g4.full_groups ? g4.tiles_full : g4.tiles_tail;
    int32_t* row0 = bnd + m4_bound_row(g4, g, 0) * 4;
    if (rank == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            row0[k] = 0;
            row0[tiles * 4 + k] = (int32_t)len[k];
        }
        return;
    }
    if (rank % kM4SamplesPerTile != 0) return;
    int32_t* rowj = row0 + (rank / kM4SamplesPerTile) * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int64_t split;
        if (k == r) {
            split = ic * G;
        } else if (cnt[k] == 0) {
            split = 0;
        } else {
            // the key count lies in [(cnt-1) G + 1, min(cnt G, len)]
            const int64_t rb = gb + k * g4.L;
            int64_t a = (cnt[k] - 1) * G + 1;
            int64_t b = cnt[k] * G < len[k] ? cnt[k] * G : len[k];
            while (a < b) {
                const int64_t mid = (a + b) >> 1;  // is key mid (0-based) before?
                const uint32_t ox = ord_key<DT>(in[rb + mid]);
                if (k < r ? ox <= ov : ox < ov) a = mid + 1; else b = mid;
            }
            split = a;
        }
        rowj[k] = (int32_t)split;
    }
}

// Byte offset of padded LDS slot i (one spare word every 32, as lds_idx):
// 4 * (i + i / 32) in one shift and one shift-add.
__device__ __forceinline__ uint32_t m4_off(uint32_t i) {
    uint32_t r;
    asm("v_add_lshl_u32 %0, %1, %2, 2" : "=v"(r) : "v"(i), "v"(i >> 5));
    return r;
}

template <typename Key>
__device__ __forceinline__ Key m4_ld(const unsigned char* sm, uint32_t i) {
    return *reinterpret_cast<const Key*>(sm + m4_off(i));
}

// Merge path co-rank in padded LDS (A at a0, B at b0): keys of A among the
// first d outputs, A first on ties.
template <typename Key>
__device__ __forceinline__ int m4_corank(const unsigned char* sm, int a0, int la, int b0, int lb,
                                         int d) {
    int lo = d > lb ? d - lb : 0;
    int hi = d < la ? d : la;
    const int kb = b0 + d - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (!(m4_ld<Key>(sm, kb - mid) < m4_ld<Key>(sm, a0 + mid)))
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// KPT outputs of the merge of two sentinel-closed LDS runs from positions
// pa, pb.  The state is the head x of the run that gave the last output (next
// key at pc) and the head y of the other run (next key at po).  Equal keys
// may come from either run: the values are those of the stable merge, which
// is all a keys-only sort keeps.
template <typename Key, int KPT>
__device__ __forceinline__ void m4_serial(const unsigned char* sm, uint32_t pa, uint32_t pb,
                                          Key (&out)[KPT]) {
    Key x = m4_ld<Key>(sm, pa);
    Key y = m4_ld<Key>(sm, pb);
    uint32_t pc = pa + 1, po = pb + 1;
#pragma unroll
    for (int k = 0; k < KPT; ++k) {
        const bool keep = x <= y;
        out[k] = keep ? x : y;
        const Key hi = keep ? y : x;
        const uint32_t p = keep ? pc : po;
        po = keep ? po : pc;
        pc = p + 1;
        x = m4_ld<Key>(sm, p);
        y = hi;
    }
}

// Merges one tile: the four run slices between two boundaries, in one LDS
// buffer that holds, in turn, the four slices, the two level-1 results, and
// the staged output (level results pass through registers between barriers).
// Slice r sits at tile position p_r + r * kM4Gap (a multiple of 64 apart),
// so a wavefront's 64 consecutive keys that lie in one slice are read from
// one scalar base and written to LDS at one scalar offset.
template <int DT, int THREADS, int KPT>
__global__ __launch_bounds__(THREADS) void k_merge4(const uint32_t* __restrict__ in,
                                                    uint32_t* __restrict__ out,
                                                    const int32_t* __restrict__ bnd, M4Geom g4,
                                                    uint32_t* __restrict__ samp_first,
                                                    uint32_t* __restrict__ samp_last) {
    static_assert(DT == kU32 || DT == kI32, "integer keys only");
    static_assert(kM4MaxTile <= THREADS * KPT && kM4MaxTile / KPT + 2 <= THREADS, "tile fits");
    static_assert(KPT == 16 || KPT == 32, "outputs of a thread stay in one padded 32-block");
    using Key = std::conditional_t<DT == kI32, int32_t, uint32_t>;
    constexpr Key kMax = DT == kI32 ? (Key)0x7fffffff : (Key)0xffffffffu;
    constexpr int kBuf = m4_buf_keys();
    constexpr uint32_t kDummy = kBuf - 1;
    // static LDS: its base is a compile-time constant the address math folds
    __shared__ __align__(16) uint32_t lds[m4_lds_words(THREADS, KPT)];
    unsigned char* smem = reinterpret_cast<unsigned char*>(lds);
    Key* b = reinterpret_cast<Key*>(lds);

    // tile -> (group, tile of the group); grids stay below 2^31 tiles
    const uint32_t t = blockIdx.x;
    int64_t g, j;
    {
        const uint32_t q = m4_udiv(t, g4.by_tiles);
        g = q < (uint64_t)g4.full_groups ? q : g4.full_groups;
        j = (int64_t)t - g * g4.tiles_full;
    }
    const int64_t row = m4_bound_row(g4, g, j);
    const int64_t gb = g * 4 * g4.L;
    int c[4], lo[4];
    int64_t ostart = gb;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        lo[r] = bnd[row * 4 + r];
        c[r] = bnd[(row + 1) * 4 + r] - lo[r];
        ostart += lo[r];
    }
    const int p1 = c[0], p2 = p1 + c[1], p3 = p2 + c[2], cnt = p3 + c[3];
    const int tid = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t lane = (uint32_t)tid & 63u;
    const uint32_t lane4 = lane * 4u;
    const uint32_t plane = 4u * (lane + (lane >> 5));  // padded byte offset in a 64-block

    // ---- load the four slices (all loads issued before the first LDS write).
    // Wave w loads tile keys [w * 64 KPT, (w + 1) * 64 KPT).  A chunk inside
    // one slice reads from one scalar base at constant offsets; a chunk that
    // crosses a slice boundary (or the tile end) picks the slice per lane.
    {
        const int pst[4] = {0, p1, p2, p3};
        auto slice_of = [&](int x) {
            return (x >= p1 ? 1 : 0) + (x >= p2 ? 1 : 0) + (x >= p3 ? 1 : 0);
        };
        // tile key x of slice r is group key x + sh_r
        const uint32_t* gin = in + gb;
        const int64_t L = g4.L;
        const int64_t sh0 = lo[0], sh1 = L + lo[1] - p1, sh2 = 2 * L + lo[2] - p2,
                      sh3 = 3 * L + lo[3] - p3;
        const int X0 = wv * 64 * KPT;
        const int r0 = slice_of(X0), r1 = slice_of(X0 + 64 * KPT - 1);
        Key rk[KPT];
        if (X0 + 64 * KPT <= cnt && r0 == r1) {
            const int64_t sh = r0 == 0 ? sh0 : r0 == 1 ? sh1 : r0 == 2 ? sh2 : sh3;
            const char* sp = reinterpret_cast<const char*>(gin + X0 + sh) + lane4;
#pragma unroll
            for (int q = 0; q < KPT; ++q) rk[q] = *reinterpret_cast<const Key*>(sp + 256 * q);
            const uint32_t base = (uint32_t)(X0 + r0 * kM4Gap);  // a multiple of 64
            unsigned char* dp = smem + plane + 4u * (base + (base >> 5));
#pragma unroll
            for (int q = 0; q < KPT; ++q) *reinterpret_cast<Key*>(dp + 264 * q) = rk[q];
        } else if (X0 < cnt) {
            // group offsets of slice starts fit 32 bits: a group spans 4L < 2^32 keys
            const uint32_t s0 = (uint32_t)sh0, s1 = (uint32_t)sh1, s2 = (uint32_t)sh2,
                           s3 = (uint32_t)sh3;
            uint32_t pos[KPT];
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                const int x = X0 + 64 * q + (int)lane;
                const int xc = min(x, cnt - 1);
                const bool c1 = xc >= p1, c2 = xc >= p2, c3 = xc >= p3;
                const uint32_t s = c3 ? s3 : c2 ? s2 : c1 ? s1 : s0;
                const uint32_t gap = c3 ? 3 * kM4Gap : c2 ? 2 * kM4Gap : c1 ? kM4Gap : 0;
                rk[q] = (Key)gin[(uint32_t)xc + s];
                pos[q] = x < cnt ? (uint32_t)x + gap : kDummy;
            }
#pragma unroll
            for (int q = 0; q < KPT; ++q) *reinterpret_cast<Key*>(smem + m4_off(pos[q])) = rk[q];
        }
        if (tid < KPT) {
#pragma unroll
            for (int r = 0; r < 4; ++r) b[lds_idx<Key>(pst[r] + r * kM4Gap + c[r] + tid)] = kMax;
        }
    }
    __syncthreads();

    // ---- level 1: X = merge(s0, s1) at 0, Y = merge(s2, s3) at ybase
    const int nx = p2, ny = cnt - p2;
    const int ybase = (nx + KPT + 31) & ~31;
    const int tx = (nx + KPT - 1) / KPT, ty = (ny + KPT - 1) / KPT;
    {
        Key o[KPT];
        const bool in_x = tid < tx;
        const bool active = tid < tx + ty;
        const int d = in_x ? tid * KPT : (tid - tx) * KPT;
        const int sa = in_x ? 0 : p2 + 2 * kM4Gap, la = in_x ? c[0] : c[2];
        const int sb = in_x ? p1 + kM4Gap : p3 + 3 * kM4Gap, lb = in_x ? c[1] : c[3];
        const int base2 = (in_x ? 0 : ybase) + d;  // a multiple of KPT
        if (active) {
            const int i = m4_corank<Key>(smem, sa, la, sb, lb, d);
            m4_serial<Key, KPT>(smem, (uint32_t)(sa + i), (uint32_t)(sb + d - i), o);
        }
        __syncthreads();
        // outputs past the end of X (Y) are key maxima: the sentinels
        if (active) {
            Key* dst = b + (base2 + (base2 >> 5));
#pragma unroll
            for (int k = 0; k < KPT; ++k) dst[k] = o[k];
        }
        if (tid < KPT) {
            b[lds_idx<Key>(nx + tid)] = kMax;
            b[lds_idx<Key>(ybase + ny + tid)] = kMax;
        }
    }
    __syncthreads();

    // ---- level 2: merge(X, Y)
    const int d = tid * KPT;
    Key o[KPT];
    if (d < cnt) {
        const int i = m4_corank<Key>(smem, 0, nx, ybase, ny, d);
        m4_serial<Key, KPT>(smem, (uint32_t)i, (uint32_t)(ybase + d - i), o);
    }
    // stage (a spare word every 16) and store lane-contiguous words
    uint32_t* st = reinterpret_cast<uint32_t*>(smem);
    __syncthreads();
    if (d < cnt) {
        uint32_t* sd = st + (d + (d >> 4));
#pragma unroll
        for (int k = 0; k < KPT; ++k) sd[k + (k >> 4)] = (uint32_t)o[k];
    }
    __syncthreads();
    uint32_t v[KPT];
    const uint32_t* sr = st + (tid + (tid >> 4));
#pragma unroll
    for (int q = 0; q < KPT; ++q) v[q] = sr[q * (THREADS + THREADS / 16)];
    // raw buffer stores: the descriptor's byte bound (cnt keys) drops the
    // stores past the tile end, so the rows need no per-lane guard
    const __amdgpu_buffer_rsrc_t ro =
        __builtin_amdgcn_make_buffer_rsrc(out + ostart, 0, cnt * 4, kRawBufferWord3);
#pragma unroll
    for (int q = 0; q < KPT; ++q)
        __builtin_amdgcn_raw_buffer_store_b32(v[q], ro, (tid + q * THREADS) * 4, 0, 0);
    // chunk samples of the output for the next pass
    constexpr int G = kSampleChunk;
    const int f0 = (int)((G - (ostart % G)) % G);             // first chunk start in the tile
    const int l0 = (int)((2 * G - 1 - (ostart % G)) % G);     // first chunk end in the tile
    if (tid < 32) {
        const int e = f0 + tid * G;
        if (e < cnt) samp_first[(ostart + e) / G] = st[e + (e >> 4)];
    } else if (tid < 64) {
        const int e = l0 + (tid - 32) * G;
        if (e < cnt) samp_last[(ostart + e) / G] = st[e + (e >> 4)];
    }
}


}  // namespace msn
