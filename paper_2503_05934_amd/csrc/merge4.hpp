// Four-way global merge passes for integer keys-only flat sorts: each pass
// merges groups of four sorted runs of length L into runs of 4L, reading and
// writing every key once -- half the HBM sweeps of binary passes.
//
// Output tiles are cut at sampled splitters rather than at fixed output
// positions, so no tile needs a four-sequence co-rank search:
//   1. the chunk samples of the input (the first key of every 256-key chunk,
//      left by the previous sweep) are runs of L/256 sorted keys; two binary
//      merge passes over them (payload = chunk index) put each group's samples
//      in total order (key, run, position);
//   2. every kM4SamplesPerTile-th merged sample is a tile boundary; k_m4_split
//      finds, for each of the four runs, how many of its keys precede it
//      (its own run: its position; earlier runs: keys <= it; later runs:
//      keys < it), searching the run's chunk samples first;
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

constexpr int kM4Threads = 512;
constexpr int kM4KPT = 16;
constexpr int kM4MaxTile = (kM4SamplesPerTile + 4) * kSampleChunk - 4;
static_assert(kM4MaxTile <= kM4Threads * kM4KPT, "a tile fits one workgroup");
// level 1 needs ceil(nx/KPT) + ceil(ny/KPT) <= kMaxTile/KPT + 2 threads
static_assert(kM4MaxTile / kM4KPT + 2 <= kM4Threads, "level-1 threads fit");

// Geometry of one four-way pass (host-computed, passed by value).
struct M4Geom {
    int64_t n;
    int64_t L;            // input run length (a multiple of the sample chunk)
    int64_t full_groups;  // groups of four full runs
    int tiles_full;       // tiles per full group
    int tiles_tail;       // tiles of the last, partial group (0 if none)
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
    M4Geom g4{n, L, n / (4 * L), 0, 0};
    g4.tiles_full = (int)m4_ceil_div(4 * L / kSampleChunk, kM4SamplesPerTile);
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

__global__ void k_iota(uint32_t* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (uint32_t)i;
}

// Splits of every tile boundary: one thread per (boundary, run).
// mkeys/mpay: each group's samples in total order, payload = global chunk
// index.  bnd[row * 4 + r] = keys of run r before the boundary.
template <int DT>
__global__ __launch_bounds__(256) void k_m4_split(const uint32_t* __restrict__ in,
                                                  const uint32_t* __restrict__ samp_first,
                                                  const uint32_t* __restrict__ mkeys,
                                                  const uint32_t* __restrict__ mpay,
                                                  int32_t* __restrict__ bnd, M4Geom g4,
                                                  int64_t nbounds) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nbounds * 4) return;
    const int64_t row = gid >> 2;
    const int r = (int)(gid & 3);
    int64_t g, j, tiles;
    if (row < g4.full_groups * (g4.tiles_full + 1)) {
        g = row / (g4.tiles_full + 1);
        j = row % (g4.tiles_full + 1);
        tiles = g4.tiles_full;
    } else {
        g = g4.full_groups;
        j = row - g4.full_groups * (g4.tiles_full + 1);
        tiles = g4.tiles_tail;
    }
    constexpr int64_t G = kSampleChunk;
    const int64_t gb = g * 4 * g4.L;
    const int64_t rb = gb + r * g4.L;
    const int64_t len = rb >= g4.n ? 0 : (g4.n - rb < g4.L ? g4.n - rb : g4.L);
    int64_t split;
    if (j == 0) {
        split = 0;
    } else if (j == tiles) {
        split = len;
    } else {
        const int64_t idx = gb / G + j * kM4SamplesPerTile;
        const uint32_t v = mkeys[idx];
        const int64_t pos = (int64_t)mpay[idx] * G;          // the splitter's position
        const int rs = (int)((pos - gb) / g4.L);
        if (r == rs) {
            split = pos - rb;
        } else {
            // keys of run r ordered before the splitter: earlier runs win ties
            const bool le = r < rs;
            const uint32_t ov = ord_key<DT>(v);
            auto before = [&](uint32_t x) {
                const uint32_t ox = ord_key<DT>(x);
                return le ? ox <= ov : ox < ov;
            };
            // chunks whose first key is before the splitter: a prefix of run r
            const int64_t nck = m4_ceil_div(len, G);
            int64_t lo = 0, hi = nck;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (before(samp_first[rb / G + mid])) lo = mid + 1; else hi = mid;
            }
            if (lo == 0) {
                split = 0;
            } else {
                // the count lies in [(lo-1)*G + 1, min(lo*G, len)]
                int64_t a = (lo - 1) * G + 1;
                int64_t b = lo * G < len ? lo * G : len;
                while (a < b) {
                    const int64_t mid = (a + b) >> 1;   // is key mid (0-based) before?
                    if (before(in[rb + mid])) a = mid + 1; else b = mid;
                }
                split = a;
            }
        }
    }
    bnd[row * 4 + r] = (int32_t)split;
}

// Merges one tile: the four run slices between two boundaries, in one LDS
// buffer that holds, in turn, the four slices, the two level-1 results, and
// the staged output (level results pass through registers between barriers).
template <int DT>
__global__ __launch_bounds__(kM4Threads) void k_merge4(const uint32_t* __restrict__ in,
                                                       uint32_t* __restrict__ out,
                                                       const int32_t* __restrict__ bnd,
                                                       M4Geom g4,
                                                       uint32_t* __restrict__ samp_first,
                                                       uint32_t* __restrict__ samp_last) {
    static_assert(DT == kU32 || DT == kI32, "integer keys only");
    using Key = std::conditional_t<DT == kI32, int32_t, uint32_t>;
    constexpr Key kMax = DT == kI32 ? (Key)0x7fffffff : (Key)0xffffffffu;
    constexpr int KPT = kM4KPT;
    constexpr int kBuf = kM4MaxTile + 4 * KPT + 8;  // keys + sentinels, unpadded
    extern __shared__ __align__(16) unsigned char smem[];
    Key* b = reinterpret_cast<Key*>(smem);

    const int64_t t = blockIdx.x;
    int64_t g, j;
    if (t < g4.full_groups * g4.tiles_full) {
        g = t / g4.tiles_full;
        j = t % g4.tiles_full;
    } else {
        g = g4.full_groups;
        j = t - g4.full_groups * g4.tiles_full;
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
    const int o1 = c[0] + KPT, o2 = o1 + c[1] + KPT, o3 = o2 + c[2] + KPT;  // slice offsets
    const int tid = threadIdx.x;

    // load the four slices (every load issued before the first LDS write).
    // Tile element x of slice r sits at group offset x + sh[r] (32-bit: a
    // group spans 4L <= 2^31 keys).
    {
        const uint32_t* gin = in + gb;
        const uint32_t L32 = (uint32_t)g4.L;
        const uint32_t sh[4] = {(uint32_t)lo[0], L32 + lo[1] - p1, 2 * L32 + lo[2] - p2,
                                3 * L32 + lo[3] - p3};
        Key rk[KPT];
        int pos[KPT];
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const int x = tid + q * kM4Threads;
            const int xc = min(x, cnt - 1);
            const int r = (xc >= p1 ? 1 : 0) + (xc >= p2 ? 1 : 0) + (xc >= p3 ? 1 : 0);
            const uint32_t s = r == 0 ? sh[0] : r == 1 ? sh[1] : r == 2 ? sh[2] : sh[3];
            rk[q] = (Key)gin[(uint32_t)xc + s];
            pos[q] = x < cnt ? x + r * KPT : kBuf - 1;
        }
#pragma unroll
        for (int q = 0; q < KPT; ++q) b[lds_idx<Key>(pos[q])] = rk[q];
        if (tid < KPT) {
            b[lds_idx<Key>(c[0] + tid)] = kMax;
            b[lds_idx<Key>(o1 + c[1] + tid)] = kMax;
            b[lds_idx<Key>(o2 + c[2] + tid)] = kMax;
            b[lds_idx<Key>(o3 + c[3] + tid)] = kMax;
        }
    }
    __syncthreads();

    // level 1: X = merge(s0, s1), Y = merge(s2, s3); then b = [X | max.. | Y | max..]
    const int nx = p2, ny = cnt - p2;
    const int tx = (nx + KPT - 1) / KPT, ty = (ny + KPT - 1) / KPT;
    {
        // one code path for both halves: per-thread run parameters
        Key o[KPT];
        const bool in_x = tid < tx;
        const bool active = tid < tx + ty;
        const int d = in_x ? tid * KPT : (tid - tx) * KPT;
        const int sa = in_x ? 0 : o2, la = in_x ? c[0] : c[2];
        const int sb = in_x ? o1 : o3, lb = in_x ? c[1] : c[3];
        const int base2 = in_x ? 0 : nx + KPT;
        const int lim = active ? (in_x ? nx : ny) : 0;
        if (active) {
            const int i = corank_lds(b, sa, la, sb, lb, d, PlainLess{});
            serial_merge_closed<Key, KPT>(b, sa + i, sb + d - i, o);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KPT; ++k) {
            const int pos = d + k < lim ? base2 + d + k : kBuf - 1;
            b[lds_idx<Key>(pos)] = o[k];
        }
        if (tid < KPT) {
            b[lds_idx<Key>(nx + tid)] = kMax;
            b[lds_idx<Key>(nx + KPT + ny + tid)] = kMax;
        }
    }
    __syncthreads();

    // level 2: merge(X, Y)
    const int d = tid * KPT;
    Key o[KPT];
    if (d < cnt) {
        const int i = corank_lds(b, 0, nx, nx + KPT, ny, d, PlainLess{});
        serial_merge_closed<Key, KPT>(b, i, nx + KPT + d - i, o);
    }
    // stage (a spare word every 16) and store lane-contiguous words
    uint32_t* st = reinterpret_cast<uint32_t*>(smem);
    __syncthreads();
    if (d < cnt) {
#pragma unroll
        for (int k = 0; k < KPT; ++k) st[(d + k) + ((d + k) >> 4)] = (uint32_t)o[k];
    }
    __syncthreads();
    uint32_t* dst = out + ostart;
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
        const int e = tid + q * kM4Threads;
        if (e < cnt) dst[e] = st[e + (e >> 4)];
    }
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

inline size_t m4_lds_bytes() {
    constexpr int kBuf = kM4MaxTile + 4 * kM4KPT + 8;
    const size_t one = (size_t)(lds_words<uint32_t>(kBuf) + 16) * 4;
    const size_t stage = (size_t)(kM4Threads * kM4KPT + kM4Threads * kM4KPT / 16 + 16) * 4;
    return one > stage ? one : stage;
}

}  // namespace msn
