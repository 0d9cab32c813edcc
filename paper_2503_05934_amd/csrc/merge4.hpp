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
// Cache policy of the passes' output row stores: nontemporal.  The rows
// start at 64-word boundaries of the output, so every 256-byte store of a
// wavefront covers two whole cache lines; the next pass's boundary search,
// which reads the chunk samples and a few keys, then finds more of them in
// the caches.
constexpr int kM4StoreNt = 2;
// Output rows of `threads` words that a tile (plus up to 63 words of
// alignment) can touch.
__host__ __device__ constexpr int m4_out_rows(int threads) {
    return (kM4MaxTile + 63 + threads - 1) / threads;
}
constexpr int kM4Gap = 64;  // slice spacing in LDS (> kM4Sent sentinels, lane-aligned)
constexpr int kM4Sent = 32;  // outputs per thread of the merge levels = sentinels per run
// LDS keys: the slices with their gaps, or X and Y with theirs (Y starts at a
// multiple of 32 at least KPT <= 32 past X), plus a dummy slot.
__host__ __device__ constexpr int m4_buf_keys() { return kM4MaxTile + 4 * kM4Gap + 8; }
// Level 1 needs ceil(nx/KPT) + ceil(ny/KPT) <= kM4MaxTile/KPT + 2 threads.
// LDS words: the padded buffer, or the staged output (a spare word every 32).
__host__ __device__ constexpr int m4_lds_words(int threads) {
    return lds_words<uint32_t>(m4_buf_keys()) + 16 >
                   m4_out_rows(threads) * threads + m4_out_rows(threads) * threads / 32 + 16
               ? lds_words<uint32_t>(m4_buf_keys()) + 16
               : m4_out_rows(threads) * threads + m4_out_rows(threads) * threads / 32 + 16;
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
    const int* skip;      // *skip set: the input is already sorted, the pass returns at once
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
    M4Geom g4{n, L, n / (4 * L), 0, 0, {}, nullptr};
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

// Tile boundaries of one four-way pass.  A chunk sample's rank in its
// group's total order (key, run, position) is its index in its own run plus,
// for each other run, how many of that run's samples precede it (earlier runs
// win ties).  Samples whose rank is a positive multiple of kM4SamplesPerTile
// are the tile boundaries; their thread turns each run's sample count into a
// key count by a search inside one chunk and writes the boundary row:
// bnd[row * 4 + r] = keys of run r before the boundary.  The group's first
// sample in that order writes the group's rows 0 and `tiles`.
struct M4Group {
    int64_t gb;       // first key of the group
    int64_t len[4];   // run lengths (short or empty runs at the array end)
    int64_t smp[4];   // chunk samples per run
    int64_t tiles;    // tiles of the group
};

__device__ __forceinline__ M4Group m4_group(const M4Geom& g4, int64_t g) {
    M4Group q;
    q.gb = g * 4 * g4.L;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t rb = q.gb + k * g4.L;
        q.len[k] = rb >= g4.n ? 0 : (g4.n - rb < g4.L ? g4.n - rb : g4.L);
        q.smp[k] = m4_ceil_div(q.len[k], kSampleChunk);
    }
    q.tiles = g < g4.full_groups ? g4.tiles_full : g4.tiles_tail;
    return q;
}

// a[k] for a run index known only at run time, without local-memory indexing
__device__ __forceinline__ int64_t m4_sel(const int64_t (&a)[4], int k) {
    return k == 0 ? a[0] : k == 1 ? a[1] : k == 2 ? a[2] : a[3];
}

// Is a key (order-mapped) of run k ordered before the sample ov of run r?
__device__ __forceinline__ bool m4_before(uint32_t ox, uint32_t ov, int k, int r) {
    return k < r ? ox <= ov : ox < ov;
}

// Keys of run `run` (len keys) before the sample, given that `cnt` of the
// run's chunk samples precede it: the count lies in [(cnt-1) G + 1,
// min(cnt G, len)].  Three rounds of independent loads narrow it: the last
// key of each 64-key block (4 loads), of each 16-key block inside the block
// found (4 loads), then the 16 keys of the block found.  Most of a chunk's
// cache lines are never fetched (the search reads about two thirds of the
// lines that reading every 16th key would).
template <int DT>
__device__ int64_t m4_key_count(const uint32_t* __restrict__ run, int64_t len, int64_t cnt,
                                uint32_t ov, int k, int r) {
    constexpr int64_t G = kSampleChunk;
    static_assert(G == 256, "three rounds of 64, 16 and 1 cover one chunk");
    if (cnt == 0) return 0;
    const int64_t A = (cnt - 1) * G + 1;
    const int64_t B = cnt * G < len ? cnt * G : len;
    // indices are clamped to B - 1 (>= A - 1, a valid key) so that the loads
    // of a round issue together; results past B are masked off
    int64_t a = A;
#pragma unroll
    for (int step = 64; step >= 16; step >>= 2) {
        uint32_t x[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int64_t idx = a + step * m + step - 1;
            x[m] = run[idx < B ? idx : B - 1];
        }
        int full = 0;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            full += (int)((a + step * m + step - 1 < B) & m4_before(ord_key<DT>(x[m]), ov, k, r));
        a += step * full;
    }
    uint32_t x[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) x[u] = run[a + u < B ? a + u : B - 1];
    int part = 0;
#pragma unroll
    for (int u = 0; u < 16; ++u)
        part += (int)((a + u < B) & m4_before(ord_key<DT>(x[u]), ov, k, r));
    return a + part;
}

// Number of entries of the sorted (order-mapped) LDS array s[0, n) ordered
// before ov under the tie rule of runs k and r.
__device__ __forceinline__ int m4_lds_count(const uint32_t* s, int n, uint32_t ov, int k, int r) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (m4_before(s[mid], ov, k, r)) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Three such counts at once, over s_j[0, m_j) with every m_j < 2^(lgmax+1):
// binary lifting with one step size for all three, so their LDS reads are
// in flight together.  k_j: the run of array j; r: the run of ov.  Each
// array has a readable word before it (s_j[-1]).  An entry x is before ov
// when x < ov + (k_j < r), compared in 64 bits.
__device__ __forceinline__ void m4_lds_count3(const uint32_t* (&s)[3], const int (&m)[3],
                                              const int (&k)[3], uint32_t ov, int r, int lgmax,
                                              int (&c)[3]) {
    int p[3] = {0, 0, 0};
    uint64_t thr[3];
    const uint32_t* base[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        thr[j] = (uint64_t)ov + (k[j] < r ? 1u : 0u);
        base[j] = s[j] - 1;
    }
    for (int b = 1 << lgmax; b > 0; b >>= 1) {
        uint32_t x[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) x[j] = base[j][min(p[j] + b, m[j])];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int q = p[j] + b;
            p[j] = ((q <= m[j]) & ((uint64_t)x[j] < thr[j])) ? q : p[j];
        }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) c[j] = p[j];
}

// Both boundary kernels rank kM4BoundsBlock samples per workgroup in LDS,
// collect the boundary samples in an LDS list, and then refine all
// (boundary, run) pairs at once, one per thread.
constexpr int kM4BoundsBlock = 1024;
constexpr int kM4MaxCuts = 64;  // boundaries per workgroup: 1024 / 27 + one per group
constexpr int kM4SmallRun = 256;  // runs of at most this many chunks: small kernel

struct M4Cut {
    int64_t g, ic, rank;
    int64_t cnt[4];
    uint32_t ov;
    int r;
};

// Key count of run k before boundary sample c, written to its row.
template <int DT>
__device__ __forceinline__ void m4_split_one(const uint32_t* __restrict__ in,
                                             int32_t* __restrict__ bnd, const M4Geom& g4,
                                             const M4Cut& c, int k) {
    const M4Group q = m4_group(g4, c.g);
    const int64_t split =
        k == c.r ? c.ic * kSampleChunk
                 : m4_key_count<DT>(in + q.gb + k * g4.L, m4_sel(q.len, k), m4_sel(c.cnt, k),
                                    c.ov, k, c.r);
    // ranks stay below 2^23 (n < 2^31 keys): 32-bit division
    bnd[(m4_bound_row(g4, c.g, 0) + (uint32_t)c.rank / kM4SamplesPerTile) * 4 + k] = (int32_t)split;
}

// Records a ranked sample: the group's first sample writes rows 0 and
// `tiles` at once; boundary samples go to the list (or, past its capacity,
// are refined on the spot).
template <int DT>
__device__ __forceinline__ void m4_note(const uint32_t* __restrict__ in,
                                        int32_t* __restrict__ bnd, const M4Geom& g4, int64_t g,
                                        const M4Group& q, int r, int64_t ic, uint32_t ov,
                                        int64_t rank, const int64_t (&cnt)[4], M4Cut* cuts,
                                        int* ncut) {
    if (rank == 0) {
        int32_t* row0 = bnd + m4_bound_row(g4, g, 0) * 4;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            row0[k] = 0;
            row0[q.tiles * 4 + k] = (int32_t)q.len[k];
        }
    } else if ((uint32_t)rank % kM4SamplesPerTile == 0) {
        M4Cut c;
        c.g = g;
        c.ic = ic;
        c.rank = rank;
#pragma unroll
        for (int k = 0; k < 4; ++k) c.cnt[k] = cnt[k];
        c.ov = ov;
        c.r = r;
        const int e = atomicAdd(ncut, 1);
        if (e < kM4MaxCuts) {
            cuts[e] = c;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) m4_split_one<DT>(in, bnd, g4, c, k);
        }
    }
}

// The listed (boundary, run) pairs, one per thread.
template <int DT>
__device__ __forceinline__ void m4_refine(const uint32_t* __restrict__ in,
                                          int32_t* __restrict__ bnd, const M4Geom& g4,
                                          const M4Cut* cuts, int ncut) {
    const int e = threadIdx.x >> 2, k = threadIdx.x & 3;
    if (e < ncut && e < kM4MaxCuts) m4_split_one<DT>(in, bnd, g4, cuts[e], k);
}

// Groups of at most kM4SmallRun chunks per run: each workgroup ranks the
// samples of kM4BoundsBlock / (4 CL) whole groups against each other in LDS.
template <int DT>
__global__ __launch_bounds__(256) void k_m4_bounds_small(const uint32_t* __restrict__ in,
                                                         const uint32_t* __restrict__ samp_first,
                                                         int32_t* __restrict__ bnd, M4Geom g4,
                                                         int lg_cl, int64_t nck) {
    const int skip = *g4.skip;  // tested once the sample loads are in flight
    __shared__ uint32_t smp_g[1 + kM4BoundsBlock];  // a guard word, then the samples
    __shared__ M4Cut cuts[kM4MaxCuts];
    __shared__ int ncut;
    uint32_t* smp = smp_g + 1;
    const int CL = 1 << lg_cl, GS = 4 * CL;
    const int gpw = kM4BoundsBlock / GS;
    const int64_t c0 = (int64_t)blockIdx.x * kM4BoundsBlock;
    const int nh = (int)(nck - c0 < kM4BoundsBlock ? nck - c0 : kM4BoundsBlock);
    if (threadIdx.x == 0) ncut = 0;
    for (int i = threadIdx.x; i < nh; i += blockDim.x) smp[i] = ord_key<DT>(samp_first[c0 + i]);
    if (skip) return;  // the input is already sorted
    __syncthreads();
    for (int i = threadIdx.x; i < nh; i += blockDim.x) {
        const int gl = i / GS, j = i - gl * GS;
        const int64_t g = (int64_t)blockIdx.x * gpw + gl;
        const M4Group q = m4_group(g4, g);
        const int r = j >> lg_cl;
        const int64_t ic = j & (CL - 1);
        const uint32_t ov = smp[i];
        const uint32_t* gs = smp + gl * GS;  // the group's runs: k CL apart
        const int o[3] = {r == 0 ? 1 : 0, r <= 1 ? 2 : 1, r <= 2 ? 3 : 2};  // the other runs
        const uint32_t* sa[3] = {gs + o[0] * CL, gs + o[1] * CL, gs + o[2] * CL};
        const int ma[3] = {(int)m4_sel(q.smp, o[0]), (int)m4_sel(q.smp, o[1]),
                           (int)m4_sel(q.smp, o[2])};
        int cj[3];
        m4_lds_count3(sa, ma, o, ov, r, lg_cl, cj);
        int64_t cnt[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            cnt[k] = k == r ? ic : k == o[0] ? cj[0] : k == o[1] ? cj[1] : cj[2];
        const int64_t rank = ic + cj[0] + cj[1] + cj[2];
        m4_note<DT>(in, bnd, g4, g, q, r, ic, ov, rank, cnt, cuts, &ncut);
    }
    __syncthreads();
    m4_refine<DT>(in, bnd, g4, cuts, ncut);
}

// Larger groups: each workgroup ranks min(kM4BoundsBlock, CL) consecutive
// samples of one run (CL, the run's chunk count, is a power of two).  For
// each other run, every cs-th sample (cs = 256, or more for runs of over
// 2^19 chunks, so that at most kM4Window are taken) is staged in LDS, which
// brackets the block's counts to within cs-sample steps; the bracket (up to
// kM4Window samples) is staged next and every count is finished in LDS.
// Wider brackets (skewed inputs) are searched in global memory.
constexpr int kM4Window = 2048;
static_assert(kM4Window < (2 << 11), "window counts use 12 lifting steps");

template <int DT>
__global__ __launch_bounds__(256) void k_m4_bounds_large(const uint32_t* __restrict__ in,
                                                         const uint32_t* __restrict__ samp_first,
                                                         int32_t* __restrict__ bnd, M4Geom g4,
                                                         int lg_cl, int64_t nck) {
    const int skip = *g4.skip;  // tested once the sample loads are in flight
    __shared__ uint32_t vs[kM4BoundsBlock];
    __shared__ uint32_t stage_g[3][1 + kM4Window];  // guard word + coarse samples / window
    __shared__ M4Cut cuts[kM4MaxCuts];
    __shared__ int64_t brk[6];
    __shared__ int ncut;
    const int tid = threadIdx.x;
    const int bs = lg_cl < 10 ? 1 << lg_cl : kM4BoundsBlock;
    const int lg_cs = lg_cl > 19 ? lg_cl - 11 : 8;  // coarse stride: at most 2^11 per run
    const int64_t cs = 1ll << lg_cs;
    const int64_t c0 = (int64_t)blockIdx.x * bs;
    const int64_t g = c0 >> (lg_cl + 2);
    const int r = (int)((c0 >> lg_cl) & 3);
    const int64_t ic0 = c0 & ((1ll << lg_cl) - 1);
    const M4Group q = m4_group(g4, g);
    const int nh = (int)(nck - c0 < bs ? nck - c0 : bs);
    const int o[3] = {r == 0 ? 1 : 0, r <= 1 ? 2 : 1, r <= 2 ? 3 : 2};  // the other runs
    int64_t nsm[3];
    const uint32_t* rs[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        nsm[j] = m4_sel(q.smp, o[j]);
        rs[j] = samp_first + (q.gb + o[j] * g4.L) / kSampleChunk;
    }
    if (tid == 0) ncut = 0;
    for (int i = tid; i < nh; i += 256) vs[i] = ord_key<DT>(samp_first[c0 + i]);
    // every cs-th sample of each other run
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int nc = (int)m4_ceil_div(nsm[j], cs);
        for (int i = tid; i < nc; i += 256) (stage_g[j] + 1)[i] = ord_key<DT>(rs[j][(int64_t)i << lg_cs]);
    }
    if (skip) return;  // the input is already sorted
    __syncthreads();
    // brackets: with c coarse samples before v, the count lies in
    // [(c - 1) cs + 1, min(c cs, n)] (or is 0 when c == 0)
    if (tid < 6) {
        const int j = tid >> 1;
        const uint32_t ov = vs[(tid & 1) ? nh - 1 : 0];
        const int nc = (int)m4_ceil_div(nsm[j], cs);
        const int64_t c = m4_lds_count((stage_g[j] + 1), nc, ov, o[j], r);
        brk[tid] = (tid & 1) ? (c * cs < nsm[j] ? c * cs : nsm[j])
                             : (c == 0 ? 0 : (c - 1) * cs + 1);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int64_t lo = brk[2 * j], hi = brk[2 * j + 1];
        if (hi - lo <= kM4Window)
            for (int i = tid; i < hi - lo; i += 256) (stage_g[j] + 1)[i] = ord_key<DT>(rs[j][lo + i]);
    }
    __syncthreads();
    const bool narrow = brk[1] - brk[0] <= kM4Window && brk[3] - brk[2] <= kM4Window &&
                        brk[5] - brk[4] <= kM4Window;
    for (int i = tid; i < nh; i += 256) {
        const uint32_t ov = vs[i];
        const int64_t ic = ic0 + i;
        int64_t cj[3];
        int64_t rank = ic;
        if (narrow) {  // all three brackets staged: counts in lockstep
            const uint32_t* sa[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) sa[j] = stage_g[j] + 1;
            const int ma[3] = {(int)(brk[1] - brk[0]), (int)(brk[3] - brk[2]),
                               (int)(brk[5] - brk[4])};
            int c3[3];
            m4_lds_count3(sa, ma, o, ov, r, 11, c3);
#pragma unroll
            for (int j = 0; j < 3; ++j) cj[j] = brk[2 * j] + c3[j];
            rank += cj[0] + cj[1] + cj[2];
        } else {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int64_t lo = brk[2 * j], hi = brk[2 * j + 1];
            if (hi - lo <= kM4Window) {
                cj[j] = lo + m4_lds_count((stage_g[j] + 1), (int)(hi - lo), ov, o[j], r);
            } else {
                int64_t a = lo, b = hi;
                while (a < b) {
                    const int64_t mid = (a + b) >> 1;
                    if (m4_before(ord_key<DT>(rs[j][mid]), ov, o[j], r)) a = mid + 1; else b = mid;
                }
                cj[j] = a;
            }
            rank += cj[j];
        }
        }
        int64_t cnt[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            cnt[k] = k == r ? ic : k == o[0] ? cj[0] : k == o[1] ? cj[1] : cj[2];
        m4_note<DT>(in, bnd, g4, g, q, r, ic, ov, rank, cnt, cuts, &ncut);
    }
    __syncthreads();
    m4_refine<DT>(in, bnd, g4, cuts, ncut);
}

// LDS slots of the merge kernel: one spare word every 2^kM4PadShift, so that
// the merge-path threads (whose runs start about 16 keys apart) begin on
// distinct banks.
constexpr int kM4PadShift = 5;
__host__ __device__ constexpr uint32_t m4_idx(uint32_t i) { return i + (i >> kM4PadShift); }
constexpr int kWin = 4 * (int)m4_idx(64);  // bytes between windows of 64 keys (64-aligned)
static_assert(kM4PadShift == 5 || kM4PadShift == 6, "padding: every 32 or 64 words");

// Byte offset of padded slot i, 4 * m4_idx(i), in one shift and one shift-add.
__device__ __forceinline__ uint32_t m4_off(uint32_t i) {
    uint32_t r;
    asm("v_add_lshl_u32 %0, %1, %2, 2" : "=v"(r) : "v"(i), "v"(i >> kM4PadShift));
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
// gin: the group's first key (run r starts L keys after run r - 1); slice r
// is gin[r * L + lo[r], + c[r]); the tile's outputs go to out[ostart, ostart
// + sum c).  SAMPLES: also record the output's chunk samples for the next
// pass.  lds: m4_lds_words(THREADS) words of static LDS.
template <int DT, int THREADS, int KPT, bool SAMPLES>
__device__ __forceinline__ void m4_merge_tile(const uint32_t* __restrict__ gin, int64_t L,
                                              const int (&lo)[4], const int (&c)[4],
                                              uint32_t* __restrict__ out, int64_t ostart,
                                              uint32_t* __restrict__ samp_first,
                                              uint32_t* __restrict__ samp_last, uint32_t* lds) {
    static_assert(DT == kU32 || DT == kI32, "integer keys only");
    static_assert(kM4MaxTile <= THREADS * KPT, "tile fits");
    static_assert(KPT == 16 || KPT == 32, "outputs of a thread stay in one padded 32-block");
    using Key = std::conditional_t<DT == kI32, int32_t, uint32_t>;
    constexpr Key kMax = DT == kI32 ? (Key)0x7fffffff : (Key)0xffffffffu;
    constexpr int kBuf = m4_buf_keys();
    constexpr uint32_t kDummy = kBuf - 1;
    unsigned char* smem = reinterpret_cast<unsigned char*>(lds);
    Key* b = reinterpret_cast<Key*>(lds);
    const int p1 = c[0], p2 = p1 + c[1], p3 = p2 + c[2], cnt = p3 + c[3];
    const int tid = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t lane = (uint32_t)tid & 63u;
    const uint32_t lane4 = lane * 4u;
    const uint32_t plane = 4u * m4_idx(lane);  // padded byte offset in a 64-key window

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
            unsigned char* dp = smem + plane + 4u * m4_idx(base);
#pragma unroll
            for (int q = 0; q < KPT; ++q) *reinterpret_cast<Key*>(dp + kWin * q) = rk[q];
        } else if (X0 + 64 * KPT <= cnt && r1 == r0 + 1) {
            // one boundary P (chunk offset) inside: slice r0 before it, r1 from
            // it.  Windows of 64 keys wholly on one side read one scalar base
            // at constant offsets; only window P / 64 picks per lane.
            const int P = __builtin_amdgcn_readfirstlane((r1 == 1 ? p1 : r1 == 2 ? p2 : p3) - X0);
            const int qb = P >> 6;
            const int64_t sa = r0 == 0 ? sh0 : r0 == 1 ? sh1 : sh2;
            const int64_t sb = r1 == 1 ? sh1 : r1 == 2 ? sh2 : sh3;
            const char* spa = reinterpret_cast<const char*>(gin + X0 + sa) + lane4;
            const char* spb = reinterpret_cast<const char*>(gin + X0 + sb) + lane4;
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                if (q < qb) {
                    rk[q] = *reinterpret_cast<const Key*>(spa + 256 * q);
                } else if (q > qb) {
                    rk[q] = *reinterpret_cast<const Key*>(spb + 256 * q);
                } else {
                    const int e = 64 * q + (int)lane;
                    rk[q] = *reinterpret_cast<const Key*>((e >= P ? spb : spa) + 256 * q);
                }
            }
            const uint32_t ga = (uint32_t)(X0 + r0 * kM4Gap);  // multiples of 64
            const uint32_t gb2 = ga + kM4Gap;
            unsigned char* dpa = smem + plane + 4u * m4_idx(ga);
            unsigned char* dpb = smem + plane + 4u * m4_idx(gb2);
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                const int e = 64 * q + (int)lane;
                unsigned char* dp = q < qb ? dpa : q > qb ? dpb : (e >= P ? dpb : dpa);
                *reinterpret_cast<Key*>(dp + kWin * q) = rk[q];
            }
        } else if (X0 < cnt && r0 == slice_of(cnt - 1)) {
            // the tile's last chunk, inside one slice: full windows read one
            // scalar base; the window holding the tile end checks each lane
            const int E = __builtin_amdgcn_readfirstlane(cnt - X0);  // 1 .. 64 KPT - 1
            const int qe = E >> 6;
            const int64_t sh = r0 == 0 ? sh0 : r0 == 1 ? sh1 : r0 == 2 ? sh2 : sh3;
            const char* sp = reinterpret_cast<const char*>(gin + X0 + sh) + lane4;
            const uint32_t base = (uint32_t)(X0 + r0 * kM4Gap);  // a multiple of 64
            unsigned char* dp = smem + plane + 4u * m4_idx(base);
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                if (q < qe) {
                    rk[q] = *reinterpret_cast<const Key*>(sp + 256 * q);
                } else if (q == qe) {
                    const int e = min(64 * q + (int)lane, E - 1);
                    rk[q] = *reinterpret_cast<const Key*>(sp - lane4 + 4 * e);
                }
            }
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                if (q < qe) {
                    *reinterpret_cast<Key*>(dp + kWin * q) = rk[q];
                } else if (q == qe && 64 * q + (int)lane < E) {
                    *reinterpret_cast<Key*>(dp + kWin * q) = rk[q];
                }
            }
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
        // kM4Sent copies of the maximum close every slice (the merge levels
        // take up to kM4Sent outputs per thread)
        if (tid < kM4Sent) {
#pragma unroll
            for (int r = 0; r < 4; ++r) b[m4_idx(pst[r] + r * kM4Gap + c[r] + tid)] = kMax;
        }
    }
    __syncthreads();

    // ---- level 1: X = merge(s0, s1) at 0, Y = merge(s2, s3) at ybase.  Both
    // merge levels give MK = 32 outputs to each of the first tiles/32 threads
    // (one co-rank search per 32 outputs); the others wait at the barriers.
    constexpr int MK = kM4Sent;
    static_assert(kM4MaxTile / MK + 2 <= THREADS && kM4Gap > MK, "merge shape");
    const int nx = p2, ny = cnt - p2;
    const int ybase = (nx + MK + 31) & ~31;
    const int tx = (nx + MK - 1) / MK, ty = (ny + MK - 1) / MK;
    {
        Key o[MK];
        const bool in_x = tid < tx;
        const bool active = tid < tx + ty;
        const int d = in_x ? tid * MK : (tid - tx) * MK;
        const int sa = in_x ? 0 : p2 + 2 * kM4Gap, la = in_x ? c[0] : c[2];
        const int sb = in_x ? p1 + kM4Gap : p3 + 3 * kM4Gap, lb = in_x ? c[1] : c[3];
        const int base2 = (in_x ? 0 : ybase) + d;  // a multiple of 32
        if (active) {
            const int i = m4_corank<Key>(smem, sa, la, sb, lb, d);
            m4_serial<Key, MK>(smem, (uint32_t)(sa + i), (uint32_t)(sb + d - i), o);
        }
        __syncthreads();
        // outputs past the end of X (Y) are key maxima: the sentinels
        if (active) {
            Key* dst = b + m4_idx(base2);
#pragma unroll
            for (int k = 0; k < MK; ++k) dst[k] = o[k];
        }
        if (tid < MK) {
            b[m4_idx(nx + tid)] = kMax;
            b[m4_idx(ybase + ny + tid)] = kMax;
        }
    }
    __syncthreads();

    // ---- level 2: merge(X, Y)
    const int d = tid * MK;
    Key o[MK];
    if (d < cnt) {
        const int i = m4_corank<Key>(smem, 0, nx, ybase, ny, d);
        m4_serial<Key, MK>(smem, (uint32_t)i, (uint32_t)(ybase + d - i), o);
    }
    // stage (a spare word every 32: a thread's 32 outputs start on distinct
    // banks) and store lane-contiguous words
    uint32_t* st = reinterpret_cast<uint32_t*>(smem);
    __syncthreads();
    if (d < cnt) {
        uint32_t* sd = st + (d + (d >> 5));
#pragma unroll
        for (int k = 0; k < MK; ++k) sd[k] = (uint32_t)o[k];
    }
    __syncthreads();
    // rows begin at the 64-word boundary at or before the tile start: the
    // first `al` words of row 0 belong to the previous tile and are skipped
    const int al = (int)(ostart & 63);
    constexpr int QR = m4_out_rows(THREADS);
    uint32_t v[QR];
    {
        const int e0 = max(tid - al, 0);
        v[0] = st[e0 + (e0 >> 5)];
        const uint32_t* sr = st + m4_idx((uint32_t)(tid - al + THREADS));
#pragma unroll
        for (int q = 1; q < QR; ++q) v[q] = sr[(q - 1) * (THREADS + THREADS / 32)];
    }
    // raw buffer stores: the descriptor's byte bound (the tile's last key)
    // drops the stores past the tile end, so only row 0 needs a lane guard
    const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
        out + (ostart - al), 0, (cnt + al) * 4, kRawBufferWord3);
#pragma unroll
    for (int q = 0; q < QR; ++q)
        if (q > 0 || tid >= al)
            __builtin_amdgcn_raw_buffer_store_b32(v[q], ro, (tid + q * THREADS) * 4, 0, kM4StoreNt);
    // chunk samples of the output for the next pass
    if constexpr (SAMPLES) {
        constexpr int G = kSampleChunk;
        const int f0 = (int)((G - (ostart % G)) % G);          // first chunk start in the tile
        const int l0 = (int)((2 * G - 1 - (ostart % G)) % G);  // first chunk end in the tile
        if (tid < 32) {
            const int e = f0 + tid * G;
            if (e < cnt) samp_first[(ostart + e) / G] = st[e + (e >> 5)];
        } else if (tid < 64) {
            const int e = l0 + (tid - 32) * G;
            if (e < cnt) samp_last[(ostart + e) / G] = st[e + (e >> 5)];
        }
    }
}

// One tile of a four-way pass of the flat sort: tile -> (group, tile of the
// group) -> its boundary rows, then the merge.
template <int DT, int THREADS, int KPT>
__global__ __launch_bounds__(THREADS) void k_merge4(const uint32_t* __restrict__ in,
                                                    uint32_t* __restrict__ out,
                                                    const int32_t* __restrict__ bnd, M4Geom g4,
                                                    uint32_t* __restrict__ samp_first,
                                                    uint32_t* __restrict__ samp_last) {
    const int skip = *g4.skip;  // tested once the boundary loads are in flight
    // static LDS: its base is a compile-time constant the address math folds
    __shared__ __align__(16) uint32_t lds[m4_lds_words(THREADS)];
    // grids stay below 2^31 tiles
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
    if (skip) return;  // the input is already sorted
    m4_merge_tile<DT, THREADS, KPT, true>(in + gb, g4.L, lo, c, out, ostart, samp_first,
                                          samp_last, lds);
}



// ---------------------------------------------------------------- pairs ---
// Four-way pass over key-value pairs (integer keys, stable).  The tiles and
// their splits are those of the keys (the boundary kernels above, whose order
// (key, run, position) is the stable order).  In LDS every key travels as the
// 64-bit composite (order-mapped key, tile position): tile positions grow
// with the run and with the position inside it, so plain composite order is
// the stable order and the merge levels need no tie rule.  Values stay in
// registers until the merge is done; then they are written to LDS by tile
// position, gathered through the positions the composites carry, staged with
// the keys and stored as rows.  Each level gives m4p_mk(threads) outputs to
// each merging thread: 8 for 1024-thread tiles, so that about 990 of the
// threads merge instead of about 500 with 16 (0.89 against 0.93 ms per pass
// over 2^28 pairs); 32 for 512-thread tiles.
__host__ __device__ constexpr int m4p_mk(int threads) { return threads >= 1024 ? 8 : 32; }
// Staged keys: every output a thread holds (up to MK - 1 past the tile end),
// a spare word every 32; the staged values follow.
__host__ __device__ constexpr int m4p_stage(int mk) {
    return kM4MaxTile + mk + (kM4MaxTile + mk) / 32 + 8;
}
// LDS: the padded composite buffer (slices kM4Gap apart, or X and Y), or the
// values by tile position, or the staged keys and values (read back as rows
// of `threads` words, the last row partly past the tile).
__host__ __device__ constexpr int m4p_lds_bytes(int threads) {
    return 8 * lds_words<uint64_t>(kM4MaxTile + 4 * kM4Gap + 8) >
                   4 * (m4p_stage(m4p_mk(threads)) + m4_out_rows(threads) * threads +
                        m4_out_rows(threads) * threads / 32)
               ? 8 * lds_words<uint64_t>(kM4MaxTile + 4 * kM4Gap + 8)
               : 4 * (m4p_stage(m4p_mk(threads)) + m4_out_rows(threads) * threads +
                      m4_out_rows(threads) * threads / 32);
}

template <int DT, int THREADS, int KPT>
__global__ __launch_bounds__(THREADS) void k_merge4_pairs(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, const int32_t* __restrict__ bnd,
    M4Geom g4, uint32_t* __restrict__ samp_first, uint32_t* __restrict__ samp_last) {
    const int skip = *g4.skip;  // tested once the boundary loads are in flight
    static_assert(DT == kU32 || DT == kI32, "integer keys only");
    static_assert(kM4MaxTile <= THREADS * KPT, "tile fits");
    constexpr int MK = m4p_mk(THREADS);
    static_assert(kM4MaxTile / MK + 2 <= THREADS && kM4Gap >= MK, "merge shape");
    constexpr uint64_t kMaxC = kCompMax;
    __shared__ __align__(16) unsigned char smem[m4p_lds_bytes(THREADS)];
    uint64_t* cs = reinterpret_cast<uint64_t*>(smem);  // composites
    uint32_t* w32 = reinterpret_cast<uint32_t*>(smem);  // values, then staging

    const uint32_t t = blockIdx.x;
    int64_t g, j;
    {
        const uint32_t q = m4_udiv(t, g4.by_tiles);
        g = q < (uint64_t)g4.full_groups ? q : g4.full_groups;
        j = (int64_t)t - g * g4.tiles_full;
    }
    const int64_t row = m4_bound_row(g4, g, j);
    const int64_t gb = g * 4 * g4.L;
    int c[4];
    uint32_t sh[4];  // tile key x of slice r is group key x + sh[r] (< 4L < 2^31)
    int64_t ostart = gb;
    int pst[5];
    pst[0] = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lo = bnd[row * 4 + r];
        c[r] = bnd[(row + 1) * 4 + r] - lo;
        ostart += lo;
        sh[r] = (uint32_t)(r * g4.L + lo - pst[r]);
        pst[r + 1] = pst[r] + c[r];
    }
    if (skip) return;  // the input is already sorted
    const int p1 = pst[1], p2 = pst[2], p3 = pst[3], cnt = pst[4];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int X0 = (tid >> 6) * 64 * KPT;

    // ---- load: thread keys and values at tile positions X0 + 64 q + lane.
    // A wave's chunk inside one slice reads from one scalar base at constant
    // offsets and writes its composites at constant LDS offsets; other chunks
    // pick the slice per lane.
    uint32_t rv[KPT];
    {
        const uint32_t* gk = kin + gb;
        const uint32_t* gv = vin + gb;
        uint32_t rk[KPT];
        auto slice_of = [&](int x) { return (x >= p1 ? 1 : 0) + (x >= p2 ? 1 : 0) + (x >= p3 ? 1 : 0); };
        const int r0 = slice_of(X0);
        if (X0 + 64 * KPT <= cnt && r0 == slice_of(X0 + 64 * KPT - 1)) {
            const uint32_t s0 = __builtin_amdgcn_readfirstlane(
                r0 == 0 ? sh[0] : r0 == 1 ? sh[1] : r0 == 2 ? sh[2] : sh[3]);
            const uint32_t* pk = gk + (uint32_t)(X0 + s0) + lane;
            const uint32_t* pv = gv + (uint32_t)(X0 + s0) + lane;
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                rk[q] = ld1_stream(pk + 64 * q);
                rv[q] = ld1_stream(pv + 64 * q);
            }
            // X0 + r0 kM4Gap is a multiple of 64: window q of the chunk sits
            // 68 q padded slots past its first slot
            uint64_t* dst = cs + lds_idx<uint64_t>((uint32_t)(X0 + r0 * kM4Gap)) + lds_idx<uint64_t>(lane);
#pragma unroll
            for (int q = 0; q < KPT; ++q)
                dst[68 * q] = comp_make(ord_key<DT>(rk[q]), (uint32_t)(X0 + 64 * q + lane));
        } else {
            uint32_t src[KPT];
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                const int x = X0 + 64 * q + lane;
                const int xc = min(x, cnt - 1);
                const bool c1 = xc >= p1, c2 = xc >= p2, c3 = xc >= p3;
                src[q] = (uint32_t)xc + (c3 ? sh[3] : c2 ? sh[2] : c1 ? sh[1] : sh[0]);
            }
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                rk[q] = ld1_stream(gk + src[q]);
                rv[q] = ld1_stream(gv + src[q]);
            }
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                const int x = X0 + 64 * q + lane;
                if (x < cnt) {
                    const int gap =
                        x >= p3 ? 3 * kM4Gap : x >= p2 ? 2 * kM4Gap : x >= p1 ? kM4Gap : 0;
                    cs[lds_idx<uint64_t>(x + gap)] = comp_make(ord_key<DT>(rk[q]), (uint32_t)x);
                }
            }
        }
        if (tid < MK) {
#pragma unroll
            for (int r = 0; r < 4; ++r) cs[lds_idx<uint64_t>(pst[r + 1] + r * kM4Gap + tid)] = kMaxC;
        }
    }
    __syncthreads();

    // ---- level 1: X = merge(s0, s1) at 0, Y = merge(s2, s3) at ybase
    const int nx = p2, ny = cnt - p2;
    const int ybase = (nx + MK + 15) & ~15;
    {
        const int tx = (nx + MK - 1) / MK, ty = (ny + MK - 1) / MK;
        uint64_t o[MK];
        const bool in_x = tid < tx;
        const bool active = tid < tx + ty;
        const int d = in_x ? tid * MK : (tid - tx) * MK;
        const int sa = in_x ? 0 : p2 + 2 * kM4Gap, la = in_x ? c[0] : c[2];
        const int sb = in_x ? p1 + kM4Gap : p3 + 3 * kM4Gap, lb = in_x ? c[1] : c[3];
        const int base2 = (in_x ? 0 : ybase) + d;  // a multiple of 16
        if (active) {
            const int i = corank_lds(cs, sa, la, sb, lb, d, PlainLess{});
            serial_merge_closed<uint64_t, MK>(cs, sa + i, sb + d - i, o);
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int k = 0; k < MK; ++k) cs[lds_idx<uint64_t>(base2 + k)] = o[k];
        }
        if (tid < MK) {
            cs[lds_idx<uint64_t>(nx + tid)] = kMaxC;
            cs[lds_idx<uint64_t>(ybase + ny + tid)] = kMaxC;
        }
    }
    __syncthreads();

    // ---- level 2: merge(X, Y)
    const int d = tid * MK;
    uint64_t o[MK];
    if (d < cnt) {
        const int i = corank_lds(cs, 0, nx, ybase, ny, d, PlainLess{});
        serial_merge_closed<uint64_t, MK>(cs, i, ybase + d - i, o);
    }
    __syncthreads();
    // values by tile position, then gathered through the composites
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
        const int x = X0 + 64 * q + lane;
        if (x < cnt) w32[x + (x >> 5)] = rv[q];
    }
    __syncthreads();
    uint32_t ok[MK], ov[MK];
#pragma unroll
    for (int k = 0; k < MK; ++k) {
        const uint32_t x = comp_pos(o[k]);
        ok[k] = unord_key<DT>(comp_ord(o[k]));
        ov[k] = d + k < cnt ? w32[x + (x >> 5)] : 0u;
    }
    // stage keys, then values (a spare word every 32), and store rows
    uint32_t* stk = w32;
    uint32_t* stv = w32 + m4p_stage(MK);
    __syncthreads();
    if (d < cnt) {
#pragma unroll
        for (int k = 0; k < MK; ++k) {
            stk[(d + k) + ((d + k) >> 5)] = ok[k];
            stv[(d + k) + ((d + k) >> 5)] = ov[k];
        }
    }
    __syncthreads();
    const int al = (int)(ostart & 63);  // as in k_merge4: 64-word-aligned rows
    constexpr int QR = m4_out_rows(THREADS);
    const __amdgpu_buffer_rsrc_t rk_out = __builtin_amdgcn_make_buffer_rsrc(
        kout + (ostart - al), 0, (cnt + al) * 4, kRawBufferWord3);
    const __amdgpu_buffer_rsrc_t rv_out = __builtin_amdgcn_make_buffer_rsrc(
        vout + (ostart - al), 0, (cnt + al) * 4, kRawBufferWord3);
#pragma unroll
    for (int q = 0; q < QR; ++q) {
        const int e = max(tid + q * THREADS - al, 0);
        const int pe = e + (e >> 5);
        if (q > 0 || tid >= al) {
            __builtin_amdgcn_raw_buffer_store_b32(stk[pe], rk_out, (tid + q * THREADS) * 4, 0,
                                                  kM4StoreNt);
            __builtin_amdgcn_raw_buffer_store_b32(stv[pe], rv_out, (tid + q * THREADS) * 4, 0,
                                                  kM4StoreNt);
        }
    }
    // chunk samples of the output keys for the next pass
    constexpr int G = kSampleChunk;
    const int f0 = (int)((G - (ostart % G)) % G);
    const int l0 = (int)((2 * G - 1 - (ostart % G)) % G);
    if (tid < 32) {
        const int e = f0 + tid * G;
        if (e < cnt) samp_first[(ostart + e) / G] = stk[e + (e >> 5)];
    } else if (tid < 64) {
        const int e = l0 + (tid - 32) * G;
        if (e < cnt) samp_last[(ostart + e) / G] = stk[e + (e >> 5)];
    }
}

}  // namespace msn
