// Backward of a row-wise sort: grad_in[r][perm[r][i]] = grad_out[r][i].
// A permutation, so no atomics and no arithmetic: the result is exact.
// Rows that fit LDS are scattered there and written back with coalesced
// stores; longer rows scatter straight to global memory.
#include "device.hpp"
#include "internal.hpp"

namespace msn {

constexpr int kBwdThreads = 256;
constexpr int kBwdMaxLdsCols = 32768;  // 128 KiB of LDS per row
constexpr int64_t kBwdMaxGrid = 1 << 20;

// Workgroups take rows in turn (the grid is capped, so that any row count
// stays within the launch limits of the dispatch).
__global__ __launch_bounds__(kBwdThreads) void k_backward_lds(const float* __restrict__ go,
                                                              const int32_t* __restrict__ perm,
                                                              float* __restrict__ gi,
                                                              int64_t rows, int cols, int vec) {
    extern __shared__ __align__(16) unsigned char smem[];
    float* s = reinterpret_cast<float*>(smem);
    const int tid = threadIdx.x;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int64_t row = r * cols;
        const float* g = go + row;
        const int32_t* p = perm + row;
        float* out = gi + row;
        for (int i = tid; i < cols; i += kBwdThreads) s[i] = 0.0f;
        __syncthreads();
        if (vec) {
            const int c4 = cols >> 2;
            for (int q = tid; q < c4; q += kBwdThreads) {
                const float4 gv = reinterpret_cast<const float4*>(g)[q];
                const int4 pv = reinterpret_cast<const int4*>(p)[q];
                if ((unsigned)pv.x < (unsigned)cols) s[pv.x] = gv.x;
                if ((unsigned)pv.y < (unsigned)cols) s[pv.y] = gv.y;
                if ((unsigned)pv.z < (unsigned)cols) s[pv.z] = gv.z;
                if ((unsigned)pv.w < (unsigned)cols) s[pv.w] = gv.w;
            }
        } else {
            for (int i = tid; i < cols; i += kBwdThreads) {
                const int32_t j = p[i];
                if ((unsigned)j < (unsigned)cols) s[j] = g[i];
            }
        }
        __syncthreads();
        if (vec) {
            const int c4 = cols >> 2;
            for (int q = tid; q < c4; q += kBwdThreads)
                reinterpret_cast<float4*>(out)[q] =
                    make_float4(s[4 * q], s[4 * q + 1], s[4 * q + 2], s[4 * q + 3]);
        } else {
            for (int i = tid; i < cols; i += kBwdThreads) out[i] = s[i];
        }
        __syncthreads();  // the next row reuses s
    }
}

__global__ __launch_bounds__(kBwdThreads) void k_backward_global(const float* __restrict__ go,
                                                                 const int32_t* __restrict__ perm,
                                                                 float* __restrict__ gi,
                                                                 int64_t rows, int64_t cols) {
    const int64_t e = (int64_t)blockIdx.x * kBwdThreads + threadIdx.x;
    if (e >= rows * cols) return;
    const int64_t r = e / cols;
    const int32_t j = perm[e];
    if ((uint64_t)(uint32_t)j < (uint64_t)cols && j >= 0) gi[r * cols + j] = go[e];
}

int launch_backward(const float* grad_out, const int32_t* perm, float* grad_in, int64_t rows,
                    int64_t cols, hipStream_t stream) {
    if (rows == 0 || cols == 0) return 0;
    if (cols <= kBwdMaxLdsCols) {
        const size_t lds = (size_t)cols * 4;
        if (int rc = set_dynamic_lds(reinterpret_cast<const void*>(&k_backward_lds),
                                     (size_t)kBwdMaxLdsCols * 4))
            return rc;
        auto al = [](const void* q) { return ((uintptr_t)q & 15u) == 0; };
        const int vec = (cols % 4 == 0) && al(grad_out) && al(perm) && al(grad_in);
        // one row per workgroup up to 2^20 rows (2^28 threads); more rows loop
        const int64_t grid = rows < kBwdMaxGrid ? rows : kBwdMaxGrid;
        LaunchTimer timer("backward", rows * cols, stream);
        hipLaunchKernelGGL(k_backward_lds, dim3((unsigned)grid), dim3(kBwdThreads), lds, stream,
                           grad_out, perm, grad_in, rows, (int)cols, vec);
    } else {
        const int64_t total = rows * cols;
        LaunchTimer timer("backward", total, stream);
        hipLaunchKernelGGL(k_backward_global,
                           dim3((unsigned)((total + kBwdThreads - 1) / kBwdThreads)),
                           dim3(kBwdThreads), 0, stream, grad_out, perm, grad_in, rows, cols);
    }
    return (int)hipGetLastError();
}

}  // namespace msn
