// Auxiliary kernels: C = beta*C for k == 0 / alpha == 0, and the grouped
// problem-table preparation.
#include <hip/hip_runtime.h>

#include "sk_internal.h"

namespace sk {

// ---------------------------------------------------------------------------
// C = beta * C over an m x n row-major view (the caller has already folded a
// column-major C into its transpose).  beta == 0 writes zeros without reading.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf16f(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ void scale_c_kernel(Problem p) {
    const int64_t total = (int64_t)p.m * p.n;
    const bool rd = p.beta != 0.0;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = idx / p.n, col = idx % p.n;
        const int64_t off = row * p.ldc + col;
        switch (p.c_type) {
        case SK_F64: {
            double *c = (double *)p.C + off;
            *c = rd ? p.beta * *c : 0.0;
            break;
        }
        case SK_F32: {
            float *c = (float *)p.C + off;
            *c = rd ? (float)p.beta * *c : 0.0f;
            break;
        }
        case SK_F16: {
            _Float16 *c = (_Float16 *)p.C + off;
            *c = rd ? (_Float16)((float)p.beta * (float)*c) : (_Float16)0.0f;
            break;
        }
        default: {
            uint16_t *c = (uint16_t *)p.C + off;
            *c = rd ? f2bf((float)p.beta * bf16f(*c)) : (uint16_t)0;
            break;
        }
        }
    }
}

int launch_scale_c(const Problem &p, void *stream) {
    const int64_t total = (int64_t)p.m * p.n;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(scale_c_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, p);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Grouped launches: turn the caller's descriptors (copied into the workspace)
// into kernel problems and prefix sums of tiles and iterations.  One
// workgroup; each thread handles a contiguous run of problems, then a scan
// over the 256 per-thread totals gives every run its offsets.
// ---------------------------------------------------------------------------
__global__ void group_prep_kernel(const sk_gemm_desc_t *raw, int32_t count, int bm, int bn, int bk,
                                  GroupTable tab) {
    __shared__ int32_t tsum[256], isum[256];
    const int t = threadIdx.x;
    const int per = (count + 255) / 256;
    const int b = t * per, e = b + per < count ? b + per : count;
    int32_t ts = 0, is = 0;
    for (int i = b; i < e; ++i) {
        Problem pr = to_problem(raw[i], bm, bn, bk);
        tab.probs[i] = pr;
        const int32_t tiles = pr.m > 0 && pr.n > 0 ? ((pr.m + bm - 1) / bm) * pr.tiles_n : 0;
        ts += tiles;
        is += tiles * pr.iters;
    }
    tsum[t] = ts;
    isum[t] = is;
    __syncthreads();
    if (t == 0) {
        int32_t a = 0, c = 0;
        for (int i = 0; i < 256; ++i) {
            int32_t x = tsum[i], y = isum[i];
            tsum[i] = a;
            isum[i] = c;
            a += x;
            c += y;
        }
        tab.tile_prefix[count] = a;
        tab.iter_prefix[count] = c;
    }
    __syncthreads();
    int32_t ta = tsum[t], ia = isum[t];
    for (int i = b; i < e; ++i) {
        const Problem &pr = tab.probs[i];
        tab.tile_prefix[i] = ta;
        tab.iter_prefix[i] = ia;
        const int32_t tiles = pr.m > 0 && pr.n > 0 ? ((pr.m + bm - 1) / bm) * pr.tiles_n : 0;
        ta += tiles;
        ia += tiles * pr.iters;
    }
}

int launch_group_prep(const sk_gemm_desc_t *raw, int32_t count, int bm, int bn, int bk,
                      const GroupTable &tab, void *stream) {
    hipLaunchKernelGGL(group_prep_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, raw, count, bm,
                       bn, bk, tab);
    return (int)hipGetLastError();
}

}  // namespace sk
