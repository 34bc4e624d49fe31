// Internal structures shared by the host planner/launcher and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "streamk.h"

namespace sk {

// One GEMM as the kernels see it: C is row-major (a column-major C has been
// turned into C^T = B^T A^T by swapping A and B), so "m" runs down C's rows.
struct Problem {
    const void *A;
    const void *B;
    void *C;
    int64_t lda, ldb, ldc;   // elements
    int32_t m, n, k;
    int32_t tiles_m;         // ceil(m / BM)
    int32_t tiles_n;         // ceil(n / BN)
    int32_t iters;           // ceil(k / BK): MAC-loop iterations per tile
    int32_t c_type;          // sk_dtype_t of C
    int32_t c_vec;           // C rows 16-byte aligned: 4-wide vector stores allowed
    double alpha;            // includes the FP8 scale product
    double beta;
};

__host__ __device__ inline int dtype_bytes(int t) {
    return t == SK_F64 ? 8 : t == SK_F32 ? 4 : t == SK_F8_E4M3 ? 1 : 2;
}

// A descriptor as the kernels see it (section 2 problem statement; the
// column-major-C case becomes C^T = B^T A^T with a row-major C^T).
// Operand contiguity is preserved by the swap: see a_kcontig / b_kcontig.
__host__ __device__ inline Problem to_problem(const sk_gemm_desc_t &d, int bm, int bn, int bk) {
    Problem p;
    const bool swap = d.c_order == SK_COL_MAJOR;
    const int64_t lda = d.lda ? d.lda : (d.a_order == SK_ROW_MAJOR ? d.k : d.m);
    const int64_t ldb = d.ldb ? d.ldb : (d.b_order == SK_ROW_MAJOR ? d.n : d.k);
    const int64_t ldc = d.ldc ? d.ldc : (d.c_order == SK_ROW_MAJOR ? d.n : d.m);
    if (!swap) {
        p.A = d.A; p.B = d.B; p.lda = lda; p.ldb = ldb;
        p.m = (int32_t)d.m; p.n = (int32_t)d.n;
    } else {
        p.A = d.B; p.B = d.A; p.lda = ldb; p.ldb = lda;
        p.m = (int32_t)d.n; p.n = (int32_t)d.m;
    }
    p.C = d.C;
    p.ldc = ldc;
    p.k = (int32_t)d.k;
    p.tiles_m = (p.m + bm - 1) / bm;
    p.tiles_n = (p.n + bn - 1) / bn;
    p.iters = (p.k + bk - 1) / bk;
    p.c_type = d.c_type;
    const int eb = dtype_bytes(d.c_type);
    p.c_vec = (((uintptr_t)d.C & 15u) == 0 && ((ldc * eb) & 15) == 0) ? 1 : 0;
    const double s = d.ab_type == SK_F8_E4M3 ? (double)d.a_scale * (double)d.b_scale : 1.0;
    p.alpha = d.alpha * s;
    p.beta = d.beta;
    return p;
}

// Kernel operand A (m rows) / B (n rows) contiguous along k?
__host__ __device__ inline bool a_kcontig(const sk_gemm_desc_t &d) {
    return d.c_order == SK_COL_MAJOR ? d.b_order == SK_COL_MAJOR : d.a_order == SK_ROW_MAJOR;
}
__host__ __device__ inline bool b_kcontig(const sk_gemm_desc_t &d) {
    return d.c_order == SK_COL_MAJOR ? d.a_order == SK_ROW_MAJOR : d.b_order == SK_COL_MAJOR;
}

// Grouped launches keep their problem table in the workspace.
struct GroupTable {
    Problem *probs;
    int32_t *tile_prefix;    // count + 1 entries
    int32_t *iter_prefix;    // count + 1 entries
    int32_t count;
};

// Everything a Stream-K / data-parallel launch needs, passed by value.
struct Params {
    Problem prob;            // single-problem launches
    GroupTable group;        // grouped launches (prob unused)
    int32_t tiles;           // output tiles over all problems
    int32_t g;               // logical workgroups
    int32_t sk_tile_begin;   // SK region in tile order
    int32_t sk_tile_end;
    int32_t sk_iter_begin;   // first iteration of the SK region
    int32_t sk_iters;        // iterations in the SK region
    int32_t dp_tiles;        // tiles outside the SK region
    int32_t dp_first;
    int32_t xcd_remap;
    int32_t band;            // tile rasterisation band (1: row-major tiles)
    int32_t fixup;           // FIXUP_SERIAL or FIXUP_SPREAD
    int32_t dyn_dp;          // 1: data-parallel tiles after the first from the per-XCD queues
    int32_t split;           // > 0: fixed split (s workgroups per tile, one problem) instead of the even split
    int64_t wait_ticks;      // bound of one fixup wait, in real-time-counter ticks (<= 0: give up at once)
    void *partials;          // partial-tile slots of BM*BN accumulators (see slot_first / slot_last)
    int32_t *flags;          // the fixed flag region, FLAG_STRIDE ints apart
    int32_t *hdr;            // workspace header: HDR_ERR, HDR_GEN, HDR_DONE
    int32_t *err;            // error word a giving-up wait sets (hdr + HDR_ERR unless the caller gives one)
    int32_t *trace;          // optional segment trace
    int64_t trace_cap;
};

constexpr int FLAG_STRIDE = 16;          // ints between flags (64 bytes)
constexpr int WS_HEADER = 256;           // header words and padding
constexpr int THREADS = 256;             // 4 wave64 per workgroup
constexpr int MAX_GRID = 1024;           // largest persistent grid
// The flag region [WS_HEADER, WS_HEADER + FLAG_REGION) is reserved in every
// workspace whatever the schedule, so nothing but flags is ever stored there:
// flag x (x < MAX_GRID) belongs to the partial tile workgroup x stores for
// its first segment, flag MAX_GRID + x to the one it stores for its last
// segment (distributed fixup only).
constexpr int FLAG_REGION = 2 * MAX_GRID * FLAG_STRIDE * 4;
// Header words.  A flag is raised by storing the call's epoch, derived from
// HDR_GEN, so flags never need clearing; the last workgroup of a Stream-K
// launch to finish (counted in HDR_DONE) advances HDR_GEN for the next call,
// and returns the eight data-parallel tile queue counters HDR_NEXT + c to 0.
constexpr int HDR_ERR = 0, HDR_GEN = 1, HDR_DONE = 2, HDR_NEXT = 3, XCDS = 8;
// Owners wait on at most this many peers (one 64-lane polling round).
constexpr int MAX_PEERS = 64;

enum Fixup { FIXUP_SERIAL = 0, FIXUP_SPREAD = 1 };

enum Role { ROLE_DP = 0, ROLE_FULL = 1, ROLE_OWNER = 2, ROLE_PRODUCER = 3, ROLE_REDUCE = 4 };

// Kernel instance selection key.
struct KernelKey {
    int ab_type;
    int bm, bn;
    bool a_kc, b_kc;     // operand contiguous along k
    bool grouped;
    bool dp_only;        // the standalone data-parallel kernel
};

// Launch one kernel instance; returns hipError_t as int.
using LaunchFn = int (*)(const Params &p, int grid, void *stream);
using OccupancyFn = int (*)(int *blocks_per_cu);

struct KernelEntry {
    LaunchFn launch;
    OccupancyFn occupancy;
};

// Lookup in the per-dtype instance tables (null launch if not built).
KernelEntry find_kernel(const KernelKey &key);

// Auxiliary launches.
int launch_scale_c(const Problem &p, void *stream);       // C = beta*C
int launch_group_prep(const sk_gemm_desc_t *raw, int32_t count, int bm, int bn, int bk,
                      const GroupTable &tab, void *stream);

}  // namespace sk
