// Host side of the C ABI: argument validation, the launch planner (tile,
// schedule, grid size, Stream-K region) and the kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "sk_internal.h"

using namespace sk;

namespace {

struct TileDef {
    int bm, bn, bk;
};

// Built tiles per input dtype; the first entry is the default.  The paper
// keeps one tile per precision, the smallest that reaches its near-peak rate
// on very large problems (section 5.1).  For FP16/BF16 and FP8 the
// automatic choice takes the second (128x128) tile unless the problem fills
// at least kBigTileWaves full waves of it (in build_call): the 256x256 tile
// moves half the operand bytes per flop, which wins once quantisation no
// longer matters (FP8 8192^3: 1994 vs 1631 TFLOP/s row/row, 2300 vs 2086
// row/col), while the 128x128 tile fills the machine on smaller problems.
// The 64x64 tiles of the 16-bit and FP8 types are never the automatic
// choice; they serve callers (and the autotuner) that pick them: a second,
// smaller-tile kernel for problems too small or too memory-bound to fill
// the machine with the larger tiles.
const TileDef kF64Tiles[] = {{128, 128, 16}, {64, 64, 16}};
const TileDef k16Tiles[] = {{256, 256, 64}, {128, 128, 64}, {64, 64, 64}};
const TileDef kF8Tiles[] = {{256, 256, 128}, {128, 128, 128}, {64, 64, 128}};

const TileDef *tiles_for(int ab, int *n) {
    switch (ab) {
    case SK_F64: *n = 2; return kF64Tiles;
    case SK_F16:
    case SK_BF16: *n = 3; return k16Tiles;
    case SK_F8_E4M3: *n = 3; return kF8Tiles;
    }
    *n = 0;
    return nullptr;
}

// Appendix A.1 grid-size model constants {a, b, c, d} in microseconds:
// a fixed per-workgroup cost, b the cost of emitting a partial tile, c one
// MAC-loop iteration, d reading and adding one peer's partial tile.  As the
// paper prescribes, they were measured once on the target (MI355X, from
// basic Stream-K timings over a range of grid sizes, least-squares fit) and
// are compiled in; only their ratios matter to the argmin over g.  The
// spread fixup has its own set: each contributor reads one tile's worth of
// partials whatever the peer count, so its d is small.
struct Model {
    double a, b, c, d;
    // optional memory term (off by default): microseconds per workgroup
    // that writes and reads back one partial tile, charged to every
    // workgroup of a plan that splits tiles -- 2 BM BN acc_bytes / bandwidth
    double mem = 0.0;
};

Model default_model(int ab, int bm, bool spread) {
    if (ab != SK_F64 && bm < 128) return spread ? Model{0.0, 6.0, 0.25, 0.02} : Model{0.0, 5.0, 0.25, 0.3};
    if (spread) {
        switch (ab) {
        case SK_F64: return bm >= 128 ? Model{15.6, 6.0, 2.03, 0.1} : Model{6.22, 2.6, 0.73, 0.05};
        case SK_F8_E4M3: return bm >= 256 ? Model{27.8, 8.0, 1.62, 0.2} : Model{0.0, 14.0, 0.82, 0.05};
        default: return bm >= 256 ? Model{25.2, 8.0, 1.41, 0.2} : Model{0.0, 12.0, 0.73, 0.05};
        }
    }
    switch (ab) {
    case SK_F64: return bm >= 128 ? Model{15.6, 4.41, 2.03, 1.65} : Model{6.22, 2.22, 0.73, 0.43};
    case SK_F8_E4M3: return bm >= 256 ? Model{27.8, 0.0, 1.62, 6.39} : Model{0.0, 13.2, 0.82, 0.64};
    default: return bm >= 256 ? Model{25.2, 0.0, 1.41, 5.47} : Model{0.0, 11.2, 0.73, 0.64};
    }
}

bool supported_pair(int ab, int c) {
    switch (ab) {
    case SK_F64: return c == SK_F64;
    case SK_F16: return c == SK_F32 || c == SK_F16;
    case SK_BF16: return c == SK_BF16 || c == SK_F32;
    case SK_F8_E4M3: return c == SK_BF16 || c == SK_F32;
    }
    return false;
}

bool is_order(int o) { return o == SK_ROW_MAJOR || o == SK_COL_MAJOR; }

// Largest leading dimension of A or B, in bytes (4 MiB: 2M FP16 elements).
constexpr int64_t kMaxRowBytes = 1LL << 22;

sk_status_t validate(const sk_gemm_desc_t &d) {
    if (d.m < 0 || d.n < 0 || d.k < 0) return SK_ERR_INVALID_VALUE;
    if (d.m > (1LL << 30) || d.n > (1LL << 30) || d.k > (1LL << 30)) return SK_ERR_INVALID_VALUE;
    if (!is_order(d.a_order) || !is_order(d.b_order) || !is_order(d.c_order)) return SK_ERR_INVALID_VALUE;
    if (d.ab_type < SK_F64 || d.ab_type > SK_F8_E4M3 || d.c_type < SK_F64 || d.c_type > SK_F8_E4M3)
        return SK_ERR_INVALID_VALUE;
    if (!supported_pair(d.ab_type, d.c_type)) return SK_ERR_UNSUPPORTED;
    if (d.ab_type == SK_F8_E4M3) {
        if (!(std::isfinite(d.a_scale) && d.a_scale > 0.0f && std::isfinite(d.b_scale) && d.b_scale > 0.0f))
            return SK_ERR_INVALID_VALUE;
    } else if (!((d.a_scale == 0.0f || d.a_scale == 1.0f) && (d.b_scale == 0.0f || d.b_scale == 1.0f))) {
        return SK_ERR_INVALID_VALUE;
    }
    if (d.lda < 0 || d.ldb < 0 || d.ldc < 0) return SK_ERR_INVALID_VALUE;
    if (d.m == 0 || d.n == 0) return SK_OK;
    // leading dimensions cover the packed extent
    const int64_t a_ext = d.a_order == SK_ROW_MAJOR ? d.k : d.m;
    const int64_t b_ext = d.b_order == SK_ROW_MAJOR ? d.n : d.k;
    const int64_t c_ext = d.c_order == SK_ROW_MAJOR ? d.n : d.m;
    if (d.ldc != 0 && d.ldc < c_ext) return SK_ERR_INVALID_VALUE;
    if (!d.C) return SK_ERR_INVALID_VALUE;
    if (((uintptr_t)d.C) % (uintptr_t)dtype_bytes(d.c_type)) return SK_ERR_MISALIGNED;
    if (d.k == 0 || d.alpha == 0.0) return SK_OK;   // A and B are not referenced
    if (d.lda != 0 && d.lda < a_ext) return SK_ERR_INVALID_VALUE;
    if (d.ldb != 0 && d.ldb < b_ext) return SK_ERR_INVALID_VALUE;
    if (!d.A || !d.B) return SK_ERR_INVALID_VALUE;
    const int vec = 16 / dtype_bytes(d.ab_type);
    const int64_t lda = d.lda ? d.lda : a_ext, ldb = d.ldb ? d.ldb : b_ext;
    if (((uintptr_t)d.A & 15u) || ((uintptr_t)d.B & 15u)) return SK_ERR_MISALIGNED;
    if (lda % vec || ldb % vec || a_ext % vec || b_ext % vec) return SK_ERR_MISALIGNED;
    // the kernels address one k-tile of an operand with 32-bit offsets
    const int64_t eb = dtype_bytes(d.ab_type);
    if (lda * eb > kMaxRowBytes || ldb * eb > kMaxRowBytes) return SK_ERR_INVALID_VALUE;
    return SK_OK;
}

// Workgroups of a tile's kernel that fit one CU by LDS alone (two k-tile
// buffers of (BM + BN) 128-byte rows; 160 KiB per CU).
int lds_wgs_per_cu(const TileDef &t) {
    const int lds = 2 * (t.bm + t.bn) * 128;
    return std::max(1, (160 * 1024) / lds);
}

// FP16/BF16 problems with at least this many full waves of 128x128 tiles
// use the 256x256 tile (its larger per-tile reuse wins once the machine is
// saturated many times over; below that the 128x128 tile's two workgroups
// per CU hide more latency).
// FP8: 8.  FP16/BF16 (eight-wave 256x256 kernel): 2 -- BF16 DP 4096^3
// 870 -> 1026 TFLOP/s, 4096x8192x4096 1002 -> 1105, 2048x8192x8192 1050 ->
// 1169, 3072x3072x8192 696 -> 801; even at 6144x6144x4096; the FP16 sweep
// is unchanged within noise (352 -> 354).
constexpr int64_t kBigTileWaves = 8;        // FP8
constexpr int64_t kBigTileWaves16 = 2;      // FP16 / BF16

// FP16/BF16 problems too small for the 128x128 tile to fill the machine
// take the 64x64 tile (measured per problem over the FP16 sweep, every
// problem under every configuration: the sum of per-GEMM times falls from
// 82.6 to 75.1 ms, geometric-mean speedup 1.25): basic Stream-K while it
// has fewer than kTinySkTiles tiles and k <= kTinySkMaxK, else
// data-parallel for problems of at most 3/4 CUs 128x128 tiles and k <=
// kTinyDpMaxK.  Deeper or larger ones keep the 128x128 tile, whose
// Stream-K split wins there (256x256x65536: 30 vs 35 us on the 64x64
// tile; 4096x1024x4096, 256 tiles: 46 vs 76 us).
constexpr int64_t kTinySkTiles = 64;
constexpr int64_t kTinySkMaxK = 8192;
constexpr int64_t kTinyDpMaxK = 4096;

// Schedule refinements of the FP16/BF16 default, measured per problem over
// two FP16 geometry sweeps (2 x 2048 GEMMs, every problem under every
// configuration; gains are of the summed per-GEMM time):
//  * 64x64 tile, fewer than 1.5 CUs' worth of tiles, at least kDeepIters
//    k-iterations per tile: basic Stream-K instead of one workgroup per tile
//    (these problems' own time -12 %, -23 % below one CU's worth; sweep
//    +1.1 %; from 1.5 CUs' worth on, one workgroup per tile is faster);
//  * 128x128 tile under Stream-K: a k-aligned split (below, sweep +1.7 %);
//  * 256x256 tile past a full wave with a last partial wave of at most
//    kTailNum / kTailDen of the slots and at least kDeepIters k-iterations
//    per tile: data-parallel waves + one-tile Stream-K (section 5.2) instead
//    of a nearly empty last data-parallel wave, its tail as a fixed split
//    (tail_split_factor) rather than the even split over all p workgroups,
//    whose pieces start at unrelated k offsets (FP16: 2048x8448x7040 with an
//    8-tile tail: DP 357, even tail 280, fixed-split tail 256 us;
//    2048x11264x4096, 96-tile tail: 211, 209, 196; 2048x12288x4096,
//    128-tile tail: 213, 207, 205).  With a tail of more than half the
//    slots no split of two or more fits and DP stays.
constexpr int64_t kDeepIters = 32;
constexpr int64_t kTailNum = 1, kTailDen = 2;
constexpr int64_t kTailMaxSplit = 16;
// A single GEMM with between kMidBigDp/kMidBigDen of the CUs and all CUs in
// 256x256 tiles and at least kDeepIters k-iterations per tile takes that
// tile, data-parallel (the 128x128 tile would give 2-4 partial waves of one
// or two workgroups per CU; these problems' own time -11 %); from
// kMidBigLo/kMidBigDen of the CUs on and with at least kMidBigSkIters
// k-iterations per tile, basic Stream-K over the model's grid (-9 %;
// shallower ones lose to the 128x128 tile).
constexpr int64_t kMidBigLo = 4, kMidBigDp = 5, kMidBigDen = 8;
constexpr int64_t kMidBigSkIters = 48;

// The fixed split of a hybrid's tail of r tiles: the largest s <= 16 with
// s r <= p and no empty piece (1: none).  Measured on 256x256 FP16 tiles:
// an 8-tile tail split 16 ways beat 32 ways (2048x8448x7040: 256 vs 260 us).
int64_t tail_split_factor(int64_t r, int64_t iters_per_tile, int p);

// Fixed split (Algorithm 4) of t tiles of I iterations on p slots: the
// largest s <= SK_MAX_PEERS + 1 with s t <= p whose pieces of ceil(I / s)
// iterations leave none of the s empty; 1 if there is none.
int64_t fixed_split_factor(int64_t tiles, int64_t iters_per_tile, int p) {
    int64_t best = 1;
    const int64_t smax = std::min<int64_t>(iters_per_tile, SK_MAX_PEERS + 1);
    for (int64_t s = 2; s <= smax; ++s)
        if (s * tiles <= p && (s - 1) * ((iters_per_tile + s - 1) / s) < iters_per_tile) best = s;
    return best;
}

int64_t tail_split_factor(int64_t r, int64_t iters_per_tile, int p) {
    int64_t best = 1;
    const int64_t smax = std::min<int64_t>(iters_per_tile, kTailMaxSplit);
    for (int64_t s = 2; s <= smax; ++s)
        if (s * r <= p && (s - 1) * ((iters_per_tile + s - 1) / s) < iters_per_tile) best = s;
    return best;
}

// k-aligned split for the automatic schedule: the fixed split above, used
// when it keeps at least half of the slots busy (2 s t >= p).  The paper's
// even split over the model's grid starts the workgroups of neighbouring
// tiles at unrelated k offsets, so concurrently running workgroups share no
// operand k-slices in their XCD's L2; with a fixed split, the workgroups of
// the same piece index run the same k-slices together.  Measured (FP16,
// 128x128 tiles, t <= CUs, k >= 4096): the summed time of the problems with
// 2 s t >= p (s dividing I) falls by 9-27 % against the model's grid (by
// more the closer s t comes to p); with fewer busy slots the model's grid
// wins.  FP8 (128x128x128): 2048x1664x4096 594 -> 894 TFLOP/s,
// 3072x1280x6144 761 -> 1242, 1152x2560x8192 657 -> 1106.  Single GEMMs
// only (a grouped call's tiles differ in I).
// On the 64x64 tile (four workgroups per CU) it pays from 5/8 of the slots
// on (FP16 sweep, the 64x64 Stream-K problems with s t >= 5/8 p: -4 to
// -6.5 %; at half of the slots +5 to +13 %).
int64_t aligned_split(int64_t tiles, int64_t iters_per_tile, int p, int64_t fill_num, int64_t fill_den) {
    const int64_t s = fixed_split_factor(tiles, iters_per_tile, p);
    return (s >= 2 && fill_den * s * tiles >= fill_num * (int64_t)p) ? s : 1;
}

sk_status_t resolve_tile(int ab, const sk_config_t *cfg, TileDef *out) {
    int n = 0;
    const TileDef *t = tiles_for(ab, &n);
    if (!t) return SK_ERR_UNSUPPORTED;
    if (!cfg || (cfg->blk_m == 0 && cfg->blk_n == 0 && cfg->blk_k == 0)) {
        *out = t[0];   // refined by pick_tile for FP16/BF16
        return SK_OK;
    }
    for (int i = 0; i < n; ++i)
        if (t[i].bm == cfg->blk_m && t[i].bn == cfg->blk_n && (cfg->blk_k == 0 || t[i].bk == cfg->blk_k)) {
            *out = t[i];
            return SK_OK;
        }
    return SK_ERR_UNSUPPORTED;
}

// Resident workgroup slots of a kernel on the current device (cached).
struct SlotKey {
    int dev, ab, bm;
    bool akc, bkc, grouped;
    bool operator==(const SlotKey &o) const {
        return dev == o.dev && ab == o.ab && bm == o.bm && akc == o.akc && bkc == o.bkc && grouped == o.grouped;
    }
};
std::mutex g_slot_mu;
std::vector<std::pair<SlotKey, int>> g_slot_cache;

std::vector<std::pair<int, int>> g_cu_cache;   // device -> CU count

sk_status_t query_cus(int *cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SK_ERR_HIP;
    {
        std::lock_guard<std::mutex> lk(g_slot_mu);
        for (auto &e : g_cu_cache)
            if (e.first == dev) {
                *cus = e.second;
                return SK_OK;
            }
    }
    if (hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || *cus <= 0)
        return SK_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_slot_mu);
    g_cu_cache.push_back({dev, *cus});
    return SK_OK;
}

sk_status_t query_slots(const KernelKey &key, int *slots) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SK_ERR_HIP;
    SlotKey sk_{dev, key.ab_type, key.bm, key.a_kc, key.b_kc, key.grouped};
    {
        std::lock_guard<std::mutex> lk(g_slot_mu);
        for (auto &e : g_slot_cache)
            if (e.first == sk_) {
                *slots = e.second;
                return SK_OK;
            }
    }
    int cus = 0;
    if (query_cus(&cus) != SK_OK) return SK_ERR_HIP;
    KernelKey k2 = key;
    k2.dp_only = false;
    KernelEntry e = find_kernel(k2);
    if (!e.occupancy) return SK_ERR_UNSUPPORTED;
    int bpc = 0;
    if (e.occupancy(&bpc) != (int)hipSuccess || bpc <= 0) return SK_ERR_HIP;
    *slots = cus * bpc;
    std::lock_guard<std::mutex> lk(g_slot_mu);
    g_slot_cache.push_back({sk_, *slots});
    return SK_OK;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Appendix A.1's per-workgroup time of basic Stream-K on g workgroups,
// a + b [peers > 1] + c ItersPerCta(g) + d (peers - 1), plus the optional
// memory term mem * g [peers > 1] for the partial-tile traffic, which grows
// with the number of workgroups that emit partials.
double model_time(int64_t T, int64_t I, int64_t g, const Model &m) {
    const int64_t ipc = cdiv(T, g);
    const int64_t peers = cdiv(I, ipc);
    const double split = peers > 1 ? 1.0 : 0.0;
    return m.a + m.b * split + m.c * (double)ipc + m.d * (double)(peers - 1) + m.mem * (double)g * split;
}

// Appendix A.1: g* = argmin over g in [1, min(p, T)] of
//   a + b [peers > 1] + c ItersPerCta(g) + d (peers - 1),
// ItersPerCta(g) = ceil(T / g), peers = ceil(I / ItersPerCta(g)); ties take
// the smallest g.  `ok(g)` excludes grids the library cannot run (an owner
// with more than SK_MAX_PEERS peers); g = 1 is always feasible.
template <class Ok>
int model_grid(int64_t T, int64_t I, int p, const Model &m, Ok ok) {
    const int64_t gmax = std::max<int64_t>(1, std::min<int64_t>(p, T));
    std::vector<std::pair<double, int>> cand;
    cand.reserve((size_t)gmax);
    for (int64_t g = 1; g <= gmax; ++g) {
        cand.push_back({model_time(T, I, g, m), (int)g});
    }
    size_t best = 0;
    for (size_t i = 1; i < cand.size(); ++i)
        if (cand[i].first < cand[best].first) best = i;
    if (cand[best].second == 1 || ok(cand[best].second)) return cand[best].second;
    std::stable_sort(cand.begin(), cand.end(),
                     [](const std::pair<double, int> &u, const std::pair<double, int> &v) { return u.first < v.first; });
    for (const auto &c : cand)
        if (c.second == 1 || ok(c.second)) return c.second;
    return 1;
}

// Host view of one call: problems (kernel form), tile, key and prefix sums.
struct Call {
    std::vector<Problem> probs;
    std::vector<int64_t> tile_prefix, iter_prefix;   // count + 1
    TileDef tile;
    KernelKey key;
    int64_t tiles = 0, iters = 0, imax = 0;

    int64_t tile_iter_begin(int64_t tile_g) const {
        // problem holding tile_g (last index with prefix <= tile_g)
        size_t lo = 0, hi = probs.size();
        while (hi - lo > 1) {
            size_t mid = (lo + hi) / 2;
            if (tile_prefix[mid] <= tile_g) lo = mid; else hi = mid;
        }
        return iter_prefix[lo] + (tile_g - tile_prefix[lo]) * probs[lo].iters;
    }
    int64_t region_iters(int64_t tb, int64_t te) const {
        if (te <= tb) return 0;
        return (te >= tiles ? iters : tile_iter_begin(te)) - tile_iter_begin(tb);
    }
    // [begin, end) in global iterations of the tile holding global iteration it
    void tile_span(int64_t it, int64_t *b, int64_t *e) const {
        size_t lo = 0, hi = probs.size();
        while (hi - lo > 1) {
            size_t mid = (lo + hi) / 2;
            if (iter_prefix[mid] <= it) lo = mid; else hi = mid;
        }
        // skip problems without tiles (their iteration range is empty)
        while (lo + 1 < probs.size() && iter_prefix[lo + 1] <= it) ++lo;
        const int64_t I = probs[lo].iters;
        *b = iter_prefix[lo] + (it - iter_prefix[lo]) / I * I;
        *e = *b + I;
    }
    // Largest number of peers any tile's owner has when the iterations
    // [ib, ib + n) are split evenly over g workgroups (section 4 partition).
    int64_t max_peers(int64_t ib, int64_t n, int64_t g) const {
        if (n <= 0 || g <= 1) return 0;
        const int64_t q = n / g, r = n % g, rq = r * (q + 1);
        auto owner = [&](int64_t i) { return i < rq ? i / (q + 1) : r + (i - rq) / q; };
        const bool one = probs.size() == 1;
        const int64_t I1 = probs[0].iters;
        int64_t best = 0;
        for (int64_t x = 0; x < g; ++x) {
            const int64_t b = x * q + std::min(x, r), e = b + q + (x < r ? 1 : 0);
            if (e <= b) continue;
            int64_t tb, te;
            if (one) {
                tb = (ib + e - 1) / I1 * I1;
                te = tb + I1;
            } else {
                tile_span(ib + e - 1, &tb, &te);
            }
            tb -= ib;
            te -= ib;
            if (tb >= b && te > e) best = std::max(best, owner(te - 1) - x);
        }
        return best;
    }
    // Whether no tile's owner has more than `lim` peers when [0, n) is split
    // evenly over g workgroups.  Ranges are q or q + 1 iterations long
    // (q = n / g), so a tile of I iterations meets at most ceil((I - 1) / q)
    // ranges after its first, and the longest tile at least
    // ceil(imax / (q + 1)) ranges in all; the exact O(g) count is only
    // needed between the two bounds.
    bool peers_within(int64_t n, int64_t g, int64_t lim) const {
        if (n <= 0 || g <= 1) return true;
        const int64_t q = n / g;
        if (q <= 0) return max_peers(0, n, g) <= lim;
        if ((imax - 1 + q - 1) / q <= lim) return true;
        if ((imax + q) / (q + 1) - 1 > lim) return false;
        return max_peers(0, n, g) <= lim;
    }
};

sk_status_t build_call(const sk_gemm_desc_t *d, int32_t count, const sk_config_t *cfg, bool grouped,
                       Call *c) {
    if (!d || count <= 0) return SK_ERR_INVALID_VALUE;
    if (cfg && (cfg->wg_slots < 0 || cfg->grid < 0 || cfg->split < 0 || cfg->sched < SK_SCHED_AUTO ||
                cfg->sched > SK_SCHED_FIXED_SPLIT))
        return SK_ERR_INVALID_VALUE;
    for (int i = 0; i < count; ++i) {
        sk_status_t s = validate(d[i]);
        if (s != SK_OK) return s;
        if (grouped) {
            if (d[i].ab_type != d[0].ab_type || d[i].c_type != d[0].c_type || d[i].a_order != d[0].a_order ||
                d[i].b_order != d[0].b_order || d[i].c_order != d[0].c_order)
                return SK_ERR_UNSUPPORTED;
            if (d[i].m > 0 && d[i].n > 0 && d[i].k == 0) return SK_ERR_UNSUPPORTED;
        }
    }
    sk_status_t s = resolve_tile(d[0].ab_type, cfg, &c->tile);
    if (s != SK_OK) return s;
    const bool tile_given = cfg && (cfg->blk_m != 0 || cfg->blk_n != 0 || cfg->blk_k != 0);
    if (!tile_given && (d[0].ab_type == SK_F16 || d[0].ab_type == SK_BF16 || d[0].ab_type == SK_F8_E4M3)) {
        // the 128x128 tile unless there are kBigTileWaves full waves of it
        int n = 0;
        const TileDef small = tiles_for(d[0].ab_type, &n)[1];
        int64_t t_small = 0;
        for (int i = 0; i < count; ++i) {
            const Problem p = to_problem(d[i], small.bm, small.bn, small.bk);
            if (p.m > 0 && p.n > 0) t_small += cdiv(p.m, small.bm) * (int64_t)p.tiles_n;
        }
        int p_small = cfg ? cfg->wg_slots : 0;
        if (p_small <= 0) {
            const KernelKey ks{d[0].ab_type, small.bm, small.bn, a_kcontig(d[0]), b_kcontig(d[0]), grouped, false};
            s = query_slots(ks, &p_small);
            if (s != SK_OK) return s;
        }
        const int64_t waves = d[0].ab_type == SK_F8_E4M3 ? kBigTileWaves : kBigTileWaves16;
        if (t_small < waves * (int64_t)p_small) c->tile = small;
        if (d[0].ab_type != SK_F8_E4M3 && c->tile.bm == small.bm && count == 1) {
            // a deep GEMM with between half and all of a CU's worth of
            // 256x256 tiles keeps the eight-wave tile (see kMidBig*)
            const TileDef big = tiles_for(d[0].ab_type, &n)[0];
            const Problem pb = to_problem(d[0], big.bm, big.bn, big.bk);
            const int64_t t_big = cdiv(pb.m, big.bm) * (int64_t)pb.tiles_n;
            int cus = 0;
            if (cfg && cfg->wg_slots > 0) {
                cus = std::max(1, cfg->wg_slots / lds_wgs_per_cu(small));
            } else {
                s = query_cus(&cus);
                if (s != SK_OK) return s;
            }
            if (t_big <= cus && ((pb.iters >= kDeepIters && kMidBigDen * t_big >= kMidBigDp * (int64_t)cus) ||
                                 (pb.iters >= kMidBigSkIters && kMidBigDen * t_big >= kMidBigLo * (int64_t)cus)))
                c->tile = big;
        }
        if (d[0].ab_type != SK_F8_E4M3 && c->tile.bm == small.bm) {
            const TileDef tiny = tiles_for(d[0].ab_type, &n)[2];
            int64_t t_tiny = 0, kmax = 0;
            for (int i = 0; i < count; ++i) {
                const Problem p = to_problem(d[i], tiny.bm, tiny.bn, tiny.bk);
                if (p.m > 0 && p.n > 0) t_tiny += cdiv(p.m, tiny.bm) * (int64_t)p.tiles_n;
                kmax = std::max<int64_t>(kmax, d[i].k);
            }
            int cus = 0;
            if (cfg && cfg->wg_slots > 0) {
                cus = std::max(1, cfg->wg_slots / lds_wgs_per_cu(small));
            } else {
                s = query_cus(&cus);
                if (s != SK_OK) return s;
            }
            if ((t_tiny < kTinySkTiles && kmax <= kTinySkMaxK) || (4 * t_small <= 3 * (int64_t)cus && kmax <= kTinyDpMaxK))
                c->tile = tiny;
        }
    }
    c->key = KernelKey{d[0].ab_type, c->tile.bm, c->tile.bn, a_kcontig(d[0]), b_kcontig(d[0]), grouped, false};
    c->probs.resize(count);
    c->tile_prefix.assign(count + 1, 0);
    c->iter_prefix.assign(count + 1, 0);
    for (int i = 0; i < count; ++i) {
        Problem p = to_problem(d[i], c->tile.bm, c->tile.bn, c->tile.bk);
        c->probs[i] = p;
        const int64_t t = (p.m > 0 && p.n > 0) ? cdiv(p.m, c->tile.bm) * (int64_t)p.tiles_n : 0;
        c->tile_prefix[i + 1] = c->tile_prefix[i] + t;
        c->iter_prefix[i + 1] = c->iter_prefix[i] + t * p.iters;
        if (t > 0) c->imax = std::max<int64_t>(c->imax, p.iters);
    }
    c->tiles = c->tile_prefix[count];
    c->iters = c->iter_prefix[count];
    if (c->tiles >= (1LL << 31) || c->iters >= (1LL << 31)) return SK_ERR_INVALID_VALUE;
    return SK_OK;
}


// Owners with at least this many peers make the automatic fixup the spread
// one (with a single peer the serial fixup moves fewer bytes for the same
// critical path).
constexpr int64_t kSpreadMinPeers = 2;

// The schedule: which tiles form the Stream-K region and how many
// workgroups run.  Section 5.2 hybrids with w = t / p full waves, r = t % p:
//  r == 0           -> whole waves of data-parallel tiles on g = p;
//  w == 0           -> basic Stream-K over every tile with the model's g;
//  two-tile SK + DP -> (w >= threshold) SK over the first r + p tiles, each
//                      workgroup getting 1..2 tiles of iterations, then DP;
//  DP + one-tile SK -> DP over the first w*p tiles, then SK over the last r.
// No plan may give a tile's owner more than SK_MAX_PEERS peers: the model's
// grid search skips such grids, the automatic schedule avoids them, and an
// explicit grid or hybrid that needs them is rejected.
sk_status_t plan_call(const Call &c, const sk_config_t *cfg, sk_plan_t *pl) {
    std::memset(pl, 0, sizeof(*pl));
    pl->blk_m = c.tile.bm;
    pl->blk_n = c.tile.bn;
    pl->blk_k = c.tile.bk;
    pl->tiles = c.tiles;
    pl->iters_total = c.iters;
    pl->fixup = SK_FIXUP_SERIAL;
    int sched = cfg ? cfg->sched : SK_SCHED_AUTO;
    if (sched < SK_SCHED_AUTO || sched > SK_SCHED_FIXED_SPLIT) return SK_ERR_INVALID_VALUE;
    if (cfg && cfg->split < 0) return SK_ERR_INVALID_VALUE;
    const bool auto_sched = sched == SK_SCHED_AUTO;
    const int user_grid = cfg ? cfg->grid : 0;
    if (user_grid < 0 || user_grid > SK_MAX_GRID) return SK_ERR_INVALID_VALUE;
    const int fix_req = cfg ? cfg->fixup : SK_FIXUP_AUTO;
    if (fix_req < SK_FIXUP_AUTO || fix_req > SK_FIXUP_SPREAD) return SK_ERR_INVALID_VALUE;
    const int threshold = (cfg && cfg->sk_threshold_waves > 0) ? cfg->sk_threshold_waves : 2;
    Model m_serial = default_model(c.key.ab_type, c.tile.bm, false);
    Model m_spread = default_model(c.key.ab_type, c.tile.bm, true);
    if (cfg && (cfg->model_a != 0.0 || cfg->model_b != 0.0 || cfg->model_c != 0.0 || cfg->model_d != 0.0))
        m_serial = m_spread = Model{cfg->model_a, cfg->model_b, cfg->model_c, cfg->model_d};
    if (cfg && cfg->model_bw > 0.0) {
        const double acc = c.key.ab_type == SK_F64 ? 8.0 : 4.0;
        m_serial.mem = m_spread.mem = 2.0 * (double)c.tile.bm * (double)c.tile.bn * acc / cfg->model_bw;
    }
    const int64_t t = c.tiles;
    pl->xcd_remap = (cfg && (cfg->flags & SK_FLAG_NO_XCD_REMAP)) ? 0 : 1;
    if (t == 0) {
        pl->sched = sched == SK_SCHED_AUTO ? SK_SCHED_DP : sched;
        return SK_OK;
    }
    if (c.iters == 0) {
        // k == 0: no MAC-loop work; sk_gemm computes C = beta*C with its own
        // kernel, so nothing persistent is planned
        pl->sched = SK_SCHED_DP;
        pl->dp_tiles = t;
        return SK_OK;
    }
    int p = 0;
    int cus = 0;
    if (sched != SK_SCHED_DP) {
        p = cfg ? cfg->wg_slots : 0;
        if (p < 0) return SK_ERR_INVALID_VALUE;
        if (p == 0) {
            sk_status_t s = query_slots(c.key, &p);
            if (s == SK_OK) s = query_cus(&cus);
            if (s != SK_OK) return s;
        } else {
            cus = p / lds_wgs_per_cu(c.tile);
        }
        pl->wg_slots = p;
        if (user_grid > p) return SK_ERR_INVALID_VALUE;   // all workgroups must be co-resident
    }
    const int pg = std::min(p, SK_MAX_GRID);   // grids the model may choose
    // Algorithm 4: s workgroups per tile, piece y of tile x on workgroup x s + y
    auto plan_fixed_split = [&](int64_t split) -> sk_status_t {
        if (c.probs.size() != 1) return SK_ERR_UNSUPPORTED;
        const int64_t I = c.imax;
        const int64_t sp = split > 0 ? split : fixed_split_factor(t, I, pg);
        if (sp > SK_MAX_PEERS + 1) return SK_ERR_UNSUPPORTED;
        if (user_grid > 0 && user_grid != sp * t) return SK_ERR_INVALID_VALUE;
        if (sp == 1) {
            // s = 1 is the data-parallel schedule (any number of tiles)
            pl->sched = SK_SCHED_DP;
            pl->grid = (int32_t)t;
            pl->dp_first = 1;
            pl->dp_tiles = t;
            return SK_OK;
        }
        if (sp * t > pg) return SK_ERR_INVALID_VALUE;   // all s t workgroups must be co-resident
        const int64_t ips = cdiv(I, sp);
        pl->sched = SK_SCHED_FIXED_SPLIT;
        pl->split = (int32_t)sp;
        pl->grid = (int32_t)(sp * t);
        pl->sk_tile_begin = 0;
        pl->sk_tile_end = t;
        pl->sk_iter_begin = 0;
        pl->sk_iters = c.iters;
        pl->dp_tiles = 0;
        pl->dp_first = 0;
        pl->max_peers = (int32_t)(cdiv(I, ips) - 1);
        pl->fixup = fix_req == SK_FIXUP_AUTO ? (pl->max_peers >= kSpreadMinPeers ? SK_FIXUP_SPREAD : SK_FIXUP_SERIAL)
                                             : fix_req;
        // as for deep-k basic Stream-K: with 8 or more pieces per tile the
        // round-robin XCD placement puts equal pieces of different tiles on
        // one XCD
        if (pl->xcd_remap && sp >= 8) pl->xcd_remap = 0;
        return SK_OK;
    };
    if (sched == SK_SCHED_FIXED_SPLIT) return plan_fixed_split(cfg ? cfg->split : 0);
    // basic Stream-K over every tile: the model's grid for a fixup mode, and
    // its predicted time
    auto sk_grid = [&](bool spread, double *val) {
        const Model &m = spread ? m_spread : m_serial;
        const int g = model_grid(c.iters, c.imax, pg, m,
                                 [&](int gg) { return c.peers_within(c.iters, gg, SK_MAX_PEERS); });
        if (val) *val = model_time(c.iters, c.imax, g, m);
        return g;
    };
    // the fixup mode and grid of basic Stream-K with the model's grid
    auto sk_model = [&](int *fix) {
        if (fix_req == SK_FIXUP_SERIAL) { *fix = SK_FIXUP_SERIAL; return sk_grid(false, nullptr); }
        if (fix_req == SK_FIXUP_SPREAD) { *fix = SK_FIXUP_SPREAD; return sk_grid(true, nullptr); }
        double vs = 0.0, vp = 0.0;
        const int gs = sk_grid(false, &vs), gp = sk_grid(true, &vp);
        // the spread fixup only for a grid that gives some owner enough peers
        if (vp < vs && c.max_peers(0, c.iters, gp) >= kSpreadMinPeers) { *fix = SK_FIXUP_SPREAD; return gp; }
        *fix = SK_FIXUP_SERIAL;
        return gs;
    };
    int fix = SK_FIXUP_SERIAL;
    int64_t tail_split = 0;    // > 1: the automatic hybrid's fixed-split tail
    if (sched == SK_SCHED_AUTO) {
        // Measured on MI355X: Stream-K pays off while the tiles give no CU
        // more than one workgroup (t <= CUs: a lone workgroup leaves its
        // CU's second slot idle, which a Stream-K split fills -- 2048^2 x
        // 8192 BF16: DP 634, SK 889 TFLOP/s); from there on, one data-parallel
        // workgroup per tile is at least as fast as the hybrids -- with two
        // or more workgroups resident per CU the last partial wave costs
        // little, while a Stream-K region loses the k-aligned L2 reuse of
        // concurrently running tiles and pays for its fixups.
        // FP64: a k-tile's MFMA work is long next to its operand traffic,
        // so lost L2 reuse costs little and Stream-K's balance wins at every
        // size (FP64 sweep: basic SK 47.5, two-tile hybrid 47.8, the rule
        // above 43.7, DP 30.6 TFLOP/s): the paper's two-tile hybrid.
        // the 64x64 tile of the 16-bit and FP8 types: Stream-K only below
        // kTinySkTiles tiles, data-parallel otherwise (see the tile choice);
        // FP16/BF16 also up to 1.5 CUs' worth of tiles with kDeepIters
        // k-iterations per tile.  The refinements of the 16-bit default
        // (kDeepIters, kMidBig*, kTail*, aligned_split) are described with
        // their constants.
        const bool half = c.key.ab_type == SK_F16 || c.key.ab_type == SK_BF16;
        const bool single = c.probs.size() == 1;
        int64_t sk_tiles = (c.tile.bm <= 64 && c.key.ab_type != SK_F64) ? kTinySkTiles - 1 : cus;
        if (half && c.tile.bm <= 64 && c.imax >= kDeepIters) sk_tiles = std::max<int64_t>(sk_tiles, 3 * (int64_t)cus / 2 - 1);
        if (c.key.ab_type == SK_F64) sched = SK_SCHED_2TILE_SK_DP;
        else if (half && single && user_grid == 0 && c.tile.bm >= 256 && t <= cus &&
                 kMidBigDen * t >= kMidBigDp * (int64_t)cus)
            sched = SK_SCHED_DP;
        else if (t <= sk_tiles) {
            sched = SK_SCHED_SK;
            // a model grid of exactly one workgroup per tile (one problem)
            // is the data-parallel schedule: run the data-parallel kernel;
            // any other model grid of a single GEMM gives way to the
            // k-aligned fixed split when that fills enough of the slots
            // (128x128, FP16/BF16/FP8: half; 64x64, FP16/BF16: 5/8)
            int f0 = 0;
            if (user_grid == 0 && single && std::min<int64_t>(sk_model(&f0), c.iters) == t) {
                sched = SK_SCHED_DP;
            } else if ((half || c.key.ab_type == SK_F8_E4M3) && single && user_grid == 0 && c.tile.bm == 128) {
                const int64_t s_al = aligned_split(t, c.imax, pg, 1, 2);
                if (s_al > 1) return plan_fixed_split(s_al);
            } else if (half && single && user_grid == 0 && c.tile.bm == 64) {
                const int64_t s_al = aligned_split(t, c.imax, pg, 5, 8);
                if (s_al > 1) return plan_fixed_split(s_al);
            }
        } else {
            sched = SK_SCHED_DP;
            const int64_t tail = t % p;
            if (half && single && user_grid == 0 && c.tile.bm >= 256 && t > p && tail > 0 &&
                kTailDen * tail <= kTailNum * (int64_t)p && c.imax >= kDeepIters) {
                tail_split = tail_split_factor(tail, c.imax, pg);
                if (tail_split > 1) sched = SK_SCHED_DP_1TILE_SK;
            }
        }
    }
    if (sched == SK_SCHED_DP) {
        pl->sched = SK_SCHED_DP;
        pl->grid = (int32_t)t;
        pl->dp_first = 1;
        pl->dp_tiles = t;
        return SK_OK;
    }
    const int64_t w = t / p, r = t % p;
    int64_t skb = 0, ske = 0;
    int64_t g = 0;
    bool model_g = false;
    if (sched == SK_SCHED_SK || (w == 0 && r != 0)) {
        sched = SK_SCHED_SK;
        skb = 0;
        ske = t;
        model_g = user_grid == 0;
        g = model_g ? sk_model(&fix) : user_grid;
    } else if (r == 0) {
        // perfect quantisation: data-parallel waves only
        sched = SK_SCHED_DP_1TILE_SK;
        skb = ske = 0;
        g = user_grid > 0 ? user_grid : pg;
    } else if (sched == SK_SCHED_2TILE_SK_DP && w >= threshold) {
        skb = 0;
        ske = r + p;
        g = user_grid > 0 ? user_grid : pg;
    } else {
        sched = SK_SCHED_DP_1TILE_SK;
        skb = w * p;
        ske = t;
        g = user_grid > 0 ? user_grid : pg;
    }
    int64_t sk_iters = c.region_iters(skb, ske);
    // basic Stream-K never launches more workgroups than iterations; a
    // hybrid's grid also carries its data-parallel waves and keeps p (some
    // workgroups then have an empty Stream-K range)
    if (sched == SK_SCHED_SK && sk_iters > 0) g = std::max<int64_t>(1, std::min<int64_t>(g, sk_iters));
    int64_t sk_ib = skb < t ? c.tile_iter_begin(skb) : c.iters;
    int64_t mp = 0;
    if (sched == SK_SCHED_DP_1TILE_SK && ((cfg && cfg->split > 1) || tail_split > 1) && ske > skb) {
        // DP + one-tile SK with a fixed-split tail (Algorithm 4 on the tail
        // tiles): s workgroups per tail tile, k-aligned; the other
        // workgroups run only their data-parallel tiles.  Single GEMMs.
        if (c.probs.size() != 1) return SK_ERR_UNSUPPORTED;
        const int64_t sp = tail_split > 1 ? tail_split : cfg->split, ips = cdiv(c.imax, sp);
        if (sp > SK_MAX_PEERS + 1) return SK_ERR_UNSUPPORTED;
        if (sp * (ske - skb) > g) return SK_ERR_INVALID_VALUE;
        pl->split = (int32_t)sp;
        mp = cdiv(c.imax, ips) - 1;
    } else {
        mp = c.max_peers(sk_ib, sk_iters, g);
    }
    if (mp > SK_MAX_PEERS) {
        // only a hybrid the automatic schedule chose (or an explicit grid)
        // gets here: the automatic schedule falls back to basic Stream-K
        if (!auto_sched || user_grid > 0) return SK_ERR_UNSUPPORTED;
        sched = SK_SCHED_SK;
        skb = 0;
        ske = t;
        model_g = true;
        g = sk_model(&fix);
        sk_iters = c.iters;
        g = std::max<int64_t>(1, std::min<int64_t>(g, sk_iters));
        sk_ib = 0;
        mp = c.max_peers(0, sk_iters, g);
    }
    if (!model_g) {
        fix = fix_req == SK_FIXUP_AUTO ? (mp >= kSpreadMinPeers ? SK_FIXUP_SPREAD : SK_FIXUP_SERIAL) : fix_req;
    }
    // Deep-k basic Stream-K (every tile split over at least 8 workgroups):
    // the hardware's round-robin placement (workgroup x on XCD x mod 8) puts
    // the workgroups that run the same k-range of different tiles on one
    // XCD, whose L2 then serves the A and B k-slices those tiles share;
    // contiguous runs per XCD would give each XCD whole tiles at unrelated
    // k offsets.  Measured (BF16, 128x128 tiles, spread fixup): 256x256x65536
    // 34.8 -> 31.4 us, 512x512x32768 45.3 -> 34.7, 1024x1024x16384 56.3 ->
    // 48.1; with two workgroups per tile (4096x1024x4096) the contiguous
    // runs stay faster (45.2 vs 51.3).
    if (pl->xcd_remap && sched == SK_SCHED_SK && ske > skb && g >= 8 * (ske - skb)) pl->xcd_remap = 0;
    pl->sched = sched;
    pl->grid = (int32_t)g;
    pl->dp_first = sched == SK_SCHED_DP_1TILE_SK ? 1 : 0;
    pl->sk_tile_begin = skb;
    pl->sk_tile_end = ske;
    pl->sk_iter_begin = sk_ib;
    pl->sk_iters = sk_iters;
    pl->dp_tiles = t - (ske - skb);
    pl->fixup = fix;
    pl->max_peers = (int32_t)mp;
    return SK_OK;
}

// Plans of single GEMMs, cached by everything planning reads (device,
// shape, types, orders, leading dimensions and the configuration fields that
// steer the plan), so a shape seen before is launched without re-planning.
struct PlanKey {
    int32_t dev;
    int32_t ab, ct, ao, bo, co;
    int64_t m, n, k, lda, ldb, ldc;
    sk_config_t cfg;       // trace, trace_capacity and wait_limit_us zeroed
    int32_t has_cfg;
};

constexpr size_t kPlanCacheSize = 64;
std::mutex g_plan_mu;
std::vector<std::pair<PlanKey, sk_plan_t>> g_plan_cache;
size_t g_plan_next = 0;

bool plan_key(const sk_gemm_desc_t &d, const sk_config_t *cfg, PlanKey *k) {
    std::memset(k, 0, sizeof(*k));
    if (hipGetDevice(&k->dev) != hipSuccess) return false;
    k->ab = d.ab_type; k->ct = d.c_type;
    k->ao = d.a_order; k->bo = d.b_order; k->co = d.c_order;
    k->m = d.m; k->n = d.n; k->k = d.k;
    k->lda = d.lda; k->ldb = d.ldb; k->ldc = d.ldc;
    if (cfg) {
        k->has_cfg = 1;
        k->cfg.sched = cfg->sched;
        k->cfg.blk_m = cfg->blk_m; k->cfg.blk_n = cfg->blk_n; k->cfg.blk_k = cfg->blk_k;
        k->cfg.grid = cfg->grid;
        k->cfg.wg_slots = cfg->wg_slots;
        k->cfg.sk_threshold_waves = cfg->sk_threshold_waves;
        k->cfg.flags = cfg->flags;
        k->cfg.model_a = cfg->model_a; k->cfg.model_b = cfg->model_b;
        k->cfg.model_c = cfg->model_c; k->cfg.model_d = cfg->model_d;
        k->cfg.fixup = cfg->fixup;
        k->cfg.model_bw = cfg->model_bw;
        k->cfg.split = cfg->split;
    }
    return true;
}

// plan_call for one GEMM, through the cache
sk_status_t plan_single(const Call &c, const sk_gemm_desc_t &d, const sk_config_t *cfg, sk_plan_t *pl) {
    PlanKey key;
    const bool keyed = plan_key(d, cfg, &key);
    if (keyed) {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        for (const auto &e : g_plan_cache)
            if (std::memcmp(&e.first, &key, sizeof(key)) == 0) {
                *pl = e.second;
                return SK_OK;
            }
    }
    sk_status_t s = plan_call(c, cfg, pl);
    if (s != SK_OK || !keyed) return s;
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (g_plan_cache.size() < kPlanCacheSize) {
        g_plan_cache.push_back({key, *pl});
    } else {
        g_plan_cache[g_plan_next] = {key, *pl};
        g_plan_next = (g_plan_next + 1) % kPlanCacheSize;
    }
    return SK_OK;
}

struct Layout {
    size_t partials = 0, raw = 0, probs = 0, tpre = 0, ipre = 0, total = 0;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace: the header words, the fixed flag region (reserved in every
// workspace, so no table or partial tile is ever stored where a later call
// looks for flags), the partial-tile slots of a Stream-K plan (g of them for
// the serial fixup, 2g for the spread one), then the grouped descriptor
// tables.  The table region is always reserved (a few hundred bytes per
// problem), so one size serves sk_gemm and sk_gemm_grouped alike, including
// a grouped call with a single problem.
Layout layout_for(const sk_plan_t &pl, int ab, int32_t count) {
    Layout L;
    size_t off = WS_HEADER + FLAG_REGION;
    if (pl.sched != SK_SCHED_DP && pl.grid > 0) {
        L.partials = off;
        const size_t acc = ab == SK_F64 ? 8 : 4;
        const size_t slots = (size_t)pl.grid * (pl.fixup == SK_FIXUP_SPREAD ? 2 : 1);
        off = align256(off + slots * pl.blk_m * pl.blk_n * acc);
    }
    L.raw = off;
    off = align256(off + (size_t)count * sizeof(sk_gemm_desc_t));
    L.probs = off;
    off = align256(off + (size_t)count * sizeof(Problem));
    L.tpre = off;
    off = align256(off + (size_t)(count + 1) * sizeof(int32_t));
    L.ipre = off;
    off = align256(off + (size_t)(count + 1) * sizeof(int32_t));
    L.total = off;
    return L;
}

// Bound of one fixup wait when the caller gives none: 2 s of real time.
constexpr int64_t kWaitLimitUs = 2000000;

// Ticks per microsecond of the counter the kernels read for their bounded
// waits (s_memrealtime), per device.
std::vector<std::pair<int, int64_t>> g_clock_cache;

int64_t wait_ticks(const sk_config_t *cfg) {
    const int64_t us = (cfg && cfg->wait_limit_us != 0) ? cfg->wait_limit_us : kWaitLimitUs;
    if (us < 0) return 0;
    int dev = 0;
    int64_t khz = 100000;    // 100 MHz unless the device says otherwise
    if (hipGetDevice(&dev) == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_slot_mu);
        bool found = false;
        for (auto &e : g_clock_cache)
            if (e.first == dev) {
                khz = e.second;
                found = true;
            }
        if (!found) {
            int rate = 0;
            if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev) == hipSuccess && rate > 0)
                khz = rate;
            g_clock_cache.push_back({dev, khz});
        }
    }
    return std::max<int64_t>(1, us * khz / 1000);
}

// Tile rasterisation: bands of this many tile rows, walked column by column,
// so consecutive tiles (and the workgroups of one XCD) share A and B panels.
constexpr int kTileBand = 8;

Params make_params(const Call &c, const sk_plan_t &pl, const Layout &L, void *ws,
                   const sk_config_t *cfg) {
    Params P;
    std::memset(&P, 0, sizeof(P));
    P.prob = c.probs[0];
    P.tiles = (int32_t)c.tiles;
    P.g = pl.grid;
    P.sk_tile_begin = (int32_t)pl.sk_tile_begin;
    P.sk_tile_end = (int32_t)pl.sk_tile_end;
    P.sk_iter_begin = (int32_t)pl.sk_iter_begin;
    P.sk_iters = (int32_t)pl.sk_iters;
    P.dp_tiles = (int32_t)pl.dp_tiles;
    P.dp_first = pl.dp_first;
    P.xcd_remap = pl.xcd_remap;
    P.band = (cfg && (cfg->flags & SK_FLAG_ROW_MAJOR_TILES)) ? 1 : kTileBand;
    P.fixup = pl.fixup == SK_FIXUP_SPREAD ? FIXUP_SPREAD : FIXUP_SERIAL;
    // per-XCD tile queues for batches of several problems (tiles of
    // different cost); a single GEMM's equal tiles keep the static order,
    // which measured faster for them (FP16 sweep, 128x128 tiles: DP +
    // one-tile SK 327 vs 316 TFLOP/s, two-tile SK + DP 317 vs 313)
    P.split = pl.split;
    P.dyn_dp = (c.probs.size() > 1 && pl.sched != SK_SCHED_DP && pl.dp_tiles > pl.grid &&
                !(cfg && (cfg->flags & SK_FLAG_STATIC_DP_TILES))) ? 1 : 0;
    P.wait_ticks = wait_ticks(cfg);
    char *w = (char *)ws;
    P.hdr = (int32_t *)w;
    P.err = P.hdr + HDR_ERR;
    P.flags = (int32_t *)(w + WS_HEADER);
    if (L.partials) P.partials = w + L.partials;
    if (cfg && cfg->trace) {
        P.trace = cfg->trace;
        P.trace_cap = cfg->trace_capacity;
    }
    return P;
}

}  // namespace

extern "C" {

const char *sk_status_string(sk_status_t s) {
    switch (s) {
    case SK_OK: return "SK_OK";
    case SK_ERR_INVALID_VALUE: return "SK_ERR_INVALID_VALUE";
    case SK_ERR_UNSUPPORTED: return "SK_ERR_UNSUPPORTED";
    case SK_ERR_WORKSPACE_TOO_SMALL: return "SK_ERR_WORKSPACE_TOO_SMALL";
    case SK_ERR_MISALIGNED: return "SK_ERR_MISALIGNED";
    case SK_ERR_HIP: return "SK_ERR_HIP";
    case SK_ERR_TIMEOUT: return "SK_ERR_TIMEOUT";
    }
    return "SK_ERR_UNKNOWN";
}

sk_status_t sk_plan(const sk_gemm_desc_t *d, int32_t count, const sk_config_t *cfg, sk_plan_t *out) {
    if (!out) return SK_ERR_INVALID_VALUE;
    Call c;
    sk_status_t s = build_call(d, count, cfg, count > 1, &c);
    if (s != SK_OK) return s;
    s = count == 1 ? plan_single(c, d[0], cfg, out) : plan_call(c, cfg, out);
    if (s != SK_OK) return s;
    out->workspace_bytes = layout_for(*out, d[0].ab_type, count).total;
    return SK_OK;
}

sk_status_t sk_workspace_size(const sk_gemm_desc_t *d, int32_t count, const sk_config_t *cfg, size_t *bytes) {
    if (!bytes) return SK_ERR_INVALID_VALUE;
    sk_plan_t pl;
    sk_status_t s = sk_plan(d, count, cfg, &pl);
    if (s != SK_OK) return s;
    *bytes = (size_t)pl.workspace_bytes;
    return SK_OK;
}

}  // extern "C"

namespace {

// sk_gemm's body.  err: the error word a giving-up fixup wait sets (NULL:
// the workspace header's).
sk_status_t gemm_on(const sk_gemm_desc_t *d, const sk_config_t *cfg, void *workspace, size_t ws_bytes,
                    int32_t *err, void *stream) {
    if (!d) return SK_ERR_INVALID_VALUE;
    sk_status_t s = validate(*d);
    if (s != SK_OK) return s;
    if (d->m == 0 || d->n == 0) return SK_OK;
    if (d->k == 0 || d->alpha == 0.0) {
        Problem p = to_problem(*d, 1, 1, 1);
        return launch_scale_c(p, stream) == (int)hipSuccess ? SK_OK : SK_ERR_HIP;
    }
    Call c;
    s = build_call(d, 1, cfg, false, &c);
    if (s != SK_OK) return s;
    sk_plan_t pl;
    s = plan_single(c, *d, cfg, &pl);
    if (s != SK_OK) return s;
    Layout L = layout_for(pl, d->ab_type, 1);
    if (!workspace || ws_bytes < L.total) return SK_ERR_WORKSPACE_TOO_SMALL;
    KernelKey key = c.key;
    key.dp_only = pl.sched == SK_SCHED_DP;
    KernelEntry e = find_kernel(key);
    if (!e.launch) return SK_ERR_UNSUPPORTED;
    Params P = make_params(c, pl, L, workspace, cfg);
    if (err) P.err = err;
    return e.launch(P, pl.grid, stream) == (int)hipSuccess ? SK_OK : SK_ERR_HIP;
}

// ---------------------------------------------------------------------------
// Workspace that needs no allocation: a fixed device array, one copy per GPU
// the library runs on, kept until the process ends.  Host code never passes
// the array's name to a kernel or a copy (on the host it is only a stand-in
// for the symbol); it uses the per-device address hipGetSymbolAddress gives.
// ---------------------------------------------------------------------------
static_assert(SK_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
static __device__ __align__(256) char scratch[SK_NOALLOC_SCRATCH_BYTES];

// Header words and flag region of a fresh workspace: zeroed by a kernel (a
// memset node would not be safe under stream capture).
__global__ void zero_words_kernel(int32_t *w, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) w[i] = 0;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The scratch address on the current device; the first call on a device
// looks it up and enqueues the zeroing of its header and flag region on
// `stream` (stream order puts it before the caller's launch).
sk_status_t scratch_for_current_device(void *stream, void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SK_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SK_ERR_HIP;
        const int words = (WS_HEADER + FLAG_REGION) / 4;
        hipLaunchKernelGGL(zero_words_kernel, dim3((words + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                           (int32_t *)ptr, words);
        if (hipGetLastError() != hipSuccess) return SK_ERR_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SK_OK;
}

}  // namespace

extern "C" {

sk_status_t sk_gemm(const sk_gemm_desc_t *d, const sk_config_t *cfg, void *workspace, size_t ws_bytes,
                    void *stream) {
    return gemm_on(d, cfg, workspace, ws_bytes, nullptr, stream);
}

sk_status_t sk_gemm_noalloc(const sk_gemm_desc_t *d, const sk_config_t *cfg, int32_t *wait_error, void *stream) {
    if (!d) return SK_ERR_INVALID_VALUE;
    sk_status_t s = validate(*d);
    if (s != SK_OK) return s;
    if (d->m == 0 || d->n == 0) return SK_OK;
    // C = beta C needs no workspace
    if (d->k == 0 || d->alpha == 0.0) return gemm_on(d, cfg, nullptr, 0, wait_error, stream);
    // the plan's workspace must fit the scratch array (checked before the
    // device is touched)
    size_t need = 0;
    s = sk_workspace_size(d, 1, cfg, &need);
    if (s != SK_OK) return s;
    if (need > (size_t)SK_NOALLOC_SCRATCH_BYTES) return SK_ERR_WORKSPACE_TOO_SMALL;
    void *ws = nullptr;
    s = scratch_for_current_device(stream, &ws);
    if (s != SK_OK) return s;
    return gemm_on(d, cfg, ws, (size_t)SK_NOALLOC_SCRATCH_BYTES, wait_error, stream);
}

sk_status_t sk_gemm_grouped(const sk_gemm_desc_t *d, int32_t count, const sk_config_t *cfg, void *workspace,
                            size_t ws_bytes, void *stream) {
    Call c;
    sk_status_t s = build_call(d, count, cfg, true, &c);
    if (s != SK_OK) return s;
    sk_plan_t pl;
    s = plan_call(c, cfg, &pl);
    if (s != SK_OK) return s;
    Layout L = layout_for(pl, d[0].ab_type, count);
    if (!workspace || ws_bytes < L.total) return SK_ERR_WORKSPACE_TOO_SMALL;
    if (c.tiles == 0) return SK_OK;
    KernelKey key = c.key;
    key.dp_only = pl.sched == SK_SCHED_DP;
    KernelEntry e = find_kernel(key);
    if (!e.launch) return SK_ERR_UNSUPPORTED;
    char *w = (char *)workspace;
    if (hipMemcpyAsync(w + L.raw, d, sizeof(sk_gemm_desc_t) * (size_t)count, hipMemcpyHostToDevice,
                       (hipStream_t)stream) != hipSuccess)
        return SK_ERR_HIP;
    GroupTable tab;
    tab.probs = (Problem *)(w + L.probs);
    tab.tile_prefix = (int32_t *)(w + L.tpre);
    tab.iter_prefix = (int32_t *)(w + L.ipre);
    tab.count = count;
    if (launch_group_prep((const sk_gemm_desc_t *)(w + L.raw), count, c.tile.bm, c.tile.bn, c.tile.bk, tab,
                          stream) != (int)hipSuccess)
        return SK_ERR_HIP;
    Params P = make_params(c, pl, L, workspace, cfg);
    P.group = tab;
    return e.launch(P, pl.grid, stream) == (int)hipSuccess ? SK_OK : SK_ERR_HIP;
}

sk_status_t sk_workspace_check(void *workspace, size_t ws_bytes, void *stream) {
    if (!workspace || ws_bytes < (size_t)(WS_HEADER + FLAG_REGION)) return SK_ERR_INVALID_VALUE;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return SK_ERR_HIP;
    int32_t err = 0;
    if (hipMemcpy(&err, workspace, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) return SK_ERR_HIP;
    if (err == 0) return SK_OK;
    // A wait gave up.  Every workgroup still finished and the generation
    // moved on, so no flag of that call can be mistaken for a later call's;
    // the header and the flag region are reset anyway, to the state of a
    // freshly zeroed workspace.
    if (hipMemsetAsync(workspace, 0, (size_t)(WS_HEADER + FLAG_REGION), (hipStream_t)stream) != hipSuccess ||
        hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return SK_ERR_HIP;
    return SK_ERR_TIMEOUT;
}

}  // extern "C"
