/*
 * streamk.h -- C ABI of the MI355X (gfx950) Stream-K GEMM library.
 *
 * The library computes the GEMM of the paper's problem statement (section 2):
 *     C = alpha * A * B + beta * C,   A: m x k,  B: k x n,  C: m x n
 * with the work-centric Stream-K decomposition (section 4, Algorithm 5): a
 * persistent grid of g workgroups splits the m->n->k linearised MAC-loop
 * iteration space evenly, a workgroup may start or stop inside an output
 * tile, and partial tiles are reconciled through a workspace with per-slot
 * ready flags.  The data-parallel schedule (section 3.2, Algorithm 2) and the
 * two hybrids of section 5.2 run in the same kernels.
 *
 * Conventions shared by every entry point:
 *  - Only plain C types and pointers cross the boundary.  Device pointers are
 *    HIP device addresses owned by the caller; `stream` is a hipStream_t
 *    passed as void* (NULL = the null stream).  The library allocates no
 *    device memory and keeps no mutable global state, so calls on distinct
 *    workspaces may be issued from several host threads.
 *  - Every entry point validates all arguments on the host before anything
 *    is enqueued and returns an sk_status_t.  Compute entry points are
 *    asynchronous: SK_OK means the work was enqueued on `stream`.
 *  - Enumerations are passed as int32_t fields so the struct layout is fixed.
 */
#ifndef STREAMK_H
#define STREAMK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SK_OK = 0,
    SK_ERR_INVALID_VALUE = 1,      /* bad dimension, pointer, ld, scale, count */
    SK_ERR_UNSUPPORTED = 2,        /* dtype / order / tile combination not built */
    SK_ERR_WORKSPACE_TOO_SMALL = 3,
    SK_ERR_MISALIGNED = 4,         /* see the alignment rule below */
    SK_ERR_HIP = 5,                /* a HIP runtime call failed (no device, launch error) */
    SK_ERR_TIMEOUT = 6             /* a fixup wait exceeded its bound (sk_workspace_check) */
} sk_status_t;

typedef enum { SK_ROW_MAJOR = 0, SK_COL_MAJOR = 1 } sk_order_t;

/* F8_E4M3 is the OCP e4m3fn format (max 448, no infinities). */
typedef enum { SK_F64 = 0, SK_F32 = 1, SK_F16 = 2, SK_BF16 = 3, SK_F8_E4M3 = 4 } sk_dtype_t;

/* Work decompositions (paper sections 3.2, 4 and 5.2). */
typedef enum {
    SK_SCHED_AUTO = 0,          /* library default, measured on MI355X: per problem a tile and one of
                                   the schedules below -- Stream-K while t <= CUs (for a single
                                   16-bit or F8 GEMM on 128x128 tiles preferably the fixed split that
                                   fills at least half of the slots), else DP, with DP + one-tile SK
                                   (its tail a fixed split) for a last wave of at most half the slots
                                   of 256x256 tiles; F64: the two-tile SK + DP hybrid */
    SK_SCHED_DP = 1,            /* data-parallel: one workgroup per output tile (Algorithm 2) */
    SK_SCHED_SK = 2,            /* basic Stream-K over all tiles (Algorithm 5), g from the model */
    SK_SCHED_DP_1TILE_SK = 3,   /* full DP waves, then SK over the remaining tiles on g = p */
    SK_SCHED_2TILE_SK_DP = 4,   /* SK over r + p tiles first (1..2 tiles per WG), then DP waves */
    SK_SCHED_FIXED_SPLIT = 5    /* fixed split (Algorithm 4): s workgroups per tile, workgroup
                                   x s + y running iterations [y ceil(I/s), min(I, (y+1) ceil(I/s)))
                                   of tile x, g = s t; single GEMMs only (grouped calls:
                                   SK_ERR_UNSUPPORTED) */
} sk_sched_t;

/*
 * One GEMM.  Element (i, j) of a rows x cols matrix X stored in order o with
 * leading dimension ld (in elements) is X[i*ld + j] (row-major) or
 * X[j*ld + i] (column-major).  ld == 0 means packed (cols resp. rows).
 *
 * Supported (ab_type -> c_type): F64 -> F64; F16 -> F32 | F16;
 * BF16 -> BF16 | F32; F8_E4M3 -> BF16 | F32.  Products accumulate in FP32
 * (FP64 for F64) and are never rounded to a narrower type before the final
 * store.  alpha and beta are applied once, by the workgroup that writes the
 * tile, in the accumulator precision; beta == 0 means C is not read.  For F8
 * the stored codes are dequantised by the per-tensor scales:
 *     C = alpha * (a_scale*A) * (b_scale*B) + beta * C;
 * a_scale and b_scale must be finite and > 0 (and 1.0 for other dtypes).
 *
 * Alignment rule: A, B and C must be aligned to their element size and A
 * and B to 16 bytes; for A and B, the leading dimension and the extent of the
 * contiguous dimension (k for row-major A, m for column-major A, n for
 * row-major B, k for column-major B) must be multiples of 16 bytes' worth of
 * elements (8 for F16/BF16, 16 for F8, 2 for F64).  Otherwise SK_ERR_MISALIGNED.
 * m == 0 or n == 0 is a no-op; k == 0 or alpha == 0 gives C = beta * C.
 */
typedef struct {
    int64_t m, n, k;
    double alpha, beta;
    int32_t ab_type, c_type;              /* sk_dtype_t */
    int32_t a_order, b_order, c_order;    /* sk_order_t */
    int32_t reserved0;
    int64_t lda, ldb, ldc;
    const void *A;
    const void *B;
    void *C;
    float a_scale, b_scale;
} sk_gemm_desc_t;

/*
 * Launch configuration; every field 0 (or NULL) selects the library default.
 *  sched            sk_sched_t.
 *  blk_m/n/k        tile shape; must be one built for the dtype.  Built:
 *                   F64 128x128x16 (default), 64x64x16; F16/BF16 256x256x64,
 *                   128x128x64, 64x64x64; F8 256x256x128, 128x128x128,
 *                   64x64x128 (the 64x64 tiles only when asked for).  F16/BF16/F8
 *                   default: the 128x128 tile unless the problem has at least 2
 *                   (F16/BF16) or 8 (F8) full waves of those tiles (t >= 2 p,
 *                   t >= 8 p), then the 256x256 tile.
 *                   AUTO's "CUs" is the device's CU count, or wg_slots divided
 *                   by the tile's workgroups per CU by LDS (160 KiB / (2 (BM +
 *                   BN) 128 B)) when wg_slots is given.
 *  grid             g, the number of persistent workgroups (SK schedules).
 *                   Must not exceed wg_slots (a fixup waits for other
 *                   workgroups, so all g must be co-resident) nor SK_MAX_GRID.
 *  wg_slots         p, resident workgroup slots (CUs x workgroups per CU for
 *                   the chosen kernel); 0 = queried from the current device.
 *  sk_threshold_waves  full waves w at and above which AUTO / 2TILE use the
 *                   two-tile hybrid (below it, DP + one-tile SK); 0 = 2.
 *  flags            SK_FLAG_* bits.
 *  model_a..d       grid-size model constants of appendix A.1 (any unit);
 *                   all zero = the library's calibrated constants.
 *  trace            optional device buffer receiving one record per executed
 *                   segment (for schedule verification); trace[0] is an
 *                   int32 record counter the caller zeroes, records of 8
 *                   int32 {wg, seq, tile, k_begin, k_end, role, last_peer, x}
 *                   start at trace[8].  Records beyond trace_capacity are
 *                   dropped (the counter still counts them).
 *                   Data-parallel tiles taken from the per-XCD queues (see
 *                   SK_FLAG_STATIC_DP_TILES) are recorded under the
 *                   workgroup that ran them, in its order.
 *                   role: 0 DP tile, 1 whole tile in one SK segment,
 *                   2 owner (its tile's later contributors end at last_peer),
 *                   3 producer (stores one partial tile), 4 slice reduction
 *                   of the spread fixup (k_begin/k_end: the 16-byte chunk
 *                   range of the tile's partial tiles it reduced; x: the
 *                   tile's first contributor; last_peer: its last).
 *  wait_limit_us    bound of one fixup wait in microseconds of real time;
 *                   0 = 2 s.  Negative: a wait gives up at once (testing
 *                   only: a call with any split tile then reports
 *                   SK_ERR_TIMEOUT and its results are undefined).
 *  fixup            SK_FIXUP_*: how split tiles are reconciled.
 *  model_bw         device bytes per microsecond for an optional memory term
 *                   of the grid model: every workgroup of a plan that splits
 *                   tiles is charged 2 BM BN acc_bytes / model_bw for writing
 *                   and reading back its partial tile; 0 = no memory term.
 *  split            SK_SCHED_FIXED_SPLIT's splitting factor s (1..SK_MAX_PEERS
 *                   + 1, s t <= wg_slots: all s t workgroups co-resident);
 *                   0 = the largest such s that leaves no workgroup without
 *                   iterations.  s = 1 is the data-parallel schedule.  A
 *                   nonzero grid must equal s t.  With SK_SCHED_DP_1TILE_SK,
 *                   s > 1 makes the Stream-K tail of r tiles a fixed split
 *                   (workgroup x < s r runs piece x mod s of tail tile x / s;
 *                   s r <= grid, single GEMMs); 0 or 1 = the even split.
 */
typedef struct {
    int32_t sched;
    int32_t blk_m, blk_n, blk_k;
    int32_t grid;
    int32_t wg_slots;
    int32_t sk_threshold_waves;
    int32_t flags;
    double model_a, model_b, model_c, model_d;
    int32_t *trace;
    int64_t trace_capacity;
    int32_t wait_limit_us;
    int32_t fixup;
    double model_bw;
    int32_t split;
} sk_config_t;

#define SK_FLAG_NO_XCD_REMAP 0x1     /* keep logical workgroup id == hardware id */
#define SK_FLAG_ROW_MAJOR_TILES 0x2  /* tile t -> (t / tiles_n, t % tiles_n) instead of banded order */
/* A persistent launch of several problems (sk_gemm_grouped, count > 1) with
 * more data-parallel tiles than workgroups gives workgroup x the
 * data-parallel tile x first, then takes the others from
 * eight per-XCD queues (contiguous eighths of the remaining tiles, each in
 * order, an emptied queue taking from the next XCDs' ones), so uneven
 * tiles (grouped problems of different k) balance over the workgroups; the
 * results are the same bits either way (no data-parallel tile is split).
 * This flag keeps the static order of section 4's data-parallel schedule
 * instead: tiles x, x + g, x + 2g, ... to workgroup x. */
#define SK_FLAG_STATIC_DP_TILES 0x4

/* Largest persistent grid, and the most peers one tile's owner may wait on
 * (plans beyond it are rejected with SK_ERR_UNSUPPORTED, or avoided when the
 * library picks the grid). */
#define SK_MAX_GRID 1024
#define SK_MAX_PEERS 64

/* Fixup of a tile split over workgroups f..l (f ran the tile's first
 * iteration).  SERIAL is Algorithm 5: f's successors store partial tiles and
 * f adds them, in ascending order, before writing the tile.  SPREAD: every
 * contributor stores its partial tile and then reduces 1/(l-f+1) of the tile
 * over all of them, in the same ascending order, so both give identical
 * bits.  AUTO (0): SPREAD when some owner has at least two peers. */
typedef enum { SK_FIXUP_AUTO = 0, SK_FIXUP_SERIAL = 1, SK_FIXUP_SPREAD = 2 } sk_fixup_t;

/* The resolved launch plan of a call (host only; no device access when
 * cfg->wg_slots > 0). */
typedef struct {
    int32_t sched;            /* resolved schedule (never AUTO) */
    int32_t blk_m, blk_n, blk_k;
    int32_t grid;             /* workgroups launched */
    int32_t wg_slots;         /* p used for the decision */
    int32_t dp_first;         /* 1: each WG runs its DP tiles before its SK range */
    int32_t xcd_remap;        /* 1: logical ids grouped per XCD */
    int64_t tiles;            /* output tiles over all problems */
    int64_t iters_total;      /* MAC-loop iterations over all problems */
    int64_t sk_tile_begin, sk_tile_end;   /* SK region, in global tile order */
    int64_t sk_iter_begin, sk_iters;      /* the same region in iterations */
    int64_t dp_tiles;         /* tiles outside the SK region */
    uint64_t workspace_bytes;
    int32_t fixup;            /* resolved sk_fixup_t (never AUTO) */
    int32_t max_peers;        /* largest peer count of any tile's owner */
    int32_t split;            /* SK_SCHED_FIXED_SPLIT: its s; SK_SCHED_DP_1TILE_SK: the
                                 fixed-split tail's s (0: even split); otherwise 0 */
} sk_plan_t;

/* Plan the call without launching it: the schedule (sections 3.2, 4, 5.2),
 * the grid (appendix A.1 model), the Stream-K region and the fixup.  d points
 * to `count` descriptors (count == 1 for sk_gemm).  Pure host computation;
 * the device is only queried for its CU count when cfg->wg_slots is 0. */
sk_status_t sk_plan(const sk_gemm_desc_t *d, int32_t count, const sk_config_t *cfg,
                    sk_plan_t *out);

/* Workspace bytes needed by sk_gemm (count == 1) or sk_gemm_grouped with the
 * same descriptors and configuration: the header and the fixed flag region,
 * then (Stream-K schedules only) the partial-tile slots of Algorithm 5's
 * StorePartials -- one BM x BN accumulator tile per workgroup, two with the
 * SPREAD fixup -- then the grouped call's descriptor and problem tables.
 * The workspace is device memory owned by the caller; it must be
 * zero-filled before its first use.  Flags are raised with a per-call epoch
 * and never cleared, so a completed call leaves the workspace ready for the
 * next one without any reset.  One workspace serves one call in flight at a
 * time; calls that overlap on one workspace race.
 * Errors: SK_ERR_INVALID_VALUE (bytes NULL, or a descriptor rejected as by
 * sk_gemm), SK_ERR_UNSUPPORTED (no such kernel, or a plan whose owner would
 * wait on more than SK_MAX_PEERS peers). */
sk_status_t sk_workspace_size(const sk_gemm_desc_t *d, int32_t count,
                              const sk_config_t *cfg, size_t *bytes);

/* One GEMM (section 2: C = alpha A B + beta C), enqueued on `stream` as one
 * kernel launch of the plan sk_plan returns: data-parallel tiles
 * (Algorithm 2), basic Stream-K (Algorithm 5, the grid from the appendix A.1
 * model unless cfg->grid is set) or a section 5.2 hybrid.  A, B, C are
 * device pointers owned by the caller; `workspace` (ws_bytes >= what
 * sk_workspace_size returns) holds the partial tiles and flags.  cfg may be
 * NULL.  All validation happens before anything is enqueued: on any status
 * other than SK_OK nothing was launched and C is untouched. */
sk_status_t sk_gemm(const sk_gemm_desc_t *d, const sk_config_t *cfg,
                    void *workspace, size_t ws_bytes, void *stream);

/* Bytes of the device scratch array behind sk_gemm_noalloc: one copy on
 * every GPU the library runs on, held until the process ends. */
#define SK_NOALLOC_SCRATCH_BYTES (80u << 20)

/* sk_gemm for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same plan, kernels and results as sk_gemm with the same d and cfg, but the
 * workspace is the library's fixed scratch array on the current device
 * (SK_NOALLOC_SCRATCH_BYTES).  Nothing is allocated by this call or by the
 * library on its behalf.  A plan whose workspace (sk_workspace_size) exceeds
 * the array is rejected with SK_ERR_WORKSPACE_TOO_SMALL before anything is
 * enqueued (choose a smaller grid, the SERIAL fixup or the DP schedule).
 * The first call on a device also enqueues, on `stream`, the zeroing of the
 * array's header and flag region.  Every call on one GPU shares its array:
 * calls that overlap on one GPU (on different streams, or from several host
 * threads without ordering) race and give undefined results.
 * wait_error: optional device int32 (NULL = not reported) into which the
 * kernels OR 1 if a fixup wait gave up (the call's results are then
 * undefined); the caller zeroes it. */
sk_status_t sk_gemm_noalloc(const sk_gemm_desc_t *d, const sk_config_t *cfg,
                            int32_t *wait_error, void *stream);

/* `count` independent GEMMs with the same ab_type, c_type and orders but any
 * shapes, pointers, alpha, beta and scales, in one persistent launch whose
 * Stream-K iteration space is the concatenation of the problems' spaces
 * (problem index outermost): section 4's even split of the MAC-loop
 * iterations applied to the union of the problems' tiles, each problem's
 * tiles linearised m -> n -> k as for one GEMM.  Problems with m, n or k
 * equal to zero contribute no tiles (k == 0 or alpha == 0: C = beta C).
 * Validation and errors as sk_gemm; a count < 1 is SK_ERR_INVALID_VALUE.  d is host memory; it is copied into the
 * workspace stream-ordered, so it must stay valid until the stream reaches
 * this call (pinned memory is required under stream capture, and replays of
 * a captured call read d again: shapes must then be unchanged). */
sk_status_t sk_gemm_grouped(const sk_gemm_desc_t *d, int32_t count,
                            const sk_config_t *cfg, void *workspace,
                            size_t ws_bytes, void *stream);

/* Synchronise `stream` and read the workspace's error word.  Returns
 * SK_ERR_TIMEOUT if a fixup wait (Algorithm 5's Wait, bounded here in real
 * time) gave up since the last check; the header and the flag region are
 * then reset to the zero-filled state, so the workspace can be used again.
 * SK_ERR_INVALID_VALUE for a NULL or undersized workspace. */
sk_status_t sk_workspace_check(void *workspace, size_t ws_bytes, void *stream);

/* Static text for a status code (never NULL; unknown codes get a generic
 * text). */
const char *sk_status_string(sk_status_t s);

#ifdef __cplusplus
}
#endif
#endif /* STREAMK_H */
