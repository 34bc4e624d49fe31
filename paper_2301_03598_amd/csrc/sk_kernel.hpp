// Stream-K GEMM kernels for gfx950 (CDNA4): MFMA mainloop, partial-tile
// fixup and the data-parallel / Stream-K / hybrid work walk.
//
// Work decomposition (paper section 4, Algorithm 5): the MAC-loop iterations
// of the Stream-K region (tiles in m->n->k order, k innermost) are split into
// g contiguous ranges whose lengths differ by at most one; each workgroup
// walks its range tile by tile.  A segment that does not start at its tile's
// first iteration stores its accumulators to its own workspace slot and
// raises its flag; the segment that does start there (the owner) adds the
// later contributors' slots in ascending workgroup order, so the summation
// order is fixed and runs are bitwise repeatable, then applies alpha/beta and
// writes the tile.  Tiles outside the Stream-K region are produced whole, in
// data-parallel waves (section 5.2 hybrids; Algorithm 2 when g = tiles).
//
// MAC loop (Algorithm 3): each k-tile of BLK_K is staged from global memory
// into LDS with 16-byte loads and consumed by MFMA instructions from LDS,
// double-buffered so the global loads of k-tile i+1 overlap the MFMAs of
// k-tile i.  LDS rows are 128 bytes of one A row (or B column) along k, the
// 16-byte chunks of a row XOR-swizzled by the row index so the MFMA operand
// reads and the stores are free of bank conflicts.  An operand that is
// contiguous along m (or n) is transposed in registers on its way to LDS.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "sk_internal.h"

namespace sk {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Bit casts go through by-value helpers: applied directly to an element of
// an ext_vector_type lvalue, __builtin_bit_cast reads element 0 of the vector.
__device__ __forceinline__ uint32_t f2u(float f) { return __builtin_bit_cast(uint32_t, f); }
__device__ __forceinline__ float u2f(uint32_t u) { return __builtin_bit_cast(float, u); }
__device__ __forceinline__ uint64_t d2u(double d) { return __builtin_bit_cast(uint64_t, d); }
__device__ __forceinline__ double u2d(uint64_t u) { return __builtin_bit_cast(double, u); }

// Compile-time loop: f(integral_constant<int, 0>), ..., f(<N-1>).  Used
// where accumulator fragments are indexed, so every index is a constant even
// when the body is too large for the loop unroller.
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

enum class Dt { F64, F16, BF16, F8 };

template <Dt D> struct DtTraits;
template <> struct DtTraits<Dt::F64> {
    static constexpr int E = 8;     // bytes per element
    static constexpr int MT = 16;   // MFMA output block edge
    using Acc = double;
    using Frag = f64x4;             // one 16x16 output block per lane
    static constexpr int FRAG_N = 4;
};
template <> struct DtTraits<Dt::F16> {
    static constexpr int E = 2, MT = 32, FRAG_N = 16;
    using Acc = float;
    using Frag = f32x16;
};
template <> struct DtTraits<Dt::BF16> {
    static constexpr int E = 2, MT = 32, FRAG_N = 16;
    using Acc = float;
    using Frag = f32x16;
};
template <> struct DtTraits<Dt::F8> {
    static constexpr int E = 1, MT = 32, FRAG_N = 16;
    using Acc = float;
    using Frag = f32x16;
};

template <Dt D, int BM_, int BN_, bool AKC_, bool BKC_, bool GROUPED_, int NW_ = 4>
struct Cfg {
    static constexpr Dt DT = D;
    static constexpr bool AKC = AKC_, BKC = BKC_, GROUPED = GROUPED_;
    // waves per workgroup, arranged 2 (along m) x NW/2 (along n); each wave
    // instruction of LDS-DMA staging moves 1 KiB, so one round of all waves
    // moves NW KiB
    static constexpr int NW = NW_, THREADS = 64 * NW_;
    static constexpr int WGM = 2, WGN = NW_ / 2;
    static constexpr int DMA_ROUND = 1024 * NW_;
    static_assert(NW_ == 4 || NW_ == 8, "four or eight waves");
    static constexpr int E = DtTraits<D>::E;
    static constexpr int VEC = 16 / E;          // elements per 16-byte load
    static constexpr int BK = 8 * VEC;          // MAC-loop iteration: 128 bytes of k
    static constexpr int BM = BM_, BN = BN_;
    // staged k-tile: KROW bytes of k per LDS row (64-byte rows -- half
    // iterations, four buffers -- were measured slower for the 256x256
    // 16-bit tile: twice the barriers, and the extra lead bought nothing)
    static constexpr int KROW = 128;
    static constexpr int BKS = KROW / E;        // k per staged k-tile
    static constexpr int SUB = BK / BKS;        // staged k-tiles per MAC-loop iteration
    static constexpr int WTM = BM / WGM, WTN = BN / WGN;   // the wave's block of C
    static constexpr int MT = DtTraits<D>::MT;
    static constexpr int FM = WTM / MT, FN = WTN / MT;
    static constexpr int FRAG_N = DtTraits<D>::FRAG_N;
    static constexpr int A_BYTES = BM * KROW, B_BYTES = BN * KROW;
    static constexpr int STAGE = A_BYTES + B_BYTES;
    // LDS k-tile buffers.  FP64 keeps three (its k-tiles carry half the
    // bytes of a 16-bit one for the same MFMA time, so its loads need two
    // k-tiles of lead to hide their latency; one workgroup per CU leaves the
    // room).
    static constexpr int NSTAGE = D == Dt::F64 ? 3 : (KROW == 64 ? 4 : 2);
    static constexpr int LDS = NSTAGE * STAGE;
    static constexpr int DMA_PER_KTILE = STAGE / DMA_ROUND;   // LDS-DMA loads per wave per staged k-tile
    // k-tile instruction order pinned for the scheduler (MFMAs interleaved
    // with the loads and fragment reads, barrier before the last k-step):
    // measured faster for the 16-bit 256x256 tile (one workgroup, so one
    // wave, per SIMD) and for FP8; slower for the 16-bit 128x128 tile (two
    // workgroups per CU cover each other's stalls) and FP64, which keep the
    // compiler's order
    static constexpr bool ORDERED = NW == 4 && (D == Dt::F8 || (E == 2 && BM >= 256));
    // the first fixup peer is staged through LDS (not for the 256x256 FP8
    // tile, whose transpose-read fragments leave no registers for it)
    static constexpr bool FIX_LDS = !(D == Dt::F8 && BM >= 256);
    // peers whose partial fragments are loaded together in the fixup (the
    // 256x256 tiles have no registers for more than one at a time)
    static constexpr int PEER_BATCH = BM >= 256 ? 1 : 4;
    using Acc = typename DtTraits<D>::Acc;
    using Frag = typename DtTraits<D>::Frag;
    static constexpr int ACC_N = FM * FN * FRAG_N;     // accumulators per thread
    static constexpr int ACC_CHUNKS = ACC_N * (int)sizeof(Acc) / 16;
    static constexpr int SLOT_BYTES = BM * BN * (int)sizeof(Acc);
    static_assert(BM * BN == THREADS * ACC_N && FM >= 1 && FN >= 1, "accumulator split");
};

// LDS byte offset of 16-byte chunk c of row r (KROW-byte rows, XOR
// swizzle).  The LDS serves a 16-byte-per-lane access 16 lanes per cycle
// across 64 banks (256 bytes): 256/KROW consecutive rows share one bank
// row, so the swizzle key is row/(256/KROW).  Then 16 lanes reading the
// same chunk of 16 consecutive rows all hit distinct banks.
template <int KROW>
__device__ __forceinline__ uint32_t lds_off(uint32_t row, uint32_t chunk) {
    if constexpr (KROW == 128) return row * 128u + (((chunk ^ (row >> 1)) & 7u) << 4);
    else return row * 64u + (((chunk ^ (row >> 2)) & 3u) << 4);
}

// ---------------------------------------------------------------------------
// global -> LDS staging of one operand tile (ROWS x BK) with LDS-DMA loads
//
// The operand is seen as a ROWS x k matrix X with element (r, p) at
// KC ? r*ld + p : p*ld + r.  Each wave instruction moves 1 KiB: lane L's 16
// bytes land at the wave's LDS block + 16 L, so the XOR swizzles are applied
// by choosing which global chunk each lane fetches.
//  KC (rows x k, k contiguous): the block is 1024/KROW rows of KROW bytes in
//    the lds_off layout; lane L fetches row L/(KROW/16), chunk
//    (L % (KROW/16)) ^ swizzle(row).
//  !KC (k x rows, rows contiguous): LDS k-row p holds the tile's ROWS
//    values (E*ROWS bytes) with 16-byte chunk c at slot c ^ sw(p) (see
//    nkc_swizzle); the block is 1024 / (E*ROWS) k-rows.
// Loads outside the matrix get an offset past the resource range and
// deposit zeros.
// ---------------------------------------------------------------------------
// Chunk swizzle of k-row p in the !KC (natural) layout, chosen so that the
// fragment reads -- 16-bit transpose reads: 4 consecutive k-rows x 32 bytes
// per 16 lanes; 8-bit: 8 consecutive k-rows x 16 bytes; FP64: 4 k-rows two
// apart x 128 bytes -- hit every bank once per 256 bytes.  A k-row of 256
// bytes fills the 64 banks; one of 128 (64) bytes shares them with 1 (3)
// neighbours.  The swizzled chunk stays inside its k-row: the value is below
// the k-row's chunk count (ROWS * E / 16).
template <int E, int ROWS>
__device__ __forceinline__ int nkc_swizzle(int p) {
    constexpr int RB = ROWS * E;     // bytes per k-row
    static_assert(RB >= 64, "at least four chunks per k-row");
    if constexpr (E == 8) {
        static_assert(RB >= 256, "FP64 swizzle needs 16 chunks");
        return 8 * ((p >> 1) & 1);
    } else if constexpr (E == 2) {
        // 256-byte k-rows: the 4 k-rows of a read share the banks;
        // 128-byte k-rows: k-rows p and p + 2 do
        if constexpr (RB >= 256) return 4 * (p & 3);
        else return 2 * ((p >> 1) & 1);
    } else {
        // 8 consecutive k-rows per read: 256-byte k-rows all share the banks,
        // 128-byte ones in fours, 64-byte ones in pairs (p and p + 4)
        if constexpr (RB >= 256) return 2 * (p & 7);
        else if constexpr (RB == 128) return 2 * ((p >> 1) & 3);
        else return 2 * ((p >> 2) & 1);
    }
}

template <class C, int ROWS, bool KC>
struct StageDma {
    static constexpr int E = C::E, VEC = C::VEC, BK = C::BKS, KROW = C::KROW;
    static constexpr int NW = C::NW;
    static constexpr int NL = ROWS * KROW / C::DMA_ROUND;   // loads per wave per staged k-tile
    static constexpr int RPB = 1024 / KROW;         // KC: rows per 1 KiB block
    static constexpr int LPR = KROW / 16;           // KC: lanes per row
    static constexpr int CPR = ROWS * E / 16;       // !KC: chunks per k-row
    static constexpr int KR = 1024 / (ROWS * E);    // !KC: k-rows per 1 KiB block
    static_assert(BK * E == KROW && KR >= 1 && NL >= 1, "whole rows per 1 KiB block");
    static constexpr uint32_t OOB = 0x80000000u;
    const char *ub;
    int64_t ustep;
    uint32_t ustride;
    uint32_t voff;
    int rows_valid;        // KC: number of valid leading loads (row edge)
    bool mn_valid;         // !KC: this lane's chunk lies inside the matrix
    int kofs;              // k offset of this lane's first load within a k-tile
    uint32_t lds_w;        // the wave's first block within the operand stage

    __device__ __forceinline__ void init(const void *ptr, int64_t ld, int row0, int rows_total, int tid) {
        const char *p = (const char *)ptr;
        const int w = __builtin_amdgcn_readfirstlane(tid >> 6), L = tid & 63;
        if constexpr (KC) {
            // rows rr + 4*RPB*i; the swizzle key is the same for every i
            const int rr = RPB * w + L / LPR;
            const int key = KROW == 128 ? (rr >> 1) & 7 : (rr >> 2) & 3;
            const int c = (L % LPR) ^ key;
            ub = p + (int64_t)row0 * ld * E;
            ustep = (int64_t)BK * E;
            ustride = (uint32_t)(NW * RPB * ld * E);
            voff = (uint32_t)(((int64_t)rr * ld + c * VEC) * E);
            const int rem = rows_total - row0 - rr;
            rows_valid = rem <= 0 ? 0 : (rem + NW * RPB - 1) / (NW * RPB);
            kofs = c * VEC;
            lds_w = (uint32_t)(w * 1024);
        } else {
            const int pr = w * KR + L / CPR;            // k-row of load 0 within the k-tile
            const int c = (L % CPR) ^ nkc_swizzle<E, ROWS>(pr);
            ub = p + (int64_t)row0 * E;
            ustep = (int64_t)BK * ld * E;
            ustride = (uint32_t)(NW * KR * ld * E);
            voff = (uint32_t)(((int64_t)pr * ld + c * VEC) * E);
            mn_valid = row0 + c * VEC < rows_total;
            kofs = pr;
            lds_w = (uint32_t)(w * 1024);
        }
    }

    __device__ __forceinline__ void dma(const __amdgpu_buffer_rsrc_t &rs, char *dst, uint32_t o, uint32_t so) const {
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)dst, 16, o, so, 0, 0);
    }

    // Issue the loads of k-tile kt into the operand stage at `lds`.  live
    // false: the loads still run (out of range, depositing zeros), so the
    // caller needs no branch around them.  interior: no row or k edge.
    // ORDERED configurations stay branch-free (a k-tile is one basic block,
    // whose loads the scheduler places between the MFMAs); the others take
    // a branch to the plain interior loads.
    __device__ __forceinline__ void issue(char *lds, int kt, int K, bool live, bool interior) const {
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void *)(ub + kt * ustep), (short)0, 0x7fffffff, 0x00020000);
        constexpr int BLK = C::DMA_ROUND;               // LDS bytes between a wave's blocks
        if (!C::ORDERED && live && interior) {
#pragma unroll
            for (int i = 0; i < NL; ++i) dma(rs, lds + lds_w + i * BLK, voff, i * ustride);
        } else if constexpr (KC) {
            const bool kv = live && (interior || kt * BK + kofs < K);
#pragma unroll
            for (int i = 0; i < NL; ++i)
                dma(rs, lds + lds_w + i * BLK, (kv && (interior || i < rows_valid)) ? voff : OOB, i * ustride);
        } else {
            const int k0 = kt * BK + kofs;
#pragma unroll
            for (int i = 0; i < NL; ++i)
                dma(rs, lds + lds_w + i * BLK, (live && (interior || (mn_valid && k0 + i * NW * KR < K))) ? voff : OOB,
                    i * ustride);
        }
    }
};

// Wait for this wave's LDS-DMA loads to land: all of them, or all but the
// newest N (vector-memory loads complete in issue order).
__device__ __forceinline__ void wait_dma() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
template <int N>
__device__ __forceinline__ void wait_dma_but() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    // s_waitcnt encoding: vmcnt[3:0] and [15:14], expcnt [6:4] = 7 and
    // lgkmcnt [11:8] = 15 (no wait on those)
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
    asm volatile("" ::: "memory");
}

// The MAC loop's LDS k-tile buffers: separate LDS objects (NSTAGE of them
// in use), selected by compile-time index.
struct LdsBufs {
    char *b0, *b1, *b2, *b3;
    template <int I>
    __device__ __forceinline__ char *get() const {
        if constexpr (I == 0) return b0;
        else if constexpr (I == 1) return b1;
        else if constexpr (I == 2) return b2;
        else return b3;
    }
};

// ---------------------------------------------------------------------------
// MFMA operand fragments
//
// 32x32 MFMAs (f16/bf16/f8): lane l feeds row (l % 32) of the A block (and
// column (l % 32) of the B block) with a contiguous run of k from lane group
// q = l / 32: 8 values (one 16-byte chunk) for f16/bf16, 32 values (two
// chunks) for f8.  A k-tile (8 chunks) is NSUB such k-steps.
// 16x16x4 f64 MFMA: lane group q = l / 16 supplies one k value per MFMA; one
// chunk read gives a lane two consecutive k values (2q and 2q+1 of an 8-k
// half of the row) consumed by two MFMAs.  A and B use the same assignment,
// so every k of the k-tile meets its partner exactly once.
// ---------------------------------------------------------------------------
template <class C>
struct Frag {
    static constexpr int CPM = (C::DT == Dt::F8) ? 2 : 1;          // chunks per lane per operand
    static constexpr int CHUNKS = C::KROW / 16;                     // chunks per staged LDS row
    static constexpr int NSUB = (C::DT == Dt::F64) ? CHUNKS / 4 : CHUNKS / (2 * CPM);   // k-steps per staged k-tile
    // MFMAs and LDS fragment reads per k-step
    static constexpr int MFMAS = C::FM * C::FN * (C::DT == Dt::F64 ? 2 : 1);
    static constexpr int READS_PER_FRAG = C::DT == Dt::F8 ? 4 : 2;   // transpose / 8-byte reads
    static constexpr int READS = (C::AKC ? C::FM * CPM : C::FM * READS_PER_FRAG) +
                                 (C::BKC ? C::FN * CPM : C::FN * READS_PER_FRAG);
    u32x4 a[C::FM][CPM], b[C::FN][CPM];
};

template <class C>
__device__ __forceinline__ int frag_chunk(int ks, int q, int s) {
    if constexpr (C::DT == Dt::F64) return ks * 4 + q;
    else return ks * 2 * Frag<C>::CPM + q * Frag<C>::CPM + s;
}

// One 16-bit MFMA operand fragment from a !KC operand stage (k-rows of ROWS
// values, chunk-swizzled): lane l needs rows base + l%32 at k = 8(l/32)..+7 of
// k-step ks.  ds_read_b64_tr_b16 hands lane l of a 16-lane group element l%4
// of the 4-value runs read by lanes 4e + (l%16)/4, e = 0..3, so source lane
// s (s16 = s%16, group g = s/16) reads k-row ks*16 + 8(g/2) + 4h + s16/4 at
// rows base + 16(g%2) + 4(s16%4); two reads (h = 0, 1) give the 8 k values.
template <class C, int ROWS>
__device__ __forceinline__ u32x4 frag_tr(const char *op, uint32_t base, int ks, int lane) {
    typedef short s16x4 __attribute__((ext_vector_type(4)));
    constexpr int RB = ROWS * 2;
    const int g = lane >> 4, s16 = lane & 15;
    const uint32_t r0 = base + 16 * (g & 1) + 4 * (s16 & 3);
    const uint32_t p = (uint32_t)(ks * 16 + 8 * (g >> 1) + (s16 >> 2));
    const uint32_t off = p * RB + (((r0 >> 3) ^ (uint32_t)nkc_swizzle<2, ROWS>((int)p)) << 4) + (r0 & 7) * 2;
    const s16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s16x4 *)(op + off));
    const s16x4 hi =
        __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s16x4 *)(op + off + 4 * RB));
    const u32x2 l2 = __builtin_bit_cast(u32x2, lo), h2 = __builtin_bit_cast(u32x2, hi);
    return u32x4{l2[0], l2[1], h2[0], h2[1]};
}

// One FP8 MFMA operand fragment (32 k values per lane) from a !KC operand
// stage: lane l needs rows base + l%32 at k = ks*64 + 32(l/32) + 0..31.
// ds_read_b64_tr_b8 hands lane l of a 16-lane group byte l%8 of the 8-byte
// runs read by lanes 2e + (l%16)/8, e = 0..7, so source lane s (group g)
// reads k-row ks*64 + 32(g/2) + 8h + s/2 at rows base + 16(g%2) + 8(s%2);
// four reads (h = 0..3) give the lane's 32 k values.
template <class C, int ROWS>
__device__ __forceinline__ void frag_tr8(u32x4 (&out)[2], const char *op, uint32_t base, int ks, int lane) {
    typedef int i32x2 __attribute__((ext_vector_type(2)));
    constexpr int RB = ROWS;
    const int g = lane >> 4, s16 = lane & 15;
    const uint32_t r0 = base + 16 * (g & 1) + 8 * (s16 & 1);
    uint32_t w[8];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        const int p = ks * 64 + 32 * (g >> 1) + 8 * h + (s16 >> 1);
        const uint32_t off = (uint32_t)p * RB + (((r0 >> 4) ^ (uint32_t)nkc_swizzle<1, ROWS>(p)) << 4) + (r0 & 15);
        const i32x2 v =
            __builtin_amdgcn_ds_read_tr8_b64_v2i32((__attribute__((address_space(3))) i32x2 *)(op + off));
        w[2 * h] = (uint32_t)v[0];
        w[2 * h + 1] = (uint32_t)v[1];
    }
    out[0] = u32x4{w[0], w[1], w[2], w[3]};
    out[1] = u32x4{w[4], w[5], w[6], w[7]};
}

// One FP64 MFMA operand fragment from a !KC operand stage: lane l (row
// base + l%16, group q = l/16) needs k = 8ks + 2q and 8ks + 2q + 1 (one per
// MFMA of the pair); 16 lanes read 128 consecutive bytes of one k-row.
template <class C, int ROWS>
__device__ __forceinline__ u32x4 frag_f64_nkc(const char *op, uint32_t base, int ks, int lane) {
    constexpr int RB = ROWS * 8;
    const int q = lane >> 4;
    const uint32_t r = base + (lane & 15);
    u32x2 h[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int p = 8 * ks + 2 * q + e;
        const uint32_t off = (uint32_t)p * RB + (((r >> 1) ^ (uint32_t)nkc_swizzle<8, ROWS>(p)) << 4) + (r & 1) * 8;
        h[e] = *(const u32x2 *)(op + off);
    }
    return u32x4{h[0][0], h[0][1], h[1][0], h[1][1]};
}

template <class C>
__device__ __forceinline__ void read_frags(Frag<C> &f, const char *ldsA, const char *ldsB, uint32_t arow,
                                           uint32_t brow, int ks, int q) {
    if constexpr (!C::AKC && C::DT == Dt::F64) {
        const int lane = (int)(arow % 16) + 16 * q;
#pragma unroll
        for (int i = 0; i < C::FM; ++i) f.a[i][0] = frag_f64_nkc<C, C::BM>(ldsA, arow - arow % 16 + i * C::MT, ks, lane);
    } else if constexpr (!C::AKC && C::DT == Dt::F8) {
        const int lane = (int)(arow % 32) + 32 * q;
#pragma unroll
        for (int i = 0; i < C::FM; ++i) frag_tr8<C, C::BM>(f.a[i], ldsA, arow - arow % 32 + i * C::MT, ks, lane);
    } else if constexpr (!C::AKC) {
        const int lane = (int)(arow % 32) + 32 * q;
#pragma unroll
        for (int i = 0; i < C::FM; ++i) f.a[i][0] = frag_tr<C, C::BM>(ldsA, arow - arow % 32 + i * C::MT, ks, lane);
    } else {
#pragma unroll
        for (int s = 0; s < Frag<C>::CPM; ++s) {
            const int c = frag_chunk<C>(ks, q, s);
#pragma unroll
            for (int i = 0; i < C::FM; ++i) f.a[i][s] = *(const u32x4 *)(ldsA + lds_off<C::KROW>(arow + i * C::MT, c));
        }
    }
    if constexpr (!C::BKC && C::DT == Dt::F64) {
        const int lane = (int)(brow % 16) + 16 * q;
#pragma unroll
        for (int j = 0; j < C::FN; ++j) f.b[j][0] = frag_f64_nkc<C, C::BN>(ldsB, brow - brow % 16 + j * C::MT, ks, lane);
    } else if constexpr (!C::BKC && C::DT == Dt::F8) {
        const int lane = (int)(brow % 32) + 32 * q;
#pragma unroll
        for (int j = 0; j < C::FN; ++j) frag_tr8<C, C::BN>(f.b[j], ldsB, brow - brow % 32 + j * C::MT, ks, lane);
    } else if constexpr (!C::BKC) {
        const int lane = (int)(brow % 32) + 32 * q;
#pragma unroll
        for (int j = 0; j < C::FN; ++j) f.b[j][0] = frag_tr<C, C::BN>(ldsB, brow - brow % 32 + j * C::MT, ks, lane);
    } else {
#pragma unroll
        for (int s = 0; s < Frag<C>::CPM; ++s) {
            const int c = frag_chunk<C>(ks, q, s);
#pragma unroll
            for (int j = 0; j < C::FN; ++j) f.b[j][s] = *(const u32x4 *)(ldsB + lds_off<C::KROW>(brow + j * C::MT, c));
        }
    }
}

__device__ __forceinline__ double lo_d(const u32x4 &x) { return u2d((uint64_t)x[0] | ((uint64_t)x[1] << 32)); }
__device__ __forceinline__ double hi_d(const u32x4 &x) { return u2d((uint64_t)x[2] | ((uint64_t)x[3] << 32)); }

// One k-step of MFMAs.  ZERO: the accumulators start from the constant 0
// (the first k-step of a segment), so they need no separate clearing.
template <class C, bool ZERO>
__device__ __forceinline__ void mfma_step(typename C::Frag (&acc)[C::FM][C::FN], const Frag<C> &f) {
#pragma unroll
    for (int i = 0; i < C::FM; ++i)
#pragma unroll
        for (int j = 0; j < C::FN; ++j) {
            const typename C::Frag cin = ZERO ? typename C::Frag{} : acc[i][j];
            if constexpr (C::DT == Dt::F64) {
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(lo_d(f.a[i][0]), lo_d(f.b[j][0]), cin, 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(hi_d(f.a[i][0]), hi_d(f.b[j][0]), acc[i][j], 0, 0, 0);
            } else if constexpr (C::DT == Dt::BF16) {
                // D = B_frag * A_frag: the transposed block (see the output layout)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    __builtin_bit_cast(bf16x8, f.b[j][0]), __builtin_bit_cast(bf16x8, f.a[i][0]), cin, 0, 0, 0);
            } else if constexpr (C::DT == Dt::F16) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                    __builtin_bit_cast(f16x8, f.b[j][0]), __builtin_bit_cast(f16x8, f.a[i][0]), cin, 0, 0, 0);
            } else {
                const i32x8 av = __builtin_shufflevector(__builtin_bit_cast(i32x4, f.a[i][0]),
                                                         __builtin_bit_cast(i32x4, f.a[i][1]), 0, 1, 2, 3, 4, 5, 6, 7);
                const i32x8 bv = __builtin_shufflevector(__builtin_bit_cast(i32x4, f.b[j][0]),
                                                         __builtin_bit_cast(i32x4, f.b[j][1]), 0, 1, 2, 3, 4, 5, 6, 7);
                // formats 0/0 = FP8 e4m3 for both operands; E8M0 scales of
                // 2^0 (127): the per-tensor FP32 scales go into alpha
                acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(bv, av, cin, 0, 0, 0, 127, 0, 127);
            }
        }
}

// ---------------------------------------------------------------------------
// The MAC loop over iterations [it0, it1) of one tile (Algorithm 3)
//
// Per k-tile i: the LDS-DMA loads of k-tile i+1 go to the other LDS buffer
// (free since the last barrier); the k-steps of k-tile i run with their
// operand fragments double-buffered in registers (the reads of step s+1
// overlap the MFMAs of step s); the wave waits for its loads, one barrier,
// then the first fragments of k-tile i+1 are read.
// ---------------------------------------------------------------------------
template <class C>
struct Ctx {
    StageDma<C, C::BM, C::AKC> sa;
    StageDma<C, C::BN, C::BKC> sb;
};

// Instruction order of one staged k-tile, for the scheduler's group
// barriers.  With one workgroup per CU each SIMD runs a single wave, which
// issues in order: a burst of loads stalls the MFMAs queued behind it.  So
// the k-tile's MFMAs go one by one, its DMA issues spread over the first
// k-step's MFMAs (early enough that they land by the k-tile's end), and
// each k-step's fragment reads for the next k-step spread over the first
// half of its MFMAs (so they have landed when the next k-step starts).
template <class C>
__device__ __forceinline__ void order_ktile() {
    constexpr int NSUB = Frag<C>::NSUB, MF = Frag<C>::MFMAS, RD = Frag<C>::READS;
    constexpr int DMA = C::DMA_PER_KTILE, SPAN = MF;
    constexpr int RSPAN = MF >= 2 ? MF / 2 : 1;     // reads go in the step's first half
    static_for<NSUB * MF>([&](auto gg) {
        constexpr int g = decltype(gg)::value, m = g % MF;
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                 // one MFMA
        constexpr int nd = g < SPAN ? (g + 1) * DMA / SPAN - g * DMA / SPAN : 0;
        if constexpr (nd > 0) __builtin_amdgcn_sched_group_barrier(0x010, nd, 0);   // DMA issues
        constexpr int nr = m < RSPAN ? (m + 1) * RD / RSPAN - m * RD / RSPAN : 0;
        if constexpr (nr > 0) __builtin_amdgcn_sched_group_barrier(0x100, nr, 0);   // fragment reads
    });
}

// Wait until at most n (< LA) staged k-tiles of this wave's loads are
// still in flight (each staged k-tile is DPK loads).
template <int LA, int DPK>
__device__ __forceinline__ void wait_landed(int n) {
    if constexpr (LA >= 3) {
        if (n >= 2) {
            wait_dma_but<2 * DPK>();
            return;
        }
    }
    if constexpr (LA >= 2) {
        if (n >= 1) {
            wait_dma_but<DPK>();
            return;
        }
    }
    wait_dma();
}

// One staged k-tile.  FIRST: the segment's first, whose first k-step starts
// the accumulators from zero.  P: which buffer holds it.  With NSTAGE
// buffers the loads run NSTAGE - 1 staged k-tiles ahead.  The buffers are
// distinct LDS objects, so the compiler can tell that the fragment reads of
// one never wait for the DMA writes into another.
//  ORDERED: one basic block -- loads past the segment's end are issued out
//  of range (they deposit zeros into a free buffer), the barrier comes
//  before the last k-step's MFMAs, which then cover the first fragment reads
//  of the next k-tile (read unconditionally: after the segment's last k-tile
//  they are dead), and order_ktile pins the interleaving.
//  Otherwise: loads and the next k-tile's first reads sit behind branches
//  and the barrier ends the k-tile.
template <class C, bool FIRST, int P>
__device__ __forceinline__ void ktile_dma(Ctx<C> &cx, Frag<C> (&f)[2], typename C::Frag (&acc)[C::FM][C::FN],
                                          const LdsBufs &bufs, int it, int it1, bool rows_in, int kfull, int K,
                                          uint32_t arow, uint32_t brow, int q) {
    constexpr int NSUB = Frag<C>::NSUB;
    constexpr int NS = C::NSTAGE, LA = NS - 1;
    const char *st = bufs.template get<P>();
    const char *nx = bufs.template get<(P + 1) % NS>();
    char *ld = bufs.template get<(P + LA) % NS>();
    const bool live = it + LA < it1;
    const bool in = rows_in && it + LA < kfull;
    if constexpr (C::ORDERED) {
        cx.sa.issue(ld, it + LA, K, live, in);
        cx.sb.issue(ld + C::A_BYTES, it + LA, K, live, in);
        static_for<NSUB - 1>([&](auto kk) {
            constexpr int ks = decltype(kk)::value;
            read_frags<C>(f[(ks + 1) & 1], st, st + C::A_BYTES, arow, brow, ks + 1, q);
            mfma_step<C, FIRST && ks == 0>(acc, f[ks & 1]);
        });
        // staged k-tile it+1 must have landed; the LA-1 after it may still
        // be in flight (every k-tile issues the same number of loads)
        wait_dma_but<(LA - 1) * C::DMA_PER_KTILE>();
        __syncthreads();
        read_frags<C>(f[0], nx, nx + C::A_BYTES, arow, brow, 0, q);
        mfma_step<C, false>(acc, f[(NSUB - 1) & 1]);
        order_ktile<C>();
    } else {
        if (live) {
            cx.sa.issue(ld, it + LA, K, true, in);
            cx.sb.issue(ld + C::A_BYTES, it + LA, K, true, in);
        }
        static_for<NSUB>([&](auto kk) {
            constexpr int ks = decltype(kk)::value;
            if constexpr (ks + 1 < NSUB) read_frags<C>(f[(ks + 1) & 1], st, st + C::A_BYTES, arow, brow, ks + 1, q);
            mfma_step<C, FIRST && ks == 0>(acc, f[ks & 1]);
        });
        // staged k-tile it+1 must have landed; newer ones may stay in flight
        const int newer = it1 - 1 - (it + 1) < LA - 1 ? it1 - 1 - (it + 1) : LA - 1;
        wait_landed<LA, C::DMA_PER_KTILE>(newer);
        __syncthreads();
        if (it + 1 < it1) read_frags<C>(f[0], nx, nx + C::A_BYTES, arow, brow, 0, q);
    }
}

template <class C>
__device__ __forceinline__ void mac_loop(const Problem &P, int tm, int tn, int it0, int it1,
                                         typename C::Frag (&acc)[C::FM][C::FN], const LdsBufs &bufs,
                                         int tid) {
    if (it0 >= it1) {
        // an empty range (never produced by the planner, which sends k == 0
        // work to the C = beta*C kernel): zero accumulators via a
        // zero-operand k-step
        Frag<C> z;
#pragma unroll
        for (int s = 0; s < Frag<C>::CPM; ++s) {
#pragma unroll
            for (int i = 0; i < C::FM; ++i) z.a[i][s] = u32x4{0u, 0u, 0u, 0u};
#pragma unroll
            for (int j = 0; j < C::FN; ++j) z.b[j][s] = u32x4{0u, 0u, 0u, 0u};
        }
        mfma_step<C, true>(acc, z);
        return;
    }
    static_assert(Frag<C>::NSUB % 2 == 0, "fragment double buffer needs an even step count");
    const int lane = tid & 63, wave = tid >> 6, wm = wave / C::WGN, wn = wave % C::WGN;
    const int q = C::MT == 16 ? (lane >> 4) : (lane >> 5);
    const uint32_t arow = (uint32_t)(wm * C::WTM + (lane % C::MT));
    const uint32_t brow = (uint32_t)(wn * C::WTN + (lane % C::MT));
    const int row0 = tm * C::BM, col0 = tn * C::BN;
    Ctx<C> cx;
    cx.sa.init(P.A, P.lda, row0, P.m, tid);
    cx.sb.init(P.B, P.ldb, col0, P.n, tid);
    const bool rows_in = (row0 + C::BM <= P.m) && (col0 + C::BN <= P.n);
    // the loop runs over staged k-tiles: SUB per MAC-loop iteration
    const int s0 = it0 * C::SUB, s1 = it1 * C::SUB;
    const int kfull = P.k / C::BKS;                // staged k-tiles with no k edge
    constexpr int NS = C::NSTAGE, LA = NS - 1;
    // ORDERED issues every prologue load (out of range past the segment's
    // end), so the loads in flight are always LA staged k-tiles
    static_for<LA>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        const bool in = rows_in && s0 + j < kfull;
        if (C::ORDERED || s0 + j < s1) {
            cx.sa.issue(bufs.template get<j>(), s0 + j, P.k, s0 + j < s1, in);
            cx.sb.issue(bufs.template get<j>() + C::A_BYTES, s0 + j, P.k, s0 + j < s1, in);
        }
    });
    if constexpr (C::ORDERED) wait_dma_but<(LA - 1) * C::DMA_PER_KTILE>();
    else wait_landed<LA, C::DMA_PER_KTILE>(s1 - 1 - s0 < LA - 1 ? s1 - 1 - s0 : LA - 1);
    __syncthreads();
    Frag<C> f[2];
    read_frags<C>(f[0], bufs.b0, bufs.b0 + C::A_BYTES, arow, brow, 0, q);
    ktile_dma<C, true, 0>(cx, f, acc, bufs, s0, s1, rows_in, kfull, P.k, arow, brow, q);
    // staged k-tiles in groups of NSTAGE so the buffer of each is a constant
    for (int it = s0 + 1; it < s1; it += NS) {
        ktile_dma<C, false, 1 % NS>(cx, f, acc, bufs, it, s1, rows_in, kfull, P.k, arow, brow, q);
        if constexpr (NS >= 2) {
            if (it + 1 < s1) ktile_dma<C, false, 2 % NS>(cx, f, acc, bufs, it + 1, s1, rows_in, kfull, P.k, arow, brow, q);
        }
        if constexpr (NS >= 3) {
            if (it + 2 < s1) ktile_dma<C, false, 3 % NS>(cx, f, acc, bufs, it + 2, s1, rows_in, kfull, P.k, arow, brow, q);
        }
        if constexpr (NS >= 4) {
            if (it + 3 < s1) ktile_dma<C, false, 4 % NS>(cx, f, acc, bufs, it + 3, s1, rows_in, kfull, P.k, arow, brow, q);
        }
    }
    // ORDERED with more than two buffers would leave the out-of-range loads
    // past the segment's end in flight; the epilogue's staging reuses the
    // buffers, so they must land first (the other path waits for every load
    // in its last k-tile)
    if constexpr (C::ORDERED && LA > 1) wait_dma();
}

// ---------------------------------------------------------------------------
// accumulator <-> (row, col) and the epilogue
// ---------------------------------------------------------------------------
// Output layout of a fragment.
// 32x32 blocks (f16/bf16/f8): the MFMAs compute D = B_frag * A_frag, the
// transposed block, so lane l holds C row (l % 32) of the block and, in
// accumulator register 4g+e, column 8g + 4(l / 32) + e: four consecutive
// columns per group g, stored as one vector.
// 16x16 f64 blocks: D = A_frag * B_frag; lane l holds column (l % 16) and,
// in register r, row 4r + (l / 16).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
    return __builtin_bit_cast(float, (uint32_t)b << 16);
}

template <int CT, class Acc>
__device__ __forceinline__ Acc load_c(const char *p) {
    if constexpr (CT == SK_F64) return (Acc)(*(const double *)p);
    else if constexpr (CT == SK_F32) return (Acc)(*(const float *)p);
    else if constexpr (CT == SK_F16) return (Acc)(float)(*(const _Float16 *)p);
    else return (Acc)bf16_to_f32(*(const uint16_t *)p);
}

template <int CT, class Acc>
__device__ __forceinline__ void put_c(char *p, Acc v) {
    if constexpr (CT == SK_F64) *(double *)p = (double)v;
    else if constexpr (CT == SK_F32) *(float *)p = (float)v;
    else if constexpr (CT == SK_F16) *(_Float16 *)p = (_Float16)(float)v;
    else *(uint16_t *)p = f32_to_bf16_rne((float)v);
}

template <int CT> struct CBytes { static constexpr int v = CT == SK_F64 ? 8 : (CT == SK_F32 ? 4 : 2); };

// Four consecutive outputs of one row, alpha*acc (+ beta*C), rounded once.
template <int CT, class Acc>
__device__ __forceinline__ void put4(char *p, const Acc (&v)[4], Acc beta, bool rd) {
    constexpr int EB = CBytes<CT>::v;
    Acc w[4];
    if (rd) {
        if constexpr (CT == SK_F64) {
            const f64x4 o = *(const f64x4 *)p;
            for (int e = 0; e < 4; ++e) w[e] = v[e] + beta * (Acc)o[e];
        } else if constexpr (CT == SK_F32) {
            const u32x4 o = *(const u32x4 *)p;
            for (int e = 0; e < 4; ++e) w[e] = v[e] + beta * (Acc)u2f(o[e]);
        } else {
            const u32x2 o = *(const u32x2 *)p;
            for (int e = 0; e < 4; ++e) {
                const uint16_t h = (uint16_t)(o[e >> 1] >> ((e & 1) * 16));
                float f = CT == SK_F16 ? (float)__builtin_bit_cast(_Float16, h) : bf16_to_f32(h);
                w[e] = v[e] + beta * (Acc)f;
            }
        }
    } else {
        for (int e = 0; e < 4; ++e) w[e] = v[e];
    }
    if constexpr (CT == SK_F64) {
        *(f64x4 *)p = f64x4{(double)w[0], (double)w[1], (double)w[2], (double)w[3]};
    } else if constexpr (CT == SK_F32) {
        *(u32x4 *)p = u32x4{f2u((float)w[0]), f2u((float)w[1]), f2u((float)w[2]), f2u((float)w[3])};
    } else {
        uint32_t h[4];
        for (int e = 0; e < 4; ++e)
            h[e] = CT == SK_F16 ? (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(float)w[e])
                                : (uint32_t)f32_to_bf16_rne((float)w[e]);
        *(u32x2 *)p = u32x2{h[0] | (h[1] << 16), h[2] | (h[3] << 16)};
    }
    (void)EB;
}

// Partial tiles: thread-fragment order, 16-byte chunk v of thread t at
// slot + (v*THREADS + t)*16, so stores and loads are fully coalesced.
template <class C>
struct PartialLayout {
    static constexpr int PER = 16 / (int)sizeof(typename C::Acc);   // accumulators per chunk
    static constexpr int CPF = C::FRAG_N / PER;                      // chunks per fragment
    __device__ static __forceinline__ int64_t off(int i, int j, int s, int tid) {
        return ((int64_t)((i * C::FN + j) * CPF + s) * C::THREADS + tid) * 16;
    }
};

// One fragment of a partial tile, as a whole vector.
// Cache policy of every partial-tile and flag access: device scope (SC1).
// The eight XCDs have separate L2 caches; accesses with device scope are
// coherent across them by themselves, so publishing a partial tile needs
// neither an L2 write-back on the producer side nor an L2 invalidate on the
// owner side (the agent-scope release/acquire fences would issue both, and
// an invalidate per poll evicts the operand tiles of every other workgroup on
// that XCD).
constexpr int CPOL_DEVICE = 16;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t slot_rsrc(const char *slot, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)slot, (short)0, bytes, 0x00020000);
}

template <class C>
__device__ __forceinline__ typename C::Frag load_partial_frag(const char *slot, int i, int j, int tid) {
    using PL = PartialLayout<C>;
    const __amdgpu_buffer_rsrc_t rs = slot_rsrc(slot, C::SLOT_BYTES);
    u32x4 c[PL::CPF];
#pragma unroll
    for (int s = 0; s < PL::CPF; ++s)
        c[s] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, (uint32_t)PL::off(i, j, s, tid),
                                                                             0, CPOL_DEVICE));
    if constexpr (PL::PER == 4) {
        const f32x8 lo = __builtin_shufflevector(__builtin_bit_cast(f32x4, c[0]), __builtin_bit_cast(f32x4, c[1]), 0,
                                                 1, 2, 3, 4, 5, 6, 7);
        const f32x8 hi = __builtin_shufflevector(__builtin_bit_cast(f32x4, c[2]), __builtin_bit_cast(f32x4, c[3]), 0,
                                                 1, 2, 3, 4, 5, 6, 7);
        return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15);
    } else {
        return __builtin_shufflevector(__builtin_bit_cast(f64x2, c[0]), __builtin_bit_cast(f64x2, c[1]), 0, 1, 2, 3);
    }
}

// v + the fragment of the partial tiles in slots [p0, p1], added in
// ascending slot order.
template <class C>
__device__ __forceinline__ typename C::Frag add_peers(typename C::Frag v, const char *slots, int p0, int p1,
                                                      int i, int j, int tid) {
    // PEER_BATCH peers' fragments are loaded before they are added (one
    // memory round trip per batch); the additions keep ascending order
    int peer = p0;
    if constexpr (C::PEER_BATCH > 1) {
        for (; peer + C::PEER_BATCH - 1 <= p1; peer += C::PEER_BATCH) {
            typename C::Frag x[C::PEER_BATCH];
#pragma unroll
            for (int u = 0; u < C::PEER_BATCH; ++u)
                x[u] = load_partial_frag<C>(slots + (int64_t)(peer + u) * C::SLOT_BYTES, i, j, tid);
#pragma unroll
            for (int u = 0; u < C::PEER_BATCH; ++u) v = v + x[u];
        }
    }
    for (; peer <= p1; ++peer)
        v = v + load_partial_frag<C>(slots + (int64_t)peer * C::SLOT_BYTES, i, j, tid);
    return v;
}

// The first peer's partial tile is staged through the (then idle) MAC-loop
// LDS buffers by LDS-DMA loads, in FIX_PH phases, so its fragments are read
// with LDS latency instead of one global round trip each.  Each wave stages
// exactly the chunks its own lanes read back (partial chunk v of thread t
// sits at v*4096 + 16t in both places), so a wave only waits for its own
// loads; a barrier after the epilogue keeps the next unit's DMA away.
template <class C>
struct FixStage {
    static constexpr int PH = C::SLOT_BYTES > 2 * C::STAGE ? C::SLOT_BYTES / (2 * C::STAGE) : 1;   // phases
    static constexpr int VPH = C::ACC_CHUNKS / PH;                    // chunks per thread per phase
    static constexpr int H = VPH / 2;                                 // chunks per buffer
    static constexpr int ROWS_PH = C::FM / PH;                        // fragment rows per phase
    static constexpr int RB = C::DMA_ROUND;                           // bytes of one chunk of every thread
    static_assert(H * RB <= C::STAGE && C::FM % PH == 0 && VPH % 2 == 0, "fixup staging fits the LDS");

    // stage chunks [ph*VPH, (ph+1)*VPH) of the slot
    __device__ static __forceinline__ void issue(const char *slot, char *lds0, char *lds1, int ph, int tid) {
        const __amdgpu_buffer_rsrc_t rs = slot_rsrc(slot, C::SLOT_BYTES);
        const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
#pragma unroll
        for (int u = 0; u < VPH; ++u) {
            char *dst = (u < H ? lds0 : lds1) + (u % H) * RB + w * 1024;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)dst, 16,
                                                     (uint32_t)tid * 16u, (uint32_t)((ph * VPH + u) * RB), 0,
                                                     CPOL_DEVICE);
        }
    }

    // fragment (i, j) of the staged slot
    __device__ static __forceinline__ typename C::Frag frag(const char *lds0, const char *lds1, int i, int j,
                                                            int tid) {
        using PL = PartialLayout<C>;
        u32x4 c[PL::CPF];
#pragma unroll
        for (int s = 0; s < PL::CPF; ++s) {
            const int u = (i * C::FN + j) * PL::CPF + s - (i / ROWS_PH) * VPH;
            c[s] = *(const u32x4 *)((u < H ? lds0 : lds1) + (u % H) * RB + tid * 16);
        }
        if constexpr (PL::PER == 4) {
            const f32x8 lo = __builtin_shufflevector(__builtin_bit_cast(f32x4, c[0]), __builtin_bit_cast(f32x4, c[1]),
                                                     0, 1, 2, 3, 4, 5, 6, 7);
            const f32x8 hi = __builtin_shufflevector(__builtin_bit_cast(f32x4, c[2]), __builtin_bit_cast(f32x4, c[3]),
                                                     0, 1, 2, 3, 4, 5, 6, 7);
            return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15);
        } else {
            return __builtin_shufflevector(__builtin_bit_cast(f64x2, c[0]), __builtin_bit_cast(f64x2, c[1]), 0, 1, 2,
                                           3);
        }
    }
};

// acc + the peers' partial fragments (i, j), ascending slot order; the first
// peer's fragment comes from the LDS staging.  The accumulator copy is made
// opaque where it is used, so the copies of all fragments are not hoisted
// to the start of the epilogue (which exhausts the VGPRs).
template <class C>
__device__ __forceinline__ typename C::Frag fix_frag(const typename C::Frag &a, const char *slots, int p0, int p1,
                                                     const char *lds0, const char *lds1, int i, int j, int tid) {
    if constexpr (!C::FIX_LDS) {
        return add_peers<C>(a, slots, p0, p1, i, j, tid);
    } else {
        typename C::Frag v = a;
        asm volatile("" : "+v"(v));
        if (p0 <= p1) {
            v = v + FixStage<C>::frag(lds0, lds1, i, j, tid);
            v = add_peers<C>(v, slots, p0 + 1, p1, i, j, tid);
        }
        return v;
    }
}

// Phase boundary of the staged fixup: stage the phase's chunks of the first
// peer (after this wave's reads of the previous phase) and wait for them.
template <class C>
__device__ __forceinline__ void fix_phase(bool staged, const char *slots, int p0, char *lds0, char *lds1, int i,
                                          int tid) {
    if (C::FIX_LDS && staged && i % FixStage<C>::ROWS_PH == 0) {
        if (i > 0) asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        FixStage<C>::issue(slots + (int64_t)p0 * C::SLOT_BYTES, lds0, lds1, i / FixStage<C>::ROWS_PH, tid);
        wait_dma();
    }
}

// Epilogue of a tile with no partial sums to add (32x32 blocks, C rows
// 16-byte aligned): the fragments pass through the idle MAC-loop LDS buffers
// so that C is written in whole rows.  Straight from the MFMA layout a store
// instruction covers 32 rows with 32 bytes each (16 with a 16-bit C), one
// write request per row; after the transpose a wave's instruction covers
// 1 KiB of consecutive bytes (512 with a 16-bit C), a few whole 128-byte
// lines, which makes small-k GEMMs (output-write bound) several times
// cheaper.  The arithmetic per element is that of store_tile_t: alpha * acc,
// then + beta * C, rounded once.  One band of 2 x 32 rows (32 rows per wave
// row) per fragment row i; each padded LDS row (BN floats + 16 bytes) starts
// 4 banks after the previous one, so the 32 rows of a fragment write land in
// distinct banks.  Rows and columns past the edge of C are not stored.
template <class C, int CT>
__device__ __forceinline__ void store_tile_rows(const Problem &P, int tm, int tn,
                                                const typename C::Frag (&acc)[C::FM][C::FN], int tid, char *lds0,
                                                char *lds1, bool interior) {
    using Acc = typename C::Acc;
    constexpr int EB = CBytes<CT>::v;
    constexpr int G = C::FRAG_N / 4;                  // column groups per fragment
    constexpr int RS = C::BN * 4 + 16;                // padded LDS row
    constexpr int Q = C::BN / 4;                      // 16-byte chunks per row
    constexpr int NCH = C::WGM * C::MT * Q / C::THREADS;   // chunks per thread per band
    static_assert(C::MT == 32 && C::WGM == 2 && C::MT * RS <= C::STAGE, "a band's half fits one k-tile buffer");
    static_assert((C::WGM * C::MT * Q) % C::THREADS == 0, "whole chunks per thread");
    const int lane = tid & 63, wave = tid >> 6, wm = wave / C::WGN, wn = wave % C::WGN;
    char *const half = wm == 0 ? lds0 : lds1;
    const int wr = (lane % C::MT) * RS + (wn * C::WTN + 4 * (lane / C::MT)) * 4;
    const Acc alpha = (Acc)P.alpha, beta = (Acc)P.beta;
    const bool rd = P.beta != 0.0;
    static_for<C::FM>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        __syncthreads();                              // LDS free: MAC-loop reads, previous band
#pragma unroll
        for (int j = 0; j < C::FN; ++j) {
            // an opaque copy where it is used, as in fix_frag: the copies of
            // all fragments are not hoisted out of the accumulator registers
            typename C::Frag f = acc[i][j];
            asm volatile("" : "+v"(f));
#pragma unroll
            for (int g = 0; g < G; ++g) {
                f32x4 v;
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = alpha * f[4 * g + e];
                *(f32x4 *)(half + wr + (j * C::MT + 8 * g) * 4) = v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NCH; ++u) {
            const int c = tid + u * C::THREADS;
            const int br = c / Q, c4 = c % Q;         // band row, chunk in the row
            const f32x4 v = *(const f32x4 *)((br < C::MT ? lds0 : lds1) + (br % C::MT) * RS + c4 * 16);
            const int row = tm * C::BM + (br / C::MT) * C::WTM + i * C::MT + br % C::MT;
            const int col = tn * C::BN + 4 * c4;
            const Acc a[4] = {v[0], v[1], v[2], v[3]};
            char *const q = (char *)P.C + ((int64_t)row * P.ldc + col) * EB;
            if (interior || (row < P.m && col + 4 <= P.n)) {
                put4<CT, Acc>(q, a, beta, rd);
            } else if (row < P.m) {
                // the last chunk of a row that ends inside it
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (col + e < P.n) {
                        Acc w = a[e];
                        if (rd) w = w + beta * load_c<CT, Acc>(q + e * EB);
                        put_c<CT, Acc>(q + e * EB, w);
                    }
                }
            }
        }
    });
    __syncthreads();                                  // LDS free for the next unit's loads
}

// C_tile = alpha * (acc + partials of slots [p0, p1]) + beta * C_tile (C read
// only when beta != 0), rounded once to the output type.  The accumulators
// are only read here: each fragment is copied, completed with the peers'
// partial sums and stored, one fragment at a time.  Interior tiles of a C
// whose rows are 16-byte aligned use 4-wide vector accesses; edge tiles test
// every element.
template <class C, int CT>
__device__ __forceinline__ void store_tile_t(const Problem &P, int tm, int tn,
                                             const typename C::Frag (&acc)[C::FM][C::FN], int tid,
                                             const char *slots, int p0, int p1, char *lds0, char *lds1) {
    using Acc = typename C::Acc;
    constexpr int EB = CBytes<CT>::v;
    constexpr int G = C::FRAG_N / 4;                 // column groups per fragment
    const int lane = tid & 63, wave = tid >> 6, wm = wave / C::WGN, wn = wave % C::WGN;
    const Acc alpha = (Acc)P.alpha, beta = (Acc)P.beta;
    const bool rd = P.beta != 0.0;
    const bool interior = (tm + 1) * C::BM <= P.m && (tn + 1) * C::BN <= P.n;
    const bool fast = P.c_vec && interior;
    if constexpr (C::MT == 16) {
        // f64: one element per store; a lane group of 16 writes 128
        // consecutive bytes of one row
        const int r0 = tm * C::BM + wm * C::WTM + (lane >> 4);
        const int c0 = tn * C::BN + wn * C::WTN + (lane & 15);
        const bool staged = p0 <= p1;
        static_for<C::FM * C::FN>([&](auto ij) {
            constexpr int i = decltype(ij)::value / C::FN, j = decltype(ij)::value % C::FN;
            if constexpr (j == 0) fix_phase<C>(staged, slots, p0, lds0, lds1, i, tid);
            const typename C::Frag v = fix_frag<C>(acc[i][j], slots, p0, p1, lds0, lds1, i, j, tid);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + i * 16 + 4 * r, col = c0 + j * 16;
                if (interior || (row < P.m && col < P.n)) {
                    char *q = (char *)P.C + ((int64_t)row * P.ldc + col) * EB;
                    Acc w = alpha * v[r];
                    if (rd) w = w + beta * load_c<CT, Acc>(q);
                    put_c<CT, Acc>(q, w);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        });
        return;
    }
    // (16-bit inputs only, from the 128x128 tile on: the staging's registers
    // would cost the 64x64 Stream-K kernel a wave per SIMD, and with it the
    // FP8 kernels' MAC loops measured 3 % slower at large k)
    if constexpr (C::MT == 32 && C::BM >= 128 && C::DT != Dt::F8) {
        if (P.c_vec && p0 > p1) {
            // whole rows through the LDS, edge tiles included (the flags are
            // uniform over the workgroup)
            store_tile_rows<C, CT>(P, tm, tn, acc, tid, lds0, lds1, interior);
            return;
        }
    }
    const int rowl = tm * C::BM + wm * C::WTM + (lane % C::MT);
    const int coll = tn * C::BN + wn * C::WTN + 4 * (lane / C::MT);
    const bool staged = p0 <= p1;
    static_for<C::FM * C::FN>([&](auto ij) {
        constexpr int i = decltype(ij)::value / C::FN, j = decltype(ij)::value % C::FN;
        if constexpr (j == 0) fix_phase<C>(staged, slots, p0, lds0, lds1, i, tid);
        const int row = rowl + i * C::MT;
        char *rp = (char *)P.C + ((int64_t)row * P.ldc + coll) * EB;
        {
            const typename C::Frag f = fix_frag<C>(acc[i][j], slots, p0, p1, lds0, lds1, i, j, tid);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int co = j * C::MT + 8 * g;         // column offset from coll
                Acc v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = alpha * f[4 * g + e];
                if (fast) {
                    put4<CT, Acc>(rp + co * EB, v, beta, rd);
                } else if (row < P.m) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (coll + co + e < P.n) {
                            char *q = rp + (co + e) * EB;
                            Acc w = v[e];
                            if (rd) w = w + beta * load_c<CT, Acc>(q);
                            put_c<CT, Acc>(q, w);
                        }
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    });
}

template <class C>
__device__ __forceinline__ void store_tile(const Problem &P, int tm, int tn,
                                           const typename C::Frag (&acc)[C::FM][C::FN], int tid,
                                           const char *slots, int p0, int p1, char *lds0, char *lds1) {
    if constexpr (C::DT == Dt::F64) {
        store_tile_t<C, SK_F64>(P, tm, tn, acc, tid, slots, p0, p1, lds0, lds1);
    } else {
        switch (P.c_type) {
        case SK_F32: store_tile_t<C, SK_F32>(P, tm, tn, acc, tid, slots, p0, p1, lds0, lds1); break;
        case SK_F16: store_tile_t<C, SK_F16>(P, tm, tn, acc, tid, slots, p0, p1, lds0, lds1); break;
        default: store_tile_t<C, SK_BF16>(P, tm, tn, acc, tid, slots, p0, p1, lds0, lds1); break;
        }
    }
    // the staged fixup used this wave's LDS regions: keep the next unit's
    // loads out until every wave is done with them
    if (C::FIX_LDS && p0 <= p1) __syncthreads();
}

template <class C>
__device__ __forceinline__ void store_partial(char *slot, const typename C::Frag (&acc)[C::FM][C::FN], int tid) {
    using PL = PartialLayout<C>;
    const __amdgpu_buffer_rsrc_t rs = slot_rsrc(slot, C::SLOT_BYTES);
    static_for<C::FM * C::FN>([&](auto ij) {
        constexpr int i = decltype(ij)::value / C::FN, j = decltype(ij)::value % C::FN;
        {
#pragma unroll
            for (int s = 0; s < PL::CPF; ++s) {
                u32x4 w;
                if constexpr (PL::PER == 4) {
                    w[0] = f2u(acc[i][j][4 * s + 0]);
                    w[1] = f2u(acc[i][j][4 * s + 1]);
                    w[2] = f2u(acc[i][j][4 * s + 2]);
                    w[3] = f2u(acc[i][j][4 * s + 3]);
                } else {
                    const uint64_t x0 = d2u(acc[i][j][2 * s + 0]);
                    const uint64_t x1 = d2u(acc[i][j][2 * s + 1]);
                    w[0] = (uint32_t)x0; w[1] = (uint32_t)(x0 >> 32);
                    w[2] = (uint32_t)x1; w[3] = (uint32_t)(x1 >> 32);
                }
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, w), rs, (uint32_t)PL::off(i, j, s, tid),
                                                       0, CPOL_DEVICE);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    });
}

// ---------------------------------------------------------------------------
// flags.  Partial tiles and flags are all device-coherent accesses (SC1):
// the producer waits until its partial stores have completed, then one
// thread raises the flag by storing the call's epoch; a waiter polls the
// flags it needs (one lane per flag) and issues its partial loads only after
// it has seen all of them.  Program order plus completion waits order the
// accesses; no cache-wide fence is needed.  A flag is never cleared: a value
// other than this call's epoch (an earlier call's, or zero) means "not yet".
// ---------------------------------------------------------------------------
__device__ __forceinline__ void signal_flag(int32_t *flag, int32_t epoch, int tid) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's partial stores are done
    __syncthreads();
    if (tid == 0) __hip_atomic_store(flag, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until the flags of contributors first..last other than `self` (at
// most MAX_PEERS of them, one per lane of wave 0) all hold `epoch`.
// Contributor c's flag is flags[c], except that contributor `first` uses
// flags[first_flag].  The other waves wait at the barrier.  Bounded in real
// time: once `ticks` of the constant-rate counter have passed (at once if
// ticks <= 0) the error word is set and the wait ends; the partial tiles of a
// contributor that has not arrived are then stale and the call reports
// SK_ERR_TIMEOUT.
__device__ __forceinline__ void wait_flags(const int32_t *flags, int first, int last, int self, int first_flag,
                                           int32_t epoch, int32_t *err, int64_t ticks, int tid) {
    if (tid < 64) {
        const int c = first + tid + (first + tid >= self && self >= first ? 1 : 0);
        const bool mine = c <= last;
        const int fi = c == first ? first_flag : c;
        const int32_t *f = flags + (int64_t)(mine ? fi : first_flag) * FLAG_STRIDE;
        bool seen = !mine;
        const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
        if (ticks > 0) {
            while (true) {
                if (!seen) seen = __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch;
                if (__all(seen)) break;
                if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > ticks) {
                    seen = false;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        // bounded: give up, report, never hang
        if (!__all(seen) && tid == 0) __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the workgroup barrier (with its compiler-level ordering) keeps every
    // wave's partial loads behind the observed flags
    __syncthreads();
}

__device__ __forceinline__ void trace_rec(const Params &p, int wg, int seq, int tile, int k0, int k1,
                                          int role, int last, int extra, int tid) {
    if (p.trace != nullptr && tid == 0) {
        int idx = __hip_atomic_fetch_add(p.trace, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (idx < p.trace_cap) {
            int32_t *rec = p.trace + 8 + (int64_t)idx * 8;
            rec[0] = wg; rec[1] = seq; rec[2] = tile; rec[3] = k0;
            rec[4] = k1; rec[5] = role; rec[6] = last; rec[7] = extra;
        }
    }
}

// ---------------------------------------------------------------------------
// Distributed fixup: every contributor of a split tile stores its partial
// tile, and contributor f + i of the s = l - f + 1 contributors f..l reduces
// chunks [i N / s, (i + 1) N / s) of the tile's N 16-byte partial chunks over
// all s partials, in ascending workgroup order -- the same additions, in the
// same order, as the owner's serial fixup, so both give identical bits --
// then applies alpha / beta and writes those elements of C.  The slices of a
// pass are staged into the (idle) MAC-loop LDS buffers with LDS-DMA loads,
// all contributors' chunks at once, so the reads of one slice take one
// memory round trip instead of one per contributor.
// ---------------------------------------------------------------------------
template <class C>
struct Spread {
    static constexpr int N = C::SLOT_BYTES / 16;                 // chunks per tile
    static constexpr int LDS_CHUNKS = C::NSTAGE * C::STAGE / 16;  // staging capacity
    static constexpr int BLK_PER_BUF = C::STAGE / 1024;           // 1 KiB DMA blocks per buffer
    static_assert(C::STAGE % 1024 == 0, "whole DMA blocks per buffer");

    __device__ static __forceinline__ char *blk(LdsBufs b, int i) {
        const int u = i / BLK_PER_BUF, o = (i % BLK_PER_BUF) * 1024;
        return (u == 0 ? b.b0 : u == 1 ? b.b1 : b.b2) + o;
    }

    // Elements of chunk c (16 bytes of the thread-fragment order) of tile
    // (tm, tn): alpha * v (+ beta * C), rounded once, masked at the edges.
    template <int CT>
    __device__ static __forceinline__ void put_chunk(const Problem &P, int tm, int tn, int c, const u32x4 &raw) {
        using Acc = typename C::Acc;
        using PL = PartialLayout<C>;
        constexpr int EB = CBytes<CT>::v;
        const int t = c % C::THREADS, vi = c / C::THREADS;
        const int sc = vi % PL::CPF, fij = vi / PL::CPF, fi = fij / C::FN, fj = fij % C::FN;
        const int lane = t & 63, wave = t >> 6, wm = wave / C::WGN, wn = wave % C::WGN;
        const Acc alpha = (Acc)P.alpha, beta = (Acc)P.beta;
        const bool rd = P.beta != 0.0;
        if constexpr (C::MT == 16) {
            // FP64: the chunk holds rows 4(2 sc) + lane/16 and 4(2 sc + 1) + lane/16 of one column
            const f64x2 v = __builtin_bit_cast(f64x2, raw);
            const int col = tn * C::BN + wn * C::WTN + fj * 16 + (lane & 15);
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int row = tm * C::BM + wm * C::WTM + fi * 16 + 4 * (2 * sc + e) + (lane >> 4);
                if (row < P.m && col < P.n) {
                    char *q = (char *)P.C + ((int64_t)row * P.ldc + col) * EB;
                    Acc w = alpha * v[e];
                    if (rd) w = w + beta * load_c<CT, Acc>(q);
                    put_c<CT, Acc>(q, w);
                }
            }
        } else {
            // 32x32 blocks: four consecutive columns of one row
            const f32x4 v = __builtin_bit_cast(f32x4, raw);
            const int row = tm * C::BM + wm * C::WTM + fi * C::MT + (lane % C::MT);
            const int col = tn * C::BN + wn * C::WTN + fj * C::MT + 8 * sc + 4 * (lane / C::MT);
            char *rp = (char *)P.C + ((int64_t)row * P.ldc + col) * EB;
            Acc a[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) a[e] = alpha * v[e];
            const bool interior = (tm + 1) * C::BM <= P.m && (tn + 1) * C::BN <= P.n;
            if (P.c_vec && interior) {
                put4<CT, Acc>(rp, a, beta, rd);
            } else if (row < P.m) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (col + e < P.n) {
                        char *q = rp + e * EB;
                        Acc w = a[e];
                        if (rd) w = w + beta * load_c<CT, Acc>(q);
                        put_c<CT, Acc>(q, w);
                    }
                }
            }
        }
    }

    // Element e of chunk c (16 bytes of the thread-fragment order) of tile
    // (tm, tn): alpha * v (+ beta * C), rounded once, masked at the edges.
    template <int CT>
    __device__ static __forceinline__ void put_elem(const Problem &P, int tm, int tn, int c, int e,
                                                    typename C::Acc v) {
        using Acc = typename C::Acc;
        using PL = PartialLayout<C>;
        constexpr int EB = CBytes<CT>::v;
        const int t = c % C::THREADS, vi = c / C::THREADS;
        const int sc = vi % PL::CPF, fij = vi / PL::CPF, fi = fij / C::FN, fj = fij % C::FN;
        const int lane = t & 63, wave = t >> 6, wm = wave / C::WGN, wn = wave % C::WGN;
        int row, col;
        if constexpr (C::MT == 16) {
            // FP64: the chunk holds rows 4(2 sc) + lane/16 and 4(2 sc + 1) + lane/16 of one column
            row = tm * C::BM + wm * C::WTM + fi * 16 + 4 * (2 * sc + e) + (lane >> 4);
            col = tn * C::BN + wn * C::WTN + fj * 16 + (lane & 15);
        } else {
            // 32x32 blocks: four consecutive columns of one row
            row = tm * C::BM + wm * C::WTM + fi * C::MT + (lane % C::MT);
            col = tn * C::BN + wn * C::WTN + fj * C::MT + 8 * sc + 4 * (lane / C::MT) + e;
        }
        if (row < P.m && col < P.n) {
            char *q = (char *)P.C + ((int64_t)row * P.ldc + col) * EB;
            Acc w = (Acc)P.alpha * v;
            if (P.beta != 0.0) w = w + (Acc)P.beta * load_c<CT, Acc>(q);
            put_c<CT, Acc>(q, w);
        }
    }

    template <int CT>
    __device__ static __forceinline__ void reduce_t(const Params &p, const Problem &P, int tm, int tn, int f,
                                                    int l, int x, LdsBufs bufs, int tid) {
        const int s = l - f + 1, i = x - f;
        const int c0 = (int)((int64_t)N * i / s), c1 = (int)((int64_t)N * (i + 1) / s);
        // chunks per pass: all s contributors' copies of them fit the LDS
        const int pc = LDS_CHUNKS / s;
        const uint32_t region = (uint32_t)(2 * p.g) * (uint32_t)C::SLOT_BYTES;
        const __amdgpu_buffer_rsrc_t rs = slot_rsrc((const char *)p.partials, (int)region);
        const int w = __builtin_amdgcn_readfirstlane(tid >> 6), L = tid & 63;
        for (int cp = c0; cp < c1; cp += pc) {
            const int n = c1 - cp < pc ? c1 - cp : pc;         // chunks this pass
            const int nblk = (s * pc + 63) / 64;              // 1 KiB staging blocks
            __syncthreads();                                   // LDS free (MAC loop / previous pass)
            for (int b = w; b < nblk; b += C::NW) {
                const int k = b * 64 + L;                      // staging index: contributor k / pc, chunk k % pc
                const int cc = k / pc, j = k % pc;
                const int slot = cc == 0 ? p.g + f : f + cc;   // the owner's is its last-segment slot
                const bool ok = cc < s && j < n;
                const uint32_t off = ok ? (uint32_t)slot * (uint32_t)C::SLOT_BYTES + (uint32_t)(cp + j) * 16u
                                        : 0x80000000u;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)blk(bufs, b),
                                                         16, off, 0, 0, CPOL_DEVICE);
            }
            wait_dma();
            __syncthreads();
            using Acc = typename C::Acc;
            constexpr int EPC = 16 / (int)sizeof(Acc);
            if (n >= C::THREADS) {
                // enough chunks for every thread: one 16-byte chunk per
                // thread, vector reads and stores
                for (int j = tid; j < n; j += C::THREADS) {
                    u32x4 raw;
                    if constexpr (sizeof(Acc) == 4) {
                        f32x4 v = *(const f32x4 *)(blk(bufs, j / 64) + (j % 64) * 16);
                        for (int cc = 1; cc < s; ++cc) {
                            const int k = cc * pc + j;
                            v = v + *(const f32x4 *)(blk(bufs, k / 64) + (k % 64) * 16);
                        }
                        raw = __builtin_bit_cast(u32x4, v);
                    } else {
                        f64x2 v = *(const f64x2 *)(blk(bufs, j / 64) + (j % 64) * 16);
                        for (int cc = 1; cc < s; ++cc) {
                            const int k = cc * pc + j;
                            v = v + *(const f64x2 *)(blk(bufs, k / 64) + (k % 64) * 16);
                        }
                        raw = __builtin_bit_cast(u32x4, v);
                    }
                    put_chunk<CT>(P, tm, tn, cp + j, raw);
                }
                continue;
            }
            // a short slice over many contributors: one element per thread
            // (the order of additions is per element, so the elements of a
            // chunk need not share a thread), the contributors' values read
            // eight at a time ahead of their additions, which stay in
            // ascending order
            for (int u = tid; u < n * EPC; u += C::THREADS) {
                const int j = u / EPC, e = u % EPC;
                auto at = [&](int cc) -> Acc {
                    const int k = cc * pc + j;
                    return *(const Acc *)(blk(bufs, k / 64) + (k % 64) * 16 + e * (int)sizeof(Acc));
                };
                Acc v = at(0);
                int cc = 1;
                for (; cc + 8 <= s; cc += 8) {
                    Acc t[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) t[i] = at(cc + i);
#pragma unroll
                    for (int i = 0; i < 8; ++i) v = v + t[i];
                }
                for (; cc < s; ++cc) v = v + at(cc);
                put_elem<CT>(P, tm, tn, cp + j, e, v);
            }
        }
        __syncthreads();                                       // LDS free for the next user
    }

    __device__ static __forceinline__ void reduce(const Params &p, const Problem &P, int tm, int tn, int f, int l,
                                                  int x, LdsBufs bufs, int tid) {
        if constexpr (C::DT == Dt::F64) {
            reduce_t<SK_F64>(p, P, tm, tn, f, l, x, bufs, tid);
        } else {
            switch (P.c_type) {
            case SK_F32: reduce_t<SK_F32>(p, P, tm, tn, f, l, x, bufs, tid); break;
            case SK_F16: reduce_t<SK_F16>(p, P, tm, tn, f, l, x, bufs, tid); break;
            default: reduce_t<SK_BF16>(p, P, tm, tn, f, l, x, bufs, tid); break;
            }
        }
    }
};

// ---------------------------------------------------------------------------
// tile lookup
// ---------------------------------------------------------------------------

// Output coordinates of a problem's tile t.  The iteration space is linearised
// tile by tile (m->n->k, section 4); the tile-to-coordinate map is a banded
// raster: bands of `band` tile rows, each walked column by column, so that a
// run of consecutive tiles covers a compact block of C and shares A and B
// panels in cache.  band == 1 is the plain row-major order.
__device__ __forceinline__ void tile_coords(const Problem &P, int t, int band, int &tm, int &tn) {
    if (band <= 1) {
        tm = t / P.tiles_n;
        tn = t % P.tiles_n;
        return;
    }
    const int per = band * P.tiles_n;
    const int m0 = (t / per) * band, r = t % per;
    const int rows = P.tiles_m - m0 < band ? P.tiles_m - m0 : band;
    tm = m0 + r % rows;
    tn = r / rows;
}

// Every field of a unit's problem is the same in all lanes; reading it through
// readfirstlane states that, so buffer resources and loop bounds derived from
// it live in scalar registers (a resource the compiler must assume divergent
// costs a readfirstlane loop around every buffer load).
__device__ __forceinline__ Problem uniform_problem(const Problem &src) {
    static_assert(sizeof(Problem) % 4 == 0, "word copy");
    uint32_t w[sizeof(Problem) / 4];
    __builtin_memcpy(w, &src, sizeof(Problem));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(Problem) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    Problem out;
    __builtin_memcpy(&out, w, sizeof(Problem));
    return out;
}
__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

struct TileRef {
    const Problem *P;
    int tile_local;     // tile index within its problem
    int it_begin;       // global iteration of the tile's first MAC iteration
};

template <bool GROUPED>
__device__ __forceinline__ TileRef tile_of_tile(const Params &p, int tile) {
    if constexpr (!GROUPED) {
        return TileRef{&p.prob, tile, tile * p.prob.iters};
    } else {
        const int32_t *tp = p.group.tile_prefix;
        int lo = 0, hi = p.group.count;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (tp[mid] <= tile) lo = mid; else hi = mid;
        }
        const Problem *P = p.group.probs + lo;
        int local = tile - tp[lo];
        return TileRef{P, local, p.group.iter_prefix[lo] + local * P->iters};
    }
}

template <bool GROUPED>
__device__ __forceinline__ int tile_of_iter(const Params &p, int it) {
    if constexpr (!GROUPED) {
        return it / p.prob.iters;
    } else {
        const int32_t *ip = p.group.iter_prefix;
        int lo = 0, hi = p.group.count;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (ip[mid] <= it) lo = mid; else hi = mid;
        }
        return p.group.tile_prefix[lo] + (it - ip[lo]) / p.group.probs[lo].iters;
    }
}

// Data-parallel tiles of a persistent launch after its first wave (tiles
// [0, g) go to workgroups 0..g-1): the tiles [g, dp_tiles) form eight
// contiguous chunks, one per XCD, each taken in order through its own
// counter, so the workgroups of one XCD keep neighbouring tiles (shared A
// and B panels) in flight as a one-workgroup-per-tile launch does, while a
// workgroup that drew short tiles simply takes more of them.  A workgroup
// whose chunk is used up moves on to the next XCDs' chunks.  Thread 0 takes
// a ticket as a tile starts (take) and resolves it after the tile's
// epilogue (resolve), so the atomic's latency hides under the MAC loop.
struct DpQueue {
    // qs: workgroup-shared {chunk tickets are taken from, chunks given up as
    // used up (8: none left)} -- shared memory, so the state costs the
    // persistent loop no registers; ticket: that of the running tile
    __device__ __forceinline__ static int take(const Params &p, const int *qs) {
        return __hip_atomic_fetch_add(p.hdr + HDR_NEXT + qs[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // index into [0, dp_tiles - g) of the next tile, or dp_tiles - g
    __device__ __forceinline__ static int resolve(const Params &p, int *qs, int ticket) {
        const int D = p.dp_tiles - p.g;
        while (qs[1] < XCDS) {
            const int c = qs[0];
            const int lo = (int)((int64_t)D * c / XCDS), hi = (int)((int64_t)D * (c + 1) / XCDS);
            if (ticket < hi - lo) return lo + ticket;
            qs[0] = (c + 1) % XCDS;
            if (++qs[1] < XCDS) ticket = take(p, qs);
        }
        return D;
    }
};

// ---------------------------------------------------------------------------
// the kernel body
// ---------------------------------------------------------------------------
// One workgroup's work is a sequence of units: whole data-parallel tiles
// (j = x, then x+g, x+2g, ... or the per-XCD queues' tiles) and the
// segments of its Stream-K range, in the phase
// order the plan asks for.  Keeping a single MAC-loop / fixup / epilogue site
// keeps the code (and its register allocation) in one piece.
//
// Fixup of a tile split over workgroups f..l (f owns the tile's k = 0):
//  serial (Algorithm 5): f..l-1's successors f+1..l store their partial tiles
//    and raise their flags; f waits for them and adds them to its own
//    accumulators in ascending order inside its epilogue;
//  spread: every contributor stores its partial tile and raises its flag as
//    its segment ends; after its last unit, each contributor waits for the
//    tile's other contributors and reduces its slice (Spread).  Only the
//    first and the last segment of a range can belong to a split tile, so a
//    workgroup has at most two slices to reduce; its partial tiles live in
//    slots x (first segment) and g + x (last segment).
template <class C, bool DP_ONLY>
__device__ __forceinline__ void sk_body(const Params &p) {
    // the k-tile buffers of the MAC loop
    __shared__ __attribute__((aligned(16))) char lds0[C::STAGE];
    __shared__ __attribute__((aligned(16))) char lds1[C::STAGE];
    __shared__ __attribute__((aligned(16))) char lds2[C::NSTAGE >= 3 ? C::STAGE : 16];
    __shared__ __attribute__((aligned(16))) char lds3[C::NSTAGE >= 4 ? C::STAGE : 16];
    __shared__ int next_dp;     // the next queued data-parallel tile, for all waves
    __shared__ int dp_queue[2]; // DpQueue state (thread 0 only)
    const LdsBufs bufs{lds0, lds1, lds2, lds3};
    const int tid0 = threadIdx.x;
    const int b = blockIdx.x;
    int x = b;
    if (p.xcd_remap) {
        // hardware dispatches workgroup b to XCD b % 8; give each XCD a
        // contiguous run of logical ids so Stream-K neighbours share an L2
        const int q8 = p.g >> 3, r8 = p.g & 7, j = b & 7;
        x = j * q8 + (j < r8 ? j : r8) + (b >> 3);
    }
    // this call's flag value: the generation word is only advanced after
    // every workgroup of the launch has finished, so all read the same value
    int32_t epoch = 0;
    if constexpr (!DP_ONLY) {
        const uint32_t gen = (uint32_t)__hip_atomic_load(p.hdr + HDR_GEN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        epoch = uniform_int((int)((gen & 0x3fffffffu) + 1u));
    }
    const bool spread = !DP_ONLY && p.fixup == FIXUP_SPREAD;
    // Stream-K range of this workgroup: [beg, end) within the SK region
    // (fixed split, Algorithm 4: workgroup x runs piece x mod s of tile
    // x / s, iterations [y ips, min(I, (y+1) ips)) with ips = ceil(I / s) --
    // again one contiguous range of the region, so everything below holds)
    const int fs = DP_ONLY ? 0 : p.split;
    int q = 0, r = 0, beg = 0, end = 0, rq = 0, fI = 1, ips = 1;
    if (!DP_ONLY && p.sk_iters > 0) {
        if (fs > 0) {
            // (a hybrid's region of fewer than g / s tiles leaves the
            // workgroups past s tiles without Stream-K work)
            fI = p.prob.iters;
            ips = (fI + fs - 1) / fs;
            const int tl = x / fs, y = x % fs;
            if (tl < p.sk_iters / fI) {
                beg = tl * fI + (y * ips < fI ? y * ips : fI);
                end = tl * fI + ((y + 1) * ips < fI ? (y + 1) * ips : fI);
            } else {
                beg = end = p.sk_iters;
            }
        } else {
            q = p.sk_iters / p.g;
            r = p.sk_iters % p.g;
            beg = x * q + (x < r ? x : r);
            end = beg + q + (x < r ? 1 : 0);
            rq = r * (q + 1);
        }
    }
    // the workgroup holding region-relative iteration i
    auto owner_of = [&](int i) {
        if (fs > 0) return (i / fI) * fs + (i % fI) / ips;
        return i < rq ? i / (q + 1) : r + (i - rq) / q;
    };
    // slices still to reduce (spread fixup): tile, first and last contributor
    int red_tile[2] = {-1, -1}, red_f[2] = {0, 0}, red_l[2] = {0, 0};
    int it = beg;          // next SK iteration
    int j = x;             // next DP tile index
    int phase = 0;         // 0, 1: the two phases; 2: done
    int seq = 0;
    const bool dp_first = DP_ONLY || p.dp_first;
    // data-parallel tiles after the first from the per-XCD queues (DpQueue):
    // thread 0 hands the next one to the workgroup after each epilogue
    const bool dyn = !DP_ONLY && p.dyn_dp;
    int ticket = 0;
    if (dyn && tid0 == 0) {
        dp_queue[0] = b % XCDS;
        dp_queue[1] = 0;
    }
    while (true) {
        const bool dp_now = (phase == 0) == dp_first;
        int tile, k0, k1;
        bool started = true, ended = true;
        if (phase >= 2) break;
        if (dp_now) {
            if (j >= p.dp_tiles) { ++phase; continue; }
            tile = j < p.sk_tile_begin ? j : j - p.sk_tile_begin + p.sk_tile_end;
            if (dyn) {
                if (tid0 == 0) ticket = DpQueue::take(p, dp_queue);
            } else {
                j += p.g;
            }
        } else {
            if (DP_ONLY || it >= end) { ++phase; continue; }
            tile = tile_of_iter<C::GROUPED>(p, p.sk_iter_begin + it);
        }
        const TileRef tr = tile_of_tile<C::GROUPED>(p, tile);
        const Problem P = uniform_problem(*tr.P);
        int t0 = 0, t1 = 0;
        if (dp_now) {
            k0 = 0;
            k1 = P.iters;
        } else {
            t0 = uniform_int(tr.it_begin) - p.sk_iter_begin;   // region-relative tile start
            t1 = t0 + P.iters;
            k0 = it - t0;
            k1 = (end < t1 ? end : t1) - t0;
            started = it == t0;
            ended = end >= t1;
            it = t1;
        }
        int tm, tn;
        tile_coords(P, uniform_int(tr.tile_local), p.band, tm, tn);
        // an opaque copy of the thread index: per-thread addresses are
        // recomputed for every unit instead of being hoisted out of this loop
        // and kept live (spilled) across the whole kernel
        int tid = tid0;
        asm volatile("" : "+v"(tid));
        typename C::Frag acc[C::FM][C::FN];
        mac_loop<C>(P, tm, tn, k0, k1, acc, bufs, tid);
        const int last = ended ? -1 : owner_of(t1 - 1);
        if (!started) {
            // the first segment of this range: partial slot and flag x
            store_partial<C>((char *)p.partials + (int64_t)x * C::SLOT_BYTES, acc, tid);
            signal_flag(p.flags + x * FLAG_STRIDE, epoch, tid);
            trace_rec(p, x, seq++, tile, k0, k1, ROLE_PRODUCER, -1, 0, tid);
            if (spread) {
                red_tile[0] = tile;
                red_f[0] = owner_of(t0);
                red_l[0] = ended ? x : last;
            }
            continue;
        }
        if (!ended && spread) {
            // the last segment of this range owns the tile: partial slot and
            // flag g + x (resp. MAX_GRID + x)
            store_partial<C>((char *)p.partials + (int64_t)(p.g + x) * C::SLOT_BYTES, acc, tid);
            signal_flag(p.flags + (MAX_GRID + x) * FLAG_STRIDE, epoch, tid);
            trace_rec(p, x, seq++, tile, k0, k1, ROLE_OWNER, last, 0, tid);
            red_tile[1] = tile;
            red_f[1] = x;
            red_l[1] = last;
            continue;
        }
        if (!ended) wait_flags(p.flags, x + 1, last, -1, x + 1, epoch, p.err, p.wait_ticks, tid);
        // peers' partial tiles are added in ascending slot order inside the
        // epilogue, fragment by fragment
        store_tile<C>(P, tm, tn, acc, tid, (const char *)p.partials, x + 1, last, lds0, lds1);
        trace_rec(p, x, seq++, tile, k0, k1, dp_now ? ROLE_DP : (ended ? ROLE_FULL : ROLE_OWNER), last, 0,
                  tid);
        if (dp_now && dyn) {
            if (tid0 == 0) next_dp = DpQueue::resolve(p, dp_queue, ticket);
            __syncthreads();
            j = p.g + next_dp;
            __syncthreads();
        }
    }
    if constexpr (!DP_ONLY) {
        if (spread) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (red_tile[u] < 0) continue;
                const int f = red_f[u], l = red_l[u];
                wait_flags(p.flags, f, l, x, MAX_GRID + f, epoch, p.err, p.wait_ticks, tid0);
                const TileRef tr = tile_of_tile<C::GROUPED>(p, red_tile[u]);
                const Problem P = uniform_problem(*tr.P);
                int tm, tn;
                tile_coords(P, uniform_int(tr.tile_local), p.band, tm, tn);
                const int s = l - f + 1, i = x - f;
                trace_rec(p, x, seq++, red_tile[u], (int)((int64_t)Spread<C>::N * i / s),
                          (int)((int64_t)Spread<C>::N * (i + 1) / s), ROLE_REDUCE, l, f, tid0);
                Spread<C>::reduce(p, P, tm, tn, f, l, x, bufs, tid0);
            }
        }
        // the last workgroup to finish advances the generation (next epoch)
        __syncthreads();
        if (tid0 == 0) {
            const int done = __hip_atomic_fetch_add(p.hdr + HDR_DONE, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (done == p.g - 1) {
                __hip_atomic_store(p.hdr + HDR_DONE, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (int c = 0; c < XCDS; ++c)
                    __hip_atomic_store(p.hdr + HDR_NEXT + c, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(p.hdr + HDR_GEN, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

template <class C>
__global__ __launch_bounds__(C::THREADS) void sk_kernel(Params p) {
    sk_body<C, false>(p);
}

template <class C>
__global__ __launch_bounds__(C::THREADS) void dp_kernel(Params p) {
    sk_body<C, true>(p);
}

template <class C>
int launch_sk(const Params &p, int grid, void *stream) {
    hipLaunchKernelGGL(sk_kernel<C>, dim3(grid), dim3(C::THREADS), 0, (hipStream_t)stream, p);
    return (int)hipGetLastError();
}

template <class C>
int launch_dp(const Params &p, int grid, void *stream) {
    hipLaunchKernelGGL(dp_kernel<C>, dim3(grid), dim3(C::THREADS), 0, (hipStream_t)stream, p);
    return (int)hipGetLastError();
}

template <class C>
int occupancy_sk(int *blocks) {
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sk_kernel<C>, C::THREADS, 0);
}

}  // namespace sk
