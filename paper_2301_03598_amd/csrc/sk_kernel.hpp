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

#include "sk_internal.h"

namespace sk {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Bit casts go through by-value helpers: applied directly to an element of
// an ext_vector_type lvalue, __builtin_bit_cast reads element 0 of the vector.
__device__ __forceinline__ uint32_t f2u(float f) { return __builtin_bit_cast(uint32_t, f); }
__device__ __forceinline__ float u2f(uint32_t u) { return __builtin_bit_cast(float, u); }
__device__ __forceinline__ uint64_t d2u(double d) { return __builtin_bit_cast(uint64_t, d); }
__device__ __forceinline__ double u2d(uint64_t u) { return __builtin_bit_cast(double, u); }

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

template <Dt D, int BM_, int BN_, bool AKC_, bool BKC_, bool GROUPED_>
struct Cfg {
    static constexpr Dt DT = D;
    static constexpr bool AKC = AKC_, BKC = BKC_, GROUPED = GROUPED_;
    static constexpr int E = DtTraits<D>::E;
    static constexpr int VEC = 16 / E;          // elements per 16-byte load
    static constexpr int BK = 8 * VEC;          // an LDS row = 8 chunks = 128 B
    static constexpr int BM = BM_, BN = BN_;
    static constexpr int WTM = BM / 2, WTN = BN / 2;   // 2 x 2 waves
    static constexpr int MT = DtTraits<D>::MT;
    static constexpr int FM = WTM / MT, FN = WTN / MT;
    static constexpr int FRAG_N = DtTraits<D>::FRAG_N;
    static constexpr int A_BYTES = BM * 128, B_BYTES = BN * 128;
    static constexpr int STAGE = A_BYTES + B_BYTES;
    static constexpr int LDS = 2 * STAGE;
    using Acc = typename DtTraits<D>::Acc;
    using Frag = typename DtTraits<D>::Frag;
    static constexpr int ACC_N = FM * FN * FRAG_N;     // accumulators per thread
    static constexpr int ACC_CHUNKS = ACC_N * (int)sizeof(Acc) / 16;
    static constexpr int SLOT_BYTES = BM * BN * (int)sizeof(Acc);
    static_assert(BM * BN == THREADS * ACC_N, "accumulator split");
};

// LDS byte offset of 16-byte chunk c of row r (128-byte rows, XOR swizzle).
__device__ __forceinline__ uint32_t lds_off(uint32_t row, uint32_t chunk) {
    return row * 128u + (((chunk ^ row) & 7u) << 4);
}

// ---------------------------------------------------------------------------
// global -> register -> LDS staging of one operand tile (ROWS x BK)
//
// The operand is seen as a ROWS x k matrix X with element (r, p) at
// KC ? r*ld + p : p*ld + r.  Every thread issues ROWS/32 16-byte loads per
// k-tile whichever way X is stored.
// ---------------------------------------------------------------------------
template <class C, int ROWS, bool KC>
struct Stage {
    static constexpr int NL = ROWS / 32;            // loads per thread
    static constexpr int E = C::E, VEC = C::VEC, BK = C::BK;
    // contiguous-along-mn layout: a thread loads L k-rows of VEC elements
    static constexpr int L = NL;
    static constexpr int KB = BK / L;               // k-blocks (threads) per mn block
    static constexpr int PIECE = L * E;             // bytes per mn-row piece

    const char *base;      // thread's first load address at k-tile 0
    int64_t kstep;         // bytes per k-tile
    int64_t lstride;       // bytes between this thread's consecutive loads
    int rows_valid;        // number of valid leading loads (row edge), KC only
    bool mn_valid;         // !KC: this thread's mn block lies inside the matrix
    int kofs;              // k offset (elements) of this thread's first load within a k-tile
    uint32_t lds0;         // LDS offset of the first store (KC) / row base (!KC)
    u32x4 r[NL];

    __device__ __forceinline__ void init(const void *ptr, int64_t ld, int row0, int rows_total,
                                         int tid) {
        const char *p = (const char *)ptr;
        if constexpr (KC) {
            int rr = tid >> 3, c = tid & 7;
            base = p + ((int64_t)(row0 + rr) * ld + c * VEC) * E;
            kstep = (int64_t)BK * E;
            lstride = (int64_t)32 * ld * E;
            int rem = rows_total - row0 - rr;           // rows left for this thread
            rows_valid = rem <= 0 ? 0 : (rem + 31) / 32;
            kofs = c * VEC;
            lds0 = lds_off(rr, c);
        } else {
            int kb = tid % KB, mb = tid / KB;
            base = p + ((int64_t)(kb * L) * ld + row0 + mb * VEC) * E;
            kstep = (int64_t)BK * ld * E;
            lstride = (int64_t)ld * E;
            mn_valid = row0 + mb * VEC < rows_total;
            kofs = kb * L;
            lds0 = (uint32_t)(mb * VEC);                // first row of the block
        }
    }

    // Issue the loads of k-tile kt.  Out-of-range data are zero.
    __device__ __forceinline__ void load(int kt, int K, bool interior) {
        const char *p = base + kt * kstep;
        if constexpr (KC) {
            if (interior) {
#pragma unroll
                for (int i = 0; i < NL; ++i) r[i] = *(const u32x4 *)(p + i * lstride);
            } else {
                bool kv = kt * BK + kofs < K;
#pragma unroll
                for (int i = 0; i < NL; ++i) {
                    if (kv && i < rows_valid) r[i] = *(const u32x4 *)(p + i * lstride);
                    else r[i] = u32x4{0u, 0u, 0u, 0u};
                }
            }
        } else {
            if (interior) {
#pragma unroll
                for (int j = 0; j < NL; ++j) r[j] = *(const u32x4 *)(p + j * lstride);
            } else {
                int k0 = kt * BK + kofs;
#pragma unroll
                for (int j = 0; j < NL; ++j) {
                    if (mn_valid && k0 + j < K) r[j] = *(const u32x4 *)(p + j * lstride);
                    else r[j] = u32x4{0u, 0u, 0u, 0u};
                }
            }
        }
    }

    // element e (0..VEC-1) of loaded vector j, as raw bits in the low E bytes
    __device__ __forceinline__ uint32_t elem_bits(int j, int e) const {
        if constexpr (E == 2) return (r[j][e >> 1] >> ((e & 1) * 16)) & 0xffffu;
        else return (r[j][e >> 2] >> ((e & 3) * 8)) & 0xffu;
    }

    __device__ __forceinline__ void store(char *lds) const {
        if constexpr (KC) {
#pragma unroll
            for (int i = 0; i < NL; ++i) *(u32x4 *)(lds + lds0 + i * 32 * 128) = r[i];
        } else {
            const int kb_byte = kofs * E;               // byte offset of the piece in a row
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const uint32_t row = lds0 + e;
                if constexpr (E == 8) {
                    // f64: element e of each load is one double (two words)
#pragma unroll
                    for (int s = 0; s < PIECE / 16; ++s) {
                        u32x4 w;
                        w[0] = r[2 * s][2 * e];
                        w[1] = r[2 * s][2 * e + 1];
                        w[2] = r[2 * s + 1][2 * e];
                        w[3] = r[2 * s + 1][2 * e + 1];
                        *(u32x4 *)(lds + lds_off(row, (kb_byte >> 4) + s)) = w;
                    }
                } else {
                    constexpr int NW = PIECE / 4;       // words in the piece
                    constexpr int PER = 4 / E;          // elements per word
                    uint32_t w[NW];
#pragma unroll
                    for (int q = 0; q < NW; ++q) {
                        uint32_t v = 0;
#pragma unroll
                        for (int b = 0; b < PER; ++b) v |= elem_bits(q * PER + b, e) << (b * 8 * E);
                        w[q] = v;
                    }
                    char *dst = lds + lds_off(row, kb_byte >> 4) + (kb_byte & 15);
                    if constexpr (NW == 4) *(u32x4 *)dst = u32x4{w[0], w[1], w[2], w[3]};
                    else if constexpr (NW == 2) *(u32x2 *)dst = u32x2{w[0], w[1]};
                    else *(uint32_t *)dst = w[0];
                }
            }
        }
    }
};

// ---------------------------------------------------------------------------
// MFMA on one k-tile held in LDS
// ---------------------------------------------------------------------------
template <class C>
__device__ __forceinline__ void mma_ktile(typename C::Frag (&acc)[C::FM][C::FN], const char *ldsA,
                                          const char *ldsB, int lane, int wm, int wn) {
    if constexpr (C::DT == Dt::F64) {
        // v_mfma_f64_16x16x4: lane group q = lane/16 supplies one k value per
        // MFMA.  One 16-byte chunk read gives a lane two consecutive k values,
        // consumed by two MFMAs (group q covers k = 2q, 2q+1 of each 8-k
        // half of the chunk row); A and B use the same assignment.
        const int r16 = lane & 15, q = lane >> 4;
        const uint32_t arow = (uint32_t)(wm * C::WTM + r16), brow = (uint32_t)(wn * C::WTN + r16);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = h * 4 + q;
            double a0[C::FM], a1[C::FM], b0[C::FN], b1[C::FN];
#pragma unroll
            for (int i = 0; i < C::FM; ++i) {
                const double *pa = (const double *)(ldsA + lds_off(arow + i * 16, c));
                a0[i] = pa[0];
                a1[i] = pa[1];
            }
#pragma unroll
            for (int j = 0; j < C::FN; ++j) {
                const double *pb = (const double *)(ldsB + lds_off(brow + j * 16, c));
                b0[j] = pb[0];
                b1[j] = pb[1];
            }
#pragma unroll
            for (int i = 0; i < C::FM; ++i)
#pragma unroll
                for (int j = 0; j < C::FN; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[i], b0[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[i], b1[j], acc[i][j], 0, 0, 0);
                }
        }
    } else {
        // 32x32 MFMAs: lane group q = lane/32 supplies a contiguous run of k
        // (8 for f16/bf16: one chunk; 32 for f8: two chunks).
        constexpr int CPM = (C::DT == Dt::F8) ? 2 : 1;    // chunks per lane per MFMA
        constexpr int NSUB = 8 / (2 * CPM);                // MFMAs along k per k-tile
        const int r32 = lane & 31, q = lane >> 5;
        const uint32_t arow = (uint32_t)(wm * C::WTM + r32), brow = (uint32_t)(wn * C::WTN + r32);
#pragma unroll
        for (int ks = 0; ks < NSUB; ++ks) {
            u32x4 a[C::FM][CPM], b[C::FN][CPM];
#pragma unroll
            for (int s = 0; s < CPM; ++s) {
                const int c = ks * 2 * CPM + q * CPM + s;
#pragma unroll
                for (int i = 0; i < C::FM; ++i) a[i][s] = *(const u32x4 *)(ldsA + lds_off(arow + i * 32, c));
#pragma unroll
                for (int j = 0; j < C::FN; ++j) b[j][s] = *(const u32x4 *)(ldsB + lds_off(brow + j * 32, c));
            }
#pragma unroll
            for (int i = 0; i < C::FM; ++i)
#pragma unroll
                for (int j = 0; j < C::FN; ++j) {
                    if constexpr (C::DT == Dt::BF16) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, b[j][0]), __builtin_bit_cast(bf16x8, a[i][0]),
                            acc[i][j], 0, 0, 0);
                    } else if constexpr (C::DT == Dt::F16) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                            __builtin_bit_cast(f16x8, b[j][0]), __builtin_bit_cast(f16x8, a[i][0]),
                            acc[i][j], 0, 0, 0);
                    } else {
                        i32x8 av, bv;
                        av[0] = a[i][0][0]; av[1] = a[i][0][1]; av[2] = a[i][0][2]; av[3] = a[i][0][3];
                        av[4] = a[i][1][0]; av[5] = a[i][1][1]; av[6] = a[i][1][2]; av[7] = a[i][1][3];
                        bv[0] = b[j][0][0]; bv[1] = b[j][0][1]; bv[2] = b[j][0][2]; bv[3] = b[j][0][3];
                        bv[4] = b[j][1][0]; bv[5] = b[j][1][1]; bv[6] = b[j][1][2]; bv[7] = b[j][1][3];
                        // formats 0/0 = FP8 e4m3 for both operands; E8M0 scales of
                        // 2^0 (127): the per-tensor FP32 scales go into alpha
                        acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                            bv, av, acc[i][j], 0, 0, 0, 127, 0, 127);
                    }
                }
        }
    }
}

// ---------------------------------------------------------------------------
// The MAC loop over iterations [it0, it1) of one tile (Algorithm 3)
// ---------------------------------------------------------------------------
template <class C>
struct Ctx {
    Stage<C, C::BM, C::AKC> sa;
    Stage<C, C::BN, C::BKC> sb;
};

template <class C>
__device__ __forceinline__ void mac_loop(const Problem &P, int tm, int tn, int it0, int it1,
                                         typename C::Frag (&acc)[C::FM][C::FN], char *lds, int tid) {
#pragma unroll
    for (int i = 0; i < C::FM; ++i)
#pragma unroll
        for (int j = 0; j < C::FN; ++j) acc[i][j] = typename C::Frag{};
    if (it0 >= it1) return;
    const int lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
    const int row0 = tm * C::BM, col0 = tn * C::BN;
    Ctx<C> cx;
    cx.sa.init(P.A, P.lda, row0, P.m, tid);
    cx.sb.init(P.B, P.ldb, col0, P.n, tid);
    const bool rows_in = (row0 + C::BM <= P.m) && (col0 + C::BN <= P.n);
    const int kfull = P.k / C::BK;                 // k-tiles with no k edge
    {
        const bool in = rows_in && it0 < kfull;
        cx.sa.load(it0, P.k, in);
        cx.sb.load(it0, P.k, in);
        cx.sa.store(lds);
        cx.sb.store(lds + C::A_BYTES);
    }
    __syncthreads();
    for (int it = it0; it < it1; ++it) {
        const int cur = (it - it0) & 1;
        const bool more = it + 1 < it1;
        if (more) {
            const bool in = rows_in && it + 1 < kfull;
            cx.sa.load(it + 1, P.k, in);
            cx.sb.load(it + 1, P.k, in);
        }
        char *st = lds + cur * C::STAGE;
        mma_ktile<C>(acc, st, st + C::A_BYTES, lane, wm, wn);
        if (more) {
            char *nx = lds + (cur ^ 1) * C::STAGE;
            cx.sa.store(nx);
            cx.sb.store(nx + C::A_BYTES);
        }
        __syncthreads();
    }
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

// C_tile = alpha * acc + beta * C_tile (C read only when beta != 0), then
// rounded once to the output type.  Interior tiles of a C whose rows are
// 16-byte aligned use 4-wide vector accesses; edge tiles test every element.
template <class C, int CT>
__device__ __forceinline__ void store_tile_t(const Problem &P, int tm, int tn,
                                             typename C::Frag (&acc)[C::FM][C::FN], int tid) {
    using Acc = typename C::Acc;
    constexpr int EB = CBytes<CT>::v;
    constexpr int G = C::FRAG_N / 4;                 // column groups per fragment
    const int lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
    const int rowl = tm * C::BM + wm * C::WTM + (lane % C::MT);
    const int coll = tn * C::BN + wn * C::WTN + 4 * (lane / C::MT);
    const Acc alpha = (Acc)P.alpha, beta = (Acc)P.beta;
    const bool rd = P.beta != 0.0;
    const bool interior = (tm + 1) * C::BM <= P.m && (tn + 1) * C::BN <= P.n;
    const bool fast = P.c_vec && interior;
    if constexpr (C::MT == 16) {
        // f64: one element per store; a lane group of 16 writes 128
        // consecutive bytes of one row
        const int r0 = tm * C::BM + wm * C::WTM + (lane >> 4);
        const int c0 = tn * C::BN + wn * C::WTN + (lane & 15);
#pragma unroll
        for (int i = 0; i < C::FM; ++i) {
#pragma unroll
            for (int j = 0; j < C::FN; ++j) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = r0 + i * 16 + 4 * r, col = c0 + j * 16;
                    if (interior || (row < P.m && col < P.n)) {
                        char *q = (char *)P.C + ((int64_t)row * P.ldc + col) * EB;
                        Acc w = alpha * acc[i][j][r];
                        if (rd) w = w + beta * load_c<CT, Acc>(q);
                        put_c<CT, Acc>(q, w);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < C::FM; ++i) {
        const int row = rowl + i * C::MT;
        char *rp = (char *)P.C + ((int64_t)row * P.ldc + coll) * EB;
#pragma unroll
        for (int j = 0; j < C::FN; ++j) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int co = j * C::MT + 8 * g;         // column offset from coll
                Acc v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = alpha * acc[i][j][4 * g + e];
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
    }
}

template <class C>
__device__ __forceinline__ void store_tile(const Problem &P, int tm, int tn,
                                           typename C::Frag (&acc)[C::FM][C::FN], int tid) {
    if constexpr (C::DT == Dt::F64) {
        store_tile_t<C, SK_F64>(P, tm, tn, acc, tid);
    } else {
        switch (P.c_type) {
        case SK_F32: store_tile_t<C, SK_F32>(P, tm, tn, acc, tid); break;
        case SK_F16: store_tile_t<C, SK_F16>(P, tm, tn, acc, tid); break;
        default: store_tile_t<C, SK_BF16>(P, tm, tn, acc, tid); break;
        }
    }
}

// Partial tiles: thread-fragment order, 16-byte chunk v of thread t at
// slot + (v*THREADS + t)*16, so stores and loads are fully coalesced.
template <class C>
__device__ __forceinline__ void store_partial(char *slot, typename C::Frag (&acc)[C::FM][C::FN], int tid) {
    constexpr int PER = 16 / (int)sizeof(typename C::Acc);   // accumulators per chunk
    constexpr int CPF = C::FRAG_N / PER;                      // chunks per fragment
#pragma unroll
    for (int i = 0; i < C::FM; ++i)
#pragma unroll
        for (int j = 0; j < C::FN; ++j)
#pragma unroll
            for (int s = 0; s < CPF; ++s) {
                const int v = (i * C::FN + j) * CPF + s;
                u32x4 w;
                if constexpr (PER == 4) {
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
                *(u32x4 *)(slot + ((int64_t)v * THREADS + tid) * 16) = w;
                if (s == CPF - 1) __builtin_amdgcn_sched_barrier(0);
            }
}

template <class C>
__device__ __forceinline__ void add_partial(const char *slot, typename C::Frag (&acc)[C::FM][C::FN], int tid) {
    constexpr int PER = 16 / (int)sizeof(typename C::Acc);
    constexpr int CPF = C::FRAG_N / PER;
#pragma unroll
    for (int i = 0; i < C::FM; ++i)
#pragma unroll
        for (int j = 0; j < C::FN; ++j)
#pragma unroll
            for (int s = 0; s < CPF; ++s) {
                const int v = (i * C::FN + j) * CPF + s;
                const u32x4 w = *(const u32x4 *)(slot + ((int64_t)v * THREADS + tid) * 16);
                if constexpr (PER == 4) {
                    acc[i][j][4 * s + 0] += u2f(w[0]);
                    acc[i][j][4 * s + 1] += u2f(w[1]);
                    acc[i][j][4 * s + 2] += u2f(w[2]);
                    acc[i][j][4 * s + 3] += u2f(w[3]);
                } else {
                    acc[i][j][2 * s + 0] += u2d((uint64_t)w[0] | ((uint64_t)w[1] << 32));
                    acc[i][j][2 * s + 1] += u2d((uint64_t)w[2] | ((uint64_t)w[3] << 32));
                }
                if (s == CPF - 1) __builtin_amdgcn_sched_barrier(0);
            }
}

// ---------------------------------------------------------------------------
// flags: release after the partial stores, acquire before reading them
// ---------------------------------------------------------------------------
__device__ __forceinline__ void signal_flag(int32_t *flag, int tid) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // this thread's partial stores
    __syncthreads();
    if (tid == 0) __hip_atomic_store(flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void wait_flag(int32_t *flag, int32_t *err, int limit, int tid) {
    if (tid == 0) {
        int n = 0;
        while (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            __builtin_amdgcn_s_sleep(1);
            if (++n >= limit) {             // bounded: give up, report, never hang
                __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __hip_atomic_store(flag, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);   // consumed
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ void trace_rec(const Params &p, int wg, int seq, int tile, int k0, int k1,
                                          int role, int last, int tid) {
    if (p.trace != nullptr && tid == 0) {
        int idx = __hip_atomic_fetch_add(p.trace, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (idx < p.trace_cap) {
            int32_t *rec = p.trace + 8 + (int64_t)idx * 8;
            rec[0] = wg; rec[1] = seq; rec[2] = tile; rec[3] = k0;
            rec[4] = k1; rec[5] = role; rec[6] = last; rec[7] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// tile lookup
// ---------------------------------------------------------------------------
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

// ---------------------------------------------------------------------------
// the kernel body
// ---------------------------------------------------------------------------
// One workgroup's work is a sequence of units: whole data-parallel tiles
// (j = x, x+g, ...) and the segments of its Stream-K range, in the phase
// order the plan asks for.  Keeping a single MAC-loop / fixup / epilogue site
// keeps the code (and its register allocation) in one piece.
template <class C, bool DP_ONLY>
__device__ __forceinline__ void sk_body(const Params &p) {
    __shared__ __attribute__((aligned(16))) char lds[C::LDS];
    const int tid0 = threadIdx.x;
    const int b = blockIdx.x;
    int x = b;
    if (!DP_ONLY && p.xcd_remap) {
        // hardware dispatches workgroup b to XCD b % 8; give each XCD a
        // contiguous run of logical ids so Stream-K neighbours share an L2
        const int q8 = p.g >> 3, r8 = p.g & 7, j = b & 7;
        x = j * q8 + (j < r8 ? j : r8) + (b >> 3);
    }
    // Stream-K range of this workgroup: [beg, end) within the SK region
    int q = 0, r = 0, beg = 0, end = 0, rq = 0;
    if (!DP_ONLY && p.sk_iters > 0) {
        q = p.sk_iters / p.g;
        r = p.sk_iters % p.g;
        beg = x * q + (x < r ? x : r);
        end = beg + q + (x < r ? 1 : 0);
        rq = r * (q + 1);
    }
    int it = beg;          // next SK iteration
    int j = x;             // next DP tile index
    int phase = 0;         // 0, 1: the two phases; 2: done
    int seq = 0;
    const bool dp_first = DP_ONLY || p.dp_first;
    while (true) {
        const bool dp_now = (phase == 0) == dp_first;
        int tile, k0, k1;
        bool started = true, ended = true;
        if (phase >= 2) break;
        if (dp_now) {
            if (j >= p.dp_tiles) { ++phase; continue; }
            tile = j < p.sk_tile_begin ? j : j - p.sk_tile_begin + p.sk_tile_end;
            j += p.g;
        } else {
            if (DP_ONLY || it >= end) { ++phase; continue; }
            tile = tile_of_iter<C::GROUPED>(p, p.sk_iter_begin + it);
        }
        const TileRef tr = tile_of_tile<C::GROUPED>(p, tile);
        int t1 = 0;
        if (dp_now) {
            k0 = 0;
            k1 = tr.P->iters;
        } else {
            const int t0 = tr.it_begin - p.sk_iter_begin;   // region-relative tile start
            t1 = t0 + tr.P->iters;
            k0 = it - t0;
            k1 = (end < t1 ? end : t1) - t0;
            started = it == t0;
            ended = end >= t1;
            it = t1;
        }
        const int tm = tr.tile_local / tr.P->tiles_n, tn = tr.tile_local % tr.P->tiles_n;
        // an opaque copy of the thread index: per-thread addresses are
        // recomputed for every unit instead of being hoisted out of this loop
        // and kept live (spilled) across the whole kernel
        int tid = tid0;
        asm volatile("" : "+v"(tid));
        typename C::Frag acc[C::FM][C::FN];
        mac_loop<C>(*tr.P, tm, tn, k0, k1, acc, lds, tid);
        if (!started) {
            store_partial<C>((char *)p.partials + (int64_t)x * C::SLOT_BYTES, acc, tid);
            signal_flag(p.flags + x * FLAG_STRIDE, tid);
            trace_rec(p, x, seq++, tile, k0, k1, ROLE_PRODUCER, -1, tid);
            continue;
        }
        int last = -1;
        if (!ended) {
            const int li = t1 - 1;
            last = li < rq ? li / (q + 1) : r + (li - rq) / q;
            for (int peer = x + 1; peer <= last; ++peer) {
                wait_flag(p.flags + peer * FLAG_STRIDE, p.err, p.spin_limit, tid);
                add_partial<C>((const char *)p.partials + (int64_t)peer * C::SLOT_BYTES, acc, tid);
            }
        }
        store_tile<C>(*tr.P, tm, tn, acc, tid);
        trace_rec(p, x, seq++, tile, k0, k1, dp_now ? ROLE_DP : (ended ? ROLE_FULL : ROLE_OWNER),
                  last, tid);
    }
}

template <class C>
__global__ __launch_bounds__(THREADS) void sk_kernel(Params p) {
    sk_body<C, false>(p);
}

template <class C>
__global__ __launch_bounds__(THREADS) void dp_kernel(Params p) {
    sk_body<C, true>(p);
}

template <class C>
int launch_sk(const Params &p, int grid, void *stream) {
    hipLaunchKernelGGL(sk_kernel<C>, dim3(grid), dim3(THREADS), 0, (hipStream_t)stream, p);
    return (int)hipGetLastError();
}

template <class C>
int launch_dp(const Params &p, int grid, void *stream) {
    hipLaunchKernelGGL(dp_kernel<C>, dim3(grid), dim3(THREADS), 0, (hipStream_t)stream, p);
    return (int)hipGetLastError();
}

template <class C>
int occupancy_sk(int *blocks) {
    return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sk_kernel<C>, THREADS, 0);
}

}  // namespace sk
