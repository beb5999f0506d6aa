// Symmetric-product kernel of the recursive Fermi-operator expansion.
//
// The hot loop of every recursion in the paper (Sec. II.B, Eq. (1) and
// Eq. (2)) multiplies two commuting symmetric matrices, so the product is
// symmetric and only its upper-triangular tiles are computed (N^2 (N+1)
// flops instead of 2 N^3); each off-diagonal tile is stored twice (mirror).
// The epilogue fuses the projection step, C = alpha*AB + beta*E + gamma*I
// with (alpha, beta, gamma) chosen on the device from the SP2 branch flag
// (X^2 or 2X - X^2), and the FP64 partial sums the next decision needs:
// Tr C, ||C||_F^2 (= Tr C^2 for symmetric C, Sec. III.B) and ||AB - E||_F^2
// (the idempotency error of X when AB = X^2 and E = X).
//
// CDNA4 mapping:
//  * 256 threads = 4 wave64s in a 2 x 2 arrangement; a block owns a BT x BT
//    (BT = 32, 64 or 128)
//    output tile, each wave a (BT/2)^2 sub-tile of 16 x 16 MFMA blocks.
//  * Both operands are read as row panels of the row-major matrices: rows
//    ti*BT.. of A and rows tj*BT.. of B (B symmetric, so B[k][j] = B[j][k]),
//    whole 128-byte lines along k (one K stage of one row), staged into
//    unpadded LDS rows with the 16-byte chunks XOR-swizzled by the row index
//    (the fragment reads hit every bank equally: 1.5x the read rate of
//    16-byte-padded rows in a probe; the 64-wide FP32 tiles keep the padded
//    rows), double buffered with one barrier per stage and the next stage's
//    loads in flight during the MFMAs.  The split forms and the 128-wide
//    tiles load straight into LDS (global_load_lds_dwordx4: no VGPR round
//    trip, no ds_write); the 64-wide FP64 / FP32 tiles stage through two
//    register sets, two stages ahead.
//  * Every lane reads a 16-byte fragment (row = lane % 16, k-chunk =
//    lane / 16).  The k order inside a fragment is irrelevant because A and
//    B use the same one: FP64 feeds 2 v_mfma_f64_16x16x4 per fragment, FP32
//    4 v_mfma_f32_16x16x4, FP16/BF16 one v_mfma_f32_16x16x32.
//  * Split forms keep an FP32 master matrix (epilogue operand, sums) and
//    16-bit hi/lo companions written once by the producer:
//    hi = round(s*x), lo = round(s*x - hi) (s = 2^12 for FP16, 1 for BF16),
//    interleaved per 32 columns so that one K stage of one row is a single
//    128-byte line; the operand stages copy them straight into LDS and
//    AB ~ (hi hi + hi lo + lo hi) / s^2 with FP32 accumulation.
//  * Workgroups go round-robin over the 8 XCDs; the block index is remapped
//    so each XCD works on a contiguous run of the tile list (shared row
//    panels stay in that XCD's L2).
//  * Working matrices are zero-padded to a multiple of 128, so no bounds
//    checks are needed; partial sums are per tile and reduced in a fixed
//    order by the decide kernel (bitwise reproducible).
#include "fdm_internal.h"

namespace fdm {
namespace {

typedef double d2_t __attribute__((ext_vector_type(2)));
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef __bf16 b4_t __attribute__((ext_vector_type(4)));
typedef __bf16 b8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u2_t __attribute__((ext_vector_type(2)));

template <class To, class From>
__device__ __forceinline__ To bitcast(const From &v) {
    static_assert(sizeof(To) == sizeof(From), "size");
    return __builtin_bit_cast(To, v);
}

template <int P>
struct PT;
template <>
struct PT<P_F64> {
    using S = double;
    using Acc = d4_t;
    static constexpr bool HALF = false, SPLIT = false, F16 = false;
};
template <>
struct PT<P_F32> {
    using S = float;
    using Acc = f4_t;
    static constexpr bool HALF = false, SPLIT = false, F16 = false;
};
template <>
struct PT<P_F16X3> {
    using S = float;
    using Acc = f4_t;
    static constexpr bool HALF = true, SPLIT = true, F16 = true;
};
template <>
struct PT<P_BF16X3> {
    using S = float;
    using Acc = f4_t;
    static constexpr bool HALF = true, SPLIT = true, F16 = false;
};
template <>
struct PT<P_F16> {
    using S = float;
    using Acc = f4_t;
    static constexpr bool HALF = true, SPLIT = false, F16 = true;
};
template <>
struct PT<P_BF16> {
    using S = float;
    using Acc = f4_t;
    static constexpr bool HALF = true, SPLIT = false, F16 = false;
};

// FP16 forms work on 2^12 * x so that small entries stay normal.
constexpr float kF16Scale = 4096.0f;
constexpr double kF16Unscale = 1.0 / (4096.0 * 4096.0);

// Split (or round) four FP32 values into 16-bit halves.
template <int P>
__device__ __forceinline__ void to_halves(const u4_t &raw, u2_t &hi, u2_t &lo) {
    const f4_t x = bitcast<f4_t>(raw);
    if constexpr (PT<P>::F16) {
        h4_t h, l;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float s = x[e] * kF16Scale;
            const _Float16 hh = (_Float16)s;
            h[e] = hh;
            l[e] = (_Float16)(s - (float)hh);
        }
        hi = bitcast<u2_t>(h);
        lo = bitcast<u2_t>(l);
    } else {
        b4_t h, l;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const __bf16 hh = (__bf16)x[e];
            h[e] = hh;
            l[e] = (__bf16)(x[e] - (float)hh);
        }
        hi = bitcast<u2_t>(h);
        lo = bitcast<u2_t>(l);
    }
}

template <int P>
__device__ __forceinline__ void split1(float x, uint16_t &hi, uint16_t &lo) {
    if constexpr (PT<P>::F16) {
        const float s = x * kF16Scale;
        const _Float16 hh = (_Float16)s;
        hi = __builtin_bit_cast(uint16_t, hh);
        lo = __builtin_bit_cast(uint16_t, (_Float16)(s - (float)hh));
    } else {
        const __bf16 hh = (__bf16)x;
        hi = __builtin_bit_cast(uint16_t, hh);
        lo = __builtin_bit_cast(uint16_t, (__bf16)(x - (float)hh));
    }
}

// Index of the hi value of (row, col) in the interleaved companion layout
// (lo is 32 further on).
__device__ __forceinline__ int64_t hl_index(int64_t row, int64_t col, int64_t ld) {
    return row * 2 * ld + (col >> 5) * 64 + (col & 31);
}

// hi/lo companions of an FP32 working matrix (elementwise, whole padded area)
template <int P>
__global__ __launch_bounds__(256) void k_split(const float *__restrict__ x,
                                               uint16_t *__restrict__ hl, int64_t ld,
                                               int64_t count) {
    const int64_t i4 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (i4 >= count) return;
    const u4_t raw = *(const u4_t *)(x + i4);
    u2_t h, l;
    to_halves<P>(raw, h, l);
    const int64_t k = hl_index(i4 / ld, i4 % ld, ld);
    *(u2_t *)(hl + k) = h;
    *(u2_t *)(hl + k + 32) = l;
}

template <int P>
__device__ __forceinline__ typename PT<P>::Acc mfma_frag(const u4_t &a, const u4_t &b,
                                                         const u4_t &alo, const u4_t &blo,
                                                         typename PT<P>::Acc c) {
    if constexpr (P == P_F64) {
        const d2_t x = bitcast<d2_t>(a), y = bitcast<d2_t>(b);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(x[0], y[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(x[1], y[1], c, 0, 0, 0);
    } else if constexpr (P == P_F32) {
        const f4_t x = bitcast<f4_t>(a), y = bitcast<f4_t>(b);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[0], y[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[1], y[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[2], y[2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[3], y[3], c, 0, 0, 0);
    } else if constexpr (PT<P>::F16) {
        const h8_t x = bitcast<h8_t>(a), y = bitcast<h8_t>(b);
        if constexpr (PT<P>::SPLIT) {
            const h8_t xl = bitcast<h8_t>(alo), yl = bitcast<h8_t>(blo);
            c = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, yl, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_f16(xl, y, c, 0, 0, 0);
        }
        c = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c, 0, 0, 0);
    } else {
        const b8_t x = bitcast<b8_t>(a), y = bitcast<b8_t>(b);
        if constexpr (PT<P>::SPLIT) {
            const b8_t xl = bitcast<b8_t>(alo), yl = bitcast<b8_t>(blo);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, yl, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, y, c, 0, 0, 0);
        }
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
    }
    return c;
}

// Workgroups go round-robin over the 8 XCDs: block b runs list entry
// xcd_remap(b), so each XCD walks a contiguous run of the list.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int xcd = b & 7, slot = b >> 3, per = nb >> 3, rem = nb & 7;
    return (xcd < rem) ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

// LDS of the 128-wide split kernels, shared by their two block shapes (one
// allocation per kernel: two blocks of 80 KiB per CU).
constexpr int kEdgePoolBytes = 2 * (256 + 64) * 128;
__device__ __forceinline__ unsigned char *lds_pool() {
    __shared__ __attribute__((aligned(16))) unsigned char pool[kEdgePoolBytes];
    return pool;
}

// One output tile (entry t of a.tiles) of one product.  KIND 0: a BT x BT
// tile with LDS of its own; KIND 1: the same from the shared pool; KIND 2
// (128-wide split forms, direct-to-LDS staging): an edge block of 256 x 64
// outputs, rows 256 q .. and columns 128 tj .. of an entry (1 << 31) |
// (q << 16) | tj, covering the last tile column where the padded extent
// ends 64 columns into it.  Its four waves are stacked (64 x 64 each, the
// same per-wave work and accumulation order as a 128-wide tile); a wave
// whose rows start below the block's columns (lower triangle) stores
// nothing.
template <int P, int BT, bool DMA, int KIND = 0>
__device__ __forceinline__ void symprod_tile(const ProdArgs &a, const int t) {
    using T = PT<P>;
    using S = typename T::S;
    using Acc = typename T::Acc;
    constexpr bool HALF = T::HALF;
    constexpr bool SPLIT = T::SPLIT;
    // LDS rows hold one K stage of one operand row.  FP64 and the split forms
    // (hi chunks 0-3, lo chunks 4-7), and every form staged straight into
    // LDS, keep the 128-byte global line as is, with chunk c of row r at slot
    // c ^ (r & 7): the fragment reads (16 rows x 4 chunks per wave) then hit
    // every bank equally (no bank-conflict stalls in the counters).  The
    // 64-wide FP32 tiles through registers keep rows padded by 16 bytes
    // (1.4% faster there: 596 vs 605 us per product at N = 4000, where their
    // LDS traffic is far from the bound), and the single-pass 16-bit forms
    // round while staging into 64-byte rows padded by 16 bytes.
    constexpr bool SWZ = DMA || SPLIT || P == P_F64;
    constexpr int RSB = SWZ ? 128 : (HALF ? 80 : 144);   // LDS row stride (bytes)
    constexpr int PANEL = BT * RSB;                // bytes of one operand panel
    constexpr int KST = (sizeof(S) == 8) ? 16 : 32;  // k elements per stage (128 B of S)
    constexpr int EPC = 16 / sizeof(S);            // S elements per 16-byte chunk
    constexpr int GROUPS = HALF ? 1 : 2;           // 64-byte fragment groups per stage
    constexpr int NL = BT * 8 / 256;               // 16-byte global chunks per thread per panel
    constexpr int WT = BT / 2;
    constexpr int FM = WT / 16;

    static_assert(!DMA || SWZ, "direct-to-LDS staging needs the swizzled rows");
    static_assert(KIND == 0 || (BT == 128 && DMA), "edge blocks: 128-wide, direct to LDS");
    constexpr bool TALL = (KIND == 2);
    constexpr int AROWS = TALL ? 256 : BT;         // operand rows staged per stage
    constexpr int BROWS = TALL ? 64 : BT;
    constexpr int STAGE = (AROWS + BROWS) * RSB;   // bytes of one LDS stage
    unsigned char *lds;
    if constexpr (KIND == 0) {
        __shared__ __attribute__((aligned(16))) unsigned char own[2 * 2 * PANEL];
        lds = own;
    } else {
        static_assert(2 * STAGE <= kEdgePoolBytes, "pool");
        lds = lds_pool();
    }

    const int tid = threadIdx.x;
    const uint32_t tt = a.tiles[t];
    const int ti = (int)(TALL ? ((tt >> 16) & 0x7fffu) : (tt >> 16)), tj = (int)(tt & 0xffffu);
    const int64_t row0 = (int64_t)ti * (TALL ? 256 : BT), col0 = (int64_t)tj * BT;
    const int64_t ld = a.ld;
    const S *__restrict__ A = (const S *)a.A;
    const S *__restrict__ B = (const S *)a.B;

    // Two register sets of staged operand chunks: with both in use the loads
    // for stage k+2 are issued while stage k is multiplied, so a CU keeps two
    // stages of panel traffic in flight.
    u4_t ga0[NL], gb0[NL], ga1[NL], gb1[NL];
    const uint16_t *__restrict__ Ahl = a.Ahl;
    const uint16_t *__restrict__ Bhl = a.Bhl;
    auto gload = [&](int kt, u4_t (&ga)[NL], u4_t (&gb)[NL]) {
        const int64_t k0 = (int64_t)kt * KST;
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int c = tid + 256 * u;
            const int r = c >> 3, ch = c & 7;
            if constexpr (SPLIT) {
                // one 128-byte line per row stage: 16-byte chunks 0-3 hold the
                // hi halves, 4-7 the lo halves (k0 = 32 kt)
                const int64_t off = (int64_t)kt * 64 + ch * 8;
                ga[u] = *(const u4_t *)(Ahl + (row0 + r) * 2 * ld + off);
                gb[u] = *(const u4_t *)(Bhl + (col0 + r) * 2 * ld + off);
            } else {
                ga[u] = *(const u4_t *)(A + (row0 + r) * ld + k0 + ch * EPC);
                gb[u] = *(const u4_t *)(B + (col0 + r) * ld + k0 + ch * EPC);
            }
        }
    };
    auto lstore = [&](int st, const u4_t (&ga)[NL], const u4_t (&gb)[NL]) {
        unsigned char *pa = lds + (st * 2 + 0) * PANEL;
        unsigned char *pb = lds + (st * 2 + 1) * PANEL;
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int c = tid + 256 * u;
            const int r = c >> 3, ch = c & 7;
            if constexpr (SWZ) {
                const int off = r * RSB + ((ch ^ (r & 7)) << 4);
                *(u4_t *)(pa + off) = ga[u];
                *(u4_t *)(pb + off) = gb[u];
            } else if constexpr (!HALF) {
                *(u4_t *)(pa + r * RSB + ch * 16) = ga[u];
                *(u4_t *)(pb + r * RSB + ch * 16) = gb[u];
            } else {
                // single-pass FP16 / BF16: round the FP32 master while staging
                u2_t h, l;
                to_halves<P>(ga[u], h, l);
                *(u2_t *)(pa + r * RSB + ch * 8) = h;
                to_halves<P>(gb[u], h, l);
                *(u2_t *)(pb + r * RSB + ch * 8) = h;
            }
        }
    };

    const int w = tid >> 6, lane = tid & 63;
    const int wr = TALL ? w : w >> 1, wc = TALL ? 0 : w & 1, lr = lane & 15, lg = lane >> 4;
    // Direct-to-LDS staging (global_load_lds_dwordx4): lane l of a wave
    // instruction writes LDS bytes [16 l, 16 l + 16) of a 1 KiB block, i.e.
    // slot l & 7 of row l >> 3 of an 8-row group, so it fetches chunk
    // (l & 7) ^ (l >> 3) of that row: whole 128-byte lines per 8 lanes, and
    // the same swizzled rows as the register path.
    auto dload = [&](int kt, int st) {
        constexpr int QB = BT / 8;                 // 8-row groups per operand panel
        constexpr int QA = AROWS / 8, NG = (AROWS + BROWS) / 8;   // (edge blocks)
        static_assert(NG % 4 == 0, "groups per wave");
#pragma unroll
        for (int u = 0; u < NG / 4; ++u) {
            const int j = w + 4 * u;               // wave-uniform
            const int op = TALL ? (j >= QA ? 1 : 0) : j / QB;
            const int q = TALL ? (op ? j - QA : j) : j % QB;
            int64_t base = (op ? col0 : row0) + 8 * q;
            // the last edge block of an odd tile count reaches 128 rows past
            // the padded matrix (ld rows): its waves there store nothing,
            // and they stage in-range rows instead
            if (TALL && !op && base >= ld) base -= 128;
            const int64_t row = base + (lane >> 3);
            const int chunk = (lane & 7) ^ (lane >> 3);
            const void *src;
            if constexpr (SPLIT)
                src = (op ? Bhl : Ahl) + row * 2 * ld + (int64_t)kt * 64 + chunk * 8;
            else
                src = (op ? B : A) + row * ld + (int64_t)kt * KST + chunk * EPC;
            __builtin_amdgcn_global_load_lds(
                src,
                (__attribute__((address_space(3))) void *)(
                    TALL ? lds + st * STAGE + op * AROWS * RSB + q * 1024
                         : lds + (st * 2 + op) * PANEL + q * 1024),
                16, 0, 0);
        }
    };

    // FP32-accumulating forms sum a run of K stages in a fresh accumulator
    // and fold it into the running sum: the accumulation error then grows
    // with N / run length instead of N, which lowers the rounding floor of
    // the low-precision SP2 iterates (the operand rounding is what remains).
    //  * FP32: a plain add of each 128-deep partial sum (4 stages).  On
    //    64-wide tiles a Kahan-compensated fold of every 32-deep stage costs
    //    64 VALU ops per lane and stage: 0.597 vs 0.542 ms per product at
    //    N = 4000 for an SP2 floor of 1.11e-5 vs 1.30e-5 (one McWeeny step
    //    either way; 1.9e-4 with no fold at N = 16000).
    //  * Split forms: a plain add of each 256-deep partial sum (8 stages;
    //    their stages carry 4x fewer MFMA cycles).  A Kahan fold every 128
    //    deep on 64-wide tiles gave the same SP2 floor (8.2e-5 at N = 4000,
    //    2.4e-5 at N = 6000) at 0.260 vs 0.241 ms per product; with no fold
    //    the FP16x3 iterate of the paper's N = 32768 matrix never got below
    //    tau.
    //  * Single-pass 16-bit forms: compensated fold of every stage on 64-wide
    //    tiles, direct accumulation on 128-wide ones.
    constexpr bool KAHAN = (P != P_F64 && P != P_F32 && !SPLIT) && BT <= 64;
    constexpr bool TWOLEVEL = (P == P_F32) || SPLIT;
    constexpr bool COMP = KAHAN || TWOLEVEL;
    constexpr int FOLD = SPLIT ? 8 : (TWOLEVEL ? 4 : 1);
    const int nk = a.kext / KST;
    Acc acc[FM][FM], cmp[FM][FM], part[FM][FM];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FM; ++j) {
            acc[i][j] = Acc{0, 0, 0, 0};
            cmp[i][j] = Acc{0, 0, 0, 0};
            part[i][j] = Acc{0, 0, 0, 0};
        }

    auto compute = [&](int st, int kt) {
        const unsigned char *pa = TALL ? lds + st * STAGE : lds + (st * 2 + 0) * PANEL;
        const unsigned char *pb = TALL ? lds + st * STAGE + AROWS * RSB : lds + (st * 2 + 1) * PANEL;
#pragma unroll
        for (int g = 0; g < GROUPS; ++g) {
            u4_t fa[FM], fb[FM], fal[FM], fbl[FM];
            // chunk slots of this lane's fragment (hi, lo for the split forms)
            const int sh = SWZ ? (((g * 4 + lg) ^ (lr & 7)) << 4) : (g * 4 + lg) * 16;
            const int sl = ((4 + lg) ^ (lr & 7)) << 4;
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const int rb = (wr * WT + i * 16 + lr) * RSB;
                fa[i] = *(const u4_t *)(pa + rb + sh);
                if constexpr (SPLIT) fal[i] = *(const u4_t *)(pa + rb + sl);
            }
#pragma unroll
            for (int j = 0; j < FM; ++j) {
                const int rb = (wc * WT + j * 16 + lr) * RSB;
                fb[j] = *(const u4_t *)(pb + rb + sh);
                if constexpr (SPLIT) fbl[j] = *(const u4_t *)(pb + rb + sl);
            }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FM; ++j) {
                    if constexpr (COMP)
                        part[i][j] = mfma_frag<P>(fa[i], fb[j], fal[i], fbl[j], part[i][j]);
                    else
                        acc[i][j] = mfma_frag<P>(fa[i], fb[j], fal[i], fbl[j], acc[i][j]);
                }
        }
        if constexpr (COMP) {
            if ((kt + 1) % FOLD == 0 || kt + 1 == nk) {
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FM; ++j) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            if constexpr (KAHAN) {
                                // Kahan: cmp holds the low-order part lost so far
                                const float y = part[i][j][q] - cmp[i][j][q];
                                const float t = acc[i][j][q] + y;
                                cmp[i][j][q] = (t - acc[i][j][q]) - y;
                                acc[i][j][q] = t;
                            } else {
                                acc[i][j][q] += part[i][j][q];
                            }
                        }
                        part[i][j] = Acc{0, 0, 0, 0};
                    }
            }
        }
    };

    // Stage kt lives in LDS buffer kt & 1; the loop is unrolled by two so
    // buffer and register-set indices are static.  FP64 and FP32 prefetch
    // two stages ahead (register set kt & 1 carries stage kt); the split
    // forms spend those registers on the running fold accumulator (two sets
    // and the fold spill: 570 -> 340 TFLOP/s) and prefetch one stage ahead.
    // kext is a multiple of 64, so nk is even and every trip runs both
    // halves.  The loads are unconditional (stages past the end reload the
    // last one, in bounds and unused): a conditional load makes the
    // compiler's in-order vmcnt accounting wait for the newer set too, which
    // serialises the loads with the MFMAs.
    if constexpr (DMA) {
        // Stage kt+1 streams into the other buffer while stage kt is
        // multiplied.  A direct-to-LDS load counts on vmcnt until its data
        // is in LDS: each wave waits for its own loads, then the barrier
        // makes every wave's part of the stage visible.
        auto stage_done = [&]() {
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), other counters untouched
            __syncthreads();
        };
        dload(0, 0);
        stage_done();
        for (int kt = 0; kt < nk; kt += 2) {
            dload(kt + 1, 1);
            compute(0, kt);
            stage_done();
            if (kt + 2 < nk) dload(kt + 2, 0);
            compute(1, kt + 1);
            stage_done();
        }
    } else if constexpr ((P == P_F32 || P == P_F64) && BT == 64) {
        gload(0, ga0, gb0);
        gload(1, ga1, gb1);
        lstore(0, ga0, gb0);
        __syncthreads();
        for (int kt = 0; kt < nk; kt += 2) {
            gload(kt + 2 < nk ? kt + 2 : nk - 1, ga0, gb0);
            compute(0, kt);
            lstore(1, ga1, gb1);
            __syncthreads();
            gload(kt + 3 < nk ? kt + 3 : nk - 1, ga1, gb1);
            compute(1, kt + 1);
            if (kt + 2 < nk) lstore(0, ga0, gb0);
            __syncthreads();
        }
    } else {
        gload(0, ga0, gb0);
        lstore(0, ga0, gb0);
        __syncthreads();
        for (int kt = 0; kt < nk; kt += 2) {
            gload(kt + 1, ga0, gb0);
            compute(0, kt);
            lstore(1, ga0, gb0);
            __syncthreads();
            gload(kt + 2 < nk ? kt + 2 : nk - 1, ga0, gb0);
            compute(1, kt + 1);
            if (kt + 2 < nk) lstore(0, ga0, gb0);
            __syncthreads();
        }
    }

    // ---- fused epilogue -------------------------------------------------
    // Accumulator lane layout of a 16x16 block (lane l, register q): column
    // l % 16 and row 4*(l/16) + q for the FP32-accumulating MFMAs, row
    // l/16 + 4*q for v_mfma_f64_16x16x4.
    constexpr bool ROWS_CONSECUTIVE = (P != P_F64);
    const int sel = (a.sel != nullptr) ? *a.sel : 0;
    const double alpha = a.coef[sel][0], beta = a.coef[sel][1], gamma = a.coef[sel][2];
    const double scale = (HALF && T::F16) ? kF16Unscale : 1.0;
    const S *__restrict__ E = (const S *)a.E;
    S *__restrict__ C = (S *)a.C;
    // a tall edge block's wave covers rows row0 + 64 wr .. of its column block
    const bool diag = TALL ? (row0 + 64 * wr == col0) : (ti == tj);
    const bool active = !TALL || row0 + 64 * wr <= col0;
    double s_tr = 0.0, s_f2 = 0.0, s_d2 = 0.0;
    if (active) {
#pragma unroll
        for (int i = 0; i < FM; ++i) {
#pragma unroll
            for (int j = 0; j < FM; ++j) {
                const int64_t rb = row0 + wr * WT + i * 16;
                const int64_t col = col0 + wc * WT + j * 16 + lr;
                S ov[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t row = rb + (ROWS_CONSECUTIVE ? 4 * lg + q : lg + 4 * q);
                    const double v = ((double)acc[i][j][q] - (double)cmp[i][j][q]) * scale;
                    const double e = (E != nullptr) ? (double)E[row * ld + col] : 0.0;
                    double o = alpha * v + beta * e;
                    if (row == col && row < a.n) o += gamma;
                    const S os = (S)o;
                    ov[q] = os;
                    // Off-diagonal tiles: every element, stored twice (mirror).
                    // Diagonal tiles: only row <= col is kept and mirrored, so C
                    // is exactly symmetric even where (i,j) and (j,i) were
                    // accumulated in different orders.
                    const double w = diag ? (row < col ? 2.0 : (row == col ? 1.0 : 0.0)) : 2.0;
                    if (w != 0.0) {
                        C[row * ld + col] = os;
                        if (diag && row < col) C[col * ld + row] = os;
                        if constexpr (SPLIT) {
                            uint16_t h, l;
                            split1<P>((float)os, h, l);
                            const int64_t k = hl_index(row, col, ld);
                            a.Chl[k] = h;
                            a.Chl[k + 32] = l;
                            if (diag && row < col) {
                                const int64_t km = hl_index(col, row, ld);
                                a.Chl[km] = h;
                                a.Chl[km + 32] = l;
                            }
                        }
                        const double od = (double)os;
                        if (row == col) s_tr += od;
                        s_f2 += w * od * od;
                        s_d2 += w * (v - e) * (v - e);
                    }
                }
                if (!diag) {
                    if constexpr (ROWS_CONSECUTIVE) {
                        S *dst = C + col * ld + rb + 4 * lg;
                        *(f4_t *)dst = f4_t{(float)ov[0], (float)ov[1], (float)ov[2], (float)ov[3]};
                        if constexpr (SPLIT) {
                            u2_t hi4, lo4;
                            to_halves<P>(bitcast<u4_t>(f4_t{(float)ov[0], (float)ov[1], (float)ov[2],
                                                            (float)ov[3]}),
                                         hi4, lo4);
                            const int64_t m = hl_index(col, rb + 4 * lg, ld);
                            *(u2_t *)(a.Chl + m) = hi4;
                            *(u2_t *)(a.Chl + m + 32) = lo4;
                        }
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) C[col * ld + rb + lg + 4 * q] = ov[q];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        s_tr += __shfl_xor(s_tr, off);
        s_f2 += __shfl_xor(s_f2, off);
        s_d2 += __shfl_xor(s_d2, off);
    }
    double *red = (double *)lds;  // every wave is past the last barrier of the k loop
    if (lane == 0) {
        red[w * 3 + 0] = s_tr;
        red[w * 3 + 1] = s_f2;
        red[w * 3 + 2] = s_d2;
    }
    __syncthreads();
    if (tid == 0) {
        double *p = a.partials + (size_t)t * 4;
        p[0] = (red[0] + red[3]) + (red[6] + red[9]);
        p[1] = (red[1] + red[4]) + (red[7] + red[10]);
        p[2] = (red[2] + red[5]) + (red[8] + red[11]);
        p[3] = 0.0;
    }
}

// 32-wide tiles (small products: more blocks) run up to eight waves per
// SIMD; 64-wide tiles are register-capped to four waves per SIMD (four
// blocks per CU); 128-wide FP64, FP32 and split tiles to two (two blocks per CU: 64 x 64
// outputs per wave, half the panel and LDS fragment traffic per flop of a
// 64-wide tile); the single-pass 16-bit 128-wide tiles run one wave per SIMD.
#define FDM_SYMPROD_ATTRS(P, BT)                                                        \
    __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(                          \
        BT == 32 ? 8 : BT == 64 ? 4 : ((P == P_F32 || P == P_F64 || PT<P>::SPLIT) ? 2 : 1), \
        BT == 32 ? 8 : BT == 64 ? 4 : ((P == P_F32 || P == P_F64 || PT<P>::SPLIT) ? 2 : 1))))

// One list entry: a tile, or for the 128-wide split forms staged straight
// into LDS an edge block (bit 31 of the entry) as well.
template <int P, int BT, bool DMA>
__device__ __forceinline__ void symprod_entry(const ProdArgs &a, const int t) {
    if constexpr (PT<P>::SPLIT && BT == 128 && DMA) {
        if (a.tiles[t] >> 31)
            symprod_tile<P, 128, true, 2>(a, t);
        else
            symprod_tile<P, 128, true, 1>(a, t);
    } else {
        symprod_tile<P, BT, DMA>(a, t);
    }
}

template <int P, int BT, bool DMA>
__global__ FDM_SYMPROD_ATTRS(P, BT) void k_symprod(ProdArgs a) {
    if (a.done != nullptr && *a.done) return;
    symprod_entry<P, BT, DMA>(a, xcd_remap(blockIdx.x, gridDim.x));
}

// Several products of one precision, tile edge and staging path in one
// launch (the serving tick): the grid covers the concatenated tile lists,
// job j owning list entries [first[j], first[j+1]).  Each tile is computed
// exactly as by k_symprod, so a product's result does not depend on what it
// was grouped with.
template <int P, int BT, bool DMA>
__global__ FDM_SYMPROD_ATTRS(P, BT) void k_symprod_grouped(ProdGroup g) {
    const int u = xcd_remap(blockIdx.x, gridDim.x);
    int j = 0;
    while (j + 1 < g.njobs && u >= g.first[j + 1]) ++j;
    const ProdArgs &a = g.job[j];
    if (a.done != nullptr && *a.done) return;
    symprod_entry<P, BT, DMA>(a, u - g.first[j]);
}

// Staging path (measured on MI355X, SP2 solves of the paper's matrix):
//  * split forms, 64-wide tiles: direct to LDS (0.32 -> 0.26 ms per product
//    at N = 4000);
//  * split forms, 128-wide tiles: direct to LDS up to N ~ 18000 (1012 ->
//    1137 TFLOP/s at N = 16384), through registers beyond, where the
//    operands stream from HBM and the register path keeps more loads in
//    flight (1042 vs 924 at N = 20480, 1056 vs 826 at N = 32768);
//  * FP64 / FP32, 128-wide tiles: direct to LDS (FP32 130.0 -> 131.7 at
//    N = 32768);
//  * FP64 / FP32, 64-wide tiles: registers, two stages ahead.
constexpr int64_t kSplitDirectMaxLd = 18432;

template <int P, int BT>
bool direct_t(int64_t ld) {
    if constexpr (PT<P>::SPLIT) return (BT <= 64) || ld <= kSplitDirectMaxLd;
    else if constexpr (P == P_F64 || P == P_F32) return BT != 64;
    return false;
}

template <int P, int BT>
hipError_t launch_t(const ProdArgs &a, hipStream_t s) {
    constexpr bool ok = (P == P_F64 || P == P_F32 || PT<P>::SPLIT);
    if (direct_t<P, BT>(a.ld))
        hipLaunchKernelGGL((k_symprod<P, BT, ok>), dim3(a.ntiles), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_symprod<P, BT, false>), dim3(a.ntiles), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int P>
hipError_t launch_p(int bt, const ProdArgs &a, hipStream_t s) {
    if (bt == 128) return launch_t<P, 128>(a, s);
    if (bt == 32) return launch_t<P, 32>(a, s);
    return launch_t<P, 64>(a, s);
}

template <int P, int BT>
hipError_t launch_grouped_t(bool direct, const ProdGroup &g, int total, hipStream_t s) {
    constexpr bool ok = (P == P_F64 || P == P_F32 || PT<P>::SPLIT);
    if (direct && ok)
        hipLaunchKernelGGL((k_symprod_grouped<P, BT, ok>), dim3(total), dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((k_symprod_grouped<P, BT, false>), dim3(total), dim3(256), 0, s, g);
    return hipGetLastError();
}

template <int P>
hipError_t launch_grouped_p(int bt, bool direct, const ProdGroup &g, int total, hipStream_t s) {
    if (bt == 128) return launch_grouped_t<P, 128>(direct, g, total, s);
    if (bt == 32) return launch_grouped_t<P, 32>(direct, g, total, s);
    return launch_grouped_t<P, 64>(direct, g, total, s);
}

}  // namespace

bool symprod_direct(int prec, int bt, int64_t ld) {
    switch (prec) {
        case P_F64:
            return bt == 128 ? direct_t<P_F64, 128>(ld)
                             : (bt == 32 ? direct_t<P_F64, 32>(ld) : direct_t<P_F64, 64>(ld));
        case P_F32:
            return bt == 128 ? direct_t<P_F32, 128>(ld)
                             : (bt == 32 ? direct_t<P_F32, 32>(ld) : direct_t<P_F32, 64>(ld));
        case P_F16X3:
            return bt == 128 ? direct_t<P_F16X3, 128>(ld)
                             : (bt == 32 ? direct_t<P_F16X3, 32>(ld) : direct_t<P_F16X3, 64>(ld));
        case P_BF16X3:
            return bt == 128 ? direct_t<P_BF16X3, 128>(ld)
                             : (bt == 32 ? direct_t<P_BF16X3, 32>(ld) : direct_t<P_BF16X3, 64>(ld));
        default: return false;
    }
}

hipError_t launch_symprod_grouped(int prec, int bt, bool direct, const ProdGroup &g,
                                  hipStream_t s) {
    if (g.njobs <= 0 || g.njobs > kMaxGroup) return hipErrorInvalidValue;
    const int total = g.first[g.njobs];
    if (total <= 0) return hipSuccess;
    switch (prec) {
        case P_F64: return launch_grouped_p<P_F64>(bt, direct, g, total, s);
        case P_F32: return launch_grouped_p<P_F32>(bt, direct, g, total, s);
        case P_F16X3: return launch_grouped_p<P_F16X3>(bt, direct, g, total, s);
        case P_BF16X3: return launch_grouped_p<P_BF16X3>(bt, direct, g, total, s);
        case P_BF16: return launch_grouped_p<P_BF16>(bt, direct, g, total, s);
        case P_F16: return launch_grouped_p<P_F16>(bt, direct, g, total, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_split(int prec, const float *x, uint16_t *hl, int64_t ld, int64_t rows,
                        hipStream_t s) {
    if (ld % 32 || rows < 0) return hipErrorInvalidValue;
    const int64_t count = ld * rows;
    const int64_t nb = (count / 4 + 255) / 256;
    if (nb == 0) return hipSuccess;
    if (prec == P_F16X3)
        hipLaunchKernelGGL((k_split<P_F16X3>), dim3((unsigned)nb), dim3(256), 0, s, x, hl, ld,
                           count);
    else if (prec == P_BF16X3)
        hipLaunchKernelGGL((k_split<P_BF16X3>), dim3((unsigned)nb), dim3(256), 0, s, x, hl, ld,
                           count);
    else
        return hipSuccess;
    return hipGetLastError();
}

hipError_t launch_symprod(int prec, int bt, const ProdArgs &a, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    switch (prec) {
        case P_F64: return launch_p<P_F64>(bt, a, s);
        case P_F32: return launch_p<P_F32>(bt, a, s);
        case P_F16X3: return launch_p<P_F16X3>(bt, a, s);
        case P_BF16X3: return launch_p<P_BF16X3>(bt, a, s);
        case P_BF16: return launch_p<P_BF16>(bt, a, s);
        case P_F16: return launch_p<P_F16>(bt, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fdm
