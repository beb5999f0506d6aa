// Internal declarations shared by the kernels, the solver driver and the
// server.  Everything here is gfx950 (CDNA4) specific.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "fermidm.h"

namespace fdm {

enum Prec : int { P_F64 = 0, P_F32 = 1, P_F16X3 = 2, P_BF16X3 = 3, P_BF16 = 4, P_F16 = 5 };

// Working matrices are padded to a multiple of this edge; the padding holds
// exact zeros at all times (every kernel writes zeros there and reads only
// inside [0, N)^2 or inside zero padding), so product kernels need no bounds
// checks.
constexpr int kPadEdge = 128;
// K is swept in stages of this many elements (all precisions divide it).
constexpr int kKStep = 64;  // K extent granule: two stages of every precision

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Product tiles are listed in bands of this many tile rows (see upper_tiles).
constexpr int kTileBand = 8;
// 32-wide tiles exist (and their list is kept) only up to this size.
constexpr int64_t kTile32MaxN = 2048;

// Tile rows (and columns) of a product of size n with bt-wide tiles.  The
// tiles cover at least the K extent round_up(n, kKStep) that the products
// read: the working matrices' padding is zero only where a kernel wrote
// zeros, and a product writes exactly its tiles, so 32-wide tiles add a
// row and column of padding tiles when ceil(n / 32) is odd.
inline int64_t tile_rows(int64_t n, int bt) {
    return bt == 32 ? (n + 63) / 64 * 2 : (n + bt - 1) / bt;
}

// 128-wide split products whose K extent round_up(n, 64) ends 64 columns
// into the last tile column cover that column with 256 x 64 edge blocks
// (two tile rows each) instead of half-padding 128-wide tiles: list entries
// upper_tiles(T - 1) followed by (1 << 31) | (q << 16) | (T - 1) for
// q < ceil(T / 2), T = tile_rows(n, 128).
inline bool edge_blocks(int64_t n) { return (n + 63) / 64 % 2 == 1; }
inline int64_t edge_ntiles(int64_t n) {
    const int64_t t = tile_rows(n, 128);
    return (t - 1) * t / 2 + (t + 1) / 2;
}

// Tile edge (32, 64 or 128) of a product of size n in precision prec; forced
// = 32 (n <= kTile32MaxN), 64 or 128 overrides the measured choice.
int choose_tile(int64_t n, int prec, int forced);

// Decide-kernel modes (what the partial sums of the preceding launch mean).
// Phase flags of DevState::switch_mode above the low three bits (which say
// 0 = plain phase, 1 = low-precision phase left at tau, 2 = FP64-first
// steps):
constexpr int kGuard = 8;      // end the phase when ||X||^2 > Tr X + 0.5 (an eigenvalue
                               // of X outside [0, 1]) or a sum is not finite
constexpr int kRelTrStop = 16; // stop when RelTr <= tau instead of the idempotency rule
constexpr int kFixedSteps = 32;// run exactly max_iter products (truncated expansion)

enum DecideMode : int {
    D_INIT = 0,     // partials: Tr X, ||X||^2 of a new iterate; resets the phase
    D_SP2 = 1,      // partials of an SP2 product: Tr X+, ||X+||^2, ||X^2 - X||^2
    D_MCW_T = 2,    // partials of T = X X with E = X: ||X^2 - X||^2 in slot 2
    D_MCW_OUT = 3,  // partials of X' = 3T - 2TX
    D_SUMS = 4,     // plain reduction of (slot0, slot1, slot2) into st->sums
    D_CERT = 5,     // slot1 (a squared Frobenius norm) appended to st->cert
};

// Device-resident solver state: every branch and stop decision is taken on
// the GPU from FP64 sums, so the host never has to read a scalar to enqueue
// the next step.
struct DevState {
    double emin, emax, trH, fro2H;   // Gershgorin bounds and moments of Hp
    double n_occ, tol, tau;
    double trace, fro2;              // of the current iterate
    double idem;                     // last measured ||X_n^2 - X_n||_F
    double idem_hist[2];             // the two before it
    double sums[4];                  // D_SUMS result
    int32_t nonfinite;
    int32_t sigma;                   // branch of the next SP2 product (1 = X^2)
    int32_t done;                    // the current phase is finished
    int32_t iter;                    // products that advanced the phase
    int32_t result_iter;             // index of the result iterate when done
    int32_t executed;                // product launches that ran in this phase
    int32_t max_iter;
    int32_t status;                  // 0 or a negative FDM_ status
    int32_t switch_mode;             // 1: low-precision phase (stop on tau / stagnation)
    int32_t gprod;                   // global SP2 product counter (branch bits)
    uint64_t bits[4];
    double mcw_idem[4], mcw_trerr[4];  // FP64 McWeeny checks: ||X^2 - X||, |Tr X - n_occ|
    double reltr;                    // |Tr X_n - Tr X_{n-1}| / |Tr X_{n-1}| of the last SP2 step
    double idem_ring[8];             // last measured ||X^2 - X||_F values (ring, nring entries)
    int32_t nring;
    int32_t ncert;                   // entries of cert[] written since the last reset
    double cert[8];                  // D_CERT: ||M_k||_F^2 of the bound certificate's powers
};

// What the host polls: written by the decide kernel into mapped pinned memory.
struct HostMirror {
    int32_t done, iter, result_iter, executed, status, sigma;
    double idem, trace;
};

struct ProdArgs {
    const void *A, *B, *E;
    void *C;
    int64_t ld;             // elements
    int32_t n;              // logical size
    int32_t kext;           // K extent (multiple of kKStep)
    const uint32_t *tiles;  // (ti << 16) | tj, ti <= tj
    int32_t ntiles;
    int32_t pad;
    double coef[2][3];      // {alpha, beta, gamma}, selected by *sel (0 if sel null)
    const int32_t *sel;
    const int32_t *done;    // nullable: exit at once if *done != 0
    double *partials;       // [ntiles][4]
    // Split forms: hi/lo 16-bit companions of A, B (read as operands) and C
    // (written by the epilogue), interleaved per 32 columns: row r of a
    // companion matrix holds 2*ld values; columns 32c..32c+31 sit at
    // [64c, 64c + 32) (hi) and [64c + 32, 64c + 64) (lo), so one K stage of
    // one row is a single 128-byte line.
    const uint16_t *Ahl, *Bhl;
    uint16_t *Chl;
};

// ---- launchers (k_symprod.hip, k_aux.hip) --------------------------------
hipError_t launch_symprod(int prec, int bt, const ProdArgs &a, hipStream_t s);

// Grouped launches of the serving tick: up to kMaxGroup products of one
// precision, tile edge and staging path (their tile lists concatenated),
// and up to kMaxGroup decisions (one block each).  Passed by value as
// kernel arguments.
constexpr int kMaxGroup = 16;
struct ProdGroup {
    int32_t njobs;
    int32_t first[kMaxGroup + 1];  // job j owns grid entries [first[j], first[j+1])
    ProdArgs job[kMaxGroup];
};
// The staging path launch_symprod takes for (prec, bt, ld): products are
// grouped only with others of the same path.
bool symprod_direct(int prec, int bt, int64_t ld);
hipError_t launch_symprod_grouped(int prec, int bt, bool direct, const ProdGroup &g,
                                  hipStream_t s);

struct DecideJob {
    DevState *st;
    HostMirror *hm;
    const double *part;
    int32_t count, mode, stride, pad;
};
struct DecideGroup {
    int32_t njobs, pad;
    DecideJob job[kMaxGroup];
};
hipError_t launch_decide_grouped(const DecideGroup &g, hipStream_t s);

// out = a * in + b * I on [0,n)^2, zeros on [0,np)^2 outside; in may be a
// double (caller layout) or a float/double working matrix.  When zt_init is
// set, (a, b) come from the Gershgorin bounds in st: a = -1/(emax-emin),
// b = emax/(emax-emin).  Writes per-block (Tr, ||.||^2) partials.
hipError_t launch_affine(int in_f32, const void *in, int64_t ldi, int out_f32, void *out,
                         int64_t ldo, int n, int np, double a, double b, int zt_init,
                         const DevState *st, double *partials, int *nparts, hipStream_t s);
int affine_blocks(int np);

hipError_t launch_gershgorin(const double *H, int64_t ldh, int n, double *partials,
                             DevState *st, hipStream_t s);
int gershgorin_blocks(int n);

hipError_t launch_decide(DevState *st, HostMirror *hm, const double *partials, int count,
                         int mode, int stride, hipStream_t s);

hipError_t launch_energy(const double *H, int64_t ldh, const double *D, int64_t ldd,
                         int d_f32, int n, double *partials, DevState *st, hipStream_t s);
int energy_blocks(int n);

hipError_t launch_copy_out(int src_f32, const void *src, int64_t lds, double *dst,
                           int64_t ldd, int n, hipStream_t s);

// out = a X + b Y + c I on [0,n)^2 of working matrices (zeros elsewhere in
// [0,np)^2), with per-block (Tr, ||.||^2) partials.
hipError_t launch_axpby2(int f32, const void *X, const void *Y, void *out, int64_t ld, int n,
                         int np, double a, double b, double c, double *partials, int *nparts,
                         hipStream_t s);

hipError_t launch_lanczos(const double *H, int64_t ldh, int n, int np, int k, double *v,
                          double *ab, hipStream_t s);
// k Lanczos steps on the projection of H - sigma I onto range(D) (unocc = 0)
// or onto range(I - D) (unocc = 1), D a density matrix: v holds 5 vectors
// of stride np, ab receives alpha[0..k) then beta[0..k).
hipError_t launch_lanczos_proj(const double *H, int64_t ldh, const double *D, int64_t ldd, int n,
                               int np, int k, int unocc, double sigma, double *v, double *ab,
                               hipStream_t s);
hipError_t launch_set_bounds(DevState *st, double emin, double emax, hipStream_t s);

// hi/lo 16-bit companions of an FP32 working matrix (split precisions):
// hi = rn(s x), lo = rn(s x - hi), s = 2^12 for FP16, 1 for BF16, in the
// interleaved layout of ProdArgs; x is rows x ld (ld a multiple of 32).
hipError_t launch_split(int prec, const float *x, uint16_t *hl, int64_t ld, int64_t rows,
                        hipStream_t s);

hipError_t launch_set_params(DevState *st, double n_occ, double tol, double tau, int max_iter,
                             int switch_mode, int reset_all, hipStream_t s);

// ---- errors ---------------------------------------------------------------
void set_error(const std::string &msg);

}  // namespace fdm
