// Solver driver and C ABI.
//
// Zero temperature (Sec. II.B.1, Eq. (1)):
//   bounds (Gershgorin, Sec. II.C) -> X_0 = (e_max I - H)/(e_max - e_min) ->
//   SP2 products, each fused with its branch update and trace sums, the
//   branch for the next product and the stop test decided on the device.
// Mixed precision (Sec. III.A): a few FP64 SP2 steps, then low-precision SP2
//   steps on an FP32 master until ||X^2 - X||_F <= tau, then FP64 McWeeny
//   steps X <- 3X^2 - 2X^3 until ||X^2 - X||_F <= tol.
// Finite temperature (Sec. II.B.3, Eq. (2)): see finite_t.hip.
//
// The host enqueues one step ahead of what it has observed: it waits on the
// event of step k-1 while step k runs, so the device never idles on a host
// round trip, and at most one step per phase is launched after convergence
// (those launches see the device "done" flag and return at once).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "fdm_internal.h"
#include "solver_internal.h"

namespace fdm {

static thread_local std::string tl_err;
void set_error(const std::string &msg) { tl_err = msg; }
const char *last_error() { return tl_err.c_str(); }

int hip_fail(hipError_t e, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return FDM_EHIP;
}

// ---------------------------------------------------------------------------
// tile lists
// ---------------------------------------------------------------------------
// Upper-triangular tiles (ti <= tj) in bands of kTileBand tile rows, each band
// walked column by column: the blocks that run at the same time on one XCD
// (a contiguous run of this list) share a few row panels of A and B, so the
// panel k-slices they stream are reused from that XCD's L2.
static std::vector<uint32_t> upper_tiles(int nt) {
    std::vector<uint32_t> v;
    v.reserve((size_t)nt * (nt + 1) / 2);
    for (int i0 = 0; i0 < nt; i0 += kTileBand)
        for (int j = i0; j < nt; ++j)
            for (int i = i0; i < std::min(i0 + kTileBand, j + 1); ++i)
                v.push_back(((uint32_t)i << 16) | (uint32_t)j);
    return v;
}

static int64_t ntiles_for(int64_t n, int bt) {
    const int64_t nt = tile_rows(n, bt);
    return nt * (nt + 1) / 2;
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
// Workspace of n64 FP64 and n32 FP32 working matrices (each FP32 one with
// its hi/lo 16-bit companions), per-tile partials, tile lists, Lanczos
// vectors and the device state, each part 256-byte aligned.
static Layout plan_mats(int64_t n, int n64, int n32) {
    Layout L;
    L.n = n;
    L.np = round_up(std::max<int64_t>(n, 1), kPadEdge);
    L.ld = L.np;
    L.n64 = n64;
    L.n32 = n32;
    const size_t mat64 = (size_t)L.np * L.ld * 8, mat32 = (size_t)L.np * L.ld * 4;
    const int64_t tiles64 = ntiles_for(n, 64), tiles128 = ntiles_for(n, 128);
    const int64_t tiles32 = n <= kTile32MaxN ? ntiles_for(n, 32) : 0;
    const int64_t parts = std::max<int64_t>({tiles32, tiles64, (L.np + 3) / 4, 1});
    size_t off = 0;
    L.off64 = off;
    off += mat64 * L.n64;
    L.off32 = off;
    off += mat32 * L.n32;
    L.off16 = off;
    off += mat32 * L.n32;  // hi + lo halves per element
    L.off_part = off;
    off += round_up(parts * 8 * sizeof(double), 256);
    L.off_tiles64 = off;
    off += round_up(tiles64 * 4, 256);
    L.off_tiles128 = off;
    off += round_up(tiles128 * 4, 256);
    L.off_tiles32 = off;
    off += round_up(std::max<int64_t>(tiles32, 1) * 4, 256);
    const int64_t tiles128e = edge_blocks(n) ? edge_ntiles(n) : 0;
    L.off_tiles128e = off;
    off += round_up(tiles128e * 4, 256);
    L.off_lanczos = off;
    off += round_up((5 * L.np + 2 * kMaxLanczos) * sizeof(double), 256);
    L.off_state = off;
    off += round_up(sizeof(DevState), 256);
    L.bytes = off;
    L.ntiles64 = (int)tiles64;
    L.ntiles128 = (int)tiles128;
    L.ntiles32 = (int)tiles32;
    L.ntiles128e = (int)tiles128e;
    L.part_cap = parts;
    return L;
}

Layout plan_layout(int64_t n, bool finite, int prec) {
    return plan_mats(n, finite ? 5 : 3, (prec == P_F64) ? 0 : (finite ? 5 : 2));
}

// A single product call: four working matrices (A, B, E, C) of the
// product's precision (FP64, or FP32 masters with companions).
Layout plan_product_layout(int64_t n, int prec) {
    return prec == P_F64 ? plan_mats(n, 4, 0) : plan_mats(n, 0, 4);
}

void Resources::view(const Layout &L, char *mem) {
    lay = L;
    x64 = (double *)(mem + L.off64);
    x32 = (float *)(mem + L.off32);
    x16 = (uint16_t *)(mem + L.off16);
    part = (double *)(mem + L.off_part);
    tiles64 = (uint32_t *)(mem + L.off_tiles64);
    tiles128 = (uint32_t *)(mem + L.off_tiles128);
    tiles32 = (uint32_t *)(mem + L.off_tiles32);
    tiles128e = L.ntiles128e > 0 ? (uint32_t *)(mem + L.off_tiles128e) : nullptr;
    st = (DevState *)(mem + L.off_state);
    lanczos = (double *)(mem + L.off_lanczos);
}

Resources::~Resources() {
    for (hipEvent_t e : ev)
        if (e) hipEventDestroy(e);
    if (entry) hipEventDestroy(entry);
    for (hipEvent_t e : tev) hipEventDestroy(e);
    if (owned && base) hipFree(base);
    // the mapped host mirror is intentionally kept until process exit
}

int Resources::init(int dev) {
    device = dev;
    hipError_t e;
    for (int i = 0; i < kEvRing; ++i) {
        e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    e = hipEventCreateWithFlags(&entry, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    e = hipHostMalloc((void **)&hm_host, sizeof(HostMirror),
                      hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
    memset((void *)hm_host, 0, sizeof(HostMirror));
    e = hipHostGetDevicePointer((void **)&hm_dev, (void *)hm_host, 0);
    if (e != hipSuccess) return hip_fail(e, "hipHostGetDevicePointer");
    return FDM_OK;
}

int Resources::bind(const Layout &L, void *user_mem, size_t user_bytes, hipStream_t s) {
    hipError_t e;
    char *mem;
    if (user_mem) {
        if (user_bytes < L.bytes) {
            set_error("workspace_bytes smaller than fdm_workspace_bytes()");
            return FDM_EINVAL;
        }
        // the product kernels read whole 16-byte chunks of 128-byte rows
        if ((uintptr_t)user_mem % 256 != 0) {
            set_error("workspace must be 256-byte aligned");
            return FDM_EINVAL;
        }
        mem = (char *)user_mem;
    } else {
        if (!owned || cap < L.bytes) {
            if (owned && base) {
                e = hipStreamSynchronize(s);
                if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
                hipFree(base);
            }
            base = nullptr;
            owned = false;
            cap = 0;
            e = hipMalloc((void **)&base, L.bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                set_error("hipMalloc of " + std::to_string(L.bytes) + " workspace bytes failed");
                return FDM_ENOMEM;
            }
            owned = true;
            cap = L.bytes;
            bound_key = -1;
        }
        mem = base;
    }
    // A caller-provided block may have been used by anyone since: always
    // re-zero it and re-upload the tile lists.
    const bool fresh = user_mem != nullptr || (mem != bound_mem) ||
                       bound_key != (L.n * 16 + L.n64 * 4 + L.n32) || bound_ld != L.ld;
    view(L, mem);
    if (fresh) {
        // zero every matrix (the padding must hold zeros) and upload tile lists
        e = hipMemsetAsync(mem, 0, L.off_part, s);  // FP64, FP32 and 16-bit companions
        if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
        e = hipMemsetAsync(st, 0, sizeof(DevState), s);
        if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
        std::vector<uint32_t> t64 = upper_tiles((int)tile_rows(L.n, 64));
        std::vector<uint32_t> t128 = upper_tiles((int)tile_rows(L.n, 128));
        e = hipMemcpyAsync(tiles64, t64.data(), t64.size() * 4, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
        e = hipMemcpyAsync(tiles128, t128.data(), t128.size() * 4, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
        std::vector<uint32_t> t128e;
        if (L.ntiles128e > 0) {
            const int t = (int)tile_rows(L.n, 128);
            t128e = upper_tiles(t - 1);
            for (int q = 0; q < (t + 1) / 2; ++q)
                t128e.push_back(0x80000000u | ((uint32_t)q << 16) | (uint32_t)(t - 1));
            if ((int64_t)t128e.size() != L.ntiles128e) {
                set_error("internal: edge-block list size");
                return FDM_EHIP;
            }
            e = hipMemcpyAsync(tiles128e, t128e.data(), t128e.size() * 4, hipMemcpyHostToDevice,
                               s);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
        }
        std::vector<uint32_t> t32;
        if (L.ntiles32 > 0) {
            t32 = upper_tiles((int)tile_rows(L.n, 32));
            e = hipMemcpyAsync(tiles32, t32.data(), t32.size() * 4, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
        }
        e = hipStreamSynchronize(s);  // the host vectors die here
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        bound_mem = mem;
        bound_key = L.n * 16 + L.n64 * 4 + L.n32;
        bound_ld = L.ld;
    }
    return FDM_OK;
}

hipEvent_t Resources::timing_event(size_t i) {
    while (tev.size() <= i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        tev.push_back(e);
    }
    return tev[i];
}

static std::mutex g_res_mu;

Resources *thread_resources(int dev) {
    thread_local std::vector<std::unique_ptr<Resources>> pool;
    if ((int)pool.size() <= dev) pool.resize(dev + 1);
    if (!pool[dev]) {
        std::unique_ptr<Resources> r(new Resources());
        if (r->init(dev) != FDM_OK) return nullptr;
        pool[dev] = std::move(r);
    }
    return pool[dev].get();
}

// ---------------------------------------------------------------------------
// context helpers
// ---------------------------------------------------------------------------
int Ctx::tile_for(int prec) const { return choose_tile(n, prec, opt.tile); }

int choose_tile(int64_t n, int prec, int forced) {
    if (forced == 64 || forced == 128) return forced;
    if (forced == 32) return n <= kTile32MaxN ? 32 : 64;
    // Small products: fewer than 128 tiles of 64 leave most of the 256 CUs
    // idle, and a product is launch- and latency-bound; 32-wide tiles give
    // four times the blocks (N = 256: 36 instead of 10).
    if (n <= kTile32MaxN && ntiles_for(n, 64) < 128) return 32;
    // Measured on MI355X.
    // FP32: 128-wide tiles (two waves per SIMD) once there are at least 16
    // waves of them for the chip (N >= ~11500): 108 -> 128 TFLOP/s on a
    // dense N = 16000 matrix, 121 -> 127 on the paper's N = 16384 one; even
    // at N = 8192, far slower at N = 4000 (528 tiles).
    // FP64: the same rule as FP32.  With direct-to-LDS staging the 128-wide
    // tiles gain 10% on the dense N = 16000 matrix (65.0 -> 58.9 ms per
    // product) and 4-5% on the paper's matrices (66.9 -> 63.9 ms at
    // N = 16384, 68.1 -> 70.6 TFLOP/s at N = 32768).
    // Split forms: 128-wide tiles at two waves per SIMD with the 256-deep
    // fold once there are 2048 of them (N >= ~8100): 615 -> 753 TFLOP/s at
    // N = 8192, 606 -> 907 at N = 16000, 673 -> 1010 on the paper's
    // N = 32768 matrix, same SP2 floor.  (Without any fold they never got
    // below tau there.)  Below that the 64-wide tiles win where both sizes
    // leave the same number of waves of blocks (N = 4000: 2016 tiles in two
    // waves of 1024 slots against 528 in two waves of 512), but where all
    // 128-wide tiles fit in one wave of 512 slots and the 64-wide ones need
    // well over one wave of 1024, the 128-wide ones are faster: 0.177 ->
    // 0.162 ms at N = 3500, 0.243 -> 0.192 ms at N = 3968 (3000: 0.129 vs
    // 0.133, 64-wide still ahead).  The single-pass 16-bit forms (reported,
    // not gated) take 128-wide tiles once there are enough to fill the chip.
    const int64_t t128 = ntiles_for(n, 128);
    if (prec == P_F64 || prec == P_F32) return (t128 >= 16 * 256) ? 128 : 64;
    if (prec == P_F16X3 || prec == P_BF16X3) {
        const int64_t t64 = ntiles_for(n, 64);
        // blocks of the 128-wide launch, with edge blocks where the K extent
        // ends 64 columns into the last tile column (N = 4000: 496 tiles and
        // 16 edge blocks, one wave, instead of 528 tiles)
        const int64_t b128 = edge_blocks(n) ? edge_ntiles(n) : t128;
        const bool one_wave_128 = b128 <= 2 * 256 && t64 >= 1400;
        return (t128 >= 8 * 256 || one_wave_128) ? 128 : 64;
    }
    return (t128 >= 4 * 256) ? 128 : 64;
}

// The tile list of edge bt for precision prec: the 128-wide split products
// staged straight into LDS take the list with edge blocks where there is one.
static void set_tiles(ProdArgs &a, const Resources *r, int bt, int prec) {
    a.tiles = (bt == 128) ? r->tiles128 : (bt == 32 ? r->tiles32 : r->tiles64);
    a.ntiles = (bt == 128) ? r->lay.ntiles128 : (bt == 32 ? r->lay.ntiles32 : r->lay.ntiles64);
    if (bt == 128 && (prec == P_F16X3 || prec == P_BF16X3) && r->tiles128e != nullptr &&
        symprod_direct(prec, 128, r->lay.ld)) {
        a.tiles = r->tiles128e;
        a.ntiles = r->lay.ntiles128e;
    }
}

int Ctx::product(int prec, const void *A, const void *B, const void *E, void *C,
                 const double c0[3], const double c1[3], bool sel, bool done_guard) {
    ProdArgs a;
    memset(&a, 0, sizeof(a));
    const int bt = tile_for(prec);
    a.A = A;
    a.B = B;
    a.E = E;
    a.C = C;
    a.ld = r->lay.ld;
    a.n = (int32_t)n;
    a.kext = (int32_t)round_up(n, kKStep);
    set_tiles(a, r, bt, prec);
    for (int k = 0; k < 3; ++k) {
        a.coef[0][k] = c0[k];
        a.coef[1][k] = c1 ? c1[k] : c0[k];
    }
    a.sel = sel ? &r->st->sigma : nullptr;
    a.done = done_guard ? &r->st->done : nullptr;
    a.partials = r->part;
    if (prec == P_F16X3 || prec == P_BF16X3) {
        const size_t m = (size_t)r->lay.np * r->lay.ld;
        auto comp = [&](const void *p) -> uint16_t * {
            const float *f = (const float *)p;
            if (f < r->x32 || f >= r->x32 + (size_t)r->lay.n32 * m) return nullptr;
            const size_t i = (size_t)(f - r->x32) / m;
            return r->x16 + i * 2 * m;
        };
        a.Ahl = comp(A);
        a.Bhl = comp(B);
        a.Chl = comp(C);
        if (!a.Ahl || !a.Bhl || !a.Chl) {
            set_error("internal: split operand outside the FP32 working buffers");
            return FDM_EHIP;
        }
    }
    last_ntiles = a.ntiles;
    used_tile = bt;
    if (cap) {
        // recorded for the serving tick (launched grouped with other solves)
        StepOp o;
        o.kind = StepOp::PRODUCT;
        o.prec = prec;
        o.bt = bt;
        o.direct = symprod_direct(prec, bt, a.ld);
        o.a = a;
        cap->ops.push_back(std::move(o));
        phase_launches.push_back(prec);
        if (cap_stream) {
            tick_post(group, &member, cap_seq++, std::move(stream_step));
            stream_step.ops.clear();
        }
        return FDM_OK;
    }
    hipError_t e;
    if (opt.timing) {
        hipEvent_t e0 = r->timing_event(2 * timed.size()), e1 = r->timing_event(2 * timed.size() + 1);
        if (!e0 || !e1) return hip_fail(hipErrorOutOfMemory, "hipEventCreate");
        e = hipEventRecord(e0, s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        e = launch_symprod(prec, bt, a, s);
        if (e != hipSuccess) return hip_fail(e, "symmetric product launch");
        e = hipEventRecord(e1, s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        timed.push_back({prec, 2 * timed.size(), 2 * timed.size() + 1, true});
    } else {
        e = launch_symprod(prec, bt, a, s);
        if (e != hipSuccess) return hip_fail(e, "symmetric product launch");
    }
    phase_launches.push_back(prec);
    return FDM_OK;
}

// Product launches of the finished phase that did work: the first `executed`
// of them.  The rest returned at once on the device's done flag.
void Ctx::close_phase(int executed) {
    const size_t keep = std::min<size_t>((size_t)std::max(executed, 0), phase_launches.size());
    for (size_t i = 0; i < keep; ++i) {
        const int p = phase_launches[i];
        stats.products[p] += 1;
        const double nn = (double)n;
        stats.flops[p] += nn * nn * (nn + 1.0) * ((p == P_F16X3 || p == P_BF16X3) ? 3.0 : 1.0);
    }
    if (opt.timing) {
        // timed entries of this phase are the last phase_launches.size() ones
        const size_t first = timed.size() - phase_launches.size();
        for (size_t i = first + keep; i < timed.size(); ++i) timed[i].real = false;
    }
    phase_launches.clear();
}

int Ctx::decide(int mode, int count, int stride) {
    if (cap) {
        StepOp o;
        o.kind = StepOp::DECIDE;
        o.d = DecideJob{r->st, r->hm_dev, r->part, count, mode, stride, 0};
        cap->ops.push_back(std::move(o));
        return FDM_OK;
    }
    hipError_t e = launch_decide(r->st, r->hm_dev, r->part, count, mode, stride, s);
    return e == hipSuccess ? FDM_OK : hip_fail(e, "decide launch");
}

int Ctx::set_params(double tau, int max_iter, int switch_mode, int reset_all) {
    hipError_t e = launch_set_params(r->st, n_occ, tol, tau, max_iter, switch_mode, reset_all, s);
    return e == hipSuccess ? FDM_OK : hip_fail(e, "set_params launch");
}

int Ctx::affine(int in_f32, const void *in, int64_t ldi, int out_f32, void *out, double a,
                double b, int zt, int *nparts) {
    if (cap) {
        // recorded for the serving tick, with the companion split it implies
        const int64_t ld = r->lay.ld, np = r->lay.np;
        const int nn = (int)n;
        const DevState *st = r->st;
        double *part = r->part;
        uint16_t *hl = nullptr;
        if (out_f32 && (split_prec == P_F16X3 || split_prec == P_BF16X3)) {
            const size_t m = (size_t)np * ld;
            const float *f = (const float *)out;
            if (f >= r->x32 && f < r->x32 + (size_t)r->lay.n32 * m)
                hl = r->x16 + (size_t)(f - r->x32) / m * 2 * m;
        }
        const int sp = split_prec;
        if (nparts) *nparts = affine_blocks((int)np);
        StepOp o;
        o.kind = StepOp::CUSTOM;
        o.custom = [=](hipStream_t st_) -> hipError_t {
            hipError_t e = launch_affine(in_f32, in, ldi, out_f32, out, ld, nn, (int)np, a, b, zt,
                                         st, part, nullptr, st_);
            if (e == hipSuccess && hl) e = launch_split(sp, (const float *)out, hl, ld, np, st_);
            return e;
        };
        cap->ops.push_back(std::move(o));
        return FDM_OK;
    }
    hipError_t e = launch_affine(in_f32, in, ldi, out_f32, out, r->lay.ld, (int)n,
                                 (int)r->lay.np, a, b, zt, r->st, r->part, nparts, s);
    if (e != hipSuccess) return hip_fail(e, "affine launch");
    if (out_f32 && (split_prec == P_F16X3 || split_prec == P_BF16X3)) {
        // an FP32 operand of split products: write its hi/lo companions
        const size_t m = (size_t)r->lay.np * r->lay.ld;
        const float *f = (const float *)out;
        if (f >= r->x32 && f < r->x32 + (size_t)r->lay.n32 * m) {
            const size_t i = (size_t)(f - r->x32) / m;
            e = launch_split(split_prec, f, r->x16 + i * 2 * m, r->lay.ld, r->lay.np, s);
            if (e != hipSuccess) return hip_fail(e, "split launch");
        }
    }
    return FDM_OK;
}

// Runs `enqueue(k)` for k = 0, 1, ... keeping exactly one step in flight
// beyond the last one observed, until the device reports done.
// FDM_PROGRESS=k (environment) prints a line to stderr after every k-th
// completed step of a phase: long solves (minutes at N = 65536) show that
// they advance.
static int progress_every() {
    static const int every = [] {
        const char *v = getenv("FDM_PROGRESS");
        return v ? std::max(0, atoi(v)) : 0;
    }();
    return every;
}

// Steps kept in flight beyond the one the host waits on (a step that starts
// after the device has decided to stop returns at once).  One is enough:
// measured on MI355X, 2, 4 or 7 steps in flight left the N = 256 solve at
// 1.06-1.12 ms and the N = 1000 ... 4000 solves within 3% (the device runs
// each step's launches back to back either way).  FDM_LOOKAHEAD=k
// (1 ... kEvRing - 1) overrides.
static int lookahead() {
    static const int look = [] {
        const char *v = getenv("FDM_LOOKAHEAD");
        const int k = v ? atoi(v) : 1;
        return std::min(std::max(k, 1), kEvRing - 1);
    }();
    return look;
}

// The same loop inside a serving tick group: the steps are recorded and
// posted, the group launches them with other solves' steps, and the host
// waits for each step's event as above.
int Ctx::run_loop_grouped(int max_steps, const std::function<int(int)> &enqueue) {
    const int every = progress_every();
    const int look = lookahead();
    volatile int32_t *done = &r->hm_host->done;
    *done = 0;
    int rc = tick_join(group, &member, s);
    if (rc) return rc;
    int issued = 0;
    auto issue = [&]() -> int {
        Step st;
        cap = &st;
        int q = enqueue(issued);
        cap = nullptr;
        if (q) return q;
        tick_post(group, &member, issued, std::move(st));
        ++issued;
        return FDM_OK;
    };
    while (rc == FDM_OK && issued < max_steps && issued <= look) rc = issue();
    for (int k = 0; rc == FDM_OK && k < max_steps; ++k) {
        rc = tick_wait(group, &member, k);
        if (rc) break;
        if (every > 0 && (k + 1) % every == 0) {
            fprintf(stderr, "[fdm] n=%lld step %d done\n", (long long)n, k + 1);
            fflush(stderr);
        }
        if (*done) break;
        if (issued < max_steps) rc = issue();
    }
    const int rc2 = tick_leave(group, &member);
    if (rc) return rc;
    if (rc2) return rc2;
    if (*done) return FDM_OK;
    set_error("internal: phase ended without a device decision");
    return FDM_EHIP;
}

// Finite-temperature evaluations inside a tick group: every launch of the
// evaluation is recorded, and a step is posted at each product; the host
// waits once, at the end.
int Ctx::begin_stream_capture() {
    if (!group) return FDM_OK;
    int rc = tick_join(group, &member, s);
    if (rc) return rc;
    stream_step.ops.clear();
    cap = &stream_step;
    cap_stream = true;
    cap_seq = 0;
    return FDM_OK;
}

int Ctx::end_stream_capture() {
    if (!group) return FDM_OK;
    if (!stream_step.ops.empty()) {
        tick_post(group, &member, cap_seq++, std::move(stream_step));
        stream_step.ops.clear();
    }
    cap = nullptr;
    cap_stream = false;
    int rc = cap_seq > 0 ? tick_wait(group, &member, cap_seq - 1) : FDM_OK;
    const int rc2 = tick_leave(group, &member);
    return rc ? rc : rc2;
}

int Ctx::run_loop(int max_steps, const std::function<int(int)> &enqueue) {
    if (group) return run_loop_grouped(max_steps, enqueue);
    const int every = progress_every();
    const int look = lookahead();
    // The device writes the mirror once, when it decides to stop; every step
    // of the previous phase has finished (the previous run_loop waited for
    // its last one), and no kernel enqueued since ends a phase.
    volatile int32_t *done = &r->hm_host->done;
    *done = 0;
    int issued = 0;  // steps 0 ... issued - 1 are enqueued, each with its event
    auto issue = [&]() -> int {
        int rc = enqueue(issued);
        if (rc) return rc;
        hipError_t e = hipEventRecord(r->ev[issued % kEvRing], s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        ++issued;
        return FDM_OK;
    };
    while (issued < max_steps && issued <= look) {
        int rc = issue();
        if (rc) return rc;
    }
    for (int k = 0; k < max_steps; ++k) {
        hipError_t e = hipEventSynchronize(r->ev[k % kEvRing]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        if (every > 0 && (k + 1) % every == 0) {
            fprintf(stderr, "[fdm] n=%lld step %d done\n", (long long)n, k + 1);
            fflush(stderr);
        }
        if (*done) {
            // The steps enqueued after the observed one see the device's done
            // flag and return at once; wait for them too, so that the mirror
            // (written by whichever decide set done) and the buffers are final
            // before the caller reads them.
            if (issued - 1 > k) {
                e = hipEventSynchronize(r->ev[(issued - 1) % kEvRing]);
                if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
            }
            return FDM_OK;
        }
        if (issued < max_steps) {
            int rc = issue();
            if (rc) return rc;
        }
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (*done) return FDM_OK;
    set_error("internal: phase ended without a device decision");
    return FDM_EHIP;
}

// Accelerated expansion (A-Z-RFOE, Sec. II.B.2): the unoccupied eigenvalues
// of X_0 lie in [0, l0], the occupied ones in [h0, 1].  Each step squares the
// larger of the errors e_u = l and e_o = 1 - h with the parabola's vertex
// moved to half of it, so the two ends of that interval land on the same
// value:
//     e_u >= e_o:  p(x) = k (x - s)^2,          s = e_u / 2
//     e_u <  e_o:  p(x) = 1 - k (1 - s - x)^2,  s = e_o / 2,  k = 1 / (1 - s)^2
// (s = 0 gives X^2 and 2X - X^2).  The interval ends' images are the next
// bounds, so the sequence depends on (l0, h0) only and is fixed up front.
void Ctx::build_az_schedule(double l, double h, int steps) {
    az_coef.assign(3 * (size_t)steps, 0.0);
    az_gap.assign(steps + 1, 0.0);
    az_gap[0] = h - l;
    az_branch.assign(steps, 0);
    for (int j = 0; j < steps; ++j) {
        const double eu = l, eo = 1.0 - h;
        double *c = &az_coef[3 * (size_t)j];
        if (eu >= eo) {
            const double sh = 0.5 * eu, k = 1.0 / ((1.0 - sh) * (1.0 - sh));
            c[0] = k;
            c[1] = -2.0 * k * sh;
            c[2] = k * sh * sh;
            az_branch[j] = 1;
            l = k * sh * sh;
            h = k * (h - sh) * (h - sh);
        } else {
            const double sh = 0.5 * eo, k = 1.0 / ((1.0 - sh) * (1.0 - sh)), u = 1.0 - sh;
            c[0] = -k;
            c[1] = 2.0 * k * u;
            c[2] = 1.0 - k * u * u;
            az_branch[j] = 0;
            l = 1.0 - k * (u - l) * (u - l);
            h = 1.0 - k * sh * sh;
        }
        az_gap[j + 1] = h - l;
    }
}

// SP2 products from X_0 in bufs[0] (its sums already reduced by D_INIT).
// sched_off >= 0: step k applies the accelerated polynomial sched_off + k;
// otherwise the device picks X^2 or 2X - X^2 from the traces.
int Ctx::sp2_phase(int prec, void *b0, void *b1, int max_iter, int switch_mode, double tau,
                   int sched_off, void **result, int *iters) {
    // An eigenvalue of X outside [0, 1] (shifted polynomials built from
    // wrong HOMO / LUMO bounds; with certified spectral bounds nothing else
    // can put one there) ends the phase with FDM_ENOCONV instead of folding
    // back into [0, 1] on the wrong side.
    int rc = set_params(tau, max_iter, switch_mode | kGuard, 0);
    if (rc) return rc;
    void *bufs[2] = {b0, b1};
    // sel = 0: 2X - X^2 ;  sel = 1: X^2
    static const double c_sub[3] = {-1.0, 2.0, 0.0};
    static const double c_sq[3] = {1.0, 0.0, 0.0};
    rc = run_loop(max_iter, [&](int k) -> int {
        int q;
        if (sched_off >= 0 && !az_branch.empty()) {
            const size_t j = std::min((size_t)(sched_off + k), az_branch.size() - 1);
            q = product(prec, bufs[k & 1], bufs[k & 1], bufs[k & 1], bufs[(k + 1) & 1],
                        &az_coef[3 * j], nullptr, false, true);
        } else {
            q = product(prec, bufs[k & 1], bufs[k & 1], bufs[k & 1], bufs[(k + 1) & 1], c_sub,
                        c_sq, true, true);
        }
        if (q) return q;
        return decide(D_SP2, last_ntiles, 4);
    });
    if (rc) return rc;
    const HostMirror hm = *r->hm_host;
    close_phase(hm.executed);
    *result = bufs[hm.result_iter & 1];
    if (iters) *iters = hm.iter;
    if (hm.status) status = hm.status;
    return FDM_OK;
}

// FP64 McWeeny steps from X in x[0]: T = X X (measures ||X^2 - X||), then
// X <- 3T - 2 T X.  Buffers x[0], x[2] alternate as X; x[1] holds T.
int Ctx::mcweeny_phase(double *x0, double *t, double *x1, int max_steps, double **result,
                       int *steps) {
    int rc = set_params(0.0, max_steps, 0, 0);
    if (rc) return rc;
    double *xs[2] = {x0, x1};
    static const double c_t[3] = {1.0, 0.0, 0.0};
    static const double c_out[3] = {-2.0, 3.0, 0.0};
    rc = run_loop(max_steps + 1, [&](int k) -> int {
        double *x = xs[k & 1], *xn = xs[(k + 1) & 1];
        int q = product(P_F64, x, x, x, t, c_t, nullptr, false, true);
        if (q) return q;
        q = decide(D_MCW_T, last_ntiles, 4);
        if (q) return q;
        q = product(P_F64, t, x, t, xn, c_out, nullptr, false, true);
        if (q) return q;
        return decide(D_MCW_OUT, last_ntiles, 4);
    });
    if (rc) return rc;
    const HostMirror hm = *r->hm_host;
    close_phase(hm.executed);
    *result = xs[hm.result_iter & 1];
    if (steps) *steps = hm.result_iter;
    if (hm.status) status = hm.status;
    stats.idempotency = hm.idem;
    return FDM_OK;
}

int Ctx::read_state(DevState *out) {
    hipError_t e = hipMemcpyAsync(r->st_host(), r->st, sizeof(DevState), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    *out = *r->st_host();
    return FDM_OK;
}

DevState *Resources::st_host() {
    if (!st_pinned) {
        if (hipHostMalloc((void **)&st_pinned, sizeof(DevState), hipHostMallocDefault) != hipSuccess)
            st_pinned = &st_fallback;
    }
    return st_pinned;
}

// Finishes a solve whose density matrix is the FP64 working matrix `dm`.
int Ctx::finish(const double *Hp, int64_t ldh, const void *dm, int dm_f32, double *D, int64_t ldd,
                double *E_band) {
    hipError_t e = launch_energy(Hp, ldh, (const double *)dm, r->lay.ld, dm_f32, (int)n, r->part,
                                 r->st, s);
    if (e != hipSuccess) return hip_fail(e, "energy launch");
    e = launch_copy_out(dm_f32, dm, r->lay.ld, D, ldd, (int)n, s);
    if (e != hipSuccess) return hip_fail(e, "copy-out launch");
    DevState h;
    int rc = read_state(&h);
    if (rc) return rc;
    stats.band_energy = h.sums[0];
    stats.trace = h.sums[1];
    stats.rel_trace = h.reltr;
    stats.idem_tail_len = std::min(h.nring, 8);
    for (int i = 0; i < stats.idem_tail_len; ++i)
        stats.idem_tail[i] = h.idem_ring[(h.nring - stats.idem_tail_len + i) & 7];
    const int sp2_steps = stats.iters_fp64 + stats.iters_fp64_first + stats.iters_low;
    for (int k = 0; k < 4; ++k) {
        stats.branch_bits[k] = h.bits[k];
        if (!az_branch.empty()) {
            // the accelerated forms follow the fixed schedule
            uint64_t b = 0;
            for (int j = 0; j < 64; ++j) {
                const int g = 64 * k + j;
                if (g < sp2_steps && g < (int)az_branch.size() && az_branch[g]) b |= 1ull << j;
            }
            stats.branch_bits[k] = b;
        }
        stats.mcweeny_idem[k] = (k <= stats.mcweeny_steps && stats.mcweeny_steps > 0) ||
                                        (k == 0 && stats.iters_low > 0)
                                    ? h.mcw_idem[k]
                                    : 0.0;
        stats.mcweeny_trace_err[k] = stats.mcweeny_idem[k] != 0.0 ? h.mcw_trerr[k] : 0.0;
    }
    if (E_band) *E_band = h.sums[0];
    return FDM_OK;
}

// ---------------------------------------------------------------------------
// zero temperature
// ---------------------------------------------------------------------------
static double unit_roundoff(int prec) {
    switch (prec) {
        case P_F64: return 1.1e-16;
        case P_F32: return 6.0e-8;
        case P_F16X3: return 6.0e-8;
        case P_BF16X3: return 1.5e-5;
        case P_F16: return 4.9e-4;
        default: return 3.9e-3;
    }
}

int Ctx::bounds(const double *Hp, int64_t ldh, DevState *h) {
    hipError_t e = launch_gershgorin(Hp, ldh, (int)n, r->part, r->st, s);
    if (e != hipSuccess) return hip_fail(e, "gershgorin launch");
    int rc = read_state(h);
    if (rc) return rc;
    stats.e_min = stats.gersh_min = h->emin;
    stats.e_max = stats.gersh_max = h->emax;
    if (h->nonfinite) {
        set_error("Hp holds NaN or Inf in " + std::to_string(h->nonfinite) + " rows");
        return FDM_ENONFINITE;
    }
    return FDM_OK;
}

// Eigenpairs of a small dense symmetric matrix (cyclic Jacobi), for the
// Lanczos tridiagonal.  a is k x k row-major (destroyed); w, V (columns).
static void small_eigh(int k, std::vector<double> &a, std::vector<double> &w,
                       std::vector<double> &V) {
    V.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) V[(size_t)i * k + i] = 1.0;
    for (int sweep = 0; sweep < 80; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                const double x = a[(size_t)i * k + j];
                tot += x * x;
                if (i != j) off += x * x;
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < k - 1; ++p)
            for (int q = p + 1; q < k; ++q) {
                const double apq = a[(size_t)p * k + q];
                if (apq == 0.0) continue;
                const double th = (a[(size_t)q * k + q] - a[(size_t)p * k + p]) / (2.0 * apq);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
                const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
                for (int r = 0; r < k; ++r) {
                    const double x = a[(size_t)r * k + p], y = a[(size_t)r * k + q];
                    a[(size_t)r * k + p] = c * x - sn * y;
                    a[(size_t)r * k + q] = sn * x + c * y;
                }
                for (int r = 0; r < k; ++r) {
                    const double x = a[(size_t)p * k + r], y = a[(size_t)q * k + r];
                    a[(size_t)p * k + r] = c * x - sn * y;
                    a[(size_t)q * k + r] = sn * x + c * y;
                }
                for (int r = 0; r < k; ++r) {
                    const double x = V[(size_t)r * k + p], y = V[(size_t)r * k + q];
                    V[(size_t)r * k + p] = c * x - sn * y;
                    V[(size_t)r * k + q] = sn * x + c * y;
                }
            }
    }
    w.resize(k);
    for (int i = 0; i < k; ++i) w[i] = a[(size_t)i * k + i];
}

// Tighter bounds: k Lanczos steps on Hp give the tridiagonal T_k; its extreme
// eigenvalues theta are Ritz values of Hp with residual |beta_k s_k| (s_k the
// last component of T_k's eigenvector).  The bounds are theta -+ (residual +
// 1% of the Ritz width), clipped to the Gershgorin interval in *h.
int Ctx::refine_bounds(const double *Hp, int64_t ldh, DevState *h) {
    int k = opt.lanczos_steps > 0 ? std::min(opt.lanczos_steps, kMaxLanczos) : 16;
    k = (int)std::min<int64_t>(k, n);
    if (k < 2) return FDM_OK;
    double *ab = r->lanczos + 5 * r->lay.np;
    hipError_t e = launch_lanczos(Hp, ldh, (int)n, (int)r->lay.np, k, r->lanczos, ab, s);
    if (e != hipSuccess) return hip_fail(e, "lanczos launch");
    std::vector<double> hab(2 * k);
    e = hipMemcpyAsync(hab.data(), ab, 2 * k * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    const double *alpha = hab.data(), *beta = hab.data() + k;
    double scale = 0.0;
    for (int j = 0; j < k; ++j) scale = std::max(scale, fabs(alpha[j]) + fabs(beta[j]));
    int m = k;  // an (almost) invariant Krylov space ends the recursion early
    for (int j = 0; j < k - 1; ++j)
        if (!(beta[j] > 1e-13 * scale)) {
            m = j + 1;
            break;
        }
    std::vector<double> T((size_t)m * m, 0.0), w, V;
    for (int j = 0; j < m; ++j) {
        T[(size_t)j * m + j] = alpha[j];
        if (j + 1 < m) T[(size_t)j * m + j + 1] = T[(size_t)(j + 1) * m + j] = beta[j];
    }
    small_eigh(m, T, w, V);
    int imin = 0, imax = 0;
    for (int i = 1; i < m; ++i) {
        if (w[i] < w[imin]) imin = i;
        if (w[i] > w[imax]) imax = i;
    }
    // Gauss quadrature of the spectral density: Ritz values with the squared
    // first components of T's eigenvectors as weights (used to start the
    // chemical-potential search at finite temperature).
    ritz.assign(w.begin(), w.end());
    ritz_w.resize(m);
    for (int i = 0; i < m; ++i) ritz_w[i] = V[i] * V[i];
    const double bk = (m == k) ? beta[k - 1] : 0.0;
    const double rmin = fabs(bk * V[(size_t)(m - 1) * m + imin]);
    const double rmax = fabs(bk * V[(size_t)(m - 1) * m + imax]);
    const double margin = 0.01 * (w[imax] - w[imin]) + 1e-12 * scale;
    const double lo = std::max(h->emin, w[imin] - rmin - margin);
    const double hi = std::min(h->emax, w[imax] + rmax + margin);
    if (!(hi > lo)) return FDM_OK;  // keep the Gershgorin interval
    h->emin = lo;
    h->emax = hi;
    stats.e_min = lo;
    stats.e_max = hi;
    stats.lanczos_steps = m;
    e = launch_set_bounds(r->st, lo, hi, s);
    return e == hipSuccess ? FDM_OK : hip_fail(e, "set_bounds launch");
}

// Certified spectral bounds (Sec. II.C needs bounds that hold).  The
// Lanczos interval c -+ r of refine_bounds comes from a Krylov space, which
// cannot see an eigenvector orthogonal to its start vector.  Every direction
// enters the Frobenius norm, so with A = (Hp - c I) / r and M_k = A^(2^k),
//     max_i |lambda_i(A)|^(2^(k+1)) <= ||M_k||_F^2 = sum_i lambda_i(A)^(2^(k+1)).
// Five squarings (FP16x3 products of the library's kernel, M_k symmetric by
// construction) and the rounding of each bounded: the stored product is
// M_{k-1}^2 + E_k with ||E_k||_2 <= ||E_k||_F <= d_k, so by Weyl's theorem
// rho(M_{k-1})^2 <= rho(M_k) + d_k, and from rho(M_5) <= ||M_5||_F a bound
// b >= rho(A) follows backwards.  The bounds used are c -+ b r (clipped to
// the Gershgorin interval): an eigenvalue the Lanczos run missed widens the
// interval instead of breaking the expansion.  d_k covers the hi/lo
// representation (relative 2^-22 per operand entry, plus 2^-37 absolute in
// the FP16 subnormal range), the FP32 accumulation (24 MFMA roundings per
// 256-deep partial sum, one per fold, and the final stores) and the
// FP32 rounding of A, each doubled.  A power that overflows FP16 (|entries|
// >= 16, i.e. rho(A) far above 1) gives non-finite sums: the Gershgorin
// interval is used then.
int Ctx::certify_bounds(const double *Hp, int64_t ldh, DevState *h) {
    const double glo = stats.gersh_min, ghi = stats.gersh_max;
    const double c = 0.5 * (h->emin + h->emax), rad = 0.5 * (h->emax - h->emin);
    stats.lanczos_min = h->emin;
    stats.lanczos_max = h->emax;
    if (!(rad > 0.0) || (h->emin <= glo && h->emax >= ghi)) return FDM_OK;
    const size_t m = (size_t)r->lay.np * r->lay.ld;
    // two (FP32 matrix, hi/lo companions) slots, carved from the FP64
    // working matrices 1 and 2 (8 bytes per element each), free before X_0
    float *mat[2];
    uint16_t *hl[2];
    for (int i = 0; i < 2; ++i) {
        char *b = (char *)(r->x64 + (size_t)(i + 1) * m);
        mat[i] = (float *)b;
        hl[i] = (uint16_t *)(b + m * sizeof(float));
    }
    int rc = set_params(0.0, 1, 0, 1);  // clears the certificate slots
    if (rc) return rc;
    int np = 0;
    hipError_t e = launch_affine(0, Hp, ldh, 1, mat[0], r->lay.ld, (int)n, (int)r->lay.np,
                                 1.0 / rad, -c / rad, 0, r->st, r->part, &np, s);
    if (e != hipSuccess) return hip_fail(e, "affine launch");
    e = launch_split(P_F16X3, mat[0], hl[0], r->lay.ld, r->lay.np, s);
    if (e != hipSuccess) return hip_fail(e, "split launch");
    rc = decide(D_CERT, np, 4);
    if (rc) return rc;
    constexpr int kSq = 5;
    const int bt = tile_for(P_F16X3);
    for (int k = 1; k <= kSq; ++k) {
        ProdArgs a;
        memset(&a, 0, sizeof(a));
        const int src = (k - 1) & 1, dst = k & 1;
        a.A = a.B = mat[src];
        a.C = mat[dst];
        a.Ahl = a.Bhl = hl[src];
        a.Chl = hl[dst];
        a.ld = r->lay.ld;
        a.n = (int32_t)n;
        a.kext = (int32_t)round_up(n, kKStep);
        set_tiles(a, r, bt, P_F16X3);
        a.coef[0][0] = a.coef[1][0] = 1.0;
        a.partials = r->part;
        e = launch_symprod(P_F16X3, bt, a, s);
        if (e != hipSuccess) return hip_fail(e, "symmetric product launch");
        rc = decide(D_CERT, a.ntiles, 4);
        if (rc) return rc;
    }
    DevState hs;
    rc = read_state(&hs);
    if (rc) return rc;
    const double nn = (double)n, K = (double)round_up(n, kKStep);
    const double cu = 2.0 * (3.0 * ldexp(1.0, -22) + (27.0 + K / 256.0) * ldexp(1.0, -24));
    double F[kSq + 1];
    bool finite = hs.ncert == kSq + 1;
    for (int k = 0; k <= kSq && finite; ++k) {
        F[k] = sqrt(hs.cert[k]);
        finite = std::isfinite(F[k]);
    }
    double b = INFINITY;
    if (finite) {
        b = F[kSq] * (1.0 + 1e-12);
        for (int k = kSq; k >= 1; --k) {
            const double d = cu * F[k - 1] * F[k - 1] + 6e-11 * nn * F[k - 1] + 1e-20 * nn * nn;
            b = sqrt(b + d);
        }
        b += 2.0 * ldexp(1.0, -24) * F[0] + 1e-14;  // FP32 rounding of A
    }
    stats.cert_radius = b;
    double lo = glo, hi = ghi;
    if (std::isfinite(b)) {
        lo = std::max(glo, c - b * rad);
        hi = std::min(ghi, c + b * rad);
        stats.bounds_certified = 1;
    } else {
        stats.bounds_certified = -1;
    }
    h->emin = lo;
    h->emax = hi;
    stats.e_min = lo;
    stats.e_max = hi;
    e = launch_set_bounds(r->st, lo, hi, s);
    return e == hipSuccess ? FDM_OK : hip_fail(e, "set_bounds launch");
}

int Ctx::tight_bounds(const double *Hp, int64_t ldh, DevState *h) {
    int rc = refine_bounds(Hp, ldh, h);
    if (rc) return rc;
    if (stats.lanczos_steps == 0) return FDM_OK;  // Gershgorin kept
    return certify_bounds(Hp, ldh, h);
}

// k Lanczos steps on the projection of Hp - sigma I onto the occupied
// (unocc = 0) or unoccupied (unocc = 1) subspace of the density matrix D.
// Returns the extreme Ritz value (largest for the occupied side, smallest
// for the unoccupied one) and its residual bound |beta_k s_k|.
int Ctx::projected_ritz(const double *Hp, int64_t ldh, const double *D, int64_t ldd, int unocc,
                        double sigma, int k, double *theta, double *resid) {
    double *ab = r->lanczos + 5 * r->lay.np;
    hipError_t e = launch_lanczos_proj(Hp, ldh, D, ldd, (int)n, (int)r->lay.np, k, unocc, sigma,
                                       r->lanczos, ab, s);
    if (e != hipSuccess) return hip_fail(e, "projected lanczos launch");
    std::vector<double> hab(2 * k);
    e = hipMemcpyAsync(hab.data(), ab, 2 * k * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    const double *alpha = hab.data(), *beta = hab.data() + k;
    double scale = 0.0;
    for (int j = 0; j < k; ++j) scale = std::max(scale, fabs(alpha[j]) + fabs(beta[j]));
    int m = k;
    for (int j = 0; j < k - 1; ++j)
        if (!(beta[j] > 1e-13 * scale)) {
            m = j + 1;
            break;
        }
    std::vector<double> T((size_t)m * m, 0.0), w, V;
    for (int j = 0; j < m; ++j) {
        T[(size_t)j * m + j] = alpha[j];
        if (j + 1 < m) T[(size_t)j * m + j + 1] = T[(size_t)(j + 1) * m + j] = beta[j];
    }
    small_eigh(m, T, w, V);
    int ie = 0;
    for (int i = 1; i < m; ++i)
        if (unocc ? w[i] < w[ie] : w[i] > w[ie]) ie = i;
    const double bk = (m == k) ? beta[k - 1] : 0.0;
    *theta = w[ie];
    *resid = fabs(bk * V[(size_t)(m - 1) * m + ie]);
    return FDM_OK;
}

// HOMO / LUMO bounds for a later accelerated solve (an SCF step after this
// one): the HOMO is the largest eigenvalue of Hp on range(D), the LUMO the
// smallest on range(I - D).  Lanczos on D (Hp - e_min) D and on
// (I - D)(Hp - e_max)(I - D) (the shifts keep the extreme eigenvalue on the
// wanted side of the projections' zero eigenvalues) gives Ritz values
// theta with residual bounds r; homo_ub = e_min + theta_max + r and
// lumo_lb = e_max + theta_min - r (40 steps: on the test workloads these bound
// the true HOMO / LUMO and keep 70-100% of the gap; 16-24 steps left one
// LUMO bound above the LUMO).  A Ritz value that has not converged can still
// miss the true extreme by more than r: the accelerated solve that uses the
// bounds guards against that (divergence guard, plain SP2 rerun).
int Ctx::estimate_gap(const double *Hp, int64_t ldh, const double *D, int64_t ldd) {
    stats.homo_ub = stats.lumo_lb = NAN;
    const int k = (int)std::min<int64_t>(40, n);
    if (k < 2) return FDM_OK;
    double th_o = 0.0, r_o = 0.0, th_u = 0.0, r_u = 0.0;
    int rc = projected_ritz(Hp, ldh, D, ldd, 0, stats.e_min, k, &th_o, &r_o);
    if (rc) return rc;
    rc = projected_ritz(Hp, ldh, D, ldd, 1, stats.e_max, k, &th_u, &r_u);
    if (rc) return rc;
    // (plus 1e-6 of the width: D is itself converged only to tol, which
    // moves the Ritz values of its subspaces by about that much)
    const double pad = 1e-6 * (stats.e_max - stats.e_min);
    const double hu = stats.e_min + th_o + r_o + pad;
    const double ll = stats.e_max + th_u - r_u - pad;
    if (std::isfinite(hu) && std::isfinite(ll) && hu < ll) {
        stats.homo_ub = hu;
        stats.lumo_lb = ll;
    }
    return FDM_OK;
}

int Ctx::solve_zero_t(const double *Hp, int64_t ldh, double *D, int64_t ldd, double *E_band) {
    const bool accel = std::isfinite(opt.homo) && std::isfinite(opt.lumo) && opt.lumo > opt.homo;
    int rc = solve_zero_t_once(Hp, ldh, D, ldd, E_band, accel);
    if (rc) return rc;
    if (stats.accelerated == 1 && status != FDM_OK) {
        // the bounds were wrong (a state on the wrong side never settles): plain SP2
        status = FDM_OK;
        rc = solve_zero_t_once(Hp, ldh, D, ldd, E_band, false);
        if (rc) return rc;
        stats.accelerated = -1;
    }
    if (low_cap) {
        // The low-precision phase used all its steps without reaching tau:
        // its rounding noise is above the HOMO-LUMO gap of X, and the
        // subspace it leaves cannot be trusted.  Solve again in FP64.
        const int keep_prec = opt.precision, keep_acc = stats.accelerated;
        opt.precision = P_F64;
        status = FDM_OK;
        rc = solve_zero_t_once(Hp, ldh, D, ldd, E_band, accel && keep_acc == 1);
        opt.precision = keep_prec;
        if (keep_acc == -1) stats.accelerated = -1;
        stats.fallback_fp64 = 1;
    }
    stats.homo_ub = stats.lumo_lb = NAN;
    const int64_t k = (int64_t)llround(n_occ);
    if (rc == FDM_OK && status == FDM_OK && opt.estimate_gap && k > 0 && k < n)
        rc = estimate_gap(Hp, ldh, D, ldd);
    return rc;
}

int Ctx::solve_zero_t_once(const double *Hp, int64_t ldh, double *D, int64_t ldd, double *E_band,
                           bool accel) {
    const int64_t k = (int64_t)llround(n_occ);
    stats.accelerated = 0;
    stats.iters_fp64_first = stats.iters_low = stats.iters_fp64 = stats.mcweeny_steps = 0;
    low_cap = false;
    DevState h;
    int rc = bounds(Hp, ldh, &h);
    if (rc) return rc;
    if (k == 0 || k == n) {
        // D = 0 or I exactly
        hipError_t e = launch_affine(0, Hp, ldh, 0, D, ldd, (int)n, (int)n, 0.0,
                                     k == 0 ? 0.0 : 1.0, 0, r->st, nullptr, nullptr, s);
        if (e != hipSuccess) return hip_fail(e, "affine launch");
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        stats.band_energy = (k == 0) ? 0.0 : h.trH;
        stats.trace = (double)k;
        stats.idempotency = 0.0;
        if (E_band) *E_band = stats.band_energy;
        return FDM_OK;
    }
    if (!(h.emax > h.emin)) {
        set_error("Hp is a multiple of the identity: no gap at n_occ");
        return FDM_ENOCONV;
    }
    if (opt.bounds == 1) {
        rc = tight_bounds(Hp, ldh, &h);
        if (rc) return rc;
    }
    const int prec = opt.precision;
    const int max_iter = opt.max_iter;
    az_coef.clear();
    az_branch.clear();
    az_gap.clear();
    if (accel) {
        const double w = h.emax - h.emin;
        const double l0 = std::min(std::max((h.emax - opt.lumo) / w, 0.0), 1.0);
        const double h0 = std::min(std::max((h.emax - opt.homo) / w, 0.0), 1.0);
        if (l0 < h0) {
            build_az_schedule(l0, h0, 2 * max_iter + 8);
            stats.accelerated = 1;
        }
    }
    const int sched = stats.accelerated == 1 ? 0 : -1;
    rc = set_params(0.0, max_iter, 0, 1);
    if (rc) return rc;
    phase_done(0);
    int np = 0;
    double *x64 = r->x64;
    const size_t m64 = (size_t)r->lay.np * r->lay.ld;
    double *X64[3] = {x64, x64 + m64, x64 + 2 * m64};
    float *X32[2] = {r->x32, r->x32 + m64};

    if (opt.reltr_schedule) {
        // The paper's schedule (Sec. III.A, Sec. IV): SP2 products in the
        // working precision until the relative trace change drops below
        // reltr_switch, then FP64 products until it drops below reltr_stop;
        // the last iterate is D.  RelTr_n = Tr(X_n - X_n^2) / Tr X_n here,
        // since both SP2 branches change the trace by Tr(X - X^2).
        stats.reltr_schedule = 1;
        void *res = nullptr;
        int it = 0;
        if (prec != P_F64) {
            split_prec = prec;
            rc = affine(0, Hp, ldh, 1, X32[0], 0, 0, 1, &np);
            if (rc) return rc;
            rc = decide(D_INIT, np, 4);
            if (rc) return rc;
            rc = sp2_phase(prec, X32[0], X32[1], max_iter, 1 | kRelTrStop, opt.reltr_switch, -1,
                           &res, &it);
            if (rc) return rc;
            stats.iters_low = it;
            phase_done(2);
            if (status) {
                stats.idempotency = r->hm_host->idem;
                return finish(Hp, ldh, res, 1, D, ldd, E_band);
            }
            rc = affine(1, res, r->lay.ld, 0, X64[0], 1.0, 0.0, 0, &np);
        } else {
            rc = affine(0, Hp, ldh, 0, X64[0], 0, 0, 1, &np);
        }
        if (rc) return rc;
        rc = decide(D_INIT, np, 4);
        if (rc) return rc;
        rc = sp2_phase(P_F64, X64[0], X64[1], max_iter, kRelTrStop, opt.reltr_stop, -1, &res, &it);
        if (rc) return rc;
        stats.iters_fp64 = it;
        stats.idempotency = r->hm_host->idem;  // of the iterate before the returned one
        return finish(Hp, ldh, res, 0, D, ldd, E_band);
    }

    if (prec == P_F64) {
        rc = affine(0, Hp, ldh, 0, X64[0], 0, 0, 1, &np);
        if (rc) return rc;
        rc = decide(D_INIT, np, 4);
        if (rc) return rc;
        void *res = nullptr;
        int it = 0;
        rc = sp2_phase(P_F64, X64[0], X64[1], max_iter, 0, 0.0, sched, &res, &it);
        if (rc) return rc;
        phase_done(1);
        stats.iters_fp64 = it;
        stats.idempotency = r->hm_host->idem;
        return finish(Hp, ldh, res, 0, D, ldd, E_band);
    }

    // ---- mixed forms ----
    split_prec = prec;
    int k64 = opt.k64;
    if (k64 < 0) {
        // FP64 steps while the Gershgorin over-estimate of the spectral width
        // keeps the HOMO-LUMO gap of X tiny: ceil(log2(W / W_est)) with
        // W_est from the exact moments (2 sqrt(3) sigma, the width of a
        // uniform spectrum).  Lanczos-tightened bounds are within a few % of
        // the true width, so there only a width above 2 W_est counts
        // (floor): the 20-band N = 4000 matrix (W / W_est = 1.02) reaches
        // the same |dE| (2.2e-10 Ha) with its first step in FP32.
        const double mean = h.trH / (double)n;
        const double var = std::max(h.fro2H / (double)n - mean * mean, 1e-300);
        const double west = 2.0 * sqrt(3.0 * var);
        const double ratio = (h.emax - h.emin) / west;
        const double l2 = ratio > 1.0 ? log2(ratio) : 0.0;
        k64 = (int)(opt.bounds == 1 ? floor(l2) : ceil(l2));
        // Larger N puts more states next to the gap and larger accumulation
        // errors into each product; measured on MI355X with FP32 bulk
        // products and Gershgorin bounds: N = 4000 passes |dE| <= 1e-6 with 5
        // FP64 steps (5.8e-8), N = 30000 needs 20 (4.8e-7; 16 gives 7.9e-6).
        if (n > 4000) k64 += (opt.bounds == 1 ? 1 : 5) * (int)ceil(log2((double)n / 4000.0));
        // The accelerated polynomials open the gap of X more slowly in their
        // first steps than X^2 / 2X - X^2 and much faster later; their FP64
        // steps run until the known gap image h - l of X reaches 1e-3 N/4000
        // (measured on the paper's matrix, FP16x3: at N = 32768, 4 FP64
        // steps left |dE| = 7.4e-7 Ha, 12 steps (gap image 0.01) 1.9e-8).
        if (!az_gap.empty()) {
            const double g = 1e-3 * std::max(1.0, (double)n / 4000.0);
            int j = 0;  // az_gap[j]: gap image after j steps
            while (j + 1 < (int)az_gap.size() && az_gap[j] < g) ++j;
            k64 = std::max(k64, j);
        }
        k64 = std::min(std::max(k64, 0), 24);
    }
    // Leave low precision once every eigenvalue of X is within tau of 0 or 1
    // (tau << 1/4 keeps each on its side).  The low-precision iterates floor
    // near ||X^2 - X||_F ~ 1e-5 (FP32) to 1e-4 (split 16-bit forms) at
    // N = 4000 (measured), and the quadratic step that takes the
    // iterate below tau lands near that floor, so a lower tau only adds
    // low-precision steps; the stagnation guard ends the phase on the floor.
    double tau = opt.tau;
    if (!(tau > 0.0)) tau = std::max(1e-3, 4.0 * unit_roundoff(prec) * sqrt(n_occ));
    void *cur32 = nullptr;
    if (k64 > 0) {
        rc = affine(0, Hp, ldh, 0, X64[0], 0, 0, 1, &np);
        if (rc) return rc;
        rc = decide(D_INIT, np, 4);
        if (rc) return rc;
        void *res = nullptr;
        int it = 0;
        rc = sp2_phase(P_F64, X64[0], X64[1], k64, 2, tau, sched, &res, &it);
        if (rc) return rc;
        phase_done(1);
        stats.iters_fp64_first = it;
        if (r->hm_host->done && r->hm_host->result_iter < k64 && r->hm_host->idem <= tol) {
            stats.idempotency = r->hm_host->idem;
            return finish(Hp, ldh, res, 0, D, ldd, E_band);
        }
        if (status) {  // the FP64 steps stagnated above tol: report the last iterate
            stats.idempotency = r->hm_host->idem;
            return finish(Hp, ldh, res, 0, D, ldd, E_band);
        }
        rc = affine(0, res, r->lay.ld, 1, X32[0], 1.0, 0.0, 0, &np);
        if (rc) return rc;
    } else {
        rc = affine(0, Hp, ldh, 1, X32[0], 0, 0, 1, &np);
        if (rc) return rc;
    }
    rc = decide(D_INIT, np, 4);
    if (rc) return rc;
    int itl = 0;
    rc = sp2_phase(prec, X32[0], X32[1], max_iter, 1, tau,
                   sched < 0 ? -1 : stats.iters_fp64_first, &cur32, &itl);
    if (rc) return rc;
    phase_done(2);
    stats.iters_low = itl;
    if (status) {  // the iterate left [0, 1]: report it
        stats.idempotency = r->hm_host->idem;
        return finish(Hp, ldh, cur32, 1, D, ldd, E_band);
    }
    if (itl >= max_iter && r->hm_host->idem > tau) {
        low_cap = true;
        return FDM_OK;
    }
    rc = affine(1, cur32, r->lay.ld, 0, X64[0], 1.0, 0.0, 0, &np);
    if (rc) return rc;
    rc = decide(D_INIT, np, 4);
    if (rc) return rc;
    double *res64 = nullptr;
    int steps = 0;
    rc = mcweeny_phase(X64[0], X64[1], X64[2], opt.mcweeny_max, &res64, &steps);
    if (rc) return rc;
    stats.mcweeny_steps = steps;
    return finish(Hp, ldh, res64, 0, D, ldd, E_band);
}

void Ctx::phase_done(int i) {
    const auto now = std::chrono::steady_clock::now();
    stats.phase_ms[i] += std::chrono::duration<double, std::milli>(now - tmark).count();
    tmark = now;
}

void Ctx::finalize_timing() {
    if (!opt.timing) return;
    for (const Timed &t : timed) {
        if (!t.real) continue;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r->tev[t.e0], r->tev[t.e1]) == hipSuccess)
            stats.prod_ms[t.prec] += ms;
    }
}

}  // namespace fdm

// ===========================================================================
// C ABI
// ===========================================================================
using namespace fdm;

namespace fdm {

bool sym_product_args_ok(int32_t precision, const double *A, const double *B, const double *E,
                         const double *C, int64_t N, int64_t ld, int32_t tile) {
    return A && B && C && N > 0 && ld >= N && N < 65535 * 64 && precision >= 0 &&
           precision < FDM_NPREC && (tile == 0 || tile == 32 || tile == 64 || tile == 128) &&
           C != A &&
           C != B && !(E && C == E);
}

// The body of fdm_sym_product on a workspace already bound to
// plan_product_layout(N, precision) (zero padding, tile lists in place).
int sym_product_bound(Resources *r, int32_t precision, const double *A, const double *B,
                      const double *E, double *C, int64_t N, int64_t ld, double alpha,
                      double beta, double gamma, double *sums, int32_t tile, hipStream_t s) {
    Ctx c;
    c.r = r;
    c.s = s;
    fdm_options_default(&c.opt);
    c.opt.tile = tile;
    c.n = N;
    const bool lo = precision != P_F64;
    c.split_prec = precision;
    // Operands are packed into zero-padded working matrices of the product's
    // precision (FP64, or the FP32 master of the low-precision forms).
    const Layout &L = r->lay;
    const size_t m = (size_t)L.np * L.ld;
    void *slot[4];
    for (int i = 0; i < 4; ++i)
        slot[i] = lo ? (void *)(r->x32 + i * m) : (void *)(r->x64 + i * m);
    const double *src[3] = {A, B, E};
    void *dst[3] = {slot[0], slot[1], slot[2]};
    if (B == A) dst[1] = slot[0];
    if (E == A) dst[2] = slot[0];
    else if (E == B) dst[2] = dst[1];
    int rc;
    for (int i = 0; i < 3; ++i) {
        if (!src[i]) continue;
        if ((i == 1 && B == A) || (i == 2 && (E == A || E == B))) continue;
        rc = c.affine(0, src[i], ld, lo ? 1 : 0, dst[i], 1.0, 0.0, 0, nullptr);
        if (rc) return rc;
    }
    const double coef[3] = {alpha, beta, gamma};
    rc = c.product(precision, dst[0], dst[1], E ? dst[2] : nullptr, slot[3], coef, nullptr, false,
                   false);
    if (rc) return rc;
    rc = c.decide(D_SUMS, c.last_ntiles, 4);
    if (rc) return rc;
    hipError_t e = launch_copy_out(lo ? 1 : 0, slot[3], L.ld, C, ld, (int)N, s);
    if (e != hipSuccess) return hip_fail(e, "copy-out launch");
    DevState h;
    rc = c.read_state(&h);
    if (rc) return rc;
    if (sums) {
        sums[0] = h.sums[0];
        sums[1] = h.sums[1];
        sums[2] = h.sums[2];
    }
    if (!std::isfinite(h.sums[0]) || !std::isfinite(h.sums[1]) || !std::isfinite(h.sums[2])) {
        set_error("non-finite product (inputs non-finite, or |entries| >= 65504/4096 in an "
                  "FP16 form)");
        return FDM_ENONFINITE;
    }
    return FDM_OK;
}

}  // namespace fdm

extern "C" {

int fdm_options_default(fdm_options *opt) {
    if (!opt) return FDM_EINVAL;
    memset(opt, 0, sizeof(*opt));
    opt->precision = FDM_FP64;
    opt->k64 = -1;
    opt->tau = 0.0;
    opt->max_iter = 100;
    opt->mcweeny_max = 6;
    opt->max_mu_evals = 12;
    opt->fd_extra_depth = 7;
    opt->fd_final_fp64 = 1;
    opt->validate = 0;
    opt->timing = 0;
    opt->tile = 0;
    opt->bounds = 1;
    opt->lanczos_steps = 16;
    opt->homo = NAN;
    opt->lumo = NAN;
    opt->mu_guess = NAN;
    opt->estimate_gap = 0;
    opt->reltr_schedule = 0;
    opt->reltr_switch = 5e-4;
    opt->reltr_stop = 5e-8;
    opt->trfoe = 0;
    opt->trfoe_depth = 0;
    return FDM_OK;
}

size_t fdm_workspace_bytes(int64_t N, double kT, int32_t precision) {
    if (N <= 0 || N > 65535 * 64 || precision < 0 || precision >= FDM_NPREC || !(kT >= 0.0))
        return 0;
    return plan_layout(N, kT > 0.0, precision).bytes;
}

const char *fdm_strerror(int code) {
    switch (code) {
        case FDM_OK: return "success";
        case FDM_EINVAL: return "invalid argument";
        case FDM_ENOMEM: return "out of device memory or above the budget";
        case FDM_ENOCONV: return "iteration did not converge";
        case FDM_EHIP: return "HIP runtime error";
        case FDM_ENONFINITE: return "input holds NaN or Inf";
        default: return "unknown status";
    }
}

const char *fdm_last_error(void) { return last_error(); }

int fermi_dm_solve(const double *Hp, int64_t N, int64_t ldh, double n_occ, double kT, double tol,
                   double *D, int64_t ldd, double *E_band, const fdm_options *opt_in,
                   fdm_stats *stats_out, void *stream) {
    return fdm::solve_impl(Hp, N, ldh, n_occ, kT, tol, D, ldd, E_band, opt_in, stats_out,
                           (hipStream_t)stream, nullptr);
}

}  // extern "C"

namespace fdm {

int solve_impl(const double *Hp, int64_t N, int64_t ldh, double n_occ, double kT, double tol,
               double *D, int64_t ldd, double *E_band, const fdm_options *opt_in,
               fdm_stats *stats_out, hipStream_t stream, TickGroup *group) {
    const auto t0 = std::chrono::steady_clock::now();
    set_error("");
    fdm_options opt;
    if (opt_in)
        opt = *opt_in;
    else
        fdm_options_default(&opt);
    if (!Hp || !D || N <= 0 || N >= 65535 * 64 || ldh < N || ldd < N || !(tol > 0.0) ||
        !(kT >= 0.0) || !std::isfinite(kT) || opt.precision < 0 || opt.precision >= FDM_NPREC ||
        opt.max_iter <= 0 ||
        (opt.tile != 0 && opt.tile != 32 && opt.tile != 64 && opt.tile != 128) ||
        opt.bounds < 0 || opt.bounds > 1 || opt.trfoe_depth < 0 ||
        (opt.reltr_schedule && !(opt.reltr_switch > 0.0 && opt.reltr_stop > 0.0))) {
        set_error("invalid argument");
        return FDM_EINVAL;
    }
    if ((const void *)Hp == (const void *)D) {
        set_error("D may not alias Hp");
        return FDM_EINVAL;
    }
    if (kT == 0.0) {
        if (!(n_occ >= 0.0 && n_occ <= (double)N) || fabs(n_occ - llround(n_occ)) > 1e-9) {
            set_error("zero temperature needs an integer n_occ in [0, N]");
            return FDM_EINVAL;
        }
    } else if (!(n_occ > 0.0 && n_occ < (double)N)) {
        set_error("finite temperature needs 0 < n_occ < N");
        return FDM_EINVAL;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    Resources *r = thread_resources(dev);
    if (!r) return FDM_EHIP;
    Ctx c;
    c.r = r;
    c.s = stream;
    c.opt = opt;
    c.n = N;
    c.n_occ = n_occ;
    c.tol = tol;
    c.kT = kT;
    if (group) {
        c.group = group;
        c.member.ev = r->ev;
        c.member.entry = r->entry;
        c.opt.timing = 0;
    }
    memset(&c.stats, 0, sizeof(c.stats));
    c.stats.homo_ub = c.stats.lumo_lb = NAN;
    c.stats.lanczos_min = c.stats.lanczos_max = c.stats.cert_radius = NAN;
    c.tmark = t0;
    const Layout L = plan_layout(N, kT > 0.0, opt.precision);
    int rc = r->bind(L, opt.workspace, opt.workspace_bytes, c.s);
    if (rc == FDM_OK && opt.validate) rc = c.validate_symmetric(Hp, ldh);
    if (rc == FDM_OK) rc = (kT == 0.0) ? c.solve_zero_t(Hp, ldh, D, ldd, E_band)
                                       : c.solve_finite_t(Hp, ldh, D, ldd, E_band);
    if (rc == FDM_OK && c.status) rc = c.status;
    if (rc == FDM_OK || rc == FDM_ENOCONV) {
        hipError_t e2 = hipStreamSynchronize(c.s);
        if (e2 != hipSuccess) rc = hip_fail(e2, "hipStreamSynchronize");
        c.finalize_timing();
        c.phase_done(3);
    }
    c.stats.status = rc;
    c.stats.tile = c.used_tile;
    c.stats.tick_steps = c.member.steps;
    c.stats.tick_shared = c.member.shared;
    c.stats.ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats_out) *stats_out = c.stats;
    if (rc == FDM_ENOCONV && fdm_last_error()[0] == 0) set_error("iteration cap or stagnation");
    return rc;
}

}  // namespace fdm

extern "C" {

int fdm_gershgorin(const double *H, int64_t N, int64_t ldh, double *out, int32_t *nonfinite,
                   void *stream) {
    set_error("");
    if (!H || !out || N <= 0 || ldh < N) return FDM_EINVAL;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    Resources *r = thread_resources(dev);
    if (!r) return FDM_EHIP;
    Ctx c;
    c.r = r;
    c.s = (hipStream_t)stream;
    fdm_options_default(&c.opt);
    c.n = N;
    int rc = r->bind(plan_layout(N, false, P_F64), nullptr, 0, c.s);
    if (rc) return rc;
    e = launch_gershgorin(H, ldh, (int)N, r->part, r->st, c.s);
    if (e != hipSuccess) return hip_fail(e, "gershgorin launch");
    DevState h;
    rc = c.read_state(&h);
    if (rc) return rc;
    out[0] = h.emin;
    out[1] = h.emax;
    out[2] = h.trH;
    out[3] = h.fro2H;
    if (nonfinite) *nonfinite = h.nonfinite;
    return FDM_OK;
}

int fdm_sym_product(int32_t precision, const double *A, const double *B, const double *E,
                    double *C, int64_t N, int64_t ld, double alpha, double beta, double gamma,
                    double *sums, int32_t tile, void *stream) {
    set_error("");
    if (!sym_product_args_ok(precision, A, B, E, C, N, ld, tile)) return FDM_EINVAL;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    Resources *r = thread_resources(dev);
    if (!r) return FDM_EHIP;
    int rc = r->bind(plan_product_layout(N, precision), nullptr, 0, (hipStream_t)stream);
    if (rc) return rc;
    return sym_product_bound(r, precision, A, B, E, C, N, ld, alpha, beta, gamma, sums, tile,
                             (hipStream_t)stream);
}

int fdm_band_energy(const double *H, int64_t ldh, const double *D, int64_t ldd, int64_t N,
                    double *out, void *stream) {
    set_error("");
    if (!H || !D || !out || N <= 0 || ldh < N || ldd < N) return FDM_EINVAL;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    Resources *r = thread_resources(dev);
    if (!r) return FDM_EHIP;
    Ctx c;
    c.r = r;
    c.s = (hipStream_t)stream;
    fdm_options_default(&c.opt);
    c.n = N;
    int rc = r->bind(plan_layout(N, false, P_F64), nullptr, 0, c.s);
    if (rc) return rc;
    e = launch_energy(H, ldh, D, ldd, 0, (int)N, r->part, r->st, c.s);
    if (e != hipSuccess) return hip_fail(e, "energy launch");
    DevState h;
    rc = c.read_state(&h);
    if (rc) return rc;
    out[0] = h.sums[0];
    out[1] = h.sums[1];
    return FDM_OK;
}

}  // extern "C"
