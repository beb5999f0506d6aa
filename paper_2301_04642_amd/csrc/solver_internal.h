// Host-side solver structures (driver internals, not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <chrono>
#include <deque>
#include <functional>
#include <vector>

#include "fdm_internal.h"

namespace fdm {

constexpr int kMaxLanczos = 64;

// Carving of one workspace allocation: n64 FP64 and n32 FP32 zero-padded
// np x ld working matrices, per-tile partial sums, two tile lists and the
// device state.
struct Layout {
    int64_t n = 0, np = 0, ld = 0;
    int n64 = 0, n32 = 0;
    size_t off64 = 0, off32 = 0, off_part = 0, off_tiles64 = 0, off_tiles128 = 0, off_state = 0;
    size_t off_tiles32 = 0;  // 32-wide tile list (small N only, else empty)
    size_t off_tiles128e = 0; // 128-wide list with edge blocks (edge_blocks(n) only)
    size_t off_lanczos = 0;  // 5 vectors of np doubles + alpha/beta (2 x kMaxLanczos)
    size_t off16 = 0;        // hi/lo 16-bit companions of the FP32 buffers
    size_t bytes = 0;
    int ntiles64 = 0, ntiles128 = 0, ntiles32 = 0, ntiles128e = 0;
    int64_t part_cap = 0;
};
Layout plan_layout(int64_t n, bool finite, int prec);
Layout plan_product_layout(int64_t n, int prec);

// Events of the steps in flight (one ring per host thread and device).
constexpr int kEvRing = 8;

struct TickGroup;

// Per host thread and device: the cached workspace, the mapped host mirror
// of the device state, and events.
struct Resources {
    int device = -1;
    char *base = nullptr;
    size_t cap = 0;
    bool owned = false;
    char *bound_mem = nullptr;
    int64_t bound_key = -1, bound_ld = -1;
    Layout lay;
    double *x64 = nullptr;
    float *x32 = nullptr;
    uint16_t *x16 = nullptr;
    double *part = nullptr;
    uint32_t *tiles64 = nullptr, *tiles128 = nullptr, *tiles32 = nullptr;
    uint32_t *tiles128e = nullptr;  // null: no edge-block list
    double *lanczos = nullptr;
    DevState *st = nullptr;
    HostMirror *hm_host = nullptr, *hm_dev = nullptr;
    DevState *st_pinned = nullptr;
    DevState st_fallback;
    hipEvent_t ev[kEvRing] = {};
    hipEvent_t entry = nullptr;  // joins a tick group (serving)
    std::vector<hipEvent_t> tev;

    ~Resources();
    int init(int dev);
    int bind(const Layout &L, void *user_mem, size_t user_bytes, hipStream_t s);
    void view(const Layout &L, char *mem);  // points the buffers into mem (no other effect)
    hipEvent_t timing_event(size_t i);
    DevState *st_host();
};
Resources *thread_resources(int dev);

bool sym_product_args_ok(int32_t precision, const double *A, const double *B, const double *E,
                         const double *C, int64_t N, int64_t ld, int32_t tile);
int sym_product_bound(Resources *r, int32_t precision, const double *A, const double *B,
                      const double *E, double *C, int64_t N, int64_t ld, double alpha,
                      double beta, double gamma, double *sums, int32_t tile, hipStream_t s);

// fermi_dm_solve with an optional serving tick group (the server's
// executors pass theirs; group == nullptr launches on `stream` directly).
int solve_impl(const double *Hp, int64_t N, int64_t ldh, double n_occ, double kT, double tol,
               double *D, int64_t ldd, double *E_band, const fdm_options *opt_in,
               fdm_stats *stats_out, hipStream_t stream, TickGroup *group);

int hip_fail(hipError_t e, const char *what);
const char *last_error();

struct Timed {
    int prec;
    size_t e0, e1;
    bool real;
};

// ---- serving tick (tick.cpp) -----------------------------------------------
// One step of a solve's hot loop as recorded for a tick group instead of
// launched: products, decisions and other launches, in order.
struct StepOp {
    enum Kind { PRODUCT, DECIDE, CUSTOM } kind;
    int prec = 0, bt = 0;
    bool direct = false;
    ProdArgs a;
    DecideJob d;
    std::function<hipError_t(hipStream_t)> custom;
};
struct Step {
    std::vector<StepOp> ops;
};

// A solve taking part in a tick group (one per solve context).
struct TickMember {
    hipEvent_t *ev = nullptr;    // ring of kEvRing events: ev[seq % kEvRing] follows step seq
    hipEvent_t entry = nullptr;  // recorded on the member's stream when it joins
    bool entered = false;        // the group stream already waits on `entry`
    std::deque<std::pair<int, Step>> posted;  // steps not yet launched, in order
    int launched = -1;           // last step launched
    int taken = 0;               // steps the ticker is launching right now
    int error = 0;
    int steps = 0, shared = 0;   // steps launched; of them, in a tick with another solve's
};

// Runs the hot-loop steps of several solves together: each tick takes the
// next posted step of every member and launches their products as grouped
// products (one launch per precision, tile edge and staging path) and their
// decisions as one grouped decision, on the group's own stream.
struct TickGroup;
TickGroup *tick_group_create(int device);
void tick_group_destroy(TickGroup *g);
// Joins g: the group stream will wait for everything enqueued on s so far.
int tick_join(TickGroup *g, TickMember *m, hipStream_t s);
void tick_post(TickGroup *g, TickMember *m, int seq, Step &&st);
// Waits until step seq has run on the device.
int tick_wait(TickGroup *g, TickMember *m, int seq);
// Drops the member's unlaunched steps, waits for its launched ones to finish
// and leaves the group.
int tick_leave(TickGroup *g, TickMember *m);

// One call's context.
struct Ctx {
    Resources *r = nullptr;
    hipStream_t s = nullptr;
    fdm_options opt;
    fdm_stats stats;
    int64_t n = 0;
    double n_occ = 0.0, tol = 0.0, kT = 0.0;
    int status = 0;
    int split_prec = -1;  // split precision whose operand companions are kept
    bool low_cap = false; // the low-precision SP2 phase ran out of steps above tau
    int last_ntiles = 0;
    int used_tile = 0;
    std::vector<int> phase_launches;
    std::vector<double> ritz, ritz_w;  // Lanczos Ritz values and Gauss weights of Hp
    // accelerated zero-T expansion: coefficients (a, b, c) of a X^2 + b X + c I
    // for SP2 step k at az_coef[3k..3k+2], and the form (1 = squaring form)
    std::vector<double> az_coef;
    std::vector<uint8_t> az_branch;
    std::vector<double> az_gap;  // h - l before the first and after each accelerated step
    std::vector<Timed> timed;
    std::chrono::steady_clock::time_point tmark = std::chrono::steady_clock::now();
    // serving tick: when group is set, the hot loops' launches are recorded
    // into *cap (a step) and run by the group instead of on s
    TickGroup *group = nullptr;
    TickMember member;
    Step *cap = nullptr;
    Step stream_step;          // the step being recorded in stream capture
    bool cap_stream = false;   // post a step at every product (finite-T evaluations)
    int cap_seq = 0;
    int begin_stream_capture();
    int end_stream_capture();

    int tile_for(int prec) const;
    int product(int prec, const void *A, const void *B, const void *E, void *C, const double c0[3],
                const double c1[3], bool sel, bool done_guard);
    void close_phase(int executed);
    int decide(int mode, int count, int stride);
    int set_params(double tau, int max_iter, int switch_mode, int reset_all);
    int affine(int in_f32, const void *in, int64_t ldi, int out_f32, void *out, double a,
               double b, int zt, int *nparts);
    int run_loop(int max_steps, const std::function<int(int)> &enqueue);
    int run_loop_grouped(int max_steps, const std::function<int(int)> &enqueue);
    int sp2_phase(int prec, void *b0, void *b1, int max_iter, int switch_mode, double tau,
                  int sched_off, void **result, int *iters);
    void build_az_schedule(double l0, double h0, int steps);
    int mcweeny_phase(double *x0, double *t, double *x1, int max_steps, double **result,
                      int *steps);
    int read_state(DevState *out);
    int bounds(const double *Hp, int64_t ldh, DevState *h);
    int refine_bounds(const double *Hp, int64_t ldh, DevState *h);
    int certify_bounds(const double *Hp, int64_t ldh, DevState *h);
    int tight_bounds(const double *Hp, int64_t ldh, DevState *h);
    int estimate_gap(const double *Hp, int64_t ldh, const double *D, int64_t ldd);
    int projected_ritz(const double *Hp, int64_t ldh, const double *D, int64_t ldd, int unocc,
                       double sigma, int k, double *theta, double *resid);
    int finish(const double *Hp, int64_t ldh, const void *dm, int dm_f32, double *D, int64_t ldd,
               double *E_band);
    int validate_symmetric(const double *Hp, int64_t ldh);
    int solve_zero_t(const double *Hp, int64_t ldh, double *D, int64_t ldd, double *E_band);
    int solve_zero_t_once(const double *Hp, int64_t ldh, double *D, int64_t ldd, double *E_band,
                          bool accel);
    int canonical_correction(void *dm, double tr, double trdd, double *mu, void **out);
    int solve_finite_t(const double *Hp, int64_t ldh, double *D, int64_t ldd, double *E_band);
    int fermi_operator(const double *Hp, int64_t ldh, double mu, int depth, int prec,
                       void **result, int *result_f32, double *trace, double *trace_dd);
    void finalize_timing();
    void phase_done(int i);  // adds the host time since the last mark to stats.phase_ms[i]
    int solve_trfoe(const double *Hp, int64_t ldh, double *D, int64_t ldd, double *E_band);
};

}  // namespace fdm
