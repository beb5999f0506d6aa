/*
 * fermidm.h -- C ABI of the MI355X (gfx950) density-matrix library.
 *
 * The library turns a dense symmetric projected Hamiltonian Hp (N x N) into
 * the density matrix D and the band energy Tr(Hp D) without diagonalising
 * Hp, by recursive Fermi-operator expansion (Khadatkar & Motamarri,
 * arXiv 2301.04642):
 *
 *  - zero temperature (Sec. II.A, D = theta(mu I - Hp)): second-order
 *    projection (SP2) steps X <- X^2 or X <- 2X - X^2, the branch chosen from
 *    traces (Sec. II.B.1, Eq. (1); Tr X^2 = ||X||_F^2 as in Sec. III.B),
 *    started from Gershgorin spectral bounds (Sec. II.C); or, given bounds
 *    on the HOMO and LUMO eigenvalues, their shifted and scaled forms
 *    (A-Z-RFOE, Sec. II.B.2);
 *  - finite temperature (Sec. II.A, D = [exp(beta(Hp - mu I)) + I]^-1): a
 *    doubling recursion of projection maps (Sec. II.B.3, Eq. (2)) that
 *    reproduces the Fermi operator, with mu fixed by Tr D = N_occ;
 *  - mixed precision (Sec. III.A): the bulk of the products in a lower
 *    precision, traces, branch decisions and bounds in FP64, and FP64
 *    refinement at the end.
 *
 * Conventions for every entry point:
 *  - Matrices are float64, row-major, with a leading dimension (in elements)
 *    ld >= N.  Pointers marked "device" must be device memory of the
 *    current HIP device; pointers marked "host" are host memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it; every call returns only when its results are
 *    ready (host outputs written, device outputs complete on `stream`).
 *  - The caller owns every buffer it passes.  The library owns its
 *    workspace (cached per host thread and device) unless the caller passes
 *    one in fdm_options.
 *  - Calls return FDM_OK (0) or a negative status; they never abort.  The
 *    text of the last error of the calling thread is fdm_last_error().
 *  - One solve per stream at a time; calls on different streams from
 *    different host threads are independent.
 *  - Environment: FDM_PROGRESS=k makes a solve print "[fdm] n=N step s
 *    done" to stderr after every k-th completed step of each phase (for
 *    solves that run for minutes); unset or 0, the library prints nothing.
 */
#ifndef FERMIDM_H
#define FERMIDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define FDM_OK 0
#define FDM_EINVAL (-1)     /* bad N, ld, n_occ, kT, tol, precision or a null pointer */
#define FDM_ENOMEM (-2)     /* device allocation failed, or request above a budget    */
#define FDM_ENOCONV (-3)    /* iteration cap or stagnation: D holds the last iterate   */
#define FDM_EHIP (-4)       /* a HIP runtime error; see fdm_last_error()               */
#define FDM_ENONFINITE (-5) /* Hp holds NaN or Inf, or a product overflowed            */

/* ---- precision of the bulk products ------------------------------------ */
#define FDM_FP64 0    /* every product in FP64 MFMA (the plain method)                     */
#define FDM_FP32 1    /* FP32 MFMA, FP32 master iterate                                    */
#define FDM_FP16X3 2  /* X = hi + lo split into two FP16 halves, 3 FP16 MFMA products,
                         FP32 accumulation (about FP32 accuracy at FP16 MFMA rate)         */
#define FDM_BF16X3 3  /* as FP16X3 with BF16 halves                                        */
#define FDM_BF16 4    /* one BF16 MFMA product, FP32 accumulation (reported, not gated)    */
#define FDM_FP16 5    /* one FP16 MFMA product, FP32 accumulation (reported, not gated)    */
#define FDM_NPREC 6

/* Options.  Fill with fdm_options_default() and change what you need. */
typedef struct fdm_options {
    int32_t precision;      /* FDM_FP64 .. FDM_FP16 (default FDM_FP64)                         */
    int32_t k64;            /* zero-T mixed forms: SP2 steps done in FP64 before the low-
                               precision phase; -1 = automatic (default)                       */
    double tau;             /* zero-T mixed forms: leave the low-precision phase once
                               ||X^2 - X||_F <= tau; <= 0 = automatic (default)               */
    int32_t max_iter;       /* SP2 products per phase (default 100)                            */
    int32_t mcweeny_max;    /* FP64 McWeeny steps in the mixed forms (default 6)               */
    int32_t max_mu_evals;   /* finite T: Fermi-operator evaluations in the mu search (12)      */
    int32_t fd_extra_depth; /* finite T: doubling depth = ceil(log2(beta*R)) + this (7)        */
    int32_t fd_final_fp64;  /* finite T, low precision: finish with one FP64 evaluation (1)    */
    int32_t validate;       /* 1: reject an Hp that is not symmetric to 1e-12 relative (0)     */
    int32_t timing;         /* 1: time every product launch with HIP events (0)                */
    int32_t tile;           /* product tile edge: 0 = automatic, or 32 (N <= 2048) / 64 / 128   */
    int32_t bounds;         /* spectral bounds (Sec. II.C): 0 = Gershgorin discs; 1 (default)
                               = a Lanczos estimate of the extreme eigenvalues (Ritz values
                               widened by their residual bounds and 1% of the width), interval
                               c -+ r, then certified: with A = (Hp - c I) / r, the powers
                               A^2, A^4, ..., A^32 (five FP16x3 products, the rounding of
                               each bounded) give b >= max |lambda(A)| from ||A^32||_F, and
                               c -+ b r is used (so an eigenvalue the estimate missed widens
                               the interval; b <= N^(1/64) max |lambda(A)|).  Powers that
                               overflow FP16 (max |lambda(A)| well above 1) fall back to the
                               Gershgorin interval (stats.bounds_certified = -1).  Never
                               outside the Gershgorin interval.                              */
    int32_t lanczos_steps;  /* Lanczos steps for bounds = 1 (default 16, at most 64)           */
    int32_t estimate_gap;   /* zero T: 1 = after the solve, estimate bounds on the HOMO and LUMO
                               eigenvalues for a later accelerated solve (stats homo_ub /
                               lumo_lb; 40 projected Lanczos steps, 4 x 40 matrix-vector
                               products with Hp and D) (0)                                     */
    double homo, lumo;      /* zero T: when homo < lumo, the accelerated expansion (A-Z-RFOE,
                               Sec. II.B.2): shifted and scaled SP2 polynomials chosen from
                               these bounds, homo >= the highest occupied eigenvalue and
                               lumo <= the lowest unoccupied one (e.g. from the previous SCF
                               step).  Bounds that turn out wrong make the expansion miss
                               n_occ or stall; the solve then repeats as plain SP2.  NaN
                               (default) = plain SP2                                           */
    double mu_guess;        /* finite T: start of the mu search (e.g. the previous SCF step's mu);
                               the mixed forms then skip their low-precision search and start
                               with the FP64 evaluation.  NaN (default) = the guess from the
                               moments of Hp                                                   */
    void *workspace;        /* optional caller-owned device memory of workspace_bytes, 256-byte
                               aligned (FDM_EINVAL otherwise)                                   */
    size_t workspace_bytes; /* at least fdm_workspace_bytes(N, kT, precision)                  */
    int32_t reltr_schedule; /* zero T: 1 = the paper's schedule (Sec. III.A, Sec. IV): SP2 in
                               `precision` until RelTr <= reltr_switch, then FP64 SP2 until
                               RelTr <= reltr_stop, where RelTr = |Tr X_n - Tr X_{n-1}| /
                               |Tr X_{n-1}|; D is the last iterate (no idempotency stop, no
                               McWeeny steps).  `tol` is not used (0)                           */
    int32_t trfoe;          /* finite T: 1 = the truncated zero-temperature expansion of Sec.
                               II.B.3, Eq. (2) (T-RFOE): `trfoe_depth` SP2 steps with trace-
                               steered branches from X_0 and no mu search; D = X_m is a smeared
                               step, not the Fermi operator (0)                               */
    double reltr_switch;    /* 5e-4 */
    double reltr_stop;      /* 5e-8 */
    int32_t trfoe_depth;    /* 0 = from beta: the smallest m with (sqrt(5) - 1)^m >= beta (e_max -
                               e_min) / 4, i.e. the slope of m SP2 steps on the unstable
                               2-cycle of X^2 / 2X - X^2 (derivative sqrt(5) - 1 per step)
                               matched to the Fermi function's slope beta / 4 at mu           */
    int32_t reserved0;
} fdm_options;

/* Per-solve report (host memory, filled by fermi_dm_solve when non-NULL). */
typedef struct fdm_stats {
    int32_t status;
    int32_t iters_fp64_first;   /* zero T: FP64 SP2 products before the low-precision phase   */
    int32_t iters_low;          /* zero T: low-precision SP2 products                          */
    int32_t iters_fp64;         /* zero T, FDM_FP64: SP2 products                              */
    int32_t mcweeny_steps;      /* zero T mixed: FP64 McWeeny steps                            */
    int32_t mu_evals;           /* finite T: Fermi-operator evaluations                        */
    int32_t depth;              /* finite T: doubling steps per evaluation                     */
    int32_t tile;               /* tile edge of the last product launch (64 or 128; each
                                   precision picks its own from N)                             */
    int32_t products[FDM_NPREC];    /* product launches that ran, per precision                */
    uint64_t branch_bits[4];    /* SP2 branch of product k (bit k; 1 = X^2), k < 256           */
    double e_min, e_max;        /* spectral bounds of Hp used by the expansion                  */
    double mu;                  /* finite T: chemical potential of D                           */
    double idempotency;         /* zero T: ||D^2 - D||_F as measured by the last product       */
    double trace;               /* Tr D                                                         */
    double band_energy;         /* Tr(Hp D)                                                     */
    double ms_total;            /* wall time of the call (host clock)                          */
    double prod_ms[FDM_NPREC];  /* summed duration of product launches (timing = 1)            */
    double flops[FDM_NPREC];    /* algorithmic flops of the products that ran: N^2 (N+1) each
                                   (3x for the split forms, which run three products)          */
    double gersh_min, gersh_max;    /* Gershgorin bounds (e_min / e_max hold the bounds used)  */
    int32_t lanczos_steps;      /* Lanczos steps run for the bounds (0 with bounds = 0)        */
    int32_t accelerated;        /* zero T: 1 = the accelerated expansion gave D; -1 = it was
                                   tried and missed, and plain SP2 gave D; 0 = plain SP2       */
    double mcweeny_idem[4];     /* zero-T mixed: ||X^2 - X||_F at each FP64 McWeeny check      */
    double mcweeny_trace_err[4];/* zero-T mixed: |Tr X - n_occ| at each FP64 McWeeny check     */
    double mu_hist[16];         /* finite T: mu of the first 16 Fermi-operator evaluations      */
    double mu_trace_err[16];    /* finite T: Tr D(mu) - n_occ at those evaluations (their own   */
                                /*   precision); mu_evals says how many entries are valid       */
    int32_t fallback_fp64;      /* zero T mixed: 1 = the low-precision phase ran out of steps
                                   without reaching tau (rounding noise above the gap of X), and
                                   the solve was repeated in FP64                              */
    int32_t reserved2;
    double homo_ub, lumo_lb;    /* zero T with estimate_gap = 1: estimated bounds on the HOMO
                                   and LUMO eigenvalues (Ritz values of Hp on the occupied and
                                   unoccupied subspaces of D, widened by their residual
                                   bounds) to pass as homo / lumo to a later solve; NaN when
                                   not asked for or when they do not separate                 */
    double rel_trace;           /* zero T: RelTr = |Tr X_n - Tr X_{n-1}| / |Tr X_{n-1}| of the
                                   last SP2 product (the paper's convergence measure, Sec.
                                   III.A)                                                     */
    double idem_tail[8];        /* ||X^2 - X||_F measured by the last idem_tail_len (<= 8) SP2
                                   or McWeeny products of the solve, oldest first             */
    int32_t idem_tail_len;
    int32_t bounds_certified;   /* 1 = the widened Lanczos bounds passed the certificate (see
                                   fdm_options.bounds); 0 = Gershgorin bounds (bounds = 0, or
                                   the widened interval was not narrower); -1 = the
                                   certificate failed and the Gershgorin bounds were used      */
    double lanczos_min, lanczos_max;  /* bounds = 1: the Lanczos estimate before widening     */
    double cert_radius;         /* bounds = 1: the certified bound on max |lambda(A)| (<= 1 when
                                   the certificate passed)                                    */
    double phase_ms[4];         /* host wall time of: bounds; the first expansion phase (FP64
                                   SP2, FP64-first SP2 steps, or the mu search in `precision`);
                                   the low-precision SP2 phase (zero T) or the FP64 mu
                                   evaluations (finite T); refinement and output (McWeeny,
                                   canonical correction, energy, copy-out)                    */
    int32_t trfoe_depth;        /* finite T with trfoe = 1: SP2 steps of the truncated expansion */
    int32_t reltr_schedule;     /* zero T: 1 when the paper's RelTr schedule produced D        */
    int32_t tick_steps;         /* served with grouped ticks: hot-loop steps of this solve that
                                   ran in ticks (0 outside a server)                           */
    int32_t tick_shared;        /* of them, steps that shared their tick (grouped product and
                                   decision launches) with another request's step              */
} fdm_stats;

/* Fills *opt with the defaults listed above.  Returns FDM_EINVAL if opt is NULL. */
int fdm_options_default(fdm_options *opt);

/* Device bytes of workspace a solve of size N needs (kT > 0 selects the
 * finite-temperature solver).  Returns 0 for invalid arguments. */
size_t fdm_workspace_bytes(int64_t N, double kT, int32_t precision);

/*
 * fermi_dm_solve -- density matrix of Hp.
 *
 *  Hp     device, N x N, leading dimension ldh >= N, symmetric (read only; the
 *         full matrix is read).
 *  n_occ  kT == 0: the number of occupied states, an integer in [0, N];
 *         kT >  0: the electron count Tr D, real in (0, N).
 *  kT     electronic temperature in Hartree (k_B T_e; beta = 1/kT).  0 selects
 *         the zero-temperature projector.
 *  tol    kT == 0: stop when ||X^2 - X||_F <= tol and |Tr X - n_occ| <= tol;
 *         kT > 0: stop the mu
 *         search when |Tr D - n_occ| <= tol or the Newton step in mu is below
 *         1e-3 kT (a second-order correction of D in mu follows).  Must be > 0.
 *  D      device, N x N, leading dimension ldd >= N: receives D (full,
 *         symmetric).  May not alias Hp.
 *  E_band host: receives Tr(Hp D) (nullable).
 *  opt    nullable (defaults).     stats  host, nullable.
 *
 * Special cases: n_occ == 0 gives D = 0; n_occ == N at zero temperature
 * gives D = I.  Returns FDM_ENONFINITE when Hp holds NaN/Inf, FDM_ENOCONV when
 * the iteration cap is reached or the iteration stagnates (D then holds the
 * last iterate and stats are filled).
 */
int fermi_dm_solve(const double *Hp, int64_t N, int64_t ldh, double n_occ, double kT,
                   double tol, double *D, int64_t ldd, double *E_band,
                   const fdm_options *opt, fdm_stats *stats, void *stream);

/* Text for a status code (static storage). */
const char *fdm_strerror(int code);

/* Text of the calling thread's last error ("" if none). */
const char *fdm_last_error(void);

/* ---- single steps of the method (for tests and for composing solvers) -- */

/*
 * fdm_gershgorin -- spectral bounds of Hp by Gershgorin discs (Sec. II.C
 * needs bounds of the spectrum before the expansion; the paper names no
 * method): e_min = min_i (H_ii - r_i), e_max = max_i (H_ii + r_i),
 * r_i = sum_{j != i} |H_ij|.
 *  H       device, N x N, leading dimension ldh.
 *  out     host double[4]: e_min, e_max, Tr H, ||H||_F^2.
 *  nonfinite host int: set to the number of rows holding NaN/Inf (nullable).
 */
int fdm_gershgorin(const double *H, int64_t N, int64_t ldh, double *out, int32_t *nonfinite,
                   void *stream);

/*
 * fdm_sym_product -- one product of two commuting symmetric matrices with the
 * fused epilogue of the hot loop (Sec. II.B.1, Eq. (1); Sec. III.B):
 *
 *     C = alpha * (A B) + beta * E + gamma * I
 *
 * computed on the upper-triangular tiles only and mirrored, so C is exactly
 * symmetric.  A B is formed in `precision` (the FP16/BF16 forms round A and B
 * as described for FDM_FP16X3 .. FDM_FP16; the FP16 forms scale by 2^12 and
 * need |entries| < 65504 / 2^12 = 15.99, beyond which the scaled value
 * overflows FP16).  The epilogue and the partial sums run in FP64.  Returns
 * FDM_ENONFINITE (C then holds Inf/NaN) when a partial sum is not finite.
 *  A, B, E  device, N x N float64, leading dimension ld (E nullable = 0).
 *  C        device, N x N float64, leading dimension ld; may not alias A/B/E.
 *  sums     host double[3] (nullable): Tr C, ||C||_F^2, ||A B - E||_F^2.
 *  tile     0 = automatic, or 32 (N <= 2048; 64 above) / 64 / 128.
 * A and B are expected to commute (for X^2, A == B); only their product's
 * upper triangle is formed.
 */
int fdm_sym_product(int32_t precision, const double *A, const double *B, const double *E,
                    double *C, int64_t N, int64_t ld, double alpha, double beta,
                    double gamma, double *sums, int32_t tile, void *stream);

/*
 * fdm_sym_product_noalloc -- fdm_sym_product for callers that cannot
 * allocate device memory (code under stream capture, serving loops that
 * forbid hipMalloc).  Same arguments, kernels, results and errors as
 * fdm_sym_product; it allocates no device or pinned host memory.  Its
 * workspace is a fixed 64 MiB device array inside the library (one per GPU,
 * held until the process ends), which limits N to 1408: larger N returns
 * FDM_EINVAL with a message.  Every call on one GPU uses that GPU's array and
 * overwrites the previous call's contents (the call clears what must start at
 * zero), so calls that overlap on one GPU -- two streams or two host threads
 * at once -- race and must be serialised by the caller.
 */
int fdm_sym_product_noalloc(int32_t precision, const double *A, const double *B, const double *E,
                            double *C, int64_t N, int64_t ld, double alpha, double beta,
                            double gamma, double *sums, int32_t tile, void *stream);

/*
 * fdm_band_energy -- Tr(H D) = sum_ij H_ij D_ij and Tr D in FP64 (the band
 * energy of Sec. III.C).
 *  H, D  device, N x N, leading dimensions ldh, ldd.   out host double[2].
 */
int fdm_band_energy(const double *H, int64_t ldh, const double *D, int64_t ldd, int64_t N,
                    double *out, void *stream);

/*
 * fdm_fermi_operator -- one evaluation of the finite-temperature recursion at
 * a given mu (Sec. II.B.3, Eq. (2), with the doubling map of the design
 * notes): Y_0 = (Hp - mu I) / (kT 2^(depth+2)), Y <- 2 Y (I + 4 Y^2)^-1 depth
 * times (the inverse by Newton-Schulz in `precision`), D = I/2 - Y.
 *  depth <= 0 selects ceil(log2(beta * max(e_max - mu, mu - e_min))) +
 *  fd_extra_depth from Gershgorin bounds.
 *  out host double[3] (nullable): Tr D, Tr(D - D^2), depth used.
 */
int fdm_fermi_operator(const double *Hp, int64_t N, int64_t ldh, double mu, double kT,
                       int32_t depth, int32_t precision, double *D, int64_t ldd, double *out,
                       void *stream);

/* ---- serving: continuous batching of independent solves --------------- */

typedef struct fdm_server fdm_server;

typedef struct fdm_server_options {
    size_t budget_bytes;    /* device memory the server may hold for resident requests      */
    int32_t max_active;     /* requests executing at once (each on its own host thread and
                               stream); 0 = 4, at most 16                                    */
    int32_t precision;      /* default precision of submitted requests                      */
    int32_t independent;    /* 0 (default): the hot-loop steps of the executing requests (SP2
                               and McWeeny products, finite-temperature evaluations) run in
                               ticks, one grouped product launch per precision and one grouped
                               decision per tick over all of them; 1: each request launches
                               on its own stream                                              */
    int32_t reserved;
} fdm_server_options;

/* Creates a server on the current device (the caller selects it with
 * hipSetDevice) with the budget and limits in *opt.  Returns NULL on failure
 * (fdm_last_error() says why). */
fdm_server *fdm_server_create(const fdm_server_options *opt);

/* Queues a request.  Hp is copied at submission (host memory if hp_on_host,
 * else device memory) into a server-owned buffer; the caller may reuse it at
 * once.  Returns FDM_ENOMEM if the request alone exceeds the budget,
 * FDM_EINVAL for bad arguments.  *ticket identifies the request. */
int fdm_submit(fdm_server *s, const double *Hp, int32_t hp_on_host, int64_t N, double n_occ,
               double kT, double tol, int32_t precision, uint64_t *ticket);

/* 0 = finished (result ready), 1 = pending, negative = unknown ticket. */
int fdm_poll(fdm_server *s, uint64_t ticket);

/* Blocks until the request finishes, copies D to D_out (host memory if
 * out_on_host, else device; leading dimension ldd) and releases it.
 * Returns the request's solve status.  times (host double[4], nullable):
 * submit, start, finish and result times in seconds on the server clock.
 * A ticket is collected once: a second call for it, concurrent or later,
 * returns FDM_EINVAL. */
int fdm_result(fdm_server *s, uint64_t ticket, double *D_out, int32_t out_on_host,
               int64_t ldd, double *E_band, fdm_stats *stats, double *times);

/* Device memory of the server (host size_t each, nullable): bytes held in
 * blocks (in use or pooled for reuse; never above the budget), bytes reserved
 * by admitted requests and results not yet collected, and pooled bytes. */
int fdm_server_memory(fdm_server *s, size_t *held, size_t *reserved, size_t *pooled);

/* Stops the server: requests that have not started are dropped, running ones
 * finish, results not collected are discarded, and every resource is freed.
 * No other call on `s` may be in progress or follow. */
void fdm_server_destroy(fdm_server *s);

#ifdef __cplusplus
}
#endif
#endif /* FERMIDM_H */
