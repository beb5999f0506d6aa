// O(N^2) kernels around the product: Gershgorin bounds (Sec. II.C), the
// scaled start X_0 and other affine maps, precision conversions, the band
// energy Tr(Hp D) (Sec. III.C), and the single-block "decide" kernel that
// reduces per-block partial sums in a fixed order and takes the SP2 branch
// and stop decisions on the device (Sec. II.B.1 picks the branch from
// traces; Sec. III.A stops on a trace/idempotency criterion).
//
// All of them are HBM-bound streaming kernels: one wave64 walks a row with
// coalesced loads; per-block partials are written to a scratch array and
// summed by one block in index order, so every result is bitwise
// reproducible run to run.
#include <math.h>

#include "fdm_internal.h"

namespace fdm {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

// ---- Gershgorin: one wave per row -----------------------------------------
// partials per block: [min(H_ii - r_i), max(H_ii + r_i), sum H_ii, sum H_ij^2,
//                      rows with a non-finite entry]
__global__ __launch_bounds__(256) void k_gersh_rows(const double *__restrict__ H, int64_t ldh,
                                                    int n, double *__restrict__ part) {
    __shared__ double red[4][5];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + w;
    double rs = 0.0, dg = 0.0, sq = 0.0, bad = 0.0;
    if (row < n) {
        const double *h = H + (int64_t)row * ldh;
        for (int j = lane; j < n; j += 64) {
            const double v = h[j];
            if (!isfinite(v)) bad = 1.0;
            sq += v * v;
            if (j == row)
                dg = v;
            else
                rs += fabs(v);
        }
    }
    rs = wave_sum(rs);
    dg = wave_sum(dg);
    sq = wave_sum(sq);
    bad = wave_max(bad);
    if (lane == 0) {
        const bool ok = row < n;
        red[w][0] = ok ? dg - rs : INFINITY;
        red[w][1] = ok ? dg + rs : -INFINITY;
        red[w][2] = dg;
        red[w][3] = sq;
        red[w][4] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *p = part + (size_t)blockIdx.x * 8;
        p[0] = fmin(fmin(red[0][0], red[1][0]), fmin(red[2][0], red[3][0]));
        p[1] = fmax(fmax(red[0][1], red[1][1]), fmax(red[2][1], red[3][1]));
        p[2] = (red[0][2] + red[1][2]) + (red[2][2] + red[3][2]);
        p[3] = (red[0][3] + red[1][3]) + (red[2][3] + red[3][3]);
        p[4] = (red[0][4] + red[1][4]) + (red[2][4] + red[3][4]);
    }
}

__global__ __launch_bounds__(256) void k_gersh_final(const double *__restrict__ part, int count,
                                                     DevState *st) {
    __shared__ double red[5][256];
    const int t = threadIdx.x;
    double lo = INFINITY, hi = -INFINITY, tr = 0.0, sq = 0.0, bad = 0.0;
    for (int i = t; i < count; i += 256) {
        const double *p = part + (size_t)i * 8;
        lo = fmin(lo, p[0]);
        hi = fmax(hi, p[1]);
        tr += p[2];
        sq += p[3];
        bad += p[4];
    }
    red[0][t] = lo;
    red[1][t] = hi;
    red[2][t] = tr;
    red[3][t] = sq;
    red[4][t] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            red[0][t] = fmin(red[0][t], red[0][t + s]);
            red[1][t] = fmax(red[1][t], red[1][t + s]);
            red[2][t] += red[2][t + s];
            red[3][t] += red[3][t + s];
            red[4][t] += red[4][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        st->emin = red[0][0];
        st->emax = red[1][0];
        st->trH = red[2][0];
        st->fro2H = red[3][0];
        st->nonfinite = (int32_t)red[4][0];
    }
}

// ---- affine maps: out = a*in + b*I on [0,n)^2, 0 elsewhere in [0,np)^2 ----
// zt_init: X_0 = (e_max I - H) / (e_max - e_min) from the device bounds.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_affine(const TI *__restrict__ in, int64_t ldi,
                                                TO *__restrict__ out, int64_t ldo, int n,
                                                int np, double a, double b, int zt_init,
                                                const DevState *st, double *__restrict__ part) {
    __shared__ double red[2][4];
    double emax = 0.0, den = 1.0;
    if (zt_init) {
        emax = st->emax;
        den = st->emax - st->emin;
    }
    double tr = 0.0, f2 = 0.0;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int row = blockIdx.x * 4 + rr;
        if (row >= np) break;
        for (int c = threadIdx.x; c < np; c += 256) {
            double v = 0.0;
            if (row < n && c < n) {
                const double x = (double)in[(int64_t)row * ldi + c];
                if (zt_init)
                    v = ((row == c ? emax : 0.0) - x) / den;
                else
                    v = a * x + (row == c ? b : 0.0);
            }
            const TO o = (TO)v;
            out[(int64_t)row * ldo + c] = o;
            const double od = (double)o;
            f2 += od * od;
            if (row == c) tr += od;
        }
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    tr = wave_sum(tr);
    f2 = wave_sum(f2);
    if (lane == 0) {
        red[0][w] = tr;
        red[1][w] = f2;
    }
    __syncthreads();
    if (threadIdx.x == 0 && part != nullptr) {
        double *p = part + (size_t)blockIdx.x * 4;
        p[0] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        p[1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        p[2] = 0.0;
        p[3] = 0.0;
    }
}

// ---- out = a*X + b*Y + c*I on [0,n)^2 (working matrices), zeros elsewhere --
template <typename T>
__global__ __launch_bounds__(256) void k_axpby2(const T *__restrict__ X, const T *__restrict__ Y,
                                                T *__restrict__ out, int64_t ld, int n, int np,
                                                double a, double b, double c,
                                                double *__restrict__ part) {
    __shared__ double red[2][4];
    double tr = 0.0, f2 = 0.0;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int row = blockIdx.x * 4 + rr;
        if (row >= np) break;
        for (int col = threadIdx.x; col < np; col += 256) {
            const int64_t k = (int64_t)row * ld + col;
            double v = 0.0;
            if (row < n && col < n)
                v = a * (double)X[k] + b * (double)Y[k] + (row == col ? c : 0.0);
            const T o = (T)v;
            out[k] = o;
            const double od = (double)o;
            f2 += od * od;
            if (row == col) tr += od;
        }
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    tr = wave_sum(tr);
    f2 = wave_sum(f2);
    if (lane == 0) {
        red[0][w] = tr;
        red[1][w] = f2;
    }
    __syncthreads();
    if (threadIdx.x == 0 && part != nullptr) {
        double *p = part + (size_t)blockIdx.x * 4;
        p[0] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        p[1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        p[2] = 0.0;
        p[3] = 0.0;
    }
}

// ---- Lanczos (tighter spectral bounds) -------------------------------------
// v_0: deterministic pseudo-random unit vector (single block).
__global__ __launch_bounds__(1024) void k_lanczos_start(double *__restrict__ v, int n) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        uint32_t h = (uint32_t)i * 2654435761u + 0x9e3779b9u;
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        const double x = ((double)(h >> 8) + 0.5) / 16777216.0 - 0.5;
        v[i] = x;
        s += x * x;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 512; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    const double inv = 1.0 / sqrt(red[0]);
    for (int i = threadIdx.x; i < n; i += 1024) v[i] *= inv;
}

// w = a (M v) - shift v + b y - beta_prev v_prev (y, beta_prev nullable),
// one wave per row of the caller's M.
__global__ __launch_bounds__(256) void k_lanczos_matvec(const double *__restrict__ H, int64_t ldh,
                                                        int n, const double *__restrict__ v,
                                                        double a, double shift,
                                                        const double *__restrict__ y, double b,
                                                        const double *__restrict__ vprev,
                                                        const double *beta_prev,
                                                        double *__restrict__ w) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + wv;
    if (row >= n) return;
    const double *h = H + (int64_t)row * ldh;
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s += h[j] * v[j];
    s = wave_sum(s);
    if (lane == 0) {
        double o = a * s - shift * v[row];
        if (y) o += b * y[row];
        if (beta_prev) o -= *beta_prev * vprev[row];
        w[row] = o;
    }
}

// alpha = w.v ; w -= alpha v ; beta = ||w|| ; w <- w / beta (single block,
// fixed-order reductions).
__global__ __launch_bounds__(1024) void k_lanczos_update(double *__restrict__ w,
                                                         const double *__restrict__ v, int n,
                                                         double *alpha, double *beta) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) s += w[i] * v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 512; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    const double a = red[0];
    __syncthreads();
    s = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        const double x = w[i] - a * v[i];
        w[i] = x;
        s += x * x;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 512; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    const double b = sqrt(red[0]);
    const double inv = b > 0.0 ? 1.0 / b : 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) w[i] *= inv;
    if (threadIdx.x == 0) {
        *alpha = a;
        *beta = b;
    }
}

__global__ void k_set_bounds(DevState *st, double emin, double emax) {
    if (threadIdx.x == 0) {
        st->emin = emin;
        st->emax = emax;
    }
}

// ---- band energy: sum_ij H_ij D_ij and Tr D -------------------------------
template <typename TD>
__global__ __launch_bounds__(256) void k_energy(const double *__restrict__ H, int64_t ldh,
                                                const TD *__restrict__ D, int64_t ldd, int n,
                                                double *__restrict__ part) {
    __shared__ double red[2][4];
    double e = 0.0, tr = 0.0;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int row = blockIdx.x * 4 + rr;
        if (row >= n) break;
        for (int c = threadIdx.x; c < n; c += 256) {
            const double d = (double)D[(int64_t)row * ldd + c];
            e += H[(int64_t)row * ldh + c] * d;
            if (row == c) tr += d;
        }
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    e = wave_sum(e);
    tr = wave_sum(tr);
    if (lane == 0) {
        red[0][w] = e;
        red[1][w] = tr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *p = part + (size_t)blockIdx.x * 4;
        p[0] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        p[1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        p[2] = 0.0;
        p[3] = 0.0;
    }
}

template <typename TS>
__global__ __launch_bounds__(256) void k_copy_out(const TS *__restrict__ src, int64_t lds,
                                                  double *__restrict__ dst, int64_t ldd, int n) {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int row = blockIdx.x * 4 + rr;
        if (row >= n) break;
        for (int c = threadIdx.x; c < n; c += 256)
            dst[(int64_t)row * ldd + c] = (double)src[(int64_t)row * lds + c];
    }
}

// ---- decide ----------------------------------------------------------------
__device__ __forceinline__ int choose_square(double trace, double fro2, double n_occ) {
    // Tr X^2 = ||X||_F^2 and Tr(2X - X^2) = 2 Tr X - ||X||_F^2: take the
    // branch whose trace lands closer to N_occ (ties -> X^2).
    return fabs(fro2 - n_occ) <= fabs(2.0 * trace - fro2 - n_occ) ? 1 : 0;
}

__device__ __forceinline__ void decide_block(DevState *st, HostMirror *hm,
                                             const double *__restrict__ part, int count, int mode,
                                             int stride) {
    if ((mode == D_SP2 || mode == D_MCW_T || mode == D_MCW_OUT) && st->done) return;
    __shared__ double red[3][256];
    const int t = threadIdx.x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int i = t; i < count; i += 256) {
        const double *p = part + (size_t)i * stride;
        s0 += p[0];
        s1 += p[1];
        s2 += p[2];
    }
    red[0][t] = s0;
    red[1][t] = s1;
    red[2][t] = s2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            red[0][t] += red[0][t + s];
            red[1][t] += red[1][t + s];
            red[2][t] += red[2][t + s];
        }
        __syncthreads();
    }
    if (t != 0) return;
    s0 = red[0][0];
    s1 = red[1][0];
    s2 = red[2][0];
    const int32_t was_done = st->done;
    switch (mode) {
        case D_INIT:
            st->trace = s0;
            st->fro2 = s1;
            st->sigma = choose_square(s0, s1, st->n_occ);
            st->done = 0;
            st->iter = 0;
            st->result_iter = 0;
            st->executed = 0;
            st->status = 0;
            st->idem = INFINITY;
            st->idem_hist[0] = INFINITY;
            st->idem_hist[1] = INFINITY;
            break;
        case D_SP2: {
            // s0, s1: Tr and ||.||^2 of X_{n+1}; s2 = ||X_n^2 - X_n||^2.
            const int n = st->iter;
            const int flags = st->switch_mode;
            const int sm = flags & 7;
            const double idem = sqrt(s2);
            const double two_back = st->idem_hist[1];  // idempotency of X_{n-2}
            st->idem_hist[0] = st->idem_hist[1];
            st->idem_hist[1] = st->idem;
            st->idem = idem;
            st->idem_ring[st->nring & 7] = idem;
            st->nring += 1;
            st->executed = n + 1;
            // relative trace change of X_{n+1} against X_n (Sec. III.A)
            const double reltr = fabs(s0 - st->trace) / fmax(fabs(st->trace), 1e-300);
            st->reltr = reltr;
            // Below 0.1 every eigenvalue is within ~0.1 of 0 or 1 and two SP2
            // steps shrink the error at least 2.5x; a smaller gain means the
            // iteration sits on its rounding floor.
            const bool stagnant = idem < 0.1 && idem >= 0.8 * two_back;
            // X_{n+1} has left [0, 1] (||X||^2 > Tr X needs eigenvalues
            // outside it): give up before it overflows
            if ((flags & kGuard) && (!(idem < INFINITY) || !(s1 <= s0 + 0.5))) {
                st->done = 1;
                st->result_iter = n;
                st->status = FDM_ENOCONV;
                break;
            }
            if (flags & kFixedSteps) {
                // a truncated expansion runs exactly max_iter products
            } else if (flags & kRelTrStop) {
                if (reltr <= st->tau) {
                    st->done = 1;
                    st->result_iter = n + 1;
                }
            } else {
                // converged: idempotent and holding n_occ electrons
                // (st->trace is still Tr X_n here)
                if (idem <= st->tol && fabs(st->trace - st->n_occ) <= st->tol) {
                    st->done = 1;
                    st->result_iter = n;
                    break;
                }
                if (sm == 1 && (idem <= st->tau || stagnant)) {
                    st->done = 1;
                    st->result_iter = n + 1;
                } else if (sm != 1 && stagnant) {
                    st->done = 1;
                    st->result_iter = n;
                    st->status = FDM_ENOCONV;
                    break;
                }
            }
            if (st->gprod < 256)
                st->bits[st->gprod >> 6] |= (uint64_t)(st->sigma & 1) << (st->gprod & 63);
            st->gprod += 1;
            st->iter = n + 1;
            st->trace = s0;
            st->fro2 = s1;
            st->sigma = choose_square(s0, s1, st->n_occ);
            if (!st->done && st->iter >= st->max_iter) {
                st->done = 1;
                st->result_iter = st->iter;
                if (sm == 0 && !(flags & kFixedSteps)) st->status = FDM_ENOCONV;
            }
            break;
        }
        case D_MCW_T: {
            const double idem = sqrt(s2);
            st->idem = idem;
            st->idem_ring[st->nring & 7] = idem;
            st->nring += 1;
            st->executed += 1;
            if (st->iter < 4) {
                st->mcw_idem[st->iter] = idem;
                st->mcw_trerr[st->iter] = fabs(st->trace - st->n_occ);
            }
            if (idem <= st->tol && fabs(st->trace - st->n_occ) <= st->tol) {
                st->done = 1;
                st->result_iter = st->iter;
            } else if (st->iter >= st->max_iter) {
                st->done = 1;
                st->result_iter = st->iter;
                st->status = FDM_ENOCONV;
            }
            break;
        }
        case D_MCW_OUT:
            st->executed += 1;
            st->iter += 1;
            st->trace = s0;
            st->fro2 = s1;
            break;
        case D_CERT:
            if (st->ncert < 8) st->cert[st->ncert] = s1;
            st->ncert += 1;
            break;
        case D_SUMS:
        default:
            st->sums[0] = s0;
            st->sums[1] = s1;
            st->sums[2] = s2;
            break;
    }
    if (hm != nullptr && st->done && !was_done) {
        // Written once per phase, by the decision that ends it (the host
        // clears `done` before the phase starts and polls it).  The host
        // reads the other fields after it sees `done`: they are written
        // first and made visible before `done` is.
        volatile HostMirror *vh = hm;
        vh->iter = st->iter;
        vh->result_iter = st->result_iter;
        vh->executed = st->executed;
        vh->status = st->status;
        vh->sigma = st->sigma;
        vh->idem = st->idem;
        vh->trace = st->trace;
        __threadfence_system();
        vh->done = st->done;
        __threadfence_system();
    }
}

__global__ __launch_bounds__(256) void k_decide(DevState *st, HostMirror *hm,
                                                const double *__restrict__ part, int count,
                                                int mode, int stride) {
    decide_block(st, hm, part, count, mode, stride);
}

// One block per decision (the serving tick); each block does exactly what
// k_decide does for its job.
__global__ __launch_bounds__(256) void k_decide_grouped(DecideGroup g) {
    const DecideJob &j = g.job[blockIdx.x];
    decide_block(j.st, j.hm, j.part, j.count, j.mode, j.stride);
}

// Parameters of the next phase; reset_all also clears the solve-wide fields.
__global__ void k_set_params(DevState *st, double n_occ, double tol, double tau, int max_iter,
                             int switch_mode, int reset_all) {
    if (threadIdx.x != 0) return;
    st->n_occ = n_occ;
    st->tol = tol;
    st->tau = tau;
    st->max_iter = max_iter;
    st->switch_mode = switch_mode;
    if (reset_all) {
        st->ncert = 0;
        st->nring = 0;
        st->reltr = 0.0;
        st->gprod = 0;
        st->bits[0] = st->bits[1] = st->bits[2] = st->bits[3] = 0;
        st->done = 0;
        st->status = 0;
    }
}

}  // namespace

int gershgorin_blocks(int n) { return (n + 3) / 4; }
int affine_blocks(int np) { return (np + 3) / 4; }
int energy_blocks(int n) { return (n + 3) / 4; }

hipError_t launch_gershgorin(const double *H, int64_t ldh, int n, double *partials,
                             DevState *st, hipStream_t s) {
    const int nb = gershgorin_blocks(n);
    hipLaunchKernelGGL(k_gersh_rows, dim3(nb), dim3(256), 0, s, H, ldh, n, partials);
    hipLaunchKernelGGL(k_gersh_final, dim3(1), dim3(256), 0, s, partials, nb, st);
    return hipGetLastError();
}

hipError_t launch_affine(int in_f32, const void *in, int64_t ldi, int out_f32, void *out,
                         int64_t ldo, int n, int np, double a, double b, int zt_init,
                         const DevState *st, double *partials, int *nparts, hipStream_t s) {
    const int nb = affine_blocks(np);
    if (nparts) *nparts = nb;
    if (nb == 0) return hipSuccess;
    if (!in_f32 && !out_f32)
        hipLaunchKernelGGL((k_affine<double, double>), dim3(nb), dim3(256), 0, s,
                           (const double *)in, ldi, (double *)out, ldo, n, np, a, b, zt_init, st,
                           partials);
    else if (!in_f32 && out_f32)
        hipLaunchKernelGGL((k_affine<double, float>), dim3(nb), dim3(256), 0, s,
                           (const double *)in, ldi, (float *)out, ldo, n, np, a, b, zt_init, st,
                           partials);
    else if (in_f32 && !out_f32)
        hipLaunchKernelGGL((k_affine<float, double>), dim3(nb), dim3(256), 0, s,
                           (const float *)in, ldi, (double *)out, ldo, n, np, a, b, zt_init, st,
                           partials);
    else
        hipLaunchKernelGGL((k_affine<float, float>), dim3(nb), dim3(256), 0, s,
                           (const float *)in, ldi, (float *)out, ldo, n, np, a, b, zt_init, st,
                           partials);
    return hipGetLastError();
}

hipError_t launch_decide_grouped(const DecideGroup &g, hipStream_t s) {
    if (g.njobs <= 0 || g.njobs > kMaxGroup) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_decide_grouped, dim3(g.njobs), dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_decide(DevState *st, HostMirror *hm, const double *partials, int count,
                         int mode, int stride, hipStream_t s) {
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(256), 0, s, st, hm, partials, count, mode, stride);
    return hipGetLastError();
}

hipError_t launch_energy(const double *H, int64_t ldh, const double *D, int64_t ldd, int d_f32,
                         int n, double *partials, DevState *st, hipStream_t s) {
    const int nb = energy_blocks(n);
    if (d_f32)
        hipLaunchKernelGGL((k_energy<float>), dim3(nb), dim3(256), 0, s, H, ldh,
                           (const float *)D, ldd, n, partials);
    else
        hipLaunchKernelGGL((k_energy<double>), dim3(nb), dim3(256), 0, s, H, ldh, D, ldd, n,
                           partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_decide(st, nullptr, partials, nb, D_SUMS, 4, s);
}

hipError_t launch_axpby2(int f32, const void *X, const void *Y, void *out, int64_t ld, int n,
                         int np, double a, double b, double c, double *partials, int *nparts,
                         hipStream_t s) {
    const int nb = affine_blocks(np);
    if (nparts) *nparts = nb;
    if (f32)
        hipLaunchKernelGGL((k_axpby2<float>), dim3(nb), dim3(256), 0, s, (const float *)X,
                           (const float *)Y, (float *)out, ld, n, np, a, b, c, partials);
    else
        hipLaunchKernelGGL((k_axpby2<double>), dim3(nb), dim3(256), 0, s, (const double *)X,
                           (const double *)Y, (double *)out, ld, n, np, a, b, c, partials);
    return hipGetLastError();
}

// k Lanczos steps on the caller's H: v holds 3 vectors of stride np; ab
// receives alpha[0..k) then beta[0..k).
hipError_t launch_lanczos(const double *H, int64_t ldh, int n, int np, int k, double *v,
                          double *ab, hipStream_t s) {
    hipLaunchKernelGGL(k_lanczos_start, dim3(1), dim3(1024), 0, s, v, n);
    const int nb = (n + 3) / 4;
    for (int j = 0; j < k; ++j) {
        double *vj = v + (size_t)(j % 3) * np;
        double *vp = v + (size_t)((j + 2) % 3) * np;
        double *vn = v + (size_t)((j + 1) % 3) * np;
        hipLaunchKernelGGL(k_lanczos_matvec, dim3(nb), dim3(256), 0, s, H, ldh, n, vj, 1.0, 0.0,
                           (const double *)nullptr, 0.0, vp,
                           j ? ab + k + j - 1 : (const double *)nullptr, vn);
        hipLaunchKernelGGL(k_lanczos_update, dim3(1), dim3(1024), 0, s, vn, vj, n, ab + j,
                           ab + k + j);
    }
    return hipGetLastError();
}

hipError_t launch_lanczos_proj(const double *H, int64_t ldh, const double *D, int64_t ldd, int n,
                               int np, int k, int unocc, double sigma, double *v, double *ab,
                               hipStream_t s) {
    double *t = v + 3 * (size_t)np, *zero = v + 4 * (size_t)np;
    hipError_t e = hipMemsetAsync(zero, 0, (size_t)np * sizeof(double), s);
    if (e != hipSuccess) return e;
    const int nb = (n + 3) / 4;
    const double *nul = nullptr;
    // v_0 = P z / ||P z||, P = D or I - D, z the fixed pseudo-random vector
    hipLaunchKernelGGL(k_lanczos_start, dim3(1), dim3(1024), 0, s, t, n);
    hipLaunchKernelGGL(k_lanczos_matvec, dim3(nb), dim3(256), 0, s, D, ldd, n, t,
                       unocc ? -1.0 : 1.0, 0.0, unocc ? (const double *)t : nul, 1.0, nul, nul, v);
    hipLaunchKernelGGL(k_lanczos_update, dim3(1), dim3(1024), 0, s, v, zero, n, ab, ab + k);
    for (int j = 0; j < k; ++j) {
        double *vj = v + (size_t)(j % 3) * np;
        double *vp = v + (size_t)((j + 2) % 3) * np;
        double *vn = v + (size_t)((j + 1) % 3) * np;
        // t = (H - sigma I) v_j ; w = P t - beta_{j-1} v_{j-1}
        hipLaunchKernelGGL(k_lanczos_matvec, dim3(nb), dim3(256), 0, s, H, ldh, n, vj, 1.0, sigma,
                           nul, 0.0, nul, nul, t);
        hipLaunchKernelGGL(k_lanczos_matvec, dim3(nb), dim3(256), 0, s, D, ldd, n, t,
                           unocc ? -1.0 : 1.0, 0.0, unocc ? (const double *)t : nul, 1.0, vp,
                           j ? ab + k + j - 1 : nul, vn);
        hipLaunchKernelGGL(k_lanczos_update, dim3(1), dim3(1024), 0, s, vn, vj, n, ab + j,
                           ab + k + j);
    }
    return hipGetLastError();
}

hipError_t launch_set_bounds(DevState *st, double emin, double emax, hipStream_t s) {
    hipLaunchKernelGGL(k_set_bounds, dim3(1), dim3(64), 0, s, st, emin, emax);
    return hipGetLastError();
}

hipError_t launch_set_params(DevState *st, double n_occ, double tol, double tau, int max_iter,
                             int switch_mode, int reset_all, hipStream_t s) {
    hipLaunchKernelGGL(k_set_params, dim3(1), dim3(64), 0, s, st, n_occ, tol, tau, max_iter,
                       switch_mode, reset_all);
    return hipGetLastError();
}

hipError_t launch_copy_out(int src_f32, const void *src, int64_t lds, double *dst, int64_t ldd,
                           int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int nb = (n + 3) / 4;
    if (src_f32)
        hipLaunchKernelGGL((k_copy_out<float>), dim3(nb), dim3(256), 0, s, (const float *)src,
                           lds, dst, ldd, n);
    else
        hipLaunchKernelGGL((k_copy_out<double>), dim3(nb), dim3(256), 0, s,
                           (const double *)src, lds, dst, ldd, n);
    return hipGetLastError();
}

}  // namespace fdm
