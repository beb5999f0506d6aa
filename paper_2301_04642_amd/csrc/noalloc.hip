// fdm_sym_product_noalloc: the product entry point for callers that cannot
// allocate device memory (code under stream capture, tight serving loops).
//
// Its workspace is a fixed device array of this file, not a hipMalloc'd
// block.  The array's host-side name is only a stand-in for the runtime's
// symbol lookup: host code uses the device address that hipGetSymbolAddress
// returns for the current device (looked up once per device, on the first
// call there) and never the name itself.  Every call on one device shares
// that device's array, so calls that overlap on one device (two streams, two
// host threads) race; calls in one stream are ordered by it.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "fdm_internal.h"
#include "solver_internal.h"

namespace fdm {

// 64 MiB: four working matrices of N_pad^2 x 8 bytes (FP64) or 4 + 4 bytes
// (FP32 masters with their hi/lo companions) for N_pad <= 1408, plus the
// partial sums, tile lists and device state.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64];

// Device address of `scratch` on device dev (the current device).
static int scratch_address(int dev, char **out) {
    if (dev < 0 || dev >= 64) {
        set_error("device ordinal out of range");
        return FDM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || (uintptr_t)p % 256 != 0) {
            set_error("scratch array has no 256-byte aligned device address");
            return FDM_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = (char *)g_scratch_ptr[dev];
    return FDM_OK;
}

// Zero-fills `words` 16-byte words (the padding of the working matrices must
// hold zeros; the array keeps the previous call's contents).
__global__ __launch_bounds__(256) void k_zero16(uint4 *p, size_t words) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// The upper-triangular tile list (ti <= tj) in the same banded order as the
// host-built lists of the cached workspace: bands of kTileBand tile rows,
// each walked column by column.  One thread; nt <= 1408 / 32 = 44 here.
__global__ void k_upper_tiles(uint32_t *out, int nt) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int k = 0;
    for (int i0 = 0; i0 < nt; i0 += kTileBand)
        for (int j = i0; j < nt; ++j) {
            const int iend = (i0 + kTileBand < j + 1) ? i0 + kTileBand : j + 1;
            for (int i = i0; i < iend; ++i) out[k++] = ((uint32_t)i << 16) | (uint32_t)j;
        }
}

}  // namespace fdm

using namespace fdm;

extern "C" {

int fdm_sym_product_noalloc(int32_t precision, const double *A, const double *B, const double *E,
                            double *C, int64_t N, int64_t ld, double alpha, double beta,
                            double gamma, double *sums, int32_t tile, void *stream) {
    set_error("");
    if (!sym_product_args_ok(precision, A, B, E, C, N, ld, tile)) {
        set_error("invalid argument");
        return FDM_EINVAL;
    }
    const Layout L = plan_product_layout(N, precision);
    if (L.bytes > kScratchBytes) {
        set_error("fdm_sym_product_noalloc: N = " + std::to_string(N) + " needs " +
                  std::to_string(L.bytes) + " workspace bytes, above the fixed " +
                  std::to_string(kScratchBytes) + " (N <= 1408)");
        return FDM_EINVAL;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    char *mem = nullptr;
    int rc = scratch_address(dev, &mem);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    // A view of the array: no events, no mapped mirror (the decide kernel
    // skips it when null), state read back into host memory of the view.
    Resources r;
    r.device = dev;
    r.view(L, mem);
    r.tiles128e = nullptr;  // no edge-block list here: 128-wide tiles only
    r.st_pinned = &r.st_fallback;
    const size_t words = L.bytes / 16;
    const int blocks = (int)std::min<size_t>((words + 255) / 256, 2048);
    hipLaunchKernelGGL(k_zero16, dim3(blocks), dim3(256), 0, s, (uint4 *)mem, words);
    hipLaunchKernelGGL(k_upper_tiles, dim3(1), dim3(1), 0, s, r.tiles64, (int)tile_rows(N, 64));
    hipLaunchKernelGGL(k_upper_tiles, dim3(1), dim3(1), 0, s, r.tiles128, (int)tile_rows(N, 128));
    hipLaunchKernelGGL(k_upper_tiles, dim3(1), dim3(1), 0, s, r.tiles32, (int)tile_rows(N, 32));
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "scratch set-up launch");
    return sym_product_bound(&r, precision, A, B, E, C, N, ld, alpha, beta, gamma, sums, tile, s);
}

}  // extern "C"
