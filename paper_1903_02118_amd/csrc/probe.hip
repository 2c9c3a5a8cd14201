// HBM read probe: one streaming read of a device buffer with the access of
// the near-field and dense kernels (16-byte non-temporal loads), timed with
// HIP events.  A measurement utility, not part of the method.
#include <hip/hip_runtime.h>

#include <string>

#include "bie_internal.hpp"

namespace bie {

typedef double probe_double2 __attribute__((ext_vector_type(2)));

constexpr int PROBE_BLOCKS = 256 * 16;  // 16 workgroups per compute unit
// The per-workgroup sums live in a static device array: the library
// allocates no device memory, the probe included.
__device__ double probe_sums[PROBE_BLOCKS];

// Grid-stride sum over the buffer; the per-block sum is written so the loads
// are not removed.  Eight independent loads per lane per pass.
__global__ __launch_bounds__(256) void k_hbm_read(const probe_double2 *__restrict__ a, int64_t n,
                                                  double *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s0 = 0.0, s1 = 0.0;
    for (; i + 7 * stride < n; i += 8 * stride) {
        probe_double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = __builtin_nontemporal_load(a + i + u * stride);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            s0 += v[u].x;
            s1 += v[u].y;
        }
    }
    for (; i < n; i += stride) {
        const probe_double2 v = __builtin_nontemporal_load(a + i);
        s0 += v.x;
        s1 += v.y;
    }
    __shared__ double red[256];
    red[threadIdx.x] = s0 + s1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace bie

extern "C" int bie_hbm_read_probe(const void *buf_dev, int64_t bytes, double *ms_out, void *stream) {
    if (!buf_dev || !ms_out || bytes <= 0 || bytes % 16 != 0 || ((uintptr_t)buf_dev & 15) != 0) {
        bie::set_error("bie_hbm_read_probe: need a 16-byte aligned buffer, a positive multiple of 16 bytes, an output");
        return BIE_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    constexpr int BLOCKS = bie::PROBE_BLOCKS;
    double *out = nullptr;  // device address of the static array (current device)
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = BIE_OK;
    float ms = 0.0f;
    if (hipGetSymbolAddress((void **)&out, HIP_SYMBOL(bie::probe_sums)) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        bie::set_error("bie_hbm_read_probe: the probe's partial-sum array or its events are not available");
        rc = BIE_EHIP;
    } else {
        const auto *a = reinterpret_cast<const bie::probe_double2 *>(buf_dev);
        hipEventRecord(e0, s);
        hipLaunchKernelGGL(bie::k_hbm_read, dim3(BLOCKS), dim3(256), 0, s, a, bytes / 16, out);
        hipEventRecord(e1, s);
        const hipError_t err = hipEventSynchronize(e1);
        if (err != hipSuccess || hipGetLastError() != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            bie::set_error(std::string("bie_hbm_read_probe: ") + hipGetErrorString(err));
            rc = BIE_EHIP;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc == BIE_OK) *ms_out = (double)ms;
    return rc;
}
