// HBM probe: streaming kernels that give the practical bandwidth ceiling the
// step kernels are judged against (a plain copy, the one-pass step's mix of
// three read and two written streams, and a write-only stream).  They do no
// part of the method.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/tdse.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// Every access carries the non-temporal hint: nothing is re-read, and on
// this device the hinted streams are the fastest measured (copy 6.5 TB/s,
// the mix 5.9 TB/s over 1 GiB streams with one vector per thread).
__global__ __launch_bounds__(256) void hbm_copy_kernel(const f4* __restrict__ a, f4* __restrict__ b,
                                                       long n4) {
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

__global__ __launch_bounds__(256) void hbm_mix_kernel(const f4* __restrict__ a, const f4* __restrict__ b,
                                                      const f4* __restrict__ c, f4* __restrict__ d,
                                                      f4* __restrict__ e, long n4) {
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        const f4 x = __builtin_nontemporal_load(a + i);
        const f4 y = __builtin_nontemporal_load(b + i);
        const f4 z = __builtin_nontemporal_load(c + i);
        __builtin_nontemporal_store(x + y * z, d + i);
        __builtin_nontemporal_store(y - x * z, e + i);
    }
}

// a write-only stream (the ceiling of a kernel that only writes, such as
// the potential interpolation)
__global__ __launch_bounds__(256) void hbm_fill_kernel(f4* __restrict__ b, float v, long n4) {
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        __builtin_nontemporal_store(f4{v, v, v, v}, b + i);
}

}  // namespace

extern "C" tdse_status tdse_hbm_probe(int32_t kind, void* const* bufs, int64_t n, int32_t grid,
                                      int32_t reps, void* stream, double* ms_per_pass) {
    if (!bufs || !ms_per_pass || n <= 0 || n % 4 != 0 || reps < 1 || grid < 0) return TDSE_ERR_ARG;
    if (kind != 0 && kind != 1 && kind != 2) return TDSE_ERR_ARG;
    const int nb = kind == 0 ? 2 : kind == 1 ? 5 : 1;
    for (int i = 0; i < nb; ++i) {
        if (!bufs[i] || reinterpret_cast<uintptr_t>(bufs[i]) % 16 != 0) return TDSE_ERR_ARG;
        for (int j = 0; j < i; ++j)
            if (bufs[i] == bufs[j]) return TDSE_ERR_ARG;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const long n4 = n / 4;
    long g = grid > 0 ? grid : (n4 + 255) / 256;   // default: one vector per thread
    g = g < (n4 + 255) / 256 ? g : (n4 + 255) / 256;
    auto launch = [&]() {
        if (kind == 0)
            hipLaunchKernelGGL(hbm_copy_kernel, dim3((unsigned)g), dim3(256), 0, st,
                               static_cast<const f4*>(bufs[0]), static_cast<f4*>(bufs[1]), n4);
        else if (kind == 2)
            hipLaunchKernelGGL(hbm_fill_kernel, dim3((unsigned)g), dim3(256), 0, st,
                               static_cast<f4*>(bufs[0]), 1.0f, n4);
        else
            hipLaunchKernelGGL(hbm_mix_kernel, dim3((unsigned)g), dim3(256), 0, st,
                               static_cast<const f4*>(bufs[0]), static_cast<const f4*>(bufs[1]),
                               static_cast<const f4*>(bufs[2]), static_cast<f4*>(bufs[3]),
                               static_cast<f4*>(bufs[4]), n4);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return TDSE_ERR_DEVICE;
    }
    tdse_status s = TDSE_OK;
    launch();  // warm-up pass
    if (hipEventRecord(e0, st) != hipSuccess) s = TDSE_ERR_DEVICE;
    for (int r = 0; r < reps && s == TDSE_OK; ++r) launch();
    if (s == TDSE_OK && hipGetLastError() != hipSuccess) s = TDSE_ERR_DEVICE;
    if (s == TDSE_OK && hipEventRecord(e1, st) != hipSuccess) s = TDSE_ERR_DEVICE;
    if (s == TDSE_OK && hipEventSynchronize(e1) != hipSuccess) s = TDSE_ERR_DEVICE;
    float ms = 0.f;
    if (s == TDSE_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) s = TDSE_ERR_DEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s == TDSE_OK) *ms_per_pass = (double)ms / reps;
    return s;
}
