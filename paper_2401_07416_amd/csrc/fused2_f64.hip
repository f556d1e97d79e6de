// Two-step (temporally blocked) sweep kernel instances for double state.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "fused2.hpp"

namespace tdse {

namespace {

template <int W, int M>
hipError_t go2(bool rec, bool pf, dim3 grid, size_t lds, hipStream_t st, const Fused2Args<double>& a,
               hipEvent_t e0, hipEvent_t e1) {
    auto run = [&](auto kern) -> hipError_t {
        if (lds > 65536) {
            // more than 64 KiB of dynamic LDS has to be allowed per kernel
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        if (e0)
            hipExtLaunchKernelGGL(kern, grid, dim3(256), lds, st, e0, e1, 0, a);
        else
            hipLaunchKernelGGL(kern, grid, dim3(256), lds, st, a);
        return hipGetLastError();
    };
    if (pf)
        return rec ? run(fused2_kernel<double, W, M, true, true>) : run(fused2_kernel<double, W, M, false, true>);
    return rec ? run(fused2_kernel<double, W, M, true, false>) : run(fused2_kernel<double, W, M, false, false>);
}

template <int W>
hipError_t go2_m(int m, bool rec, bool pf, dim3 grid, size_t lds, hipStream_t st,
                 const Fused2Args<double>& a, hipEvent_t e0, hipEvent_t e1) {
    switch (m) {
        case 2: return go2<W, 2>(rec, pf, grid, lds, st, a, e0, e1);
        default: return go2<W, 3>(rec, pf, grid, lds, st, a, e0, e1);
    }
}

}  // namespace

hipError_t launch_fused2_f64(int w, int m, bool rec, bool pf, dim3 grid, size_t lds, hipStream_t st,
                             const Fused2Args<double>& a, hipEvent_t e0, hipEvent_t e1) {
    switch (w) {
        case 2: return go2_m<2>(m, rec, pf, grid, lds, st, a, e0, e1);
        case 1: return go2_m<1>(m, rec, pf, grid, lds, st, a, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

namespace {

template <int W, int M>
hipError_t gob2(bool rec, bool pf, dim3 grid, size_t lds, hipStream_t st, const Batch2Step<double>& b) {
    if (pf) {
        if (rec) hipLaunchKernelGGL((fused2_batch_kernel<double, W, M, true, true>), grid, dim3(256), lds, st, b);
        else hipLaunchKernelGGL((fused2_batch_kernel<double, W, M, false, true>), grid, dim3(256), lds, st, b);
    } else {
        if (rec) hipLaunchKernelGGL((fused2_batch_kernel<double, W, M, true, false>), grid, dim3(256), lds, st, b);
        else hipLaunchKernelGGL((fused2_batch_kernel<double, W, M, false, false>), grid, dim3(256), lds, st, b);
    }
    return hipGetLastError();
}

template <int W>
hipError_t gob2_m(int m, bool rec, bool pf, dim3 grid, size_t lds, hipStream_t st, const Batch2Step<double>& b) {
    switch (m) {
        case 2: return gob2<W, 2>(rec, pf, grid, lds, st, b);
        default: return gob2<W, 3>(rec, pf, grid, lds, st, b);
    }
}

template <int W, int M>
hipError_t allow2(size_t lds) {
    const void* k[4] = {reinterpret_cast<const void*>(fused2_batch_kernel<double, W, M, true, true>),
                        reinterpret_cast<const void*>(fused2_batch_kernel<double, W, M, false, true>),
                        reinterpret_cast<const void*>(fused2_batch_kernel<double, W, M, true, false>),
                        reinterpret_cast<const void*>(fused2_batch_kernel<double, W, M, false, false>)};
    for (const void* f : k) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int W>
hipError_t allow2_m(int m, size_t lds) {
    return m == 2 ? allow2<W, 2>(lds) : allow2<W, 3>(lds);
}

}  // namespace

hipError_t launch_fused2_batch_f64(int w, int m, bool rec, bool pf, dim3 grid, size_t lds, hipStream_t st,
                                   const Batch2Step<double>& b) {
    switch (w) {
        case 2: return gob2_m<2>(m, rec, pf, grid, lds, st, b);
        case 1: return gob2_m<1>(m, rec, pf, grid, lds, st, b);
        default: return hipErrorInvalidValue;
    }
}

// Allow the batch instances more than 64 KiB of dynamic LDS (before capture).
hipError_t fused2_batch_allow_lds_f64(int w, int m, size_t lds) {
    switch (w) {
        case 2: return allow2_m<2>(m, lds);
        case 1: return allow2_m<1>(m, lds);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tdse
