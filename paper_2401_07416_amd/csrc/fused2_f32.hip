// Two-step (temporally blocked) sweep kernel instances for float state:
// (rows per thread, threads per workgroup) in {(2, 256), (3, 256), (1, 512), (2, 512), (1, 1024)}.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "fused2.hpp"

namespace tdse {

namespace {

template <int W, int M, int NT>
hipError_t go2(bool rec, bool pf, dim3 grid, size_t lds, hipStream_t st, const Fused2Args<float>& a,
               hipEvent_t e0, hipEvent_t e1) {
    auto run = [&](auto kern) -> hipError_t {
        if (lds > 65536) {
            // more than 64 KiB of dynamic LDS has to be allowed per kernel
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        if (e0)
            hipExtLaunchKernelGGL(kern, grid, dim3(NT), lds, st, e0, e1, 0, a);
        else
            hipLaunchKernelGGL(kern, grid, dim3(NT), lds, st, a);
        return hipGetLastError();
    };
    if (pf)
        return rec ? run(fused2_kernel<float, W, M, true, true, NT>) : run(fused2_kernel<float, W, M, false, true, NT>);
    return rec ? run(fused2_kernel<float, W, M, true, false, NT>) : run(fused2_kernel<float, W, M, false, false, NT>);
}

template <int W>
hipError_t go2_m(int m, int nt, bool rec, bool pf, dim3 grid, size_t lds, hipStream_t st,
                 const Fused2Args<float>& a, hipEvent_t e0, hipEvent_t e1) {
    if (m == 2 && nt == 256) return go2<W, 2, 256>(rec, pf, grid, lds, st, a, e0, e1);
    if (m == 3 && nt == 256) return go2<W, 3, 256>(rec, pf, grid, lds, st, a, e0, e1);
    if (m == 1 && nt == 512) return go2<W, 1, 512>(rec, pf, grid, lds, st, a, e0, e1);
    if (m == 2 && nt == 512) return go2<W, 2, 512>(rec, pf, grid, lds, st, a, e0, e1);
    if (m == 1 && nt == 1024) return go2<W, 1, 1024>(rec, pf, grid, lds, st, a, e0, e1);
    return hipErrorInvalidValue;
}

template <int W, int M, int NT>
hipError_t gob2(bool rec, bool pf, dim3 grid, size_t lds, hipStream_t st, const Batch2Step<float>& b) {
    if (pf) {
        if (rec) hipLaunchKernelGGL((fused2_batch_kernel<float, W, M, true, true, NT>), grid, dim3(NT), lds, st, b);
        else hipLaunchKernelGGL((fused2_batch_kernel<float, W, M, false, true, NT>), grid, dim3(NT), lds, st, b);
    } else {
        if (rec) hipLaunchKernelGGL((fused2_batch_kernel<float, W, M, true, false, NT>), grid, dim3(NT), lds, st, b);
        else hipLaunchKernelGGL((fused2_batch_kernel<float, W, M, false, false, NT>), grid, dim3(NT), lds, st, b);
    }
    return hipGetLastError();
}

template <int W>
hipError_t gob2_m(int m, int nt, bool rec, bool pf, dim3 grid, size_t lds, hipStream_t st,
                  const Batch2Step<float>& b) {
    if (m == 2 && nt == 256) return gob2<W, 2, 256>(rec, pf, grid, lds, st, b);
    if (m == 3 && nt == 256) return gob2<W, 3, 256>(rec, pf, grid, lds, st, b);
    if (m == 1 && nt == 512) return gob2<W, 1, 512>(rec, pf, grid, lds, st, b);
    if (m == 2 && nt == 512) return gob2<W, 2, 512>(rec, pf, grid, lds, st, b);
    if (m == 1 && nt == 1024) return gob2<W, 1, 1024>(rec, pf, grid, lds, st, b);
    return hipErrorInvalidValue;
}

template <int W, int M, int NT>
hipError_t allow2(size_t lds) {
    const void* k[4] = {reinterpret_cast<const void*>(fused2_batch_kernel<float, W, M, true, true, NT>),
                        reinterpret_cast<const void*>(fused2_batch_kernel<float, W, M, false, true, NT>),
                        reinterpret_cast<const void*>(fused2_batch_kernel<float, W, M, true, false, NT>),
                        reinterpret_cast<const void*>(fused2_batch_kernel<float, W, M, false, false, NT>)};
    for (const void* f : k) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int W>
hipError_t allow2_m(int m, int nt, size_t lds) {
    if (m == 2 && nt == 256) return allow2<W, 2, 256>(lds);
    if (m == 3 && nt == 256) return allow2<W, 3, 256>(lds);
    if (m == 1 && nt == 512) return allow2<W, 1, 512>(lds);
    if (m == 2 && nt == 512) return allow2<W, 2, 512>(lds);
    if (m == 1 && nt == 1024) return allow2<W, 1, 1024>(lds);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_fused2_f32(int w, int m, int nt, bool rec, bool pf, dim3 grid, size_t lds, hipStream_t st,
                             const Fused2Args<float>& a, hipEvent_t e0, hipEvent_t e1) {
    switch (w) {
        case 4: return go2_m<4>(m, nt, rec, pf, grid, lds, st, a, e0, e1);
        case 2: return go2_m<2>(m, nt, rec, pf, grid, lds, st, a, e0, e1);
        case 1: return go2_m<1>(m, nt, rec, pf, grid, lds, st, a, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fused2_batch_f32(int w, int m, int nt, bool rec, bool pf, dim3 grid, size_t lds,
                                   hipStream_t st, const Batch2Step<float>& b) {
    switch (w) {
        case 4: return gob2_m<4>(m, nt, rec, pf, grid, lds, st, b);
        case 2: return gob2_m<2>(m, nt, rec, pf, grid, lds, st, b);
        case 1: return gob2_m<1>(m, nt, rec, pf, grid, lds, st, b);
        default: return hipErrorInvalidValue;
    }
}

// Allow the batch instances more than 64 KiB of dynamic LDS (before capture).
hipError_t fused2_batch_allow_lds_f32(int w, int m, int nt, size_t lds) {
    switch (w) {
        case 4: return allow2_m<4>(m, nt, lds);
        case 2: return allow2_m<2>(m, nt, lds);
        case 1: return allow2_m<1>(m, nt, lds);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tdse
