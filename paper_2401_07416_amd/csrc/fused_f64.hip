// One-pass step kernel instances for double state.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "fused.hpp"

namespace tdse {

namespace {

template <int W, int M>
hipError_t go(bool rec, bool pf, dim3 grid, int nt, size_t lds, hipStream_t st, const FusedArgs<double>& a,
              hipEvent_t e0, hipEvent_t e1) {
    auto run = [&](auto kern) -> hipError_t {
        if (e0)
            hipExtLaunchKernelGGL(kern, grid, dim3(nt), lds, st, e0, e1, 0, a);
        else
            hipLaunchKernelGGL(kern, grid, dim3(nt), lds, st, a);
        return hipGetLastError();
    };
    if (pf)
        return rec ? run(fused_step_kernel<double, W, M, true, true>)
                   : run(fused_step_kernel<double, W, M, false, true>);
    return rec ? run(fused_step_kernel<double, W, M, true, false>)
               : run(fused_step_kernel<double, W, M, false, false>);
}

template <int W>
hipError_t go_m(int m, bool rec, bool pf, dim3 grid, int nt, size_t lds, hipStream_t st,
                const FusedArgs<double>& a, hipEvent_t e0, hipEvent_t e1) {
    switch (m) {
        case 2: return go<W, 2>(rec, pf, grid, nt, lds, st, a, e0, e1);
        case 3: return go<W, 3>(rec, pf, grid, nt, lds, st, a, e0, e1);
        case 4: return go<W, 4>(rec, pf, grid, nt, lds, st, a, e0, e1);
        default: return go<W, 6>(rec, pf, grid, nt, lds, st, a, e0, e1);
    }
}

}  // namespace

hipError_t launch_fused_f64(int w, int m, bool rec, bool pf, dim3 grid, int nt, size_t lds, hipStream_t st,
                             const FusedArgs<double>& a, hipEvent_t e0, hipEvent_t e1) {
    switch (w) {
        case 2: return go_m<2>(m, rec, pf, grid, nt, lds, st, a, e0, e1);
        default: return go_m<1>(m, rec, pf, grid, nt, lds, st, a, e0, e1);
    }
}

namespace {

template <int W, int M>
hipError_t gob(bool rec, bool pf, dim3 grid, int nt, size_t lds, hipStream_t st, const BatchStep<double>& b) {
    if (pf) {
        if (rec) hipLaunchKernelGGL((fused_batch_kernel<double, W, M, true, true>), grid, dim3(nt), lds, st, b);
        else hipLaunchKernelGGL((fused_batch_kernel<double, W, M, false, true>), grid, dim3(nt), lds, st, b);
    } else {
        if (rec) hipLaunchKernelGGL((fused_batch_kernel<double, W, M, true, false>), grid, dim3(nt), lds, st, b);
        else hipLaunchKernelGGL((fused_batch_kernel<double, W, M, false, false>), grid, dim3(nt), lds, st, b);
    }
    return hipGetLastError();
}

template <int W>
hipError_t gob_m(int m, bool rec, bool pf, dim3 grid, int nt, size_t lds, hipStream_t st,
                 const BatchStep<double>& b) {
    switch (m) {
        case 2: return gob<W, 2>(rec, pf, grid, nt, lds, st, b);
        case 3: return gob<W, 3>(rec, pf, grid, nt, lds, st, b);
        case 4: return gob<W, 4>(rec, pf, grid, nt, lds, st, b);
        default: return gob<W, 6>(rec, pf, grid, nt, lds, st, b);
    }
}

}  // namespace

hipError_t launch_fused_batch_f64(int w, int m, bool rec, bool pf, dim3 grid, int nt, size_t lds,
                                  hipStream_t st, const BatchStep<double>& b) {
    switch (w) {
        case 2: return gob_m<2>(m, rec, pf, grid, nt, lds, st, b);
        default: return gob_m<1>(m, rec, pf, grid, nt, lds, st, b);
    }
}

}  // namespace tdse
