// One-pass adjoint step instances for float state.
#include <hip/hip_runtime.h>

#include "adjoint_fused.hpp"

namespace tdse {

namespace {

template <int W>
hipError_t goa(int m, dim3 grid, size_t lds, hipStream_t st, const AdjFusedArgs<float>& a) {
    if (m == 2)
        hipLaunchKernelGGL((adjoint_fused_kernel<float, W, 2>), grid, dim3(256), lds, st, a);
    else
        hipLaunchKernelGGL((adjoint_fused_kernel<float, W, 3>), grid, dim3(256), lds, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint_fused_f32(int w, int m, dim3 grid, size_t lds, hipStream_t st,
                                    const AdjFusedArgs<float>& a) {
    switch (w) {
        case 4: return goa<4>(m, grid, lds, st, a);
        case 2: return goa<2>(m, grid, lds, st, a);
        case 1: return goa<1>(m, grid, lds, st, a);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tdse
