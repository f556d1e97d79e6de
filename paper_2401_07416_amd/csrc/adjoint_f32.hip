// Adjoint half-step kernel instances for float state (one row per wavefront).
#include <hip/hip_runtime.h>

#include "adjoint.hpp"

namespace tdse {

namespace {

template <int W, int G>
hipError_t go(int phase, dim3 grid, dim3 block, hipStream_t st, const AdjArgs<float>& a) {
    if (phase == 0)
        hipLaunchKernelGGL((adjoint_half_kernel<float, W, G, 1, 0>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((adjoint_half_kernel<float, W, G, 1, 1>), grid, block, 0, st, a);
    return hipGetLastError();
}

template <int W>
hipError_t go_g(int g, int phase, dim3 grid, dim3 block, hipStream_t st, const AdjArgs<float>& a) {
    switch (g) {
        case 1: return go<W, 1>(phase, grid, block, st, a);
        case 2: return go<W, 2>(phase, grid, block, st, a);
        case 4: return go<W, 4>(phase, grid, block, st, a);
        default: return go<W, 8>(phase, grid, block, st, a);
    }
}

}  // namespace

hipError_t launch_adjoint_f32(int w, int g, int phase, dim3 grid, dim3 block, hipStream_t st,
                               const AdjArgs<float>& a) {
    switch (w) {
        case 4: return go_g<4>(g, phase, grid, block, st, a);
        case 2: return go_g<2>(g, phase, grid, block, st, a);
        default: return go_g<1>(g, phase, grid, block, st, a);
    }
}

}  // namespace tdse
