// Half-step kernel instances for double state, 1-element vectors.
#include "dispatch.hpp"

namespace tdse {

hipError_t launch_half_f64_w1(int g, int rows, int mode, dim3 grid, dim3 block, hipStream_t st,
                              const HalfArgs<double>& a, hipEvent_t e0, hipEvent_t e1) {
    return launch_groups<double, 1>(g, rows, mode, grid, block, st, a, e0, e1);
}

}  // namespace tdse
