// Half-step kernel instances for float state, 2-element vectors.
#include "dispatch.hpp"

namespace tdse {

hipError_t launch_half_f32_w2(int g, int rows, int mode, dim3 grid, dim3 block, hipStream_t st,
                              const HalfArgs<float>& a, hipEvent_t e0, hipEvent_t e1) {
    return launch_groups<float, 2>(g, rows, mode, grid, block, st, a, e0, e1);
}

}  // namespace tdse
