// Template dispatch of the half-step kernel over (rows per wave, mode).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace tdse {

template <typename T, int W, int G, int RY>
hipError_t launch_mode(int mode, dim3 grid, dim3 block, hipStream_t st, const HalfArgs<T>& a,
                       hipEvent_t e0, hipEvent_t e1) {
    auto go = [&](auto kern) -> hipError_t {
        if (e0) {
            hipExtLaunchKernelGGL(kern, grid, block, 0, st, e0, e1, 0, a);
        } else {
            hipLaunchKernelGGL(kern, grid, block, 0, st, a);
        }
        return hipGetLastError();
    };
    switch (mode) {
        case MODE_I: return go(half_step_kernel<T, W, G, RY, MODE_I>);
        case MODE_R: return go(half_step_kernel<T, W, G, RY, MODE_R>);
        case MODE_R_REC: return go(half_step_kernel<T, W, G, RY, MODE_R_REC>);
        default: return go(half_step_kernel<T, W, G, RY, MODE_I_PEEK>);
    }
}

template <typename T, int W, int G>
hipError_t launch_rows(int rows, int mode, dim3 grid, dim3 block, hipStream_t st,
                       const HalfArgs<T>& a, hipEvent_t e0, hipEvent_t e1) {
    switch (rows) {
        case 1: return launch_mode<T, W, G, 1>(mode, grid, block, st, a, e0, e1);
        case 2: return launch_mode<T, W, G, 2>(mode, grid, block, st, a, e0, e1);
        case 4: return launch_mode<T, W, G, 4>(mode, grid, block, st, a, e0, e1);
        default: return launch_mode<T, W, G, 8>(mode, grid, block, st, a, e0, e1);
    }
}

template <typename T, int W>
hipError_t launch_groups(int g, int rows, int mode, dim3 grid, dim3 block, hipStream_t st,
                         const HalfArgs<T>& a, hipEvent_t e0, hipEvent_t e1) {
    switch (g) {
        case 1: return launch_rows<T, W, 1>(rows, mode, grid, block, st, a, e0, e1);
        case 2: return launch_rows<T, W, 2>(rows, mode, grid, block, st, a, e0, e1);
        case 4: return launch_rows<T, W, 4>(rows, mode, grid, block, st, a, e0, e1);
        default: return launch_rows<T, W, 8>(rows, mode, grid, block, st, a, e0, e1);
    }
}

}  // namespace tdse
