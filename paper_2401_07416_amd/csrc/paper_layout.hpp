// Arguments and launchers of the z-fastest half-step kernels that follow the
// GPU design of arXiv 2401.07416 section 2.2 (eq. (12) mapping, no shared
// memory, one launch per half-step).
#pragma once

#include <hip/hip_runtime.h>

namespace tdse {

template <typename T>
struct ZArgs {
    T* U;          // own-cell operand, updated in place
    const T* S;    // stencil operand
    const T* V;
    const T* ca;   // [nz] CAP tables
    const T* cb;
    T cx, cy, cz, cv;
    T d0, dlo;     // 2 (cx + cy + cz) as hi + lo parts
    int nx, ny, nz;
    int bcx, bcy, bcz;
    int nyb;       // blocks of Bz planes along y
};

hipError_t launch_zfast_f32(bool is_r, dim3 grid, dim3 block, hipStream_t st, const ZArgs<float>& a);
hipError_t launch_zfast_f64(bool is_r, dim3 grid, dim3 block, hipStream_t st, const ZArgs<double>& a);

}  // namespace tdse
