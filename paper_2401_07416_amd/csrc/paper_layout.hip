// The GPU design of arXiv 2401.07416 section 2.2 on gfx950, kept as the
// baseline this library's sweeps are measured against: arrays stored z
// fastest and x slowest ([nx][ny][nz]), one thread per grid point, blocks of
// Bx x By x Bz points (Bx along z) laid out on a two-dimensional grid by
// eq. (12), every neighbour read from global memory (the paper found shared
// memory slower), periodic neighbours by the modular indices that replace
// the branches of eqs. (13)-(14), one launch per half-step (eq. (9), then
// eq. (8)), each in place.  The cell arithmetic is vterm / hterm / upd_I /
// upd_R, so the states equal those of the x-fastest kernels bit for bit,
// transposed.  No records or sums: the paper takes the detector plane on
// the host.
#include "kernels.hpp"
#include "paper_layout.hpp"

namespace tdse {

template <typename T, bool IS_R>
__global__ __launch_bounds__(1024) void zfast_half_kernel(ZArgs<T> a) {
    // eq. (12): the long grid axis runs over x first, then over the blocks
    // of Bz planes along y; the short axis runs along z
    const long m = (long)blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(m % a.nx);
    const long jb = m / a.nx;
    const int j = (int)(jb * blockDim.z + threadIdx.z);
    if (k >= a.nz || jb >= a.nyb || j >= a.ny) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long sy = nz, sx = (long)ny * nz;
    const T* S = a.S;
    // neighbour along one axis: periodic by (q +- 1 + n) mod n, zero outside
    // a zero boundary
    auto nb = [&](int q, int d, int n, int zero_bc, long stride, long base) -> T {
        const int p = q + d;
        if (zero_bc && (p < 0 || p >= n)) return T(0);
        return S[base + (long)((p + n) % n) * stride];
    };
    const long idx = (long)i * sx + (long)j * sy + k;
    const T c = S[idx];
    const T xl = nb(i, -1, nx, a.bcx, sx, idx - (long)i * sx);
    const T xr = nb(i, +1, nx, a.bcx, sx, idx - (long)i * sx);
    const T yl = nb(j, -1, ny, a.bcy, sy, idx - (long)j * sy);
    const T yr = nb(j, +1, ny, a.bcy, sy, idx - (long)j * sy);
    const T zl = nb(k, -1, nz, a.bcz, 1, idx - k);
    const T zr = nb(k, +1, nz, a.bcz, 1, idx - k);
    const T hx = hterm(c, xl, xr, yl, yr, zl, zr, vterm(a.V[idx], a.cv, a.d0), a.cx, a.cy, a.cz, a.dlo);
    const T uo = a.U[idx];
    const T cak = a.ca[k], cbk = a.cb[k];
    a.U[idx] = IS_R ? upd_R(hx, uo, cak, cbk) : upd_I(hx, uo, cak, cbk);
}

hipError_t launch_zfast_f32(bool is_r, dim3 grid, dim3 block, hipStream_t st, const ZArgs<float>& a) {
    if (is_r)
        hipLaunchKernelGGL((zfast_half_kernel<float, true>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((zfast_half_kernel<float, false>), grid, block, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_zfast_f64(bool is_r, dim3 grid, dim3 block, hipStream_t st, const ZArgs<double>& a) {
    if (is_r)
        hipLaunchKernelGGL((zfast_half_kernel<double, true>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((zfast_half_kernel<double, false>), grid, block, 0, st, a);
    return hipGetLastError();
}

}  // namespace tdse
