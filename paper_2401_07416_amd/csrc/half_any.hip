// Half-step kernel for any x extent (arXiv 2401.07416 section 2.1, eq. (9)
// or eq. (8) with the time-centred CAP of eq. (10), periodic or zero
// boundaries of eqs. (13)-(14)).  The vector kernel of kernels.hpp spreads a
// row over the lanes of one wavefront and needs nx = W * G * L with L <= 64;
// this one takes any nx: a workgroup of 256 threads owns one y row of a
// chunk of z planes, each thread the x columns tid, tid + 256, ..., and
// marches z with the stencil array's z neighbours in registers; the x and y
// neighbours are plain loads (the neighbouring threads and rows read the
// same lines, so they come from the caches).  The cell arithmetic is that of
// every other step kernel (vterm / hterm / upd_*), so the states are the
// same bits.  The flux and record partials of a row are reduced in a fixed
// order into slot j of the row (one slot per row and plane, as the vector
// kernel's y tiles of one row each), so finalize_kernel folds them as usual.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace tdse {

template <typename T, int MODE>
__global__ __launch_bounds__(256) void half_any_kernel(HalfArgs<T> a) {
    constexpr bool IS_R = (MODE == MODE_R || MODE == MODE_R_REC);
    constexpr bool REC = (MODE == MODE_R_REC || MODE == MODE_I_PEEK);
    __shared__ double red[4];
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int L = xcd_remap(blockIdx.x, a.nwg);
    const int zchunk = L / ny;
    const int j = L - zchunk * ny;
    const int k0 = zchunk * a.zc;
    const int k1 = min(k0 + a.zc, nz);
    const long plane = (long)nx * ny;
    const int jl = j > 0 ? j - 1 : (a.bcy ? -1 : ny - 1);
    const int jr = j + 1 < ny ? j + 1 : (a.bcy ? -1 : 0);
    auto kwrap = [&](int kk) -> int {
        if (kk < 0) return a.bcz ? -1 : kk + nz;
        if (kk >= nz) return a.bcz ? -1 : kk - nz;
        return kk;
    };
    // S at (plane kk, row jj, column xx); an index of -1 reads zero
    auto at = [&](int kk, int jj, int xx) -> T {
        if (kk < 0 || jj < 0 || xx < 0) return T(0);
        return a.S[(long)kk * plane + (long)jj * nx + xx];
    };
    double f0 = 0.0, f1 = 0.0, q = 0.0, nv = 0.0, pl = 0.0;
    for (int x = threadIdx.x; x < nx; x += 256) {
        const int xl_i = x > 0 ? x - 1 : (a.bcx ? -1 : nx - 1);
        const int xr_i = x + 1 < nx ? x + 1 : (a.bcx ? -1 : 0);
        T sp = at(kwrap(k0 - 1), j, x);
        T sc = at(k0, j, x);
        for (int k = k0; k < k1; ++k) {
            const T sn = at(kwrap(k + 1), j, x);
            const T xl = at(k, j, xl_i), xr = at(k, j, xr_i);
            const T yl = at(k, jl, x), yr = at(k, jr, x);
            const long idx = (long)k * plane + (long)j * nx + x;
            const T uo = a.U[idx];
            const T cak = ld_uniform(a.ca, k);
            const T cbk = ld_uniform(a.cb, k);
            const T hx = hterm(sc, xl, xr, yl, yr, sp, sn, vterm(a.V[idx], a.cv, a.d0), a.cx, a.cy, a.cz,
                               a.dlo);
            const T un = IS_R ? upd_R(hx, uo, cak, cbk) : upd_I(hx, uo, cak, cbk);
            if (MODE != MODE_I_PEEK) a.U[idx] = un;
            if (IS_R) {
                if (k == a.k_det) f0 += (double)sn * ((double)uo + (double)un);
                if (k == a.k_up) f1 += (double)sp * ((double)uo + (double)un);
            }
            if (REC) {
                const double dc = (double)sc, du = (double)uo, dn = (double)un;
                q += dc * dc + du * dn;
                nv += IS_R ? (dn * dn + dc * dc) : (dc * dc + du * du);
                if (k == a.k_det) {
                    const double dr = IS_R ? dn : du;
                    const double rho = dr * dr + dc * dc;
                    a.rec_plane[(long)j * nx + x] = (T)rho;
                    pl += rho;
                    if (a.pixel) a.pixel[(long)j * nx + x] += a.pixel_w * rho;
                }
            }
            sp = sc;
            sc = sn;
        }
    }
    const bool has_det = a.k_det >= k0 && a.k_det < k1;
    const bool has_up = a.k_up >= k0 && a.k_up < k1;
    if (IS_R) {
        if (has_det) {
            const double s = block_sum(f0, red, 4);
            if (threadIdx.x == 0) a.flux_slots[j] = s;
        }
        if (has_up) {
            const double s = block_sum(f1, red, 4);
            if (threadIdx.x == 0) a.flux_slots[a.ytiles + j] = s;
        }
    }
    if (REC) {
        const double sq = block_sum(q, red, 4);
        const double sn_ = block_sum(nv, red, 4);
        if (threadIdx.x == 0) {
            a.part_q[(long)zchunk * a.ytiles + j] = sq;
            a.part_naive[(long)zchunk * a.ytiles + j] = sn_;
        }
        if (has_det) {
            const double sp_ = block_sum(pl, red, 4);
            if (threadIdx.x == 0) a.part_plane[j] = sp_;
        }
    }
}

template <typename T>
hipError_t launch_half_any(int mode, dim3 grid, hipStream_t st, const HalfArgs<T>& a, hipEvent_t e0,
                           hipEvent_t e1) {
    auto go = [&](auto kern) -> hipError_t {
        if (e0)
            hipExtLaunchKernelGGL(kern, grid, dim3(256), 0, st, e0, e1, 0, a);
        else
            hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, a);
        return hipGetLastError();
    };
    switch (mode) {
        case MODE_I: return go(half_any_kernel<T, MODE_I>);
        case MODE_R: return go(half_any_kernel<T, MODE_R>);
        case MODE_R_REC: return go(half_any_kernel<T, MODE_R_REC>);
        default: return go(half_any_kernel<T, MODE_I_PEEK>);
    }
}

hipError_t launch_half_any_f32(int mode, dim3 grid, hipStream_t st, const HalfArgs<float>& a,
                               hipEvent_t e0, hipEvent_t e1) {
    return launch_half_any<float>(mode, grid, st, a, e0, e1);
}

hipError_t launch_half_any_f64(int mode, dim3 grid, hipStream_t st, const HalfArgs<double>& a,
                               hipEvent_t e0, hipEvent_t e1) {
    return launch_half_any<double>(mode, grid, st, a, e0, e1);
}

}  // namespace tdse
