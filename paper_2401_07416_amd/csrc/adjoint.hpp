// Reverse-mode adjoint of the leapfrog of arXiv 2401.07416 section 2.1.
//
// With G X = -(cx dxx + cy dyy + cz dzz) X + cv V X (symmetric), A = diag(ca_k),
// B = diag(cb_k), one forward step is
//   I^{n+1/2} = A I^{n-1/2} - B G R^n            (eq. (9) with the CAP)
//   R^{n+1}   = A R^n + B G I^{n+1/2}            (eq. (8) with the CAP)
// and its transpose, applied from r = dL/dR^{n+1}, i = dL/dI^{n+1/2}, is
//   i_t = i + G (B r)                              adjoint phase A
//   r  <- A r - G (B i_t),   i <- A i_t            adjoint phase B
//   dL/dV += cv (B r) o I^{n+1/2} - cv (B i_t) o R^n
// followed by the record injections of level n.  Phase A is a stencil of r,
// phase B a stencil of i_t; each kernel updates its own-cell operand in
// place (it is never a stencil input of the same kernel) and phase B writes
// A i_t to a second buffer.  The mapping is that of the two-pass kernel: a
// wavefront owns RY full x rows and marches a chunk of z planes, z
// neighbours in registers, x neighbours by lane permutes.  The per-plane
// scaling by cb is applied to each loaded value (cb_p * X(p)), exactly the
// product the reference forms before its stencil.
#pragma once

#include "kernels.hpp"

namespace tdse {

template <typename T>
struct AdjArgs {
    const T* S;      // stencil input: r (phase A) or i_t (phase B)
    T* U;            // in place: i (A) or r (B)
    T* U2;           // phase B: A i_t
    const T* V;
    const T* Rn;     // phase B: R^n
    const T* Ih;     // phase B: I^{n+1/2}
    T* gv;           // phase B: dL/dV accumulator (state precision)
    const T* ca;
    const T* cb;
    T cx, cy, cz, cv;
    int nx, ny, nz, nl;
    int ytiles, wpg, ywg, zc, nzc, nwg;
    int bcx, bcy, bcz;
};

template <typename T, int W, int G, int RY, int PHASE>
__global__ __launch_bounds__(256) void adjoint_half_kernel(AdjArgs<T> a) {
    using VT = vec_t<T, W>;
    const int lane = threadIdx.x;
    const int L = xcd_remap(blockIdx.x, a.nwg);
    const int zchunk = L / a.ywg;
    const int ytile = (L - zchunk * a.ywg) * a.wpg + threadIdx.y;
    if (ytile >= a.ytiles) return;
    const bool act = lane < a.nl;
    const int lc = act ? lane : 0;
    const int nx = a.nx, ny = a.ny, nz = a.nz, nl = a.nl;
    const long plane = (long)nx * ny;
    const int j0 = ytile * RY;
    const int k0 = zchunk * a.zc;
    const int k1 = min(k0 + a.zc, nz);
    int jrow[RY];
    bool real[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int jj = j0 + r;
        real[r] = jj < ny;
        jrow[r] = real[r] ? jj : (a.bcy ? -1 : jj % ny);
    }
    const int jlo = (j0 > 0) ? j0 - 1 : (a.bcy ? -1 : ny - 1);
    const int jhi = (j0 + RY < ny) ? j0 + RY : (a.bcy ? -1 : (j0 + RY) % ny);
    auto kwrap = [&](int kk) -> int {
        if (kk < 0) return a.bcz ? -1 : kk + nz;
        if (kk >= nz) return a.bcz ? -1 : kk - nz;
        return kk;
    };
    // row of X at plane kk scaled by cb_kk (zero outside a zero boundary)
    auto load_scaled = [&](const T* base, int jj, int kk, VT(&out)[G]) {
        if (jj < 0 || kk < 0) {
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int e = 0; e < W; ++e) out[g].v[e] = T(0);
            return;
        }
        const T s = ld_uniform(a.cb, kk);
        const T* p = base + (long)kk * plane + (long)jj * nx + (long)lc * W;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            VT v = ldv<T, W>(p + (long)g * nl * W);
#pragma unroll
            for (int e = 0; e < W; ++e) out[g].v[e] = s * v.v[e];
        }
    };
    auto load_row = [&](const T* base, int jj, int kk, VT(&out)[G]) {
        const T* p = base + (long)kk * plane + (long)jj * nx + (long)lc * W;
#pragma unroll
        for (int g = 0; g < G; ++g) out[g] = ldv<T, W>(p + (long)g * nl * W);
    };

    VT sp[RY][G], sc[RY][G], sn[RY][G];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        load_scaled(a.S, jrow[r], kwrap(k0 - 1), sp[r]);
        load_scaled(a.S, jrow[r], k0, sc[r]);
    }
    const int src_l = (lane == 0) ? nl - 1 : lane - 1;
    const int src_r = (lane == nl - 1) ? 0 : lane + 1;
    for (int k = k0; k < k1; ++k) {
        VT hl[G], hh[G];
#pragma unroll
        for (int r = 0; r < RY; ++r) load_scaled(a.S, jrow[r], kwrap(k + 1), sn[r]);
        load_scaled(a.S, jlo, k, hl);
        load_scaled(a.S, jhi, k, hh);
        const T cak = ld_uniform(a.ca, k);
        const T cbk = ld_uniform(a.cb, k);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (!real[r]) continue;
            VT u[G], vv[G], rn[G], ih[G], gv[G], un[G], u2[G];
            load_row(a.U, jrow[r], k, u);
            load_row(a.V, jrow[r], k, vv);
            if (PHASE == 1) {
                load_row(a.Rn, jrow[r], k, rn);
                load_row(a.Ih, jrow[r], k, ih);
                load_row(a.gv, jrow[r], k, gv);
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const T give_l = (lane == nl - 1) ? sc[r][(g + G - 1) % G].v[W - 1] : sc[r][g].v[W - 1];
                const T give_r = (lane == 0) ? sc[r][(g + 1) % G].v[0] : sc[r][g].v[0];
                T xl_edge = __shfl(give_l, src_l, 64);
                T xr_edge = __shfl(give_r, src_r, 64);
                if (a.bcx) {
                    if (lane == 0 && g == 0) xl_edge = T(0);
                    if (lane == nl - 1 && g == G - 1) xr_edge = T(0);
                }
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    const T c = sc[r][g].v[e];  // cb_k * X
                    const T xl = (e > 0) ? sc[r][g].v[e - 1] : xl_edge;
                    const T xr = (e < W - 1) ? sc[r][g].v[e + 1] : xr_edge;
                    const T yl = (r > 0) ? sc[r - 1][g].v[e] : hl[g].v[e];
                    const T yr = (r < RY - 1) ? sc[r + 1][g].v[e] : hh[g].v[e];
                    const T lap = lap7(c, xl, xr, yl, yr, sp[r][g].v[e], sn[r][g].v[e], a.cx, a.cy, a.cz);
                    const T gX = -lap + a.cv * vv[g].v[e] * c;  // G (B X) at the cell
                    const T uo = u[g].v[e];
                    if (PHASE == 0) {
                        un[g].v[e] = uo + gX;                     // i_t = i + G (B r)
                    } else {
                        un[g].v[e] = cak * uo - gX;               // r <- A r - G (B i_t)
                        // A i_t: the unscaled own value is the stencil centre / cb, so
                        // reload it from memory instead of dividing
                        const T tr = cbk * uo;                    // B r (old r)
                        gv[g].v[e] = (gv[g].v[e] + a.cv * tr * ih[g].v[e]) - a.cv * c * rn[g].v[e];
                    }
                }
            }
            if (act) {
                const long off = (long)k * plane + (long)jrow[r] * nx + (long)lc * W;
#pragma unroll
                for (int g = 0; g < G; ++g) stv<T, W>(a.U + off + (long)g * nl * W, un[g]);
                if (PHASE == 1) {
                    VT it[G];
                    load_row(a.S, jrow[r], k, it);
#pragma unroll
                    for (int g = 0; g < G; ++g) {
#pragma unroll
                        for (int e = 0; e < W; ++e) u2[g].v[e] = cak * it[g].v[e];
                        stv<T, W>(a.U2 + off + (long)g * nl * W, u2[g]);
                        stv<T, W>(a.gv + off + (long)g * nl * W, gv[g]);
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int g = 0; g < G; ++g) {
                sp[r][g] = sc[r][g];
                sc[r][g] = sn[r][g];
            }
    }
}

// Record injection at level m on plane k_det:
//   r += 2 R^m o rho_bar,  i += 2 I^{m-1/2} o rho_bar
template <typename T>
__global__ __launch_bounds__(256) void adjoint_inject_kernel(T* r, T* i, const T* Rm, const T* Im,
                                                             const T* rho_bar, long plane_off,
                                                             long n) {
    const long c = (long)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    const long o = plane_off + c;
    const T w = rho_bar[c];
    r[o] = r[o] + T(2) * Rm[o] * w;
    i[o] = i[o] + T(2) * Im[o] * w;
}

// dL/dV in FP64 += the state-precision segment accumulator, which restarts.
template <typename T>
__global__ __launch_bounds__(256) void adjoint_fold_kernel(double* out, T* acc, long n) {
    const long c = (long)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    out[c] += (double)acc[c];
    acc[c] = T(0);
}

}  // namespace tdse
