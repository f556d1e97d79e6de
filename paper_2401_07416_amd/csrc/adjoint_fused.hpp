// One-pass reverse step of the adjoint (arXiv 2401.07416 section 2.1, the
// transpose of one leapfrog step; see adjoint.hpp for the two-phase form):
//   i_t   = i + G (B r)                       phase A, plane p+1
//   r'    = A r - G (B i_t),  i' = A i_t      phase B, plane p
//   dL/dV += cv (B r) o I^{n+1/2} - cv (B i_t) o R^n
// in one z-marching sweep with the band mapping of the one-pass forward step
// (fused.hpp): a workgroup owns TY full x rows of a chunk of planes; phase A
// forms i_t on the band plus one halo row each side from the r window in
// registers and the centre plane of r in LDS, phase B forms r', i' and the
// dL/dV update on the band from the i_t window and its centre plane in LDS.
// It reads r, i, V, R^n, I^{n+1/2}, dL/dV once and writes r', i', dL/dV once
// (36 B per cell-step in FP32) where the two phase kernels move 52 B; r' and
// i' go to second buffers because neighbouring workgroups still read r.
//
// The products, sums and their order are those of the two phase kernels
// (each neighbour is scaled by cb of its plane before the 7-point sum), so
// both forms give the same bits.
#pragma once

#include "kernels.hpp"

namespace tdse {

template <typename T>
struct AdjFusedArgs {
    const T* r;    // dL/dR^{n+1}
    const T* i;    // dL/dI^{n+1/2}
    T* r_out;      // dL/dR^n
    T* i_out;      // dL/dI^{n-1/2}
    const T* V;
    const T* Rn;   // R^n
    const T* Ih;   // I^{n+1/2}
    T* gv;         // dL/dV accumulator (state precision), in place
    const T* ca;
    const T* cb;
    T cx, cy, cz, cv;
    int nx, ny, nz;
    int tpr, rpp, ty, nbands, zc, nzc, nwg;
    int bcx, bcy, bcz;
};

template <typename T, int W, int M>
__global__ __launch_bounds__(256) void adjoint_fused_kernel(AdjFusedArgs<T> a) {
    using VT = vec_t<T, W>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* LR = reinterpret_cast<T*>(smem_raw);                  // [ty + 4][nx] raw r
    T* LI = LR + (size_t)(a.ty + 4) * a.nx;                   // [2][ty + 2][nx] raw i_t
    const int L = xcd_remap(blockIdx.x, a.nwg);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int tid = threadIdx.x;
    const int rs = tid / a.tpr;
    const int xs = tid - rs * a.tpr;
    const bool live = rs < a.rpp;
    const int x0 = (live ? xs : 0) * W;
    const int zchunk = L / a.nbands;
    const int band = L - zchunk * a.nbands;
    const int j0 = band * a.ty;
    const int k0 = zchunk * a.zc;
    const int k1 = min(k0 + a.zc, nz);
    const int TY = a.ty;

    auto grow = [&](int b) -> int {
        int j = j0 - 1 + b;
        if (j < 0) return a.bcy ? -1 : ((j % ny) + ny) % ny;
        if (j >= ny) return a.bcy ? -1 : j % ny;
        return j;
    };
    auto gplane = [&](int p) -> int {
        if (p < 0) {
            if (a.bcz) return -1;
            do p += nz; while (p < 0);
        } else if (p >= nz) {
            if (a.bcz) return -1;
            do p -= nz; while (p >= nz);
        }
        return p;
    };
    const int pbytes = (int)((long)nx * ny * (long)sizeof(T));
    auto prs = [&](const T* base, int gp) {
        return plane_rsrc(base + (long)(gp < 0 ? 0 : gp) * nx * ny, gp < 0 ? 0 : pbytes);
    };
    // cb of a plane; a zero plane only ever scales zeros
    auto cb_of = [&](int gp) -> T { return gp >= 0 ? ld_uniform(a.cb, gp) : T(0); };

    int rowb[M], rowj[M], voff[M], voffB[M];
    bool isB[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        rowb[i] = rs + i * a.rpp;
        rowj[i] = grow(rowb[i]);
        isB[i] = live && rowb[i] >= 1 && rowb[i] <= TY && (j0 - 1 + rowb[i]) < ny;
        voff[i] = (live && rowj[i] >= 0) ? (rowj[i] * nx + x0) * (int)sizeof(T) : OOB;
        voffB[i] = isB[i] ? voff[i] : OOB;
    }
    const bool halo_lo = live && rs == 0;
    const bool halo_hi = live && rs == a.rpp - 1;
    const int jh_lo = grow(-1), jh_hi = grow(TY + 2);
    const int voff_lo = (halo_lo && jh_lo >= 0) ? (jh_lo * nx + x0) * (int)sizeof(T) : OOB;
    const int voff_hi = (halo_hi && jh_hi >= 0) ? (jh_hi * nx + x0) * (int)sizeof(T) : OOB;

    auto lr_row = [&](int b) -> T* { return LR + (size_t)(b + 1) * nx; };
    auto li_row = [&](int buf, int b) -> T* { return LI + ((size_t)buf * (TY + 2) + b) * nx; };
    auto xl_of = [&](const T* row) -> T {
        const int x = x0 - 1;
        if (x < 0) return a.bcx ? T(0) : row[nx - 1];
        return row[x];
    };
    auto xr_of = [&](const T* row) -> T {
        const int x = x0 + W;
        if (x >= nx) return a.bcx ? T(0) : row[0];
        return row[x];
    };

    VT Rz[3][M], Iz[3][M], Vk[M];
    auto load_a = [&](int p, VT(&io)[M], VT(&vv)[M], VT& hlo, VT& hhi) {
        const int gp = gplane(p);
        const auto rI = prs(a.i, gp), rV = prs(a.V, gp), rR = prs(a.r, gp);
#pragma unroll
        for (int i = 0; i < M; ++i) {
            io[i] = bload<T, W>(rI, voff[i]);
            vv[i] = bload<T, W>(rV, voff[i]);
        }
        hlo = bload<T, W>(rR, voff_lo);
        hhi = bload<T, W>(rR, voff_hi);
    };
    auto load_r = [&](int p, VT(&out)[M]) {
        const auto rR = prs(a.r, gplane(p));
#pragma unroll
        for (int i = 0; i < M; ++i) out[i] = bload<T, W>(rR, voff[i]);
    };
    auto stage = [&](const VT& hlo, const VT& hhi) {
        if (live) {
#pragma unroll
            for (int i = 0; i < M; ++i)
                if (rowb[i] <= TY + 1) *reinterpret_cast<VT*>(lr_row(rowb[i]) + x0) = Rz[1][i];
            if (halo_lo) *reinterpret_cast<VT*>(lr_row(-1) + x0) = hlo;
            if (halo_hi) *reinterpret_cast<VT*>(lr_row(TY + 2) + x0) = hhi;
        }
    };
    // phase A on plane p: i_t = i + G (B r) from the r window (planes p-1,
    // p, p+1 in Rz, centre plane in LDS); into outI and the LDS buffer of p
    auto compute_a = [&](int p, const VT(&io)[M], const VT(&vv)[M], VT(&outI)[M]) {
        const int gp = gplane(p);
        const T cbc = cb_of(gp), cbl = cb_of(gplane(p - 1)), cbh = cb_of(gplane(p + 1));
        const int buf = (p - k0 + 2) & 1;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            VT out;
            const int b = rowb[i];
            const bool zero = (gp < 0) || (rowj[i] < 0);
            if (live && b <= TY + 1) {
                const T* rc = lr_row(b);
                const VT yl = *reinterpret_cast<const VT*>(lr_row(b - 1) + x0);
                const VT yr = *reinterpret_cast<const VT*>(lr_row(b + 1) + x0);
                const T xle = xl_of(rc), xre = xr_of(rc);
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    const T c = cbc * Rz[1][i].v[e];
                    const T xl = cbc * (e > 0 ? Rz[1][i].v[e - 1] : xle);
                    const T xr = cbc * (e < W - 1 ? Rz[1][i].v[e + 1] : xre);
                    const T lap = lap7(c, xl, xr, cbc * yl.v[e], cbc * yr.v[e], cbl * Rz[0][i].v[e],
                                       cbh * Rz[2][i].v[e], a.cx, a.cy, a.cz);
                    const T gX = -lap + a.cv * vv[i].v[e] * c;
                    out.v[e] = zero ? T(0) : io[i].v[e] + gX;
                }
                *reinterpret_cast<VT*>(li_row(buf, b) + x0) = out;
            } else {
#pragma unroll
                for (int e = 0; e < W; ++e) out.v[e] = T(0);
            }
            outI[i] = out;
        }
    };

    VT io[M], vv[M], hlo, hhi;
    load_r(k0 - 2, Rz[0]);
    load_r(k0 - 1, Rz[1]);
    load_r(k0, Rz[2]);
    load_a(k0 - 1, io, vv, hlo, hhi);
    stage(hlo, hhi);
    __syncthreads();
    compute_a(k0 - 1, io, vv, Iz[0]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < M; ++i) {
        Rz[0][i] = Rz[1][i];
        Rz[1][i] = Rz[2][i];
    }
    load_r(k0 + 1, Rz[2]);
    load_a(k0, io, vv, hlo, hhi);
    stage(hlo, hhi);
    __syncthreads();
    compute_a(k0, io, vv, Iz[1]);
#pragma unroll
    for (int i = 0; i < M; ++i) Vk[i] = vv[i];

    for (int k = k0; k < k1; ++k) {
#pragma unroll
        for (int i = 0; i < M; ++i) {
            Rz[0][i] = Rz[1][i];
            Rz[1][i] = Rz[2][i];
        }
        load_r(k + 2, Rz[2]);
        load_a(k + 1, io, vv, hlo, hhi);
        VT vk[M];
#pragma unroll
        for (int i = 0; i < M; ++i) vk[i] = Vk[i];
        __syncthreads();
        stage(hlo, hhi);
        __syncthreads();
        compute_a(k + 1, io, vv, Iz[2]);
#pragma unroll
        for (int i = 0; i < M; ++i) Vk[i] = vv[i];
        // phase B on plane k
        const int buf = (k - k0 + 2) & 1;
        const T cak = ld_uniform(a.ca, k);
        const T cbk = ld_uniform(a.cb, k);
        const T cbl = cb_of(gplane(k - 1)), cbh = cb_of(gplane(k + 1));
        const auto rRn = prs(a.Rn, k), rIh = prs(a.Ih, k), rG = prs(a.gv, k);
#pragma unroll
        for (int i = 0; i < M; ++i) {
            if (!isB[i]) continue;
            const int b = rowb[i];
            const VT rn = bload<T, W>(rRn, voffB[i]);
            const VT ih = bload<T, W>(rIh, voffB[i]);
            VT gv = bload<T, W>(rG, voffB[i]);
            const T* ic = li_row(buf, b);
            const VT yl = *reinterpret_cast<const VT*>(li_row(buf, b - 1) + x0);
            const VT yr = *reinterpret_cast<const VT*>(li_row(buf, b + 1) + x0);
            const T xle = xl_of(ic), xre = xr_of(ic);
            VT rout, iout;
#pragma unroll
            for (int e = 0; e < W; ++e) {
                const T c = cbk * Iz[1][i].v[e];
                const T xl = cbk * (e > 0 ? Iz[1][i].v[e - 1] : xle);
                const T xr = cbk * (e < W - 1 ? Iz[1][i].v[e + 1] : xre);
                const T lap = lap7(c, xl, xr, cbk * yl.v[e], cbk * yr.v[e], cbl * Iz[0][i].v[e],
                                   cbh * Iz[2][i].v[e], a.cx, a.cy, a.cz);
                const T gX = -lap + a.cv * vk[i].v[e] * c;
                const T uo = Rz[0][i].v[e];
                rout.v[e] = cak * uo - gX;
                const T tr = cbk * uo;
                gv.v[e] = (gv.v[e] + a.cv * tr * ih.v[e]) - a.cv * c * rn.v[e];
                iout.v[e] = cak * Iz[1][i].v[e];
            }
            bstore<T, W>(prs(a.r_out, k), voffB[i], rout);
            bstore<T, W>(prs(a.i_out, k), voffB[i], iout);
            bstore<T, W>(rG, voffB[i], gv);
        }
#pragma unroll
        for (int i = 0; i < M; ++i) {
            Iz[0][i] = Iz[1][i];
            Iz[1][i] = Iz[2][i];
        }
    }
}

}  // namespace tdse
