// One-pass leapfrog step: eq. (9) and eq. (8) of arXiv 2401.07416 section
// 2.1 fused into one sweep, reading (R^n, I^{n-1/2}, V) once and writing
// (R^{n+1}, I^{n+1/2}) once into a second pair of buffers (ping-pong: the
// sweep reads neighbours of cells other workgroups update, so it cannot work
// in place).  It moves 20 B per cell-step in FP32 (40 in FP64) instead of the
// 32 (64) of two in-place half-step sweeps.
//
// Mapping.  A workgroup owns a band of TY consecutive full x rows and a chunk
// of zc planes and marches z.  Per plane p it first forms I^{n+1/2}(p+1) on
// the band plus one halo row on each side (phase A), then R^{n+1}(p) on the
// band (phase B).  Each thread owns M rows of phase A (rows rs, rs + RPP, ...
// of the band+halo, RPP = rows per pass) and W consecutive x values of each;
// it keeps the z neighbours in registers: R at planes p, p+1, p+2 and
// I^{n+1/2} at p-1, p, p+1.  The x and y neighbours of the centre planes go
// through LDS: R(p+1) on the band plus two halo rows, I^{n+1/2}(p) on the
// band plus one halo row (double-buffered).  Two barriers per plane.
//
// Cell arithmetic is the same expression as the two-pass kernel (lap7,
// update_I, update_R of kernels.hpp), so both paths give identical bits.
#pragma once

#include "kernels.hpp"

namespace tdse {

template <typename T>
struct FusedArgs {
    const T* R0;  // R^n
    const T* I0;  // I^{n-1/2}
    T* R1;        // R^{n+1}
    T* I1;        // I^{n+1/2}
    const T* V;
    const T* ca;
    const T* cb;
    T cx, cy, cz, cv;
    int nx, ny, nz;
    int tpr, rpp, ty;      // threads per row, rows per pass, band rows
    int nbands, zc, nzc, nwg;
    int bcx, bcy, bcz;
    int k_det, k_up;
    double* flux_slots;    // [2][nbands]
    T* rec_plane;
    double* part_q;        // [nzc][nbands]
    double* part_naive;
    double* part_plane;    // [nbands]
    double* pixel;
    double pixel_w;
};

template <typename T, int W, int M, bool REC>
__global__ __launch_bounds__(256) void fused_step_kernel(FusedArgs<T> a) {
    using VT = vec_t<T, W>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* LR = reinterpret_cast<T*>(smem_raw);                  // [ty + 4][nx]
    T* LI = LR + (size_t)(a.ty + 4) * a.nx;                   // [2][ty + 2][nx]
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long plane = (long)nx * ny;
    const int tid = threadIdx.x;
    const int rs = tid / a.tpr;            // row slot within a pass
    const int xs = tid - rs * a.tpr;       // x slot
    const bool live = rs < a.rpp;          // threads past the last full row idle
    const int x0 = (live ? xs : 0) * W;
    const int L = xcd_remap(blockIdx.x, a.nwg);
    const int zchunk = L / a.nbands;
    const int band = L - zchunk * a.nbands;
    const int j0 = band * a.ty;
    const int k0 = zchunk * a.zc;
    const int k1 = min(k0 + a.zc, nz);
    const int TY = a.ty;

    // global row of band row b (b = 0 is the halo row j0 - 1); -1 = zero row
    // (the halo reaches two rows / planes out, which can wrap more than once
    // on an axis of length 1)
    auto grow = [&](int b) -> int {
        int j = j0 - 1 + b;
        if (j < 0) return a.bcy ? -1 : ((j % ny) + ny) % ny;
        if (j >= ny) return a.bcy ? -1 : j % ny;
        return j;
    };
    auto gplane = [&](int p) -> int {
        if (p < 0) return a.bcz ? -1 : ((p % nz) + nz) % nz;
        if (p >= nz) return a.bcz ? -1 : p % nz;
        return p;
    };
    auto ld = [&](const T* base, int j, int p) -> VT {
        VT r;
        if (j < 0 || p < 0 || !live) {
#pragma unroll
            for (int e = 0; e < W; ++e) r.v[e] = T(0);
            return r;
        }
        return ldv<T, W>(base + (long)p * plane + (long)j * nx + x0);
    };

    int rowb[M];   // band row of owned row i
    int rowj[M];   // its global row (-1: zero row)
    bool isB[M];   // phase-B row inside the grid
#pragma unroll
    for (int i = 0; i < M; ++i) {
        rowb[i] = rs + i * a.rpp;
        rowj[i] = grow(rowb[i]);
        isB[i] = live && rowb[i] >= 1 && rowb[i] <= TY && (j0 - 1 + rowb[i]) < ny;
    }
    // the two extra R rows of the LDS band (global j0 - 2 and j0 + TY + 1)
    const bool halo_lo = live && rs == 0;
    const bool halo_hi = live && rs == a.rpp - 1;
    const int jh_lo = grow(-1), jh_hi = grow(TY + 2);

    VT Rz[3][M], Iz[3][M], Vk[M];

    // LDS accessors: LR rows are band rows -1 .. TY+2 (index b + 1), LI rows
    // are band rows 0 .. TY+1
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

    // phase A for plane p: I^{n+1/2}(p) on the owned rows from the R window
    // (planes p-1, p, p+1 in Rz[0..2]); result into Iz[slot] and LDS buffer.
    auto phase_a = [&](int p, int slot, bool store) {
        const int gp = gplane(p);
        // stage R(p) of the band (+ halo rows) in LDS
        if (live) {
#pragma unroll
            for (int i = 0; i < M; ++i)
                if (rowb[i] <= TY + 1) *reinterpret_cast<VT*>(lr_row(rowb[i]) + x0) = Rz[1][i];
            if (halo_lo) *reinterpret_cast<VT*>(lr_row(-1) + x0) = ld(a.R0, jh_lo, gp);
            if (halo_hi) *reinterpret_cast<VT*>(lr_row(TY + 2) + x0) = ld(a.R0, jh_hi, gp);
        }
        VT io[M], vv[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
            io[i] = ld(a.I0, rowj[i], gp);
            vv[i] = ld(a.V, rowj[i], gp);
        }
        __syncthreads();
        const T cap = gp >= 0 ? a.ca[gp] : T(1);
        const T cbp = gp >= 0 ? a.cb[gp] : T(1);
        const int buf = (p - k0 + 2) & 1;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            VT out;
            const int b = rowb[i];
            const bool zero = (gp < 0) || (rowj[i] < 0);
            if (live && b <= TY + 1) {
                const T* rc = lr_row(b);
                const T* ru = lr_row(b - 1);
                const T* rd = lr_row(b + 1);
                const VT yl = *reinterpret_cast<const VT*>(ru + x0);
                const VT yr = *reinterpret_cast<const VT*>(rd + x0);
                const T xle = xl_of(rc), xre = xr_of(rc);
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    const T c = Rz[1][i].v[e];
                    const T xl = e > 0 ? Rz[1][i].v[e - 1] : xle;
                    const T xr = e < W - 1 ? Rz[1][i].v[e + 1] : xre;
                    const T lap = lap7(c, xl, xr, yl.v[e], yr.v[e], Rz[0][i].v[e], Rz[2][i].v[e],
                                       a.cx, a.cy, a.cz);
                    out.v[e] = zero ? T(0) : update_I(lap, vv[i].v[e], c, io[i].v[e], a.cv, cap, cbp);
                }
                *reinterpret_cast<VT*>(li_row(buf, b) + x0) = out;
                if (store && isB[i])
                    stv<T, W>(a.I1 + (long)gp * plane + (long)rowj[i] * nx + x0, out);
            } else {
#pragma unroll
                for (int e = 0; e < W; ++e) out.v[e] = T(0);
            }
            Iz[slot][i] = out;
            Vk[i] = vv[i];
        }
    };

    // R window for the prologue: planes k0-2, k0-1, k0
#pragma unroll
    for (int i = 0; i < M; ++i) {
        Rz[0][i] = ld(a.R0, rowj[i], gplane(k0 - 2));
        Rz[1][i] = ld(a.R0, rowj[i], gplane(k0 - 1));
        Rz[2][i] = ld(a.R0, rowj[i], gplane(k0));
    }
    phase_a(k0 - 1, 0, false);       // I^{n+1/2}(k0-1), neighbour only
    __syncthreads();                  // LR is rewritten next
#pragma unroll
    for (int i = 0; i < M; ++i) {
        Rz[0][i] = Rz[1][i];
        Rz[1][i] = Rz[2][i];
        Rz[2][i] = ld(a.R0, rowj[i], gplane(k0 + 1));
    }
    phase_a(k0, 1, true);             // I^{n+1/2}(k0)
    // Vk now holds V(k0)

    double f0 = 0.0, f1 = 0.0, q = 0.0, nv = 0.0, pl = 0.0;
    for (int k = k0; k < k1; ++k) {
        // R window to planes k, k+1, k+2
#pragma unroll
        for (int i = 0; i < M; ++i) {
            Rz[0][i] = Rz[1][i];
            Rz[1][i] = Rz[2][i];
            Rz[2][i] = ld(a.R0, rowj[i], gplane(k + 2));
        }
        VT vk[M];
#pragma unroll
        for (int i = 0; i < M; ++i) vk[i] = Vk[i];
        __syncthreads();                 // all phase-B reads of the previous plane done
        phase_a(k + 1, 2, k + 1 < k1);   // I^{n+1/2}(k+1); barrier inside
        // phase B for plane k: R^{n+1}(k) = eq. (8) from I^{n+1/2}(k-1..k+1)
        const int buf = (k - k0 + 2) & 1;
        const T cak = a.ca[k];
        const T cbk = a.cb[k];
        const bool at_det = (k == a.k_det), at_up = (k == a.k_up);
#pragma unroll
        for (int i = 0; i < M; ++i) {
            if (!isB[i]) continue;
            const int b = rowb[i];
            const T* ic = li_row(buf, b);
            const VT yl = *reinterpret_cast<const VT*>(li_row(buf, b - 1) + x0);
            const VT yr = *reinterpret_cast<const VT*>(li_row(buf, b + 1) + x0);
            const T xle = xl_of(ic), xre = xr_of(ic);
            VT out;
#pragma unroll
            for (int e = 0; e < W; ++e) {
                const T c = Iz[1][i].v[e];
                const T xl = e > 0 ? Iz[1][i].v[e - 1] : xle;
                const T xr = e < W - 1 ? Iz[1][i].v[e + 1] : xre;
                const T lap = lap7(c, xl, xr, yl.v[e], yr.v[e], Iz[0][i].v[e], Iz[2][i].v[e],
                                   a.cx, a.cy, a.cz);
                const T uo = Rz[0][i].v[e];
                const T un = update_R(lap, vk[i].v[e], c, uo, a.cv, cak, cbk);
                out.v[e] = un;
                if (at_det) f0 += (double)Iz[2][i].v[e] * ((double)uo + (double)un);
                if (at_up) f1 += (double)Iz[0][i].v[e] * ((double)uo + (double)un);
                if (REC) {
                    const double dc = (double)c, du = (double)uo, dn = (double)un;
                    q += dc * dc + du * dn;
                    nv += dn * dn + dc * dc;
                }
            }
            const long off = (long)k * plane + (long)rowj[i] * nx + x0;
            stv<T, W>(a.R1 + off, out);
            if (REC && at_det) {
                VT rv;
                const long poff = (long)rowj[i] * nx + x0;
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    const double dn = (double)out.v[e], dc = (double)Iz[1][i].v[e];
                    const double rho = dn * dn + dc * dc;
                    rv.v[e] = (T)rho;
                    pl += rho;
                    if (a.pixel) a.pixel[poff + e] += a.pixel_w * rho;
                }
                stv<T, W>(a.rec_plane + poff, rv);
            }
        }
        // shift the I window
#pragma unroll
        for (int i = 0; i < M; ++i) {
            Iz[0][i] = Iz[1][i];
            Iz[1][i] = Iz[2][i];
        }
    }

    // fixed-order workgroup sums of the partials
    __shared__ double red[256];
    const bool has_det = (a.k_det >= k0 && a.k_det < k1);
    const bool has_up = (a.k_up >= k0 && a.k_up < k1);
    auto wg_sum = [&](double v) -> double {
        __syncthreads();
        red[tid] = v;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (tid < o && tid + o < (int)blockDim.x) red[tid] += red[tid + o];
            __syncthreads();
        }
        return red[0];
    };
    if (has_det) {
        const double s = wg_sum(f0);
        if (tid == 0) a.flux_slots[band] = s;
    }
    if (has_up) {
        const double s = wg_sum(f1);
        if (tid == 0) a.flux_slots[a.nbands + band] = s;
    }
    if (REC) {
        const double sq = wg_sum(q);
        const double sn = wg_sum(nv);
        const long slot = (long)zchunk * a.nbands + band;
        if (tid == 0) {
            a.part_q[slot] = sq;
            a.part_naive[slot] = sn;
        }
        if (has_det) {
            const double sp = wg_sum(pl);
            if (tid == 0) a.part_plane[band] = sp;
        }
    }
}

}  // namespace tdse
