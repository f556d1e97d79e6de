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
// Cell arithmetic is the same expression as the two-pass kernel (vterm,
// hterm, upd_I, upd_R of kernels.hpp), so both paths give identical bits.
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
    T d0, dlo;             // 2 (cx + cy + cz) as hi + lo parts
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
    int nt_out;           // non-temporal hint on the R^{n+1}, I^{n+1/2} stores
};

// PF: issue the loads of the next plane (R three planes ahead, I^{n-1/2}
// and V two ahead, the LDS halo rows) before the eq. (8) part of the
// current plane, so their latency hides behind it.
// The body of one workgroup of the one-pass step: logical workgroup L of
// the grid described by a (z chunk L / nbands, band L % nbands), with the
// dynamic LDS at smem_raw.
template <typename T, int W, int M, bool REC, bool PF>
__device__ __forceinline__ void fused_step_body(const FusedArgs<T>& a, int L,
                                                unsigned char* smem_raw) {
    using VT = vec_t<T, W>;
    T* LR = reinterpret_cast<T*>(smem_raw);                  // [ty + 4][nx]
    T* LI = LR + (size_t)(a.ty + 4) * a.nx;                   // [2][ty + 2][nx]
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long plane = (long)nx * ny;
    const int tid = threadIdx.x;
    const int rs = tid / a.tpr;            // row slot within a pass
    const int xs = tid - rs * a.tpr;       // x slot
    const bool live = rs < a.rpp;          // threads past the last full row idle
    const int x0 = (live ? xs : 0) * W;
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
        if (p < 0) {
            if (a.bcz) return -1;
            do p += nz; while (p < 0);
        } else if (p >= nz) {
            if (a.bcz) return -1;
            do p -= nz; while (p >= nz);
        }
        return p;
    };
    // plane resource of an array (size 0 for a zero plane)
    const int pbytes = (int)(plane * (long)sizeof(T));
    auto prs = [&](const T* base, int gp) {
        return plane_rsrc(base + (long)(gp < 0 ? 0 : gp) * plane, gp < 0 ? 0 : pbytes);
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
    // byte offsets within a plane: loads of owned rows, stores of band rows,
    // halo rows; OOB reads zero / drops the store
    int voff[M], voffB[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        voff[i] = (live && rowj[i] >= 0) ? (rowj[i] * nx + x0) * (int)sizeof(T) : OOB;
        voffB[i] = isB[i] ? voff[i] : OOB;
    }
    const int voff_lo = (halo_lo && jh_lo >= 0) ? (jh_lo * nx + x0) * (int)sizeof(T) : OOB;
    const int voff_hi = (halo_hi && jh_hi >= 0) ? (jh_hi * nx + x0) * (int)sizeof(T) : OOB;

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

    // load the plane-p inputs of phase A: I^{n-1/2}(p), V(p), and the two
    // extra R(p) rows of the LDS band
    auto load_a = [&](int p, VT(&io)[M], VT(&vv)[M], VT& hlo, VT& hhi) {
        const int gp = gplane(p);
        const auto rI = prs(a.I0, gp), rV = prs(a.V, gp), rR = prs(a.R0, gp);
#pragma unroll
        for (int i = 0; i < M; ++i) {
            io[i] = bload<T, W>(rI, voff[i]);
            vv[i] = bload<T, W>(rV, voff[i]);
        }
        hlo = bload<T, W>(rR, voff_lo);
        hhi = bload<T, W>(rR, voff_hi);
    };
    auto load_r = [&](int p, VT(&out)[M]) {
        const auto rR = prs(a.R0, gplane(p));
#pragma unroll
        for (int i = 0; i < M; ++i) out[i] = bload<T, W>(rR, voff[i]);
    };
    // stage R(p) = Rz[1] of the band and its halo rows in LDS
    auto stage = [&](const VT& hlo, const VT& hhi) {
        if (live) {
#pragma unroll
            for (int i = 0; i < M; ++i)
                if (rowb[i] <= TY + 1) *reinterpret_cast<VT*>(lr_row(rowb[i]) + x0) = Rz[1][i];
            if (halo_lo) *reinterpret_cast<VT*>(lr_row(-1) + x0) = hlo;
            if (halo_hi) *reinterpret_cast<VT*>(lr_row(TY + 2) + x0) = hhi;
        }
    };
    // phase A for plane p: I^{n+1/2}(p) on the owned rows from the R window
    // (planes p-1, p, p+1 in Rz[0..2], centre plane staged in LDS); result
    // into outI and the LDS buffer of plane p; stored if p is in the chunk.
    auto compute_a = [&](int p, const VT(&io)[M], const VT(&vv)[M], VT(&outI)[M], bool store) {
        const int gp = gplane(p);
        const T cap = gp >= 0 ? ld_uniform(a.ca, gp) : T(1);
        const T cbp = gp >= 0 ? ld_uniform(a.cb, gp) : T(1);
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
                    const T c = Rz[1][i].v[e];
                    const T xl = e > 0 ? Rz[1][i].v[e - 1] : xle;
                    const T xr = e < W - 1 ? Rz[1][i].v[e + 1] : xre;
                    const T hx = hterm(c, xl, xr, yl.v[e], yr.v[e], Rz[0][i].v[e], Rz[2][i].v[e],
                                       vterm(vv[i].v[e], a.cv, a.d0), a.cx, a.cy, a.cz, a.dlo);
                    out.v[e] = zero ? T(0) : upd_I(hx, io[i].v[e], cap, cbp);
                }
                *reinterpret_cast<VT*>(li_row(buf, b) + x0) = out;
                if (store) bstore_out<T, W>(prs(a.I1, gp), voffB[i], out, a.nt_out);
            } else {
#pragma unroll
                for (int e = 0; e < W; ++e) out.v[e] = T(0);
            }
            outI[i] = out;
        }
    };

    VT io[M], vv[M], hlo, hhi, Rn[M];
    // prologue: I^{n+1/2} at planes k0-1 (neighbour only) and k0
    load_r(k0 - 2, Rz[0]);
    load_r(k0 - 1, Rz[1]);
    load_r(k0, Rz[2]);
    load_a(k0 - 1, io, vv, hlo, hhi);
    stage(hlo, hhi);
    __syncthreads();
    compute_a(k0 - 1, io, vv, Iz[0], false);
    __syncthreads();                  // LR is rewritten next
#pragma unroll
    for (int i = 0; i < M; ++i) {
        Rz[0][i] = Rz[1][i];
        Rz[1][i] = Rz[2][i];
    }
    load_r(k0 + 1, Rz[2]);
    load_a(k0, io, vv, hlo, hhi);
    stage(hlo, hhi);
    __syncthreads();
    compute_a(k0, io, vv, Iz[1], true);
#pragma unroll
    for (int i = 0; i < M; ++i) Vk[i] = vv[i];  // V(k0)
    if (PF) {
        load_r(k0 + 2, Rn);
        load_a(k0 + 1, io, vv, hlo, hhi);
    }

    double f0 = 0.0, f1 = 0.0, q = 0.0, nv = 0.0, pl = 0.0;
    for (int k = k0; k < k1; ++k) {
        // R window to planes k, k+1, k+2 and the phase-A inputs of plane k+1
#pragma unroll
        for (int i = 0; i < M; ++i) {
            Rz[0][i] = Rz[1][i];
            Rz[1][i] = Rz[2][i];
            if (PF) Rz[2][i] = Rn[i];
        }
        if (!PF) {
            load_r(k + 2, Rz[2]);
            load_a(k + 1, io, vv, hlo, hhi);
        }
        VT vk[M];
#pragma unroll
        for (int i = 0; i < M; ++i) vk[i] = Vk[i];
        __syncthreads();                 // all reads of the previous plane's LDS done
        stage(hlo, hhi);
        __syncthreads();
        compute_a(k + 1, io, vv, Iz[2], k + 1 < k1);   // I^{n+1/2}(k+1)
#pragma unroll
        for (int i = 0; i < M; ++i) Vk[i] = vv[i];      // V(k+1)
        if (PF && k + 1 < k1) {
            load_r(k + 3, Rn);
            load_a(k + 2, io, vv, hlo, hhi);
        }
        // phase B for plane k: R^{n+1}(k) = eq. (8) from I^{n+1/2}(k-1..k+1)
        const int buf = (k - k0 + 2) & 1;
        const T cak = ld_uniform(a.ca, k);
        const T cbk = ld_uniform(a.cb, k);
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
                const T hx = hterm(c, xl, xr, yl.v[e], yr.v[e], Iz[0][i].v[e], Iz[2][i].v[e],
                                   vterm(vk[i].v[e], a.cv, a.d0), a.cx, a.cy, a.cz, a.dlo);
                const T uo = Rz[0][i].v[e];
                const T un = upd_R(hx, uo, cak, cbk);
                out.v[e] = un;
                if (at_det) f0 += (double)Iz[2][i].v[e] * ((double)uo + (double)un);
                if (at_up) f1 += (double)Iz[0][i].v[e] * ((double)uo + (double)un);
                if (REC) {
                    const double dc = (double)c, du = (double)uo, dn = (double)un;
                    q += dc * dc + du * dn;
                    nv += dn * dn + dc * dc;
                }
            }
            bstore_out<T, W>(prs(a.R1, k), voffB[i], out, a.nt_out);
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
    __shared__ double red[4];
    const bool has_det = (a.k_det >= k0 && a.k_det < k1);
    const bool has_up = (a.k_up >= k0 && a.k_up < k1);
    auto wg_sum = [&](double v) -> double { return block_sum(v, red, (int)blockDim.x >> 6); };
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

template <typename T, int W, int M, bool REC, bool PF>
__global__ __launch_bounds__(256) void fused_step_kernel(FusedArgs<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    fused_step_body<T, W, M, REC, PF>(a, xcd_remap(blockIdx.x, a.nwg), smem_raw);
}

// Many grids in one launch.  cfg[c] is the step of configuration c from its
// state pair 0 into pair 1 (parity 0) or back (parity 1); its workgroups are
// wg_start[c] .. wg_start[c+1]-1 of the launch, the whole launch remapped so
// that neighbouring tiles of one grid share an XCD.  Record slots come from
// the device counter *rec_idx so a captured graph can be replayed.
template <typename T>
struct BatchStep {
    const FusedArgs<T>* cfg;
    const int* wg_start;
    const long* rec_idx;
    int n, total_wg, parity, flux_slot;
};

template <typename T, int W, int M, bool REC, bool PF>
__global__ __launch_bounds__(256) void fused_batch_kernel(BatchStep<T> b) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int Lg = xcd_remap(blockIdx.x, b.total_wg);
    int lo = 0, hi = b.n;  // wg_start[lo] <= Lg < wg_start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (b.wg_start[mid] <= Lg) lo = mid; else hi = mid;
    }
    FusedArgs<T> a = b.cfg[lo];
    if (b.parity) {
        const T* r0 = a.R0;
        const T* i0 = a.I0;
        a.R0 = a.R1;
        a.I0 = a.I1;
        a.R1 = const_cast<T*>(r0);
        a.I1 = const_cast<T*>(i0);
    }
    a.flux_slots += (long)b.flux_slot * 2 * a.nbands;
    if (REC) a.rec_plane += (*b.rec_idx) * (long)a.nx * a.ny;
    fused_step_body<T, W, M, REC, PF>(a, Lg - b.wg_start[lo], smem_raw);
}

}  // namespace tdse
