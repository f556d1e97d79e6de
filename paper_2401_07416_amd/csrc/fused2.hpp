// Two leapfrog steps per sweep: eqs. (9), (8), (9), (8) of arXiv 2401.07416
// section 2.1 chained in one z-marching pass (temporal blocking of depth
// two).  The sweep reads (R^n, I^{n-1/2}, V) once and writes (R^{n+2},
// I^{n+3/2}) once, 20 B per cell in FP32 for two steps, where the one-pass
// step moves 20 B per step.  The intermediate level (I^{n+1/2}, R^{n+1})
// never leaves the chip.
//
// Mapping.  A workgroup (NT = 256, 512 or 1024 threads) owns an interior
// tile of tx x ty cells of every plane of a z chunk, and works on the tile
// extended by four cells on each side in x and y (ex = tx + 8, ey = ty + 8,
// ey = M rows per thread x the rows one pass of NT threads covers): each of
// the four half-steps needs its input one cell further out than its output,
// so the region on which a phase result is exact shrinks by one cell per
// phase, from the whole extension for the loaded R^n to the interior for
// R^{n+2}.  Results on the shrinking rim are computed and discarded.
//
// Per iteration k of the z march the four phases run one plane apart:
//   A1  I^{n+1/2}(k+3)  from R^n(k+2..k+4)
//   B1  R^{n+1}(k+2)    from I^{n+1/2}(k+1..k+3)
//   A2  I^{n+3/2}(k+1)  from R^{n+1}(k..k+2)
//   B2  R^{n+2}(k)      from I^{n+3/2}(k-1..k+1)
// Each thread keeps the z windows of the four fields (the new plane of each
// plus the two below it that the next phases read, in rings of three
// register slots) and four planes of the potential term vterm(V) in
// registers (its W-wide x vectors of M extended rows).  The x and y
// neighbours of each phase's centre plane come from LDS, where the previous
// iteration left them: every phase reads the LDS buffers of parity k and
// writes those of parity k + 1, so one barrier per iteration orders all
// reads and writes.  The march starts six planes before the chunk so
// that every stored plane is exact.
//
// The cell arithmetic is vterm / hterm / upd_* of kernels.hpp, so the
// states are bitwise identical to those of the one-pass and two-pass steps.
// The flux partials of both steps (every step) and, on the second step only,
// the record fields are reduced per workgroup in a fixed order.
#pragma once

#include <type_traits>

#include "kernels.hpp"

namespace tdse {

template <typename T>
struct Fused2Args {
    const T* R0;  // R^n
    const T* I0;  // I^{n-1/2}
    T* R1;        // R^{n+2}
    T* I1;        // I^{n+3/2}
    const T* V;
    const T* ca;
    const T* cb;
    T cx, cy, cz, cv;
    T d0, dlo;            // 2 (cx + cy + cz) as hi + lo parts
    int nx, ny, nz;
    int tx, ty, ex, ey;   // interior and extended tile extents
    int tpr, rpp;         // threads per extended row, extended rows per pass
    int ntx, ntiles, zc, nzc, nwg;
    int bcx, bcy, bcz;
    int k_det, k_up;
    int ulo, uhi;         // planes [ulo, uhi) have no absorption (ca = cb = 1)
    double* flux_a;       // [2][ntiles], step n -> n+1
    double* flux_b;       // [2][ntiles], step n+1 -> n+2
    // record of level n+2 (REC instances only)
    T* rec_plane;
    double* part_q;       // [nzc][ntiles]
    double* part_naive;
    double* part_plane;   // [ntiles]
    double* pixel;
    double pixel_w;
    int nt_out;           // non-temporal hint on the R^{n+2}, I^{n+3/2} stores
};

template <typename T, int W, int M, bool REC, bool PF, int NT>
__device__ __forceinline__ void fused2_body(const Fused2Args<T>& a, int L, unsigned char* smem_raw) {
    using VT = vec_t<T, W>;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int ex = a.ex, ey = a.ey;
    const int pbytes = (int)((long)nx * ny * (long)sizeof(T));
    const long fstride = (long)(ey + 2) * ex;   // one LDS buffer with a pad row on each side
    T* lds = reinterpret_cast<T*>(smem_raw);
    // field f (0 R^n, 1 I^{n+1/2}, 2 R^{n+1}, 3 I^{n+3/2}), parity q: row 0
    auto buf = [&](int f, int q) -> T* { return lds + (2 * f + q) * fstride + ex; };

    const int zchunk = L / a.ntiles;
    const int tile = L - zchunk * a.ntiles;
    const int tyi = tile / a.ntx;
    const int txi = tile - tyi * a.ntx;
    const int x0 = txi * a.tx, y0 = tyi * a.ty;
    const int k0 = zchunk * a.zc;
    const int k1 = min(k0 + a.zc, nz);
    const int tid = threadIdx.x;
    const int rs0 = tid / a.tpr;
    const bool live = rs0 < a.rpp;             // threads past the last full row idle
    const int rs = live ? rs0 : 0;
    const int c0 = (live ? tid - rs0 * a.tpr : 0) * W;   // extended column of the vector
    const int gx = x0 - 4 + c0;                          // unwrapped grid column
    int colg = gx;
    if (gx < 0 || gx >= nx) colg = a.bcx ? -1 : ((gx % nx) + nx) % nx;
    const bool xin = c0 >= 4 && c0 < 4 + a.tx && gx < nx;

    int rowb[M], voff[M], soff[M], voff_iv[M];
    bool zc_cell[M];   // cell outside a zero-boundary axis (or idle thread): forced to 0
#pragma unroll
    for (int i = 0; i < M; ++i) {
        rowb[i] = rs + i * a.rpp;
        const int gy = y0 - 4 + rowb[i];
        int rj = gy;
        if (gy < 0 || gy >= ny) rj = a.bcy ? -1 : ((gy % ny) + ny) % ny;
        const bool ok = live && rj >= 0 && colg >= 0;
        zc_cell[i] = !ok;
        voff[i] = ok ? (rj * nx + colg) * (int)sizeof(T) : OOB;
        const bool st = live && xin && rowb[i] >= 4 && rowb[i] < 4 + a.ty && gy < ny;
        soff[i] = st ? voff[i] : OOB;
        // I^{n-1/2} and V of the outermost extended rows feed only the
        // first phase's results there, which are discarded: not read
        voff_iv[i] = (rowb[i] >= 1 && rowb[i] < ey - 1) ? voff[i] : OOB;
    }
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
    auto prs = [&](const T* base, int gp) {
        return plane_rsrc(base + (long)(gp < 0 ? 0 : gp) * nx * ny, gp < 0 ? 0 : pbytes);
    };
    auto zero_vec = [&]() {
        VT z;
#pragma unroll
        for (int e = 0; e < W; ++e) z.v[e] = T(0);
        return z;
    };

    // z windows.  The four fields live in rings of three register slots,
    // plane p of a field in slot (p + off) mod 3, so that an iteration
    // writes each new plane over the one that has gone out of use and
    // nothing moves between iterations; the march is unrolled three times
    // so that every slot index is a compile-time constant.  At iteration k:
    // R^n holds planes k+2, k+3 and receives k+4; I^{n+1/2} holds k+1, k+2
    // and receives k+3; R^{n+1} holds k, k+1 and receives k+2; I^{n+3/2}
    // holds k-1, k and receives k+1.  Vw[0..3] holds the potential term of
    // V(k..k+3) (V(k+3) arrives in the iteration), io I^{n-1/2}(k+3).
    VT Rn[3][M], Ia[3][M], Rb[3][M], Ib[3][M], Vw[4][M], io[M];
    VT pR[M], pI[M], pV[M];   // prefetched inputs of the next iteration
#pragma unroll
    for (int i = 0; i < M; ++i) {
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            Ia[s][i] = zero_vec();
            Rb[s][i] = zero_vec();
            Ib[s][i] = zero_vec();
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) Vw[s][i] = zero_vec();
    }

    // one phase on plane p: centre c, z neighbours zl / zr, x / y neighbours
    // from LDS buffer src (the centre plane), old value uo, potential term
    // vterm(V) in vtv;
    // IS_R selects eq. (8), else eq. (9).  The result goes to out and, from
    // live threads, to LDS buffer dst (if not null).  A plane outside a zero
    // z boundary is zero.  Workgroups of 512 and 1024 threads (one or two
    // per CU, where the VALU work is least hidden) also take two uniform
    // shortcuts: no zero-boundary select without zero x / y boundaries (idle
    // threads' results are never stored or read), and no CAP factors on
    // planes without absorption (ca = cb = 1); the bits are the same.
    const bool sel_xy = NT < 512 || a.bcx || a.bcy;
    // Phase d (1..4) is exact on extended rows [d, ey - d); with one row per
    // thread, a wavefront none of whose rows lie there skips it (its rows
    // are all discarded rim, and no needed cell of the next phase reads
    // them): two of 16 wavefronts in the last phase of a 1024-thread tile.
    const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63);
    const int wlo = wbase / a.tpr;
    const int whi = min((wbase + 63) / a.tpr, a.rpp - 1);
    auto wave_needed = [&](int d) -> bool {
#pragma unroll
        for (int i = 0; i < M; ++i)
            if (whi + i * a.rpp >= d && wlo + i * a.rpp < ey - d) return true;
        return false;
    };
    auto phase = [&](auto is_r, int depth, int p, const VT(&zl)[M], const VT(&c)[M], const VT(&zr)[M],
                     const T* src, const VT(&uo)[M], const VT(&vtv)[M], VT(&out)[M], T* dst) {
        constexpr bool IS_R = decltype(is_r)::value;
        // the march's first iterations reach planes below those the stored
        // planes [k0, k1) depend on: phase d needs planes >= k0 - (4 - d)
        if (p < k0 - (4 - depth) || (M == 1 && !wave_needed(depth))) {
#pragma unroll
            for (int i = 0; i < M; ++i) out[i] = zero_vec();
            return;
        }
        const int gp = gplane(p);
        if (gp < 0) {
#pragma unroll
            for (int i = 0; i < M; ++i) {
                out[i] = zero_vec();
                if (dst && live) *reinterpret_cast<VT*>(dst + rowb[i] * ex + c0) = out[i];
            }
            return;
        }
        const T cap = ld_uniform(a.ca, gp);
        const T cbp = ld_uniform(a.cb, gp);
        auto cells = [&](auto sel, auto unit) {
            constexpr bool SEL = decltype(sel)::value, UNIT = decltype(unit)::value;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const T* row = src + rowb[i] * ex + c0;
                const VT yl = *reinterpret_cast<const VT*>(row - ex);
                const VT yr = *reinterpret_cast<const VT*>(row + ex);
                const T xle = row[-1], xre = row[W];
                VT o;
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    const T cc = c[i].v[e];
                    const T xl = e > 0 ? c[i].v[e - 1] : xle;
                    const T xr = e < W - 1 ? c[i].v[e + 1] : xre;
                    const T hx = hterm(cc, xl, xr, yl.v[e], yr.v[e], zl[i].v[e], zr[i].v[e], vtv[i].v[e],
                                       a.cx, a.cy, a.cz, a.dlo);
                    T u;
                    if constexpr (UNIT)
                        u = IS_R ? upd_R_unit(hx, uo[i].v[e]) : upd_I_unit(hx, uo[i].v[e]);
                    else
                        u = IS_R ? upd_R(hx, uo[i].v[e], cap, cbp) : upd_I(hx, uo[i].v[e], cap, cbp);
                    if constexpr (SEL)
                        o.v[e] = zc_cell[i] ? T(0) : u;
                    else
                        o.v[e] = u;
                }
                out[i] = o;
                if (dst && live) *reinterpret_cast<VT*>(dst + rowb[i] * ex + c0) = o;
            }
        };
        using Yes = std::true_type;
        using No = std::false_type;
        const bool unit = NT >= 512 && cap == T(1) && cbp == T(1);
        if (sel_xy) {
            if (unit) cells(Yes{}, Yes{});
            else cells(Yes{}, No{});
        } else {
            if (unit) cells(No{}, Yes{});
            else cells(No{}, No{});
        }
    };
    using IsR = std::integral_constant<bool, true>;
    using IsI = std::integral_constant<bool, false>;

    // The straight-line iteration (one row per thread, 512 or 1024
    // threads): the cells of one phase with unit CAP factors from the LDS
    // buffer src, and the write slot of each buffer (wslot + buffer index x
    // wstep; idle threads: the slot past the eight buffers, wstep 0).
    constexpr bool FAST = M == 1 && NT >= 512;
    const bool fast_grid = !sel_xy;
    const bool need4 = M != 1 || wave_needed(4);
    const bool wave_live = wlo < a.rpp;   // some thread of the wavefront owns a row
    T* const wslot = live ? buf(0, 0) + rowb[0] * ex + c0 : lds + 8 * fstride;
    const long wstep = live ? fstride : 0;
    const int rofs = rowb[0] * ex + c0;
    auto fast_cells = [&](auto is_r, const VT& zl, const VT& c, const VT& zr, const T* src, const VT& uo,
                          const VT& vtv, VT& out) {
        constexpr bool IS_R = decltype(is_r)::value;
        const T* row = src + rofs;
        const VT yl = *reinterpret_cast<const VT*>(row - ex);
        const VT yr = *reinterpret_cast<const VT*>(row + ex);
        const T xle = row[-1], xre = row[W];
#pragma unroll
        for (int e = 0; e < W; ++e) {
            const T cc = c.v[e];
            const T xl = e > 0 ? c.v[e - 1] : xle;
            const T xr = e < W - 1 ? c.v[e + 1] : xre;
            const T hx = hterm(cc, xl, xr, yl.v[e], yr.v[e], zl.v[e], zr.v[e], vtv.v[e], a.cx, a.cy, a.cz,
                               a.dlo);
            out.v[e] = IS_R ? upd_R_unit(hx, uo.v[e]) : upd_I_unit(hx, uo.v[e]);
        }
    };

    auto load3 = [&](int pr, int pi, VT(&r)[M], VT(&iv)[M], VT(&vv)[M]) {
        const int gr = gplane(pr), gi = gplane(pi);
        const auto rR = prs(a.R0, gr), rI = prs(a.I0, gi), rV = prs(a.V, gi);
#pragma unroll
        for (int i = 0; i < M; ++i) {
            r[i] = bload<T, W>(rR, voff[i]);
            iv[i] = bload<T, W>(rI, voff_iv[i]);
            vv[i] = bload<T, W>(rV, voff_iv[i]);
        }
    };

    const int ks = k0 - 6;
    // ring slot of plane p: R^n and I^{n+1/2} by (p - ks) mod 3, R^{n+1} and
    // I^{n+3/2} the same (their planes trail by one and two); as a
    // compile-time function of the unrolled iteration u = (k - ks) mod 3
    // and the plane's offset j from k
    auto slot = [](int u, int j) -> int { return ((u + j) % 3 + 3) % 3; };
    // prologue: R^n(ks+2), R^n(ks+3) into the ring, R^n(ks+3) staged for A1
    {
        const auto r2 = prs(a.R0, gplane(ks + 2)), r3 = prs(a.R0, gplane(ks + 3));
#pragma unroll
        for (int i = 0; i < M; ++i) {
            Rn[slot(0, 2)][i] = bload<T, W>(r2, voff[i]);
            Rn[slot(0, 3)][i] = bload<T, W>(r3, voff[i]);
        }
        if (live) {
#pragma unroll
            for (int i = 0; i < M; ++i)
                *reinterpret_cast<VT*>(buf(0, 0) + rowb[i] * ex + c0) = Rn[slot(0, 3)][i];
        }
        if (PF) load3(ks + 4, ks + 3, pR, pI, pV);
    }
    __syncthreads();

    double fa0 = 0.0, fa1 = 0.0, fb0 = 0.0, fb1 = 0.0, q = 0.0, nv = 0.0, pl = 0.0;
    // one iteration of the march; U = (k - ks) mod 3 as a type
    auto iteration = [&](auto uc, int k) {
        constexpr int U = decltype(uc)::value;
        const int par = (k - ks) & 1;
        VT(&rN)[M] = Rn[slot(U, 4)];   // R^n(k+4), arriving
        VT(&rC)[M] = Rn[slot(U, 3)];
        VT(&rL)[M] = Rn[slot(U, 2)];
        VT(&nA)[M] = Ia[slot(U, 3)];   // I^{n+1/2}(k+3), formed by A1
        VT(&iC)[M] = Ia[slot(U, 2)];
        VT(&iL)[M] = Ia[slot(U, 1)];
        VT(&nB)[M] = Rb[slot(U, 2)];   // R^{n+1}(k+2), formed by B1
        VT(&bC)[M] = Rb[slot(U, 1)];
        VT(&bL)[M] = Rb[slot(U, 0)];
        VT(&nC)[M] = Ib[slot(U, 1)];   // I^{n+3/2}(k+1), formed by A2
        VT(&jC)[M] = Ib[slot(U, 0)];
        VT(&jL)[M] = Ib[slot(U, -1)];
        if (PF) {
#pragma unroll
            for (int i = 0; i < M; ++i) {
                rN[i] = pR[i];
                io[i] = pI[i];
                Vw[3][i] = pV[i];
            }
            if (k + 1 < k1) load3(k + 5, k + 4, pR, pI, pV);
        } else {
            load3(k + 4, k + 3, rN, io, Vw[3]);
        }
        // the window keeps the potential term of the update (vterm),
        // formed once per plane instead of per phase
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int e = 0; e < W; ++e) Vw[3][i].v[e] = vterm(Vw[3][i].v[e], a.cv, a.d0);
        VT nD[M];   // R^{n+2}(k), formed by B2
        if (FAST && fast_grid && k >= k0 && k >= a.ulo && k + 3 < a.uhi) {
            // the common iteration as one straight-line block: all four
            // planes inside the chunk's dependence range and the grid, no
            // absorption on them, periodic x and y.  Every LDS read of the
            // iteration comes before its first LDS write (the reads take
            // parity k, the writes parity k + 1), so the compiler may issue
            // a phase's neighbour reads ahead of the previous phase's
            // arithmetic; idle threads write a slot past the buffers
            // instead of branching around the writes.  Same bits as the
            // phases below.
            if (wave_live) {
                fast_cells(IsI{}, rL[0], rC[0], rN[0], buf(0, par), io[0], Vw[3][0], nA[0]);
                fast_cells(IsR{}, iL[0], iC[0], nA[0], buf(1, par), rL[0], Vw[2][0], nB[0]);
                fast_cells(IsI{}, bL[0], bC[0], nB[0], buf(2, par), iL[0], Vw[1][0], nC[0]);
                if (need4)
                    fast_cells(IsR{}, jL[0], jC[0], nC[0], buf(3, par), bL[0], Vw[0][0], nD[0]);
                else
                    nD[0] = zero_vec();
                *reinterpret_cast<VT*>(wslot + (0 * 2 + (par ^ 1)) * wstep) = rN[0];
                *reinterpret_cast<VT*>(wslot + (1 * 2 + (par ^ 1)) * wstep) = nA[0];
                *reinterpret_cast<VT*>(wslot + (2 * 2 + (par ^ 1)) * wstep) = nB[0];
                *reinterpret_cast<VT*>(wslot + (3 * 2 + (par ^ 1)) * wstep) = nC[0];
            } else {
                // a wavefront of idle threads (a tile shorter than the
                // threads cover): nothing of it is stored or read
                nA[0] = nB[0] = nC[0] = nD[0] = zero_vec();
            }
        } else {
            // stage R^n(k+4) for the next iteration's A1
            if (live) {
#pragma unroll
                for (int i = 0; i < M; ++i)
                    *reinterpret_cast<VT*>(buf(0, par ^ 1) + rowb[i] * ex + c0) = rN[i];
            }
            // A1: I^{n+1/2}(k+3)
            phase(IsI{}, 1, k + 3, rL, rC, rN, buf(0, par), io, Vw[3], nA, buf(1, par ^ 1));
            // B1: R^{n+1}(k+2)
            phase(IsR{}, 2, k + 2, iL, iC, nA, buf(1, par), rL, Vw[2], nB, buf(2, par ^ 1));
            // A2: I^{n+3/2}(k+1)
            phase(IsI{}, 3, k + 1, bL, bC, nB, buf(2, par), iL, Vw[1], nC, buf(3, par ^ 1));
            // B2: R^{n+2}(k)
            phase(IsR{}, 4, k, jL, jC, nC, buf(3, par), bL, Vw[0], nD, nullptr);
        }
        const int pB = k + 2, pC = k + 1, pD = k;
        if (pC >= k0 && pC < k1) {
            const auto rI = prs(a.I1, pC);
#pragma unroll
            for (int i = 0; i < M; ++i) bstore_out<T, W>(rI, soff[i], nC[i], a.nt_out);
        }
        if (pD >= k0) {
            const auto rR = prs(a.R1, pD);
#pragma unroll
            for (int i = 0; i < M; ++i) bstore_out<T, W>(rR, soff[i], nD[i], a.nt_out);
        }
        // flux partials of both steps over the stored cells
        const bool inB = pB >= k0 && pB < k1;
        // (the two faces are the same plane when nz = 1)
        if (inB && (pB == a.k_det || pB == a.k_up)) {
            const bool det = pB == a.k_det, up = pB == a.k_up;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                if (soff[i] == OOB) continue;
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    const double s = (double)rL[i].v[e] + (double)nB[i].v[e];
                    if (det) fa0 += (double)nA[i].v[e] * s;
                    if (up) fa1 += (double)iL[i].v[e] * s;
                }
            }
        }
        if (pD >= k0 && (pD == a.k_det || pD == a.k_up)) {
            const bool det = pD == a.k_det, up = pD == a.k_up;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                if (soff[i] == OOB) continue;
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    const double s = (double)bL[i].v[e] + (double)nD[i].v[e];
                    if (det) fb0 += (double)nC[i].v[e] * s;
                    if (up) fb1 += (double)jL[i].v[e] * s;
                }
            }
        }
        if (REC && pD >= k0) {
#pragma unroll
            for (int i = 0; i < M; ++i) {
                if (soff[i] == OOB) continue;
#pragma unroll
                for (int e = 0; e < W; ++e) {
                    const double dc = (double)jC[i].v[e], du = (double)bL[i].v[e];
                    const double dn = (double)nD[i].v[e];
                    q += dc * dc + du * dn;
                    nv += dn * dn + dc * dc;
                }
                if (pD == a.k_det) {
                    VT rv;
                    const long poff = soff[i] / (int)sizeof(T);
#pragma unroll
                    for (int e = 0; e < W; ++e) {
                        const double dn = (double)nD[i].v[e], dc = (double)jC[i].v[e];
                        const double rho = dn * dn + dc * dc;
                        rv.v[e] = (T)rho;
                        pl += rho;
                        if (a.pixel) a.pixel[poff + e] += a.pixel_w * rho;
                    }
                    stv<T, W>(a.rec_plane + poff, rv);
                }
            }
        }
        // shift the potential window one plane up
#pragma unroll
        for (int i = 0; i < M; ++i) {
            Vw[0][i] = Vw[1][i];
            Vw[1][i] = Vw[2][i];
            Vw[2][i] = Vw[3][i];
        }
        __syncthreads();
    };
    using U0 = std::integral_constant<int, 0>;
    using U1 = std::integral_constant<int, 1>;
    using U2 = std::integral_constant<int, 2>;
    // k1 - ks >= 7 iterations; every exit is uniform over the workgroup
    for (int k = ks;; k += 3) {
        iteration(U0{}, k);
        if (k + 1 >= k1) break;
        iteration(U1{}, k + 1);
        if (k + 2 >= k1) break;
        iteration(U2{}, k + 2);
        if (k + 3 >= k1) break;
    }

    // fixed-order workgroup sums of the partials
    __shared__ double red[NT / 64];
    const bool has_det = a.k_det >= k0 && a.k_det < k1;
    const bool has_up = a.k_up >= k0 && a.k_up < k1;
    auto wg_sum = [&](double v) -> double { return block_sum(v, red, NT / 64); };
    if (has_det) {
        const double sa = wg_sum(fa0);
        const double sb = wg_sum(fb0);
        if (tid == 0) {
            a.flux_a[tile] = sa;
            a.flux_b[tile] = sb;
        }
    }
    if (has_up) {
        const double sa = wg_sum(fa1);
        const double sb = wg_sum(fb1);
        if (tid == 0) {
            a.flux_a[a.ntiles + tile] = sa;
            a.flux_b[a.ntiles + tile] = sb;
        }
    }
    if (REC) {
        const double sq = wg_sum(q);
        const double sn = wg_sum(nv);
        const long slot = (long)zchunk * a.ntiles + tile;
        if (tid == 0) {
            a.part_q[slot] = sq;
            a.part_naive[slot] = sn;
        }
        if (has_det) {
            const double sp = wg_sum(pl);
            if (tid == 0) a.part_plane[tile] = sp;
        }
    }
}

template <typename T, int W, int M, bool REC, bool PF, int NT>
__global__ __launch_bounds__(NT) void fused2_kernel(Fused2Args<T> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    fused2_body<T, W, M, REC, PF, NT>(a, xcd_remap(blockIdx.x, a.nwg), smem_raw);
}

// Two steps of many grids in one launch (the batch form of the sweep).
// cfg[c] describes grid c from its state pair 0 into pair 1 (parity 0) or
// back (parity 1), with flux_a at its ring's slot 0; the launch takes ring
// slots flux_slot and flux_slot + 1.  Workgroups wg_start[c] ..
// wg_start[c+1]-1 of the launch (after an XCD remap over the whole launch)
// belong to grid c.  The record slot comes from the device counter so a
// captured graph can be replayed.
template <typename T>
struct Batch2Step {
    const Fused2Args<T>* cfg;
    const int* wg_start;
    const long* rec_idx;
    int n, total_wg, parity, flux_slot;
};

template <typename T, int W, int M, bool REC, bool PF, int NT>
__global__ __launch_bounds__(NT) void fused2_batch_kernel(Batch2Step<T> b) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int Lg = xcd_remap(blockIdx.x, b.total_wg);
    int lo = 0, hi = b.n;  // wg_start[lo] <= Lg < wg_start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (b.wg_start[mid] <= Lg) lo = mid; else hi = mid;
    }
    Fused2Args<T> a = b.cfg[lo];
    if (b.parity) {
        const T* r0 = a.R0;
        const T* i0 = a.I0;
        a.R0 = a.R1;
        a.I0 = a.I1;
        a.R1 = const_cast<T*>(r0);
        a.I1 = const_cast<T*>(i0);
    }
    a.flux_a += (long)b.flux_slot * 2 * a.ntiles;
    a.flux_b = a.flux_a + 2 * a.ntiles;
    if (REC) a.rec_plane += (*b.rec_idx) * (long)a.nx * a.ny;
    fused2_body<T, W, M, REC, PF, NT>(a, Lg - b.wg_start[lo], smem_raw);
}

}  // namespace tdse
