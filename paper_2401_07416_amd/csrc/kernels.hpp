// Device code of libtdse for gfx950 (CDNA4, wave64).
//
// Half-step kernels of the staggered leapfrog, arXiv 2401.07416 section 2.1:
//   eq. (9): I <- ca_k I + cb_k ( L(R) - c_v V R )   (imaginary half-step)
//   eq. (8): R <- ca_k R - cb_k ( L(I) - c_v V I )   (real half-step)
// (hterm / upd_* below give the per-precision evaluation order)
// with L(X) = c_x dxx X + c_y dyy X + c_z dzz X (3-point second differences,
// periodic wrap as in eqs. (13)-(14) or zero outside), and ca_k, cb_k the
// time-centred damping of the per-plane absorbing rate (eq. (10)).
//
// Mapping.  Arrays are [nz][ny][nx], x fastest.  One wavefront owns a tile of
// RY consecutive full x-rows and marches through a chunk of zc planes.  A row
// of nx values is spread over the wave as G groups of W-element vectors:
// lane l, group g, element e holds x = (g * nl + l) * W + e, so every vector
// load instruction of a wave covers one contiguous run of nl * W * sizeof(T)
// bytes.  z neighbours live in registers (planes k-1, k, k+1 of the stencil
// array), y neighbours are the tile's own rows plus two halo rows, and the x
// neighbours at vector edges come from the adjacent lane through a lane
// permute, with the wrap across groups and across the row handled by which
// value the edge lanes hand out.  Each of R, I and V is read from HBM about
// once per half-step; the halo rows are re-read by the neighbouring tile and
// the workgroup order keeps neighbouring tiles on one XCD so those re-reads
// hit its L2.
//
// The real half-step also produces the FP64 partial sums of the detection
// face flux (every step) and, on record steps, the detection-plane density,
// the pixel integral and the partial sums of Q, the naive norm and the plane
// density.  Every partial goes to its own slot (no atomics) and is reduced in
// a fixed order by finalize_kernel, so results are bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdse {

enum Mode : int {
    MODE_I = 0,       // eq. (9), store I
    MODE_R = 1,       // eq. (8), store R, flux partials
    MODE_R_REC = 2,   // eq. (8) + record: rho plane, Q, naive norm, pixel
    MODE_I_PEEK = 3   // eq. (9) evaluated, not stored: record 0 (Q^0, rho^0)
};

template <typename T, int W>
struct alignas(sizeof(T) * W) vec_t {
    T v[W];
};

template <typename T>
struct HalfArgs {
    T* U;              // array updated in place (I for eq. (9), R for eq. (8))
    const T* S;        // stencil array (R for eq. (9), I for eq. (8))
    const T* V;
    const T* ca;       // [nz]
    const T* cb;       // [nz]
    T cx, cy, cz, cv;
    T d0, dlo;         // 2 (cx + cy + cz) as hi + lo parts (FP32 form)
    int nx, ny, nz, nl;
    int ytiles, wpg, ywg, zc, nzc, nwg;
    int bcx, bcy, bcz;  // 1 = zero boundary on that axis
    int k_det, k_up;    // detection plane and the plane above it (-1: none)
    double* flux_slots; // [2][ytiles] for this step
    T* rec_plane;       // [ny][nx] record slot
    double* part_q;     // [nzc][ytiles]
    double* part_naive; // [nzc][ytiles]
    double* part_plane; // [ytiles]
    double* pixel;      // [ny][nx] or null
    double pixel_w;     // h * dt
    int nt_in;          // non-temporal hint on the U and V loads
};

// Workgroup id -> logical tile index such that the workgroups the hardware
// places on one XCD (ids congruent mod 8) get a contiguous range of logical
// tiles, i.e. neighbouring y-tiles of the same z-chunk.
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int q = n >> 3, rem = n & 7;
    const int x = b & 7, r = b >> 3;
    return (x < rem) ? x * (q + 1) + r : rem * (q + 1) + (x - rem) * q + r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Fixed-order workgroup sum for 1D workgroups of whole wavefronts: the
// butterfly above within each wavefront (every lane ends with the same bits,
// since each level adds x_i + x_(i^o) and addition commutes), then the
// wavefront totals in wavefront order.  red holds one double per
// wavefront; every thread of the workgroup calls this and gets the sum.
__device__ __forceinline__ double block_sum(double v, double* red, int nwaves) {
    v = wave_sum(v);
    __syncthreads();  // the previous call's reads of red are done
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nwaves; ++w) s += red[w];
    return s;
}

template <typename T, int W>
__device__ __forceinline__ vec_t<T, W> ldv(const T* p) {
    return *reinterpret_cast<const vec_t<T, W>*>(p);
}

// Load with the non-temporal hint, for streams read once per launch.
template <typename T, int W>
__device__ __forceinline__ vec_t<T, W> ldv_nt(const T* p) {
    constexpr int B = (int)sizeof(T) * W;
    if constexpr (B == 16) {
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        return __builtin_bit_cast(vec_t<T, W>, __builtin_nontemporal_load(reinterpret_cast<const u4*>(p)));
    } else if constexpr (B == 8) {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(vec_t<T, W>, __builtin_nontemporal_load(reinterpret_cast<const u2*>(p)));
    } else {
        return __builtin_bit_cast(vec_t<T, W>, __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p)));
    }
}

template <typename T, int W>
__device__ __forceinline__ void stv(T* p, const vec_t<T, W>& x) {
    *reinterpret_cast<vec_t<T, W>*>(p) = x;
}

// Buffer accesses through a resource spanning one z-plane of an array: the
// 32-bit byte offset of a row is the same for every plane and every array
// of the grid, and an offset past the plane (or a plane of size 0) reads
// as zero and drops stores, so zero rows and planes cost no branches.
// 0x00020000 is the gfx9 word-3 setting of a raw (stride 0) buffer.
constexpr int OOB = 0x7ffffff0;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}

template <typename T, int W>
__device__ __forceinline__ vec_t<T, W> bload(__amdgpu_buffer_rsrc_t r, int off) {
    constexpr int B = (int)sizeof(T) * W;
    static_assert(B == 4 || B == 8 || B == 16, "vector of 4, 8 or 16 bytes");
    if constexpr (B == 16) {
        return __builtin_bit_cast(vec_t<T, W>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    } else if constexpr (B == 8) {
        return __builtin_bit_cast(vec_t<T, W>, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    } else {
        return __builtin_bit_cast(vec_t<T, W>, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
}

// AUX is the cache-policy immediate: 0, or CPOL_NT, the non-temporal hint
// of gfx950 (bit 1).
constexpr int CPOL_NT = 2;

template <typename T, int W, int AUX = 0>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, int off, const vec_t<T, W>& v) {
    constexpr int B = (int)sizeof(T) * W;
    if constexpr (B == 16) {
        using U = __attribute__((ext_vector_type(4))) unsigned int;
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U, v), r, off, 0, AUX);
    } else if constexpr (B == 8) {
        using U = __attribute__((ext_vector_type(2))) unsigned int;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, v), r, off, 0, AUX);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, AUX);
    }
}

// Store of a result that no other workgroup of the launch reads: with nt
// set (grids whose arrays are far larger than the 256 MB memory-side cache)
// it carries the non-temporal hint, so the written lines do not displace
// inputs that neighbouring tiles are still to re-read.
template <typename T, int W>
__device__ __forceinline__ void bstore_out(__amdgpu_buffer_rsrc_t r, int off, const vec_t<T, W>& v, bool nt) {
    if (nt)
        bstore<T, W, CPOL_NT>(r, off, v);
    else
        bstore<T, W>(r, off, v);
}

// Load of a read-only table entry at a wave-uniform index through the
// scalar cache (constant address space), so that it never waits behind the
// vector loads in flight (a vector load of the same entry would, and a
// prefetch issued before it would be drained by that wait).
template <typename T>
__device__ __forceinline__ T ld_uniform(const T* p, int i) {
    using CT = const __attribute__((address_space(4))) T;
    return reinterpret_cast<CT*>(reinterpret_cast<uintptr_t>(p))[__builtin_amdgcn_readfirstlane(i)];
}

// Cell arithmetic shared by every step kernel (two-pass, one-pass, two-step,
// batch, the section 2.2 layout), so all of them produce the same bits.
//   L(X) = cx (X(i+1) - 2X + X(i-1)) + cy (...) + cz (...)
template <typename T>
__device__ __forceinline__ T lap7(T c, T xl, T xr, T yl, T yr, T zl, T zr, T cx, T cy, T cz) {
    return cx * ((xr - T(2) * c) + xl) + cy * ((yr - T(2) * c) + yl) + cz * ((zr - T(2) * c) + zl);
}

// The update term H X = L(X) - cv V X of eqs. (8)-(9) from the 7-point
// neighbourhood of X and a per-cell potential term vt = vterm(V), which a
// kernel forms once per cell and plane.
//  FP64: vt = cv V and H X = L(X) - vt X with L grouped as printed above,
//        every operation rounded on its own: the oracle's rounding sequence.
//  FP32: the diagonal of the Laplacian is folded into the potential term,
//        vt = 2 (cx + cy + cz)_hi + cv V (one fused multiply-add from V),
//          H X = cx (X(i+1) + X(i-1)) + cy (...) + cz (...) - vt X - dlo X,
//        three adds and five fused multiply-adds instead of twelve
//        operations: the same operator, regrouped.  The diagonal
//        2 (cx + cy + cz) of the FP32 coefficients is exact in FP64 and is
//        carried as hi + lo FP32 parts (d0 = hi, dlo = lo): a diagonal
//        rounded to FP32 alone would disagree with the neighbour weights
//        by up to an FP32 ulp, a constant energy shift that turns into a
//        global phase growing linearly with the step count (measured:
//        1.5e-4 relative L2 after 20,000 steps of the surface workload).
template <typename T>
__device__ __forceinline__ T vterm(T v, T cv, T d0) {
    if constexpr (sizeof(T) == 4)
        return __builtin_fmaf(cv, v, d0);
    else
        return cv * v;
}

template <typename T>
__device__ __forceinline__ T hterm(T c, T xl, T xr, T yl, T yr, T zl, T zr, T vt, T cx, T cy, T cz,
                                   T dlo) {
    if constexpr (sizeof(T) == 4) {
        float s = cx * (xl + xr);
        s = __builtin_fmaf(cy, yl + yr, s);
        s = __builtin_fmaf(cz, zl + zr, s);
        s = __builtin_fmaf(-vt, c, s);
        return __builtin_fmaf(-dlo, c, s);
    } else {
        (void)dlo;
        return lap7(c, xl, xr, yl, yr, zl, zr, cx, cy, cz) - vt * c;
    }
}

// eq. (9) with the time-centred CAP: I' = ca I + cb H R; eq. (8):
// R' = ca R - cb H I; and their forms on planes without absorption (ca =
// cb = 1, where both forms give the same bits: 1 * x = x exactly, and
// fma(1, u, x) rounds u + x once).
template <typename T>
__device__ __forceinline__ T upd_I(T hx, T uo, T ca, T cb) {
    if constexpr (sizeof(T) == 4)
        return __builtin_fmaf(ca, uo, cb * hx);
    else
        return ca * uo + cb * hx;
}

template <typename T>
__device__ __forceinline__ T upd_R(T hx, T uo, T ca, T cb) {
    if constexpr (sizeof(T) == 4)
        return __builtin_fmaf(ca, uo, -(cb * hx));
    else
        return ca * uo - cb * hx;
}

template <typename T>
__device__ __forceinline__ T upd_I_unit(T hx, T uo) {
    return uo + hx;
}

template <typename T>
__device__ __forceinline__ T upd_R_unit(T hx, T uo) {
    return uo - hx;
}

template <typename T, int W, int G, int RY, int MODE>
__global__ __launch_bounds__(256) void half_step_kernel(HalfArgs<T> a) {
    using VT = vec_t<T, W>;
    constexpr bool IS_R = (MODE == MODE_R || MODE == MODE_R_REC);
    constexpr bool REC = (MODE == MODE_R_REC || MODE == MODE_I_PEEK);
    const int lane = threadIdx.x;
    const int L = xcd_remap(blockIdx.x, a.nwg);
    const int zchunk = L / a.ywg;
    const int ytile = (L - zchunk * a.ywg) * a.wpg + threadIdx.y;
    if (ytile >= a.ytiles) return;  // whole wave leaves: no barriers below

    const bool act = lane < a.nl;
    const int lc = act ? lane : 0;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const long plane = (long)nx * ny;
    const int j0 = ytile * RY;
    const int k0 = zchunk * a.zc;
    const int k1 = min(k0 + a.zc, nz);

    // tile rows: real rows are stored; rows past ny are wrapped copies (or
    // zero rows) that only serve as y neighbours
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
    auto load_row = [&](const T* base, int jj, int kk, VT(&out)[G]) {
        if (jj < 0 || kk < 0) {
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int e = 0; e < W; ++e) out[g].v[e] = T(0);
            return;
        }
        const T* p = base + (long)kk * plane + (long)jj * nx + (long)lc * W;
#pragma unroll
        for (int g = 0; g < G; ++g) out[g] = ldv<T, W>(p + (long)g * a.nl * W);
    };
    // U and V are read once per launch (no neighbour reads them): with nt_in
    // (grids far beyond the memory-side cache) they stream past it
    auto load_own = [&](const T* base, int jj, int kk, VT(&out)[G]) {
        const T* p = base + (long)kk * plane + (long)jj * nx + (long)lc * W;
        if (a.nt_in) {
#pragma unroll
            for (int g = 0; g < G; ++g) out[g] = ldv_nt<T, W>(p + (long)g * a.nl * W);
        } else {
#pragma unroll
            for (int g = 0; g < G; ++g) out[g] = ldv<T, W>(p + (long)g * a.nl * W);
        }
    };

    VT sp[RY][G], sc[RY][G], sn[RY][G];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        load_row(a.S, jrow[r], kwrap(k0 - 1), sp[r]);
        load_row(a.S, jrow[r], k0, sc[r]);
    }

    double f0 = 0.0, f1 = 0.0, q = 0.0, nv = 0.0, pl = 0.0;
    const int nl = a.nl;
    const int src_l = (lane == 0) ? nl - 1 : lane - 1;
    const int src_r = (lane == nl - 1) ? 0 : lane + 1;

    for (int k = k0; k < k1; ++k) {
        const int kn = kwrap(k + 1);
        VT hl[G], hh[G], u[RY][G], vv[RY][G];
#pragma unroll
        for (int r = 0; r < RY; ++r) load_row(a.S, jrow[r], kn, sn[r]);
        load_row(a.S, jlo, k, hl);
        load_row(a.S, jhi, k, hh);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (real[r]) {
                load_own(a.U, jrow[r], k, u[r]);
                load_own(a.V, jrow[r], k, vv[r]);
            }
        }
        const T cak = ld_uniform(a.ca, k);
        const T cbk = ld_uniform(a.cb, k);
        const bool at_det = (k == a.k_det);
        const bool at_up = (k == a.k_up);

#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (!real[r]) continue;
            VT un[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                // x neighbours across vector edges
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
                    const T c = sc[r][g].v[e];
                    const T xl = (e > 0) ? sc[r][g].v[e - 1] : xl_edge;
                    const T xr = (e < W - 1) ? sc[r][g].v[e + 1] : xr_edge;
                    const T yl = (r > 0) ? sc[r - 1][g].v[e] : hl[g].v[e];
                    const T yr = (r < RY - 1) ? sc[r + 1][g].v[e] : hh[g].v[e];
                    const T zl = sp[r][g].v[e];
                    const T zr = sn[r][g].v[e];
                    const T hx = hterm(c, xl, xr, yl, yr, zl, zr, vterm(vv[r][g].v[e], a.cv, a.d0),
                                       a.cx, a.cy, a.cz, a.dlo);
                    const T uo = u[r][g].v[e];
                    const T unew = IS_R ? upd_R(hx, uo, cak, cbk) : upd_I(hx, uo, cak, cbk);
                    un[g].v[e] = unew;
                    if (act) {
                        if (IS_R) {
                            if (at_det) f0 += (double)zr * ((double)uo + (double)unew);
                            if (at_up) f1 += (double)zl * ((double)uo + (double)unew);
                        }
                        if (REC) {
                            const double dc = (double)c, du = (double)uo, dn = (double)unew;
                            q += dc * dc + du * dn;
                            nv += IS_R ? (dn * dn + dc * dc) : (dc * dc + du * du);
                        }
                    }
                }
            }
            if (act) {
                const long off = (long)k * plane + (long)jrow[r] * nx + (long)lc * W;
                if (MODE != MODE_I_PEEK) {
#pragma unroll
                    for (int g = 0; g < G; ++g) stv<T, W>(a.U + off + (long)g * nl * W, un[g]);
                }
                if (REC && at_det) {
                    const long poff = (long)jrow[r] * nx + (long)lc * W;
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        VT rv;
#pragma unroll
                        for (int e = 0; e < W; ++e) {
                            const double dc = (double)sc[r][g].v[e];
                            const double dr = IS_R ? (double)un[g].v[e] : (double)u[r][g].v[e];
                            const double rho = dr * dr + dc * dc;
                            rv.v[e] = (T)rho;
                            pl += rho;
                            if (a.pixel) a.pixel[poff + (long)g * nl * W + e] += a.pixel_w * rho;
                        }
                        stv<T, W>(a.rec_plane + poff + (long)g * nl * W, rv);
                    }
                }
            }
        }
        // rotate the z window
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int g = 0; g < G; ++g) {
                sp[r][g] = sc[r][g];
                sc[r][g] = sn[r][g];
            }
    }

    const bool has_det = (a.k_det >= k0 && a.k_det < k1);
    const bool has_up = (a.k_up >= k0 && a.k_up < k1);
    if (IS_R) {
        if (has_det) {
            const double s = wave_sum(f0);
            if (lane == 0) a.flux_slots[ytile] = s;
        }
        if (has_up) {
            const double s = wave_sum(f1);
            if (lane == 0) a.flux_slots[a.ytiles + ytile] = s;
        }
    }
    if (REC) {
        const double sq = wave_sum(q);
        const double sn_ = wave_sum(nv);
        const long slot = (long)zchunk * a.ytiles + ytile;
        if (lane == 0) {
            a.part_q[slot] = sq;
            a.part_naive[slot] = sn_;
        }
        if (has_det) {
            const double sp_ = wave_sum(pl);
            if (lane == 0) a.part_plane[ytile] = sp_;
        }
    }
}

}  // namespace tdse
