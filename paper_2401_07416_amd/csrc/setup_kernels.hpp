// Device code of libtdse outside the half-step kernels: the fixed-order
// finalisation of the FP64 partial sums and the setup passes (potential,
// Gaussian packet, min/max of V).  Included by the runtime only.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.hpp"

namespace tdse {

// Fixed-order FP64 sum over a workgroup of 256 threads (wavefront
// butterflies, then the four wavefront totals in order).
__device__ __forceinline__ double block_sum256(double v, double* red) { return block_sum(v, red, 4); }

struct FinArgs {
    const double* flux_ring;  // [n_pending][2][ytiles]
    int n_pending, ytiles, has_up, record;
    long rec_idx;
    double dv_cz, dV;
    double* acc;              // acc[0] = accumulated flux
    const double* part_q;
    const double* part_naive;
    long n_part;
    const double* part_plane;
    double* scalars;          // [max_records][4]
};

// Folds the pending per-step flux partials into the accumulator in step
// order and, on record steps, writes {plane_sum, naive_norm, Q, flux_acc}.
__device__ __forceinline__ void finalize_body(const FinArgs& a) {
    __shared__ double red[4];
    const int t = threadIdx.x;
    double acc = a.acc[0];
    for (int s = 0; s < a.n_pending; ++s) {
        const double* f = a.flux_ring + (long)s * 2 * a.ytiles;
        double v = 0.0;
        for (int i = t; i < a.ytiles; i += 256) v += f[i] - f[a.ytiles + i];
        v = block_sum256(v, red);
        if (a.has_up) acc += a.dv_cz * v;
    }
    if (a.record) {
        double vq = 0.0, vn = 0.0, vp = 0.0;
        for (long i = t; i < a.n_part; i += 256) {
            vq += a.part_q[i];
            vn += a.part_naive[i];
        }
        for (int i = t; i < a.ytiles; i += 256) vp += a.part_plane[i];
        vq = block_sum256(vq, red);
        vn = block_sum256(vn, red);
        vp = block_sum256(vp, red);
        if (t == 0) {
            double* o = a.scalars + 4 * a.rec_idx;
            o[0] = a.dV * vp;
            o[1] = a.dV * vn;
            o[2] = a.dV * vq;
            o[3] = acc;
        }
    }
    if (t == 0) a.acc[0] = acc;
}

__global__ __launch_bounds__(256) void finalize_kernel(FinArgs a) { finalize_body(a); }

// One workgroup per configuration of a batch; pending count, record flag and
// the device record counter are shared by the launch.
struct BatchFin {
    const FinArgs* cfg;
    const long* rec_idx;
    int n_pending, record;
};

__global__ __launch_bounds__(256) void finalize_batch_kernel(BatchFin b) {
    FinArgs a = b.cfg[blockIdx.x];
    a.n_pending = b.n_pending;
    a.record = b.record;
    a.rec_idx = b.record ? *b.rec_idx : 0;
    finalize_body(a);
}

// Advance / set the device record counter of a batch (one lane, vector store).
__global__ void bump_counter_kernel(long* c) {
    if (threadIdx.x == 0) c[0] = c[0] + 1;
}

__global__ void set_counter_kernel(long* c, long v) {
    if (threadIdx.x == 0) c[0] = v;
}

// ---------------------------------------------------------------------------
// Setup kernels
// ---------------------------------------------------------------------------

// Per-block min, max and non-finite count of V (FP64), for E_max.
template <typename T>
__global__ __launch_bounds__(256) void minmax_kernel(const T* V, long n, double* out) {
    __shared__ double smin[256], smax[256], sbad[256];
    const int t = threadIdx.x;
    double mn = 1e308, mx = -1e308, bad = 0.0;
    for (long i = (long)blockIdx.x * 256 + t; i < n; i += (long)gridDim.x * 256) {
        const double v = (double)V[i];
        if (!isfinite(v)) {
            bad += 1.0;
            continue;
        }
        mn = fmin(mn, v);
        mx = fmax(mx, v);
    }
    smin[t] = mn;
    smax[t] = mx;
    sbad[t] = bad;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
            smin[t] = fmin(smin[t], smin[t + o]);
            smax[t] = fmax(smax[t], smax[t + o]);
            sbad[t] += sbad[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[3 * blockIdx.x + 0] = smin[0];
        out[3 * blockIdx.x + 1] = smax[0];
        out[3 * blockIdx.x + 2] = sbad[0];
    }
}

struct PotArgs {
    int nx, ny, nz;
    double dx, dy, dz, Lx, Ly, Lz;
    int bcx, bcy, bcz, screened;
    const double* atoms;    // [n][5] in caller order
    const int* plane_ptr;   // [nz + 1]
    const int* plane_idx;   // candidate atoms per plane, ascending atom index
    double soft, cutoff, kappa, a0;
};

__device__ __forceinline__ double min_image(double u, double L) { return u - L * rint(u / L); }

// V(r) = sum_a amp_a v_Z(d_a) over the plane's candidate atoms in atom order,
// v_Z(d) = -Z kappa exp(-d/lam_Z) / sqrt(d^2 + s^2), lam_Z = 0.8853 a0 Z^(-1/3).
template <typename T>
__global__ __launch_bounds__(256) void potential_kernel(PotArgs p, T* V) {
    const int k = blockIdx.y;
    const long c = (long)blockIdx.x * 256 + threadIdx.x;
    const long nxy = (long)p.nx * p.ny;
    if (c >= nxy) return;
    const int i = (int)(c % p.nx), j = (int)(c / p.nx);
    const double r0 = i * p.dx, r1 = j * p.dy, r2 = k * p.dz;
    double v = 0.0;
    for (int q = p.plane_ptr[k]; q < p.plane_ptr[k + 1]; ++q) {
        const double* at = p.atoms + 5 * (long)p.plane_idx[q];
        double u0 = r0 - at[0], u1 = r1 - at[1], u2 = r2 - at[2];
        if (!p.bcx) u0 = min_image(u0, p.Lx);
        if (!p.bcy) u1 = min_image(u1, p.Ly);
        if (!p.bcz) u2 = min_image(u2, p.Lz);
        const double d = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
        if (d >= p.cutoff) continue;
        const double Z = at[3];
        const double e = p.screened ? exp(-d / (0.8853 * p.a0 * pow(Z, -1.0 / 3.0))) : 1.0;
        v += at[4] * (-Z * p.kappa * e / sqrt(d * d + p.soft * p.soft));
    }
    V[(long)k * nxy + c] = (T)v;
}

struct GaussAxisArgs {
    int n[3];
    double d[3], L[3], r0[3], k0[3];
    int periodic[3];
    double sigma, hbar, mass, t0, t1;
    double* fac;  // [2 times][nx + ny + nz][2] complex
};

// One factor of eq. (3) evolved freely to time t (closed form), summed over
// periodic images |m| <= 2:
//   phi = (pi s^2)^(-1/4) (1 + i tau)^(-1/2)
//         exp(-(x - x0 - v t)^2 / (2 s^2 (1 + i tau)) + i k (x - x0) - i hbar k^2 t / 2m)
__device__ void gauss_phi(double x, double x0, double k, double s, double t, double hbar,
                          double mass, double* re, double* im) {
    const double tau = hbar * t / (mass * s * s);
    const double v = hbar * k / mass;
    const double u = x - x0 - v * t;
    const double den = 2.0 * s * s * (1.0 + tau * tau);
    const double are = -(u * u) / den;
    const double aim = (u * u) * tau / den + k * (x - x0) - hbar * k * k * t / (2.0 * mass);
    // (1 + i tau)^(-1/2) = (1 + tau^2)^(-1/4) exp(-i atan(tau) / 2)
    const double mod = pow(1.0 + tau * tau, -0.25) * pow(M_PI * s * s, -0.25) * exp(are);
    const double ph = aim - 0.5 * atan(tau);
    double sn, cs;
    sincos(ph, &sn, &cs);
    *re = mod * cs;
    *im = mod * sn;
}

__global__ __launch_bounds__(256) void gauss_axis_kernel(GaussAxisArgs a) {
    const int tot = a.n[0] + a.n[1] + a.n[2];
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= 2 * tot) return;
    const int which = idx / tot;
    int m = idx % tot;
    int ax = 0;
    while (m >= a.n[ax]) {
        m -= a.n[ax];
        ++ax;
    }
    const double t = which ? a.t1 : a.t0;
    const double x = m * a.d[ax];
    double sre = 0.0, sim = 0.0;
    const int ni = a.periodic[ax] ? 2 : 0;
    for (int im = -ni; im <= ni; ++im) {
        double re, imv;
        gauss_phi(x + im * a.L[ax], a.r0[ax], a.k0[ax], a.sigma, t, a.hbar, a.mass, &re, &imv);
        sre += re;
        sim += imv;
    }
    a.fac[2 * idx] = sre;
    a.fac[2 * idx + 1] = sim;
}

struct GaussCellArgs {
    int nx, ny, nz;
    const double* fac;  // as written by gauss_axis_kernel
    double scale;
    double* partial;    // [gridDim.x * gridDim.y] (norm pass)
};

__device__ __forceinline__ void cmul(double ar, double ai, double br, double bi, double* cr,
                                     double* ci) {
    *cr = ar * br - ai * bi;
    *ci = ar * bi + ai * br;
}

__device__ __forceinline__ void psi_cell(const double* f, int nx, int ny, int i, int j, int k,
                                         double* re, double* im) {
    double r, m;
    cmul(f[2 * i], f[2 * i + 1], f[2 * (nx + j)], f[2 * (nx + j) + 1], &r, &m);
    cmul(r, m, f[2 * (nx + ny + k)], f[2 * (nx + ny + k) + 1], re, im);
}

// Per-block partial of sum |psi(r, 0)|^2.
__global__ __launch_bounds__(256) void gauss_norm_kernel(GaussCellArgs a) {
    __shared__ double red[256];
    const int k = blockIdx.y;
    const long c = (long)blockIdx.x * 256 + threadIdx.x;
    const long nxy = (long)a.nx * a.ny;
    double v = 0.0;
    if (c < nxy) {
        double re, im;
        psi_cell(a.fac, a.nx, a.ny, (int)(c % a.nx), (int)(c / a.nx), k, &re, &im);
        v = re * re + im * im;
    }
    v = block_sum256(v, red);
    if (threadIdx.x == 0) a.partial[(long)k * gridDim.x + blockIdx.x] = v;
}

// R = s Re psi(r, t0), I = s Im psi(r, t1).
template <typename T>
__global__ __launch_bounds__(256) void gauss_write_kernel(GaussCellArgs a, T* R, T* I) {
    const int k = blockIdx.y;
    const long c = (long)blockIdx.x * 256 + threadIdx.x;
    const long nxy = (long)a.nx * a.ny;
    if (c >= nxy) return;
    const int i = (int)(c % a.nx), j = (int)(c / a.nx);
    double re0, im0, re1, im1;
    psi_cell(a.fac, a.nx, a.ny, i, j, k, &re0, &im0);
    const long off = (long)(a.nx + a.ny + a.nz);
    psi_cell(a.fac + 2 * off, a.nx, a.ny, i, j, k, &re1, &im1);
    R[(long)k * nxy + c] = (T)(a.scale * re0);
    I[(long)k * nxy + c] = (T)(a.scale * im1);
}

}  // namespace tdse

namespace tdse {

struct VjpArgs {
    int nx, ny, nz;
    double dx, dy, dz, Lx, Ly, Lz;
    int bcx, bcy, bcz, screened;
    const double* atoms;  // [n][5]
    const double* gV;     // dL/dV [nz][ny][nx]
    double soft, cutoff, kappa, a0;
    double* out;          // [n][4]: dL/dx, dL/dy, dL/dz, dL/damp
};

// Index range of one axis around coordinate x within the cutoff: the cells
// i0 .. i0 + cnt - 1 (wrapped on a periodic axis, clipped on a zero one),
// each cell of the axis at most once.
__device__ __forceinline__ void axis_range(double x, double cut, double d, int n, int zero,
                                           int* i0, int* cnt) {
    int lo = (int)ceil((x - cut) / d), hi = (int)floor((x + cut) / d);
    if (zero) {
        lo = max(lo, 0);
        hi = min(hi, n - 1);
        *i0 = lo;
        *cnt = max(0, hi - lo + 1);
        return;
    }
    if (hi - lo + 1 >= n) {
        *i0 = 0;
        *cnt = n;
        return;
    }
    *i0 = lo;
    *cnt = hi - lo + 1;
}

// Chain rule from dL/dV to the atoms:
//   dL/dX_a = sum_r gV(r) (-amp_a v'(d) u / d),  dL/damp_a = sum_r gV(r) v(d),
// u = r - X_a (minimum image), d = |u| < cutoff; a cell exactly on the atom
// adds nothing to dL/dX_a (cusp of the screened potential).  One workgroup
// per atom, fixed-order reduction.
__global__ __launch_bounds__(256) void potential_vjp_kernel(VjpArgs p) {
    __shared__ double red[256];
    const double* at = p.atoms + 5 * (long)blockIdx.x;
    int i0, ci, j0, cj, k0, ck;
    axis_range(at[0], p.cutoff, p.dx, p.nx, p.bcx, &i0, &ci);
    axis_range(at[1], p.cutoff, p.dy, p.ny, p.bcy, &j0, &cj);
    axis_range(at[2], p.cutoff, p.dz, p.nz, p.bcz, &k0, &ck);
    const long tot = (long)ci * cj * ck;
    double sx = 0.0, sy = 0.0, sz = 0.0, sa = 0.0;
    const double Z = at[3], amp = at[4];
    const double lam = 0.8853 * p.a0 * pow(Z, -1.0 / 3.0);
    for (long c = threadIdx.x; c < tot; c += 256) {
        const int ii = (int)(c % ci), jj = (int)((c / ci) % cj), kk = (int)(c / ((long)ci * cj));
        int i = i0 + ii, j = j0 + jj, k = k0 + kk;
        if (!p.bcx) i = ((i % p.nx) + p.nx) % p.nx;
        if (!p.bcy) j = ((j % p.ny) + p.ny) % p.ny;
        if (!p.bcz) k = ((k % p.nz) + p.nz) % p.nz;
        double ux = i * p.dx - at[0], uy = j * p.dy - at[1], uz = k * p.dz - at[2];
        if (!p.bcx) ux = min_image(ux, p.Lx);
        if (!p.bcy) uy = min_image(uy, p.Ly);
        if (!p.bcz) uz = min_image(uz, p.Lz);
        const double d = sqrt(ux * ux + uy * uy + uz * uz);
        if (d >= p.cutoff) continue;
        const double w = p.gV[((long)k * p.ny + j) * p.nx + i];
        const double e = p.screened ? exp(-d / lam) : 1.0;
        const double v = -Z * p.kappa * e / sqrt(d * d + p.soft * p.soft);
        sa += w * v;
        if (d > 0.0) {
            const double inv_lam = p.screened ? 1.0 / lam : 0.0;
            const double dv = v * (-inv_lam - d / (d * d + p.soft * p.soft));
            const double f = -amp * dv / d;
            sx += w * f * ux;
            sy += w * f * uy;
            sz += w * f * uz;
        }
    }
    sx = block_sum256(sx, red);
    sy = block_sum256(sy, red);
    sz = block_sum256(sz, red);
    sa = block_sum256(sa, red);
    if (threadIdx.x == 0) {
        double* o = p.out + 4 * (long)blockIdx.x;
        o[0] = sx;
        o[1] = sy;
        o[2] = sz;
        o[3] = sa;
    }
}

// Potential from a table over one unit cell (section 2.3: the cell's
// potential is repeated in x and y and interpolated onto the mesh points),
// trilinear.  Sample (a, b, c) of the table [uz][uy][ux] sits at origin +
// (a sx, b sy, c sz); the cell repeats in x and y, and the table is held
// constant beyond its first and last z planes.
struct InterpArgs {
    const double* table;
    int ux, uy, uz;
    double sx, sy, sz, ox, oy, oz;
    int nx, ny, nz;
    double dx, dy, dz;
};

// Per-axis samples and weight of one mesh index: the lower table sample a0,
// the upper a1 and the weight t of a1.
struct AxisW {
    int a0, a1;
    double t;
};

// fractional table coordinate u -> lower sample (wrapped), upper sample and weight
__device__ __forceinline__ AxisW cell_axis(double u, int n) {
    const double f = floor(u);
    AxisW w;
    w.t = u - f;
    long a = (long)f % n;
    if (a < 0) a += n;
    w.a0 = (int)a;
    w.a1 = (int)((a + 1) % n);
    return w;
}

// The weights of every mesh index of the three axes, once per call:
// ax[0 .. nx) for x, ax[nx .. nx+ny) for y (both periodic over the cell),
// ax[nx+ny .. nx+ny+nz) for z (clamped to the table's z range).
__global__ __launch_bounds__(256) void interp_axes_kernel(InterpArgs a, AxisW* ax) {
    const long n = (long)a.nx + a.ny + a.nz;
    for (long c = (long)blockIdx.x * 256 + threadIdx.x; c < n; c += (long)gridDim.x * 256) {
        AxisW w{0, 0, 0.0};
        if (c < a.nx) {
            w = cell_axis(((double)c * a.dx - a.ox) / a.sx, a.ux);
        } else if (c < (long)a.nx + a.ny) {
            w = cell_axis(((double)(c - a.nx) * a.dy - a.oy) / a.sy, a.uy);
        } else if (a.uz > 1) {
            const long k = c - a.nx - a.ny;
            double u = ((double)k * a.dz - a.oz) / a.sz;
            u = fmin(fmax(u, 0.0), (double)(a.uz - 1));
            w.a0 = min((int)floor(u), a.uz - 2);
            w.t = u - (double)w.a0;
            w.a1 = w.a0 + 1;
        }
        ax[c] = w;
    }
}

// One workgroup: plane k = blockIdx.y, a segment of 256 x columns and rows
// [j0, j0 + rows) (blockIdx.x = segment + nseg * row group).  Each thread
// holds its column's x weights and reads the row's y and the plane's z
// weights as wave-uniform values, so a cell costs its eight table samples
// (four table rows that the whole row shares, from the caches), the blends
// in x, then y, then z, and one coalesced store.
template <typename T>
__global__ __launch_bounds__(256) void interp_potential_kernel(InterpArgs a, const AxisW* ax, int nseg,
                                                               int rows, T* V) {
    const int seg = blockIdx.x % nseg;
    const int j0 = (blockIdx.x / nseg) * rows;
    const int k = blockIdx.y;
    const int i = seg * 256 + threadIdx.x;
    if (i >= a.nx) return;   // no barriers below
    const AxisW wx = ax[i];
    const AxisW wz = ax[a.nx + a.ny + k];
    const double tx = wx.t, sx = 1.0 - tx;
    const double tz = wz.t;
    const long plane = (long)a.uy * a.ux;
    const double* p0 = a.table + (long)wz.a0 * plane;
    const double* p1 = a.table + (long)wz.a1 * plane;
    T* out = V + ((long)k * a.ny) * a.nx + i;
    const int j1 = min(j0 + rows, a.ny);
    for (int j = j0; j < j1; ++j) {
        const AxisW wy = ax[a.nx + j];
        const double ty = wy.t;
        const long r0 = (long)wy.a0 * a.ux, r1 = (long)wy.a1 * a.ux;
        const double b00 = sx * p0[r0 + wx.a0] + tx * p0[r0 + wx.a1];
        const double b10 = sx * p0[r1 + wx.a0] + tx * p0[r1 + wx.a1];
        const double b01 = sx * p1[r0 + wx.a0] + tx * p1[r0 + wx.a1];
        const double b11 = sx * p1[r1 + wx.a0] + tx * p1[r1 + wx.a1];
        const double c0 = (1.0 - ty) * b00 + ty * b10;
        const double c1 = (1.0 - ty) * b01 + ty * b11;
        out[(long)j * a.nx] = (T)((1.0 - tz) * c0 + tz * c1);
    }
}

// The same with the z blend of the workgroup's mesh plane done once per
// table sample, Z[b][a] = (1 - tz) T[c0][b][a] + tz T[c1][b][a], and then
// the y blend of each of its rows once per sample of the row,
// Y[r][a] = (1 - ty_r) Z[b0_r][a] + ty_r Z[b1_r][a], both staged in LDS
// when they fit (rows of ux + 1 samples, the last a copy of the first, so
// the upper x sample is always the next one).  A cell then costs one paired
// LDS read and the x blend (3 FP64 operations instead of 21).  The same
// trilinear value, blended z, y, x instead of x, y, z: it differs from that
// order by FP64 rounding only.
template <typename T>
__global__ __launch_bounds__(256) void interp_potential_lds_kernel(InterpArgs a, const AxisW* ax, int nseg,
                                                                   int rows, T* V) {
    extern __shared__ double zl[];   // Z: [uy][ux + 1], then Y: [rows][ux + 1]
    const int seg = blockIdx.x % nseg;
    const int j0 = (blockIdx.x / nseg) * rows;
    const int k = blockIdx.y;
    const int ux1 = a.ux + 1;
    const int per = a.uy * ux1;
    const int j1 = min(j0 + rows, a.ny);
    const AxisW wz = ax[a.nx + a.ny + k];
    const long plane = (long)a.uy * a.ux;
    const double* t0 = a.table + (long)wz.a0 * plane;
    const double* t1 = a.table + (long)wz.a1 * plane;
    for (int t = threadIdx.x; t < per; t += 256) {
        const int r = t / ux1, q = t - r * ux1;
        const long src = (long)r * a.ux + (q == a.ux ? 0 : q);
        zl[t] = (1.0 - wz.t) * t0[src] + wz.t * t1[src];
    }
    __syncthreads();
    double* yl = zl + per;
    const int ny1 = (j1 - j0) * ux1;
    for (int t = threadIdx.x; t < ny1; t += 256) {
        const int r = t / ux1, q = t - r * ux1;
        const AxisW wy = ax[a.nx + j0 + r];
        yl[t] = (1.0 - wy.t) * zl[wy.a0 * ux1 + q] + wy.t * zl[wy.a1 * ux1 + q];
    }
    __syncthreads();
    const int i = seg * 256 + threadIdx.x;
    if (i >= a.nx) return;   // after the last barrier
    const AxisW wx = ax[i];
    const double tx = wx.t, sx = 1.0 - tx;
    const double* yx = yl + wx.a0;
    T* out = V + ((long)k * a.ny) * a.nx + i;
    for (int j = j0; j < j1; ++j) {
        const double* y = yx + (j - j0) * ux1;
        __builtin_nontemporal_store((T)(sx * y[0] + tx * y[1]), out + (long)j * a.nx);
    }
}

}  // namespace tdse
