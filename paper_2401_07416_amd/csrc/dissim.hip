// Trajectory dissimilarity of eq. (16), arXiv 2401.07416 section 3.2: for
// every pair (k, j) of trajectories, the time average of the L2 distance
// between their detector-plane densities,
//   d_kj = sum_t w_t sqrt(dA sum_p (rho_k,t,p - rho_j,t,p)^2),
// with the quadrature weights w_t carrying 1 / (t1 - t0).
//
// The pixel sum is formed directly from the differences, not from the Gram
// expansion |a|^2 + |b|^2 - 2 a.b: trajectories that are close (the pairs a
// dissimilarity is for) would lose their distance to cancellation in the
// FP32 cross term.  So the contraction runs on the vector ALU, register
// tiled like a GEMM: a workgroup owns a 64 x 64 block of pairs, each thread a
// 4 x 4 sub-block, and pixels stream through LDS in chunks of 32; per chunk
// the squared differences are summed in the frame precision (fused
// multiply-adds) and then added to an FP64 accumulator.  Each workgroup covers a range of frames and
// writes its partial time sum; a second kernel adds the partials in a fixed
// order, so the result is bitwise reproducible and exactly symmetric.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/tdse.h"

namespace {

constexpr int BK = 64;   // trajectories per block side
constexpr int PC = 32;   // pixels per LDS chunk
constexpr int LS = BK + 4;  // LDS row stride (pixel-major rows of BK values)

template <typename T>
struct alignas(4 * sizeof(T)) vec_of {
    T v[4];
};

struct DissimArgs {
    const void* frames;   // [K][T][P]
    const double* w;      // [T]
    double dA;
    int K, T;
    long P;
    int nb;               // row blocks
    int npb;              // pair blocks (upper triangle with diagonal)
    int tpc;              // frames per workgroup
    double* part;         // [ntc][K][K]
};

// e * e + s with one rounding (a fused multiply-add): two instructions per
// pair and pixel with the subtraction, and a sum at least as accurate as
// the separately rounded product and add.
__device__ __forceinline__ float fma_of(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_of(double a, double b, double c) { return __builtin_fma(a, b, c); }

// pair block index -> (row block, column block), column >= row
__device__ __forceinline__ void pair_block(int q, int nb, int* bi, int* bj) {
    int r = 0;
    while (q >= nb - r) {
        q -= nb - r;
        ++r;
    }
    *bi = r;
    *bj = r + q;
}

// LDS tiles are pixel-major ([PC][BK], stride LS) so that each thread reads
// its 4 consecutive trajectories of a pixel with one vector read.
template <typename T>
__global__ __launch_bounds__(256) void dissim_kernel(DissimArgs a) {
    __shared__ __align__(16) T As[PC * LS];
    __shared__ __align__(16) T Bs[PC * LS];
    using V4 = vec_of<T>;
    const T* F = static_cast<const T*>(a.frames);
    const int q = blockIdx.x % a.npb;
    const int tc = blockIdx.x / a.npb;
    int bi, bj;
    pair_block(q, a.nb, &bi, &bj);
    const int r0 = bi * BK, c0 = bj * BK;
    const int tid = threadIdx.x;
    const int tr = tid >> 4, tcl = tid & 15;   // rows 4 tr .. 4 tr + 3, columns 4 tcl .. 4 tcl + 3
    const int t0 = tc * a.tpc;
    const int t1 = min(t0 + a.tpc, a.T);
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;

    // chunks of PC pixels of the workgroup's frames, in (frame, pixel) order;
    // the next chunk's values are loaded into registers while the current
    // one is summed from LDS
    constexpr int PER = BK * PC / 256;   // values per thread and tile
    const long cpt = (a.P + PC - 1) / PC;  // chunks per frame
    const long nch = cpt * (t1 - t0);
    T ra[PER], rb[PER];
    // value i of a thread's tile share: row (tid / PC) + i (256 / PC), pixel tid % PC
    constexpr int RSTEP = 256 / PC;
    const int row0 = tid / PC, col = tid - row0 * PC;
    const long rstride = (long)RSTEP * a.T * a.P;
    const T* pa = F + ((long)(r0 + row0) * a.T) * a.P + col;
    const T* pb = F + ((long)(c0 + row0) * a.T) * a.P + col;
    auto fetch = [&](long c) {
        const int t = t0 + (int)(c / cpt);
        const long p0 = (c % cpt) * PC;
        const bool pin = p0 + col < a.P;
        const long off = (long)t * a.P + p0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            ra[i] = (pin && r0 + row0 + RSTEP * i < a.K) ? pa[off + i * rstride] : T(0);
            rb[i] = (pin && c0 + row0 + RSTEP * i < a.K) ? pb[off + i * rstride] : T(0);
        }
    };
    double s64[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) s64[x][y] = 0.0;
    if (nch > 0) fetch(0);
    for (long c = 0; c < nch; ++c) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            As[col * LS + row0 + RSTEP * i] = ra[i];
            Bs[col * LS + row0 + RSTEP * i] = rb[i];
        }
        __syncthreads();
        if (c + 1 < nch) fetch(c + 1);
        T s[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) s[x][y] = T(0);
#pragma unroll 8
        for (int p = 0; p < PC; ++p) {
            const V4 av = *reinterpret_cast<const V4*>(As + p * LS + 4 * tr);
            const V4 bv = *reinterpret_cast<const V4*>(Bs + p * LS + 4 * tcl);
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    const T e = av.v[x] - bv.v[y];
                    s[x][y] = fma_of(e, e, s[x][y]);
                }
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) s64[x][y] += (double)s[x][y];
        if (c % cpt == cpt - 1) {
            // the frame is complete
            const double wt = a.w[t0 + (int)(c / cpt)];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    acc[x][y] += wt * sqrt(a.dA * s64[x][y]);
                    s64[x][y] = 0.0;
                }
        }
        __syncthreads();
    }
    double* out = a.part + (long)tc * a.K * a.K;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int k = r0 + 4 * tr + x, j = c0 + 4 * tcl + y;
            if (k < a.K && j < a.K) {
                out[(long)k * a.K + j] = acc[x][y];
                out[(long)j * a.K + k] = acc[x][y];
            }
        }
}

__global__ __launch_bounds__(256) void dissim_reduce_kernel(const double* part, int ntc, long kk,
                                                            double* out) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < kk; i += (long)gridDim.x * 256) {
        double s = 0.0;
        for (int c = 0; c < ntc; ++c) s += part[(long)c * kk + i];
        out[i] = s;
    }
}

struct Plan {
    int nb, npb, tpc, ntc;
};

Plan plan_of(int K, int T) {
    Plan p;
    p.nb = (K + BK - 1) / BK;
    p.npb = p.nb * (p.nb + 1) / 2;
    // enough workgroups to fill the chip: split the frames into chunks
    const int want = std::max(1, (2048 + p.npb - 1) / p.npb);
    p.ntc = std::min(T, want);
    p.tpc = (T + p.ntc - 1) / p.ntc;
    p.ntc = (T + p.tpc - 1) / p.tpc;
    return p;
}

}  // namespace

extern "C" tdse_status tdse_dissimilarity_workspace_size(int32_t K, int32_t T, size_t* bytes) {
    if (!bytes || K < 1 || T < 1) return TDSE_ERR_ARG;
    const Plan p = plan_of(K, T);
    *bytes = (size_t)p.ntc * K * K * sizeof(double);
    return TDSE_OK;
}

extern "C" tdse_status tdse_dissimilarity(int32_t precision, const void* frames, int32_t K, int32_t T,
                                          int64_t P, const double* weights, double dA, double* out,
                                          void* workspace, size_t workspace_bytes, void* stream) {
    if (!frames || !weights || !out || !workspace || K < 1 || T < 1 || P < 1) return TDSE_ERR_ARG;
    if (precision != TDSE_F32 && precision != TDSE_F64) return TDSE_ERR_ARG;
    if (!(dA > 0)) return TDSE_ERR_ARG;
    const Plan p = plan_of(K, T);
    if (workspace_bytes < (size_t)p.ntc * K * K * sizeof(double)) return TDSE_ERR_ARG;
    if ((long)p.npb * p.ntc > (1L << 31) - 1) return TDSE_ERR_ARG;
    DissimArgs a;
    a.frames = frames;
    a.w = weights;
    a.dA = dA;
    a.K = K;
    a.T = T;
    a.P = P;
    a.nb = p.nb;
    a.npb = p.npb;
    a.tpc = p.tpc;
    a.part = static_cast<double*>(workspace);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const dim3 grid((unsigned)(p.npb * p.ntc));
    if (precision == TDSE_F64)
        hipLaunchKernelGGL(dissim_kernel<double>, grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(dissim_kernel<float>, grid, dim3(256), 0, st, a);
    if (hipGetLastError() != hipSuccess) return TDSE_ERR_DEVICE;
    const long kk = (long)K * K;
    const unsigned g = (unsigned)std::min<long>((kk + 255) / 256, 4096);
    hipLaunchKernelGGL(dissim_reduce_kernel, dim3(g), dim3(256), 0, st,
                       static_cast<const double*>(workspace), p.ntc, kk, out);
    return hipGetLastError() == hipSuccess ? TDSE_OK : TDSE_ERR_DEVICE;
}
