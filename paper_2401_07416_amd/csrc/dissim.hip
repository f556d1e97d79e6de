// Trajectory dissimilarity of eq. (16), arXiv 2401.07416 section 3.2: for
// every pair (k, j) of trajectories, the time average of the L2 distance
// between their detector-plane densities,
//   d_kj = sum_t w_t sqrt(dA sum_p (rho_k,t,p - rho_j,t,p)^2),
// with the quadrature weights w_t carrying 1 / (t1 - t0).
//
// FP32 frames (the records) go to the FP64 matrix cores as a Gram
// contraction of shifted frames (dissim_gram_kernel, below).  FP64 frames
// keep the direct form on the vector ALU, where an FP64 Gram expansion
// would lose close pairs to cancellation: register tiled like a GEMM, a
// workgroup owns a 64 x 64 block of pairs, each thread a 4 x 4 sub-block,
// pixels stream through LDS in chunks of 32, and the squared differences of
// a chunk are summed with fused multiply-adds.  Each workgroup covers a
// range of frames and writes its partial time sums; a second kernel adds
// the partials in a fixed order, so the result is bitwise reproducible and
// exactly symmetric.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>

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

// FP32 frames on the matrix cores.  The distance does not change when every
// frame of a time t is shifted by the same image c_t, and with x_k = rho_k - c
//   sum_p (rho_k - rho_j)^2 = |x_k|^2 + |x_j|^2 - 2 x_k . x_j,
// a Gram contraction.  Formed in FP64 from FP32 frames: x = rho - c is exact
// in FP64 with the shift c_t = the frame of trajectory 0, and the
// cancellation in the expansion costs a few FP64 ulps of |x_k|^2 + |x_j|^2:
// a squared frame distance d^2 carries a relative error of about
// eps64 (|x_k|^2 + |x_j|^2) / d^2, tiny while a pair's distance is not far
// below the distances to trajectory 0 (1e-15 for random frames), larger for
// a tight cluster far from trajectory 0 (pairs 1e-6 apart at unit distance
// from it: about 1e-4 in d^2); the FP64-frame form below has no such
// cancellation.  The Gram block of a workgroup (GB x GB pairs, sixteen wavefronts
// of 32 x 32 pairs: four per SIMD) accumulates on v_mfma_f64_16x16x4_f64
// over chunks of GPC pixels staged in LDS as FP64 rows; the squared norms
// come from the same FP64 values as they are staged.
constexpr int GB = 128;           // trajectories per block side
constexpr int GPC = 32;           // pixels per LDS chunk
constexpr int GLS = GPC + 2;      // LDS row stride in doubles (16-byte rows, spread banks)
constexpr int GTHREADS = 1024;
constexpr int GWN = GTHREADS == 1024 ? 2 : 4;  // 16-column tiles per wavefront (2 row tiles)
constexpr int GWC = GB / (16 * GWN);            // wavefronts across a block's columns
static_assert((GB / 32) * GWC * 64 == GTHREADS, "wavefront grid");
static_assert(GPC % 4 == 0 && GB % (GTHREADS / (GPC / 4)) == 0 && GPC / 4 <= 64, "staging map");
constexpr int GQ = GPC / 4;            // 4-pixel vectors per row and chunk
constexpr int GRP = GTHREADS / GQ;     // rows staged per pass
constexpr int GNP = GB / GRP;          // passes per side

typedef double dbl4 __attribute__((ext_vector_type(4)));

struct GramArgs {
    const float* frames;  // [K][T][P]
    const double* w;      // [T]
    double dA;
    int K, T;
    long P;
    int nb, npb, tpc;
    double tau;           // a frame's d^2 below tau (|x_k|^2 + |x_j|^2) marks the pair
    double* part;         // [ntc][K][K]
    unsigned* count;      // length of the list of marked pairs (zeroed here)
};

// four consecutive pixels p0 .. p0 + 3 of a row (zero past P)
template <bool VEC>
__device__ __forceinline__ float4 load4(const float* row, long p0, long P) {
    if (VEC) {
        if (p0 < P) return *reinterpret_cast<const float4*>(row + p0);
        return make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float4 r;
    r.x = p0 < P ? row[p0] : 0.f;
    r.y = p0 + 1 < P ? row[p0 + 1] : 0.f;
    r.z = p0 + 2 < P ? row[p0 + 2] : 0.f;
    r.w = p0 + 3 < P ? row[p0 + 3] : 0.f;
    return r;
}

// VEC: P is a multiple of 4 (whole float4 loads)
template <bool VEC>
__global__ __launch_bounds__(GTHREADS) void dissim_gram_kernel(GramArgs a) {
    __shared__ __align__(16) double As[2 * GB * GLS];
    __shared__ __align__(16) double Bs[2 * GB * GLS];
    __shared__ double nrm[2 * 2 * GB];
    const int q = blockIdx.x % a.npb;
    const int tc = blockIdx.x / a.npb;
    int bi, bj;
    pair_block(q, a.nb, &bi, &bj);
    const int r0 = bi * GB, c0 = bj * GB;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int wr = (wv / GWC) * 32, wc = (wv % GWC) * 16 * GWN;  // the wavefront's 32 x 16 GWN pairs
    const int li = lane & 15, lk = lane >> 4;
    const int t0 = tc * a.tpc;
    const int t1 = min(t0 + a.tpc, a.T);
    const long TP = (long)a.T * a.P;
    const long cpt = (a.P + GPC - 1) / GPC;
    const long nch = cpt * (t1 - t0);
    // the reduction that follows on the stream appends the marked pairs
    if (blockIdx.x == 0 && tid == 0) *a.count = 0u;

    // staging: rows srow + GRP i of each side, pixels 4 quad .. 4 quad + 3
    const int quad = tid % GQ, srow = tid / GQ;
    float4 ra[GNP], rb[GNP], rc;
    bool va[GNP], vb[GNP];
#pragma unroll
    for (int i = 0; i < GNP; ++i) {
        va[i] = r0 + srow + GRP * i < a.K;
        vb[i] = c0 + srow + GRP * i < a.K;
    }
    // chunk pc of frame t0 + f of the workgroup's frames (positions are
    // advanced incrementally: no 64-bit division in the loop)
    auto fetch = [&](int f, long pc) {
        const long p0 = pc * GPC + 4 * quad;
        const long off = (long)(t0 + f) * a.P;
#pragma unroll
        for (int i = 0; i < GNP; ++i) {
            ra[i] = va[i] ? load4<VEC>(a.frames + (long)(r0 + srow + GRP * i) * TP + off, p0, a.P)
                          : make_float4(0.f, 0.f, 0.f, 0.f);
            rb[i] = vb[i] ? load4<VEC>(a.frames + (long)(c0 + srow + GRP * i) * TP + off, p0, a.P)
                          : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        rc = load4<VEC>(a.frames + off, p0, a.P);   // the shift: trajectory 0
    };

    dbl4 g[2][GWN];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < GWN; ++n) g[m][n] = dbl4{0.0, 0.0, 0.0, 0.0};
    // the time sums live in this workgroup's own slab of the partials (the
    // pairs k <= j of its block), one read-modify-write per frame
    double* out = a.part + (long)tc * a.K * a.K;
    double na[GNP], nbv[GNP];
#pragma unroll
    for (int i = 0; i < GNP; ++i) na[i] = nbv[i] = 0.0;

    // one row's four staged values as FP64 x = rho - c (exact), into LDS,
    // with their squares added to the row's partial norm
    auto stage = [&](double* L, int row, const float4& v, bool valid, double& nacc) {
        double x0 = 0.0, x1 = 0.0, x2 = 0.0, x3 = 0.0;
        if (valid) {
            x0 = (double)v.x - (double)rc.x;
            x1 = (double)v.y - (double)rc.y;
            x2 = (double)v.z - (double)rc.z;
            x3 = (double)v.w - (double)rc.w;
        }
        nacc = __builtin_fma(x0, x0, nacc);
        nacc = __builtin_fma(x1, x1, nacc);
        nacc = __builtin_fma(x2, x2, nacc);
        nacc = __builtin_fma(x3, x3, nacc);
        double2* d = reinterpret_cast<double2*>(L + row * GLS + 4 * quad);
        d[0] = make_double2(x0, x1);
        d[1] = make_double2(x2, x3);
    };

    // a row's norm over the frame: its GQ quad lanes (adjacent lanes)
    // combined by a butterfly, the same bits in each, into the frame's half
    // of nrm (halves alternate with the frame, so that a wavefront still in
    // the previous frame's end reads its own half)
    auto frame_norms = [&](int f) {
        double* nf = nrm + (f & 1) * 2 * GB;
#pragma unroll
        for (int i = 0; i < GNP; ++i) {
            double x = na[i], y = nbv[i];
#pragma unroll
            for (int s = 1; s < GQ; s <<= 1) {
                x += __shfl_xor(x, s);
                y += __shfl_xor(y, s);
            }
            if (quad == 0) {
                nf[srow + GRP * i] = x;
                nf[GB + srow + GRP * i] = y;
            }
            na[i] = 0.0;
            nbv[i] = 0.0;
        }
    };
    auto stage_chunk = [&](int buf) {
#pragma unroll
        for (int i = 0; i < GNP; ++i) {
            stage(As + buf * GB * GLS, srow + GRP * i, ra[i], va[i], na[i]);
            stage(Bs + buf * GB * GLS, srow + GRP * i, rb[i], vb[i], nbv[i]);
        }
    };

    // two LDS buffers: chunk c + 1 is staged into the other buffer while
    // chunk c is contracted (late in it: its loads, issued a chunk ahead,
    // have landed), one barrier per chunk
    auto advance = [&](int& f, long& pc) {
        if (++pc == cpt) {
            pc = 0;
            ++f;
        }
    };
    int fc = 0, fn = 0;     // frame of the current chunk and of the next one to fetch
    long pcc = 0, pn = 0;   // their chunks within the frame
    if (nch > 0) {
        fetch(fn, pn);
        stage_chunk(0);
        advance(fn, pn);
        if (nch > 1) {
            fetch(fn, pn);
            advance(fn, pn);
        }
    }
    __syncthreads();
    for (long c = 0; c < nch; ++c) {
        const int cur = (int)(c & 1);
        const double* Ac = As + cur * GB * GLS;
        const double* Bc = Bs + cur * GB * GLS;
        const bool frame_done = pcc == cpt - 1;
#pragma unroll
        for (int kk = 0; kk < GPC / 4; ++kk) {
            double av[2], bv[GWN];
#pragma unroll
            for (int m = 0; m < 2; ++m) av[m] = Ac[(wr + 16 * m + li) * GLS + 4 * kk + lk];
#pragma unroll
            for (int n = 0; n < GWN; ++n) bv[n] = Bc[(wc + 16 * n + li) * GLS + 4 * kk + lk];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int n = 0; n < GWN; ++n)
                    g[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[m], bv[n], g[m][n], 0, 0, 0);
            if (kk == GPC * 3 / 16) {
                // the staged norms so far cover the frame's chunks up to c
                if (frame_done) frame_norms(fc);
                if (c + 1 < nch) {
                    stage_chunk(cur ^ 1);
                    if (c + 2 < nch) {
                        fetch(fn, pn);
                        advance(fn, pn);
                    }
                }
            }
        }
        __syncthreads();
        if (frame_done) {
            const int f = fc;
            const double wt = a.w[t0 + f];
            const double* nf = nrm + (f & 1) * 2 * GB;
            // element r of a lane's accumulator is pair (4 r + lk, li) of the 16 x 16 tile
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int n = 0; n < GWN; ++n)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = wr + 16 * m + 4 * r + lk, col = wc + 16 * n + li;
                        const double ns = nf[row] + nf[GB + col];
                        const double d2 = ns - 2.0 * g[m][n][r];
                        const double v = wt * sqrt(a.dA * fmax(d2, 0.0));
                        g[m][n][r] = 0.0;
                        const int k = r0 + row, j = c0 + col;
                        if (k < a.K && j < a.K && k <= j) {
                            // a d^2 this small against the norms may be
                            // mostly the expansion's rounding: the partial
                            // turns negative (no contribution is) and stays
                            // so, and the pair goes to the direct form
                            double* o = out + (long)k * a.K + j;
                            const double prev = f == 0 ? 0.0 : *o;
                            const bool mark = k < j && d2 < a.tau * ns;
                            *o = (mark || prev < 0.0) ? -1.0 : prev + v;
                        }
                    }
            // nothing of the frame's epilogue stays in flight: the loop's
            // wait bookkeeping then never holds the next chunk's LDS reads
            // or the prefetch behind these accesses
            __builtin_amdgcn_s_waitcnt(0);
        }
        advance(fc, pcc);
    }
    // a diagonal block holds both (k, j) and (j, k): the pair with k < j
    // writes both, so the result is exactly symmetric; d_kk = 0
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < GWN; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = r0 + wr + 16 * m + 4 * r + lk, j = c0 + wc + 16 * n + li;
                if (k < a.K && j < a.K && k <= j) {
                    if (k == j)
                        out[(long)k * a.K + k] = 0.0;
                    else
                        out[(long)j * a.K + k] = out[(long)k * a.K + j];
                }
            }
}

// Adds the partial time sums in a fixed order.  A pair with a negative
// partial (marked by the Gram kernel) is appended to list (k < j, once per
// pair; the order of the list does not matter, each entry is evaluated on
// its own) and its entries are left for dissim_pairs_kernel.
__global__ __launch_bounds__(256) void dissim_reduce_kernel(const double* part, int ntc, int K,
                                                            double* out, int2* list, unsigned* count) {
    const long kk = (long)K * K;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < kk; i += (long)gridDim.x * 256) {
        double s = 0.0;
        bool marked = false;
        for (int c = 0; c < ntc; ++c) {
            const double v = part[(long)c * kk + i];
            marked |= v < 0.0;
            s += v;
        }
        out[i] = marked ? 0.0 : s;
        if (marked && list) {
            const int k = (int)(i / K), j = (int)(i - (long)k * K);
            if (k < j) list[atomicAdd(count, 1u)] = make_int2(k, j);
        }
    }
}

// The marked pairs in the direct form of eq. (16): per frame the sum over
// pixels of (rho_k - rho_j)^2, the differences of the FP32 values exact in
// FP64, fused multiply-adds.  A workgroup per pair of the list (a strided
// loop over the list), pixels strided over its threads, then a butterfly in
// each wavefront and the four wavefronts in order: the same bits on every
// run.  Writes d_kj and d_jk.
__global__ __launch_bounds__(256) void dissim_pairs_kernel(const float* frames, const double* w, double dA,
                                                           int K, int T, long P, const int2* list,
                                                           const unsigned* count, double* out) {
    __shared__ double red[4];
    const unsigned n = *count;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long TP = (long)T * P;
    for (unsigned it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 kj = list[it];
        const float* fa = frames + (long)kj.x * TP;
        const float* fb = frames + (long)kj.y * TP;
        double acc = 0.0;
        for (int t = 0; t < T; ++t) {
            double s = 0.0;
            for (long p = threadIdx.x; p < P; p += 256) {
                const double e = (double)fa[(long)t * P + p] - (double)fb[(long)t * P + p];
                s = __builtin_fma(e, e, s);
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
            if (lane == 0) red[wv] = s;
            __syncthreads();
            if (threadIdx.x == 0) acc += w[t] * sqrt(dA * (((red[0] + red[1]) + red[2]) + red[3]));
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            out[(long)kj.x * K + kj.y] = acc;
            out[(long)kj.y * K + kj.x] = acc;
        }
    }
}

struct Plan {
    int nb, npb, tpc, ntc;
};

// Gram kernel: frames per workgroup chosen so that the last round of
// workgroups over the compute units is as full as possible (cost = rounds x
// frames per workgroup, for 256 compute units; ties to more frames, less
// workspace)
Plan plan_gram(int K, int T) {
    Plan p;
    p.nb = (K + GB - 1) / GB;
    p.npb = p.nb * (p.nb + 1) / 2;
    constexpr long CUS = 256;
    long best = -1;
    p.tpc = 1;
    for (int tpc = 1; tpc <= T; ++tpc) {
        const long ntc = (T + tpc - 1) / tpc;
        const long cost = (p.npb * ntc + CUS - 1) / CUS * tpc;
        if (best < 0 || cost <= best) {
            best = cost;
            p.tpc = tpc;
        }
    }
    p.ntc = (T + p.tpc - 1) / p.tpc;
    return p;
}

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

// Workspace of a call: the partial sums (ntc x K x K doubles), and for FP32
// frames behind them the count and list of the pairs marked for the direct
// form (room for every pair k < j).
constexpr size_t kListHead = 256;
size_t part_bytes(const Plan& p, int K) { return (size_t)p.ntc * K * K * sizeof(double); }
size_t list_bytes(int K) { return kListHead + (size_t)K * (K - 1) / 2 * sizeof(int2); }
size_t need_bytes(int32_t precision, int K, int T) {
    return precision == TDSE_F32 ? part_bytes(plan_gram(K, T), K) + list_bytes(K)
                                 : part_bytes(plan_of(K, T), K);
}

}  // namespace

extern "C" tdse_status tdse_dissimilarity_workspace_size(int32_t K, int32_t T, size_t* bytes) {
    if (!bytes || K < 1 || T < 1) return TDSE_ERR_ARG;
    // the larger of the two precisions' needs
    *bytes = std::max(need_bytes(TDSE_F32, K, T), need_bytes(TDSE_F64, K, T));
    return TDSE_OK;
}

namespace {

// The launches of tdse_dissimilarity with its workspace at `ws` (laid out
// as need_bytes says; every entry a kernel reads is written first by an
// earlier one on the stream, so stale contents do no harm).
tdse_status dissim_launch(int32_t precision, const void* frames, int32_t K, int32_t T, int64_t P,
                          const double* weights, double dA, double* out, void* ws, hipStream_t st) {
    const Plan p = precision == TDSE_F32 ? plan_gram(K, T) : plan_of(K, T);
    const dim3 grid((unsigned)(p.npb * p.ntc));
    double* part = static_cast<double*>(ws);
    unsigned* count = nullptr;
    int2* list = nullptr;
    if (precision == TDSE_F32) {
        char* tail = static_cast<char*>(ws) + part_bytes(p, K);
        count = reinterpret_cast<unsigned*>(tail);
        list = reinterpret_cast<int2*>(tail + kListHead);
    }
    if (precision == TDSE_F32) {
        GramArgs g;
        g.frames = static_cast<const float*>(frames);
        g.w = weights;
        g.dA = dA;
        g.K = K;
        g.T = T;
        g.P = P;
        g.nb = p.nb;
        g.npb = p.npb;
        g.tpc = p.tpc;
        // The expansion's rounding error in a frame's d^2 is below about
        // 0.4 P eps64 (|x_k|^2 + |x_j|^2) (sequential sums of P / 8 pixels
        // per lane for the norms, P / 4 matrix steps for the cross term), so
        // an unmarked d^2 is good to 0.4 eps64 / 2^-30 = 5e-8 of itself.
        g.tau = std::ldexp((double)P, -30);
        g.part = part;
        g.count = count;
        const bool vec = P % 4 == 0 && (reinterpret_cast<uintptr_t>(frames) & 15) == 0;
        if (vec)
            hipLaunchKernelGGL(dissim_gram_kernel<true>, grid, dim3(GTHREADS), 0, st, g);
        else
            hipLaunchKernelGGL(dissim_gram_kernel<false>, grid, dim3(GTHREADS), 0, st, g);
    } else {
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
        a.part = part;
        hipLaunchKernelGGL(dissim_kernel<double>, grid, dim3(256), 0, st, a);
    }
    if (hipGetLastError() != hipSuccess) return TDSE_ERR_DEVICE;
    const long kk = (long)K * K;
    const unsigned g = (unsigned)std::min<long>((kk + 255) / 256, 4096);
    hipLaunchKernelGGL(dissim_reduce_kernel, dim3(g), dim3(256), 0, st,
                       static_cast<const double*>(part), p.ntc, (int)K, out, list, count);
    if (hipGetLastError() != hipSuccess) return TDSE_ERR_DEVICE;
    if (precision == TDSE_F32 && K > 1) {
        // usually an empty list: every workgroup reads the count and ends
        const unsigned gp = (unsigned)std::min<long>((long)K * (K - 1) / 2, 1024);
        hipLaunchKernelGGL(dissim_pairs_kernel, dim3(gp), dim3(256), 0, st,
                           static_cast<const float*>(frames), weights, dA, (int)K, (int)T, (long)P,
                           static_cast<const int2*>(list), static_cast<const unsigned*>(count), out);
    }
    return hipGetLastError() == hipSuccess ? TDSE_OK : TDSE_ERR_DEVICE;
}

// Checks shared by both entry points; *need = bytes of partial sums.
tdse_status dissim_check(int32_t precision, const void* frames, int32_t K, int32_t T, int64_t P,
                         const double* weights, double dA, const double* out, size_t* need) {
    if (!frames || !weights || !out || K < 1 || T < 1 || P < 1) return TDSE_ERR_ARG;
    if (precision != TDSE_F32 && precision != TDSE_F64) return TDSE_ERR_ARG;
    if (!(dA > 0)) return TDSE_ERR_ARG;
    const Plan p = precision == TDSE_F32 ? plan_gram(K, T) : plan_of(K, T);
    if ((long)p.npb * p.ntc > (1L << 31) - 1) return TDSE_ERR_ARG;
    *need = need_bytes(precision, K, T);
    return TDSE_OK;
}

// Partial sums of tdse_dissimilarity_noalloc: one fixed array per GPU,
// allocated with the code object, never by a call.  Host code must not use
// this name as a device address (on the host it names a stand-in); it uses
// the address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoallocScratchBytes = (size_t)TDSE_DISSIM_NOALLOC_MAX_BYTES;
static __device__ __align__(256) double scratch[kNoallocScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device.
tdse_status scratch_on_current_device(double** ptr) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return TDSE_ERR_DEVICE;
    if (dev >= kMaxDevices) return TDSE_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TDSE_ERR_DEVICE;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *ptr = g_scratch_ptr[dev];
    return TDSE_OK;
}

}  // namespace

extern "C" tdse_status tdse_dissimilarity(int32_t precision, const void* frames, int32_t K, int32_t T,
                                          int64_t P, const double* weights, double dA, double* out,
                                          void* workspace, size_t workspace_bytes, void* stream) {
    size_t need = 0;
    const tdse_status st = dissim_check(precision, frames, K, T, P, weights, dA, out, &need);
    if (st != TDSE_OK) return st;
    if (!workspace || workspace_bytes < need) return TDSE_ERR_ARG;
    return dissim_launch(precision, frames, K, T, P, weights, dA, out, workspace,
                         static_cast<hipStream_t>(stream));
}

extern "C" tdse_status tdse_dissimilarity_noalloc(int32_t precision, const void* frames, int32_t K,
                                                  int32_t T, int64_t P, const double* weights, double dA,
                                                  double* out, void* stream) {
    size_t need = 0;
    tdse_status st = dissim_check(precision, frames, K, T, P, weights, dA, out, &need);
    if (st != TDSE_OK) return st;
    if (need > kNoallocScratchBytes) return TDSE_ERR_CAPACITY;
    double* part = nullptr;
    st = scratch_on_current_device(&part);
    if (st != TDSE_OK) return st;
    return dissim_launch(precision, frames, K, T, P, weights, dA, out, part,
                         static_cast<hipStream_t>(stream));
}
