// libtdse runtime: the C ABI declared in include/tdse.h.
//
// The host side validates descriptions, carves the caller's workspace,
// builds the coefficient tables, picks the x layout and tile shape of the
// half-step kernels and drives the step loop on the handle's stream.  All
// arithmetic of the method runs in the kernels of kernels.hpp.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include <unistd.h>

#include "../../include/tdse.h"
#include "kernels.hpp"
#include "setup_kernels.hpp"
#include "fused.hpp"
#include "fused2.hpp"
#include "adjoint.hpp"
#include "adjoint_fused.hpp"
#include "paper_layout.hpp"

using namespace tdse;

struct tdse_batch_ctx;

struct tdse_ctx {
    tdse_desc d;
    // whole record intervals of one-pass steps replay a captured graph (an
    // internal one-member batch) when the stream is not the null stream
    bool graph_on = true;
    tdse_batch_ctx* gb = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    // x layout and tile: W-element vectors; the vector half-step kernel's
    // row of G groups of NL lanes when half_vec (nx = W G NL, NL <= 64),
    // else the any-width half-step kernel
    int W = 1, G = 1, NL = 1;
    bool half_vec = true;
    int rows = 2, waves = 4, zc = 16;
    // one-pass (fused) step: rows per thread M, z chunk, enabled flag
    int fm = 3, fzc = 64, ft = 256;
    bool fpf = false;
    bool fused = false;
    // two-step sweep: interior tile width, rows per thread, z chunk
    bool two = false;
    int t2x = 56, t2m = 2, t2zc = 64, t2t = 256;
    int t2ty = 0;   // requested interior tile height (0: the tallest the threads cover)
    bool t2pf = false;
    int lds_max = 65536;   // dynamic + static LDS per workgroup of the device
    int cus = 256;         // compute units of the device
    // adjoint: checkpoints every adj_K steps of an adj_N-step forward run
    void* adj_ws = nullptr;
    int64_t adj_N = 0;
    // a second stream (default priority) on which the adjoint recomputes
    // the next segment while the handle's stream sweeps the current one
    // backwards, and the events that order the two
    hipStream_t adj_stream = nullptr;
    hipEvent_t adj_ev[5] = {};
    int adj_K = 0;
    // bound memory
    void* R = nullptr;
    void* I = nullptr;
    void* V = nullptr;
    void* R2 = nullptr;  // second state pair of the one-pass step
    void* I2 = nullptr;
    void* ws = nullptr;
    void* rec = nullptr;
    double* scal = nullptr;
    double* pix = nullptr;
    size_t ws_bytes = 0;
    // workspace carve
    void* ca = nullptr;
    void* cb = nullptr;
    double* acc = nullptr;
    double* flux_ring = nullptr;
    double* part_q = nullptr;
    double* part_naive = nullptr;
    double* part_plane = nullptr;
    double* red = nullptr;
    double* gfac = nullptr;
    int F = 1;
    // state machine
    bool bound = false, finalized = false, ready = false;
    double dt = 0.0, emax = 0.0;
    double c[4] = {0, 0, 0, 0};
    std::vector<double> wcap;
    std::vector<double> ca_h, cb_h;
    std::vector<float> caf_h, cbf_h;
    // the longest run of planes [unit_lo, unit_hi) without absorption (ca =
    // cb = 1 exactly in the state precision)
    int unit_lo = 0, unit_hi = 0;
    int64_t step = 0;
    int pending = 0;
    std::string err;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_kind;
    size_t ev_used = 0;
};

// A batch: many handles stepped together by one launch per step, the steps
// of one record interval captured in a HIP graph.
struct tdse_batch_ctx {
    std::vector<tdse_ctx*> members;
    hipStream_t stream = nullptr;
    int precision = TDSE_F32;
    int64_t h = 0;       // record interval shared by the members
    int S = 0;           // steps per graph replay
    int W = 0, M = 3, zc = 64, nt = 256;
    bool pf = false;
    // two-step sweep for the whole batch (when every member fits it)
    bool two = true;
    int t2x = 80, t2zc = 32, t2m = 1, t2t = 1024;
    bool t2pf = true;
    bool use2 = false;  // chosen at prepare
    int par = 0;        // state pair holding the members' current level
    size_t lds = 0;
    int total_wg = 0;
    void* d_cfg = nullptr;     // FusedArgs<T>[n] or Fused2Args<T>[n]
    int* d_wg = nullptr;       // [n + 1]
    long* d_rec = nullptr;     // record counter
    void* d_fin = nullptr;     // FinArgs[n]
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph1 = nullptr;     // the interval starting from pair 1 (two-step, odd S/2)
    hipGraphExec_t exec1 = nullptr;
    bool prepared = false;
    bool owns = true;    // members are destroyed with the batch
    // device memory of the tables (d_cfg, d_fin, d_wg, d_rec), borrowed
    // from the caller (tdse_batch_bind_workspace) or, for a handle's own
    // graph replays, from the handle's workspace
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int64_t step = 0;
    std::string err;
};

namespace {

constexpr size_t ALIGN = 256;
constexpr int RED_SLOTS = 3 * 4096;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Bytes of the device tables of an n-member batch: the per-member kernel
// arguments (either form), the finalisation arguments, the workgroup
// starts and the record counter, each 256-byte aligned.
size_t batch_tables_bytes(size_t n) {
    const size_t cfg = std::max({sizeof(FusedArgs<float>), sizeof(FusedArgs<double>),
                                 sizeof(Fused2Args<float>), sizeof(Fused2Args<double>)});
    return align_up(n * cfg) + align_up(n * sizeof(FinArgs)) + align_up((n + 1) * sizeof(int)) +
           align_up(sizeof(long));
}


size_t elem_size(const tdse_desc& d) { return d.precision == TDSE_F64 ? 8 : 4; }

tdse_status fail(tdse_ctx* h, tdse_status s, const std::string& msg) {
    if (h) h->err = msg;
    return s;
}

tdse_status hip_check(tdse_ctx* h, hipError_t e, const char* what) {
    if (e == hipSuccess) return TDSE_OK;
    return fail(h, TDSE_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(h, call)                                          \
    do {                                                          \
        tdse_status s_ = hip_check((h), (call), #call);           \
        if (s_ != TDSE_OK) return s_;                             \
    } while (0)

// Step outputs (and the half-step's own-cell inputs) carry the
// non-temporal hint when the five state-sized arrays a step touches exceed
// the 256 MB memory-side cache (MALL): they are evicted before the next
// step reads them in any case, and without the hint they displace input
// lines that neighbouring tiles re-read.
constexpr size_t MALL_BYTES = (size_t)256 << 20;

bool stream_outputs(size_t state_bytes_total) { return 5 * state_bytes_total > MALL_BYTES; }

// The diagonal 2 (cx + cy + cz) of the 7-point Laplacian in the state
// precision's coefficients, as hi + lo parts: FP32 coefficients sum exactly
// in FP64, and hi + lo holds that sum exactly; FP64 kernels do not use it.
template <typename T>
void diag_parts(const tdse_ctx* h, T* hi, T* lo) {
    const double d = 2.0 * ((double)(T)h->c[0] + (double)(T)h->c[1] + (double)(T)h->c[2]);
    *hi = (T)d;
    *lo = (T)(d - (double)*hi);
}

size_t state_bytes(const tdse_desc& d) {
    return (size_t)d.nx * d.ny * d.nz * (d.precision == TDSE_F64 ? 8 : 4);
}

struct Layout {
    size_t ca, cb, acc, flux, part_q, part_n, part_p, red, gfac, gtab, total;
    int F;
};

int flux_ring_steps(const tdse_desc& d) {
    if (d.record_every > 0) return (int)std::min<int64_t>(d.record_every, 256);
    return 256;
}

Layout layout_of(const tdse_desc& d) {
    Layout L{};
    const size_t es = elem_size(d);
    const size_t nz = (size_t)d.nz, ny = (size_t)d.ny;
    L.F = flux_ring_steps(d);
    size_t o = 0;
    L.ca = o; o = align_up(o + nz * es);
    L.cb = o; o = align_up(o + nz * es);
    L.acc = o; o = align_up(o + 8 * sizeof(double));
    L.flux = o; o = align_up(o + (size_t)L.F * 2 * ny * sizeof(double));
    // partial-sum slots: one per (z chunk, y tile) of any tile shape, and
    // one per (256-cell block, plane) for the packet normalisation
    const size_t nparts = std::max(ny * nz, ((size_t)d.nx * ny + 255) / 256 * nz);
    L.part_q = o; o = align_up(o + nparts * sizeof(double));
    L.part_n = o; o = align_up(o + nparts * sizeof(double));
    L.part_p = o; o = align_up(o + ny * sizeof(double));
    L.red = o; o = align_up(o + (size_t)RED_SLOTS * sizeof(double));
    L.gfac = o; o = align_up(o + 2 * 2 * ((size_t)d.nx + ny + nz) * sizeof(double));
    // tables of the one-member batch behind the handle's graph replays
    L.gtab = o; o = align_up(o + batch_tables_bytes(1));
    L.total = o;
    return L;
}

// Widest vector of the precision's widths (4, 2, 1 floats; 2, 1 doubles)
// that divides nx, so every row starts on a vector boundary.
int vector_width(const tdse_desc& d) {
    const int w0 = d.precision == TDSE_F64 ? 2 : 4;
    for (int w = w0; w > 1; w /= 2)
        if (d.nx % w == 0) return w;
    return 1;
}

// The extents the kernels take: byte offsets within one z plane are 32-bit
// (buffer resources of one plane, out-of-range reads as zero), so a plane
// must stay below OOB = 0x7ffffff0 bytes; y and z extents within the
// launch-grid and table limits.
tdse_status supported_shape(const tdse_desc& d) {
    const int64_t es = d.precision == TDSE_F64 ? 8 : 4;
    if ((double)d.nx * (double)d.ny * (double)es >= (double)0x7ffffff0) return TDSE_ERR_UNSUPPORTED;
    if (d.ny > (int64_t)1 << 24 || d.nz > 65535) return TDSE_ERR_UNSUPPORTED;
    return TDSE_OK;
}

// nx = W * G * NL with NL <= 64 lanes; widest vectors first, fewest groups.
bool choose_x_layout(const tdse_desc& d, int* W, int* G, int* NL) {
    const int ws32[3] = {4, 2, 1};
    const int ws64[2] = {2, 1};
    const int* wl = d.precision == TDSE_F64 ? ws64 : ws32;
    const int nw = d.precision == TDSE_F64 ? 2 : 3;
    for (int a = 0; a < nw; ++a) {
        const int w = wl[a];
        if (d.nx % w) continue;
        const int64_t m = d.nx / w;
        for (int g : {1, 2, 4, 8}) {
            if (m % g) continue;
            if (m / g <= 64) {
                *W = w;
                *G = g;
                *NL = (int)(m / g);
                return true;
            }
        }
    }
    return false;
}

// Default half-step tile: 2 rows per wavefront, 4 wavefronts, 2-plane z
// chunks.  Short chunks give many workgroups whose plane loads overlap
// (neighbouring chunks' planes come from the L2), which beats long z
// marches on small, cache-resident grids (2-3x) and on large ones alike
// (7% on 512x512x1024 FP32, 21% on 256x256x512 FP32; 3% slower on
// 1024x1024x256 FP32, whose long rows already make the workgroups many).
// Below two workgroups per CU the chunks go to one plane, then the rows
// to one (64^3: 24 -> 30, 48^3: 10 -> 14 Gcell-steps/s).
void default_tile(tdse_ctx* h) {
    const tdse_desc& d = h->d;
    auto nwg = [&](int rows, int zc) {
        const int64_t ytiles = (d.ny + rows - 1) / rows;
        return ((ytiles + 3) / 4) * ((d.nz + zc - 1) / zc);
    };
    h->rows = d.ny >= 2 ? 2 : 1;
    h->waves = 4;
    h->zc = (int)std::min<int64_t>(2, d.nz);
    const int64_t want = 2L * h->cus;
    if (nwg(h->rows, h->zc) < want) h->zc = 1;
    if (nwg(h->rows, h->zc) < want) h->rows = 1;
}

// Default one-pass tile: the first band shape and z chunk, longest chunks
// first, whose workgroups keep the CUs busy.
void default_fused_tile(tdse_ctx* h);

struct TileDims {
    int ytiles, ywg, nzc, nwg, zc;
};

// Geometry of the half-step kernels: the vector kernel's y tiles of `rows`
// rows, `waves` tiles per workgroup, z chunks of zc planes; without a vector
// layout of nx, the any-width kernel's one row per workgroup and z chunks
// sized for about 2048 workgroups (rows, waves and zc do not apply).
TileDims tile_dims(const tdse_ctx* h, int rows, int waves, int zc) {
    TileDims t;
    if (!h->half_vec) {
        const int64_t ny = h->d.ny, nz = h->d.nz;
        const int64_t want = std::max<int64_t>(1, (2048 + ny - 1) / ny);
        t.zc = (int)std::max<int64_t>(1, (nz + want - 1) / want);
        t.ytiles = (int)ny;
        t.ywg = (int)ny;
        t.nzc = (int)((nz + t.zc - 1) / t.zc);
        t.nwg = t.ywg * t.nzc;
        return t;
    }
    t.zc = zc;
    t.ytiles = (int)((h->d.ny + rows - 1) / rows);
    t.ywg = (t.ytiles + waves - 1) / waves;
    t.nzc = (int)((h->d.nz + zc - 1) / zc);
    t.nwg = t.ywg * t.nzc;
    return t;
}

}  // namespace

namespace tdse {
// Half-step launchers, one translation unit per (precision, vector width)
// so the many template instances compile in parallel (half_*.hip).
hipError_t launch_half_any_f32(int mode, dim3 grid, hipStream_t st, const HalfArgs<float>& a,
                               hipEvent_t e0, hipEvent_t e1);
hipError_t launch_half_any_f64(int mode, dim3 grid, hipStream_t st, const HalfArgs<double>& a,
                               hipEvent_t e0, hipEvent_t e1);
hipError_t launch_half_f32_w4(int g, int rows, int mode, dim3 grid, dim3 block, hipStream_t st,
                              const HalfArgs<float>& a, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_half_f32_w2(int g, int rows, int mode, dim3 grid, dim3 block, hipStream_t st,
                              const HalfArgs<float>& a, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_half_f32_w1(int g, int rows, int mode, dim3 grid, dim3 block, hipStream_t st,
                              const HalfArgs<float>& a, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_half_f64_w2(int g, int rows, int mode, dim3 grid, dim3 block, hipStream_t st,
                              const HalfArgs<double>& a, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_half_f64_w1(int g, int rows, int mode, dim3 grid, dim3 block, hipStream_t st,
                              const HalfArgs<double>& a, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_fused_f32(int w, int m, bool rec, bool pf, dim3 grid, int nt, size_t lds, hipStream_t st,
                            const FusedArgs<float>& a, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_adjoint_f32(int w, int g, int phase, dim3 grid, dim3 block, hipStream_t st,
                              const AdjArgs<float>& a);
hipError_t launch_adjoint_f64(int w, int g, int phase, dim3 grid, dim3 block, hipStream_t st,
                              const AdjArgs<double>& a);
hipError_t launch_fused_batch_f32(int w, int m, bool rec, bool pf, dim3 grid, int nt, size_t lds,
                                  hipStream_t st, const BatchStep<float>& b);
hipError_t launch_fused_batch_f64(int w, int m, bool rec, bool pf, dim3 grid, int nt, size_t lds,
                                  hipStream_t st, const BatchStep<double>& b);
hipError_t launch_fused_f64(int w, int m, bool rec, bool pf, dim3 grid, int nt, size_t lds, hipStream_t st,
                            const FusedArgs<double>& a, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_fused2_f32(int w, int m, int nt, bool rec, bool pf, dim3 grid, size_t lds, hipStream_t st,
                             const Fused2Args<float>& a, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_fused2_f64(int w, int m, int nt, bool rec, bool pf, dim3 grid, size_t lds, hipStream_t st,
                             const Fused2Args<double>& a, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_fused2_batch_f32(int w, int m, int nt, bool rec, bool pf, dim3 grid, size_t lds,
                                   hipStream_t st, const Batch2Step<float>& b);
hipError_t launch_fused2_batch_f64(int w, int m, int nt, bool rec, bool pf, dim3 grid, size_t lds,
                                   hipStream_t st, const Batch2Step<double>& b);
hipError_t fused2_batch_allow_lds_f32(int w, int m, int nt, size_t lds);
hipError_t launch_adjoint_fused_f32(int w, int m, dim3 grid, size_t lds, hipStream_t st,
                                    const AdjFusedArgs<float>& a);
hipError_t launch_adjoint_fused_f64(int w, int m, dim3 grid, size_t lds, hipStream_t st,
                                    const AdjFusedArgs<double>& a);
hipError_t fused2_batch_allow_lds_f64(int w, int m, int nt, size_t lds);
}  // namespace tdse

namespace {

hipError_t launch_half_f32(int w, int g, int rows, int mode, dim3 grid, dim3 block, hipStream_t st,
                           const HalfArgs<float>& a, hipEvent_t e0, hipEvent_t e1) {
    switch (w) {
        case 4: return launch_half_f32_w4(g, rows, mode, grid, block, st, a, e0, e1);
        case 2: return launch_half_f32_w2(g, rows, mode, grid, block, st, a, e0, e1);
        default: return launch_half_f32_w1(g, rows, mode, grid, block, st, a, e0, e1);
    }
}

hipError_t launch_half_f64(int w, int g, int rows, int mode, dim3 grid, dim3 block, hipStream_t st,
                           const HalfArgs<double>& a, hipEvent_t e0, hipEvent_t e1) {
    switch (w) {
        case 2: return launch_half_f64_w2(g, rows, mode, grid, block, st, a, e0, e1);
        default: return launch_half_f64_w1(g, rows, mode, grid, block, st, a, e0, e1);
    }
}

// Fill a HalfArgs for one half-step.  mode selects the kernel; rec_idx is
// the record slot for record modes; flux_slot the ring row for eq. (8).
template <typename T>
HalfArgs<T> make_args(tdse_ctx* h, int mode, int rows, int waves, int zc, long rec_idx,
                      int flux_slot) {
    const tdse_desc& d = h->d;
    const TileDims td = tile_dims(h, rows, waves, zc);
    HalfArgs<T> a;
    const bool isR = (mode == MODE_R || mode == MODE_R_REC);
    a.U = static_cast<T*>(isR ? h->R : h->I);
    a.S = static_cast<const T*>(isR ? h->I : h->R);
    a.V = static_cast<const T*>(h->V);
    a.ca = static_cast<const T*>(h->ca);
    a.cb = static_cast<const T*>(h->cb);
    a.cx = (T)h->c[0];
    a.cy = (T)h->c[1];
    a.cz = (T)h->c[2];
    a.cv = (T)h->c[3];
    diag_parts(h, &a.d0, &a.dlo);
    a.nx = (int)d.nx;
    a.ny = (int)d.ny;
    a.nz = (int)d.nz;
    a.nl = h->NL;
    a.ytiles = td.ytiles;
    a.wpg = waves;
    a.ywg = td.ywg;
    a.zc = td.zc;
    a.nzc = td.nzc;
    a.nwg = td.nwg;
    a.bcx = d.bc[0] == TDSE_BC_ZERO;
    a.bcy = d.bc[1] == TDSE_BC_ZERO;
    a.bcz = d.bc[2] == TDSE_BC_ZERO;
    a.k_det = (int)d.k_det;
    const bool has_up = !(a.bcz && d.k_det + 1 >= d.nz);
    a.k_up = has_up ? (int)((d.k_det + 1) % d.nz) : -1;
    a.flux_slots = h->flux_ring + (size_t)flux_slot * 2 * td.ytiles;
    const size_t es = sizeof(T);
    a.rec_plane = h->rec ? reinterpret_cast<T*>(static_cast<char*>(h->rec) +
                                                (size_t)rec_idx * d.nx * d.ny * es)
                         : nullptr;
    a.part_q = h->part_q;
    a.part_naive = h->part_naive;
    a.part_plane = h->part_plane;
    a.pixel = (d.flags & TDSE_FLAG_PIXEL_INTEGRAL) ? h->pix : nullptr;
    a.pixel_w = (double)d.record_every * h->dt;
    a.nt_in = stream_outputs(state_bytes(d));
    if (mode == MODE_I || mode == MODE_R) a.pixel = nullptr;
    return a;
}

// Event pair around the next launch when timing is on.  kind: 0 = eq. (9)
// half-step, 1 = eq. (8) half-step, 2 = one-pass step, 3 = two-step sweep;
// plus 4 for a launch that writes a record.
tdse_status timing_events(tdse_ctx* h, int kind, hipEvent_t* e0, hipEvent_t* e1) {
    *e0 = *e1 = nullptr;
    if (!h->timing) return TDSE_OK;
    while (h->ev.size() < h->ev_used + 2) {
        hipEvent_t e;
        HIPCHK(h, hipEventCreate(&e));
        h->ev.push_back(e);
        h->ev_kind.push_back(0);
    }
    *e0 = h->ev[h->ev_used];
    *e1 = h->ev[h->ev_used + 1];
    h->ev_kind[h->ev_used] = kind;
    h->ev_used += 2;
    return TDSE_OK;
}

tdse_status launch_half(tdse_ctx* h, int mode, int rows, int waves, int zc, long rec_idx,
                        int flux_slot) {
    const TileDims td = tile_dims(h, rows, waves, zc);
    dim3 grid(td.nwg), block(64, waves);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (mode != MODE_I_PEEK) {
        tdse_status s = timing_events(h, mode == MODE_I ? 0 : (mode == MODE_R_REC ? 5 : 1), &e0, &e1);
        if (s != TDSE_OK) return s;
    }
    hipError_t e;
    if (h->d.precision == TDSE_F64) {
        HalfArgs<double> a = make_args<double>(h, mode, rows, waves, zc, rec_idx, flux_slot);
        e = h->half_vec ? launch_half_f64(h->W, h->G, rows, mode, grid, block, h->stream, a, e0, e1)
                        : launch_half_any_f64(mode, grid, h->stream, a, e0, e1);
    } else {
        HalfArgs<float> a = make_args<float>(h, mode, rows, waves, zc, rec_idx, flux_slot);
        e = h->half_vec ? launch_half_f32(h->W, h->G, rows, mode, grid, block, h->stream, a, e0, e1)
                        : launch_half_any_f32(mode, grid, h->stream, a, e0, e1);
    }
    return hip_check(h, e, "half-step launch");
}

// Geometry of the one-pass kernel: W-element vectors, tpr threads per row,
// rpp rows per pass of a 256-thread workgroup, band of ty = rpp*m - 2 rows.
struct FusedDims {
    int W, tpr, rpp, ty, nbands, nzc, nwg, threads;
    int zcu;  // the z chunk the geometry was made for
    size_t lds;
    bool ok;
};

FusedDims fused_dims(const tdse_ctx* h, int m, int zc, int threads = 0) {
    const tdse_desc& d = h->d;
    FusedDims f{};
    const int es = d.precision == TDSE_F64 ? 8 : 4;
    const int wl32[3] = {4, 2, 1}, wl64[2] = {2, 1};
    const int* wl = es == 8 ? wl64 : wl32;
    const int nw = es == 8 ? 2 : 3;
    f.threads = threads > 0 ? threads : h->ft;
    f.ok = false;
    for (int i = 0; i < nw; ++i) {
        if (d.nx % wl[i] == 0 && d.nx / wl[i] <= f.threads) {
            f.W = wl[i];
            f.ok = true;
            break;
        }
    }
    if (!f.ok) return f;
    f.tpr = (int)(d.nx / f.W);
    f.rpp = f.threads / f.tpr;
    f.ty = f.rpp * m - 2;
    f.nbands = f.ty > 0 ? (int)((d.ny + f.ty - 1) / f.ty) : 0;
    f.zcu = zc;
    f.nzc = (int)((d.nz + zc - 1) / zc);
    f.nwg = f.nbands * f.nzc;
    f.lds = (size_t)(3 * f.ty + 8) * d.nx * es;
    // dynamic LDS plus the 2 KB static reduction buffer stay under 64 KB
    f.ok = f.ty >= 1 && f.lds <= 65536 - 4096;
    return f;
}

template <typename T>
FusedArgs<T> make_fused_args(tdse_ctx* h, const FusedDims& f, bool rec, long rec_idx,
                             int flux_slot) {
    const tdse_desc& d = h->d;
    FusedArgs<T> a;
    a.R0 = static_cast<const T*>(h->R);
    a.I0 = static_cast<const T*>(h->I);
    a.R1 = static_cast<T*>(h->R2);
    a.I1 = static_cast<T*>(h->I2);
    a.V = static_cast<const T*>(h->V);
    a.ca = static_cast<const T*>(h->ca);
    a.cb = static_cast<const T*>(h->cb);
    a.cx = (T)h->c[0];
    a.cy = (T)h->c[1];
    a.cz = (T)h->c[2];
    a.cv = (T)h->c[3];
    diag_parts(h, &a.d0, &a.dlo);
    a.nx = (int)d.nx;
    a.ny = (int)d.ny;
    a.nz = (int)d.nz;
    a.tpr = f.tpr;
    a.rpp = f.rpp;
    a.ty = f.ty;
    a.nbands = f.nbands;
    a.zc = h->fzc;
    a.nzc = f.nzc;
    a.nwg = f.nwg;
    a.bcx = d.bc[0] == TDSE_BC_ZERO;
    a.bcy = d.bc[1] == TDSE_BC_ZERO;
    a.bcz = d.bc[2] == TDSE_BC_ZERO;
    a.k_det = (int)d.k_det;
    const bool has_up = !(a.bcz && d.k_det + 1 >= d.nz);
    a.k_up = has_up ? (int)((d.k_det + 1) % d.nz) : -1;
    a.flux_slots = h->flux_ring + (size_t)flux_slot * 2 * f.nbands;
    a.rec_plane = (rec && h->rec) ? reinterpret_cast<T*>(static_cast<char*>(h->rec) +
                                                         (size_t)rec_idx * d.nx * d.ny * sizeof(T))
                                  : nullptr;
    a.part_q = h->part_q;
    a.part_naive = h->part_naive;
    a.part_plane = h->part_plane;
    a.pixel = (rec && (d.flags & TDSE_FLAG_PIXEL_INTEGRAL)) ? h->pix : nullptr;
    a.pixel_w = (double)d.record_every * h->dt;
    a.nt_out = stream_outputs(state_bytes(d));
    return a;
}

// One one-pass step from (R, I) into (R2, I2); the caller swaps the pairs.
tdse_status launch_fused(tdse_ctx* h, const FusedDims& f, bool rec, long rec_idx, int flux_slot) {
    hipEvent_t e0, e1;
    tdse_status s = timing_events(h, rec ? 6 : 2, &e0, &e1);
    if (s != TDSE_OK) return s;
    hipError_t e;
    if (h->d.precision == TDSE_F64) {
        FusedArgs<double> a = make_fused_args<double>(h, f, rec, rec_idx, flux_slot);
        e = launch_fused_f64(f.W, h->fm, rec, h->fpf, dim3(f.nwg), f.threads, f.lds, h->stream, a, e0, e1);
    } else {
        FusedArgs<float> a = make_fused_args<float>(h, f, rec, rec_idx, flux_slot);
        e = launch_fused_f32(f.W, h->fm, rec, h->fpf, dim3(f.nwg), f.threads, f.lds, h->stream, a, e0, e1);
    }
    return hip_check(h, e, "one-pass step launch");
}

// Geometry of the two-step sweep for interior tile width tx, rows per
// thread m, z chunk zc and nt threads per workgroup; the supported
// (m, nt) are (2, 256), (3, 256), (1, 512), (2, 512) and (1, 1024).
struct Fused2Dims {
    int W, tx, ty, ex, ey, tpr, rpp, ntx, nty, ntiles, nzc, nwg, nt;
    size_t lds;
    bool ok;
};

// ty_req > 0 asks for a shorter tile than the threads cover (fewer rows per
// pass, the threads past them idle): a tile count that fills the last round
// of workgroups can outweigh the larger rim share.
Fused2Dims fused2_dims(const tdse_ctx* h, int tx, int m, int zc, int nt, int ty_req) {
    const tdse_desc& d = h->d;
    Fused2Dims f{};
    f.ok = false;
    const int es = d.precision == TDSE_F64 ? 8 : 4;
    const int wl32[3] = {4, 2, 1}, wl64[2] = {2, 1};
    const int* wl = es == 8 ? wl64 : wl32;
    const int nw = es == 8 ? 2 : 3;
    const bool pair_ok = (nt == 256 && (m == 2 || m == 3)) || (nt == 512 && (m == 1 || m == 2)) ||
                         (nt == 1024 && m == 1);
    if (tx < 8 || !pair_ok || zc < 1) return f;
    f.nt = nt;
    f.W = 0;
    for (int i = 0; i < nw; ++i) {
        if (d.nx % wl[i] == 0 && tx % wl[i] == 0 && (tx + 8) / wl[i] <= nt) {
            f.W = wl[i];
            break;
        }
    }
    if (!f.W) return f;
    f.tx = tx;
    f.ex = tx + 8;
    f.tpr = f.ex / f.W;
    f.rpp = nt / f.tpr;
    if (ty_req > 0) f.rpp = std::min(f.rpp, (ty_req + 8 + m - 1) / m);
    f.ey = f.rpp * m;
    f.ty = f.ey - 8;
    if (f.ty < 1) return f;
    f.ntx = (int)((d.nx + tx - 1) / tx);
    f.nty = (int)((d.ny + f.ty - 1) / f.ty);
    f.ntiles = f.ntx * f.nty;
    f.nzc = (int)((d.nz + zc - 1) / zc);
    f.nwg = f.ntiles * f.nzc;
    // eight buffers and one vector slot that idle threads write
    f.lds = (size_t)8 * (f.ey + 2) * f.ex * es + 16;
    // flux and partial slots are sized for ny per step / plane; 8 B per
    // wavefront of static LDS for the reductions
    f.ok = f.ntiles <= d.ny && f.lds + 8 * (size_t)(nt / 64) <= (size_t)h->lds_max &&
           (long)f.nwg < (1L << 31);
    return f;
}

template <typename T>
Fused2Args<T> make_fused2_args(tdse_ctx* h, const Fused2Dims& f, bool rec, long rec_idx,
                               int flux_slot) {
    const tdse_desc& d = h->d;
    Fused2Args<T> a;
    a.R0 = static_cast<const T*>(h->R);
    a.I0 = static_cast<const T*>(h->I);
    a.R1 = static_cast<T*>(h->R2);
    a.I1 = static_cast<T*>(h->I2);
    a.V = static_cast<const T*>(h->V);
    a.ca = static_cast<const T*>(h->ca);
    a.cb = static_cast<const T*>(h->cb);
    a.cx = (T)h->c[0];
    a.cy = (T)h->c[1];
    a.cz = (T)h->c[2];
    a.cv = (T)h->c[3];
    diag_parts(h, &a.d0, &a.dlo);
    a.nx = (int)d.nx;
    a.ny = (int)d.ny;
    a.nz = (int)d.nz;
    a.tx = f.tx;
    a.ty = f.ty;
    a.ex = f.ex;
    a.ey = f.ey;
    a.tpr = f.tpr;
    a.rpp = f.rpp;
    a.ntx = f.ntx;
    a.ntiles = f.ntiles;
    a.zc = h->t2zc;
    a.nzc = f.nzc;
    a.nwg = f.nwg;
    a.bcx = d.bc[0] == TDSE_BC_ZERO;
    a.bcy = d.bc[1] == TDSE_BC_ZERO;
    a.bcz = d.bc[2] == TDSE_BC_ZERO;
    a.k_det = (int)d.k_det;
    const bool has_up = !(a.bcz && d.k_det + 1 >= d.nz);
    a.k_up = has_up ? (int)((d.k_det + 1) % d.nz) : -1;
    a.flux_a = h->flux_ring + (size_t)flux_slot * 2 * f.ntiles;
    a.flux_b = h->flux_ring + (size_t)(flux_slot + 1) * 2 * f.ntiles;
    a.rec_plane = rec ? static_cast<T*>(h->rec) + (size_t)rec_idx * d.nx * d.ny : nullptr;
    a.part_q = h->part_q;
    a.part_naive = h->part_naive;
    a.part_plane = h->part_plane;
    a.pixel = (rec && (d.flags & TDSE_FLAG_PIXEL_INTEGRAL)) ? h->pix : nullptr;
    a.pixel_w = (double)d.record_every * h->dt;
    a.nt_out = stream_outputs(state_bytes(d));
    a.ulo = h->unit_lo;
    a.uhi = h->unit_hi;
    return a;
}

// Two steps n -> n+2 into the second state pair; the record of level n+2
// if rec.  Flux partials go to ring slots flux_slot and flux_slot + 1.
tdse_status launch_fused2(tdse_ctx* h, const Fused2Dims& f, bool rec, long rec_idx, int flux_slot) {
    hipEvent_t e0, e1;
    tdse_status s = timing_events(h, rec ? 7 : 3, &e0, &e1);
    if (s != TDSE_OK) return s;
    hipError_t e;
    if (h->d.precision == TDSE_F64) {
        Fused2Args<double> a = make_fused2_args<double>(h, f, rec, rec_idx, flux_slot);
        e = launch_fused2_f64(f.W, h->t2m, f.nt, rec, h->t2pf, dim3(f.nwg), f.lds, h->stream, a, e0, e1);
    } else {
        Fused2Args<float> a = make_fused2_args<float>(h, f, rec, rec_idx, flux_slot);
        e = launch_fused2_f32(f.W, h->t2m, f.nt, rec, h->t2pf, dim3(f.nwg), f.lds, h->stream, a, e0, e1);
    }
    return hip_check(h, e, "two-step sweep launch");
}

// Fold n_pending steps of flux partials (slots per step each) into the
// accumulator; on record steps also write the record scalars from n_part
// partial slots.
tdse_status launch_finalize(tdse_ctx* h, int n_pending, bool record, long rec_idx, int slots,
                            long n_part) {
    const tdse_desc& d = h->d;
    FinArgs a;
    a.flux_ring = h->flux_ring;
    a.n_pending = n_pending;
    a.ytiles = slots;
    a.has_up = !(d.bc[2] == TDSE_BC_ZERO && d.k_det + 1 >= d.nz);
    a.record = record ? 1 : 0;
    a.rec_idx = rec_idx;
    a.dV = d.dx * d.dy * d.dz;
    a.dv_cz = a.dV * h->c[2];
    a.acc = h->acc;
    a.part_q = h->part_q;
    a.part_naive = h->part_naive;
    a.n_part = n_part;
    a.part_plane = h->part_plane;
    a.scalars = h->scal;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, h->stream, a);
    return hip_check(h, hipGetLastError(), "finalize launch");
}

// Record 0 of a freshly set state: rho^0, Q^0 with a non-storing peek of
// eq. (9), the naive norm; flux and record count reset.
tdse_status begin_records(tdse_ctx* h) {
    HIPCHK(h, hipMemsetAsync(h->acc, 0, 8 * sizeof(double), h->stream));
    h->pending = 0;
    if (h->d.record_every <= 0) return TDSE_OK;
    if (h->d.flags & TDSE_FLAG_PIXEL_INTEGRAL) {
        HIPCHK(h, hipMemsetAsync(h->pix, 0, (size_t)h->d.nx * h->d.ny * sizeof(double), h->stream));
    }
    tdse_status s = launch_half(h, MODE_I_PEEK, h->rows, h->waves, h->zc, 0, 0);
    if (s != TDSE_OK) return s;
    const TileDims td = tile_dims(h, h->rows, h->waves, h->zc);
    return launch_finalize(h, 0, true, 0, td.ytiles, (long)td.nzc * td.ytiles);
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) % ALIGN) == 0; }

// Adjoint workspace: checkpoints of levels 0, K, 2K, ... < N, the K + 1
// states of one recomputed segment, r and its second buffer, i and A i_t,
// and (FP32) the segment accumulator of dL/dV.  Each array is [nz][ny][nx]
// in the state precision.
struct AdjLayout {
    size_t arr, nck, ckpt, seg, rb, rc, ia, ib, gv, total;
};

AdjLayout adj_layout(const tdse_desc& d, int64_t N, int K) {
    AdjLayout L{};
    L.arr = align_up((size_t)d.nx * d.ny * d.nz * elem_size(d));
    L.nck = (size_t)((N + K - 1) / K);
    size_t o = 0;
    L.ckpt = o; o += 2 * L.nck * L.arr;
    // two banks of segment states: one recomputed while the other is swept
    L.seg = o; o += 2 * 2 * ((size_t)K + 1) * L.arr;
    L.rb = o; o += L.arr;
    L.rc = o; o += L.arr;
    L.ia = o; o += L.arr;
    L.ib = o; o += L.arr;
    L.gv = o; o += L.arr;
    L.total = o;
    return L;
}

template <typename T>
AdjArgs<T> make_adj_args(tdse_ctx* h, const T* S, T* U, T* U2, const T* Rn, const T* Ih, T* gv) {
    const tdse_desc& d = h->d;
    const TileDims td = tile_dims(h, 1, h->waves, h->zc);
    AdjArgs<T> a;
    a.S = S;
    a.U = U;
    a.U2 = U2;
    a.V = static_cast<const T*>(h->V);
    a.Rn = Rn;
    a.Ih = Ih;
    a.gv = gv;
    a.ca = static_cast<const T*>(h->ca);
    a.cb = static_cast<const T*>(h->cb);
    a.cx = (T)h->c[0];
    a.cy = (T)h->c[1];
    a.cz = (T)h->c[2];
    a.cv = (T)h->c[3];
    a.nx = (int)d.nx;
    a.ny = (int)d.ny;
    a.nz = (int)d.nz;
    a.nl = h->NL;
    a.ytiles = td.ytiles;
    a.wpg = h->waves;
    a.ywg = td.ywg;
    a.zc = h->zc;
    a.nzc = td.nzc;
    a.nwg = td.nwg;
    a.bcx = d.bc[0] == TDSE_BC_ZERO;
    a.bcy = d.bc[1] == TDSE_BC_ZERO;
    a.bcz = d.bc[2] == TDSE_BC_ZERO;
    return a;
}

template <typename T>
tdse_status launch_adj(tdse_ctx* h, int phase, const AdjArgs<T>& a) {
    const TileDims td = tile_dims(h, 1, h->waves, h->zc);
    hipError_t e;
    if constexpr (sizeof(T) == 8)
        e = launch_adjoint_f64(h->W, h->G, phase, dim3(td.nwg), dim3(64, h->waves), h->stream, a);
    else
        e = launch_adjoint_f32(h->W, h->G, phase, dim3(td.nwg), dim3(64, h->waves), h->stream, a);
    return hip_check(h, e, "adjoint launch");
}

// One forward step from (Rs, Is) into (Rd, Id), no records, no flux
// accumulation (the flux ring slot 0 is scratch here).
// zc > 0: the one-pass step's z chunk for this call where that geometry is
// valid (the chunking does not change any cell's arithmetic)
tdse_status forward_step_explicit(tdse_ctx* h, void* Rs, void* Is, void* Rd, void* Id, int zc = 0) {
    const int szc = h->fzc;
    if (zc > 0 && fused_dims(h, h->fm, zc).ok) h->fzc = zc;
    const FusedDims fd = fused_dims(h, h->fm, h->fzc);
    void* sR = h->R;
    void* sI = h->I;
    void* sR2 = h->R2;
    void* sI2 = h->I2;
    tdse_status st = TDSE_OK;
    if (fd.ok) {
        h->R = Rs;
        h->I = Is;
        h->R2 = Rd;
        h->I2 = Id;
        st = launch_fused(h, fd, false, 0, 0);
    } else {
        const size_t bytes = (size_t)h->d.nx * h->d.ny * h->d.nz * elem_size(h->d);
        st = hip_check(h, hipMemcpyAsync(Rd, Rs, bytes, hipMemcpyDeviceToDevice, h->stream), "copy");
        if (st == TDSE_OK)
            st = hip_check(h, hipMemcpyAsync(Id, Is, bytes, hipMemcpyDeviceToDevice, h->stream), "copy");
        h->R = Rd;
        h->I = Id;
        if (st == TDSE_OK) st = launch_half(h, MODE_I, h->rows, h->waves, h->zc, 0, 0);
        if (st == TDSE_OK) st = launch_half(h, MODE_R, h->rows, h->waves, h->zc, 0, 0);
    }
    h->R = sR;
    h->I = sI;
    h->R2 = sR2;
    h->I2 = sI2;
    h->fzc = szc;
    return st;
}

// Geometry of the one-pass reverse step (the forward band mapping with 256
// threads, z chunks from 64 planes down to 2 until there are 1024
// workgroups: on 128x128x256 the 2-plane chunks make 1280 and the reverse
// pass 1.5% faster than 8-plane ones); not ok where the one-pass forward
// step is off.
FusedDims adj_fused_dims(const tdse_ctx* h) {
    FusedDims best{};
    best.ok = false;
    if (!h->fused) return best;
    for (int zc0 : {64, 32, 16, 8, 4, 2}) {
        const int zc = (int)std::min<int64_t>(zc0, h->d.nz);
        const FusedDims f = fused_dims(h, 2, zc, 256);
        if (!f.ok) return best;
        best = f;
        best.zcu = zc;
        if ((long)f.nwg >= 1024) break;
    }
    return best;
}

template <typename T>
tdse_status launch_adj_fused(tdse_ctx* h, const FusedDims& f, const T* r, const T* i, T* r_out,
                             T* i_out, const T* Rn, const T* Ih, T* gv) {
    const tdse_desc& d = h->d;
    AdjFusedArgs<T> a;
    a.r = r;
    a.i = i;
    a.r_out = r_out;
    a.i_out = i_out;
    a.V = static_cast<const T*>(h->V);
    a.Rn = Rn;
    a.Ih = Ih;
    a.gv = gv;
    a.ca = static_cast<const T*>(h->ca);
    a.cb = static_cast<const T*>(h->cb);
    a.cx = (T)h->c[0];
    a.cy = (T)h->c[1];
    a.cz = (T)h->c[2];
    a.cv = (T)h->c[3];
    a.nx = (int)d.nx;
    a.ny = (int)d.ny;
    a.nz = (int)d.nz;
    a.tpr = f.tpr;
    a.rpp = f.rpp;
    a.ty = f.ty;
    a.nbands = f.nbands;
    a.zc = f.zcu;
    a.nzc = f.nzc;
    a.nwg = f.nwg;
    a.bcx = d.bc[0] == TDSE_BC_ZERO;
    a.bcy = d.bc[1] == TDSE_BC_ZERO;
    a.bcz = d.bc[2] == TDSE_BC_ZERO;
    hipError_t e;
    if constexpr (sizeof(T) == 8)
        e = launch_adjoint_fused_f64(f.W, 2, dim3(f.nwg), f.lds, h->stream, a);
    else
        e = launch_adjoint_fused_f32(f.W, 2, dim3(f.nwg), f.lds, h->stream, a);
    return hip_check(h, e, "one-pass adjoint launch");
}

template <typename T>
tdse_status run_adjoint(tdse_ctx* h, const T* rho_bar, double* gV64, T* gR0, T* gI0) {
    const tdse_desc& d = h->d;
    const int64_t N = h->adj_N;
    const int K = h->adj_K;
    const AdjLayout L = adj_layout(d, N, K);
    char* w = static_cast<char*>(h->adj_ws);
    const long n = (long)d.nx * d.ny * d.nz;
    const long nxy = (long)d.nx * d.ny;
    auto ck = [&](size_t c, int which) { return reinterpret_cast<T*>(w + L.ckpt + (2 * c + which) * L.arr); };
    // state (which = 0: psiR, 1: psiI) of level s0 + m of the segment in bank b
    auto sgb = [&](int b, size_t m, int which) {
        return reinterpret_cast<T*>(w + L.seg + ((size_t)b * 2 * ((size_t)K + 1) + 2 * m + which) * L.arr);
    };
    T* rb = reinterpret_cast<T*>(w + L.rb);
    T* rc = reinterpret_cast<T*>(w + L.rc);
    T* ia = reinterpret_cast<T*>(w + L.ia);
    T* ib = reinterpret_cast<T*>(w + L.ib);
    T* gv = sizeof(T) == 8 ? reinterpret_cast<T*>(gV64) : reinterpret_cast<T*>(w + L.gv);
    const size_t bytes = (size_t)n * sizeof(T);
    HIPCHK(h, hipMemsetAsync(rb, 0, bytes, h->stream));
    HIPCHK(h, hipMemsetAsync(ia, 0, bytes, h->stream));
    HIPCHK(h, hipMemsetAsync(gV64, 0, (size_t)n * sizeof(double), h->stream));
    if (sizeof(T) != 8) HIPCHK(h, hipMemsetAsync(gv, 0, bytes, h->stream));
    const int64_t hrec = d.record_every;
    const long poff = (long)d.k_det * nxy;
    const unsigned gi = (unsigned)((nxy + 255) / 256);
    auto inject = [&](int64_t lev, const T* Rm, const T* Im) -> tdse_status {
        if (hrec <= 0 || lev % hrec != 0) return TDSE_OK;
        hipLaunchKernelGGL(adjoint_inject_kernel<T>, dim3(gi), dim3(256), 0, h->stream, rb, ia, Rm,
                           Im, rho_bar + (lev / hrec) * nxy, poff, nxy);
        return hip_check(h, hipGetLastError(), "inject launch");
    };
    // the one-pass reverse step where the one-pass forward step is on
    const FusedDims af = adj_fused_dims(h);
    // Segments are swept last to first.  Segment c's states are recomputed
    // from its checkpoint into bank c mod 2 on the second stream while the
    // handle's stream sweeps segment c + 1 (bank (c + 1) mod 2) backwards:
    // ev[b] (recompute into bank b done) gates the sweep, ev[2 + b] (sweep
    // of bank b done) gates the next recompute into it, ev[4] hands the
    // forward run's checkpoints to the second stream.  The kernels and their
    // order per stream are those of one stream, so the bits are the same.
    if (!h->adj_stream) {
        HIPCHK(h, hipStreamCreateWithFlags(&h->adj_stream, hipStreamNonBlocking));
        for (hipEvent_t& e : h->adj_ev) HIPCHK(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    hipStream_t s1 = h->stream, s2 = h->adj_stream;
    hipEvent_t* ev = h->adj_ev;
    // The recompute shares the GPU with the reverse sweep, so it takes z
    // chunks twice as long as the forward run's (half the workgroups, fewer
    // re-read chunk starts; 128x128x256 FP32: 8 -> 16 planes, adjoint 232
    // -> 220 ms over 4000 steps).
    const int rzc = (int)std::min<int64_t>(std::min(2 * h->fzc, 64), d.nz);
    auto recompute = [&](int64_t c) -> tdse_status {
        const int b = (int)(c & 1);
        const int64_t s0 = c * K;
        const int64_t s1_ = std::min<int64_t>(s0 + K, N);
        HIPCHK(h, hipMemcpyAsync(sgb(b, 0, 0), ck(c, 0), bytes, hipMemcpyDeviceToDevice, s2));
        HIPCHK(h, hipMemcpyAsync(sgb(b, 0, 1), ck(c, 1), bytes, hipMemcpyDeviceToDevice, s2));
        h->stream = s2;
        tdse_status st = TDSE_OK;
        for (int64_t m = s0; m < s1_ && st == TDSE_OK; ++m)
            st = forward_step_explicit(h, sgb(b, m - s0, 0), sgb(b, m - s0, 1), sgb(b, m - s0 + 1, 0),
                                       sgb(b, m - s0 + 1, 1), rzc);
        h->stream = s1;
        if (st != TDSE_OK) return st;
        HIPCHK(h, hipEventRecord(ev[b], s2));
        return TDSE_OK;
    };
    HIPCHK(h, hipEventRecord(ev[4], s1));
    HIPCHK(h, hipStreamWaitEvent(s2, ev[4], 0));
    {
        const tdse_status st = recompute((int64_t)L.nck - 1);
        if (st != TDSE_OK) return st;
    }
    bool first = true;
    for (int64_t c = (int64_t)L.nck - 1; c >= 0; --c) {
        const int b = (int)(c & 1);
        const int64_t s0 = c * K;
        const int64_t s1_ = std::min<int64_t>(s0 + K, N);
        if (c >= 1) {
            // the previous segment into the other bank, once its last sweep is done
            if (c + 1 < (int64_t)L.nck) HIPCHK(h, hipStreamWaitEvent(s2, ev[2 + (b ^ 1)], 0));
            const tdse_status st = recompute(c - 1);
            if (st != TDSE_OK) return st;
        }
        HIPCHK(h, hipStreamWaitEvent(s1, ev[b], 0));
        if (first) {
            tdse_status st = inject(N, sgb(b, s1_ - s0, 0), sgb(b, s1_ - s0, 1));
            if (st != TDSE_OK) return st;
            first = false;
        }
        for (int64_t m = s1_ - 1; m >= s0; --m) {
            const T* Rn = sgb(b, m - s0, 0);
            const T* Ih = sgb(b, m - s0 + 1, 1);
            tdse_status st;
            if (af.ok) {
                st = launch_adj_fused<T>(h, af, rb, ia, rc, ib, Rn, Ih, gv);
                if (st != TDSE_OK) return st;
                std::swap(rb, rc);
            } else {
                st = launch_adj<T>(h, 0, make_adj_args<T>(h, rb, ia, nullptr, nullptr, nullptr, nullptr));
                if (st != TDSE_OK) return st;
                st = launch_adj<T>(h, 1, make_adj_args<T>(h, ia, rb, ib, Rn, Ih, gv));
                if (st != TDSE_OK) return st;
            }
            std::swap(ia, ib);
            st = inject(m, sgb(b, m - s0, 0), sgb(b, m - s0, 1));
            if (st != TDSE_OK) return st;
        }
        HIPCHK(h, hipEventRecord(ev[2 + b], s1));
        if (sizeof(T) != 8) {
            hipLaunchKernelGGL(adjoint_fold_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                               h->stream, gV64, gv, n);
            HIPCHK(h, hipGetLastError());
        }
    }
    if (gR0) HIPCHK(h, hipMemcpyAsync(gR0, rb, bytes, hipMemcpyDeviceToDevice, h->stream));
    if (gI0) HIPCHK(h, hipMemcpyAsync(gI0, ia, bytes, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return TDSE_OK;
}


// Below 2^24 cells: the widest band that fits (256 threads first), two
// rows per thread (the lowest of 2, 3, 4 whose band is at least 4 rows
// tall; none: the occupancy rule below), and the longest z
// chunk of 64 planes down to 1 that gives two workgroups per CU, else
// 1-plane chunks.  Measured against the occupancy rule below it: 160^3
// FP32 91 -> 189, 192^3 FP32 151 -> 222, 200^3 FP32 149 -> 229, 128^3 FP64
// 84 -> 95 Gcell-steps/s; 3 rows per thread at the same chunk was slower
// on all of these but 160^3 FP64 (6% faster there).
bool model_fused_tile(tdse_ctx* h) {
    const tdse_desc& d = h->d;
    const long want = 2L * h->cus;
    for (int ft : {256, 128, 64}) {
        for (int m : {2, 3, 4}) {
            const FusedDims f1 = fused_dims(h, m, 1, ft);
            if (!f1.ok || f1.ty < 4) continue;
            h->ft = ft;
            h->fm = m;
            h->fzc = 1;
            for (int zc0 : {64, 32, 16, 8, 4, 2}) {
                const int zc = (int)std::min<int64_t>(zc0, d.nz);
                if ((long)fused_dims(h, m, zc, ft).nwg >= want) {
                    h->fzc = zc;
                    break;
                }
            }
            return true;
        }
    }
    return false;
}

void default_fused_tile(tdse_ctx* h) {
    // first (threads per workgroup, rows per thread, z chunk) in order of
    // preference that keeps at least ~8 waves per CU busy, z chunks of 8
    // only if nothing longer does
    const tdse_desc& d = h->d;
    if (d.nx * d.ny * d.nz < (int64_t(1) << 24) && model_fused_tile(h)) return;
    const long target = 256L * 512;
    for (int pass = 0; pass < 2; ++pass) {
        for (int ft : {256, 128, 64}) {
            for (int m : {3, 4, 2}) {
                for (int zc0 : {64, 32, 16, 8}) {
                    if ((pass == 0) != (zc0 >= 16)) continue;
                    const int zc = (int)std::min<int64_t>(zc0, d.nz);
                    const FusedDims f = fused_dims(h, m, zc, ft);
                    if (f.ok && (long)f.nwg * ft >= target) {
                        h->ft = ft;
                        h->fm = m;
                        h->fzc = zc;
                        return;
                    }
                }
            }
        }
    }
    // small grids: the z march of each workgroup, not HBM, sets the time,
    // so the chunks go to 2 planes, or 1 below two workgroups per CU; the
    // widest band that fits (narrow bands reload most of their rows as
    // halo), with the most workgroups when none reaches two per CU
    h->ft = 256;
    h->fm = 3;
    h->fzc = (int)std::min<int64_t>(64, d.nz);
    for (int ft : {256, 128, 64}) {
        long most = -1;
        for (int zc0 : {2, 1}) {
            for (int m : {3, 4, 2}) {
                const int zc = (int)std::min<int64_t>(zc0, d.nz);
                const FusedDims f = fused_dims(h, m, zc, ft);
                if (!f.ok) continue;
                if ((long)f.nwg >= 2L * h->cus) {
                    h->ft = ft;
                    h->fm = m;
                    h->fzc = zc;
                    return;
                }
                if (f.nwg > most) {
                    most = f.nwg;
                    h->ft = ft;
                    h->fm = m;
                    h->fzc = zc;
                }
            }
        }
        if (most >= 0) return;
    }
}

// Workgroups of a two-step tile one CU holds at once: LDS, and the
// wavefronts per SIMD the kernel's registers allow (one row per thread:
// <= 128 VGPRs, 4 per SIMD; two rows: 2 per SIMD; three rows: 1).
int fused2_wg_per_cu(const tdse_ctx* h, const Fused2Dims& f, int m) {
    const int waves = f.nt / 64;
    const int per_simd = m == 1 ? 4 : (m == 2 ? 2 : 1);
    const int by_regs = std::max(1, 4 * per_simd / waves);
    const size_t lds = f.lds + 8 * (size_t)(f.nt / 64);
    const int by_lds = std::max(1, (int)((size_t)h->lds_max / lds));
    return std::min(by_regs, by_lds);
}

// Modelled time of a two-step tile: the workgroups run in ceil(nwg / slots)
// waves, slots = CUs x workgroups per CU; each takes (zc + 6) planes of its
// extended tile, at a rate shared by the workgroups of a CU.  On the grids
// measured this ranks the tiles and chunks as the timings do (the chunk
// that makes the last wave full matters most on mid-size grids).
double fused2_cost(const tdse_ctx* h, const Fused2Dims& f, int m, int zc) {
    const int k = fused2_wg_per_cu(h, f, m);
    const long slots = (long)k * h->cus;
    const long waves = (f.nwg + slots - 1) / slots;
    return (double)waves * k * (zc + 6) * (double)f.ex * f.ey;
}

// The one-round two-step tile of interior width tx: 1024 threads, one row
// each, a height of at least 16 rows and z chunks of at least 32 planes (up
// to 16 of them) whose workgroups fill 90-100% of one round of the CUs.
// In one round the time is that of one workgroup, so the tile taken is the
// one whose workgroup sweeps the fewest cells, (zc + 6) planes of its
// extended tile (ex x ey), then the one with more workgroups.  All
// workgroups then march the same planes at about the same time and the L2
// serves the rims that neighbouring tiles re-read; wide tiles read long
// contiguous rows.  False if no such tile exists.
bool one_round_tile(tdse_ctx* h, int tx, int* ty_out, int* zc_out) {
    const tdse_desc& d = h->d;
    const Fused2Dims tall = fused2_dims(h, tx, 1, (int)std::min<int64_t>(d.nz, 32), 1024, 0);
    if (!tall.ok) return false;
    long bwg = 0;
    double bper = 0.0;
    for (int ty = tall.ty; ty >= 16; --ty) {
        for (int nzc = 1; nzc <= 16; ++nzc) {
            const int zc = (int)((d.nz + nzc - 1) / nzc);
            if (zc < 32 && nzc > 1) break;
            const Fused2Dims f = fused2_dims(h, tx, 1, zc, 1024, ty);
            if (!f.ok || f.ty != ty || f.nwg > h->cus || 10L * f.nwg < 9L * h->cus) continue;
            const double per = (double)(zc + 6) * f.ex * f.ey;
            if (bwg == 0 || per < bper || (per == bper && f.nwg > bwg)) {
                bwg = f.nwg;
                bper = per;
                *ty_out = ty;
                *zc_out = zc;
            }
        }
    }
    return bwg > 0;
}

// The default on grids of 2^24 cells or more: the one-round tile of the
// first width of the list that divides nx and has one (128, 80, 64, the
// widths measured best, then the other multiples of 8 from 120 down to 72;
// FP64: 64, 32, then 56, 48, 40).  On the grids measured (512x512x1024 FP32
// and FP64, 256x256x512, the 512x512x128 z-slab, the 240x240x520 grid) it
// is the fastest tile or within 1-2% of it, and on 208x208x416,
// 224x224x448, 320x320x640 and 384x384x768 4-30% faster than the cost
// model's tiles; below 2^24 cells (128x128x256: no faster than the
// one-pass step) it is not used.  False where no such tile exists (e.g.
// 1024x1024x256, whose planes need more than one round of tiles).
bool one_round_two_step(tdse_ctx* h) {
    const tdse_desc& d = h->d;
    if (d.nx * d.ny * d.nz < (int64_t)1 << 24) return false;
    const bool f64 = d.precision == TDSE_F64;
    const int w32[9] = {128, 80, 64, 120, 112, 104, 96, 88, 72}, w64[5] = {64, 32, 56, 48, 40};
    for (int iw = 0; iw < (f64 ? 5 : 9); ++iw) {
        const int tx = f64 ? w64[iw] : w32[iw];
        int ty = 0, zc = 0;
        if (d.nx % tx != 0 || !one_round_tile(h, tx, &ty, &zc)) continue;
        h->two = true;
        h->t2x = tx;
        h->t2m = 1;
        h->t2t = 1024;
        h->t2pf = true;
        h->t2zc = zc;
        h->t2ty = ty;
        return true;
    }
    return false;
}

// The default two-step tile: a one-round tile where the grid has one, else
// the lowest modelled time over the built (rows, threads) pairs, a few tile
// widths and z chunks of 32 .. 256 planes (shorter chunks spend too much on
// the six-plane start), where the tile fits and its workgroups fill at
// least three quarters of the CUs' slots.
void default_two_step(tdse_ctx* h) {
    const tdse_desc& d = h->d;
    if (one_round_two_step(h)) return;
    const bool f64 = d.precision == TDSE_F64;
    struct Cand {
        int tx, m, nt;
    };
    // on a tie of the model the earlier candidate stays (512 threads first:
    // two workgroups per CU hide more latency than one)
    const Cand c32[10] = {{64, 1, 512}, {56, 1, 512}, {48, 1, 512}, {32, 1, 512}, {64, 1, 1024},
                          {120, 1, 1024}, {32, 1, 1024}, {64, 2, 256}, {56, 2, 256}, {24, 2, 256}};
    const Cand c64[8] = {{32, 1, 512}, {64, 1, 512}, {32, 1, 1024}, {64, 1, 1024}, {16, 1, 1024},
                         {56, 2, 512}, {32, 2, 256}, {16, 2, 256}};
    const Cand* cl = f64 ? c64 : c32;
    const int nc = f64 ? 8 : 10;
    h->two = false;
    h->t2x = cl[0].tx;
    h->t2m = cl[0].m;
    h->t2t = cl[0].nt;
    h->t2pf = true;
    h->t2zc = (int)std::min<int64_t>(64, d.nz);
    h->t2ty = 0;
    // below about 5 M cells the one-pass default is faster (128x128x256
    // FP64: 120.6 against 98.5 Gcell-steps/s, 160^3 FP64: 105.9 against
    // 97.2); from 192^3 up the sweep wins (192^3 FP64: 145.9 against 94.4)
    if (d.nx * d.ny * d.nz < (int64_t(5) << 20)) return;
    double best = 0.0;
    for (int i = 0; i < nc; ++i) {
        const Fused2Dims tall = fused2_dims(h, cl[i].tx, cl[i].m, 64, cl[i].nt, 0);
        if (tall.ty < 1) continue;
        // the tallest tile the threads cover and up to a sixth shorter (a
        // tile count that fills the last round of workgroups)
        const int rmax = tall.rpp, rmin = std::max(1, rmax - rmax / 6);
        for (int r = rmax; r >= rmin; --r) {
            const int ty_req = r == rmax ? 0 : r * cl[i].m - 8;
            if (r != rmax && ty_req < 1) break;
            for (int zc0 = 32; zc0 <= 256; zc0 += 4) {
                if (zc0 > d.nz) break;
                const Fused2Dims f = fused2_dims(h, cl[i].tx, cl[i].m, zc0, cl[i].nt, ty_req);
                // at least three quarters of one wave of workgroups, else the
                // one-pass step (more, smaller workgroups) keeps the CUs busier
                if (!f.ok || 4L * f.nwg < 3L * fused2_wg_per_cu(h, f, cl[i].m) * h->cus) continue;
                const double c = fused2_cost(h, f, cl[i].m, zc0);
                if (!h->two || c < best) {
                    best = c;
                    h->two = true;
                    h->t2x = cl[i].tx;
                    h->t2m = cl[i].m;
                    h->t2t = cl[i].nt;
                    h->t2zc = zc0;
                    h->t2ty = ty_req;
                }
            }
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------

static tdse_status bfail(tdse_batch_ctx* b, tdse_status s, const std::string& m) {
    b->err = m;
    return s;
}

static void batch_free_device(tdse_batch_ctx* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->exec1) (void)hipGraphExecDestroy(b->exec1);
    if (b->graph1) (void)hipGraphDestroy(b->graph1);
    b->exec1 = nullptr;
    b->graph1 = nullptr;
    // the tables live in borrowed memory: nothing to free
    b->exec = nullptr;
    b->graph = nullptr;
    b->d_cfg = b->d_fin = nullptr;
    b->d_wg = nullptr;
    b->d_rec = nullptr;
    b->prepared = false;
}

// Point the tables into the batch's workspace; false if none is bound or it
// is short.
static bool batch_carve_tables(tdse_batch_ctx* b) {
    const size_t n = b->members.size();
    if (!b->ws || b->ws_bytes < batch_tables_bytes(n)) return false;
    char* w = static_cast<char*>(b->ws);
    const size_t cfg = std::max({sizeof(FusedArgs<float>), sizeof(FusedArgs<double>),
                                 sizeof(Fused2Args<float>), sizeof(Fused2Args<double>)});
    b->d_cfg = w;
    w += align_up(n * cfg);
    b->d_fin = w;
    w += align_up(n * sizeof(FinArgs));
    b->d_wg = reinterpret_cast<int*>(w);
    w += align_up((n + 1) * sizeof(int));
    b->d_rec = reinterpret_cast<long*>(w);
    return true;
}

// the members run together, so their summed footprint decides the hint
static int batch_streams(const tdse_batch_ctx* b) {
    size_t tot = 0;
    for (const tdse_ctx* m : b->members) tot += state_bytes(m->d);
    return stream_outputs(tot) ? 1 : 0;
}

template <typename T>
static hipError_t batch_enqueue_interval(tdse_batch_ctx* b) {
    const size_t n = b->members.size();
    for (int j = 0; j < b->S; ++j) {
        BatchStep<T> st;
        st.cfg = static_cast<const FusedArgs<T>*>(b->d_cfg);
        st.wg_start = b->d_wg;
        st.rec_idx = b->d_rec;
        st.n = (int)n;
        st.total_wg = b->total_wg;
        st.parity = j & 1;
        st.flux_slot = j;
        const bool rec = b->h > 0 && j == b->S - 1;
        hipError_t e;
        if constexpr (sizeof(T) == 8)
            e = launch_fused_batch_f64(b->W, b->M, rec, b->pf, dim3(b->total_wg), b->nt, b->lds, b->stream, st);
        else
            e = launch_fused_batch_f32(b->W, b->M, rec, b->pf, dim3(b->total_wg), b->nt, b->lds, b->stream, st);
        if (e != hipSuccess) return e;
    }
    BatchFin f;
    f.cfg = static_cast<const FinArgs*>(b->d_fin);
    f.rec_idx = b->d_rec;
    f.n_pending = b->S;
    f.record = b->h > 0 ? 1 : 0;
    hipLaunchKernelGGL(finalize_batch_kernel, dim3((unsigned)n), dim3(256), 0, b->stream, f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (b->h > 0) {
        hipLaunchKernelGGL(bump_counter_kernel, dim3(1), dim3(64), 0, b->stream, b->d_rec);
        e = hipGetLastError();
    }
    return e;
}

// One record interval of two-step sweeps: S / 2 launches (the last one
// writes the record), the per-member finalisation and the counter bump.
// par0 = the state pair the interval starts from.
template <typename T>
static hipError_t batch_enqueue_interval2(tdse_batch_ctx* b, int par0) {
    const size_t n = b->members.size();
    const int launches = b->S / 2;
    for (int j = 0; j < launches; ++j) {
        Batch2Step<T> st;
        st.cfg = static_cast<const Fused2Args<T>*>(b->d_cfg);
        st.wg_start = b->d_wg;
        st.rec_idx = b->d_rec;
        st.n = (int)n;
        st.total_wg = b->total_wg;
        st.parity = (par0 + j) & 1;
        st.flux_slot = 2 * j;
        const bool rec = b->h > 0 && j == launches - 1;
        hipError_t e;
        if constexpr (sizeof(T) == 8)
            e = launch_fused2_batch_f64(b->W, b->t2m, b->t2t, rec, b->t2pf, dim3(b->total_wg), b->lds,
                                        b->stream, st);
        else
            e = launch_fused2_batch_f32(b->W, b->t2m, b->t2t, rec, b->t2pf, dim3(b->total_wg), b->lds,
                                        b->stream, st);
        if (e != hipSuccess) return e;
    }
    BatchFin f;
    f.cfg = static_cast<const FinArgs*>(b->d_fin);
    f.rec_idx = b->d_rec;
    f.n_pending = b->S;
    f.record = b->h > 0 ? 1 : 0;
    hipLaunchKernelGGL(finalize_batch_kernel, dim3((unsigned)n), dim3(256), 0, b->stream, f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (b->h > 0) {
        hipLaunchKernelGGL(bump_counter_kernel, dim3(1), dim3(64), 0, b->stream, b->d_rec);
        e = hipGetLastError();
    }
    return e;
}

// Tables and graphs of the two-step form; false (nothing allocated) if a
// member does not fit the sweep's tile.
// A member's tile in the batch sweep: the batch's rows per thread, threads
// per workgroup and z chunk, vector width W, and an interior width of at
// most txmax (txmax, then multiples of 8 below it) with the height that
// covers the plane with the fewest rows of tiles; the tile with the fewest
// tiles per plane wins (a workgroup takes about the same time whatever its
// tile), then the one that sweeps the fewest cells (rim included), then the
// wider.  Grids of uneven sizes then each get a tiling without a mostly
// empty last row or column of tiles.
Fused2Dims batch_member_tile(const tdse_ctx* h, int txmax, int m, int zc, int nt, int W) {
    Fused2Dims best{};
    best.ok = false;
    long bt = 0, bc = 0;
    for (int tx = txmax; tx >= 8; tx = (tx == txmax ? txmax - 1 : tx - 1) / 8 * 8) {
        const Fused2Dims tall = fused2_dims(h, tx, m, zc, nt, 0);
        if (!tall.ok || tall.W != W) continue;
        const long nty = (h->d.ny + tall.ty - 1) / tall.ty;
        const Fused2Dims f = fused2_dims(h, tx, m, zc, nt, (int)((h->d.ny + nty - 1) / nty));
        if (!f.ok || f.W != W) continue;
        const long cells = (long)f.ntx * f.ex * f.nty * f.ey;
        if (!best.ok || f.ntiles < bt || (f.ntiles == bt && cells < bc)) {
            best = f;
            bt = f.ntiles;
            bc = cells;
        }
    }
    return best;
}

template <typename T>
static tdse_status batch_prepare2_t(tdse_batch_ctx* b, bool* used) {
    *used = false;
    const size_t n = b->members.size();
    std::vector<Fused2Args<T>> cfg(n);
    std::vector<FinArgs> fin(n);
    std::vector<int> wg(n + 1, 0);
    size_t lds = 0;
    int W = 0;
    for (size_t i = 0; i < n; ++i) {
        tdse_ctx* h = b->members[i];
        const int zc = (int)std::min<int64_t>(b->t2zc, h->d.nz);
        // the vector width of the batch's nominal tile on its first member
        if (W == 0) W = fused2_dims(h, b->t2x, b->t2m, zc, b->t2t, 0).W;
        const Fused2Dims f = batch_member_tile(h, b->t2x, b->t2m, zc, b->t2t, W);
        if (!f.ok) return TDSE_OK;
        // the member's own tile is kept for its single-grid steps
        const int sx = h->t2x, sm = h->t2m, sz = h->t2zc, st = h->t2t;
        const bool spf = h->t2pf;
        h->t2x = b->t2x;
        h->t2m = b->t2m;
        h->t2zc = zc;
        h->t2pf = b->t2pf;
        h->t2t = b->t2t;
        cfg[i] = make_fused2_args<T>(h, f, b->h > 0, 0, 0);
        h->t2x = sx;
        h->t2m = sm;
        h->t2zc = sz;
        h->t2pf = spf;
        h->t2t = st;
        cfg[i].nt_out = batch_streams(b);
        cfg[i].rec_plane = static_cast<T*>(h->rec);  // record 0; the kernel adds the counter
        lds = std::max(lds, f.lds);
        wg[i + 1] = wg[i] + f.nwg;
        const tdse_desc& d = h->d;
        FinArgs& a = fin[i];
        a.flux_ring = h->flux_ring;
        a.n_pending = 0;
        a.ytiles = f.ntiles;
        a.has_up = !(d.bc[2] == TDSE_BC_ZERO && d.k_det + 1 >= d.nz);
        a.record = 0;
        a.rec_idx = 0;
        a.dV = d.dx * d.dy * d.dz;
        a.dv_cz = a.dV * h->c[2];
        a.acc = h->acc;
        a.part_q = h->part_q;
        a.part_naive = h->part_naive;
        a.n_part = (long)f.nzc * f.ntiles;
        a.part_plane = h->part_plane;
        a.scalars = h->scal;
    }
    if ((long)wg[n] >= (1L << 31)) return TDSE_OK;
    b->W = W;
    b->lds = lds;
    b->total_wg = wg[n];
    hipError_t e = sizeof(T) == 8 ? fused2_batch_allow_lds_f64(W, b->t2m, b->t2t, lds)
                                  : fused2_batch_allow_lds_f32(W, b->t2m, b->t2t, lds);
    if (e != hipSuccess) return bfail(b, TDSE_ERR_DEVICE, std::string("batch LDS: ") + hipGetErrorString(e));
    if (!batch_carve_tables(b))
        return bfail(b, TDSE_ERR_STATE, "bind a batch workspace of tdse_batch_workspace_size bytes first");
    e = hipMemcpyAsync(b->d_cfg, cfg.data(), n * sizeof(Fused2Args<T>), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_fin, fin.data(), n * sizeof(FinArgs), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_wg, wg.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        batch_free_device(b);
        return bfail(b, TDSE_ERR_DEVICE, std::string("batch tables: ") + hipGetErrorString(e));
    }
    // one interval from pair 0 and, when an interval swaps the pairs an odd
    // number of times, one from pair 1
    const int ngraphs = ((b->S / 2) % 2) ? 2 : 1;
    for (int g = 0; g < ngraphs && e == hipSuccess; ++g) {
        hipGraph_t* gr = g ? &b->graph1 : &b->graph;
        hipGraphExec_t* ex = g ? &b->exec1 : &b->exec;
        e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e2 = batch_enqueue_interval2<T>(b, g);
            e = hipStreamEndCapture(b->stream, gr);
            if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(ex, *gr, nullptr, nullptr, 0);
    }
    if (e != hipSuccess) {
        batch_free_device(b);
        return bfail(b, TDSE_ERR_DEVICE, std::string("batch graph: ") + hipGetErrorString(e));
    }
    b->prepared = true;
    *used = true;
    return TDSE_OK;
}

template <typename T>
static tdse_status batch_prepare_t(tdse_batch_ctx* b) {
    const size_t n = b->members.size();
    std::vector<FusedArgs<T>> cfg(n);
    std::vector<FinArgs> fin(n);
    std::vector<int> wg(n + 1, 0);
    size_t lds = 0;
    int W = 0;
    for (size_t i = 0; i < n; ++i) {
        tdse_ctx* h = b->members[i];
        // the member's own tile is kept for its single-grid steps
        const int sm = h->fm, sz = h->fzc, st = h->ft;
        h->fm = b->M;
        h->fzc = (int)std::min<int64_t>(b->zc, h->d.nz);
        h->ft = b->nt;
        const FusedDims fd = fused_dims(h, b->M, h->fzc, b->nt);
        struct Restore {
            tdse_ctx* h;
            int m, z, t;
            ~Restore() {
                h->fm = m;
                h->fzc = z;
                h->ft = t;
            }
        } restore{h, sm, sz, st};
        if (!fd.ok) return bfail(b, TDSE_ERR_UNSUPPORTED, "member grid does not fit the one-pass tile");
        if (W == 0) W = fd.W;
        if (fd.W != W) return bfail(b, TDSE_ERR_UNSUPPORTED, "members need the same vector width");
        cfg[i] = make_fused_args<T>(h, fd, b->h > 0, 0, 0);
        cfg[i].nt_out = batch_streams(b);
        cfg[i].rec_plane = static_cast<T*>(h->rec);  // record 0; the kernel adds the counter
        lds = std::max(lds, fd.lds);
        wg[i + 1] = wg[i] + fd.nwg;
        const tdse_desc& d = h->d;
        FinArgs& a = fin[i];
        a.flux_ring = h->flux_ring;
        a.n_pending = 0;
        a.ytiles = fd.nbands;
        a.has_up = !(d.bc[2] == TDSE_BC_ZERO && d.k_det + 1 >= d.nz);
        a.record = 0;
        a.rec_idx = 0;
        a.dV = d.dx * d.dy * d.dz;
        a.dv_cz = a.dV * h->c[2];
        a.acc = h->acc;
        a.part_q = h->part_q;
        a.part_naive = h->part_naive;
        a.n_part = (long)fd.nzc * fd.nbands;
        a.part_plane = h->part_plane;
        a.scalars = h->scal;
    }
    b->W = W;
    b->lds = lds;
    b->total_wg = wg[n];
    if (!batch_carve_tables(b))
        return bfail(b, TDSE_ERR_STATE, "bind a batch workspace of tdse_batch_workspace_size bytes first");
    hipError_t e = hipMemcpyAsync(b->d_cfg, cfg.data(), n * sizeof(FusedArgs<T>), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_fin, fin.data(), n * sizeof(FinArgs), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_wg, wg.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        batch_free_device(b);
        return bfail(b, TDSE_ERR_DEVICE, std::string("batch tables: ") + hipGetErrorString(e));
    }
    // capture one interval of S steps + finalisation + counter bump
    e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e2 = batch_enqueue_interval<T>(b);
        e = hipStreamEndCapture(b->stream, &b->graph);
        if (e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        batch_free_device(b);
        return bfail(b, TDSE_ERR_DEVICE, std::string("batch graph: ") + hipGetErrorString(e));
    }
    b->prepared = true;
    return TDSE_OK;
}

// Drop the captured single-grid graph (tables and graph of the internal
// one-member batch) after anything it baked in changes.
static void graph_invalidate(tdse_ctx* h) {
    if (!h->gb) return;
    batch_free_device(h->gb);
    delete h->gb;
    h->gb = nullptr;
}

namespace {

// The tile cache of tdse_autotune: a text file, one line per tuned case,
//   tdse-tune-v1 <nx ny nz precision bcx bcy bcz families pingpong CUs arch> : <15 tile fields>
// read and rewritten whole (through a temporary file renamed over it).
constexpr const char* TUNE_TAG = "tdse-tune-v1";

std::string tune_key(const tdse_ctx* h, int families) {
    const tdse_desc& d = h->d;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) arch = prop.gcnArchName;
    for (char& c : arch)
        if (c == ' ' || c == ':') c = '_';
    char buf[256];
    std::snprintf(buf, sizeof buf, "%lld %lld %lld %d %d %d %d %d %d %d %s", (long long)d.nx,
                  (long long)d.ny, (long long)d.nz, d.precision, d.bc[0], d.bc[1], d.bc[2], families,
                  h->R2 ? 1 : 0, h->cus, arch.c_str());
    return buf;
}

void tile_fields(const tdse_tile& t, int v[15]) {
    const int f[15] = {t.rows, t.waves, t.zc, t.fused, t.fused_rows, t.fused_zc, t.fused_prefetch,
                       t.graph, t.fused_threads, t.two_step, t.two_step_tx, t.two_step_rows,
                       t.two_step_zc, t.two_step_prefetch, t.two_step_threads};
    for (int i = 0; i < 15; ++i) v[i] = f[i];
}

void tile_from_fields(tdse_tile* t, const int v[15]) {
    t->rows = v[0];
    t->waves = v[1];
    t->zc = v[2];
    t->fused = v[3];
    t->fused_rows = v[4];
    t->fused_zc = v[5];
    t->fused_prefetch = v[6];
    t->graph = v[7];
    t->fused_threads = v[8];
    t->two_step = v[9];
    t->two_step_tx = v[10];
    t->two_step_rows = v[11];
    t->two_step_zc = v[12];
    t->two_step_prefetch = v[13];
    t->two_step_threads = v[14];
}

std::vector<std::string> read_lines(const char* path) {
    std::vector<std::string> lines;
    FILE* f = std::fopen(path, "r");
    if (!f) return lines;
    char buf[1024];
    while (std::fgets(buf, sizeof buf, f)) {
        std::string l(buf);
        while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
        if (!l.empty()) lines.push_back(l);
    }
    std::fclose(f);
    return lines;
}

// The cached tile of key, if the file has a well-formed line for it.
bool tune_cache_lookup(const char* path, const std::string& key, tdse_tile* t) {
    const std::string head = std::string(TUNE_TAG) + " " + key + " :";
    for (const std::string& l : read_lines(path)) {
        if (l.compare(0, head.size(), head) != 0) continue;
        int v[15];
        int used = 0;
        const char* p = l.c_str() + head.size();
        int i = 0;
        for (; i < 15; ++i) {
            if (std::sscanf(p, "%d%n", &v[i], &used) != 1) break;
            p += used;
        }
        if (i == 15) {
            tile_from_fields(t, v);
            return true;
        }
    }
    return false;
}

// Replace (or add) the line of key; false if the file cannot be written.
bool tune_cache_store(const char* path, const std::string& key, const tdse_tile& t) {
    const std::string head = std::string(TUNE_TAG) + " " + key + " :";
    std::vector<std::string> lines;
    for (const std::string& l : read_lines(path))
        if (l.compare(0, head.size(), head) != 0) lines.push_back(l);
    int v[15];
    tile_fields(t, v);
    std::string line = head;
    for (int i = 0; i < 15; ++i) line += " " + std::to_string(v[i]);
    lines.push_back(line);
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    bool ok = true;
    for (const std::string& l : lines) ok = ok && std::fprintf(f, "%s\n", l.c_str()) > 0;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

}  // namespace

extern "C" {

int32_t tdse_abi_version(void) { return 1; }

const char* tdse_status_string(tdse_status s) {
    switch (s) {
        case TDSE_OK: return "ok";
        case TDSE_ERR_ARG: return "invalid argument";
        case TDSE_ERR_STATE: return "call out of order";
        case TDSE_ERR_UNSTABLE: return "time step above the stability bound";
        case TDSE_ERR_NONFINITE: return "non-finite value in the FP64 sums";
        case TDSE_ERR_DEVICE: return "HIP device error";
        case TDSE_ERR_OOM: return "device allocation failed";
        case TDSE_ERR_UNSUPPORTED: return "unsupported shape or option";
        case TDSE_ERR_CAPACITY: return "record buffer or fixed scratch too small";
        default: return "unknown status";
    }
}

const char* tdse_last_error(tdse_handle h) { return h ? h->err.c_str() : ""; }

}  // extern "C"

namespace {

tdse_status check_desc(const tdse_desc* d) {
    if (!d) return TDSE_ERR_ARG;
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return TDSE_ERR_ARG;
    if (d->nx > (1 << 20) || d->ny > (1 << 20) || d->nz > (1 << 20)) return TDSE_ERR_ARG;
    if ((double)d->nx * d->ny * d->nz > 9.0e18) return TDSE_ERR_ARG;
    if (!(d->dx > 0) || !(d->dy > 0) || !(d->dz > 0)) return TDSE_ERR_ARG;
    if (!std::isfinite(d->dx) || !std::isfinite(d->dy) || !std::isfinite(d->dz)) return TDSE_ERR_ARG;
    if (!(d->hbar > 0) || !(d->mass > 0) || !std::isfinite(d->hbar) || !std::isfinite(d->mass))
        return TDSE_ERR_ARG;
    for (int a = 0; a < 3; ++a)
        if (d->bc[a] != TDSE_BC_PERIODIC && d->bc[a] != TDSE_BC_ZERO) return TDSE_ERR_ARG;
    if (d->precision != TDSE_F32 && d->precision != TDSE_F64) return TDSE_ERR_ARG;
    if (d->k_det < 0 || d->k_det >= d->nz) return TDSE_ERR_ARG;
    if (d->record_every < 0) return TDSE_ERR_ARG;
    if (d->record_every > 0 && d->max_records < 1) return TDSE_ERR_ARG;
    if (!(d->dt > 0) && !(d->dt_frac > 0)) return TDSE_ERR_ARG;
    if (!std::isfinite(d->dt) || !std::isfinite(d->dt_frac)) return TDSE_ERR_ARG;
    if (d->flags & ~(uint32_t)(TDSE_FLAG_ALLOW_UNSTABLE | TDSE_FLAG_PIXEL_INTEGRAL))
        return TDSE_ERR_ARG;
    return supported_shape(*d);
}

// The kinetic part of the Gershgorin bound: (hbar^2/2m) sum_d 4/d^2 over
// the axes that couple cells (a periodic axis of length 1 adds nothing).
double kinetic_bound(const tdse_desc* d) {
    const int64_t n[3] = {d->nx, d->ny, d->nz};
    const double sp[3] = {d->dx, d->dy, d->dz};
    double kin = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (n[a] == 1 && d->bc[a] == TDSE_BC_PERIODIC) continue;
        kin += 4.0 / (sp[a] * sp[a]);
    }
    return kin * d->hbar * d->hbar / (2.0 * d->mass);
}

}  // namespace

extern "C" {

tdse_status tdse_validate_desc(const tdse_desc* d, double* dt_bound) {
    const tdse_status s = check_desc(d);
    if (s != TDSE_OK) return s;
    if (dt_bound) {
        const double kin = kinetic_bound(d);
        *dt_bound = kin > 0 ? d->hbar / kin : INFINITY;
    }
    return TDSE_OK;
}

tdse_status tdse_time_step_bound(const tdse_desc* d, double vmin, double vmax, double* e_max,
                                 double* dt_bound) {
    tdse_status s = check_desc(d);
    if (s != TDSE_OK) return s;
    if (!std::isfinite(vmin) || !std::isfinite(vmax) || vmin > vmax) return TDSE_ERR_ARG;
    const double kin = kinetic_bound(d);
    const double em = std::max(std::fabs(vmin), std::fabs(vmax + kin));
    if (!(em > 0)) return TDSE_ERR_ARG;
    if (e_max) *e_max = em;
    if (dt_bound) *dt_bound = d->hbar / em;
    return TDSE_OK;
}

tdse_status tdse_workspace_size(const tdse_desc* d, size_t* bytes) {
    tdse_status s = check_desc(d);
    if (s != TDSE_OK) return s;
    if (!bytes) return TDSE_ERR_ARG;
    *bytes = layout_of(*d).total;
    return TDSE_OK;
}

tdse_status tdse_create(const tdse_desc* d, void* stream, tdse_handle* out) {
    if (!out) return TDSE_ERR_ARG;
    *out = nullptr;
    tdse_status s = check_desc(d);
    if (s != TDSE_OK) return s;
    s = supported_shape(*d);
    if (s != TDSE_OK) return s;
    int W = 1, G = 0, NL = 0;
    const bool half_vec = choose_x_layout(*d, &W, &G, &NL);
    if (!half_vec) W = vector_width(*d);
    tdse_ctx* h = new (std::nothrow) tdse_ctx();
    if (!h) return TDSE_ERR_OOM;
    h->d = *d;
    h->stream = static_cast<hipStream_t>(stream);
    h->W = W;
    h->G = G;
    h->NL = NL;
    h->half_vec = half_vec;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return TDSE_ERR_DEVICE;
    }
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) == hipSuccess &&
        lds > 0)
        h->lds_max = lds;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess &&
        cus > 0)
        h->cus = cus;
    default_tile(h);
    default_fused_tile(h);
    default_two_step(h);
    h->wcap.assign((size_t)d->nz, 0.0);
    *out = h;
    return TDSE_OK;
}

tdse_status tdse_destroy(tdse_handle h) {
    if (!h) return TDSE_OK;
    graph_invalidate(h);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->adj_ev)
        if (e) (void)hipEventDestroy(e);
    if (h->adj_stream) (void)hipStreamDestroy(h->adj_stream);
    delete h;
    return TDSE_OK;
}

tdse_status tdse_bind(tdse_handle h, void* psi_r, void* psi_i, void* v, void* workspace,
                      size_t workspace_bytes, void* records, double* scalars, double* pixel) {
    if (!h) return TDSE_ERR_ARG;
    const tdse_desc& d = h->d;
    if (!psi_r || !psi_i || !v || !workspace) return fail(h, TDSE_ERR_ARG, "null pointer");
    if (psi_r == psi_i || psi_r == v || psi_i == v) return fail(h, TDSE_ERR_ARG, "aliased arrays");
    const Layout L = layout_of(d);
    if (workspace_bytes < L.total) return fail(h, TDSE_ERR_ARG, "workspace too small");
    if (d.record_every > 0 && (!records || !scalars))
        return fail(h, TDSE_ERR_ARG, "records and scalars are required when record_every > 0");
    if ((d.flags & TDSE_FLAG_PIXEL_INTEGRAL) && !pixel)
        return fail(h, TDSE_ERR_ARG, "pixel buffer required by TDSE_FLAG_PIXEL_INTEGRAL");
    for (const void* p : {(const void*)psi_r, (const void*)psi_i, (const void*)v, (const void*)workspace})
        if (!aligned(p)) return fail(h, TDSE_ERR_ARG, "pointer not 256-byte aligned");
    if (records && !aligned(records)) return fail(h, TDSE_ERR_ARG, "records not 256-byte aligned");
    if (scalars && !aligned(scalars)) return fail(h, TDSE_ERR_ARG, "scalars not 256-byte aligned");
    if ((d.flags & TDSE_FLAG_PIXEL_INTEGRAL) && !aligned(pixel))
        return fail(h, TDSE_ERR_ARG, "pixel not 256-byte aligned");
    graph_invalidate(h);
    h->R = psi_r;
    h->I = psi_i;
    h->V = v;
    h->R2 = nullptr;
    h->I2 = nullptr;
    h->fused = false;
    h->adj_ws = nullptr;
    h->ws = workspace;
    h->ws_bytes = workspace_bytes;
    h->rec = records;
    h->scal = scalars;
    h->pix = pixel;
    char* w = static_cast<char*>(workspace);
    h->ca = w + L.ca;
    h->cb = w + L.cb;
    h->acc = reinterpret_cast<double*>(w + L.acc);
    h->flux_ring = reinterpret_cast<double*>(w + L.flux);
    h->part_q = reinterpret_cast<double*>(w + L.part_q);
    h->part_naive = reinterpret_cast<double*>(w + L.part_n);
    h->part_plane = reinterpret_cast<double*>(w + L.part_p);
    h->red = reinterpret_cast<double*>(w + L.red);
    h->gfac = reinterpret_cast<double*>(w + L.gfac);
    h->F = L.F;
    h->bound = true;
    h->finalized = false;
    h->ready = false;
    h->step = 0;
    h->pending = 0;
    return TDSE_OK;
}

tdse_status tdse_build_potential(tdse_handle h, const tdse_atom* atoms, int64_t n,
                                 const tdse_pot_params* p) {
    if (!h || !p || n < 0 || (n > 0 && !atoms)) return TDSE_ERR_ARG;
    if (!h->bound) return fail(h, TDSE_ERR_STATE, "bind before building the potential");
    if (!(p->cutoff > 0) || !(p->soft >= 0) || !(p->kappa > 0) || !(p->a0 > 0))
        return fail(h, TDSE_ERR_ARG, "bad potential parameters");
    if (n > (int64_t)1 << 26) return fail(h, TDSE_ERR_ARG, "too many atoms");
    const tdse_desc& d = h->d;
    for (int64_t a = 0; a < n; ++a) {
        const tdse_atom& t = atoms[a];
        if (!std::isfinite(t.x) || !std::isfinite(t.y) || !std::isfinite(t.z) || !(t.Z > 0) ||
            !std::isfinite(t.amp))
            return fail(h, TDSE_ERR_ARG, "bad atom");
    }
    // per-plane candidate lists: atoms whose z distance (minimum image on a
    // periodic z axis) is below the cutoff, in ascending atom order
    const double Lz = d.nz * d.dz;
    std::vector<int> ptr((size_t)d.nz + 1, 0);
    std::vector<int> idx;
    for (int64_t k = 0; k < d.nz; ++k) {
        const double z = k * d.dz;
        for (int64_t a = 0; a < n; ++a) {
            double u = z - atoms[a].z;
            if (d.bc[2] == TDSE_BC_PERIODIC) u -= Lz * std::nearbyint(u / Lz);
            if (std::fabs(u) < p->cutoff) idx.push_back((int)a);
        }
        ptr[(size_t)k + 1] = (int)idx.size();
    }
    if (idx.empty()) idx.push_back(0);
    double* d_atoms = nullptr;
    int* d_ptr = nullptr;
    int* d_idx = nullptr;
    auto cleanup = [&]() {
        if (d_atoms) (void)hipFree(d_atoms);
        if (d_ptr) (void)hipFree(d_ptr);
        if (d_idx) (void)hipFree(d_idx);
    };
    const size_t na = std::max<int64_t>(n, 1);
    if (hipMalloc(&d_atoms, na * 5 * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_ptr, ptr.size() * sizeof(int)) != hipSuccess ||
        hipMalloc(&d_idx, idx.size() * sizeof(int)) != hipSuccess) {
        cleanup();
        return fail(h, TDSE_ERR_OOM, "potential temporaries");
    }
    std::vector<double> flat(na * 5, 0.0);
    for (int64_t a = 0; a < n; ++a) {
        flat[5 * a + 0] = atoms[a].x;
        flat[5 * a + 1] = atoms[a].y;
        flat[5 * a + 2] = atoms[a].z;
        flat[5 * a + 3] = atoms[a].Z;
        flat[5 * a + 4] = atoms[a].amp;
    }
    hipError_t e = hipMemcpyAsync(d_atoms, flat.data(), flat.size() * sizeof(double),
                                  hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_ptr, ptr.data(), ptr.size() * sizeof(int), hipMemcpyHostToDevice,
                           h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_idx, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice,
                           h->stream);
    PotArgs a;
    a.nx = (int)d.nx;
    a.ny = (int)d.ny;
    a.nz = (int)d.nz;
    a.dx = d.dx;
    a.dy = d.dy;
    a.dz = d.dz;
    a.Lx = d.nx * d.dx;
    a.Ly = d.ny * d.dy;
    a.Lz = Lz;
    a.bcx = d.bc[0] == TDSE_BC_ZERO;
    a.bcy = d.bc[1] == TDSE_BC_ZERO;
    a.bcz = d.bc[2] == TDSE_BC_ZERO;
    a.screened = p->screened;
    a.atoms = d_atoms;
    a.plane_ptr = d_ptr;
    a.plane_idx = d_idx;
    a.soft = p->soft;
    a.cutoff = p->cutoff;
    a.kappa = p->kappa;
    a.a0 = p->a0;
    const long nxy = (long)d.nx * d.ny;
    dim3 grid((unsigned)((nxy + 255) / 256), (unsigned)d.nz);
    if (e == hipSuccess) {
        if (d.precision == TDSE_F64)
            hipLaunchKernelGGL(potential_kernel<double>, grid, dim3(256), 0, h->stream, a,
                               static_cast<double*>(h->V));
        else
            hipLaunchKernelGGL(potential_kernel<float>, grid, dim3(256), 0, h->stream, a,
                               static_cast<float*>(h->V));
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    cleanup();
    h->finalized = false;
    h->ready = false;
    return hip_check(h, e, "build_potential");
}

static tdse_status upload_tables(tdse_ctx* h) {
    const tdse_desc& d = h->d;
    const size_t nz = (size_t)d.nz;
    h->ca_h.assign(nz, 1.0);
    h->cb_h.assign(nz, 1.0);
    for (size_t k = 0; k < nz; ++k) {
        const double gam = h->wcap[k] * h->dt / d.hbar;
        h->ca_h[k] = (1.0 - 0.5 * gam) / (1.0 + 0.5 * gam);
        h->cb_h[k] = 1.0 / (1.0 + 0.5 * gam);
    }
    if (d.precision == TDSE_F64) {
        HIPCHK(h, hipMemcpyAsync(h->ca, h->ca_h.data(), nz * 8, hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(h->cb, h->cb_h.data(), nz * 8, hipMemcpyHostToDevice, h->stream));
    } else {
        h->caf_h.assign(h->ca_h.begin(), h->ca_h.end());
        h->cbf_h.assign(h->cb_h.begin(), h->cb_h.end());
        HIPCHK(h, hipMemcpyAsync(h->ca, h->caf_h.data(), nz * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipMemcpyAsync(h->cb, h->cbf_h.data(), nz * 4, hipMemcpyHostToDevice, h->stream));
    }
    h->unit_lo = h->unit_hi = 0;
    for (size_t k = 0; k < nz;) {
        auto unit = [&](size_t q) {
            return d.precision == TDSE_F64 ? (h->ca_h[q] == 1.0 && h->cb_h[q] == 1.0)
                                           : (h->caf_h[q] == 1.0f && h->cbf_h[q] == 1.0f);
        };
        if (!unit(k)) {
            ++k;
            continue;
        }
        size_t e = k;
        while (e < nz && unit(e)) ++e;
        if (e - k > (size_t)(h->unit_hi - h->unit_lo)) {
            h->unit_lo = (int)k;
            h->unit_hi = (int)e;
        }
        k = e;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return TDSE_OK;
}

tdse_status tdse_interpolate_potential(tdse_handle h, const double* table, int32_t ux, int32_t uy,
                                      int32_t uz, const double* spacing, const double* origin) {
    if (!h || !table || !spacing || !origin || ux < 1 || uy < 1 || uz < 1) return TDSE_ERR_ARG;
    if (!h->bound) return fail(h, TDSE_ERR_STATE, "bind before building the potential");
    for (int c = 0; c < 3; ++c)
        if (!(spacing[c] > 0) || !std::isfinite(spacing[c]) || !std::isfinite(origin[c]))
            return fail(h, TDSE_ERR_ARG, "bad table spacing or origin");
    if ((int64_t)ux * uy * uz > ((int64_t)1 << 31)) return fail(h, TDSE_ERR_ARG, "table too large");
    const tdse_desc& d = h->d;
    InterpArgs a;
    a.table = table;
    a.ux = ux;
    a.uy = uy;
    a.uz = uz;
    a.sx = spacing[0];
    a.sy = spacing[1];
    a.sz = spacing[2];
    a.ox = origin[0];
    a.oy = origin[1];
    a.oz = origin[2];
    a.nx = (int)d.nx;
    a.ny = (int)d.ny;
    a.nz = (int)d.nz;
    a.dx = d.dx;
    a.dy = d.dy;
    a.dz = d.dz;
    // axis weights into the workspace's setup scratch (16 B per mesh index
    // of the three axes; the region holds 32 B per index)
    AxisW* ax = reinterpret_cast<AxisW*>(h->gfac);
    const long nax = (long)d.nx + d.ny + d.nz;
    hipLaunchKernelGGL(interp_axes_kernel, dim3((unsigned)std::min<long>((nax + 255) / 256, 4096)),
                       dim3(256), 0, h->stream, a, ax);
    HIPCHK(h, hipGetLastError());
    // the z-blended table plane of a mesh plane and the y-blended rows of
    // the workgroup in LDS when they fit (48 KB); rows of one plane per
    // workgroup: 64 with the staging (it is paid once per workgroup), 16
    // without, fewer on small grids
    const int nseg = (int)((d.nx + 255) / 256);
    int rows = 64;
    const size_t lds_z = (size_t)uy * (ux + 1) * sizeof(double);
    const bool staged = lds_z + (size_t)rows * (ux + 1) * sizeof(double) <= 48 * 1024;
    if (!staged) rows = 16;
    while (rows > 1 && (long)nseg * ((d.ny + rows - 1) / rows) * d.nz < 4096) rows /= 2;
    // the z-blended plane, then the y-blended rows of the workgroup
    const size_t lds = lds_z + (size_t)rows * (ux + 1) * sizeof(double);
    const long ngx = (long)nseg * ((d.ny + rows - 1) / rows);
    if (ngx >= (1L << 31)) return fail(h, TDSE_ERR_UNSUPPORTED, "grid too large for the interpolation launch");
    const dim3 grid((unsigned)ngx, (unsigned)d.nz);
    if (staged) {
        if (d.precision == TDSE_F64)
            hipLaunchKernelGGL(interp_potential_lds_kernel<double>, grid, dim3(256), lds, h->stream, a, ax,
                               nseg, rows, static_cast<double*>(h->V));
        else
            hipLaunchKernelGGL(interp_potential_lds_kernel<float>, grid, dim3(256), lds, h->stream, a, ax,
                               nseg, rows, static_cast<float*>(h->V));
    } else if (d.precision == TDSE_F64) {
        hipLaunchKernelGGL(interp_potential_kernel<double>, grid, dim3(256), 0, h->stream, a, ax, nseg,
                           rows, static_cast<double*>(h->V));
    } else {
        hipLaunchKernelGGL(interp_potential_kernel<float>, grid, dim3(256), 0, h->stream, a, ax, nseg,
                           rows, static_cast<float*>(h->V));
    }
    return hip_check(h, hipGetLastError(), "interpolation launch");
}

tdse_status tdse_set_cap(tdse_handle h, const double* w, int64_t nz) {
    if (!h) return TDSE_ERR_ARG;
    if (nz != h->d.nz) return fail(h, TDSE_ERR_ARG, "CAP length must equal nz");
    if (w) {
        for (int64_t k = 0; k < nz; ++k)
            if (!(w[k] >= 0) || !std::isfinite(w[k])) return fail(h, TDSE_ERR_ARG, "CAP rates must be finite and >= 0");
        h->wcap.assign(w, w + nz);
    } else {
        h->wcap.assign((size_t)nz, 0.0);
    }
    if (h->finalized) {
        graph_invalidate(h);
        tdse_status s = upload_tables(h);
        if (s != TDSE_OK) return s;
        h->ready = false;
    }
    return TDSE_OK;
}

tdse_status tdse_set_cap_quadratic(tdse_handle h, int64_t n_bottom, int64_t n_top, double w_max) {
    if (!h) return TDSE_ERR_ARG;
    const int64_t nz = h->d.nz;
    if (n_bottom < 0 || n_top < 0 || n_bottom + n_top > nz || !(w_max >= 0) || !std::isfinite(w_max))
        return fail(h, TDSE_ERR_ARG, "bad CAP ramp");
    std::vector<double> w((size_t)nz, 0.0);
    for (int64_t k = 0; k < n_bottom; ++k) {
        const double t = (double)(n_bottom - k) / (double)n_bottom;
        w[(size_t)k] += w_max * t * t;
    }
    for (int64_t k = nz - n_top; k < nz; ++k) {
        const double t = (double)(k - (nz - 1 - n_top)) / (double)n_top;
        w[(size_t)k] += w_max * t * t;
    }
    return tdse_set_cap(h, w.data(), nz);
}

tdse_status tdse_set_cap_paper(tdse_handle h, double alpha, double r_cut) {
    if (!h) return TDSE_ERR_ARG;
    if (!(alpha >= 0) || !std::isfinite(alpha) || !(r_cut >= 0) || !std::isfinite(r_cut))
        return fail(h, TDSE_ERR_ARG, "bad CAP parameters");
    const int64_t nz = h->d.nz;
    const double dz = h->d.dz;
    std::vector<double> w((size_t)nz, 0.0);
    for (int64_t k = 0; k < nz; ++k) {
        const double u = r_cut - (double)k * dz;
        if ((double)k * dz < r_cut) w[(size_t)k] = alpha / dz * u * u;
    }
    return tdse_set_cap(h, w.data(), nz);
}

tdse_status tdse_time_step_paper(const tdse_desc* d, double* dt) {
    tdse_status s = check_desc(d);
    if (s != TDSE_OK) return s;
    if (!dt) return TDSE_ERR_ARG;
    const double dmin = std::min(d->dx, std::min(d->dy, d->dz));
    *dt = d->mass / (5.0 * d->hbar) * dmin * dmin;
    return TDSE_OK;
}

tdse_status tdse_finalize_setup(tdse_handle h, double* dt_out, double* e_max_out) {
    if (!h) return TDSE_ERR_ARG;
    if (!h->bound) return fail(h, TDSE_ERR_STATE, "bind before finalize");
    const tdse_desc& d = h->d;
    const long n = (long)d.nx * d.ny * d.nz;
    const int blocks = (int)std::min<long>(4096, (n + 255) / 256);
    if (d.precision == TDSE_F64)
        hipLaunchKernelGGL(minmax_kernel<double>, dim3(blocks), dim3(256), 0, h->stream,
                           static_cast<const double*>(h->V), n, h->red);
    else
        hipLaunchKernelGGL(minmax_kernel<float>, dim3(blocks), dim3(256), 0, h->stream,
                           static_cast<const float*>(h->V), n, h->red);
    HIPCHK(h, hipGetLastError());
    std::vector<double> part((size_t)3 * blocks);
    HIPCHK(h, hipMemcpyAsync(part.data(), h->red, part.size() * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    double vmin = 1e308, vmax = -1e308, bad = 0.0;
    for (int b = 0; b < blocks; ++b) {
        vmin = std::min(vmin, part[3 * b]);
        vmax = std::max(vmax, part[3 * b + 1]);
        bad += part[3 * b + 2];
    }
    if (bad > 0) return fail(h, TDSE_ERR_NONFINITE, "V holds NaN or Inf");
    double em, bound;
    tdse_status s = tdse_time_step_bound(&d, vmin, vmax, &em, &bound);
    if (s != TDSE_OK) return fail(h, s, "time step bound");
    double dt = d.dt > 0 ? d.dt : d.dt_frac * bound;
    if (dt > bound * (1.0 + 1e-12) && !(d.flags & TDSE_FLAG_ALLOW_UNSTABLE))
        return fail(h, TDSE_ERR_UNSTABLE, "dt exceeds hbar / E_max");
    graph_invalidate(h);
    h->dt = dt;
    h->emax = em;
    h->c[0] = d.hbar * dt / (2.0 * d.mass * d.dx * d.dx);
    h->c[1] = d.hbar * dt / (2.0 * d.mass * d.dy * d.dy);
    h->c[2] = d.hbar * dt / (2.0 * d.mass * d.dz * d.dz);
    h->c[3] = dt / d.hbar;
    s = upload_tables(h);
    if (s != TDSE_OK) return s;
    h->finalized = true;
    h->ready = false;
    if (dt_out) *dt_out = dt;
    if (e_max_out) *e_max_out = em;
    return TDSE_OK;
}

tdse_status tdse_init_gaussian(tdse_handle h, const double r0[3], const double k0[3], double sigma,
                               int32_t mode) {
    if (!h || !r0 || !k0) return TDSE_ERR_ARG;
    if (!h->finalized) return fail(h, TDSE_ERR_STATE, "finalize_setup before init_gaussian");
    if (!(sigma > 0) || !std::isfinite(sigma)) return fail(h, TDSE_ERR_ARG, "sigma must be > 0");
    if (mode != TDSE_INIT_HALFSTEP && mode != TDSE_INIT_NAIVE) return fail(h, TDSE_ERR_ARG, "bad mode");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(r0[a]) || !std::isfinite(k0[a])) return fail(h, TDSE_ERR_ARG, "non-finite packet");
    const tdse_desc& d = h->d;
    GaussAxisArgs ga;
    ga.n[0] = (int)d.nx;
    ga.n[1] = (int)d.ny;
    ga.n[2] = (int)d.nz;
    ga.d[0] = d.dx;
    ga.d[1] = d.dy;
    ga.d[2] = d.dz;
    for (int a = 0; a < 3; ++a) {
        ga.L[a] = ga.n[a] * ga.d[a];
        ga.r0[a] = r0[a];
        ga.k0[a] = k0[a];
        ga.periodic[a] = d.bc[a] == TDSE_BC_PERIODIC;
    }
    ga.sigma = sigma;
    ga.hbar = d.hbar;
    ga.mass = d.mass;
    ga.t0 = 0.0;
    ga.t1 = (mode == TDSE_INIT_HALFSTEP) ? -0.5 * h->dt : 0.0;
    ga.fac = h->gfac;
    const int tot = 2 * (ga.n[0] + ga.n[1] + ga.n[2]);
    hipLaunchKernelGGL(gauss_axis_kernel, dim3((tot + 255) / 256), dim3(256), 0, h->stream, ga);
    HIPCHK(h, hipGetLastError());
    const long nxy = (long)d.nx * d.ny;
    const unsigned gx = (unsigned)((nxy + 255) / 256);
    GaussCellArgs gc;
    gc.nx = (int)d.nx;
    gc.ny = (int)d.ny;
    gc.nz = (int)d.nz;
    gc.fac = h->gfac;
    gc.scale = 1.0;
    // norm partials: one per (block, plane); reuse part_q (>= ny*nz slots)
    gc.partial = h->part_q;
    hipLaunchKernelGGL(gauss_norm_kernel, dim3(gx, (unsigned)d.nz), dim3(256), 0, h->stream, gc);
    HIPCHK(h, hipGetLastError());
    std::vector<double> part((size_t)gx * d.nz);
    HIPCHK(h, hipMemcpyAsync(part.data(), h->part_q, part.size() * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    double tot_norm = 0.0;
    for (double v : part) tot_norm += v;
    const double dV = d.dx * d.dy * d.dz;
    if (!(tot_norm > 0) || !std::isfinite(tot_norm)) return fail(h, TDSE_ERR_NONFINITE, "packet norm");
    gc.scale = 1.0 / std::sqrt(dV * tot_norm);
    if (d.precision == TDSE_F64)
        hipLaunchKernelGGL(gauss_write_kernel<double>, dim3(gx, (unsigned)d.nz), dim3(256), 0,
                           h->stream, gc, static_cast<double*>(h->R), static_cast<double*>(h->I));
    else
        hipLaunchKernelGGL(gauss_write_kernel<float>, dim3(gx, (unsigned)d.nz), dim3(256), 0,
                           h->stream, gc, static_cast<float*>(h->R), static_cast<float*>(h->I));
    HIPCHK(h, hipGetLastError());
    h->step = 0;
    tdse_status s = begin_records(h);
    if (s != TDSE_OK) return s;
    h->ready = true;
    return TDSE_OK;
}

tdse_status tdse_set_state(tdse_handle h, const void* psi_r, const void* psi_i, int64_t step,
                           double flux_acc) {
    if (!h || !psi_r || !psi_i || step < 0 || !std::isfinite(flux_acc)) return TDSE_ERR_ARG;
    if (!h->finalized) return fail(h, TDSE_ERR_STATE, "finalize_setup before set_state");
    const tdse_desc& d = h->d;
    const size_t bytes = (size_t)d.nx * d.ny * d.nz * elem_size(d);
    if (psi_r != h->R)
        HIPCHK(h, hipMemcpyAsync(h->R, psi_r, bytes, hipMemcpyDeviceToDevice, h->stream));
    if (psi_i != h->I)
        HIPCHK(h, hipMemcpyAsync(h->I, psi_i, bytes, hipMemcpyDeviceToDevice, h->stream));
    h->step = step;
    h->pending = 0;
    if (step == 0) {
        tdse_status s = begin_records(h);
        if (s != TDSE_OK) return s;
    } else {
        if (d.record_every > 0 && step / d.record_every + 1 > d.max_records)
            return fail(h, TDSE_ERR_CAPACITY, "records of the resumed run exceed the buffer");
        double acc[8] = {flux_acc, 0, 0, 0, 0, 0, 0, 0};
        HIPCHK(h, hipMemcpyAsync(h->acc, acc, sizeof(acc), hipMemcpyHostToDevice, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    h->ready = true;
    return TDSE_OK;
}

tdse_status tdse_get_state(tdse_handle h, void* psi_r, void* psi_i, int64_t* step,
                           double* flux_acc) {
    if (!h) return TDSE_ERR_ARG;
    if (!h->ready) return fail(h, TDSE_ERR_STATE, "no state");
    const tdse_desc& d = h->d;
    const size_t bytes = (size_t)d.nx * d.ny * d.nz * elem_size(d);
    if (psi_r && psi_r != h->R)
        HIPCHK(h, hipMemcpyAsync(psi_r, h->R, bytes, hipMemcpyDeviceToDevice, h->stream));
    if (psi_i && psi_i != h->I)
        HIPCHK(h, hipMemcpyAsync(psi_i, h->I, bytes, hipMemcpyDeviceToDevice, h->stream));
    double acc = 0.0;
    HIPCHK(h, hipMemcpyAsync(&acc, h->acc, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (step) *step = h->step;
    if (flux_acc) *flux_acc = acc;
    return TDSE_OK;
}

// The step loop.  Each step runs as one of: OP_H, the two in-place
// half-step kernels; OP_F1, the one-pass kernel into the second state pair;
// OP_F2, the two-step sweep into the second pair.  F1 and F2 swap the pairs,
// so the plan keeps their count even and the state ends in the bound
// arrays.  A pair of steps goes to F2 unless the level between them is
// recorded or checkpointed.
enum StepOp : char { OP_H = 0, OP_F1 = 1, OP_F2 = 2 };

static tdse_status step_plain(tdse_ctx* h, int64_t n) {
    const tdse_desc& d = h->d;
    const int64_t hrec = d.record_every;
    const FusedDims fd = fused_dims(h, h->fm, h->fzc);
    const bool use_fused = h->fused && h->R2 && fd.ok;
    const Fused2Dims f2 = fused2_dims(h, h->t2x, h->t2m, h->t2zc, h->t2t, h->t2ty);
    // the two-step sweep tiles x, so it also runs where the one-pass band
    // (whole x rows in LDS) does not fit; single steps are then half-steps
    const bool use_f2 = h->fused && h->R2 && h->two && f2.ok;
    const TileDims td = tile_dims(h, h->rows, h->waves, h->zc);
    auto is_rec = [&](int64_t s) { return hrec > 0 && (s + 1) % hrec == 0; };
    auto ckpt_at = [&](int64_t level) {
        return h->adj_ws && level < h->adj_N && level % h->adj_K == 0;
    };
    std::vector<char> ops;
    ops.reserve((size_t)n);
    for (int64_t i = 0; i < n;) {
        const int64_t s = h->step + i;
        if (use_f2 && i + 1 < n && !is_rec(s) && !ckpt_at(s + 1)) {
            ops.push_back(OP_F2);
            i += 2;
        } else {
            ops.push_back(use_fused ? OP_F1 : OP_H);
            i += 1;
        }
    }
    // every one-pass step and sweep swaps the state pairs: an even number of
    // them leaves the state in the buffers of tdse_bind
    const size_t swaps = (size_t)std::count_if(ops.begin(), ops.end(), [](char o) { return o != OP_H; });
    if (swaps % 2 == 1) {
        size_t j = ops.size();
        while (j > 0 && ops[j - 1] != OP_F1) --j;
        if (j > 0) {
            ops[j - 1] = OP_H;
        } else {
            // the last sweep as two single steps (one-pass, which swap, or
            // half-steps, which do not: either way one swap more or less)
            j = ops.size();
            while (ops[j - 1] != OP_F2) --j;
            const char single = use_fused ? OP_F1 : OP_H;
            ops[j - 1] = single;
            ops.insert(ops.begin() + (long)j, single);
        }
    }
    // flux slots per step and partial slots per record of each kind
    auto slots_of = [&](char op) { return op == OP_F2 ? f2.ntiles : op == OP_F1 ? fd.nbands : td.ytiles; };
    auto parts_of = [&](char op) {
        return op == OP_F2 ? (long)f2.nzc * f2.ntiles
                           : op == OP_F1 ? (long)fd.nzc * fd.nbands : (long)td.nzc * td.ytiles;
    };
    char pend_op = OP_H;
    tdse_status st;
    for (char op : ops) {
        const int64_t s = h->step;
        const int k = op == OP_F2 ? 2 : 1;
        if (ckpt_at(s)) {
            // checkpoint of level s for the adjoint
            const AdjLayout L = adj_layout(d, h->adj_N, h->adj_K);
            char* w = static_cast<char*>(h->adj_ws) + L.ckpt + 2 * (size_t)(s / h->adj_K) * L.arr;
            const size_t bytes = (size_t)d.nx * d.ny * d.nz * elem_size(d);
            HIPCHK(h, hipMemcpyAsync(w, h->R, bytes, hipMemcpyDeviceToDevice, h->stream));
            HIPCHK(h, hipMemcpyAsync(w + L.arr, h->I, bytes, hipMemcpyDeviceToDevice, h->stream));
        }
        // partial slots of another kind or a full ring: fold them first
        if (h->pending > 0 && (op != pend_op || h->pending + k > h->F)) {
            st = launch_finalize(h, h->pending, false, 0, slots_of(pend_op), 0);
            if (st != TDSE_OK) return st;
            h->pending = 0;
        }
        pend_op = op;
        const bool record = is_rec(s + k - 1);
        const long rec_idx = record ? (long)((s + k) / hrec) : 0;
        if (op == OP_F2) {
            st = launch_fused2(h, f2, record, rec_idx, h->pending);
            if (st != TDSE_OK) return st;
            std::swap(h->R, h->R2);
            std::swap(h->I, h->I2);
        } else if (op == OP_F1) {
            st = launch_fused(h, fd, record, rec_idx, h->pending);
            if (st != TDSE_OK) return st;
            std::swap(h->R, h->R2);
            std::swap(h->I, h->I2);
        } else {
            st = launch_half(h, MODE_I, h->rows, h->waves, h->zc, 0, 0);
            if (st != TDSE_OK) return st;
            st = launch_half(h, record ? MODE_R_REC : MODE_R, h->rows, h->waves, h->zc, rec_idx,
                             h->pending);
            if (st != TDSE_OK) return st;
        }
        h->pending += k;
        h->step += k;
        if (record || h->pending == h->F) {
            st = launch_finalize(h, h->pending, record, rec_idx, slots_of(op), parts_of(op));
            if (st != TDSE_OK) return st;
            h->pending = 0;
        }
    }
    if (h->pending > 0) {
        st = launch_finalize(h, h->pending, false, 0, slots_of(pend_op), 0);
        if (st != TDSE_OK) return st;
        h->pending = 0;
    }
    return TDSE_OK;
}

tdse_status tdse_step(tdse_handle h, int64_t n) {
    if (!h || n < 0) return TDSE_ERR_ARG;
    if (!h->ready) return fail(h, TDSE_ERR_STATE, "no state: init_gaussian or set_state first");
    const tdse_desc& d = h->d;
    const int64_t hrec = d.record_every;
    if (hrec > 0 && (h->step + n) / hrec + 1 > d.max_records)
        return fail(h, TDSE_ERR_CAPACITY, "record buffer would overflow");
    const FusedDims fd = fused_dims(h, h->fm, h->fzc);
    const bool two = h->two && fused2_dims(h, h->t2x, h->t2m, h->t2zc, h->t2t, h->t2ty).ok;
    const bool graph_ok = h->fused && h->R2 && fd.ok && h->graph_on && h->stream != nullptr &&
                          !h->timing && !h->adj_ws && !two && hrec > 0 && hrec % 2 == 0 &&
                          hrec <= 256;
    if (!graph_ok) return step_plain(h, n);
    // plain steps up to the next record level, graph replays of whole
    // intervals, plain steps for the rest
    const int64_t pre = std::min<int64_t>((hrec - h->step % hrec) % hrec, n);
    tdse_status st = step_plain(h, pre);
    if (st != TDSE_OK) return st;
    const int64_t q = (n - pre) / hrec;
    if (q > 0) {
        if (!h->gb) {
            tdse_batch_ctx* b = new (std::nothrow) tdse_batch_ctx();
            if (!b) return fail(h, TDSE_ERR_OOM, "graph context");
            b->members.push_back(h);
            b->owns = false;
            const Layout L = layout_of(d);
            b->ws = static_cast<char*>(h->ws) + L.gtab;
            b->ws_bytes = L.total - L.gtab;
            b->two = false;
            b->stream = h->stream;
            b->precision = d.precision;
            b->h = hrec;
            b->S = (int)hrec;
            b->M = h->fm;
            b->zc = h->fzc;
            b->pf = h->fpf;
            b->nt = h->ft;
            b->step = h->step;
            st = d.precision == TDSE_F64 ? batch_prepare_t<double>(b) : batch_prepare_t<float>(b);
            if (st != TDSE_OK) {
                std::string m = b->err;
                batch_free_device(b);
                delete b;
                return fail(h, st, "graph capture: " + m);
            }
            h->gb = b;
        }
        tdse_batch_ctx* b = h->gb;
        hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(64), 0, h->stream, b->d_rec,
                           (long)(h->step / hrec + 1));
        hipError_t e = hipGetLastError();
        for (int64_t r = 0; r < q && e == hipSuccess; ++r) e = hipGraphLaunch(b->exec, h->stream);
        if (e != hipSuccess) return hip_check(h, e, "graph launch");
        h->step += q * hrec;
        b->step = h->step;
    }
    return step_plain(h, n - pre - q * hrec);
}

tdse_status tdse_detect(tdse_handle h, tdse_detect_out* out) {
    if (!h || !out) return TDSE_ERR_ARG;
    if (!h->ready) return fail(h, TDSE_ERR_STATE, "no state");
    const tdse_desc& d = h->d;
    double acc = 0.0;
    HIPCHK(h, hipMemcpyAsync(&acc, h->acc, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    const int64_t nrec = d.record_every > 0 ? h->step / d.record_every + 1 : 0;
    std::vector<double> sc((size_t)nrec * 4);
    if (nrec > 0)
        HIPCHK(h, hipMemcpyAsync(sc.data(), h->scal, sc.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    out->step = h->step;
    out->n_records = nrec;
    out->flux_acc = acc;
    out->dt = h->dt;
    out->e_max = h->emax;
    out->records = h->rec;
    out->scalars = h->scal;
    out->pixel = (d.flags & TDSE_FLAG_PIXEL_INTEGRAL) ? h->pix : nullptr;
    if (!std::isfinite(acc)) return fail(h, TDSE_ERR_NONFINITE, "flux accumulator not finite");
    for (double v : sc)
        if (!std::isfinite(v)) return fail(h, TDSE_ERR_NONFINITE, "record scalar not finite");
    return TDSE_OK;
}

tdse_status tdse_copy_scalars(tdse_handle h, double* host, int64_t n) {
    if (!h || !host || n < 0) return TDSE_ERR_ARG;
    if (n > h->d.max_records) return fail(h, TDSE_ERR_ARG, "n exceeds max_records");
    if (n == 0) return TDSE_OK;
    if (!h->scal) return fail(h, TDSE_ERR_STATE, "no record scalars bound");
    HIPCHK(h, hipMemcpyAsync(host, h->scal, (size_t)n * 4 * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return TDSE_OK;
}

tdse_status tdse_set_timing(tdse_handle h, int32_t enable) {
    if (!h) return TDSE_ERR_ARG;
    h->timing = enable != 0;
    return TDSE_OK;
}

namespace {

// Sum the timed launches per kind into ms[nk], count[nk]: nk = 8 keeps the
// record flag, nk = 4 folds it.
tdse_status timing_collect(tdse_handle h, double* ms, int64_t* count, int nk) {
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int k = 0; k < nk; ++k) {
        ms[k] = 0.0;
        count[k] = 0;
    }
    for (size_t e = 0; e + 1 < h->ev_used; e += 2) {
        float t = 0.f;
        HIPCHK(h, hipEventElapsedTime(&t, h->ev[e], h->ev[e + 1]));
        const int k = h->ev_kind[e] % nk;
        ms[k] += t;
        count[k] += 1;
    }
    h->ev_used = 0;
    return TDSE_OK;
}

}  // namespace

tdse_status tdse_timing_read(tdse_handle h, double* ms, int64_t* count) {
    if (!h || !ms || !count) return TDSE_ERR_ARG;
    return timing_collect(h, ms, count, 4);
}

tdse_status tdse_timing_read_split(tdse_handle h, double* ms, int64_t* count) {
    if (!h || !ms || !count) return TDSE_ERR_ARG;
    return timing_collect(h, ms, count, 8);
}

tdse_status tdse_paper_layout_run(tdse_handle h, void* psi_r, void* psi_i, const void* v, int64_t n,
                                  int32_t bx, int32_t by, int32_t bz) {
    if (!h || !psi_r || !psi_i || !v || n < 0) return TDSE_ERR_ARG;
    if (!h->finalized) return fail(h, TDSE_ERR_STATE, "finalize_setup before paper_layout_run");
    if (bx < 1 || by < 1 || bz < 1 || (long)bx * by * bz > 1024)
        return fail(h, TDSE_ERR_ARG, "block Bx x By x Bz must hold 1..1024 threads");
    if (psi_r == psi_i || psi_r == v || psi_i == v)
        return fail(h, TDSE_ERR_ARG, "psi_r, psi_i and v must be distinct");
    const tdse_desc& d = h->d;
    const long nyb = (d.ny + bz - 1) / bz;
    const long gy = ((long)d.nx * nyb + by - 1) / by;
    const long gx = (d.nz + bx - 1) / bx;
    int maxy = 0, maxx = 0;
    HIPCHK(h, hipDeviceGetAttribute(&maxy, hipDeviceAttributeMaxGridDimY, h->device));
    HIPCHK(h, hipDeviceGetAttribute(&maxx, hipDeviceAttributeMaxGridDimX, h->device));
    if (gy > maxy || gx > maxx)
        return fail(h, TDSE_ERR_UNSUPPORTED, "grid of blocks exceeds the device's grid dimensions");
    const dim3 grid((unsigned)gx, (unsigned)gy), block((unsigned)bx, (unsigned)by, (unsigned)bz);
    auto run = [&](auto* tag) -> tdse_status {
        using T = std::remove_pointer_t<decltype(tag)>;
        tdse::ZArgs<T> a;
        a.V = static_cast<const T*>(v);
        a.ca = static_cast<const T*>(h->ca);
        a.cb = static_cast<const T*>(h->cb);
        a.cx = (T)h->c[0];
        a.cy = (T)h->c[1];
        a.cz = (T)h->c[2];
        a.cv = (T)h->c[3];
        diag_parts(h, &a.d0, &a.dlo);
        a.nx = (int)d.nx;
        a.ny = (int)d.ny;
        a.nz = (int)d.nz;
        a.bcx = d.bc[0] == TDSE_BC_ZERO;
        a.bcy = d.bc[1] == TDSE_BC_ZERO;
        a.bcz = d.bc[2] == TDSE_BC_ZERO;
        a.nyb = (int)nyb;
        for (int64_t s = 0; s < n; ++s) {
            for (int half = 0; half < 2; ++half) {
                const bool is_r = half == 1;   // eq. (9), then eq. (8)
                a.U = static_cast<T*>(is_r ? psi_r : psi_i);
                a.S = static_cast<const T*>(is_r ? psi_i : psi_r);
                hipError_t e;
                if constexpr (sizeof(T) == 8)
                    e = tdse::launch_zfast_f64(is_r, grid, block, h->stream, a);
                else
                    e = tdse::launch_zfast_f32(is_r, grid, block, h->stream, a);
                HIPCHK(h, e);
            }
        }
        return TDSE_OK;
    };
    if (d.precision == TDSE_F64) return run((double*)nullptr);
    return run((float*)nullptr);
}

tdse_status tdse_get_tile(tdse_handle h, tdse_tile* out) {
    if (!h || !out) return TDSE_ERR_ARG;
    out->rows = h->rows;
    out->waves = h->waves;
    out->zc = h->zc;
    out->fused = (h->fused && h->R2) ? 1 : 0;
    out->fused_rows = h->fm;
    out->fused_zc = h->fzc;
    out->fused_prefetch = h->fpf ? 1 : 0;
    out->graph = h->graph_on ? 1 : 0;
    out->fused_threads = h->ft;
    out->two_step = (h->two && out->fused) ? 1 : 0;
    out->two_step_tx = h->t2x;
    out->two_step_rows = h->t2m;
    out->two_step_zc = h->t2zc;
    out->two_step_prefetch = h->t2pf ? 1 : 0;
    out->two_step_threads = h->t2t;
    const Fused2Dims f2 = fused2_dims(h, h->t2x, h->t2m, h->t2zc, h->t2t, h->t2ty);
    out->two_step_ty = f2.ok ? f2.ty : 0;
    out->vec_elems = h->W;
    out->vec_groups = h->G;
    out->lanes = h->NL;
    const FusedDims f = fused_dims(h, h->fm, h->fzc);
    out->band_rows = f.ok ? f.ty : 0;
    return TDSE_OK;
}

tdse_status tdse_set_tile(tdse_handle h, const tdse_tile* t) {
    if (!h || !t) return TDSE_ERR_ARG;
    if (t->rows != 1 && t->rows != 2 && t->rows != 4 && t->rows != 8)
        return fail(h, TDSE_ERR_ARG, "rows must be 1, 2, 4 or 8");
    if (t->waves < 1 || t->waves > 4) return fail(h, TDSE_ERR_ARG, "waves must be 1..4");
    if (t->zc < 1 || t->fused_zc < 1) return fail(h, TDSE_ERR_ARG, "z chunks must be >= 1");
    if (t->fused_rows != 2 && t->fused_rows != 3 && t->fused_rows != 4 && t->fused_rows != 6)
        return fail(h, TDSE_ERR_ARG, "fused_rows must be 2, 3, 4 or 6");
    if (h->pending != 0) return fail(h, TDSE_ERR_STATE, "pending flux partials");
    const int fzc = (int)std::min<int64_t>(t->fused_zc, h->d.nz);
    if (t->fused_threads != 64 && t->fused_threads != 128 && t->fused_threads != 256)
        return fail(h, TDSE_ERR_ARG, "fused_threads must be 64, 128 or 256");
    if (t->fused) {
        if (!h->R2) return fail(h, TDSE_ERR_STATE, "one-pass step needs tdse_bind_pingpong");
        // without a fitting one-pass band the pair still serves the two-step
        // sweep, with half-steps for the single steps
        if (!fused_dims(h, t->fused_rows, fzc, t->fused_threads).ok && !t->two_step)
            return fail(h, TDSE_ERR_UNSUPPORTED, "one-pass tile does not fit this grid");
    }
    if (t->two_step_zc < 1) return fail(h, TDSE_ERR_ARG, "z chunks must be >= 1");
    if (t->two_step_threads != 256 && t->two_step_threads != 512 && t->two_step_threads != 1024)
        return fail(h, TDSE_ERR_ARG, "two_step_threads must be 256, 512 or 1024");
    const int t2zc = (int)std::min<int64_t>(t->two_step_zc, h->d.nz);
    if (t->two_step) {
        if (!t->fused) return fail(h, TDSE_ERR_ARG, "the two-step sweep runs with the one-pass step");
        const int pm = t->two_step_rows, pt = t->two_step_threads;
        if (!((pt == 256 && (pm == 2 || pm == 3)) || (pt == 512 && (pm == 1 || pm == 2)) ||
              (pt == 1024 && pm == 1)))
            return fail(h, TDSE_ERR_UNSUPPORTED,
                        "two-step (rows, threads) must be (2,256), (3,256), (1,512), (2,512) or (1,1024)");
        if (t->two_step_ty < 0) return fail(h, TDSE_ERR_ARG, "two_step_ty must be >= 0");
        if (!fused2_dims(h, t->two_step_tx, t->two_step_rows, t2zc, t->two_step_threads, t->two_step_ty).ok)
            return fail(h, TDSE_ERR_UNSUPPORTED, "two-step tile does not fit this grid");
    }
    graph_invalidate(h);
    h->rows = t->rows;
    h->waves = t->waves;
    h->zc = (int)std::min<int64_t>(t->zc, h->d.nz);
    h->fused = t->fused != 0;
    h->graph_on = t->graph != 0;
    h->fm = t->fused_rows;
    h->fzc = fzc;
    h->fpf = t->fused_prefetch != 0;
    h->ft = t->fused_threads;
    h->two = t->two_step != 0;
    h->t2x = t->two_step_tx;
    h->t2m = t->two_step_rows;
    h->t2zc = t2zc;
    h->t2pf = t->two_step_prefetch != 0;
    h->t2t = t->two_step_threads;
    h->t2ty = t->two_step ? std::max(0, t->two_step_ty) : 0;
    return TDSE_OK;
}


tdse_status tdse_autotune(tdse_handle h, int32_t steps, int32_t flags, tdse_tile* out) {
    if (!h || !out || steps < 1) return TDSE_ERR_ARG;
    if (flags & ~(int32_t)(1 | 2 | 4 | TDSE_TUNE_REFRESH)) return TDSE_ERR_ARG;
    if (!h->ready) return fail(h, TDSE_ERR_STATE, "no state: init_gaussian or set_state first");
    if (h->pending != 0) return fail(h, TDSE_ERR_STATE, "pending flux partials");
    if (h->adj_ws) return fail(h, TDSE_ERR_STATE, "unbind the adjoint before tuning");
    const int families = (flags & 7) ? (flags & 7) : 7;
    const char* cache = std::getenv("TDSE_TUNE_CACHE");
    if (cache && !*cache) cache = nullptr;
    const std::string key = cache ? tune_key(h, families) : std::string();
    if (cache && !(flags & TDSE_TUNE_REFRESH)) {
        tdse_tile hit;
        tdse_get_tile(h, &hit);
        if (tune_cache_lookup(cache, key, &hit) && tdse_set_tile(h, &hit) == TDSE_OK)
            return tdse_get_tile(h, out);
    }
    const bool want2p = families & 1, want1p = families & 2, want2s = families & 4;
    tdse_tile base;
    tdse_get_tile(h, &base);
    std::vector<tdse_tile> cands;
    if (want2p) {
        // (one plane per workgroup: small, cache-resident grids, where the
        // z march's load latency and not the bytes set the time)
        const int c[5][3] = {{2, 4, 64}, {4, 4, 64}, {2, 4, 16}, {1, 4, 32}, {1, 4, 1}};
        for (const auto& x : c) {
            tdse_tile t = base;
            t.fused = 0;
            t.two_step = 0;
            t.rows = x[0];
            t.waves = x[1];
            t.zc = x[2];
            cands.push_back(t);
        }
    }
    if (want1p && h->R2) {
        const int c[6][3] = {{3, 64, 256}, {2, 32, 256}, {4, 64, 256}, {2, 8, 128}, {3, 16, 256},
                             {2, 1, 128}};
        for (const auto& x : c) {
            tdse_tile t = base;
            t.fused = 1;
            t.two_step = 0;
            t.fused_rows = x[0];
            t.fused_zc = x[1];
            t.fused_threads = x[2];
            t.fused_prefetch = 0;
            cands.push_back(t);
        }
    }
    if (want2s && h->R2) {
        const int c[9][4] = {{64, 1, 512, 64}, {56, 1, 512, 64}, {56, 2, 512, 128},
                             {64, 2, 256, 64}, {32, 1, 512, 32}, {32, 2, 256, 128},
                             {64, 1, 1024, 128}, {32, 1, 1024, 32}, {120, 1, 1024, 64}};
        for (const auto& x : c) {
            tdse_tile t = base;
            t.fused = 1;
            t.two_step = 1;
            t.two_step_tx = x[0];
            t.two_step_rows = x[1];
            t.two_step_threads = x[2];
            t.two_step_zc = x[3];
            t.two_step_prefetch = 1;
            cands.push_back(t);
        }
        // the one-round tile (one_round_tile) of each of a few widths
        const bool f64 = h->d.precision == TDSE_F64;
        const int w1[3] = {128, 80, 64}, w2[2] = {64, 32};
        for (int iw = 0; iw < (f64 ? 2 : 3); ++iw) {
            const int tx = f64 ? w2[iw] : w1[iw];
            int ty = 0, zc = 0;
            if (!one_round_tile(h, tx, &ty, &zc)) continue;
            tdse_tile t = base;
            t.fused = 1;
            t.two_step = 1;
            t.two_step_tx = tx;
            t.two_step_rows = 1;
            t.two_step_threads = 1024;
            t.two_step_zc = zc;
            t.two_step_ty = ty;
            t.two_step_prefetch = 1;
            cands.push_back(t);
        }
        // and the cost model's choice for this grid (its z chunk fills the
        // last wave of workgroups)
        const bool two0 = h->two;
        const bool pf0 = h->t2pf;
        const int x0 = h->t2x, m0 = h->t2m, t0 = h->t2t, z0 = h->t2zc;
        default_two_step(h);
        if (h->two) {
            tdse_tile t = base;
            t.fused = 1;
            t.two_step = 1;
            t.two_step_tx = h->t2x;
            t.two_step_rows = h->t2m;
            t.two_step_threads = h->t2t;
            t.two_step_zc = h->t2zc;
            t.two_step_prefetch = 1;
            cands.push_back(t);
        }
        h->two = two0;
        h->t2pf = pf0;
        h->t2x = x0;
        h->t2m = m0;
        h->t2t = t0;
        h->t2zc = z0;
    }
    // no records while tuning (the state is given up anyway)
    const int64_t hrec = h->d.record_every;
    h->d.record_every = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    tdse_status st = hip_check(h, hipEventCreate(&e0), "event");
    if (st == TDSE_OK) st = hip_check(h, hipEventCreate(&e1), "event");
    float best = -1.f;
    tdse_tile win = base;
    for (const tdse_tile& t : cands) {
        if (st != TDSE_OK) break;
        if (tdse_set_tile(h, &t) != TDSE_OK) continue;  // does not fit this grid
        st = step_plain(h, 2);
        if (st == TDSE_OK) st = hip_check(h, hipEventRecord(e0, h->stream), "event");
        if (st == TDSE_OK) st = step_plain(h, steps);
        if (st == TDSE_OK) st = hip_check(h, hipEventRecord(e1, h->stream), "event");
        if (st == TDSE_OK) st = hip_check(h, hipEventSynchronize(e1), "event");
        float ms = 0.f;
        if (st == TDSE_OK) st = hip_check(h, hipEventElapsedTime(&ms, e0, e1), "event");
        if (st == TDSE_OK && (best < 0 || ms < best)) {
            best = ms;
            win = t;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    h->d.record_every = hrec;
    h->ready = false;
    if (st != TDSE_OK) return st;
    st = tdse_set_tile(h, &win);
    if (st != TDSE_OK) return st;
    if (cache && !tune_cache_store(cache, key, win))
        return fail(h, TDSE_ERR_ARG, std::string("cannot write the tile cache ") + cache);
    return tdse_get_tile(h, out);
}

tdse_status tdse_bind_pingpong(tdse_handle h, void* psi_r2, void* psi_i2) {
    if (!h) return TDSE_ERR_ARG;
    if (!h->bound) return fail(h, TDSE_ERR_STATE, "bind before bind_pingpong");
    if (!psi_r2 || !psi_i2) return fail(h, TDSE_ERR_ARG, "null pointer");
    if (!aligned(psi_r2) || !aligned(psi_i2)) return fail(h, TDSE_ERR_ARG, "pointer not 256-byte aligned");
    void* used[5] = {h->R, h->I, h->V, psi_r2, psi_i2};
    for (int i = 0; i < 5; ++i)
        for (int j = i + 1; j < 5; ++j)
            if (used[i] == used[j]) return fail(h, TDSE_ERR_ARG, "aliased arrays");
    graph_invalidate(h);
    h->R2 = psi_r2;
    h->I2 = psi_i2;
    h->fused = fused_dims(h, h->fm, h->fzc).ok ||
               (h->two && fused2_dims(h, h->t2x, h->t2m, h->t2zc, h->t2t, h->t2ty).ok);
    return TDSE_OK;
}

tdse_status tdse_adjoint_workspace_size(const tdse_desc* d, int64_t n_steps, int32_t ckpt_every,
                                        size_t* bytes) {
    tdse_status s = check_desc(d);
    if (s != TDSE_OK) return s;
    if (!bytes || n_steps < 1 || ckpt_every < 1) return TDSE_ERR_ARG;
    *bytes = adj_layout(*d, n_steps, ckpt_every).total;
    return TDSE_OK;
}

tdse_status tdse_bind_adjoint(tdse_handle h, void* adj_ws, size_t bytes, int64_t n_steps,
                              int32_t ckpt_every) {
    if (!h) return TDSE_ERR_ARG;
    if (!adj_ws) {
        h->adj_ws = nullptr;
        return TDSE_OK;
    }
    if (!h->bound) return fail(h, TDSE_ERR_STATE, "bind before bind_adjoint");
    if (n_steps < 1 || ckpt_every < 1) return fail(h, TDSE_ERR_ARG, "n_steps and ckpt_every must be >= 1");
    if (!aligned(adj_ws)) return fail(h, TDSE_ERR_ARG, "adjoint workspace not 256-byte aligned");
    if (bytes < adj_layout(h->d, n_steps, ckpt_every).total)
        return fail(h, TDSE_ERR_ARG, "adjoint workspace too small");
    if (h->step != 0) return fail(h, TDSE_ERR_STATE, "bind the adjoint before stepping from level 0");
    h->adj_ws = adj_ws;
    h->adj_N = n_steps;
    h->adj_K = ckpt_every;
    return TDSE_OK;
}

tdse_status tdse_adjoint(tdse_handle h, const void* dL_drho, double* dL_dV, void* dL_dR0,
                         void* dL_dI0) {
    if (!h || !dL_dV) return TDSE_ERR_ARG;
    if (!h->adj_ws) return fail(h, TDSE_ERR_STATE, "tdse_bind_adjoint first");
    if (h->step != h->adj_N) return fail(h, TDSE_ERR_STATE, "run exactly n_steps forward before the adjoint");
    if (h->d.record_every > 0 && !dL_drho) return fail(h, TDSE_ERR_ARG, "dL_drho required");
    if (h->pending != 0) return fail(h, TDSE_ERR_STATE, "pending flux partials");
    if (!h->half_vec && !adj_fused_dims(h).ok)
        return fail(h, TDSE_ERR_UNSUPPORTED,
                    "the reverse step of this x extent needs the one-pass band (tdse_bind_pingpong, "
                    "nx / vector width <= 256 and its rows in LDS)");
    if (h->d.precision == TDSE_F64)
        return run_adjoint<double>(h, static_cast<const double*>(dL_drho), dL_dV,
                                   static_cast<double*>(dL_dR0), static_cast<double*>(dL_dI0));
    return run_adjoint<float>(h, static_cast<const float*>(dL_drho), dL_dV,
                              static_cast<float*>(dL_dR0), static_cast<float*>(dL_dI0));
}

tdse_status tdse_potential_vjp(tdse_handle h, const tdse_atom* atoms, int64_t n,
                               const tdse_pot_params* p, const double* dL_dV, double* dL_dpos,
                               double* dL_damp) {
    if (!h || !p || !dL_dV || n < 0 || (n > 0 && (!atoms || !dL_dpos || !dL_damp))) return TDSE_ERR_ARG;
    if (n == 0) return TDSE_OK;
    const tdse_desc& d = h->d;
    if (!(p->cutoff > 0) || !(p->soft >= 0) || !(p->kappa > 0) || !(p->a0 > 0))
        return fail(h, TDSE_ERR_ARG, "bad potential parameters");
    std::vector<double> flat((size_t)n * 5);
    for (int64_t a = 0; a < n; ++a) {
        flat[5 * a + 0] = atoms[a].x;
        flat[5 * a + 1] = atoms[a].y;
        flat[5 * a + 2] = atoms[a].z;
        flat[5 * a + 3] = atoms[a].Z;
        flat[5 * a + 4] = atoms[a].amp;
        if (!(atoms[a].Z > 0)) return fail(h, TDSE_ERR_ARG, "bad atom");
    }
    double* d_atoms = nullptr;
    double* d_out = nullptr;
    if (hipMalloc(&d_atoms, flat.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_out, (size_t)n * 4 * sizeof(double)) != hipSuccess) {
        if (d_atoms) (void)hipFree(d_atoms);
        return fail(h, TDSE_ERR_OOM, "vjp temporaries");
    }
    hipError_t e = hipMemcpyAsync(d_atoms, flat.data(), flat.size() * sizeof(double),
                                  hipMemcpyHostToDevice, h->stream);
    VjpArgs a;
    a.nx = (int)d.nx;
    a.ny = (int)d.ny;
    a.nz = (int)d.nz;
    a.dx = d.dx;
    a.dy = d.dy;
    a.dz = d.dz;
    a.Lx = d.nx * d.dx;
    a.Ly = d.ny * d.dy;
    a.Lz = d.nz * d.dz;
    a.bcx = d.bc[0] == TDSE_BC_ZERO;
    a.bcy = d.bc[1] == TDSE_BC_ZERO;
    a.bcz = d.bc[2] == TDSE_BC_ZERO;
    a.screened = p->screened;
    a.atoms = d_atoms;
    a.gV = dL_dV;
    a.soft = p->soft;
    a.cutoff = p->cutoff;
    a.kappa = p->kappa;
    a.a0 = p->a0;
    a.out = d_out;
    std::vector<double> out((size_t)n * 4);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(potential_vjp_kernel, dim3((unsigned)n), dim3(256), 0, h->stream, a);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(out.data(), d_out, out.size() * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(d_atoms);
    (void)hipFree(d_out);
    if (e != hipSuccess) return hip_check(h, e, "potential_vjp");
    for (int64_t a2 = 0; a2 < n; ++a2) {
        dL_dpos[3 * a2 + 0] = out[4 * a2 + 0];
        dL_dpos[3 * a2 + 1] = out[4 * a2 + 1];
        dL_dpos[3 * a2 + 2] = out[4 * a2 + 2];
        dL_damp[a2] = out[4 * a2 + 3];
    }
    return TDSE_OK;
}

tdse_status tdse_batch_create(const tdse_desc* descs, int32_t n, void* stream, tdse_batch* out) {
    if (!descs || n < 1 || !out) return TDSE_ERR_ARG;
    *out = nullptr;
    tdse_batch_ctx* b = new (std::nothrow) tdse_batch_ctx();
    if (!b) return TDSE_ERR_OOM;
    b->stream = static_cast<hipStream_t>(stream);
    b->precision = descs[0].precision;
    b->h = descs[0].record_every;
    for (int32_t i = 0; i < n; ++i) {
        if (descs[i].precision != b->precision || descs[i].record_every != b->h) {
            for (tdse_ctx* m : b->members) tdse_destroy(m);
            delete b;
            return TDSE_ERR_ARG;
        }
        tdse_handle h = nullptr;
        tdse_status s = tdse_create(&descs[i], stream, &h);
        if (s != TDSE_OK) {
            for (tdse_ctx* m : b->members) tdse_destroy(m);
            delete b;
            return s;
        }
        b->members.push_back(h);
    }
    if (b->h > 256 || (b->h > 0 && b->h % 2)) {
        for (tdse_ctx* m : b->members) tdse_destroy(m);
        delete b;
        return TDSE_ERR_UNSUPPORTED;
    }
    b->S = b->h > 0 ? (int)b->h : 64;
    *out = b;
    return TDSE_OK;
}

tdse_status tdse_batch_member(tdse_batch b, int32_t i, tdse_handle* h) {
    if (!b || !h || i < 0 || i >= (int32_t)b->members.size()) return TDSE_ERR_ARG;
    *h = b->members[(size_t)i];
    return TDSE_OK;
}

tdse_status tdse_batch_bind(tdse_batch b, int32_t i, void* psi_r, void* psi_i, void* v, void* workspace,
                            size_t workspace_bytes, void* records, double* scalars, double* pixel,
                            void* psi_r2, void* psi_i2) {
    if (!b || i < 0 || i >= (int32_t)b->members.size()) return TDSE_ERR_ARG;
    tdse_handle h = b->members[(size_t)i];
    // the captured graph holds the member's old pointers
    batch_free_device(b);
    tdse_status s = tdse_bind(h, psi_r, psi_i, v, workspace, workspace_bytes, records, scalars, pixel);
    if (s != TDSE_OK) return bfail(b, s, h->err);
    s = tdse_bind_pingpong(h, psi_r2, psi_i2);
    if (s != TDSE_OK) return bfail(b, s, h->err);
    return TDSE_OK;
}

tdse_status tdse_batch_detect(tdse_batch b, int32_t i, tdse_detect_out* out) {
    if (!b || i < 0 || i >= (int32_t)b->members.size()) return TDSE_ERR_ARG;
    return tdse_detect(b->members[(size_t)i], out);
}

tdse_status tdse_batch_set_tile(tdse_batch b, int32_t fused_rows, int32_t fused_zc, int32_t prefetch,
                                int32_t threads) {
    if (!b) return TDSE_ERR_ARG;
    if (threads != 64 && threads != 128 && threads != 256) return bfail(b, TDSE_ERR_ARG, "threads");
    if (fused_rows != 2 && fused_rows != 3 && fused_rows != 4 && fused_rows != 6) return bfail(b, TDSE_ERR_ARG, "fused_rows");
    if (fused_zc < 1) return bfail(b, TDSE_ERR_ARG, "fused_zc");
    batch_free_device(b);
    b->M = fused_rows;
    b->zc = fused_zc;
    b->pf = prefetch != 0;
    b->nt = threads;
    return TDSE_OK;
}

tdse_status tdse_batch_set_two_step(tdse_batch b, int32_t enable, int32_t tx, int32_t rows,
                                    int32_t zc, int32_t prefetch, int32_t threads) {
    if (!b) return TDSE_ERR_ARG;
    const bool pair_ok = (threads == 256 && (rows == 2 || rows == 3)) ||
                         (threads == 512 && (rows == 1 || rows == 2)) || (threads == 1024 && rows == 1);
    if (tx < 8 || zc < 1 || !pair_ok) return bfail(b, TDSE_ERR_ARG, "two-step tile");
    batch_free_device(b);
    b->two = enable != 0;
    b->t2x = tx;
    b->t2m = rows;
    b->t2zc = zc;
    b->t2pf = prefetch != 0;
    b->t2t = threads;
    return TDSE_OK;
}

tdse_status tdse_batch_workspace_size(tdse_batch b, size_t* bytes) {
    if (!b || !bytes) return TDSE_ERR_ARG;
    *bytes = batch_tables_bytes(b->members.size());
    return TDSE_OK;
}

tdse_status tdse_batch_bind_workspace(tdse_batch b, void* ws, size_t bytes) {
    if (!b) return TDSE_ERR_ARG;
    if (ws && (!aligned(ws) || bytes < batch_tables_bytes(b->members.size())))
        return bfail(b, TDSE_ERR_ARG, "batch workspace short or not 256-byte aligned");
    batch_free_device(b);
    b->ws = ws;
    b->ws_bytes = ws ? bytes : 0;
    return TDSE_OK;
}

tdse_status tdse_batch_prepare(tdse_batch b) {
    if (!b) return TDSE_ERR_ARG;
    batch_free_device(b);
    int64_t step = -1;
    for (tdse_ctx* h : b->members) {
        if (!h->ready || !h->R2) return bfail(b, TDSE_ERR_STATE, "every member needs a state and tdse_bind_pingpong");
        if (h->pending) return bfail(b, TDSE_ERR_STATE, "pending flux partials");
        if (step < 0) step = h->step;
        if (h->step != step) return bfail(b, TDSE_ERR_STATE, "members at different steps");
    }
    if (b->h > 0 && step % b->h) return bfail(b, TDSE_ERR_STATE, "members must sit on a record level");
    b->step = step;
    b->par = 0;
    b->use2 = false;
    if (b->two) {
        bool used = false;
        tdse_status s = b->precision == TDSE_F64 ? batch_prepare2_t<double>(b, &used)
                                                 : batch_prepare2_t<float>(b, &used);
        if (s != TDSE_OK) return s;
        if (used) {
            b->use2 = true;
            return TDSE_OK;
        }
    }
    return b->precision == TDSE_F64 ? batch_prepare_t<double>(b) : batch_prepare_t<float>(b);
}

tdse_status tdse_batch_run(tdse_batch b, int64_t n) {
    if (!b || n < 0) return TDSE_ERR_ARG;
    if (!b->prepared) return bfail(b, TDSE_ERR_STATE, "tdse_batch_prepare first");
    if (n % b->S) return bfail(b, TDSE_ERR_ARG, "n must be a multiple of the record interval (64 without records)");
    for (tdse_ctx* h : b->members) {
        if (h->step != b->step) return bfail(b, TDSE_ERR_STATE, "a member was stepped outside the batch");
        if (b->h > 0 && (b->step + n) / b->h + 1 > h->d.max_records)
            return bfail(b, TDSE_ERR_CAPACITY, "record buffer would overflow");
    }
    if (n == 0) return TDSE_OK;
    const long next = b->h > 0 ? (long)(b->step / b->h + 1) : 0;
    hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(64), 0, b->stream, b->d_rec, next);
    hipError_t e = hipGetLastError();
    const bool flips = b->use2 && (b->S / 2) % 2 == 1;
    for (int64_t r = 0; r < n / b->S && e == hipSuccess; ++r) {
        e = hipGraphLaunch(b->par ? b->exec1 : b->exec, b->stream);
        if (flips) b->par ^= 1;
    }
    // an odd number of swaps left the levels in the second pair: copy them
    // back so that the members' bound arrays hold the state
    for (size_t i = 0; i < b->members.size() && e == hipSuccess && b->par; ++i) {
        tdse_ctx* h = b->members[i];
        const size_t bytes = (size_t)h->d.nx * h->d.ny * h->d.nz * elem_size(h->d);
        e = hipMemcpyAsync(h->R, h->R2, bytes, hipMemcpyDeviceToDevice, b->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(h->I, h->I2, bytes, hipMemcpyDeviceToDevice, b->stream);
    }
    if (e == hipSuccess) b->par = 0;
    if (e != hipSuccess) return bfail(b, TDSE_ERR_DEVICE, std::string("batch run: ") + hipGetErrorString(e));
    b->step += n;
    for (tdse_ctx* h : b->members) h->step += n;
    return TDSE_OK;
}

tdse_status tdse_batch_status(tdse_batch b, int32_t* per_config) {
    if (!b || !per_config) return TDSE_ERR_ARG;
    tdse_status worst = TDSE_OK;
    for (size_t i = 0; i < b->members.size(); ++i) {
        tdse_detect_out o;
        tdse_status s = tdse_detect(b->members[i], &o);
        per_config[i] = s;
        if (s != TDSE_OK && worst == TDSE_OK) worst = s;
    }
    return worst;
}

const char* tdse_batch_last_error(tdse_batch b) { return b ? b->err.c_str() : ""; }

tdse_status tdse_batch_destroy(tdse_batch b) {
    if (!b) return TDSE_OK;
    batch_free_device(b);
    if (b->owns)
        for (tdse_ctx* h : b->members) tdse_destroy(h);
    delete b;
    return TDSE_OK;
}

}  // extern "C"
