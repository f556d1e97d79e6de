/*
 * libtdse: FDTD integration of the 3D time-dependent Schrodinger equation on
 * one AMD Instinct MI355X (gfx950).
 *
 * The method is the staggered leapfrog of Nagaya, Omatsu and Packwood,
 * arXiv 2401.07416, section 2.1:
 *   eq. (2)   i hbar dpsi/dt = -(hbar^2/2m) lap psi + V psi
 *   eq. (5)   psi = psiR + i psiI, psiR at integer and psiI at half-integer
 *             time levels
 *   eq. (9)   psiI^{n+1/2} = psiI^{n-1/2} + sum_d c_d delta_d^2 psiR^n
 *                            - c_v V psiR^n
 *   eq. (8)   psiR^{n+1}   = psiR^n - sum_d c_d delta_d^2 psiI^{n+1/2}
 *                            + c_v V psiI^{n+1/2}
 *             c_d = hbar dt / (2 m d^2), c_v = dt / hbar
 *   eq. (10)  a complex absorbing potential near the z ends, here a
 *             per-plane rate W_k >= 0 applied time-centred:
 *             gamma = W_k dt / hbar, ca = (1 - gamma/2)/(1 + gamma/2),
 *             cb = 1/(1 + gamma/2), U_new = ca U_old + cb (update term)
 *   eqs. (13)-(14)  periodic wrap (i +- 1) mod N; a zero (Dirichlet)
 *             boundary per axis is also offered
 *   eq. (15)  detection-plane density rho = psiR^2 + psiI^2 on plane k_det,
 *             stored every h steps starting at n = 0; the density at level n
 *             is psiR^n^2 + psiI^{n-1/2}^2 (section 2.1)
 *   eqs. (3)-(4)  Gaussian initial packet.
 * Added to the paper's outputs, always accumulated in FP64:
 *   Q   = dV sum[psiI^{n-1/2}^2 + psiR^{n-1} psiR^n]  (record 0:
 *         dV sum[psiR^0^2 + psiI^{-1/2} psiI^{+1/2}]), the quadratic form the
 *         leapfrog conserves exactly when W = 0;
 *   naive norm = dV sum[psiR^n^2 + psiI^{n-1/2}^2];
 *   flux through the face between planes k_det and k_det+1, accumulated
 *         over steps: Phi^{n+1/2} = dV c_z sum_ij[I_{k+1}(R^n_k + R^{n+1}_k)
 *         - I_k(R^n_{k+1} + R^{n+1}_{k+1})], I = psiI^{n+1/2}, k = k_det
 *         (positive towards +z), the scheme's exact discrete current.
 *
 * Conventions for every call
 *  - Status: every call returns tdse_status (0 = TDSE_OK); nothing aborts or
 *    throws across this boundary.  tdse_last_error(h) keeps the message of
 *    the last failure on a handle.
 *  - Layout: every 3D array is [nz][ny][nx], x fastest, contiguous, in the
 *    handle's precision (float for TDSE_F32, double for TDSE_F64), with a
 *    base address aligned to 256 bytes.  Grid point (i, j, k) sits at
 *    r = (i dx, j dy, k dz).
 *  - Ownership: all large device memory belongs to the caller.  A handle
 *    borrows the pointers passed to tdse_bind and never frees them.  Its
 *    internal scratch lives in the caller's workspace (tdse_workspace_size).
 *    Setup calls (tdse_build_potential) may allocate and free temporary
 *    device memory before they return; the stepping calls allocate nothing.
 *  - Streams: each handle launches on one HIP stream given at creation (NULL
 *    = the null stream).  Launching calls are asynchronous.  Calls that
 *    return host data synchronise that stream first.
 *  - Threads: a handle is not thread-safe; distinct handles are independent.
 *  - Units: the caller chooses them through hbar and mass (atomic units:
 *    hbar = m = 1; eV-Angstrom-fs: hbar = 0.6582119569, m = hbar^2/7.619964).
 *  - Extents: any nx, ny <= 2^24 and nz <= 65535 (each <= 2^20 as a
 *    description), with one z plane below 0x7ffffff0 bytes (nx ny x 4 in
 *    FP32, x 8 in FP64: the kernels keep 32-bit byte offsets within a
 *    plane); larger planes return TDSE_ERR_UNSUPPORTED from
 *    tdse_validate_desc and tdse_create.  Where nx = W G L (W in {1, 2, 4}
 *    floats or {1, 2} doubles, G in {1, 2, 4, 8}, L <= 64 lanes) the
 *    half-steps spread a row over one wavefront; other nx take a half-step
 *    kernel for any width (the same bits, slower), and the one-pass and
 *    two-step kernels tile x either way.
 */
#ifndef TDSE_H
#define TDSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tdse_status;

enum {
    TDSE_OK = 0,
    TDSE_ERR_ARG = 1,         /* bad argument: null, size, alignment, range */
    TDSE_ERR_STATE = 2,       /* call made out of order */
    TDSE_ERR_UNSTABLE = 3,    /* dt above hbar / E_max without the override flag */
    TDSE_ERR_NONFINITE = 4,   /* a NaN or Inf reached the FP64 sums */
    TDSE_ERR_DEVICE = 5,      /* HIP runtime error; message kept */
    TDSE_ERR_OOM = 6,         /* device allocation failed (setup temporaries) */
    TDSE_ERR_UNSUPPORTED = 7, /* shape or option the library does not handle */
    TDSE_ERR_CAPACITY = 8     /* the record buffer (or the no-alloc scratch) would overflow */
};

enum { TDSE_BC_PERIODIC = 0, TDSE_BC_ZERO = 1 };
enum { TDSE_F32 = 0, TDSE_F64 = 1 };
enum { TDSE_INIT_HALFSTEP = 0, TDSE_INIT_NAIVE = 1 };
enum {
    TDSE_FLAG_ALLOW_UNSTABLE = 1u, /* accept dt above the bound */
    TDSE_FLAG_PIXEL_INTEGRAL = 2u  /* accumulate P_ij += h dt rho_ij (FP64) */
};

/* Problem description (section 2.1 grid, eq. (11) time step, eq. (15)
 * detection).  dt > 0 is used as given; otherwise dt = dt_frac * hbar /
 * E_max with E_max the Gershgorin bound of tdse_time_step_bound. */
typedef struct tdse_desc {
    int64_t nx, ny, nz;
    double dx, dy, dz;
    double hbar, mass;
    double dt;
    double dt_frac;
    int32_t bc[3];          /* TDSE_BC_* per axis x, y, z */
    int32_t precision;      /* TDSE_F32 or TDSE_F64 (state, V and records) */
    int64_t k_det;          /* detection plane index, 0 <= k_det < nz */
    int64_t record_every;   /* h >= 0; 0 = no records */
    int64_t max_records;    /* capacity of the record buffers */
    uint32_t flags;         /* TDSE_FLAG_* */
    uint32_t reserved;
} tdse_desc;

/* One atom of the synthetic potential: position, nuclear charge, amplitude. */
typedef struct tdse_atom {
    double x, y, z, Z, amp;
} tdse_atom;

/* V(r) = sum_a amp_a v_Z(|r - X_a|) over atoms closer than cutoff, minimum
 * image along periodic axes, with
 *   v_Z(d) = -Z kappa exp(-d / lam_Z) / sqrt(d^2 + soft^2),
 *   lam_Z = 0.8853 a0 Z^(-1/3) if screened, else no exponential. */
typedef struct tdse_pot_params {
    double soft, cutoff, kappa, a0;
    int32_t screened;
    int32_t reserved;
} tdse_pot_params;

/* Result of tdse_detect.  Pointers are the caller's own bound buffers. */
typedef struct tdse_detect_out {
    int64_t step;            /* global step counter n */
    int64_t n_records;       /* records written so far (record 0 included) */
    double flux_acc;         /* accumulated flux through face k_det + 1/2 */
    double dt, e_max;
    const void* records;     /* device [max_records][ny][nx], state precision */
    const double* scalars;   /* device [max_records][4]: plane_sum, naive_norm, Q, flux_acc */
    const double* pixel;     /* device [ny][nx] or NULL */
} tdse_detect_out;

typedef struct tdse_ctx* tdse_handle;

/* Version of this interface. */
int32_t tdse_abi_version(void);

/* Human-readable name of a status code (static storage). */
const char* tdse_status_string(tdse_status s);

/* Last error message recorded on h ("" if none; static "" for NULL). */
const char* tdse_last_error(tdse_handle h);

/* Host-only check of a description: sizes > 0, spacings, hbar, mass > 0,
 * boundary and precision codes, 0 <= k_det < nz, record settings, and
 * dt or dt_frac > 0.  Touches no device.  dt_bound (may be NULL): hbar /
 * E_kin with E_kin = (hbar^2/2m) sum_d 4/d^2, the time-step bound of
 * section 2.1 for V = 0 (the potential enters E_max only once it is known:
 * tdse_time_step_bound for a range of V, tdse_finalize_setup for the bound
 * V); +inf when no axis couples cells. */
tdse_status tdse_validate_desc(const tdse_desc* d, double* dt_bound);

/* Host-only Gershgorin bound on max |E| of the discrete Hamiltonian of the
 * section 2.1 scheme for a potential with range [vmin, vmax]:
 *   E_max = max(|vmin|, |vmax + (hbar^2/2m) sum_d 4/d^2|)
 * (a periodic axis of length 1 adds nothing), and dt_bound = hbar / E_max.
 * The leapfrog is stable for dt < 2 hbar / max|E|, so dt_bound leaves at
 * least a factor 2 of margin.  Either output pointer may be NULL. */
tdse_status tdse_time_step_bound(const tdse_desc* d, double vmin, double vmax, double* e_max,
                                 double* dt_bound);

/* Bytes of device workspace a handle for d needs (host only). */
tdse_status tdse_workspace_size(const tdse_desc* d, size_t* bytes);

/* Create a handle on the current HIP device, launching on `stream` (a
 * hipStream_t, NULL for the null stream).  Host memory only. */
tdse_status tdse_create(const tdse_desc* d, void* stream, tdse_handle* out);

/* Destroy a handle (NULL is accepted).  Does not free bound memory. */
tdse_status tdse_destroy(tdse_handle h);

/* Attach caller device memory:
 *   psi_r, psi_i, v : [nz][ny][nx] in the handle's precision;
 *   workspace       : >= tdse_workspace_size bytes;
 *   records         : [max_records][ny][nx] in the handle's precision, or
 *                     NULL when record_every == 0;
 *   scalars         : double [max_records][4], or NULL when
 *                     record_every == 0;
 *   pixel           : double [ny][nx] when TDSE_FLAG_PIXEL_INTEGRAL is set,
 *                     else ignored.
 * All pointers 256-byte aligned.  Rebinding resets the handle to the
 * "potential not set" state. */
tdse_status tdse_bind(tdse_handle h, void* psi_r, void* psi_i, void* v, void* workspace,
                      size_t workspace_bytes, void* records, double* scalars, double* pixel);

/* Fill the bound V with the atom-sum potential (setup; asynchronous on the
 * handle's stream except for a short host sort).  atoms is host memory
 * [n].  Alternatively the caller writes V itself and skips this call. */
tdse_status tdse_build_potential(tdse_handle h, const tdse_atom* atoms, int64_t n,
                                 const tdse_pot_params* p);

/* Fill the bound V by interpolating a potential given on one unit cell
 * (section 2.3: the potential of one cell is repeated in x and y and
 * interpolated onto the mesh points; the paper does not name the scheme,
 * this is trilinear).  table: device memory, double [uz][uy][ux], x
 * fastest, owned by the caller and read only; its sample (a, b, c) sits at
 * origin + (a sx, b sy, c sz) with spacing = {sx, sy, sz} > 0 and origin
 * host arrays of 3.  The cell repeats in x and y with periods ux sx and
 * uy sy; beyond the first and last table planes in z the table is held
 * constant.  Mesh point (i, j, k) sits at (i dx, j dy, k dz).  Computed in
 * FP64, stored in the state precision; asynchronous on the handle's stream
 * (the table must stay valid until the stream reaches the call).  Like
 * tdse_build_potential it replaces V before tdse_finalize_setup.
 * TDSE_ERR_ARG for null pointers, sizes < 1 or more than 2^31 samples,
 * non-positive spacing; TDSE_ERR_STATE before tdse_bind. */
tdse_status tdse_interpolate_potential(tdse_handle h, const double* table, int32_t ux, int32_t uy,
                                      int32_t uz, const double* spacing, const double* origin);

/* CAP rates W[nz] >= 0 (host memory, energy units); NULL clears the CAP. */
tdse_status tdse_set_cap(tdse_handle h, const double* w, int64_t nz);

/* Quadratic CAP ramp (the shape of eq. (10)) over n_bottom planes at the
 * bottom and n_top planes at the top of z:
 *   W_k = w_max ((n_bottom - k)/n_bottom)^2 for k < n_bottom,
 *   W_k = w_max ((k - (nz-1-n_top))/n_top)^2 for k >= nz - n_top. */
tdse_status tdse_set_cap_quadratic(tdse_handle h, int64_t n_bottom, int64_t n_top, double w_max);

/* The CAP as eq. (10) prints it, one-sided at the bottom of the domain:
 * W_k = (alpha / dz) (r_cut - k dz)^2 for k dz < r_cut, else 0 (rates in
 * energy units, applied as in tdse_set_cap).  The paper's constant is
 * garbled (alpha = 1e8 eV with an electron charge, and r_cut = 0, which
 * would leave the region empty; section 2.3 instead appends 100 planes at
 * the bottom for the CAP); here alpha is energy per length and r_cut a
 * length, both >= 0, so r_cut = 100 dz over an appended region of 100
 * planes reproduces the paper's set-up.  TDSE_ERR_ARG for negative or
 * non-finite values. */
tdse_status tdse_set_cap_paper(tdse_handle h, double alpha, double r_cut);

/* The time step eq. (11) recommends, dt = m min(dx, dy, dz)^2 / (5 hbar),
 * for d's spacings and units (host only).  It exceeds the Gershgorin
 * bound hbar / E_max that tdse_finalize_setup enforces (by 1.2x on a cubic
 * grid with V = 0, more with a deep V) while staying inside the exact
 * leapfrog limit 2 hbar / max|E| when V is shallow: to run with it, pass it
 * as d->dt with TDSE_FLAG_ALLOW_UNSTABLE. */
tdse_status tdse_time_step_paper(const tdse_desc* d, double* dt);

/* Reduce min/max of V on the device, form E_max and dt, and build the
 * per-plane coefficient tables.  Synchronises.  Returns TDSE_ERR_UNSTABLE
 * if an absolute dt exceeds hbar / E_max and TDSE_FLAG_ALLOW_UNSTABLE is
 * not set, TDSE_ERR_NONFINITE if V holds NaN or Inf.  Outputs may be NULL. */
tdse_status tdse_finalize_setup(tdse_handle h, double* dt_out, double* e_max_out);

/* Write the packet of eqs. (3)-(4) into the bound state, with k0 the wave
 * vector (eq. (3) has k0 = -2 pi / lambda along z, eq. (4) for lambda) and
 * sigma the amplitude width.  The periodic images |m| <= 2 are summed
 * along periodic axes, and the state is scaled so dV sum |psi(r,0)|^2 = 1.
 * TDSE_INIT_HALFSTEP: psiI^{-1/2} = Im psi(r, -dt/2) of the free-particle
 * closed form; TDSE_INIT_NAIVE: psiI^{-1/2} = Im psi(r, 0).  Resets the
 * step counter, the flux and the records, and writes record 0.  Requires
 * tdse_finalize_setup. */
tdse_status tdse_init_gaussian(tdse_handle h, const double r0[3], const double k0[3],
                               double sigma, int32_t mode);

/* Load a state (device pointers in the handle's precision, copied into the
 * bound arrays unless they are the same) at global step `step`.  step == 0
 * resets the flux and records and writes record 0.  step > 0 resumes: the
 * records of earlier levels are taken to be in the bound buffers already
 * and the flux accumulator is set to flux_acc. */
tdse_status tdse_set_state(tdse_handle h, const void* psi_r, const void* psi_i, int64_t step,
                           double flux_acc);

/* Copy the state into caller device buffers (either may be NULL) and return
 * the step counter and flux accumulator (either may be NULL).  Synchronises. */
tdse_status tdse_get_state(tdse_handle h, void* psi_r, void* psi_i, int64_t* step,
                           double* flux_acc);

/* Advance n >= 0 steps (eq. (9) then eq. (8) per step) with the records,
 * sums and flux fused in.  Asynchronous.  Returns TDSE_ERR_CAPACITY before
 * launching anything if the records would overflow. */
tdse_status tdse_step(tdse_handle h, int64_t n);

/* Synchronise and report the counters and the caller's record buffers.
 * Returns TDSE_ERR_NONFINITE if the flux or any record scalar is not
 * finite. */
tdse_status tdse_detect(tdse_handle h, tdse_detect_out* out);

/* Copy the first n rows of the record scalars [n][4] to host memory.
 * Synchronises. */
tdse_status tdse_copy_scalars(tdse_handle h, double* host, int64_t n);

/* Second state pair for the one-pass step: psi_r2, psi_i2 as psi_r, psi_i
 * (caller-owned, 256-byte aligned, distinct from every other bound array).
 * The one-pass step fuses eq. (9) and eq. (8) into one sweep that reads
 * (psiR^n, psiI^{n-1/2}, V) and writes (psiR^{n+1}, psiI^{n+1/2}) into the
 * other pair, 20 B per cell-step in FP32 instead of 32.  Steps run in pairs
 * so that after every tdse_step call the state is back in the buffers bound
 * by tdse_bind; an odd step runs as the two in-place half-steps.  Binding
 * enables the one-pass step when the grid fits it (tdse_tile.fused). */
tdse_status tdse_bind_pingpong(tdse_handle h, void* psi_r2, void* psi_i2);

/* Reverse-mode gradient of a loss of the detection records (eq. (15))
 * through the leapfrog of eqs. (8)-(9) with the CAP.
 *
 * tdse_adjoint_workspace_size: bytes of the adjoint workspace for a forward
 * run of n_steps steps with checkpoints every ckpt_every steps: 2 ceil(N/K)
 * checkpoint arrays, 4 (K + 1) segment arrays (two banks: one segment is
 * recomputed while the next is swept) and 5 work arrays, each
 * [nz][ny][nx] in the state precision (host only).
 *
 * tdse_bind_adjoint: attach that caller-owned device workspace (256-byte
 * aligned; NULL detaches) to a handle whose state is at level 0.  The next
 * n_steps steps store (psiR, psiI) of levels 0, K, 2K, ... as checkpoints.
 *
 * tdse_adjoint: after exactly n_steps steps, form
 *   dL_dV  (device, double [nz][ny][nx])       dL/dV
 *   dL_dR0 (device, state precision, nullable) dL/dpsiR^0
 *   dL_dI0 (device, state precision, nullable) dL/dpsiI^{-1/2}
 * from dL_drho (device, state precision, [n_rec][ny][nx], the derivative of
 * the loss with respect to each record, n_rec = n_steps/h + 1).  Each
 * segment between checkpoints is recomputed forward (bit-identical to the
 * forward run; on a second stream of the handle's device, created at the
 * first call, overlapping the backward sweep of the segment after it) and
 * then swept backwards:
 *   i_t = i + G (B r);  dL/dV += cv (B r) o psiI^{n+1/2} - cv (B i_t) o psiR^n;
 *   r <- A r - G (B i_t);  i <- A i_t;  then record injections of level n,
 * G X = -(cx dxx + cy dyy + cz dzz) X + cv V X, A = diag(ca_k),
 * B = diag(cb_k).  In FP32 dL/dV is summed per segment in FP32 and folded
 * into FP64.  The handle's state is left at level n_steps.  Synchronises.
 * TDSE_ERR_UNSUPPORTED where nx has no layout over 64 lanes and the
 * one-pass reverse step does not fit either (no tdse_bind_pingpong, or
 * whole rows beyond 256 vectors). */
tdse_status tdse_adjoint_workspace_size(const tdse_desc* d, int64_t n_steps, int32_t ckpt_every,
                                        size_t* bytes);
tdse_status tdse_bind_adjoint(tdse_handle h, void* adj_ws, size_t bytes, int64_t n_steps,
                              int32_t ckpt_every);
tdse_status tdse_adjoint(tdse_handle h, const void* dL_drho, double* dL_dV, void* dL_dR0,
                         void* dL_dI0);

/* Chain rule from dL/dV (device, double [nz][ny][nx]) to the atoms of
 * tdse_build_potential (host [n]):
 *   dL_dpos[a][0..2] = sum_r dL/dV(r) (-amp_a v'(d) u/d),
 *   dL_damp[a]       = sum_r dL/dV(r) v(d),
 * u = r - X_a (minimum image), d = |u| < cutoff; a grid point exactly on an
 * atom adds nothing to dL_dpos (the screened potential has a cusp there).
 * Outputs are host memory.  Allocates and frees a small temporary;
 * synchronises. */
tdse_status tdse_potential_vjp(tdse_handle h, const tdse_atom* atoms, int64_t n,
                               const tdse_pot_params* p, const double* dL_dV, double* dL_dpos,
                               double* dL_damp);

/* Batches: many grids of uneven size stepped together, one launch per step
 * for all of them, the steps of one record interval captured in a HIP graph
 * that is replayed (the data-generation use of section 3.2: many
 * configurations, the same detection schedule).
 *
 * tdse_batch_create: one member handle per description (all with the same
 * precision and record_every h, h even and <= 256; h = 0 runs intervals
 * of 64 steps), all launching on `stream`, which must not be the null stream
 * (graphs are captured on it).  Host memory only.
 * tdse_batch_member: the i-th handle, set up with the single-grid calls
 * (tdse_bind, tdse_bind_pingpong (required), potential, CAP, finalize,
 * initial state); its outputs are read with tdse_detect as usual.
 * tdse_batch_set_tile: one-pass tile shared by the members (fused_rows 2, 3,
 * 4 or 6; fused_zc >= 1; prefetch flag; threads per workgroup 64, 128 or
 * 256); invalidates a prepared batch.
 * tdse_batch_workspace_size / tdse_batch_bind_workspace: the device memory
 * of the batch's tables (per-member kernel and finalisation arguments,
 * workgroup starts, the record counter: about 1 KB per member), owned by
 * the caller, 256-byte aligned, bound before tdse_batch_prepare and valid
 * until the batch is destroyed or another workspace is bound (NULL
 * unbinds; binding drops a prepared graph).  TDSE_ERR_ARG for a short or
 * misaligned workspace.
 * tdse_batch_prepare: all members at the same record level; writes the
 * tables into the bound workspace (TDSE_ERR_STATE without one) and captures
 * the graph of one interval; allocates no device memory.
 * tdse_batch_run: n steps, a multiple of the interval; asynchronous.
 * tdse_batch_status: synchronise; per_config[i] = tdse_detect's status of
 * member i (TDSE_ERR_NONFINITE flags a configuration whose sums went
 * non-finite while the others finish); returns the first failure.
 * tdse_batch_destroy: frees the tables, graph and member handles. */
typedef struct tdse_batch_ctx* tdse_batch;

tdse_status tdse_batch_create(const tdse_desc* descs, int32_t n, void* stream, tdse_batch* out);
tdse_status tdse_batch_member(tdse_batch b, int32_t i, tdse_handle* h);
/* tdse_batch_bind: tdse_bind and tdse_bind_pingpong of member i in one call
 * (the same arguments, rules and errors; psi_r2, psi_i2 the member's second
 * state pair, which a batch requires); drops a prepared graph.
 * tdse_batch_detect: tdse_detect of member i. */
tdse_status tdse_batch_bind(tdse_batch b, int32_t i, void* psi_r, void* psi_i, void* v, void* workspace,
                            size_t workspace_bytes, void* records, double* scalars, double* pixel,
                            void* psi_r2, void* psi_i2);
tdse_status tdse_batch_detect(tdse_batch b, int32_t i, tdse_detect_out* out);
tdse_status tdse_batch_set_tile(tdse_batch b, int32_t fused_rows, int32_t fused_zc,
                                int32_t prefetch, int32_t threads);
/* Two-step sweeps for the whole batch (on by default, with tx 80, one row,
 * z chunk 32, prefetch, 1024 threads): when every member
 * fits the sweep's tile (interior width at most tx, rows per thread, z
 * chunk zc, prefetch and threads per workgroup as for tdse_tile) and the
 * members share the vector width; each member takes the interior width
 * (tx or a multiple of 8 below it) and height that cover its plane with the
 * fewest tiles, then with the fewest cells swept,
 * tdse_batch_prepare captures intervals of S/2 two-step launches instead of
 * S one-pass launches; otherwise it falls back to the one-pass form.  When
 * S/2 is odd a second graph covers intervals that start from the second
 * state pair, and a run that ends there copies the members' state back
 * into their bound arrays. */
tdse_status tdse_batch_set_two_step(tdse_batch b, int32_t enable, int32_t tx, int32_t rows,
                                    int32_t zc, int32_t prefetch, int32_t threads);
tdse_status tdse_batch_workspace_size(tdse_batch b, size_t* bytes);
tdse_status tdse_batch_bind_workspace(tdse_batch b, void* workspace, size_t bytes);
tdse_status tdse_batch_prepare(tdse_batch b);
tdse_status tdse_batch_run(tdse_batch b, int64_t n);
tdse_status tdse_batch_status(tdse_batch b, int32_t* per_config);
const char* tdse_batch_last_error(tdse_batch b);
tdse_status tdse_batch_destroy(tdse_batch b);

/* Kernel timing for measurement: when enabled, each step kernel launch is
 * bracketed by HIP events on the handle's stream.  tdse_timing_read
 * synchronises and returns, per kernel kind (0: eq. (9) half-step, 1: eq. (8)
 * half-step, 2: one-pass step, 3: two-step sweep), the summed kernel
 * milliseconds ms[4] and launch counts count[4] since the last read, and
 * clears them. */
tdse_status tdse_set_timing(tdse_handle h, int32_t enable);
tdse_status tdse_timing_read(tdse_handle h, double* ms, int64_t* count);
/* The same with the launches that write a detection record (eq. (15))
 * kept apart: ms[8], count[8], kinds 0-3 as above for launches without a
 * record, 4 + kind for those with one (the eq. (8) half-step, one-pass step
 * or two-step sweep whose last level is recorded).  Synchronises; clears. */
tdse_status tdse_timing_read_split(tdse_handle h, double* ms, int64_t* count);

/* Trajectory dissimilarity, eq. (16) (section 3.2): for trajectories k, j
 * the time average over [t0, t1] of the L2 distance between their
 * detector-plane densities,
 *   out[k][j] = sum_t w[t] sqrt(dA sum_p (frames[k][t][p] - frames[j][t][p])^2),
 * the time integral as a quadrature over the frames with weights w (which
 * carry the 1 / (t1 - t0)), the plane integral as dA (pixel area) times the
 * pixel sum.  frames: device, [K][T][P] in precision (TDSE_F32 or
 * TDSE_F64), the trajectories on a common detector grid and common frame
 * times (records of configurations with equal grids and time steps);
 * weights: device double [T]; out: device double [K][K] (symmetric, zero
 * diagonal); workspace: device, >= tdse_dissimilarity_workspace_size bytes.
 * All caller-owned.  FP64 frames: the sums are formed from the
 * differences on the vector ALU.  FP32 frames: on the FP64 matrix cores as
 * |x_k|^2 + |x_j|^2 - 2 x_k . x_j with x = frame - (the frame of trajectory
 * 0 at the same time), exact in FP64 (the shift leaves every distance
 * unchanged).  The expansion's rounding error in a frame's d^2 is below
 * about 0.4 P eps64 (|x_k|^2 + |x_j|^2); a pair with a frame whose d^2 is
 * below P 2^-30 (|x_k|^2 + |x_j|^2) (pairs much closer to each other than
 * to trajectory 0) is evaluated again in the direct form, from the
 * differences, for all its frames; so every d^2 the result uses is good to
 * about 5e-8 of itself, and identical trajectories are at distance 0.  The
 * result is bitwise reproducible and exactly symmetric.  Workspace: the
 * partial sums, and for FP32 frames the list of such pairs (room for all K
 * (K - 1) / 2).  Asynchronous on stream (a hipStream_t, may be null).
 * TDSE_ERR_ARG for null pointers, sizes < 1, dA <= 0 or a short workspace;
 * TDSE_ERR_DEVICE for launch errors. */
tdse_status tdse_dissimilarity_workspace_size(int32_t K, int32_t T, size_t* bytes);
tdse_status tdse_dissimilarity(int32_t precision, const void* frames, int32_t K, int32_t T, int64_t P,
                               const double* weights, double dA, double* out, void* workspace,
                               size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and launches as tdse_dissimilarity, with the partial sums in
 * a fixed device array inside the library instead of a caller workspace.
 * The array holds TDSE_DISSIM_NOALLOC_MAX_BYTES on every GPU the library
 * runs on, from the load of its code object until the process ends; the
 * first call on a device looks up its address there (hipGetSymbolAddress),
 * later calls reuse it.  No call allocates or frees anything.  Arguments
 * as tdse_dissimilarity without the workspace; the kernels run on the
 * current device, on stream (a hipStream_t of that device, may be null);
 * the result is bitwise that of tdse_dissimilarity.  Every call on one GPU
 * shares its array and leaves its partial sums there (each call writes
 * every entry it reads, so nothing needs clearing): calls whose executions
 * can overlap on one GPU (unordered streams, host threads) race and give
 * wrong results; calls on one stream are ordered.  TDSE_ERR_CAPACITY when
 * the precision's workspace would exceed the maximum, checked before
 * anything is launched: ceil(T / frames per chunk) x K x K doubles of
 * partial sums, and for FP32 frames the pair list, at most
 * tdse_dissimilarity_workspace_size(K, T) (FP32 frames of K = 879
 * trajectories x T = 77 frames need 56 MiB and fit; FP64 frames of that
 * size need 118 MiB and do not).  Other errors as tdse_dissimilarity;
 * TDSE_ERR_UNSUPPORTED on a device index >= 64. */
#define TDSE_DISSIM_NOALLOC_MAX_BYTES (64u << 20)
tdse_status tdse_dissimilarity_noalloc(int32_t precision, const void* frames, int32_t K, int32_t T,
                                       int64_t P, const double* weights, double dA, double* out,
                                       void* stream);

/* HBM probe: the practical bandwidth ceiling of this device, measured by
 * streaming kernels that do no part of the method.  kind 0: a copy, bufs[0]
 * -> bufs[1]; kind 1: the one-pass step's mix, three read streams bufs[0..2]
 * and two written streams bufs[3..4] (d = a + b c, e = b - a c, elementwise);
 * kind 2: a write-only stream, bufs[0] filled with 1.0f.
 * Each buffer is n floats (n a multiple of 4) of device memory, 16-byte
 * aligned, all distinct, owned by the caller; the written buffers are
 * overwritten.  All accesses carry the non-temporal hint.  grid = workgroups
 * of 256 threads in a grid-stride loop (0: one 16-byte vector per thread,
 * the fastest form measured).  Runs one warm-up
 * pass and reps timed passes on stream (a hipStream_t, may be null),
 * synchronises it and returns the average milliseconds per pass in
 * *ms_per_pass.  TDSE_ERR_ARG for bad arguments, TDSE_ERR_DEVICE for HIP
 * errors. */
tdse_status tdse_hbm_probe(int32_t kind, void* const* bufs, int64_t n, int32_t grid, int32_t reps,
                           void* stream, double* ms_per_pass);

/* Tile shapes.  Two-pass half-step kernels: rows = y rows per wavefront (1,
 * 2, 4 or 8), waves = wavefronts per workgroup (1..4), zc = z planes per
 * workgroup.  One-pass kernel: fused != 0 selects it (needs
 * tdse_bind_pingpong), fused_rows = rows per thread (2, 3, 4 or 6),
 * fused_threads = threads per workgroup (64, 128 or 256), so the band is
 * band_rows = (fused_threads / threads per row) * fused_rows - 2 rows;
 * fused_zc = z planes per workgroup, fused_prefetch != 0 issues the next
 * plane's loads before the current plane's eq. (8) part.  graph != 0
 * (default) lets tdse_step replay a captured HIP graph for whole record
 * intervals of one-pass steps when the handle's stream is not the null
 * stream, timing is off, no adjoint is bound and the two-step sweep is off
 * (h even, <= 256).
 *
 * Two-step sweep (temporal blocking: eqs. (9), (8), (9), (8) in one pass,
 * 20 B per cell per two steps in FP32): two_step != 0 selects it on top of
 * the one-pass kernel (which still takes single steps: a step whose level
 * is recorded first, an odd last step, the level before an adjoint
 * checkpoint).  two_step_tx = interior tile width (a multiple of the vector
 * width, >= 8), two_step_threads = threads per workgroup (256, 512 or 1024),
 * two_step_rows = rows per thread (2 or 3 with 256 threads, 1 or 2 with
 * 512, 1 with 1024), so the interior tile height is at most (threads /
 * ((tx + 8) / vector width)) * rows - 8; two_step_ty > 0 asks for a
 * shorter tile (rounded up to whole rows per pass; the threads past the
 * last row idle), 0 for the tallest, and tdse_get_tile returns the height
 * in use; two_step_zc = z planes per workgroup, two_step_prefetch != 0
 * loads the next plane's inputs one iteration ahead.  The sweep needs at most ny tiles per plane
 * and its LDS ((2 x 4) buffers of (ty + 10) x (tx + 8) values, plus 8 bytes
 * per wavefront) within the device's per-workgroup limit.  TDSE_ERR_ARG for
 * a thread count other than 256, 512 or 1024; TDSE_ERR_UNSUPPORTED for a
 * (rows, threads) pair without a kernel or a tile that does not fit.
 *
 * tdse_create picks defaults; tdse_set_tile checks and replaces them.
 * vec_elems, vec_groups, lanes and band_rows are read-only (and
 * two_step_ty as described above); vec_groups and lanes are 0 where nx has
 * no layout over 64 lanes (the any-width half-step kernel runs).  fused != 0
 * with a one-pass band that does not fit (whole x rows in LDS: nx / W <=
 * fused_threads) is accepted together with two_step: the sweep then takes
 * the step pairs and half-steps the single steps. */
typedef struct tdse_tile {
    int32_t rows, waves, zc;
    int32_t fused, fused_rows, fused_zc, fused_prefetch, graph, fused_threads;
    int32_t two_step, two_step_tx, two_step_rows, two_step_zc, two_step_prefetch, two_step_threads;
    int32_t vec_elems, vec_groups, lanes, band_rows, two_step_ty;
} tdse_tile;

tdse_status tdse_get_tile(tdse_handle h, tdse_tile* out);

/* Tile autotuner: times a built-in list of candidate tiles on the handle's
 * own grid and state (flags: bit 0 two-pass, bit 1 one-pass, bit 2 two-step
 * sweep; none of the three = all; the one-pass and two-step candidates need
 * tdse_bind_pingpong; the two-step list includes, for a few tile widths,
 * the tile height and z chunk whose workgroups fill one round of the
 * compute units most fully), each for 2 warm-up and `steps` timed steps with HIP
 * events on the handle's stream, without records; keeps the fastest, sets
 * it and returns it in *out.  The state is spent: afterwards the handle
 * needs tdse_init_gaussian or tdse_set_state before tdse_step
 * (TDSE_ERR_STATE until then).  TDSE_ERR_STATE without a state, with
 * pending sums or with an adjoint bound; TDSE_ERR_ARG for unknown flag bits.
 *
 * Cache: when the environment variable TDSE_TUNE_CACHE names a file, the
 * tuner first looks there for this case (extents, precision, boundaries,
 * candidate families, ping-pong pair bound or not, compute units and
 * device architecture); on a hit it sets that tile, runs nothing and keeps
 * the state.  Otherwise (or with TDSE_TUNE_REFRESH in flags) it times the
 * candidates and writes the winner into the file (one text line per case,
 * the file rewritten through a temporary and a rename; TDSE_ERR_ARG if it
 * cannot be written). */
#define TDSE_TUNE_REFRESH 8
tdse_status tdse_autotune(tdse_handle h, int32_t steps, int32_t flags, tdse_tile* out);
tdse_status tdse_set_tile(tdse_handle h, const tdse_tile* t);

/* The GPU design of section 2.2 as a baseline: n leapfrog steps (eq. (9),
 * then eq. (8), each a launch that updates its array in place) on arrays
 * stored z fastest and x slowest, [nx][ny][nz], with one thread per grid
 * point in blocks of bx x by x bz points (bx along z, by along x, bz along
 * y) laid out on a two-dimensional grid by eq. (12), every neighbour read
 * from global memory and periodic neighbours taken modulo N (eqs.
 * (13)-(14)).  Grid, boundaries, coefficients and CAP tables are the
 * handle's (tdse_finalize_setup first); psi_r, psi_i and v are device
 * arrays of the handle's precision owned by the caller, distinct from each
 * other; psi_r and psi_i are overwritten.  The cell arithmetic is the
 * library's, so the result is bitwise the transpose of n tdse_step steps
 * from the transposed state.  No records, sums or step count: the handle's
 * own state is not touched.  Asynchronous on the handle's stream.
 * TDSE_ERR_ARG for null or aliased arrays, n < 0 or a block of more than
 * 1024 threads; TDSE_ERR_STATE before finalize; TDSE_ERR_UNSUPPORTED when
 * the block grid exceeds the device's grid dimensions. */
tdse_status tdse_paper_layout_run(tdse_handle h, void* psi_r, void* psi_i, const void* v, int64_t n,
                                  int32_t bx, int32_t by, int32_t bz);

#ifdef __cplusplus
}
#endif

#endif /* TDSE_H */
