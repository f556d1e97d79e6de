/*
 * FP64 CPU oracle for the FDTD leapfrog of the 3D time-dependent
 * Schrodinger equation (Nagaya, Omatsu, Packwood, arXiv 2401.07416).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the HIP path, and it never
 * reads anything the HIP path produced.
 *
 * Everything is double precision, round-to-nearest, compiled without FP
 * contraction.  Loops run k -> j -> i over the x-fastest layout
 * idx = (k*ny + j)*nx + i.  Sums are formed per z-plane in (j, i) order and the
 * plane sums are then added in k order, so every result is independent of
 * the OpenMP thread count.
 *
 * Readings of the paper used here (the paper is silent or garbled on them):
 *  - state at level n is (psiR^n, psiI^{n-1/2}); one step applies eq. (9)
 *    (imaginary half-step) and then eq. (8) (real half-step);
 *  - the complex absorbing potential of eq. (10) is a per-plane rate W_k >= 0
 *    applied time-centred: gamma_k = W_k dt/hbar,
 *    ca_k = (1 - gamma_k/2)/(1 + gamma_k/2), cb_k = 1/(1 + gamma_k/2);
 *    with W = 0 the update is exactly eqs. (8)-(9);
 *  - the density at level n is psiR^n^2 + psiI^{n-1/2}^2 (section 2.1, after
 *    eqs. (8)-(9)); the detection plane of eq. (15) stores it every h steps,
 *    starting with n = 0;
 *  - grid points sit at r = (i dx, j dy, k dz) (section 2.1), periodic wrap
 *    (i +- 1) mod N as in eqs. (13)-(14); a per-axis zero (Dirichlet)
 *    boundary is also offered;
 *  - the time step bound uses a Gershgorin estimate of the largest
 *    |eigenvalue| of the discrete Hamiltonian (the CAP excluded);
 *  - the conserved quadratic form of the leapfrog and the discrete
 *    probability current through the detection face are not in the paper;
 *    they are the scheme's own exact invariants (see og_step).
 */
#include <complex.h>
#undef I /* the imaginary unit is written _Complex_I below */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OG_PERIODIC 0
#define OG_ZERO 1

#define OG_INIT_HALFSTEP 0
#define OG_INIT_NAIVE 1

typedef struct {
    int64_t nx, ny, nz;
    double dx, dy, dz;
    double hbar, mass;
    int32_t bc[3];
    int32_t pad_;
} og_grid;

/* Simulation state.  Every array is owned by the caller. */
typedef struct {
    og_grid g;
    double dt;
    double cx, cy, cz, cv;     /* section 2.1, definitions after eq. (9) */
    const double* ca;          /* [nz] CAP damping, time-centred */
    const double* cb;          /* [nz] */
    double* psiR;              /* [nz][ny][nx], level n */
    double* psiI;              /* [nz][ny][nx], level n - 1/2 */
    const double* V;           /* [nz][ny][nx] */
    int64_t k_det;             /* detection plane index (eq. (15)) */
    int64_t h;                 /* record every h steps (eq. (15)) */
    int64_t step;              /* global step counter n */
    double flux_acc;           /* accumulated flux through face k_det + 1/2 */
    double* rec_rho;           /* [max_rec][ny][nx] */
    double* rec_scalars;       /* [max_rec][4]: plane_sum, naive_norm, Q, flux_acc */
    int64_t max_rec;
    int64_t n_rec;
    double* pixel;             /* [ny][nx] time-integrated intensity, or NULL */
    double* scratch_cell;      /* [nz][ny][nx] copy of psiR^n (record steps) */
    double* plane_buf;         /* [nz] per-plane partial sums */
} og_sim;

int og_abi_version(void) { return 3; }

void og_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int og_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static inline int64_t og_idx(const og_grid* g, int64_t i, int64_t j, int64_t k) {
    return (k * g->ny + j) * g->nx + i;
}

/* Value of array a at (i, j, k) where each index may be one step outside the
 * grid; periodic wrap as in eqs. (13)-(14), or zero outside for OG_ZERO. */
static inline double og_at(const og_grid* g, const double* a, int64_t i, int64_t j, int64_t k) {
    if (i < 0 || i >= g->nx) {
        if (g->bc[0] == OG_ZERO) return 0.0;
        i = (i + g->nx) % g->nx;
    }
    if (j < 0 || j >= g->ny) {
        if (g->bc[1] == OG_ZERO) return 0.0;
        j = (j + g->ny) % g->ny;
    }
    if (k < 0 || k >= g->nz) {
        if (g->bc[2] == OG_ZERO) return 0.0;
        k = (k + g->nz) % g->nz;
    }
    return a[og_idx(g, i, j, k)];
}

/* The three second-difference terms of eqs. (8)-(9) applied to array a:
 *   cx (a(i+1) - 2a(i) + a(i-1)) + cy (...) + cz (...)                      */
static inline double og_laplace_terms(const og_sim* s, const double* a, int64_t i, int64_t j,
                                      int64_t k) {
    const og_grid* g = &s->g;
    double c = a[og_idx(g, i, j, k)];
    double tx = og_at(g, a, i + 1, j, k) - 2.0 * c + og_at(g, a, i - 1, j, k);
    double ty = og_at(g, a, i, j + 1, k) - 2.0 * c + og_at(g, a, i, j - 1, k);
    double tz = og_at(g, a, i, j, k + 1) - 2.0 * c + og_at(g, a, i, j, k - 1);
    return s->cx * tx + s->cy * ty + s->cz * tz;
}

/* ---------------------------------------------------------------------- */
/* Coefficients and time step                                              */
/* ---------------------------------------------------------------------- */

/* Gershgorin bound on max |E| of the discrete Hamiltonian
 *   H = -(hbar^2/2m) (second differences) + V
 * Each axis adds (hbar^2/2m) * 4/d^2 to the upper bound (diagonal 2/d^2 plus
 * two off-diagonal 1/d^2), except a periodic axis of length 1 whose second
 * difference vanishes identically.  The CAP is excluded. */
double og_emax(const og_grid* g, const double* V) {
    int64_t n = g->nx * g->ny * g->nz;
    double vmin = V[0], vmax = V[0];
    for (int64_t c = 1; c < n; ++c) {
        if (V[c] < vmin) vmin = V[c];
        if (V[c] > vmax) vmax = V[c];
    }
    double kin = 0.0;
    const int64_t nd[3] = {g->nx, g->ny, g->nz};
    const double dd[3] = {g->dx, g->dy, g->dz};
    for (int d = 0; d < 3; ++d) {
        if (nd[d] == 1 && g->bc[d] == OG_PERIODIC) continue;
        kin += 4.0 / (dd[d] * dd[d]);
    }
    kin *= g->hbar * g->hbar / (2.0 * g->mass);
    double lo = fabs(vmin);
    double hi = fabs(vmax + kin);
    return lo > hi ? lo : hi;
}

/* Update coefficients of section 2.1 (after eq. (9)) and the per-plane CAP
 * factors.  c4 = {cx, cy, cz, cv}.  W may be NULL (no CAP). */
void og_coeffs(const og_grid* g, double dt, const double* W, double* c4, double* ca, double* cb) {
    c4[0] = g->hbar * dt / (2.0 * g->mass * g->dx * g->dx);
    c4[1] = g->hbar * dt / (2.0 * g->mass * g->dy * g->dy);
    c4[2] = g->hbar * dt / (2.0 * g->mass * g->dz * g->dz);
    c4[3] = dt / g->hbar;
    for (int64_t k = 0; k < g->nz; ++k) {
        double w = W ? W[k] : 0.0;
        double gam = w * dt / g->hbar;
        ca[k] = (1.0 - 0.5 * gam) / (1.0 + 0.5 * gam);
        cb[k] = 1.0 / (1.0 + 0.5 * gam);
    }
}

/* Quadratic CAP ramp (the shape of eq. (10)) over nbot planes at the bottom
 * and ntop planes at the top of the z axis:
 *   bottom k = 0..nbot-1:           W_k = wmax ((nbot - k)/nbot)^2
 *   top    k = nz-ntop..nz-1:       W_k = wmax ((k - (nz-1-ntop))/ntop)^2 */
void og_cap_quadratic(int64_t nz, int64_t nbot, int64_t ntop, double wmax, double* W) {
    for (int64_t k = 0; k < nz; ++k) W[k] = 0.0;
    for (int64_t k = 0; k < nbot && k < nz; ++k) {
        double d = (double)(nbot - k) / (double)nbot;
        W[k] += wmax * d * d;
    }
    for (int64_t k = nz - ntop; k < nz; ++k) {
        if (k < 0) continue;
        double d = (double)(k - (nz - 1 - ntop)) / (double)ntop;
        W[k] += wmax * d * d;
    }
}

/* ---------------------------------------------------------------------- */
/* Potential: screened softened Coulomb atoms                              */
/* ---------------------------------------------------------------------- */

/* Radial atomic potential and its derivative:
 *   v_Z(d)  = -Z kappa exp(-d/lam) / sqrt(d^2 + s^2)
 *   v_Z'(d) = v_Z(d) (-1/lam - d/(d^2 + s^2))
 * lam = 0.8853 a0 Z^(-1/3) (Thomas-Fermi) when screened, else infinite. */
static double og_lambda(double Z, double a0, int screened) {
    return screened ? 0.8853 * a0 * pow(Z, -1.0 / 3.0) : INFINITY;
}

double og_vatom(double d, double Z, double soft, double kappa, double a0, int screened) {
    double lam = og_lambda(Z, a0, screened);
    double e = screened ? exp(-d / lam) : 1.0;
    return -Z * kappa * e / sqrt(d * d + soft * soft);
}

double og_dvatom(double d, double Z, double soft, double kappa, double a0, int screened) {
    double lam = og_lambda(Z, a0, screened);
    double v = og_vatom(d, Z, soft, kappa, a0, screened);
    double inv_lam = screened ? 1.0 / lam : 0.0;
    return v * (-inv_lam - d / (d * d + soft * soft));
}

/* Minimum-image displacement along a periodic axis of length L. */
static double og_min_image(double u, double L) {
    return u - L * nearbyint(u / L);
}

/* V(r) = sum_a amp_a v_{Z_a}(|r - X_a|) over atoms within the cutoff, in
 * atom order, evaluated on a window of the grid: window cell (ii, jj, kk)
 * is grid point ((i0+ii) mod nx, (j0+jj) mod ny, (k0+kk) mod nz) and out is
 * [wnz][wny][wnx].  atoms is [n][5] = {x, y, z, Z, amp}.  Minimum image
 * along periodic axes.  Per plane, atoms whose z distance alone reaches the
 * cutoff are dropped, and per row those whose y distance does; they could
 * not contribute, so the sum and its order are those of the plain
 * definition. */
void og_potential_window(const og_grid* g, const double* atoms, int64_t n, double soft,
                         double cutoff, double kappa, double a0, int screened, int64_t i0,
                         int64_t j0, int64_t k0, int64_t wnx, int64_t wny, int64_t wnz,
                         double* out) {
    const double L[3] = {g->nx * g->dx, g->ny * g->dy, g->nz * g->dz};
#pragma omp parallel for schedule(dynamic)
    for (int64_t kk = 0; kk < wnz; ++kk) {
        const int64_t k = ((k0 + kk) % g->nz + g->nz) % g->nz;
        const double rz = k * g->dz;
        int64_t* cand = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
        int64_t* rowc = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
        int64_t nc = 0;
        for (int64_t a = 0; a < n; ++a) {
            double uz = rz - atoms[5 * a + 2];
            if (g->bc[2] == OG_PERIODIC) uz = og_min_image(uz, L[2]);
            if (fabs(uz) < cutoff) cand[nc++] = a;
        }
        for (int64_t jj = 0; jj < wny; ++jj) {
            const int64_t j = ((j0 + jj) % g->ny + g->ny) % g->ny;
            const double ry = j * g->dy;
            int64_t nr = 0;
            for (int64_t c = 0; c < nc; ++c) {
                double uy = ry - atoms[5 * cand[c] + 1];
                if (g->bc[1] == OG_PERIODIC) uy = og_min_image(uy, L[1]);
                if (fabs(uy) < cutoff) rowc[nr++] = cand[c];
            }
            for (int64_t ii = 0; ii < wnx; ++ii) {
                const int64_t i = ((i0 + ii) % g->nx + g->nx) % g->nx;
                const double r[3] = {i * g->dx, ry, rz};
                double v = 0.0;
                for (int64_t c = 0; c < nr; ++c) {
                    const double* at = atoms + 5 * rowc[c];
                    double u[3];
                    for (int d = 0; d < 3; ++d) {
                        u[d] = r[d] - at[d];
                        if (g->bc[d] == OG_PERIODIC) u[d] = og_min_image(u[d], L[d]);
                    }
                    double dist = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                    if (dist >= cutoff) continue;
                    v += at[4] * og_vatom(dist, at[3], soft, kappa, a0, screened);
                }
                out[(kk * wny + jj) * wnx + ii] = v;
            }
        }
        free(cand);
        free(rowc);
    }
}

void og_potential(const og_grid* g, const double* atoms, int64_t n, double soft, double cutoff,
                  double kappa, double a0, int screened, double* V) {
    og_potential_window(g, atoms, n, soft, cutoff, kappa, a0, screened, 0, 0, 0, g->nx, g->ny,
                        g->nz, V);
}

/* Same potential at an explicit list of points pts[m][3] (positions, not
 * necessarily grid points), looping over every atom. */
void og_potential_points(const og_grid* g, const double* atoms, int64_t n, double soft,
                         double cutoff, double kappa, double a0, int screened,
                         const double* pts, int64_t m, double* out) {
    const double L[3] = {g->nx * g->dx, g->ny * g->dy, g->nz * g->dz};
    for (int64_t p = 0; p < m; ++p) {
        double v = 0.0;
        for (int64_t a = 0; a < n; ++a) {
            const double* at = atoms + 5 * a;
            double u[3];
            for (int d = 0; d < 3; ++d) {
                u[d] = pts[3 * p + d] - at[d];
                if (g->bc[d] == OG_PERIODIC) u[d] = og_min_image(u[d], L[d]);
            }
            double dist = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            if (dist >= cutoff) continue;
            v += at[4] * og_vatom(dist, at[3], soft, kappa, a0, screened);
        }
        out[p] = v;
    }
}

/* ---------------------------------------------------------------------- */
/* Gaussian wave packet (eqs. (3)-(4))                                     */
/* ---------------------------------------------------------------------- */

/* Free-particle evolution of the 1D factor of eq. (3), with the continuum
 * normalisation (pi sigma^2)^(-1/4):
 *   phi(x,t) = (pi s^2)^(-1/4) (1 + i tau)^(-1/2)
 *              exp(-(x - x0 - v t)^2 / (2 s^2 (1 + i tau)) + i k (x - x0)
 *                  - i hbar k^2 t / (2m)),
 *   tau = hbar t/(m s^2), v = hbar k / m.                                  */
static double complex og_phi(double x, double x0, double k, double sigma, double t, double hbar,
                             double mass) {
    double tau = hbar * t / (mass * sigma * sigma);
    double v = hbar * k / mass;
    double complex one_itau = 1.0 + _Complex_I * tau;
    double u = x - x0 - v * t;
    double complex arg = -(u * u) / (2.0 * sigma * sigma * one_itau) + _Complex_I * k * (x - x0) -
                         _Complex_I * hbar * k * k * t / (2.0 * mass);
    return pow(M_PI * sigma * sigma, -0.25) / csqrt(one_itau) * cexp(arg);
}

/* Per-axis image sum (periodic axes) of phi. */
static double complex og_phi_axis(const og_grid* g, int d, double x, double x0, double k,
                                  double sigma, double t, int nimg) {
    const double L = d == 0 ? g->nx * g->dx : (d == 1 ? g->ny * g->dy : g->nz * g->dz);
    if (g->bc[d] != OG_PERIODIC) return og_phi(x, x0, k, sigma, t, g->hbar, g->mass);
    double complex s = 0.0;
    for (int m = -nimg; m <= nimg; ++m) s += og_phi(x + m * L, x0, k, sigma, t, g->hbar, g->mass);
    return s;
}

/* psi(r, t) on the grid: product of the three axis factors, each summed over
 * periodic images |m| <= nimg.  No discrete normalisation. */
void og_gaussian_closed(const og_grid* g, const double* r0, const double* k0, double sigma,
                        double t, int nimg, double* re, double* im) {
    double complex* fx = malloc(sizeof(double complex) * g->nx);
    double complex* fy = malloc(sizeof(double complex) * g->ny);
    double complex* fz = malloc(sizeof(double complex) * g->nz);
    for (int64_t i = 0; i < g->nx; ++i) fx[i] = og_phi_axis(g, 0, i * g->dx, r0[0], k0[0], sigma, t, nimg);
    for (int64_t j = 0; j < g->ny; ++j) fy[j] = og_phi_axis(g, 1, j * g->dy, r0[1], k0[1], sigma, t, nimg);
    for (int64_t k = 0; k < g->nz; ++k) fz[k] = og_phi_axis(g, 2, k * g->dz, r0[2], k0[2], sigma, t, nimg);
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                double complex p = fx[i] * fy[j] * fz[k];
                re[og_idx(g, i, j, k)] = creal(p);
                im[og_idx(g, i, j, k)] = cimag(p);
            }
    free(fx);
    free(fy);
    free(fz);
}

/* Initial state of the staggered scheme from the packet of eq. (3).
 * psiR^0 = s Re psi(r, 0).  HALFSTEP: psiI^{-1/2} = s Im psi(r, -dt/2);
 * NAIVE: psiI^{-1/2} = s Im psi(r, 0).  s makes dV sum |psi(r,0)|^2 = 1
 * (eq. (3)'s prefactor does not normalise a 3D packet, so the scale is set
 * discretely). */
void og_init_gaussian(const og_grid* g, const double* r0, const double* k0, double sigma, double dt,
                      int mode, int nimg, double* R, double* I) {
    int64_t n = g->nx * g->ny * g->nz;
    double* tmp = malloc(sizeof(double) * n);
    og_gaussian_closed(g, r0, k0, sigma, 0.0, nimg, R, tmp);
    double dV = g->dx * g->dy * g->dz;
    double tot = 0.0;
    for (int64_t k = 0; k < g->nz; ++k) {
        double ps = 0.0;
        for (int64_t c = k * g->nx * g->ny; c < (k + 1) * g->nx * g->ny; ++c)
            ps += R[c] * R[c] + tmp[c] * tmp[c];
        tot += ps;
    }
    double s = 1.0 / sqrt(dV * tot);
    if (mode == OG_INIT_HALFSTEP) {
        double* tmpr = malloc(sizeof(double) * n);
        og_gaussian_closed(g, r0, k0, sigma, -0.5 * dt, nimg, tmpr, I);
        free(tmpr);
    } else {
        memcpy(I, tmp, sizeof(double) * n);
    }
    for (int64_t c = 0; c < n; ++c) {
        R[c] *= s;
        I[c] *= s;
    }
    free(tmp);
}

/* The initial state of og_init_gaussian evaluated only on a window of the
 * grid (window cell (ii, jj, kk) is grid point ((i0+ii) mod nx, ...)), with
 * the normalisation s summed over the whole grid exactly as there.  Used to
 * check large grids on a few windows. */
void og_init_gaussian_window(const og_grid* g, const double* r0, const double* k0, double sigma,
                             double dt, int mode, int nimg, int64_t i0, int64_t j0, int64_t k0w,
                             int64_t wnx, int64_t wny, int64_t wnz, double* psiR0,
                             double* psiIh) {
    double complex* f0[3];
    double complex* fh[3];
    const int64_t nd[3] = {g->nx, g->ny, g->nz};
    const double dd[3] = {g->dx, g->dy, g->dz};
    const double th = mode == OG_INIT_HALFSTEP ? -0.5 * dt : 0.0;
    for (int d = 0; d < 3; ++d) {
        f0[d] = malloc(sizeof(double complex) * nd[d]);
        fh[d] = malloc(sizeof(double complex) * nd[d]);
        for (int64_t i = 0; i < nd[d]; ++i) {
            f0[d][i] = og_phi_axis(g, d, i * dd[d], r0[d], k0[d], sigma, 0.0, nimg);
            fh[d][i] = og_phi_axis(g, d, i * dd[d], r0[d], k0[d], sigma, th, nimg);
        }
    }
    double tot = 0.0;
    for (int64_t k = 0; k < g->nz; ++k) {
        double ps = 0.0;
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                double complex p = f0[0][i] * f0[1][j] * f0[2][k];
                ps += creal(p) * creal(p) + cimag(p) * cimag(p);
            }
        tot += ps;
    }
    const double s = 1.0 / sqrt(g->dx * g->dy * g->dz * tot);
    for (int64_t kk = 0; kk < wnz; ++kk) {
        const int64_t k = ((k0w + kk) % g->nz + g->nz) % g->nz;
        for (int64_t jj = 0; jj < wny; ++jj) {
            const int64_t j = ((j0 + jj) % g->ny + g->ny) % g->ny;
            for (int64_t ii = 0; ii < wnx; ++ii) {
                const int64_t i = ((i0 + ii) % g->nx + g->nx) % g->nx;
                const int64_t c = (kk * wny + jj) * wnx + ii;
                psiR0[c] = creal(f0[0][i] * f0[1][j] * f0[2][k]) * s;
                psiIh[c] = cimag(fh[0][i] * fh[1][j] * fh[2][k]) * s;
            }
        }
    }
    for (int d = 0; d < 3; ++d) {
        free(f0[d]);
        free(fh[d]);
    }
}

/* ---------------------------------------------------------------------- */
/* The leapfrog                                                            */
/* ---------------------------------------------------------------------- */

void og_sim_init(og_sim* s) {
    s->step = 0;
    s->flux_acc = 0.0;
    s->n_rec = 0;
}

static double og_sum_planes(const og_sim* s) {
    double t = 0.0;
    for (int64_t k = 0; k < s->g.nz; ++k) t += s->plane_buf[k];
    return t;
}

/* Eq. (9) with the CAP, at one cell: returns psiI^{n+1/2}. */
static inline double og_new_I(const og_sim* s, int64_t i, int64_t j, int64_t k) {
    int64_t c = og_idx(&s->g, i, j, k);
    double lap = og_laplace_terms(s, s->psiR, i, j, k);
    return s->ca[k] * s->psiI[c] + s->cb[k] * (lap - s->cv * s->V[c] * s->psiR[c]);
}

/* Eq. (8) with the CAP, at one cell: returns psiR^{n+1}. */
static inline double og_new_R(const og_sim* s, int64_t i, int64_t j, int64_t k) {
    int64_t c = og_idx(&s->g, i, j, k);
    double lap = og_laplace_terms(s, s->psiI, i, j, k);
    return s->ca[k] * s->psiR[c] + s->cb[k] * (-lap + s->cv * s->V[c] * s->psiI[c]);
}

/* Store one detection record at the current level n = s->step:
 *   rho_ij = psiR^n(i,j,k_det)^2 + psiI^{n-1/2}(i,j,k_det)^2
 *   plane_sum = dV sum rho, naive_norm = dV sum (psiR^2 + psiI^2),
 *   q = the conserved form supplied by the caller, flux_acc.
 * The pixel integral adds h dt rho. */
static int og_store_record(og_sim* s, double q) {
    if (s->n_rec >= s->max_rec) return -1;
    const og_grid* g = &s->g;
    double dV = g->dx * g->dy * g->dz;
    double* rho = s->rec_rho + s->n_rec * g->nx * g->ny;
    double psum = 0.0;
    for (int64_t j = 0; j < g->ny; ++j)
        for (int64_t i = 0; i < g->nx; ++i) {
            int64_t c = og_idx(g, i, j, s->k_det);
            double r = s->psiR[c] * s->psiR[c] + s->psiI[c] * s->psiI[c];
            rho[j * g->nx + i] = r;
            psum += r;
            if (s->pixel) s->pixel[j * g->nx + i] += (double)s->h * s->dt * r;
        }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < g->nz; ++k) {
        double p = 0.0;
        for (int64_t c = k * g->nx * g->ny; c < (k + 1) * g->nx * g->ny; ++c)
            p += s->psiR[c] * s->psiR[c] + s->psiI[c] * s->psiI[c];
        s->plane_buf[k] = p;
    }
    double naive = og_sum_planes(s);
    double* sc = s->rec_scalars + 4 * s->n_rec;
    sc[0] = dV * psum;
    sc[1] = dV * naive;
    sc[2] = q;
    sc[3] = s->flux_acc;
    s->n_rec += 1;
    return 0;
}

/* Record 0 at the initial level: Q^0 = dV sum[psiR^0^2 + psiI^{-1/2} psiI^{+1/2}]
 * with psiI^{+1/2} evaluated but not stored. */
int og_record0(og_sim* s) {
    const og_grid* g = &s->g;
    double dV = g->dx * g->dy * g->dz;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < g->nz; ++k) {
        double p = 0.0;
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                int64_t c = og_idx(g, i, j, k);
                double inext = og_new_I(s, i, j, k);
                p += s->psiR[c] * s->psiR[c] + s->psiI[c] * inext;
            }
        s->plane_buf[k] = p;
    }
    return og_store_record(s, dV * og_sum_planes(s));
}

/* Advance nsteps steps.  One step n -> n+1:
 *  1. psiI^{n+1/2} from eq. (9) (+ CAP), everywhere, in place;
 *  2. psiR^{n+1} from eq. (8) (+ CAP), everywhere, in place;
 *  3. flux through the face between planes k_det and k_det+1 (k_det+1
 *     wrapped on a periodic axis, absent on a zero boundary):
 *       Phi = dV cz sum_ij [ I_{k+1} (R^n_k + R^{n+1}_k)
 *                           - I_k (R^n_{k+1} + R^{n+1}_{k+1}) ],
 *     I = psiI^{n+1/2}; positive means towards +z.  It is the exact
 *     discrete current of the scheme: for W = 0 the quantity
 *     q^n = psiR^n^2 + psiI^{n-1/2} psiI^{n+1/2} changes inside a slab of
 *     planes by exactly the difference of the face fluxes;
 *  4. if (n+1) mod h == 0, a record at level n+1 with
 *       Q = dV sum[psiI^{n+1/2}^2 + psiR^n psiR^{n+1}],
 *     the same conserved form written at a half-integer level.
 * Returns 0, or -1 if the record buffer overflows. */
int og_step(og_sim* s, int64_t nsteps) {
    const og_grid* g = &s->g;
    const int64_t nxy = g->nx * g->ny;
    const double dV = g->dx * g->dy * g->dz;
    const int64_t kd = s->k_det;
    const int has_up = !(g->bc[2] == OG_ZERO && kd + 1 >= g->nz);
    const int64_t ku = (kd + 1) % g->nz;
    double* rlo = malloc(sizeof(double) * nxy); /* psiR^n on plane k_det */
    double* rhi = malloc(sizeof(double) * nxy); /* psiR^n on plane k_det+1 */
    int rc = 0;
    for (int64_t it = 0; it < nsteps; ++it) {
        const int record = s->h > 0 && ((s->step + 1) % s->h == 0);
        memcpy(rlo, s->psiR + kd * nxy, sizeof(double) * nxy);
        if (has_up) memcpy(rhi, s->psiR + ku * nxy, sizeof(double) * nxy);
        if (record) memcpy(s->scratch_cell, s->psiR, sizeof(double) * nxy * g->nz);

        /* eq. (9): imaginary half-step */
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < g->nz; ++k)
            for (int64_t j = 0; j < g->ny; ++j)
                for (int64_t i = 0; i < g->nx; ++i)
                    s->psiI[og_idx(g, i, j, k)] = og_new_I(s, i, j, k);

        /* eq. (8): real half-step */
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < g->nz; ++k)
            for (int64_t j = 0; j < g->ny; ++j)
                for (int64_t i = 0; i < g->nx; ++i)
                    s->psiR[og_idx(g, i, j, k)] = og_new_R(s, i, j, k);

        /* flux through face k_det + 1/2 */
        double phi = 0.0;
        if (has_up) {
            for (int64_t j = 0; j < g->ny; ++j)
                for (int64_t i = 0; i < g->nx; ++i) {
                    int64_t p = j * g->nx + i;
                    double Ik = s->psiI[kd * nxy + p];
                    double Iu = s->psiI[ku * nxy + p];
                    double Rk1 = s->psiR[kd * nxy + p];
                    double Ru1 = s->psiR[ku * nxy + p];
                    phi += Iu * (rlo[p] + Rk1) - Ik * (rhi[p] + Ru1);
                }
        }
        s->flux_acc += dV * s->cz * phi;
        s->step += 1;

        if (record) {
#pragma omp parallel for schedule(static)
            for (int64_t k = 0; k < g->nz; ++k) {
                double p = 0.0;
                for (int64_t c = k * nxy; c < (k + 1) * nxy; ++c)
                    p += s->psiI[c] * s->psiI[c] + s->scratch_cell[c] * s->psiR[c];
                s->plane_buf[k] = p;
            }
            if (og_store_record(s, dV * og_sum_planes(s)) != 0) {
                rc = -1;
                break;
            }
        }
    }
    free(rlo);
    free(rhi);
    return rc;
}

/* Exact inverse of nsteps steps (time reversal of the leapfrog):
 *   psiR^n       = (psiR^{n+1} - cb G psiI^{n+1/2}) / ca
 *   psiI^{n-1/2} = (psiI^{n+1/2} + cb G psiR^n) / ca
 * with G X = -(cx dxx + cy dyy + cz dzz) X + cv V X.  Records and the flux
 * accumulator are left untouched. */
void og_unstep(og_sim* s, int64_t nsteps) {
    const og_grid* g = &s->g;
    for (int64_t it = 0; it < nsteps; ++it) {
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < g->nz; ++k)
            for (int64_t j = 0; j < g->ny; ++j)
                for (int64_t i = 0; i < g->nx; ++i) {
                    int64_t c = og_idx(g, i, j, k);
                    double gI = -og_laplace_terms(s, s->psiI, i, j, k) + s->cv * s->V[c] * s->psiI[c];
                    s->psiR[c] = (s->psiR[c] - s->cb[k] * gI) / s->ca[k];
                }
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < g->nz; ++k)
            for (int64_t j = 0; j < g->ny; ++j)
                for (int64_t i = 0; i < g->nx; ++i) {
                    int64_t c = og_idx(g, i, j, k);
                    double gR = -og_laplace_terms(s, s->psiR, i, j, k) + s->cv * s->V[c] * s->psiR[c];
                    s->psiI[c] = (s->psiI[c] + s->cb[k] * gR) / s->ca[k];
                }
        s->step -= 1;
    }
}

/* ---------------------------------------------------------------------- */
/* Discrete adjoint of the leapfrog                                        */
/* ---------------------------------------------------------------------- */

/* G X = -(cx dxx + cy dyy + cz dzz) X + cv V X, the operator both half-steps
 * apply (eq. (9): I' = A I - B G R; eq. (8): R' = A R + B G I', with
 * A = diag(ca_k), B = diag(cb_k)).  G is symmetric. */
static void og_apply_G(const og_sim* s, const double* X, double* out) {
    const og_grid* g = &s->g;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                int64_t c = og_idx(g, i, j, k);
                out[c] = -og_laplace_terms(s, X, i, j, k) + s->cv * s->V[c] * X[c];
            }
}

/* Gradient of a loss of the detection records through nsteps steps of the
 * leapfrog started from the state in s (level 0), by reverse mode on the
 * discrete scheme.  dL_drho is [n_rec][ny][nx] for the records at levels
 * 0, h, 2h, ... <= nsteps (record m is rho at level m h on plane k_det).
 * Forward states are recomputed from checkpoints stored every K steps.
 * Backward step n (from r = dL/dR^{n+1}, i = dL/dI^{n+1/2}):
 *   i_t = i + G (B r)
 *   g_V += cv (B r) o I^{n+1/2} - cv (B i_t) o R^n
 *   r  <- A r - G (B i_t),   i <- A i_t
 * then the record injections at level n: r += 2 R^n rho_bar, i += 2 I^{n-1/2}
 * rho_bar on plane k_det.  Outputs gV [nz][ny][nx] (dL/dV), gR0 = dL/dR^0,
 * gI0 = dL/dI^{-1/2}.  s is left unchanged.  Returns 0 or -1 (allocation). */
int og_adjoint(og_sim* s, int64_t nsteps, const double* dL_drho, int64_t K, double* gV,
               double* gR0, double* gI0) {
    const og_grid* g = &s->g;
    const int64_t n = g->nx * g->ny * g->nz;
    const int64_t nxy = g->nx * g->ny;
    if (K < 1) K = 1;
    const int64_t nck = nsteps / K + 1;
    double* ckR = malloc(sizeof(double) * n * nck);
    double* ckI = malloc(sizeof(double) * n * nck);
    double* segR = malloc(sizeof(double) * n * (K + 1));
    double* segI = malloc(sizeof(double) * n * (K + 1));
    double* rb = calloc(n, sizeof(double));
    double* ib = calloc(n, sizeof(double));
    double* t1 = malloc(sizeof(double) * n);
    double* t2 = malloc(sizeof(double) * n);
    double* saveR = malloc(sizeof(double) * n);
    double* saveI = malloc(sizeof(double) * n);
    if (!ckR || !ckI || !segR || !segI || !rb || !ib || !t1 || !t2 || !saveR || !saveI) return -1;
    memcpy(saveR, s->psiR, sizeof(double) * n);
    memcpy(saveI, s->psiI, sizeof(double) * n);
    const int64_t step0 = s->step;
    const double flux0 = s->flux_acc;
    const int64_t h_save = s->h;
    s->h = 0; /* no records while replaying */

    /* forward pass: checkpoints at 0, K, 2K, ... */
    for (int64_t c = 0; c < nck; ++c) {
        memcpy(ckR + c * n, s->psiR, sizeof(double) * n);
        memcpy(ckI + c * n, s->psiI, sizeof(double) * n);
        int64_t todo = (c + 1) * K <= nsteps ? K : nsteps - c * K;
        if (c + 1 < nck) og_step(s, todo);
    }
    for (int64_t c = 0; c < n; ++c) gV[c] = 0.0;

    /* record injection at level lev using state (R, I) = (R^lev, I^{lev-1/2}) */
#define OG_INJECT(lev, Rl, Il)                                                        \
    do {                                                                              \
        if (h_save > 0 && (lev) % h_save == 0) {                                      \
            const double* rbar = dL_drho + ((lev) / h_save) * nxy;                    \
            for (int64_t p = 0; p < nxy; ++p) {                                       \
                int64_t cc = s->k_det * nxy + p;                                      \
                rb[cc] += 2.0 * (Rl)[cc] * rbar[p];                                   \
                ib[cc] += 2.0 * (Il)[cc] * rbar[p];                                   \
            }                                                                         \
        }                                                                             \
    } while (0)

    for (int64_t c = nck - 1; c >= 0; --c) {
        const int64_t s0 = c * K;
        const int64_t s1 = (s0 + K < nsteps) ? s0 + K : nsteps;
        /* recompute the states s0..s1 of this segment */
        memcpy(s->psiR, ckR + c * n, sizeof(double) * n);
        memcpy(s->psiI, ckI + c * n, sizeof(double) * n);
        memcpy(segR, s->psiR, sizeof(double) * n);
        memcpy(segI, s->psiI, sizeof(double) * n);
        for (int64_t m = s0; m < s1; ++m) {
            og_step(s, 1);
            memcpy(segR + (m - s0 + 1) * n, s->psiR, sizeof(double) * n);
            memcpy(segI + (m - s0 + 1) * n, s->psiI, sizeof(double) * n);
        }
        if (s1 == nsteps) OG_INJECT(nsteps, segR + (s1 - s0) * n, segI + (s1 - s0) * n);
        for (int64_t m = s1 - 1; m >= s0; --m) {
            const double* Rn = segR + (m - s0) * n;         /* R^m */
            const double* Ih = segI + (m - s0 + 1) * n;     /* I^{m+1/2} */
            /* t1 = B r, i_t = i + G t1 */
            for (int64_t cc = 0; cc < n; ++cc) t1[cc] = s->cb[cc / nxy] * rb[cc];
            og_apply_G(s, t1, t2);
            for (int64_t cc = 0; cc < n; ++cc) {
                gV[cc] += s->cv * t1[cc] * Ih[cc];
                ib[cc] += t2[cc];
            }
            /* t1 = B i_t; r <- A r - G t1; i <- A i_t */
            for (int64_t cc = 0; cc < n; ++cc) t1[cc] = s->cb[cc / nxy] * ib[cc];
            og_apply_G(s, t1, t2);
            for (int64_t cc = 0; cc < n; ++cc) {
                gV[cc] -= s->cv * t1[cc] * Rn[cc];
                const double a = s->ca[cc / nxy];
                rb[cc] = a * rb[cc] - t2[cc];
                ib[cc] = a * ib[cc];
            }
            OG_INJECT(m, Rn, segI + (m - s0) * n);
        }
    }
#undef OG_INJECT
    memcpy(gR0, rb, sizeof(double) * n);
    memcpy(gI0, ib, sizeof(double) * n);
    /* restore the simulation */
    memcpy(s->psiR, saveR, sizeof(double) * n);
    memcpy(s->psiI, saveI, sizeof(double) * n);
    s->step = step0;
    s->flux_acc = flux0;
    s->h = h_save;
    free(ckR); free(ckI); free(segR); free(segI); free(rb); free(ib);
    free(t1); free(t2); free(saveR); free(saveI);
    return 0;
}

/* Chain rule from dL/dV to the atoms of og_potential:
 *   dL/dX_a = sum_r gV(r) dV(r)/dX_a,  dV/dX_a = -amp_a v'(d) u/d,
 *   dL/damp_a = sum_r gV(r) v(d),
 * u = r - X_a (minimum image), d = |u| < cutoff.  A grid point exactly on an
 * atom (d = 0) adds nothing to dL/dX_a: the screened potential has a cusp
 * there and the symmetric subgradient is zero. */
void og_potential_vjp(const og_grid* g, const double* atoms, int64_t n, double soft,
                      double cutoff, double kappa, double a0, int screened, const double* gV,
                      double* dpos, double* damp) {
    const double L[3] = {g->nx * g->dx, g->ny * g->dy, g->nz * g->dz};
#pragma omp parallel for schedule(dynamic)
    for (int64_t a = 0; a < n; ++a) {
        const double* at = atoms + 5 * a;
        double sx = 0.0, sy = 0.0, sz = 0.0, sa = 0.0;
        for (int64_t k = 0; k < g->nz; ++k) {
            double uz = k * g->dz - at[2];
            if (g->bc[2] == OG_PERIODIC) uz = og_min_image(uz, L[2]);
            if (fabs(uz) >= cutoff) continue;
            for (int64_t j = 0; j < g->ny; ++j) {
                double uy = j * g->dy - at[1];
                if (g->bc[1] == OG_PERIODIC) uy = og_min_image(uy, L[1]);
                if (fabs(uy) >= cutoff) continue;
                for (int64_t i = 0; i < g->nx; ++i) {
                    double ux = i * g->dx - at[0];
                    if (g->bc[0] == OG_PERIODIC) ux = og_min_image(ux, L[0]);
                    const double d = sqrt(ux * ux + uy * uy + uz * uz);
                    if (d >= cutoff) continue;
                    const double w = gV[og_idx(g, i, j, k)];
                    sa += w * og_vatom(d, at[3], soft, kappa, a0, screened);
                    if (d > 0.0) {
                        const double f = -at[4] * og_dvatom(d, at[3], soft, kappa, a0, screened) / d;
                        sx += w * f * ux;
                        sy += w * f * uy;
                        sz += w * f * uz;
                    }
                }
            }
        }
        dpos[3 * a + 0] = sx;
        dpos[3 * a + 1] = sy;
        dpos[3 * a + 2] = sz;
        damp[a] = sa;
    }
}

/*
 * Potential on the mesh from a table over one unit cell (section 2.3: the
 * potential of one cell, repeated in x and y and interpolated onto the mesh
 * points; the interpolation is step (ii) of section 3.2).  The paper does not
 * name the interpolation; this is trilinear.
 *
 * table is [uz][uy][ux], x fastest; sample (a, b, c) sits at
 * (origin[0] + a sx, origin[1] + b sy, origin[2] + c sz) with s = spacing.
 * The cell repeats in x and y with periods ux sx and uy sy; in z the table is
 * held constant beyond its first and last sample planes.  Mesh point
 * (i, j, k) sits at (i dx, j dy, k dz).
 */
static void og_axis_weights_periodic(double u, int64_t n, int64_t* a0, int64_t* a1, double* t) {
    const double f = floor(u);
    *t = u - f;
    int64_t a = (int64_t)f % n;
    if (a < 0) a += n;
    *a0 = a;
    *a1 = (a + 1) % n;
}

void og_interp_potential(const og_grid* g, const double* table, int64_t ux, int64_t uy, int64_t uz,
                         const double* spacing, const double* origin, double* V) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < g->nz; ++k) {
        /* z: clamp to the table's z range */
        int64_t c0 = 0, c1 = 0;
        double tz = 0.0;
        if (uz > 1) {
            double w = (k * g->dz - origin[2]) / spacing[2];
            if (w < 0.0) w = 0.0;
            if (w > (double)(uz - 1)) w = (double)(uz - 1);
            c0 = (int64_t)floor(w);
            if (c0 > uz - 2) c0 = uz - 2;
            tz = w - (double)c0;
            c1 = c0 + 1;
        }
        for (int64_t j = 0; j < g->ny; ++j) {
            int64_t b0, b1;
            double ty;
            og_axis_weights_periodic((j * g->dy - origin[1]) / spacing[1], uy, &b0, &b1, &ty);
            for (int64_t i = 0; i < g->nx; ++i) {
                int64_t a0, a1;
                double tx;
                og_axis_weights_periodic((i * g->dx - origin[0]) / spacing[0], ux, &a0, &a1, &tx);
#define OG_T(a, b, c) table[((c) * uy + (b)) * ux + (a)]
                /* x, then y, then z */
                const double v00 = (1.0 - tx) * OG_T(a0, b0, c0) + tx * OG_T(a1, b0, c0);
                const double v10 = (1.0 - tx) * OG_T(a0, b1, c0) + tx * OG_T(a1, b1, c0);
                const double v01 = (1.0 - tx) * OG_T(a0, b0, c1) + tx * OG_T(a1, b0, c1);
                const double v11 = (1.0 - tx) * OG_T(a0, b1, c1) + tx * OG_T(a1, b1, c1);
#undef OG_T
                const double v0 = (1.0 - ty) * v00 + ty * v10;
                const double v1 = (1.0 - ty) * v01 + ty * v11;
                V[og_idx(g, i, j, k)] = (1.0 - tz) * v0 + tz * v1;
            }
        }
    }
}

/*
 * Dissimilarity of detection-plane trajectories, eq. (16): for trajectories
 * k and j, the time average over [t0, t1] of the L2 distance between their
 * detector-plane densities.  frames is [K][T][P] (trajectory, frame, pixel);
 * the time integral is the quadrature sum over frames with weights w[T]
 * (which carry the 1/(t1 - t0)); the plane integral is dA times the pixel
 * sum.  out[k][j] = sum_t w_t sqrt(dA sum_p (rho_k,t,p - rho_j,t,p)^2).
 */
void og_dissimilarity(const double* frames, int64_t K, int64_t T, int64_t P, const double* w,
                      double dA, double* out) {
#pragma omp parallel for schedule(dynamic)
    for (int64_t k = 0; k < K; ++k) {
        for (int64_t j = 0; j < K; ++j) {
            double d = 0.0;
            for (int64_t t = 0; t < T; ++t) {
                const double* a = frames + (k * T + t) * P;
                const double* b = frames + (j * T + t) * P;
                double s = 0.0;
                for (int64_t p = 0; p < P; ++p) {
                    const double e = a[p] - b[p];
                    s += e * e;
                }
                d += w[t] * sqrt(dA * s);
            }
            out[k * K + j] = d;
        }
    }
}

/*
 * The CAP of eq. (10) taken literally, one-sided at the bottom: a rate
 * W_k = (alpha / dz) (r_cut - k dz)^2 where k dz < r_cut, else 0.  The
 * paper's constant is garbled; alpha is read as energy per length.
 */
void og_cap_paper(int64_t nz, double dz, double alpha, double r_cut, double* W) {
    for (int64_t k = 0; k < nz; ++k) {
        const double z = k * dz;
        W[k] = (z < r_cut) ? alpha / dz * (r_cut - z) * (r_cut - z) : 0.0;
    }
}

/* The time step eq. (11) recommends: m min(dx, dy, dz)^2 / (5 hbar). */
double og_dt_paper(const og_grid* g) {
    double d = g->dx;
    if (g->dy < d) d = g->dy;
    if (g->dz < d) d = g->dz;
    return g->mass / (5.0 * g->hbar) * d * d;
}
