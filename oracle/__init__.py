"""FP64 CPU oracle for the FDTD leapfrog of the 3D time-dependent Schrodinger
equation (arXiv 2401.07416, section 2.1, eqs. (2)-(11) and (15)).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the HIP library and never consumes anything the HIP library produced.
The arithmetic lives in ``tdse_oracle.c``; this module only marshals numpy
arrays into it through ctypes.

Parity status of each function (the pins live in ``tests/test_oracle_*.py``):
  step / unstep / records / Q / flux : pinned (exact discrete solutions by FFT
      and by dense eigen-decomposition, conserved Q, time reversal, discrete
      continuity, continuum convergence)
  emax                                : pinned (dense eigenvalues)
  gaussian_closed / init_gaussian     : pinned (free Schrodinger residual,
      normalisation, moments, group velocity)
  potential                           : pinned (on-node value, symmetries,
      periodic images, brute-force points)
  adjoint / potential_vjp             : pinned (central finite differences of the
      forward oracle, directional derivatives, checkpoint-interval invariance)
  interp_potential                    : pinned (coincident grids copy the table,
      fields linear in each axis are reproduced, cell periodicity, a
      library trilinear interpolator on a periodically padded table)
  cap_paper / dt_paper                : pinned (support, value at the bottom plane,
      constant second difference; the 0.48 as of the paper's grid and the
      1.2 ratio to the Gershgorin step on a free cubic grid)
  dissimilarity                       : pinned (metric axioms, a closed form
      for constant frames, brute force with numpy)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tdse_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PERIODIC = 0
ZERO = 1
INIT_HALFSTEP = 0
INIT_NAIVE = 1

# physical constants (eV, Angstrom, fs)
HBAR_EV_FS = 0.6582119569
HBAR2_OVER_ME = 7.619964  # eV * Angstrom^2
KAPPA_EV_A = 14.3996454784  # e^2 / (4 pi eps0), eV * Angstrom
BOHR_A = 0.529177210903


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("hbar", ctypes.c_double), ("mass", ctypes.c_double),
                ("bc", ctypes.c_int32 * 3), ("pad_", ctypes.c_int32)]


_dp = ctypes.POINTER(ctypes.c_double)


class _Sim(ctypes.Structure):
    _fields_ = [("g", _Grid), ("dt", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("cz", ctypes.c_double),
                ("cv", ctypes.c_double), ("ca", _dp), ("cb", _dp),
                ("psiR", _dp), ("psiI", _dp), ("V", _dp),
                ("k_det", ctypes.c_int64), ("h", ctypes.c_int64), ("step", ctypes.c_int64),
                ("flux_acc", ctypes.c_double),
                ("rec_rho", _dp), ("rec_scalars", _dp), ("max_rec", ctypes.c_int64),
                ("n_rec", ctypes.c_int64), ("pixel", _dp), ("scratch_cell", _dp),
                ("plane_buf", _dp)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        gp = ctypes.POINTER(_Grid)
        sp = ctypes.POINTER(_Sim)
        L.og_abi_version.restype = ctypes.c_int
        L.og_set_threads.argtypes = [ctypes.c_int]
        L.og_get_threads.restype = ctypes.c_int
        L.og_emax.argtypes = [gp, _dp]
        L.og_emax.restype = ctypes.c_double
        L.og_coeffs.argtypes = [gp, ctypes.c_double, _dp, _dp, _dp, _dp]
        L.og_cap_quadratic.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_double, _dp]
        L.og_vatom.argtypes = [ctypes.c_double] * 5 + [ctypes.c_int]
        L.og_vatom.restype = ctypes.c_double
        L.og_dvatom.argtypes = [ctypes.c_double] * 5 + [ctypes.c_int]
        L.og_dvatom.restype = ctypes.c_double
        L.og_potential.argtypes = [gp, _dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp]
        L.og_potential_window.argtypes = [gp, _dp, ctypes.c_int64, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_int] + [ctypes.c_int64] * 6 + [_dp]
        L.og_init_gaussian_window.argtypes = [gp, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_int, ctypes.c_int] + \
            [ctypes.c_int64] * 6 + [_dp, _dp]
        L.og_potential_points.argtypes = [gp, _dp, ctypes.c_int64, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_int, _dp, ctypes.c_int64, _dp]
        L.og_gaussian_closed.argtypes = [gp, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, _dp, _dp]
        L.og_init_gaussian.argtypes = [gp, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.og_sim_init.argtypes = [sp]
        L.og_record0.argtypes = [sp]
        L.og_record0.restype = ctypes.c_int
        L.og_step.argtypes = [sp, ctypes.c_int64]
        L.og_step.restype = ctypes.c_int
        L.og_unstep.argtypes = [sp, ctypes.c_int64]
        L.og_adjoint.argtypes = [sp, ctypes.c_int64, _dp, ctypes.c_int64, _dp, _dp, _dp]
        L.og_adjoint.restype = ctypes.c_int
        L.og_cap_paper.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, _dp]
        L.og_dt_paper.argtypes = [gp]
        L.og_dt_paper.restype = ctypes.c_double
        L.og_interp_potential.argtypes = [gp, _dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                          _dp, _dp, _dp]
        L.og_dissimilarity.argtypes = [_dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _dp,
                                       ctypes.c_double, _dp]
        L.og_potential_vjp.argtypes = [gp, _dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp, _dp,
                                       _dp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def set_threads(n: int) -> None:
    lib().og_set_threads(int(n))


def get_threads() -> int:
    return int(lib().og_get_threads())


class Grid:
    """Regular grid r = (i dx, j dy, k dz), arrays [nz][ny][nx] (x fastest)."""

    def __init__(self, nx, ny, nz, dx, dy, dz, hbar=1.0, mass=1.0, bc=(PERIODIC,) * 3):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dx, self.dy, self.dz = float(dx), float(dy), float(dz)
        self.hbar, self.mass = float(hbar), float(mass)
        self.bc = tuple(int(b) for b in bc)
        self._c = _Grid(self.nx, self.ny, self.nz, self.dx, self.dy, self.dz, self.hbar,
                        self.mass, (ctypes.c_int32 * 3)(*self.bc), 0)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def dV(self):
        return self.dx * self.dy * self.dz

    def ref(self):
        return ctypes.byref(self._c)


def emax(grid: Grid, V: np.ndarray) -> float:
    V = np.ascontiguousarray(V, dtype=np.float64)
    return float(lib().og_emax(grid.ref(), _ptr(V)))


def coeffs(grid: Grid, dt: float, W=None):
    c4 = np.zeros(4)
    ca = np.zeros(grid.nz)
    cb = np.zeros(grid.nz)
    Wp = None
    if W is not None:
        W = np.ascontiguousarray(W, dtype=np.float64)
        Wp = _ptr(W)
    lib().og_coeffs(grid.ref(), float(dt), Wp, _ptr(c4), _ptr(ca), _ptr(cb))
    return c4, ca, cb


def cap_quadratic(nz: int, nbot: int, ntop: int, wmax: float) -> np.ndarray:
    W = np.zeros(nz)
    lib().og_cap_quadratic(int(nz), int(nbot), int(ntop), float(wmax), _ptr(W))
    return W


def vatom(d, Z, soft, kappa=KAPPA_EV_A, a0=BOHR_A, screened=True):
    return float(lib().og_vatom(float(d), float(Z), float(soft), float(kappa), float(a0),
                                int(screened)))


def dvatom(d, Z, soft, kappa=KAPPA_EV_A, a0=BOHR_A, screened=True):
    return float(lib().og_dvatom(float(d), float(Z), float(soft), float(kappa), float(a0),
                                 int(screened)))


def potential(grid: Grid, atoms: np.ndarray, soft=0.1, cutoff=6.0, kappa=KAPPA_EV_A,
              a0=BOHR_A, screened=True) -> np.ndarray:
    atoms = np.ascontiguousarray(atoms, dtype=np.float64).reshape(-1, 5)
    V = np.zeros(grid.shape)
    lib().og_potential(grid.ref(), _ptr(atoms), atoms.shape[0], float(soft), float(cutoff),
                       float(kappa), float(a0), int(screened), _ptr(V))
    return V


def potential_points(grid: Grid, atoms: np.ndarray, pts: np.ndarray, soft=0.1, cutoff=6.0,
                     kappa=KAPPA_EV_A, a0=BOHR_A, screened=True) -> np.ndarray:
    atoms = np.ascontiguousarray(atoms, dtype=np.float64).reshape(-1, 5)
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(pts.shape[0])
    lib().og_potential_points(grid.ref(), _ptr(atoms), atoms.shape[0], float(soft),
                              float(cutoff), float(kappa), float(a0), int(screened), _ptr(pts),
                              pts.shape[0], _ptr(out))
    return out


def potential_window(grid: Grid, atoms: np.ndarray, origin, size, soft=0.1, cutoff=6.0,
                     kappa=KAPPA_EV_A, a0=BOHR_A, screened=True) -> np.ndarray:
    """V on the window of grid points ((i0+ii) mod nx, ...), shape [wnz][wny][wnx];
    origin = (i0, j0, k0), size = (wnx, wny, wnz)."""
    atoms = np.ascontiguousarray(atoms, dtype=np.float64).reshape(-1, 5)
    out = np.zeros((int(size[2]), int(size[1]), int(size[0])))
    lib().og_potential_window(grid.ref(), _ptr(atoms), atoms.shape[0], float(soft),
                              float(cutoff), float(kappa), float(a0), int(screened),
                              *[int(x) for x in origin], *[int(x) for x in size], _ptr(out))
    return out


def init_gaussian_window(grid: Grid, r0, k0, sigma, dt, origin, size, mode=INIT_HALFSTEP,
                         nimg=2):
    """init_gaussian restricted to a window (normalised over the whole grid)."""
    shape = (int(size[2]), int(size[1]), int(size[0]))
    R = np.zeros(shape)
    I = np.zeros(shape)
    r0 = np.ascontiguousarray(r0, dtype=np.float64)
    k0 = np.ascontiguousarray(k0, dtype=np.float64)
    lib().og_init_gaussian_window(grid.ref(), _ptr(r0), _ptr(k0), float(sigma), float(dt),
                                  int(mode), int(nimg), *[int(x) for x in origin],
                                  *[int(x) for x in size], _ptr(R), _ptr(I))
    return R, I


def potential_vjp(grid: Grid, atoms: np.ndarray, gV: np.ndarray, soft=0.1, cutoff=6.0,
                  kappa=KAPPA_EV_A, a0=BOHR_A, screened=True):
    """(dL/dpositions [n][3], dL/damplitudes [n]) from dL/dV."""
    atoms = np.ascontiguousarray(atoms, dtype=np.float64).reshape(-1, 5)
    gV = np.ascontiguousarray(gV, dtype=np.float64)
    dpos = np.zeros((atoms.shape[0], 3))
    damp = np.zeros(atoms.shape[0])
    lib().og_potential_vjp(grid.ref(), _ptr(atoms), atoms.shape[0], float(soft), float(cutoff),
                           float(kappa), float(a0), int(screened), _ptr(gV), _ptr(dpos),
                           _ptr(damp))
    return dpos, damp


def gaussian_closed(grid: Grid, r0, k0, sigma, t, nimg=2):
    re = np.zeros(grid.shape)
    im = np.zeros(grid.shape)
    r0 = np.ascontiguousarray(r0, dtype=np.float64)
    k0 = np.ascontiguousarray(k0, dtype=np.float64)
    lib().og_gaussian_closed(grid.ref(), _ptr(r0), _ptr(k0), float(sigma), float(t), int(nimg),
                             _ptr(re), _ptr(im))
    return re, im


def init_gaussian(grid: Grid, r0, k0, sigma, dt, mode=INIT_HALFSTEP, nimg=2):
    R = np.zeros(grid.shape)
    I = np.zeros(grid.shape)
    r0 = np.ascontiguousarray(r0, dtype=np.float64)
    k0 = np.ascontiguousarray(k0, dtype=np.float64)
    lib().og_init_gaussian(grid.ref(), _ptr(r0), _ptr(k0), float(sigma), float(dt), int(mode),
                           int(nimg), _ptr(R), _ptr(I))
    return R, I


def wavevector(energy: float, hbar: float, mass: float) -> float:
    """|k| = 2 pi / lambda with lambda from eq. (4)."""
    lam = np.sqrt(2.0 * hbar ** 2 * np.pi ** 2 / (mass * energy))
    return 2.0 * np.pi / lam


class Sim:
    """The oracle leapfrog with its records.  Owns numpy copies of R, I, V."""

    def __init__(self, grid: Grid, V, R, I, dt, W=None, k_det=0, record_every=0,
                 max_records=0, pixel=False):
        self.grid = grid
        self.V = np.ascontiguousarray(V, dtype=np.float64).copy()
        self.R = np.ascontiguousarray(R, dtype=np.float64).copy()
        self.I = np.ascontiguousarray(I, dtype=np.float64).copy()
        assert self.V.shape == grid.shape and self.R.shape == grid.shape
        self.dt = float(dt)
        self.c4, self.ca, self.cb = coeffs(grid, dt, W)
        nrec = max(int(max_records), 1)
        self.rec_rho = np.zeros((nrec, grid.ny, grid.nx))
        self.rec_scalars = np.zeros((nrec, 4))
        self.pixel = np.zeros((grid.ny, grid.nx)) if pixel else None
        self.scratch = np.zeros(grid.shape)
        self.plane_buf = np.zeros(grid.nz)
        s = _Sim()
        s.g = grid._c
        s.dt = self.dt
        s.cx, s.cy, s.cz, s.cv = [float(x) for x in self.c4]
        s.ca, s.cb = _ptr(self.ca), _ptr(self.cb)
        s.psiR, s.psiI, s.V = _ptr(self.R), _ptr(self.I), _ptr(self.V)
        s.k_det = int(k_det)
        s.h = int(record_every)
        s.rec_rho, s.rec_scalars = _ptr(self.rec_rho), _ptr(self.rec_scalars)
        s.max_rec = int(max_records)
        s.pixel = _ptr(self.pixel) if pixel else ctypes.cast(None, _dp)
        s.scratch_cell, s.plane_buf = _ptr(self.scratch), _ptr(self.plane_buf)
        self._s = s
        lib().og_sim_init(ctypes.byref(s))

    @property
    def step_count(self) -> int:
        return int(self._s.step)

    @property
    def flux(self) -> float:
        return float(self._s.flux_acc)

    @property
    def n_records(self) -> int:
        return int(self._s.n_rec)

    def record0(self):
        if lib().og_record0(ctypes.byref(self._s)) != 0:
            raise RuntimeError("record buffer full")

    def step(self, n: int):
        if lib().og_step(ctypes.byref(self._s), int(n)) != 0:
            raise RuntimeError("record buffer full")

    def unstep(self, n: int):
        lib().og_unstep(ctypes.byref(self._s), int(n))

    def records(self):
        n = self.n_records
        return self.rec_rho[:n].copy(), self.rec_scalars[:n].copy()

    def adjoint(self, nsteps: int, dL_drho: np.ndarray, ckpt_every: int = 100):
        """Gradient of a loss of the records of an nsteps run started from the
        current state: returns (dL/dV, dL/dR^0, dL/dI^{-1/2})."""
        g = self.grid
        nrec = (nsteps // self._s.h + 1) if self._s.h > 0 else 0
        rb = np.ascontiguousarray(dL_drho, dtype=np.float64).reshape(max(nrec, 1), g.ny, g.nx)
        gV, gR, gI = np.zeros(g.shape), np.zeros(g.shape), np.zeros(g.shape)
        if lib().og_adjoint(ctypes.byref(self._s), int(nsteps), _ptr(rb), int(ckpt_every),
                            _ptr(gV), _ptr(gR), _ptr(gI)) != 0:
            raise MemoryError("oracle adjoint allocation")
        return gV, gR, gI


def interp_potential(grid: Grid, table: np.ndarray, spacing, origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Trilinear interpolation of a unit-cell table [uz][uy][ux] (periodic in
    x and y, held constant beyond its z range) onto the mesh (section 2.3)."""
    table = np.ascontiguousarray(table, dtype=np.float64)
    uz, uy, ux = table.shape
    sp = np.ascontiguousarray(spacing, dtype=np.float64)
    org = np.ascontiguousarray(origin, dtype=np.float64)
    V = np.zeros(grid.shape)
    lib().og_interp_potential(grid.ref(), _ptr(table), ux, uy, uz, _ptr(sp), _ptr(org), _ptr(V))
    return V


def dissimilarity(frames: np.ndarray, weights, dA: float) -> np.ndarray:
    """d_kj of eq. (16) for frames [K][T][P] with time-quadrature weights w[T]
    (including 1 / (t1 - t0)) and pixel area dA."""
    frames = np.ascontiguousarray(frames, dtype=np.float64)
    K, T, P = frames.shape
    w = np.ascontiguousarray(weights, dtype=np.float64)
    assert w.shape == (T,)
    out = np.zeros((K, K))
    lib().og_dissimilarity(_ptr(frames), K, T, P, _ptr(w), float(dA), _ptr(out))
    return out


def cap_paper(nz: int, dz: float, alpha: float, r_cut: float) -> np.ndarray:
    """Eq. (10) as printed, one-sided at the bottom (alpha: energy / length)."""
    W = np.zeros(int(nz))
    lib().og_cap_paper(int(nz), float(dz), float(alpha), float(r_cut), _ptr(W))
    return W


def dt_paper(grid: Grid) -> float:
    """Eq. (11): m min(dx, dy, dz)^2 / (5 hbar)."""
    return float(lib().og_dt_paper(grid.ref()))
