"""Python binding of libtdse (include/tdse.h) through ctypes.

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libtdse.so``.  PyTorch provides the device memory (caller-owned tensors
bound to a handle) and the stream (torch's current stream).  There is no CPU
fallback: if the library is missing, ``load()`` raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdse.so")

OK, ERR_ARG, ERR_STATE, ERR_UNSTABLE, ERR_NONFINITE, ERR_DEVICE, ERR_OOM, ERR_UNSUPPORTED, \
    ERR_CAPACITY = range(9)
BC_PERIODIC, BC_ZERO = 0, 1
F32, F64 = 0, 1
INIT_HALFSTEP, INIT_NAIVE = 0, 1
FLAG_ALLOW_UNSTABLE, FLAG_PIXEL_INTEGRAL = 1, 2
TUNE_REFRESH = 8   # tdse_autotune flag: time the candidates even on a cache hit

# every symbol include/tdse.h declares
EXPORTS = [
    "tdse_abi_version", "tdse_status_string", "tdse_last_error", "tdse_validate_desc",
    "tdse_time_step_bound", "tdse_workspace_size", "tdse_create", "tdse_destroy", "tdse_bind",
    "tdse_build_potential", "tdse_set_cap", "tdse_set_cap_quadratic", "tdse_finalize_setup",
    "tdse_init_gaussian", "tdse_set_state", "tdse_get_state", "tdse_step", "tdse_detect",
    "tdse_copy_scalars", "tdse_set_timing", "tdse_timing_read", "tdse_get_tile", "tdse_set_tile",
    "tdse_bind_pingpong", "tdse_adjoint_workspace_size", "tdse_bind_adjoint", "tdse_adjoint",
    "tdse_potential_vjp", "tdse_batch_create", "tdse_batch_member", "tdse_batch_set_tile",
    "tdse_batch_prepare", "tdse_batch_run", "tdse_batch_status", "tdse_batch_last_error",
    "tdse_batch_destroy", "tdse_hbm_probe", "tdse_interpolate_potential",
    "tdse_dissimilarity_workspace_size", "tdse_dissimilarity", "tdse_set_cap_paper",
    "tdse_time_step_paper", "tdse_batch_set_two_step", "tdse_autotune", "tdse_paper_layout_run",
    "tdse_dissimilarity_noalloc", "tdse_timing_read_split", "tdse_batch_workspace_size",
    "tdse_batch_bind_workspace", "tdse_batch_bind", "tdse_batch_detect",
]


class TdseError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("hbar", ctypes.c_double), ("mass", ctypes.c_double),
                ("dt", ctypes.c_double), ("dt_frac", ctypes.c_double),
                ("bc", ctypes.c_int32 * 3), ("precision", ctypes.c_int32),
                ("k_det", ctypes.c_int64), ("record_every", ctypes.c_int64),
                ("max_records", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class Atom(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double), ("y", ctypes.c_double), ("z", ctypes.c_double),
                ("Z", ctypes.c_double), ("amp", ctypes.c_double)]


class PotParams(ctypes.Structure):
    _fields_ = [("soft", ctypes.c_double), ("cutoff", ctypes.c_double),
                ("kappa", ctypes.c_double), ("a0", ctypes.c_double),
                ("screened", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class DetectOut(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("n_records", ctypes.c_int64),
                ("flux_acc", ctypes.c_double), ("dt", ctypes.c_double),
                ("e_max", ctypes.c_double), ("records", ctypes.c_void_p),
                ("scalars", ctypes.c_void_p), ("pixel", ctypes.c_void_p)]


class Tile(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("waves", ctypes.c_int32), ("zc", ctypes.c_int32),
                ("fused", ctypes.c_int32), ("fused_rows", ctypes.c_int32),
                ("fused_zc", ctypes.c_int32), ("fused_prefetch", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("fused_threads", ctypes.c_int32),
                ("two_step", ctypes.c_int32), ("two_step_tx", ctypes.c_int32),
                ("two_step_rows", ctypes.c_int32), ("two_step_zc", ctypes.c_int32),
                ("two_step_prefetch", ctypes.c_int32), ("two_step_threads", ctypes.c_int32),
                ("vec_elems", ctypes.c_int32),
                ("vec_groups", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("band_rows", ctypes.c_int32), ("two_step_ty", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


_lib = None


def load():
    """Load libtdse.so (raises if it has not been built).

    torch is imported first: the PyTorch wheel carries its own HIP runtime,
    and the library must resolve its HIP symbols to that one, the runtime
    that owns the device memory and streams it is handed.  Loaded before
    torch, the library would pull in a second HIP runtime whose calls fail
    in a process where torch has initialised the device."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2401_07416_amd.build` (no CPU fallback exists)")
    import torch  # noqa: F401  (one HIP runtime per process, torch's)
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "tdse_abi_version": (i32, []),
        "tdse_status_string": (ctypes.c_char_p, [i32]),
        "tdse_last_error": (ctypes.c_char_p, [vp]),
        "tdse_validate_desc": (i32, [ctypes.POINTER(Desc), dp]),
        "tdse_time_step_bound": (i32, [ctypes.POINTER(Desc), dbl, dbl, dp, dp]),
        "tdse_workspace_size": (i32, [ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_size_t)]),
        "tdse_create": (i32, [ctypes.POINTER(Desc), vp, ctypes.POINTER(vp)]),
        "tdse_destroy": (i32, [vp]),
        "tdse_bind": (i32, [vp, vp, vp, vp, vp, ctypes.c_size_t, vp, vp, vp]),
        "tdse_build_potential": (i32, [vp, ctypes.POINTER(Atom), i64, ctypes.POINTER(PotParams)]),
        "tdse_set_cap": (i32, [vp, dp, i64]),
        "tdse_set_cap_quadratic": (i32, [vp, i64, i64, dbl]),
        "tdse_finalize_setup": (i32, [vp, dp, dp]),
        "tdse_init_gaussian": (i32, [vp, dp, dp, dbl, i32]),
        "tdse_set_state": (i32, [vp, vp, vp, i64, dbl]),
        "tdse_get_state": (i32, [vp, vp, vp, ctypes.POINTER(i64), dp]),
        "tdse_step": (i32, [vp, i64]),
        "tdse_detect": (i32, [vp, ctypes.POINTER(DetectOut)]),
        "tdse_copy_scalars": (i32, [vp, dp, i64]),
        "tdse_set_timing": (i32, [vp, i32]),
        "tdse_timing_read": (i32, [vp, dp, ctypes.POINTER(i64)]),
        "tdse_timing_read_split": (i32, [vp, dp, ctypes.POINTER(i64)]),
        "tdse_bind_pingpong": (i32, [vp, vp, vp]),
        "tdse_adjoint_workspace_size": (i32, [ctypes.POINTER(Desc), i64, i32,
                                              ctypes.POINTER(ctypes.c_size_t)]),
        "tdse_bind_adjoint": (i32, [vp, vp, ctypes.c_size_t, i64, i32]),
        "tdse_adjoint": (i32, [vp, vp, vp, vp, vp]),
        "tdse_potential_vjp": (i32, [vp, ctypes.POINTER(Atom), i64, ctypes.POINTER(PotParams), vp,
                                     dp, dp]),
        "tdse_batch_create": (i32, [ctypes.POINTER(Desc), i32, vp, ctypes.POINTER(vp)]),
        "tdse_batch_member": (i32, [vp, i32, ctypes.POINTER(vp)]),
        "tdse_batch_bind": (i32, [vp, i32, vp, vp, vp, vp, ctypes.c_size_t, vp, vp, vp, vp, vp]),
        "tdse_batch_detect": (i32, [vp, i32, ctypes.POINTER(DetectOut)]),
        "tdse_batch_set_tile": (i32, [vp, i32, i32, i32, i32]),
        "tdse_batch_set_two_step": (i32, [vp, i32, i32, i32, i32, i32, i32]),
        "tdse_batch_workspace_size": (i32, [vp, ctypes.POINTER(ctypes.c_size_t)]),
        "tdse_batch_bind_workspace": (i32, [vp, vp, ctypes.c_size_t]),
        "tdse_batch_prepare": (i32, [vp]),
        "tdse_batch_run": (i32, [vp, i64]),
        "tdse_batch_status": (i32, [vp, ctypes.POINTER(i32)]),
        "tdse_batch_last_error": (ctypes.c_char_p, [vp]),
        "tdse_batch_destroy": (i32, [vp]),
        "tdse_get_tile": (i32, [vp, ctypes.POINTER(Tile)]),
        "tdse_set_tile": (i32, [vp, ctypes.POINTER(Tile)]),
        "tdse_autotune": (i32, [vp, i32, i32, ctypes.POINTER(Tile)]),
        "tdse_paper_layout_run": (i32, [vp, vp, vp, vp, i64, i32, i32, i32]),
        "tdse_hbm_probe": (i32, [i32, ctypes.POINTER(vp), i64, i32, i32, vp, dp]),
        "tdse_interpolate_potential": (i32, [vp, vp, i32, i32, i32, dp, dp]),
        "tdse_set_cap_paper": (i32, [vp, ctypes.c_double, ctypes.c_double]),
        "tdse_time_step_paper": (i32, [ctypes.POINTER(Desc), dp]),
        "tdse_dissimilarity_workspace_size": (i32, [i32, i32, ctypes.POINTER(ctypes.c_size_t)]),
        "tdse_dissimilarity": (i32, [i32, vp, i32, i32, i64, vp, ctypes.c_double, vp, vp,
                                     ctypes.c_size_t, vp]),
        "tdse_dissimilarity_noalloc": (i32, [i32, vp, i32, i32, i64, vp, ctypes.c_double, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def make_desc(nx, ny, nz, dx, dy, dz, hbar=1.0, mass=1.0, dt=0.0, dt_frac=0.9,
              bc=(BC_PERIODIC,) * 3, precision="f32", k_det=0, record_every=0, max_records=0,
              flags=0) -> Desc:
    d = Desc()
    d.nx, d.ny, d.nz = int(nx), int(ny), int(nz)
    d.dx, d.dy, d.dz = float(dx), float(dy), float(dz)
    d.hbar, d.mass = float(hbar), float(mass)
    d.dt, d.dt_frac = float(dt), float(dt_frac)
    d.bc = (ctypes.c_int32 * 3)(*[int(b) for b in bc])
    d.precision = F64 if precision in ("f64", F64) else F32
    d.k_det, d.record_every, d.max_records = int(k_det), int(record_every), int(max_records)
    d.flags = int(flags)
    return d


def validate_desc(d: Desc) -> int:
    return int(load().tdse_validate_desc(ctypes.byref(d), None))


def validate_desc_bound(d: Desc):
    """(status, dt bound for V = 0) of tdse_validate_desc."""
    b = ctypes.c_double()
    st = int(load().tdse_validate_desc(ctypes.byref(d), ctypes.byref(b)))
    return st, b.value


def time_step_bound(d: Desc, vmin: float, vmax: float):
    em, dtb = ctypes.c_double(), ctypes.c_double()
    st = load().tdse_time_step_bound(ctypes.byref(d), float(vmin), float(vmax), ctypes.byref(em),
                                     ctypes.byref(dtb))
    if st != OK:
        raise TdseError(st, status_string(st))
    return em.value, dtb.value


def workspace_size(d: Desc) -> int:
    n = ctypes.c_size_t()
    st = load().tdse_workspace_size(ctypes.byref(d), ctypes.byref(n))
    if st != OK:
        raise TdseError(st, status_string(st))
    return int(n.value)


def status_string(st: int) -> str:
    return load().tdse_status_string(int(st)).decode()


def wavevector(energy: float, hbar: float, mass: float) -> float:
    """|k| for kinetic energy E (eq. (4): lambda = sqrt(2 hbar^2 pi^2 / (m E)))."""
    return float(np.sqrt(2.0 * mass * energy) / hbar)


@dataclass
class Detect:
    step: int
    n_records: int
    flux: float
    dt: float
    e_max: float


class Sim:
    """One FDTD simulation on the current CUDA (HIP) device.

    Owns the torch tensors it binds: psi_r, psi_i, v ([nz][ny][nx]), the
    workspace, the records [max_records][ny][nx], the FP64 record scalars
    [max_records][4] and optionally the FP64 pixel integral [ny][nx]."""

    def __init__(self, desc: Desc, device=None, stream=None, pingpong=True, handle=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libtdse needs a HIP device")
        self.torch = torch
        self.lib = load()
        self.desc = desc
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        dt = torch.float64 if desc.precision == F64 else torch.float32
        self.dtype = dt
        shape = (desc.nz, desc.ny, desc.nx)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream()
            self.psi_r = torch.zeros(shape, dtype=dt, device=self.device)
            self.psi_i = torch.zeros(shape, dtype=dt, device=self.device)
            self.v = torch.zeros(shape, dtype=dt, device=self.device)
            self.workspace = torch.zeros(workspace_size(desc), dtype=torch.uint8,
                                         device=self.device)
            nrec = max(int(desc.max_records), 1)
            self.records = torch.zeros((nrec, desc.ny, desc.nx), dtype=dt, device=self.device)
            self.scalars = torch.zeros((nrec, 4), dtype=torch.float64, device=self.device)
            self.pixel = (torch.zeros((desc.ny, desc.nx), dtype=torch.float64, device=self.device)
                          if desc.flags & FLAG_PIXEL_INTEGRAL else None)
            if handle is None:
                h = ctypes.c_void_p()
                self._check(self.lib.tdse_create(ctypes.byref(desc),
                                                 ctypes.c_void_p(self.stream.cuda_stream),
                                                 ctypes.byref(h)), None)
                self.owned = True
            else:
                h = handle
                self.owned = False
            self.h = h
            self._check(self.lib.tdse_bind(
                self.h, self.psi_r.data_ptr(), self.psi_i.data_ptr(), self.v.data_ptr(),
                self.workspace.data_ptr(), self.workspace.numel(), self.records.data_ptr(),
                self.scalars.data_ptr(), self.pixel.data_ptr() if self.pixel is not None else None))
            self.psi_r2 = self.psi_i2 = None
            if pingpong:
                self.psi_r2 = torch.empty(shape, dtype=dt, device=self.device)
                self.psi_i2 = torch.empty(shape, dtype=dt, device=self.device)
                self._check(self.lib.tdse_bind_pingpong(self.h, self.psi_r2.data_ptr(),
                                                        self.psi_i2.data_ptr()))
        self.dt = None
        self.e_max = None

    # -- plumbing --------------------------------------------------------
    def _check(self, st, h="self"):
        if st != OK:
            handle = self.h if h == "self" else h
            msg = self.lib.tdse_last_error(handle).decode() if handle else ""
            raise TdseError(st, f"{status_string(st)}: {msg}")

    def close(self):
        if getattr(self, "h", None):
            if getattr(self, "owned", True):
                self.lib.tdse_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup -------------------------------------------------------------
    def build_potential(self, atoms: np.ndarray, soft=0.1, cutoff=6.0, kappa=14.3996454784,
                        a0=0.529177210903, screened=True):
        atoms = np.ascontiguousarray(atoms, dtype=np.float64).reshape(-1, 5)
        arr = (Atom * max(len(atoms), 1))()
        for i, a in enumerate(atoms):
            arr[i] = Atom(*[float(x) for x in a])
        p = PotParams(float(soft), float(cutoff), float(kappa), float(a0), int(bool(screened)), 0)
        self._check(self.lib.tdse_build_potential(self.h, arr, len(atoms), ctypes.byref(p)))

    def interpolate_potential(self, table, spacing, origin=(0.0, 0.0, 0.0)):
        """Fill V by trilinear interpolation of a unit-cell table [uz][uy][ux]
        (FP64; a numpy array or a device tensor), periodic in x and y."""
        import torch
        t = torch.as_tensor(table, dtype=torch.float64).to(self.device).contiguous()
        uz, uy, ux = t.shape
        sp = (ctypes.c_double * 3)(*[float(x) for x in spacing])
        org = (ctypes.c_double * 3)(*[float(x) for x in origin])
        with torch.cuda.device(self.device):
            cur = torch.cuda.current_stream(self.device)
            if self.stream != cur:
                self.stream.wait_stream(cur)   # the table as written on torch's stream
            self._check(self.lib.tdse_interpolate_potential(self.h, ctypes.c_void_p(t.data_ptr()),
                                                            ux, uy, uz, sp, org))
            # the table's memory is not reused before the launch has read it
            t.record_stream(self.stream)
            if self.stream != cur:
                cur.wait_stream(self.stream)   # torch work queued next sees V

    def set_cap(self, w: Optional[np.ndarray]):
        if w is None:
            self._check(self.lib.tdse_set_cap(self.h, None, self.desc.nz))
            return
        w = np.ascontiguousarray(w, dtype=np.float64)
        self._check(self.lib.tdse_set_cap(
            self.h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(w)))

    def set_cap_paper(self, alpha: float, r_cut: float):
        """Eq. (10) as printed: W_k = (alpha / dz) (r_cut - k dz)^2 below r_cut."""
        self._check(self.lib.tdse_set_cap_paper(self.h, float(alpha), float(r_cut)))

    def set_cap_quadratic(self, n_bottom: int, n_top: int, w_max: float):
        self._check(self.lib.tdse_set_cap_quadratic(self.h, int(n_bottom), int(n_top),
                                                    float(w_max)))

    def finalize(self):
        dt, em = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.tdse_finalize_setup(self.h, ctypes.byref(dt), ctypes.byref(em)))
        self.dt, self.e_max = dt.value, em.value
        return self.dt, self.e_max

    def init_gaussian(self, r0, k0, sigma, mode=INIT_HALFSTEP):
        r = (ctypes.c_double * 3)(*[float(x) for x in r0])
        k = (ctypes.c_double * 3)(*[float(x) for x in k0])
        self._check(self.lib.tdse_init_gaussian(self.h, r, k, float(sigma), int(mode)))

    def set_state(self, psi_r, psi_i, step=0, flux=0.0):
        t = self.torch
        pr = psi_r.to(self.device, self.dtype).contiguous()
        pi = psi_i.to(self.device, self.dtype).contiguous()
        self._keep = (pr, pi)  # alive until the asynchronous copy has run
        t.cuda.synchronize(self.device)  # the copies above ran on torch's stream
        self._check(self.lib.tdse_set_state(self.h, pr.data_ptr(), pi.data_ptr(), int(step),
                                            float(flux)))
        t.cuda.current_stream(self.device).synchronize()

    def get_state(self):
        step, flux = ctypes.c_int64(), ctypes.c_double()
        self._check(self.lib.tdse_get_state(self.h, None, None, ctypes.byref(step),
                                            ctypes.byref(flux)))
        return self.psi_r.clone(), self.psi_i.clone(), step.value, flux.value

    # -- run -----------------------------------------------------------
    def step(self, n: int):
        self._check(self.lib.tdse_step(self.h, int(n)))

    def detect(self) -> Detect:
        o = DetectOut()
        self._check(self.lib.tdse_detect(self.h, ctypes.byref(o)))
        return Detect(int(o.step), int(o.n_records), float(o.flux_acc), float(o.dt),
                      float(o.e_max))

    def records_host(self):
        d = self.detect()
        n = d.n_records
        return (self.records[:n].double().cpu().numpy(), self.scalars[:n].cpu().numpy())

    # -- adjoint -----------------------------------------------------------
    def bind_adjoint(self, n_steps: int, ckpt_every: int = 100):
        """Allocate and attach the adjoint workspace; the next n_steps steps
        (from level 0) store checkpoints every ckpt_every steps."""
        n = ctypes.c_size_t()
        self._check(self.lib.tdse_adjoint_workspace_size(ctypes.byref(self.desc), int(n_steps),
                                                         int(ckpt_every), ctypes.byref(n)), None)
        self.adj_ws = self.torch.empty(int(n.value), dtype=self.torch.uint8, device=self.device)
        self._check(self.lib.tdse_bind_adjoint(self.h, self.adj_ws.data_ptr(), self.adj_ws.numel(),
                                               int(n_steps), int(ckpt_every)))

    def adjoint(self, dL_drho):
        """(dL/dV [nz][ny][nx] float64, dL/dpsiR^0, dL/dpsiI^{-1/2}) for a loss
        whose derivative with respect to the records is dL_drho."""
        t = self.torch
        rb = dL_drho.to(self.device, self.dtype).contiguous()
        shape = (self.desc.nz, self.desc.ny, self.desc.nx)
        gV = t.empty(shape, dtype=t.float64, device=self.device)
        gR = t.empty(shape, dtype=self.dtype, device=self.device)
        gI = t.empty(shape, dtype=self.dtype, device=self.device)
        self._check(self.lib.tdse_adjoint(self.h, rb.data_ptr(), gV.data_ptr(), gR.data_ptr(),
                                          gI.data_ptr()))
        return gV, gR, gI

    def potential_vjp(self, atoms: np.ndarray, dL_dV, soft=0.1, cutoff=6.0,
                      kappa=14.3996454784, a0=0.529177210903, screened=True):
        """(dL/dpositions [n][3], dL/damplitudes [n]) as numpy arrays."""
        atoms = np.ascontiguousarray(atoms, dtype=np.float64).reshape(-1, 5)
        arr = (Atom * max(len(atoms), 1))()
        for i, a in enumerate(atoms):
            arr[i] = Atom(*[float(x) for x in a])
        p = PotParams(float(soft), float(cutoff), float(kappa), float(a0), int(bool(screened)), 0)
        gv = dL_dV.to(self.device, self.torch.float64).contiguous()
        dpos = np.zeros((len(atoms), 3))
        damp = np.zeros(len(atoms))
        dp_ = ctypes.POINTER(ctypes.c_double)
        self._check(self.lib.tdse_potential_vjp(self.h, arr, len(atoms), ctypes.byref(p),
                                                gv.data_ptr(), dpos.ctypes.data_as(dp_),
                                                damp.ctypes.data_as(dp_)))
        return dpos, damp

    # -- measurement / tuning ------------------------------------------------
    def set_timing(self, on: bool):
        self._check(self.lib.tdse_set_timing(self.h, int(bool(on))))

    def timing_read(self):
        """{kind: (ms, launches)} for 'half_i', 'half_r', 'fused', 'two_step'
        since the last read."""
        ms = (ctypes.c_double * 4)()
        n = (ctypes.c_int64 * 4)()
        self._check(self.lib.tdse_timing_read(self.h, ms, n))
        return {k: (ms[i], n[i]) for i, k in enumerate(("half_i", "half_r", "fused", "two_step"))}

    def timing_read_split(self):
        """As timing_read, with the launches that write a record under the
        same names plus '_rec'."""
        ms = (ctypes.c_double * 8)()
        n = (ctypes.c_int64 * 8)()
        self._check(self.lib.tdse_timing_read_split(self.h, ms, n))
        names = ("half_i", "half_r", "fused", "two_step")
        names = names + tuple(k + "_rec" for k in names)
        return {k: (ms[i], n[i]) for i, k in enumerate(names)}

    def autotune(self, steps: int = 10, flags: int = 0) -> Tile:
        """Library autotuner: times its candidate tiles on this grid, keeps the
        fastest.  The state is spent (set a new one before stepping)."""
        t = Tile()
        self._check(self.lib.tdse_autotune(self.h, int(steps), int(flags), ctypes.byref(t)))
        return t

    def paper_layout_run(self, psi_r, psi_i, v, n: int, block=(16, 4, 4)):
        """n steps of the section 2.2 design on z-fastest arrays [nx][ny][nz]
        (this handle's grid, coefficients and CAP; its own state untouched);
        block = (Bx, By, Bz) with Bx along z."""
        for a in (psi_r, psi_i, v):
            if (a.dtype != self.dtype or a.device != self.psi_r.device or not a.is_contiguous()
                    or tuple(a.shape) != (self.desc.nx, self.desc.ny, self.desc.nz)):
                raise ValueError("arrays must be contiguous [nx][ny][nz] of the handle's dtype "
                                 "and device")
        bx, by, bz = (int(b) for b in block)
        self._check(self.lib.tdse_paper_layout_run(self.h, psi_r.data_ptr(), psi_i.data_ptr(),
                                                   v.data_ptr(), int(n), bx, by, bz))

    def get_tile(self) -> Tile:
        t = Tile()
        self._check(self.lib.tdse_get_tile(self.h, ctypes.byref(t)))
        return t

    def set_tile(self, rows=None, waves=None, zc=None, fused=None, fused_rows=None,
                 fused_zc=None, fused_prefetch=None, graph=None, fused_threads=None,
                 two_step=None, two_step_tx=None, two_step_rows=None, two_step_zc=None,
                 two_step_prefetch=None, two_step_threads=None, two_step_ty=None):
        """Replace some tile fields, keep the rest.  two_step_ty: the sweep's
        interior tile height (0 = the tallest its threads cover); when the
        sweep's shape changes and no height is given, the tallest."""
        t = self.get_tile()
        shape = (two_step_tx, two_step_rows, two_step_threads)
        if two_step_ty is None and any(v is not None for v in shape):
            two_step_ty = 0
        for name, v in (("rows", rows), ("waves", waves), ("zc", zc), ("fused", fused),
                        ("fused_rows", fused_rows), ("fused_zc", fused_zc),
                        ("fused_prefetch", fused_prefetch), ("graph", graph),
                        ("fused_threads", fused_threads), ("two_step", two_step),
                        ("two_step_tx", two_step_tx), ("two_step_rows", two_step_rows),
                        ("two_step_zc", two_step_zc), ("two_step_prefetch", two_step_prefetch),
                        ("two_step_threads", two_step_threads), ("two_step_ty", two_step_ty)):
            if v is not None:
                setattr(t, name, int(v))
        self._check(self.lib.tdse_set_tile(self.h, ctypes.byref(t)))


def hbm_probe(kind: str = "copy", gib: float = 1.0, grid: int = 0, reps: int = 5, device=None):
    """Practical HBM bandwidth of the device in GB/s: 'copy' (one read and
    one written stream), 'mix' (the one-pass step's three read and two
    written streams) or 'fill' (one written stream), over buffers of `gib`
    GiB each."""
    import torch
    lib = load()
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    n = int(gib * (1 << 30)) // 16 * 4
    k = {"copy": 0, "mix": 1, "fill": 2}[kind]
    bufs = [torch.ones(n, dtype=torch.float32, device=dev) for _ in range((2, 5, 1)[k])]
    ptrs = (ctypes.c_void_p * len(bufs))(*[b.data_ptr() for b in bufs])
    ms = ctypes.c_double()
    stream = torch.cuda.current_stream(dev).cuda_stream
    st = lib.tdse_hbm_probe(k, ptrs, n, int(grid), int(reps), ctypes.c_void_p(stream), ctypes.byref(ms))
    if st != OK:
        raise TdseError(st, lib.tdse_status_string(st).decode())
    nbytes = len(bufs) * n * 4
    del bufs
    return nbytes / (ms.value * 1e-3) / 1e9


def time_step_paper(desc) -> float:
    """Eq. (11): m min(dx, dy, dz)^2 / (5 hbar) for the description's grid."""
    lib = load()
    dt = ctypes.c_double()
    st = lib.tdse_time_step_paper(ctypes.byref(desc), ctypes.byref(dt))
    if st != OK:
        raise TdseError(st, lib.tdse_status_string(st).decode())
    return dt.value


def dissimilarity(frames, weights, dA: float):
    """d_kj of eq. (16) on the GPU: frames [K][T][P] (a float32 or float64
    CUDA tensor), time-quadrature weights [T] (with the 1 / (t1 - t0)), pixel
    area dA.  Returns a [K][K] float64 CUDA tensor."""
    import torch
    lib = load()
    if frames.dim() != 3 or not frames.is_cuda:
        raise ValueError("frames must be a [K][T][P] CUDA tensor")
    prec = {torch.float32: F32, torch.float64: F64}[frames.dtype]
    frames = frames.contiguous()
    K, T, P = frames.shape
    dev = frames.device
    w = torch.as_tensor(weights, dtype=torch.float64).to(dev).contiguous()
    if w.shape != (T,):
        raise ValueError("weights must have one entry per frame")
    nb = ctypes.c_size_t()
    st = lib.tdse_dissimilarity_workspace_size(K, T, ctypes.byref(nb))
    if st != OK:
        raise TdseError(st, lib.tdse_status_string(st).decode())
    ws = torch.empty(max(1, nb.value // 8), dtype=torch.float64, device=dev)
    out = torch.empty((K, K), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    st = lib.tdse_dissimilarity(prec, ctypes.c_void_p(frames.data_ptr()), K, T, P,
                                ctypes.c_void_p(w.data_ptr()), float(dA),
                                ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                nb.value, ctypes.c_void_p(stream))
    if st != OK:
        raise TdseError(st, lib.tdse_status_string(st).decode())
    return out


# TDSE_DISSIM_NOALLOC_MAX_BYTES of include/tdse.h
DISSIM_NOALLOC_MAX_BYTES = 64 << 20


def dissimilarity_noalloc(frames, weights, dA: float, out=None):
    """d_kj of eq. (16) through tdse_dissimilarity_noalloc: the library's
    fixed per-GPU scratch instead of a workspace (for callers that cannot
    allocate; the binding itself allocates `out` unless one is given, a
    contiguous [K][K] float64 CUDA tensor).  frames and weights as for
    dissimilarity(); weights must already be a float64 CUDA tensor."""
    import torch
    lib = load()
    if frames.dim() != 3 or not frames.is_cuda or not frames.is_contiguous():
        raise ValueError("frames must be a contiguous [K][T][P] CUDA tensor")
    prec = {torch.float32: F32, torch.float64: F64}[frames.dtype]
    K, T, P = frames.shape
    if not (weights.is_cuda and weights.dtype == torch.float64 and weights.shape == (T,)
            and weights.is_contiguous()):
        raise ValueError("weights must be a contiguous float64 CUDA tensor of one entry per frame")
    if out is None:
        out = torch.empty((K, K), dtype=torch.float64, device=frames.device)
    elif not (out.is_cuda and out.dtype == torch.float64 and out.shape == (K, K) and out.is_contiguous()):
        raise ValueError("out must be a contiguous [K][K] float64 CUDA tensor")
    stream = torch.cuda.current_stream(frames.device).cuda_stream
    st = lib.tdse_dissimilarity_noalloc(prec, ctypes.c_void_p(frames.data_ptr()), K, T, P,
                                        ctypes.c_void_p(weights.data_ptr()), float(dA),
                                        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream))
    if st != OK:
        raise TdseError(st, lib.tdse_status_string(st).decode())
    return out


def sim_from_workload(w, precision: Optional[str] = None, steps: Optional[int] = None,
                      pixel=False, device=None, max_records: Optional[int] = None,
                      pingpong=True, stream=None) -> Sim:
    """Set up a simulation from a seeded workload description (potential on
    the device, CAP, dt, Gaussian packet)."""
    prec = precision or w.precision
    nsteps = w.steps if steps is None else steps
    nrec = w.n_records(nsteps) if max_records is None else max_records
    flags = FLAG_PIXEL_INTEGRAL if pixel else 0
    d = make_desc(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.hbar, w.mass, dt_frac=w.dt_frac,
                  bc=w.bc, precision=prec, k_det=w.k_det, record_every=w.record_every,
                  max_records=nrec, flags=flags)
    if w.dt_eq11:
        # eq. (11) exceeds the Gershgorin bound that finalize enforces
        d = make_desc(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.hbar, w.mass,
                      dt=time_step_paper(d), bc=w.bc, precision=prec, k_det=w.k_det,
                      record_every=w.record_every, max_records=nrec,
                      flags=flags | FLAG_ALLOW_UNSTABLE)
    s = Sim(d, device=device, pingpong=pingpong, stream=stream)
    if stream is not None:
        import torch
        torch.cuda.synchronize()
    if w.cell_table is not None:
        from .workloads import cell_table_of
        table, spacing, origin = cell_table_of(w)
        s.interpolate_potential(table, spacing, origin)
    if w.atoms is not None and len(w.atoms):
        s.build_potential(w.atoms, soft=w.soft, cutoff=w.cutoff, kappa=w.kappa, a0=w.a0,
                          screened=w.screened)
    if w.cap_paper is not None:
        s.set_cap_paper(*w.cap_paper)
    if w.cap is not None:
        s.set_cap_quadratic(*w.cap)
    s.finalize()
    if w.k0 is not None:
        k0 = w.k0
    else:
        kk = wavevector(w.energy, w.hbar, w.mass)
        k0 = tuple(kk * c for c in w.k_dir)
    s.init_gaussian(w.r0, k0, w.sigma)
    return s


class Batch:
    """Many simulations of uneven grid size stepped together (one launch per
    step for all of them, one HIP graph per record interval).  Members are
    Sim objects sharing the batch's stream; set each one up with the usual
    calls, then prepare() and run()."""

    def __init__(self, descs, device=None):
        import torch
        self.torch = torch
        self.lib = load()
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self.stream = torch.cuda.Stream(device=self.device)
        arr = (Desc * len(descs))(*descs)
        b = ctypes.c_void_p()
        st = self.lib.tdse_batch_create(arr, len(descs), ctypes.c_void_p(self.stream.cuda_stream),
                                        ctypes.byref(b))
        if st != OK:
            raise TdseError(st, f"{status_string(st)}: batch_create")
        self.b = b
        self.members = []
        for i, d in enumerate(descs):
            h = ctypes.c_void_p()
            self._check(self.lib.tdse_batch_member(self.b, i, ctypes.byref(h)))
            self.members.append(Sim(d, device=self.device, stream=self.stream, handle=h))
        # the batch's device tables: caller-owned memory bound to the batch
        nb = ctypes.c_size_t()
        self._check(self.lib.tdse_batch_workspace_size(self.b, ctypes.byref(nb)))
        self.ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        self._check(self.lib.tdse_batch_bind_workspace(self.b, ctypes.c_void_p(self.ws.data_ptr()),
                                                       int(nb.value)))
        torch.cuda.synchronize(self.device)

    def _check(self, st):
        if st != OK:
            raise TdseError(st, f"{status_string(st)}: {self.lib.tdse_batch_last_error(self.b).decode()}")

    def set_tile(self, fused_rows=3, fused_zc=64, prefetch=False, threads=256):
        self._check(self.lib.tdse_batch_set_tile(self.b, int(fused_rows), int(fused_zc),
                                                 int(bool(prefetch)), int(threads)))

    def set_two_step(self, enable=True, tx=80, zc=32, prefetch=True, rows=1, threads=1024):
        """Two-step sweeps for the whole batch where every member fits them."""
        self._check(self.lib.tdse_batch_set_two_step(self.b, int(bool(enable)), int(tx), int(rows),
                                                     int(zc), int(bool(prefetch)), int(threads)))

    def prepare(self):
        self.torch.cuda.synchronize(self.device)
        self._check(self.lib.tdse_batch_prepare(self.b))

    def run(self, n: int):
        self._check(self.lib.tdse_batch_run(self.b, int(n)))

    def status(self):
        out = (ctypes.c_int32 * len(self.members))()
        self.lib.tdse_batch_status(self.b, out)
        return list(out)

    def close(self):
        if getattr(self, "b", None):
            for m in self.members:
                m.h = None
            self.lib.tdse_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_from_workloads(ws, precision="f32", steps=None, device=None) -> Batch:
    """A batch whose members are set up from seeded workload descriptions."""
    descs = []
    for w in ws:
        n = w.steps if steps is None else steps
        descs.append(make_desc(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.hbar, w.mass,
                               dt_frac=w.dt_frac, bc=w.bc, precision=precision, k_det=w.k_det,
                               record_every=w.record_every, max_records=w.n_records(n)))
    b = Batch(descs, device=device)
    for w, s in zip(ws, b.members):
        with b.torch.cuda.stream(b.stream):
            if w.atoms is not None and len(w.atoms):
                s.build_potential(w.atoms, soft=w.soft, cutoff=w.cutoff, kappa=w.kappa, a0=w.a0,
                                  screened=w.screened)
            if w.cap is not None:
                s.set_cap_quadratic(*w.cap)
            s.finalize()
            k0 = w.k0 if w.k0 is not None else tuple(wavevector(w.energy, w.hbar, w.mass) * c
                                                     for c in w.k_dir)
            s.init_gaussian(w.r0, k0, w.sigma)
    b.torch.cuda.synchronize(b.device)
    return b
