"""Seeded synthetic workloads for the FDTD path (stand-ins for the paper's
DFT-derived Cu(111) and Au(111)-C6SAM systems of section 2.3).

This module only *describes* inputs: grid shapes, units, atom lists drawn
from seeded generators, packet parameters, CAP settings and run lengths.  It
holds none of the method's arithmetic (no potential values, no packet values,
no coefficients), so both the HIP library and the CPU oracle can consume the
same inputs while sharing no computation.

Units: ``ATOMIC`` uses hbar = m = 1 (bohr, hartree); ``EV_ANGSTROM`` uses eV,
Angstrom and fs with hbar = 0.6582119569 eV fs and the electron mass
m = hbar^2 / (7.619964 eV A^2).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

HBAR_EV_FS = 0.6582119569
HBAR2_OVER_ME = 7.619964
ME_EV_FS2_A2 = HBAR_EV_FS ** 2 / HBAR2_OVER_ME

PERIODIC = 0
ZERO = 1


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    hbar: float
    mass: float
    atoms: Optional[np.ndarray]          # [n][5] = x, y, z, Z, amplitude
    soft: float = 0.1                    # softening length s
    cutoff: float = 6.0
    screened: bool = True
    cap: Optional[Tuple[int, int, float]] = None   # (planes at bottom, planes at top, W_max)
    r0: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    sigma: float = 1.0
    energy: Optional[float] = None       # kinetic energy; wave vector along k_dir
    k_dir: Tuple[float, float, float] = (0.0, 0.0, -1.0)
    k0: Optional[Tuple[float, float, float]] = None  # explicit wave vector (overrides energy)
    dt_frac: float = 0.9
    steps: int = 100
    k_det: int = 0
    record_every: int = 0
    bc: Tuple[int, int, int] = (PERIODIC, PERIODIC, PERIODIC)
    precision: str = "f32"
    kappa: float = 14.3996454784
    a0: float = 0.529177210903
    notes: str = ""
    # potential from a unit-cell table instead of atoms: keyword arguments of
    # unit_cell_table plus "spacing" and "origin" of its samples
    cell_table: Optional[dict] = None
    cap_paper: Optional[Tuple[float, float]] = None  # eq. (10) as printed: (alpha, r_cut)
    dt_eq11: bool = False                # eq. (11) time step instead of dt_frac

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def n_records(self, steps: Optional[int] = None) -> int:
        s = self.steps if steps is None else steps
        return (s // self.record_every + 1) if self.record_every > 0 else 0

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def slab_atoms(seed: int, nsite_x: int, nsite_y: int, lx: float, ly: float, z_top: float,
               n_layers: int = 3, layer_gap: float = 2.5, species=(6, 8, 14),
               jitter: float = 0.05) -> np.ndarray:
    """Square slab of ``n_layers`` layers of nsite_x x nsite_y sites, the
    lattice stretched to lx/nsite_x so it stays periodic in the box; each site
    gets a species drawn uniformly from ``species`` and an isotropic Gaussian
    jitter of standard deviation ``jitter`` per coordinate."""
    rng = np.random.default_rng(seed)
    ax, ay = lx / nsite_x, ly / nsite_y
    out = []
    for layer in range(n_layers):
        z = z_top - layer * layer_gap
        for j in range(nsite_y):
            for i in range(nsite_x):
                out.append([(i + 0.5) * ax, (j + 0.5) * ay, z, 0.0, 1.0])
    atoms = np.array(out, dtype=np.float64)
    atoms[:, 3] = rng.choice(np.array(species, dtype=np.float64), size=atoms.shape[0])
    atoms[:, 0:3] += rng.normal(0.0, jitter, size=(atoms.shape[0], 3))
    return atoms


def tile_atoms(atoms: np.ndarray, lx: float, ly: float, rx: int, ry: int) -> np.ndarray:
    """Replicate an atom list rx x ry times in the xy plane."""
    parts = []
    for b in range(ry):
        for a in range(rx):
            t = atoms.copy()
            t[:, 0] += a * lx
            t[:, 1] += b * ly
            parts.append(t)
    return np.concatenate(parts, axis=0)


def c1_free_gaussian() -> Workload:
    """Free 3D Gaussian packet, atomic units, 64^3, dx = 0.2 bohr, periodic,
    V = 0, sigma = 2 bohr, k0 = (0, 0, 1.5), dt = 0.5 x bound, 200 steps."""
    return Workload(name="free-gaussian-64^3-fp64", nx=64, ny=64, nz=64, dx=0.2, dy=0.2,
                    dz=0.2, hbar=1.0, mass=1.0, atoms=None, r0=(6.4, 6.4, 6.4), sigma=2.0,
                    k0=(0.0, 0.0, 1.5), dt_frac=0.5, steps=200, k_det=48, record_every=10,
                    precision="f64")


def c2_surface(seed: int = 2401) -> Workload:
    """Electron diffraction from a synthetic 3-layer slab: 256x256x512 grid,
    dx = 0.2 A, Z in {6, 8, 14}, softening 0.1 A, 20x20 sites per layer
    (2.56 A), jitter 0.05 A, 24-plane CAP at both z ends (W_max = 50 eV),
    10 eV packet with sigma = 8 A at normal incidence, 20000 steps at
    0.9 x bound, detection plane every 50 steps."""
    L = 51.2
    atoms = slab_atoms(seed, 20, 20, L, L, z_top=36.0)
    return Workload(name="surface-256x256x512", nx=256, ny=256, nz=512, dx=0.2, dy=0.2,
                    dz=0.2, hbar=HBAR_EV_FS, mass=ME_EV_FS2_A2, atoms=atoms,
                    cap=(24, 24, 50.0), r0=(25.6, 25.6, 70.0), sigma=8.0, energy=10.0,
                    dt_frac=0.9, steps=20000, k_det=250, record_every=50)


def c2_reduced(seed: int = 2401) -> Workload:
    """The surface-diffraction physics on a 64x64x128 box (12.8 x 12.8 x 25.6 A):
    5x5 sites per layer, sigma = 2 A, 12-plane CAP, 2000 steps."""
    L = 12.8
    atoms = slab_atoms(seed, 5, 5, L, L, z_top=10.0)
    return Workload(name="surface-64x64x128", nx=64, ny=64, nz=128, dx=0.2, dy=0.2, dz=0.2,
                    hbar=HBAR_EV_FS, mass=ME_EV_FS2_A2, atoms=atoms, cap=(12, 12, 50.0),
                    r0=(6.4, 6.4, 18.0), sigma=2.0, energy=10.0, dt_frac=0.9, steps=2000,
                    k_det=70, record_every=20)


def c3_headline(seed: int = 2401) -> Workload:
    """Headline throughput run: 512x512x1024, FP32 state with FP64 reductions,
    the surface slab tiled 2x2 in xy, 32-plane CAP, 10 eV packet, 10000 steps."""
    base = slab_atoms(seed, 20, 20, 51.2, 51.2, z_top=36.0)
    atoms = tile_atoms(base, 51.2, 51.2, 2, 2)
    return Workload(name="surface-512x512x1024", nx=512, ny=512, nz=1024, dx=0.2, dy=0.2,
                    dz=0.2, hbar=HBAR_EV_FS, mass=ME_EV_FS2_A2, atoms=atoms,
                    cap=(32, 32, 50.0), r0=(51.2, 51.2, 70.0), sigma=8.0, energy=10.0,
                    dt_frac=0.9, steps=10000, k_det=250, record_every=50)


def c3_shard(gpus: int = 8, index: int = 1, seed: int = 2401) -> Workload:
    """One GPU's share of the 512x512x1024 headline grid split into z-slabs
    over `gpus` GPUs: slab `index` of 1024 / gpus planes, the same tiled
    surface atoms shifted into the slab's frame, periodic z standing in for
    the halo planes the neighbouring GPUs would send, no absorbing planes (an
    interior slab has none), the packet in the middle of the slab."""
    w = c3_headline(seed)
    nz = w.nz // gpus
    atoms = w.atoms.copy()
    atoms[:, 2] -= index * nz * w.dz
    return w.with_(name=f"shard{index}of{gpus}-512x512x{nz}", nz=nz, atoms=atoms, cap=None,
                   r0=(51.2, 51.2, 0.5 * nz * w.dz), k_det=nz // 2)


def c5_adjoint(seed: int = 5, nxy: int = 128, nz: int = 256, steps: int = 4000) -> Workload:
    """Adjoint-gradient workload: 128x128x256 (25.6 x 25.6 x 51.2 A), FP32
    forward, a 3 x 8 x 8 slab at a = 3.2 A (top layer z = 18 A, layers 2.5 A
    apart, Z in {6, 8, 14}), amplitudes 1, 24-plane CAP, 10 eV packet with
    sigma = 4 A at z = 34 A, detection plane at z = 26 A every 20 steps,
    4000 steps with checkpoints every 100."""
    L = 0.2 * nxy
    atoms = slab_atoms(seed, 8, 8, L, L, z_top=18.0)
    return Workload(name=f"adjoint-{nxy}x{nxy}x{nz}", nx=nxy, ny=nxy, nz=nz, dx=0.2, dy=0.2,
                    dz=0.2, hbar=HBAR_EV_FS, mass=ME_EV_FS2_A2, atoms=atoms,
                    cap=(24, 24, 50.0), r0=(L / 2, L / 2, 34.0), sigma=4.0, energy=10.0,
                    dt_frac=0.9, steps=steps, k_det=130, record_every=20)


def perturbed_positions(atoms: np.ndarray, seed: int = 6, scale: float = 0.05) -> np.ndarray:
    """The atom list with every coordinate moved by N(0, scale) (the target
    configuration of the adjoint workload)."""
    rng = np.random.default_rng(seed)
    out = atoms.copy()
    out[:, 0:3] += rng.normal(0.0, scale, size=(atoms.shape[0], 3))
    return out


def hydroxyhexyl() -> np.ndarray:
    """A rigid HO(CH2)6 chain (20 atoms: 6 C, 12 H, O, H) along +z from the
    origin, from textbook bond lengths (C-C 1.54, C-H 1.09, C-O 1.43,
    O-H 0.96 A) and tetrahedral angles: an all-trans zigzag in the xz plane
    with the methylene hydrogens above and below that plane.  Rows are
    x, y, z, Z."""
    half = np.deg2rad(109.47) / 2
    dz, dx = 1.54 * np.sin(half), 1.54 * np.cos(half) / 2
    out = []
    for c in range(6):
        x = dx if c % 2 else -dx
        z = c * dz
        out.append([x, 0.0, z, 6.0])
        # the two hydrogens point away from the chain, out of the zigzag plane
        hx = np.sign(x) * 1.09 * np.cos(np.deg2rad(54.75))
        hy = 1.09 * np.sin(np.deg2rad(54.75))
        out.append([x + hx, hy, z, 1.0])
        out.append([x + hx, -hy, z, 1.0])
    xo = -dx if 6 % 2 == 0 else dx
    zo = 5 * dz + 1.43 * np.sin(half)
    out.append([xo, 0.0, zo, 8.0])
    out.append([xo + 0.96 * np.cos(half), 0.0, zo + 0.96 * np.sin(half), 1.0])
    return np.array(out, dtype=np.float64)


def film_atoms(seed: int, lx: float, ly: float, z_base: float, n_side: int = 4,
               displacement: float = 0.2) -> np.ndarray:
    """Monolayer of rigid 20-atom molecules on an n_side x n_side lattice,
    each rotated in plane by an angle uniform in [0, 2 pi) and shifted by
    `displacement` in a uniform random direction; amplitudes 1."""
    rng = np.random.default_rng(seed)
    mol = hydroxyhexyl()
    out = []
    for j in range(n_side):
        for i in range(n_side):
            th = rng.uniform(0.0, 2 * np.pi)
            ph = rng.uniform(0.0, 2 * np.pi)
            c, s_ = np.cos(th), np.sin(th)
            x0 = (i + 0.5) * lx / n_side + displacement * np.cos(ph)
            y0 = (j + 0.5) * ly / n_side + displacement * np.sin(ph)
            for x, y, z, Z in mol:
                out.append([x0 + c * x - s_ * y, y0 + s_ * x + c * y, z_base + z, Z, 1.0])
    return np.array(out, dtype=np.float64)


def c4_film(b: int, steps: int = 8000) -> Workload:
    """Configuration b of the batched data-generation set: N_x = N_y =
    128 + 16 m (m uniform in 0..8, seed 7416 + b), N_z = 2 N_x, dx = 0.2 A; a
    4 x 4 film of HO(CH2)6 chains based at z = 0.25 L_z; 15 eV packet with
    sigma = min(8 A, L_z/16) at z = 0.65 L_z; detection at 0.55 L_z every 50
    steps; 24-plane CAP."""
    rng = np.random.default_rng(7416 + b)
    n = 128 + 16 * int(rng.integers(0, 9))
    nz = 2 * n
    L, Lz = 0.2 * n, 0.2 * nz
    atoms = film_atoms(7416 + b, L, L, 0.25 * Lz)
    return Workload(name=f"film-{b}-{n}x{n}x{nz}", nx=n, ny=n, nz=nz, dx=0.2, dy=0.2, dz=0.2,
                    hbar=HBAR_EV_FS, mass=ME_EV_FS2_A2, atoms=atoms, cap=(24, 24, 50.0),
                    r0=(L / 2, L / 2, 0.65 * Lz), sigma=min(8.0, Lz / 16), energy=15.0,
                    dt_frac=0.9, steps=steps, k_det=int(round(0.55 * nz)), record_every=50)


def c4_batch(n: int = 64, steps: int = 8000):
    return [c4_film(b, steps) for b in range(n)]


def ragged(precision: str = "f64", seed: int = 11) -> Workload:
    """Odd, non-power-of-two box (37 x 29 x 53) that leaves ragged tiles in
    every direction; a few atoms, a CAP and a packet."""
    rng = np.random.default_rng(seed)
    L = (37 * 0.2, 29 * 0.23, 53 * 0.21)
    atoms = np.zeros((6, 5))
    atoms[:, 0] = rng.uniform(0, L[0], 6)
    atoms[:, 1] = rng.uniform(0, L[1], 6)
    atoms[:, 2] = rng.uniform(3.0, 4.0, 6)
    atoms[:, 3] = rng.choice([6.0, 8.0, 14.0], 6)
    atoms[:, 4] = 1.0
    return Workload(name="ragged-37x29x53", nx=37, ny=29, nz=53, dx=0.2, dy=0.23, dz=0.21,
                    hbar=HBAR_EV_FS, mass=ME_EV_FS2_A2, atoms=atoms, cap=(6, 5, 40.0),
                    r0=(3.7, 3.3, 7.5), sigma=1.2, energy=12.0, dt_frac=0.9, steps=300,
                    k_det=20, record_every=7, precision=precision)


def unit_cell_table(seed: int = 7, ux: int = 24, uy: int = 28, uz: int = 360,
                    cell=(2.556, 4.427), z_top: float = 28.35, wells: int = 6, zs: float = 0.2):
    """Synthetic stand-in for a DFT potential of one surface unit cell (the
    paper's tables are DFT output, not available here): a table [uz][uy][ux]
    in eV on a cell of cell[0] x cell[1] A and uz planes zs A apart, with
    a few deep periodic wells per layer below z_top and a smooth decay into
    the vacuum above it.  Seeded; no part of the method."""
    rng = np.random.default_rng(seed)
    x = np.arange(ux) * cell[0] / ux
    y = np.arange(uy) * cell[1] / uy
    z = np.arange(uz) * zs
    X, Y = np.meshgrid(x, y)
    t = np.zeros((uz, uy, ux))
    for layer in range(4):
        zl = z_top - 2.1 * layer
        for _ in range(wells):
            cx, cy = rng.uniform(0, cell[0]), rng.uniform(0, cell[1])
            dx = (X - cx + cell[0] / 2) % cell[0] - cell[0] / 2
            dy = (Y - cy + cell[1] / 2) % cell[1] - cell[1] / 2
            r2 = dx ** 2 + dy ** 2
            depth = rng.uniform(20.0, 60.0)
            t -= depth * np.exp(-r2[None] / 0.18 - (z[:, None, None] - zl) ** 2 / 0.18)
    t -= 8.0 / (1.0 + np.exp((z - z_top) / 0.7))[:, None, None]
    return t


def cell_table_of(w: Workload):
    """(table, spacing, origin) of a workload whose potential comes from a
    unit-cell table."""
    kw = dict(w.cell_table)
    spacing, origin = kw.pop("spacing"), kw.pop("origin", (0.0, 0.0, 0.0))
    return unit_cell_table(**kw), spacing, origin


def paper_cu111(reduced: bool = False, seed: int = 7) -> Workload:
    """The paper's own set-up of section 2.1 / 2.3 (first set of runs): a
    40.9 x 40.9 x 70 A domain on a 240 x 240 x 420 grid, the surface
    potential of one cell repeated 15 x 15 and interpolated onto the mesh,
    100 planes appended at the bottom for the one-sided CAP of eq. (10),
    the eq. (11) time step, a 60 eV packet with sigma = 1.8 A at z = 42 A,
    the detector at 37.6 A, records every 20 steps, 8000 steps.  The DFT
    cell potential is replaced by the synthetic unit_cell_table; all z
    positions shift up by the appended 100 dz.  reduced: a 48 x 48 x (84 +
    20) grid over an 8.18 x 8.18 x 14 A domain (3 x 3 cells), 300 steps."""
    L, Lz = 40.9, 70.0
    n, nz, napp, cells = 240, 420, 100, 15
    if reduced:
        L, Lz, n, nz, napp, cells = 40.9 / 5, 14.0, 48, 84, 20, 3
    dx, dz = L / n, Lz / nz
    off = napp * dz
    cell = L / cells
    z_top = 28.35 if not reduced else 6.0
    uz = nz + napp
    table = dict(seed=seed, ux=24, uy=24, uz=uz, cell=(cell, cell), z_top=z_top + off, wells=4,
                 spacing=(cell / 24, cell / 24, dz), origin=(0.0, 0.0, 0.0))
    # the table's z planes sit at c * 0.2 in unit_cell_table; use the mesh spacing
    table["zs"] = dz
    z0 = (42.0 if not reduced else 10.5) + off
    zdet = (37.6 if not reduced else 9.0) + off
    alpha_rcut = 50.0 * dz / (napp * dz) ** 2  # W at the bottom plane = 50 eV
    return Workload(name=("paper-cu111-reduced-48x48x104" if reduced else "paper-cu111-240x240x520"),
                    nx=n, ny=n, nz=nz + napp, dx=dx, dy=dx, dz=dz, hbar=HBAR_EV_FS,
                    mass=ME_EV_FS2_A2, atoms=None, r0=(L / 2, L / 2, z0),
                    sigma=1.8 if not reduced else 1.2, energy=60.0, steps=8000 if not reduced else 300,
                    k_det=int(round(zdet / dz)), record_every=20, cell_table=table,
                    cap_paper=(alpha_rcut, napp * dz), dt_eq11=True,
                    notes="synthetic cell potential stands in for the DFT one")


def random_state(shape, seed: int):
    """Seeded smooth-ish random initial arrays (for pins that need generic data)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape), rng.standard_normal(shape)


ALL = {
    "free-gaussian": c1_free_gaussian,
    "surface": c2_surface,
    "surface-reduced": c2_reduced,
    "headline": c3_headline,
    "headline-shard8": c3_shard,
    "ragged": ragged,
    "adjoint": c5_adjoint,
    "paper-cu111": paper_cu111,
}
