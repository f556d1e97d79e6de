"""torch.autograd bridge for gradients of detection-plane losses with respect
to the atoms of the synthetic potential (positions and amplitudes).

Forward: build V from the atoms on the device, run the leapfrog with
checkpoints, return the time-integrated detection intensity
P_ij = h dt sum_m rho^m_ij (FP64, [ny][nx]).  Backward: dL/drho^m = h dt dL/dP
for every record m, the library's reverse sweep gives dL/dV, and the
potential chain rule gives dL/dpositions and dL/damplitudes.  All arithmetic
runs in libtdse; this module only moves tensors.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import tdse


@dataclass
class Problem:
    """A fixed simulation setup whose potential comes from the atoms: the
    workload (grid, CAP, packet, records), the species, an absolute time
    step (so dt does not move with the atoms) and the checkpoint interval.
    Moved atoms can deepen a well past the bound that fixed dt; the
    leapfrog's own limit is twice that bound, so the simulations accept it
    (TDSE_FLAG_ALLOW_UNSTABLE)."""
    workload: object
    Z: np.ndarray
    dt: float
    precision: str = "f32"
    ckpt_every: int = 100

    def make_sim(self) -> tdse.Sim:
        w = self.workload
        d = tdse.make_desc(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.hbar, w.mass, dt=self.dt,
                           bc=w.bc, precision=self.precision, k_det=w.k_det,
                           record_every=w.record_every, max_records=w.n_records(),
                           flags=tdse.FLAG_PIXEL_INTEGRAL | tdse.FLAG_ALLOW_UNSTABLE)
        return tdse.Sim(d)

    def k0(self):
        w = self.workload
        if w.k0 is not None:
            return w.k0
        k = tdse.wavevector(w.energy, w.hbar, w.mass)
        return tuple(k * c for c in w.k_dir)


def problem_for(w, precision="f32", ckpt_every=100) -> Problem:
    """Problem with the time step of the workload's own atoms."""
    d = tdse.make_desc(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.hbar, w.mass, dt_frac=w.dt_frac,
                       bc=w.bc, precision=precision, k_det=w.k_det)
    s = tdse.Sim(d, pingpong=False)
    s.build_potential(w.atoms, soft=w.soft, cutoff=w.cutoff, kappa=w.kappa, a0=w.a0,
                      screened=w.screened)
    dt, _ = s.finalize()
    s.close()
    return Problem(w, np.asarray(w.atoms[:, 3], dtype=np.float64), dt, precision, ckpt_every)


def forward_sim(problem: Problem, atoms: np.ndarray, adjoint=True) -> tdse.Sim:
    w = problem.workload
    sim = problem.make_sim()
    sim.build_potential(atoms, soft=w.soft, cutoff=w.cutoff, kappa=w.kappa, a0=w.a0,
                        screened=w.screened)
    if w.cap is not None:
        sim.set_cap_quadratic(*w.cap)
    sim.finalize()
    sim.init_gaussian(w.r0, problem.k0(), w.sigma)
    if adjoint:
        sim.bind_adjoint(w.steps, problem.ckpt_every)
    sim.step(w.steps)
    return sim


class DetectionIntegral(torch.autograd.Function):
    @staticmethod
    def forward(ctx, positions, amplitudes, problem: Problem):
        atoms = np.column_stack([positions.detach().cpu().double().numpy(), problem.Z,
                                 amplitudes.detach().cpu().double().numpy()])
        sim = forward_sim(problem, atoms, adjoint=True)
        ctx.sim, ctx.atoms, ctx.problem = sim, atoms, problem
        ctx.dev = positions.device
        return sim.pixel.clone().to(positions.device)

    @staticmethod
    def backward(ctx, dP):
        sim, w = ctx.sim, ctx.problem.workload
        nrec = w.n_records()
        g = (w.record_every * sim.dt) * dP.to(sim.device, torch.float64)
        rho_bar = g.unsqueeze(0).expand(nrec, w.ny, w.nx).contiguous()
        gV, _, _ = sim.adjoint(rho_bar)
        dpos, damp = sim.potential_vjp(ctx.atoms, gV, soft=w.soft, cutoff=w.cutoff,
                                       kappa=w.kappa, a0=w.a0, screened=w.screened)
        ctx.sim = None
        sim.close()
        return (torch.from_numpy(dpos).to(ctx.dev), torch.from_numpy(damp).to(ctx.dev), None)


def detection_integral(positions, amplitudes, problem: Problem):
    return DetectionIntegral.apply(positions, amplitudes, problem)
