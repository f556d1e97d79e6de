"""GPU parity at the configurations' own run lengths (arXiv 2401.07416,
section 2.1, eqs. (8)-(10) and (15); section 2.3 runs 8000 and 5000 steps):
the surface-diffraction physics on its 64x64x128 box for 20,000 steps with a
record every 50 steps (401 records), compared with the FP64 oracle at 2k,
5k, 10k and 20k steps, and the full 256x256x512 grid after 1,000 steps, both
precisions, on two-step sweeps (the plan the library takes on large grids;
the 64x64x128 box is given the 1024-thread sweep tile of the headline grid's
kernel at a narrower width, the full grid runs its tuned tile).  Tolerances as
everywhere: FP64 relative L2 <= 1e-11 (state, records), FP64 sums <= 1e-12;
FP32 state <= 1e-4, records <= 1e-3.  The printed error at each checkpoint
shows how the FP32 rounding error grows with the step count."""
import sys

import pytest

from paper_2401_07416_amd import workloads
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu

FP64 = dict(tol_state=1e-11, tol_rec=1e-11, tol_scal=1e-12, tol_flux=1e-12)
FP32 = dict(tol_state=1e-4, tol_rec=1e-3, tol_scal=1e-4, tol_flux=1e-5)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_in_checkpoints(w, prec, checkpoints, tile):
    from paper_2401_07416_amd import tdse
    g, V, W, dt, R, I = H.oracle_setup(w)
    import oracle
    ref = oracle.Sim(g, V, R, I, dt, W=W, k_det=w.k_det, record_every=w.record_every,
                     max_records=w.n_records(checkpoints[-1]), pixel=True)
    ref.record0()
    gpu = tdse.sim_from_workload(w, precision=prec, steps=checkpoints[-1], pixel=True)
    gpu.set_tile(**tile)
    assert gpu.get_tile().two_step == 1
    done = 0
    rows = []
    for c in checkpoints:
        ref.step(c - done)
        gpu.step(c - done)
        done = c
        res = H.compare(gpu, ref, **(FP64 if prec == "f64" else FP32))
        pix = H.rel_l2(gpu.pixel.cpu().numpy(), ref.pixel)
        assert pix <= (1e-11 if prec == "f64" else 1e-3), pix
        res["pixel"] = pix
        say(f"{w.name} {prec} after {c} steps:",
            {k: float(f"{v:.3e}") for k, v in res.items()})
        rows.append((c, res))
    return rows


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_surface_physics_20000_steps(prec):
    w = workloads.c2_reduced().with_(steps=20000, record_every=50)
    say("surface physics 64x64x128", prec, "20000 steps, h = 50")
    tile = dict(fused=1, two_step=1, two_step_tx=32, two_step_rows=1, two_step_zc=32,
                two_step_prefetch=1, two_step_threads=1024)
    rows = run_in_checkpoints(w, prec, [2000, 5000, 10000, 20000], tile)
    assert rows[-1][0] == 20000


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_full_surface_grid_1000_steps(prec):
    w = workloads.c2_surface().with_(steps=1000)
    say("surface 256x256x512", prec, "1000 steps, h = 50")
    from paper_2401_07416_amd import tuning
    run_in_checkpoints(w, prec, [1000], tuning.tile_for(w, prec))
