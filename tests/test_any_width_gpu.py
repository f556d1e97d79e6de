"""GPU parity on x extents outside the vector half-step layout (nx = W G L
with L <= 64 lanes): section 2.3 lets the user choose the number of
divisions along each axis.  nx = 67 (a prime), 130 and 1100 run the
any-width half-step kernel for single steps and record 0, the one-pass step
where its band of whole rows fits LDS (nx = 67, 130), and the two-step sweep,
which tiles x, also where it does not (nx = 1100).  Against the FP64 oracle
at the usual tolerances, and bitwise across the step paths (the cell
arithmetic is shared)."""
import sys

import numpy as np
import pytest

from paper_2401_07416_amd import workloads
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu

FP64 = dict(tol_state=1e-11, tol_rec=1e-11, tol_scal=1e-12, tol_flux=1e-12)
FP32 = dict(tol_state=1e-4, tol_rec=1e-3, tol_scal=1e-4, tol_flux=1e-5)
SWEEP = dict(fused=1, two_step=1, two_step_tx=16, two_step_rows=1, two_step_zc=20,
             two_step_prefetch=1, two_step_threads=1024)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def case(nx, prec, ny=13, nz=30, steps=61):
    return workloads.ragged(prec).with_(nx=nx, ny=ny, nz=nz, steps=steps)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nx", [67, 130])
def test_any_width_paths_vs_oracle(nx, prec):
    w = case(nx, prec)
    tol = FP64 if prec == "f64" else FP32
    say("any width", nx, prec)
    ref = H.oracle_run(w, w.steps)
    runs = {}
    for name, kw in (("half-steps", dict(pingpong=False)), ("one-pass", dict(tile=dict(fused=1, two_step=0))),
                     ("two-step", dict(tile=SWEEP))):
        g = H.gpu_run(w, w.steps, precision=prec, **kw)
        assert g.get_tile().lanes == 0, "no lane layout: the any-width half-step kernel"
        say(" ", name, H.compare(g, ref, **tol))
        runs[name] = g
    a = runs["half-steps"]
    for name in ("one-pass", "two-step"):
        b = runs[name]
        assert bool((a.psi_r == b.psi_r).all()) and bool((a.psi_i == b.psi_i).all()), name
        np.testing.assert_array_equal(a.records_host()[0], b.records_host()[0])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_wide_rows_run_the_sweep_without_the_one_pass_band(prec):
    """nx = 1100: the one-pass band (whole rows, nx / W <= 256 threads) does
    not fit, the two-step sweep does; single steps (record levels, the odd
    last step) are half-steps."""
    w = case(1100, prec, ny=64, nz=30, steps=57)
    say("nx 1100", prec)
    ref = H.oracle_run(w, w.steps)
    g = H.gpu_run(w, w.steps, precision=prec, tile=dict(SWEEP, two_step_tx=56))
    t = g.get_tile()
    assert t.two_step == 1 and t.lanes == 0
    say(" ", H.compare(g, ref, **(FP64 if prec == "f64" else FP32)))
    h = H.gpu_run(w, w.steps, precision=prec, pingpong=False)
    assert bool((g.psi_r == h.psi_r).all()) and bool((g.psi_i == h.psi_i).all())
