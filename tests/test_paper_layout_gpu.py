"""GPU design of arXiv 2401.07416 section 2.2 (arrays z fastest, the eq. (12)
thread mapping, neighbours from global memory, one launch per half-step),
kept as the baseline this library's kernels are measured against.  Its cell
arithmetic is the library's, so n steps of it on the transposed state must
equal n library steps bit for bit, on ragged blocks, every boundary mix and
degenerate extents, and match the FP64 oracle to the usual tolerance."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2401_07416_amd import tdse, workloads
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def zfast(t):
    """[nz][ny][nx] -> [nx][ny][nz]"""
    return t.permute(2, 1, 0).contiguous()


def paper_vs_library(w, prec, steps, block, tile=None):
    s = tdse.sim_from_workload(w, precision=prec, steps=steps)
    if tile is not None:
        s.set_tile(**tile)
    R, I, V = zfast(s.psi_r), zfast(s.psi_i), zfast(s.v)
    s.paper_layout_run(R, I, V, steps, block)
    s.step(steps)
    torch.cuda.synchronize()
    return s, R, I


def assert_same(s, R, I):
    assert torch.equal(R.permute(2, 1, 0), s.psi_r)
    assert torch.equal(I.permute(2, 1, 0), s.psi_i)


BLOCKS = [(16, 4, 4), (16, 4, 2), (16, 8, 8), (7, 3, 5), (64, 1, 1), (1, 1, 1)]


@pytest.mark.parametrize("block", BLOCKS)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_paper_layout_equals_library_steps(prec, block):
    w = workloads.ragged(prec)
    say("paper layout ragged 37x29x53", prec, "block", block)
    s, R, I = paper_vs_library(w, prec, 40, block)
    assert_same(s, R, I)


@pytest.mark.parametrize("bc", [(1, 1, 1), (1, 0, 1), (0, 1, 0)])
def test_paper_layout_boundaries_and_oracle(bc):
    w = workloads.ragged("f64").with_(bc=bc)
    say("paper layout ragged f64 bc", bc)
    s, R, I = paper_vs_library(w, "f64", w.steps, (16, 4, 4))
    assert_same(s, R, I)
    ref = H.oracle_run(w, w.steps)
    got = np.concatenate([R.permute(2, 1, 0).cpu().numpy().ravel(),
                          I.permute(2, 1, 0).cpu().numpy().ravel()])
    want = np.concatenate([np.asarray(ref.R).ravel(), np.asarray(ref.I).ravel()])
    assert H.rel_l2(got, want) <= 1e-11


@pytest.mark.parametrize("shape,kdet", [((1, 1, 96), 60), ((4, 1, 64), 63), ((8, 3, 1), 0),
                                        ((2, 5, 40), 39)])
def test_paper_layout_degenerate_extents(shape, kdet):
    nx, ny, nz = shape
    w = workloads.ragged("f64").with_(nx=nx, ny=ny, nz=nz, k_det=kdet, cap=(3, 3, 20.0)
                                      if nz >= 8 else None,
                                      r0=(0.1, 0.1, 0.2 * nz / 2), atoms=None, steps=60)
    for bc in [(0, 0, 0), (0, 0, 1)]:
        say("paper layout degenerate", shape, "bc", bc)
        s, R, I = paper_vs_library(w.with_(bc=bc), "f64", w.steps, (16, 4, 4))
        assert_same(s, R, I)


def test_paper_layout_on_the_paper_grid():
    """The paper's own set-up (240 x 240 x 420 + 100 CAP planes, FP32) in the
    block shape of its measurements, against the two-step sweep that the
    library runs on it, after 6 steps."""
    w = workloads.paper_cu111()
    say("paper layout paper-cu111", (w.nx, w.ny, w.nz))
    s, R, I = paper_vs_library(w, "f32", 6, (16, 4, 4))
    assert s.get_tile().two_step == 1
    assert_same(s, R, I)


def test_paper_layout_rejects_bad_arguments():
    w = workloads.ragged("f64")
    s = tdse.sim_from_workload(w, precision="f64", steps=4)
    R, I, V = zfast(s.psi_r), zfast(s.psi_i), zfast(s.v)
    lib = tdse.load()
    for args in [(R.data_ptr(), I.data_ptr(), V.data_ptr(), -1, 16, 4, 4),
                 (R.data_ptr(), I.data_ptr(), V.data_ptr(), 1, 32, 8, 8),
                 (R.data_ptr(), I.data_ptr(), V.data_ptr(), 1, 0, 4, 4),
                 (R.data_ptr(), R.data_ptr(), V.data_ptr(), 1, 16, 4, 4),
                 (None, I.data_ptr(), V.data_ptr(), 1, 16, 4, 4)]:
        assert lib.tdse_paper_layout_run(s.h, *args) == tdse.ERR_ARG
    with pytest.raises(ValueError):
        s.paper_layout_run(s.psi_r, I, V, 1)
    # a failed call leaves the arrays as they were
    torch.cuda.synchronize()
    assert torch.equal(R, zfast(s.psi_r))
    h = ctypes.c_void_p()
    assert lib.tdse_create(ctypes.byref(s.desc), None, ctypes.byref(h)) == tdse.OK
    try:
        assert lib.tdse_paper_layout_run(h, R.data_ptr(), I.data_ptr(), V.data_ptr(), 1, 16, 4,
                                         4) == tdse.ERR_STATE
    finally:
        lib.tdse_destroy(h)
