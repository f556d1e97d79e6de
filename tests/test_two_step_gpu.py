"""GPU two-step sweep: two leapfrog steps (eqs. (9), (8), (9), (8) of arXiv
2401.07416 section 2.1) per pass over the grid.  The cell arithmetic is the
one-pass step's, so states and records must be bitwise identical to it (sums
to 1e-13, reduced over other tiles), and match the FP64 oracle to the usual
tolerances on ragged, degenerate and zero-boundary grids, with odd record
intervals and odd step counts that mix two-step, one-pass and half-step
launches."""
import sys

import numpy as np
import pytest
import torch

from paper_2401_07416_amd import tdse, workloads
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu

FP64 = dict(tol_state=1e-11, tol_rec=1e-11, tol_scal=1e-12, tol_flux=1e-12)
FP32 = dict(tol_state=1e-4, tol_rec=1e-3, tol_scal=1e-4, tol_flux=1e-5)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def two(tx, rows, zc, pf=0, threads=256):
    return dict(fused=1, two_step=1, two_step_tx=tx, two_step_rows=rows, two_step_zc=zc,
                two_step_prefetch=pf, two_step_threads=threads)


TILES2 = [two(56, 2, 64), two(24, 2, 16, 1), two(8, 3, 7), two(120, 3, 33, 1),
          two(64, 1, 64, 1, 512), two(24, 2, 32, 1, 512), two(8, 1, 9, 0, 512),
          two(64, 1, 32, 1, 1024), two(16, 1, 11, 0, 1024)]


def same_run(a, b):
    assert bool((a.psi_r == b.psi_r).all()) and bool((a.psi_i == b.psi_i).all())
    ra, sa = a.records_host()
    rb, sb = b.records_host()
    np.testing.assert_array_equal(ra, rb)
    np.testing.assert_allclose(sa, sb, rtol=1e-13, atol=1e-15)
    assert a.detect().flux == pytest.approx(b.detect().flux, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_two_step_is_bitwise_the_one_pass_step(prec):
    w = workloads.c2_reduced().with_(steps=120)
    say("two-step vs one-pass 64x64x128", prec)
    base = H.gpu_run(w, w.steps, precision=prec, pixel=True, tile=dict(fused=1, two_step=0))
    for tile in TILES2:
        say(" tile", tile)
        g = H.gpu_run(w, w.steps, precision=prec, pixel=True, tile=tile)
        t = g.get_tile()
        assert t.two_step == 1 and t.two_step_ty > 0
        same_run(g, base)
        np.testing.assert_allclose(g.pixel.cpu().numpy(), base.pixel.cpu().numpy(), rtol=1e-12,
                                   atol=0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1), (1, 0, 1), (0, 1, 0)])
def test_two_step_ragged_boundaries_vs_oracle(prec, bc):
    """37 x 29 x 53, record interval 7 (records on odd and even levels)."""
    w = workloads.ragged(prec).with_(bc=bc)
    say("two-step ragged", prec, "bc", bc)
    ref = H.oracle_run(w, w.steps)
    for tile in (two(8, 2, 16), two(16, 3, 53, 1), two(16, 1, 20, 1, 512), two(16, 1, 20, 1, 1024)):
        gpu = H.gpu_run(w, w.steps, precision=prec, tile=tile)
        say(" tile", tile, H.compare(gpu, ref, **(FP64 if prec == "f64" else FP32)))


@pytest.mark.parametrize("shape,kdet", [((1, 1, 96), 60), ((4, 1, 64), 63), ((8, 3, 1), 0),
                                        ((2, 5, 40), 39)])
def test_two_step_degenerate_extents(shape, kdet):
    nx, ny, nz = shape
    w = workloads.ragged("f64").with_(nx=nx, ny=ny, nz=nz, k_det=kdet, cap=(3, 3, 20.0)
                                      if nz >= 8 else None,
                                      r0=(0.1, 0.1, 0.2 * nz / 2), atoms=None, steps=150)
    for bc in [(0, 0, 0), (0, 0, 1), (1, 1, 0)]:
        ww = w.with_(bc=bc)
        say("two-step degenerate", shape, "bc", bc)
        ref = H.oracle_run(ww, ww.steps)
        for tile in (two(8, 2, 8), two(8, 1, 8, 0, 1024)):
            gpu = H.gpu_run(ww, ww.steps, precision="f64", tile=tile)
            say(" tile", tile, H.compare(gpu, ref, **FP64))


def test_two_step_odd_chunks_and_resume():
    """Calls of 1, 2, 3, 7 and 13 steps (odd counts, pairs split by record
    levels) give the bits of one call on the one-pass path."""
    w = workloads.c2_reduced().with_(steps=300, record_every=5)
    say("two-step chunks, record interval 5")
    full = H.gpu_run(w, 300, precision="f32", tile=dict(fused=1, two_step=0))
    chunked = H.gpu_run(w, 300, precision="f32", chunks=[1, 2, 3, 7, 13, 49], tile=two(56, 2, 32))
    same_run(chunked, full)
    first = H.gpu_run(w, 141, precision="f32", tile=two(56, 2, 32))
    r, i, step, flux = first.get_state()
    second = tdse.sim_from_workload(w, precision="f32", steps=300)
    second.set_tile(**two(24, 2, 64))
    nr = first.records.shape[0]
    second.records[:nr].copy_(first.records)
    second.scalars[:nr].copy_(first.scalars)
    second.set_state(r, i, step=step, flux=flux)
    second.step(159)
    assert bool((full.psi_r == second.psi_r).all()) and bool((full.psi_i == second.psi_i).all())
    assert bool((full.records == second.records).all())
    assert second.detect().flux == pytest.approx(full.detect().flux, rel=1e-12)


def test_two_step_with_adjoint_checkpoints():
    """A forward run with checkpoints every 7 steps (odd: pairs may not
    straddle a checkpoint level) gives the same gradient with the two-step
    sweep on and off."""
    nx, ny, nz = 16, 12, 40
    rng = np.random.default_rng(0)
    V = -30.0 * np.abs(rng.standard_normal((nz, ny, nx)))
    R0, I0 = rng.standard_normal((nz, ny, nx)), rng.standard_normal((nz, ny, nx))
    N, K, h = 61, 7, 4
    rho_bar = rng.standard_normal((N // h + 1, ny, nx))
    out = []
    for tile in (dict(fused=1, two_step=0), two(8, 2, 16)):
        d = tdse.make_desc(nx, ny, nz, 0.22, 0.25, 0.2, hbar=0.6582119569, mass=0.0568563,
                           dt_frac=0.9, precision="f64", k_det=22, record_every=h,
                           max_records=N // h + 1)
        s = tdse.Sim(d)
        s.v.copy_(torch.from_numpy(V))
        s.set_cap_quadratic(5, 4, 40.0)
        s.finalize()
        s.set_tile(**tile)
        s.set_state(torch.from_numpy(R0), torch.from_numpy(I0), step=0)
        s.bind_adjoint(N, K)
        s.step(N)
        gV, gR, gI = s.adjoint(torch.from_numpy(rho_bar))
        out.append((s.psi_r.clone(), gV.clone(), gR.clone(), gI.clone()))
    say("adjoint with two-step")
    for a, b in zip(out[0], out[1]):
        assert bool((a == b).all())


def test_two_step_timing_counts_launches():
    w = workloads.c2_reduced().with_(steps=100)
    s = tdse.sim_from_workload(w, precision="f32", steps=100)
    s.set_tile(**two(56, 2, 64))
    s.set_timing(True)
    s.step(100)
    kt = s.timing_read()
    say("timing", kt)
    # record interval 20: pairs up to each record level, the record level's
    # pair carries the record, so 50 two-step launches
    assert kt["two_step"][1] == 50 and kt["fused"][1] == 0
    assert kt["two_step"][0] > 0


def test_two_step_rejects_bad_tiles():
    w = workloads.c2_reduced().with_(steps=10)
    s = tdse.sim_from_workload(w, precision="f32", steps=10)
    for bad in (two(4, 2, 8), two(56, 4, 8), two(2040, 2, 8), dict(fused=0, two_step=1),
                two(56, 3, 8, 0, 512), two(56, 2, 8, 0, 128), two(56, 2, 8, 0, 1024)):
        with pytest.raises(tdse.TdseError):
            s.set_tile(**bad)
    # a (rows, threads) pair that has no kernel names the pairs that do
    with pytest.raises(tdse.TdseError, match=r"\(1,1024\)") as e:
        s.set_tile(**two(56, 2, 8, 0, 1024))
    assert e.value.status == tdse.ERR_UNSUPPORTED
    # the handle still steps with its previous tile
    s.step(2)
    assert s.detect().n_records >= 1


def test_library_autotuner_picks_a_tile_and_spends_the_state():
    w = workloads.c2_reduced().with_(steps=100)
    s = tdse.sim_from_workload(w, precision="f32", steps=100)
    t = s.autotune(steps=6)
    say("autotuned", t.as_dict())
    assert t.fused in (0, 1) and (t.two_step == 0 or t.two_step_ty > 0)
    with pytest.raises(tdse.TdseError) as e:
        s.step(2)
    assert e.value.status == tdse.ERR_STATE
    # a fresh state on the tuned tile gives the bits of the default run
    ref = H.gpu_run(w, 100, precision="f32")
    r0 = tdse.sim_from_workload(w, precision="f32", steps=100)
    s.set_state(r0.psi_r, r0.psi_i, step=0)
    s.step(100)
    assert bool((s.psi_r == ref.psi_r).all()) and bool((s.psi_i == ref.psi_i).all())


def test_autotuner_cache_round_trip(tmp_path, monkeypatch):
    """TDSE_TUNE_CACHE: the first tuning of a case times the candidates and
    writes one line for it; the next finds the line, sets that tile without
    running anything (the state is kept); TDSE_TUNE_REFRESH times again and
    leaves one line per case."""
    path = tmp_path / "tiles.txt"
    monkeypatch.setenv("TDSE_TUNE_CACHE", str(path))
    w = workloads.c2_reduced().with_(steps=100)
    s = tdse.sim_from_workload(w, precision="f32", steps=100)
    t1 = s.autotune(steps=4, flags=6)
    lines = path.read_text().splitlines()
    say("cache after tuning", lines)
    assert len(lines) == 1 and lines[0].startswith("tdse-tune-v1 64 64 128 0 ")
    s2 = tdse.sim_from_workload(w, precision="f32", steps=100)
    t2 = s2.autotune(steps=4, flags=6)
    assert t2.as_dict() == t1.as_dict()
    s2.step(10)   # a hit keeps the state
    assert s2.detect().step == 10
    s3 = tdse.sim_from_workload(w, precision="f32", steps=100)
    s3.autotune(steps=4, flags=6 | tdse.TUNE_REFRESH)
    with pytest.raises(tdse.TdseError) as e:   # timed again: the state is spent
        s3.step(2)
    assert e.value.status == tdse.ERR_STATE
    assert len(path.read_text().splitlines()) == 1
    s4 = tdse.sim_from_workload(w.with_(nx=48), precision="f32", steps=100)
    s4.autotune(steps=4, flags=6)
    assert len(path.read_text().splitlines()) == 2


@pytest.mark.parametrize("prec,shape,want", [
    ("f32", (512, 512, 1024), (128, 16, 512)),
    ("f64", (512, 512, 1024), (64, 16, 1024)),
    ("f32", (512, 512, 128), (128, 16, 64)),
    ("f32", (240, 240, 520), (80, 35, 44)),
    ("f64", (256, 256, 512), (64, 16, 128)),
    ("f32", (208, 208, 416), (104, 19, 38)),
    ("f32", (224, 224, 448), (112, 25, 32)),
    ("f32", (320, 320, 640), (80, 36, 92)),
])
def test_default_tile_on_large_grids_fills_one_round(prec, shape, want):
    """The library's default two-step tile on grids of 2^24 cells or more:
    1024 threads, the first width of its list that divides nx, and, among
    the heights and z chunks whose workgroups fill 90-100% of one round of
    the CUs (on the MI355X's 256), the one whose workgroup sweeps the fewest
    cells."""
    props = torch.cuda.get_device_properties(0)
    if props.multi_processor_count != 256:
        pytest.skip("the expected tiles are those of a 256-CU device")
    d = tdse.make_desc(*shape, 0.2, 0.2, 0.2, precision=prec)
    s = tdse.Sim(d)
    t = s.get_tile()
    say("default tile", prec, shape, t.as_dict())
    assert t.two_step == 1 and t.two_step_threads == 1024 and t.two_step_rows == 1
    assert (t.two_step_tx, t.two_step_ty, t.two_step_zc) == want
    s.close()


def test_default_tile_on_small_grids_keeps_the_cost_model():
    """Below 2^24 cells the one-round rule is not used (a 128x128x256 grid
    stays off the one-round sweep tiles)."""
    d = tdse.make_desc(128, 128, 256, 0.2, 0.2, 0.2, precision="f64")
    s = tdse.Sim(d)
    t = s.get_tile()
    say("default tile 128x128x256 f64", t.as_dict())
    assert not (t.two_step == 1 and t.two_step_threads == 1024 and t.two_step_ty == 16
                and t.two_step_zc == 32)
    s.close()


@pytest.mark.gpu
def test_default_one_pass_chunks_shorten_on_small_grids():
    """Where no chunk of 8 planes or more gives about 8 waves per CU, the
    one-pass default takes the widest band in 2- or 1-plane chunks (the z
    march of each workgroup sets the time on a cache-resident grid); grids
    that reach the occupancy with long chunks keep them."""
    for n, nz, prec, short in ((32, 32, "f64", True), (64, 64, "f32", True), (64, 64, "f64", True),
                               (64, 512, "f32", True), (128, 128, "f64", False), (256, 256, "f32", False)):
        s = tdse.Sim(tdse.make_desc(n, n, nz, 0.2, 0.2, 0.2, precision=prec))
        t = s.get_tile()
        say(f"default one-pass tile {n}x{n}x{nz} {prec}", t.as_dict())
        assert (t.fused_zc <= 2) == short
        if short:
            assert t.fused_threads == 256
        s.close()
