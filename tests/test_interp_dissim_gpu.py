"""GPU unit-cell interpolation (section 2.3: the cell potential repeated in x
and y and interpolated onto the mesh; trilinear) and trajectory
dissimilarity (eq. (16)) against the oracle, through the C ABI.
Tolerances: interpolated V in FP64 <= 1e-13 of max|V| (FP32: one rounding,
<= 1e-7); d_kj FP64 <= 1e-12 relative, FP32 frames <= 1e-6 relative."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2401_07416_amd import analysis, tdse, workloads
from tests import gpu_harness as H

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def interp_sim(nx, ny, nz, dx, dy, dz, prec):
    d = tdse.make_desc(nx, ny, nz, dx, dy, dz, hbar=oracle.HBAR_EV_FS,
                       mass=oracle.HBAR_EV_FS ** 2 / oracle.HBAR2_OVER_ME, precision=prec)
    return tdse.Sim(d, pingpong=False)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(37, 29, 53), (40, 29, 53), (1100, 5, 7)])
def test_interpolated_potential_matches_oracle(prec, shape):
    """Odd rows (one cell per thread), rows of whole 16-byte vectors, and
    rows longer than one workgroup's segment with a partial last one."""
    table = workloads.unit_cell_table(uz=80, z_top=10.0)
    sp = (2.556 / 24, 4.427 / 28, 0.2)
    org = (0.031, -0.27, 0.15)
    nx, ny, nz = shape
    say("interpolation", shape, prec)
    s = interp_sim(nx, ny, nz, 0.21, 0.19, 0.23, prec)
    s.interpolate_potential(table, sp, org)
    g = oracle.Grid(nx, ny, nz, 0.21, 0.19, 0.23, hbar=1.0, mass=1.0)
    ref = oracle.interp_potential(g, table, sp, org)
    got = s.v.double().cpu().numpy()
    scale = np.max(np.abs(ref))
    tol = 1e-13 if prec == "f64" else 1e-7
    err = float(np.max(np.abs(got - ref)) / scale)
    say(" max err / max|V|", err)
    assert err <= tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_interpolated_potential_large_table_matches_oracle(prec):
    """A cell table whose z-blended plane does not fit the LDS staging
    (96 x 80 samples): the gather kernel with the separate weights launch."""
    table = workloads.unit_cell_table(ux=96, uy=80, uz=40, z_top=6.0)
    sp = (2.556 / 96, 4.427 / 80, 0.2)
    org = (0.013, 0.4, -0.05)
    nx, ny, nz = 45, 31, 23
    say("interpolation, large table", prec)
    s = interp_sim(nx, ny, nz, 0.21, 0.19, 0.23, prec)
    s.interpolate_potential(table, sp, org)
    g = oracle.Grid(nx, ny, nz, 0.21, 0.19, 0.23, hbar=1.0, mass=1.0)
    ref = oracle.interp_potential(g, table, sp, org)
    got = s.v.double().cpu().numpy()
    scale = np.max(np.abs(ref))
    tol = 1e-13 if prec == "f64" else 1e-7
    err = float(np.max(np.abs(got - ref)) / scale)
    say(" max err / max|V|", err)
    assert err <= tol


def test_interpolated_potential_headline_grid_sampled():
    """512 x 512 x 1024 FP32 mesh from a 24 x 28 x 360 cell table: planes
    sampled across the grid against the oracle on the same planes (the
    value at a mesh point depends only on its position)."""
    table = workloads.unit_cell_table()
    sp = (2.556 / 24, 4.427 / 28, 0.2)
    s = interp_sim(512, 512, 1024, 0.2, 0.2, 0.2, "f32")
    s.interpolate_potential(table, sp)
    torch.cuda.synchronize()
    say("interpolation 512x512x1024 sampled planes")
    for k0 in (0, 141, 357, 700, 1019):
        g = oracle.Grid(512, 512, 4, 0.2, 0.2, 0.2, hbar=1.0, mass=1.0)
        ref = oracle.interp_potential(g, table, sp, origin=(0.0, 0.0, -k0 * 0.2))
        got = s.v[k0:k0 + 4].double().cpu().numpy()
        err = float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-30))
        assert err <= 1e-6, (k0, err)


def test_run_on_an_interpolated_potential_matches_oracle():
    """The interpolated V feeds the step exactly as a built one: a reduced
    surface run (FP64) on the interpolated potential against the oracle run
    on the oracle's interpolation."""
    w = workloads.c2_reduced().with_(steps=300, atoms=None)
    table = workloads.unit_cell_table(uz=128, z_top=10.0, cell=(3.2, 3.2))
    sp = (3.2 / 24, 3.2 / 28, 0.2)
    d = tdse.make_desc(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.hbar, w.mass, dt_frac=w.dt_frac,
                       bc=w.bc, precision="f64", k_det=w.k_det, record_every=w.record_every,
                       max_records=w.n_records(w.steps))
    s = tdse.Sim(d)
    s.interpolate_potential(table, sp)
    s.set_cap_quadratic(*w.cap)
    s.finalize()
    kk = tdse.wavevector(w.energy, w.hbar, w.mass)
    s.init_gaussian(w.r0, tuple(kk * c for c in w.k_dir), w.sigma)
    s.step(w.steps)
    g = oracle.Grid(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.hbar, w.mass)
    V = oracle.interp_potential(g, table, sp)
    ref = H.oracle_run(w, w.steps, V=V)
    say("run on interpolated V", H.compare(s, ref, tol_state=1e-11, tol_rec=1e-11,
                                           tol_scal=1e-12, tol_flux=1e-12))


# ---- eq. (16) ---------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_dissimilarity_matches_oracle(prec):
    K, T, P = 70, 9, 1000        # ragged against the 64-trajectory blocks and 32-pixel chunks
    rng = np.random.default_rng(21)
    f = np.abs(rng.standard_normal((K, T, P)))
    if prec == "f32":
        f = f.astype(np.float32).astype(np.float64)
    w = rng.uniform(0.05, 0.2, T)
    dA = 0.04
    ref = oracle.dissimilarity(f, w, dA)
    ft = torch.from_numpy(f).to("cuda", torch.float32 if prec == "f32" else torch.float64)
    d = tdse.dissimilarity(ft, torch.from_numpy(w), dA).cpu().numpy()
    say("dissimilarity", prec, "max rel", float(np.max(np.abs(d - ref) / np.maximum(ref, 1e-300))))
    assert np.all(np.diag(d) == 0.0)
    np.testing.assert_array_equal(d, d.T)
    np.testing.assert_allclose(d, ref, rtol=1e-12 if prec == "f64" else 1e-6, atol=0)


def test_dissimilarity_keeps_close_pairs_accurate():
    """Pairs that differ by 1e-4 of the signal keep their relative
    accuracy (an FP32 Gram expansion would lose it to cancellation; the
    library's FP64 expansion of shifted frames does not)."""
    K, T, P = 8, 3, 65536
    rng = np.random.default_rng(22)
    base = np.abs(rng.standard_normal((1, T, P)))
    f = base + 1e-4 * rng.standard_normal((K, T, P))
    f = f.astype(np.float32).astype(np.float64)
    w = np.full(T, 1.0 / T)
    ref = oracle.dissimilarity(f, w, 1.0)
    d = tdse.dissimilarity(torch.from_numpy(f).to("cuda", torch.float32), torch.from_numpy(w),
                           1.0).cpu().numpy()
    off = ~np.eye(K, dtype=bool)
    err = float(np.max(np.abs(d[off] - ref[off]) / ref[off]))
    say("close pairs max rel", err)
    assert err <= 1e-5


def test_dissimilarity_of_a_tight_cluster_far_from_trajectory_0():
    """Trajectories 1e-6 apart at unit distance from trajectory 0 (the shift
    of the FP32 Gram form): the expansion alone would leave about 1e-4 of
    relative error in their d^2, so these pairs are evaluated in the direct
    form, and keep the oracle's accuracy; pairs with trajectory 0 stay on the
    matrix cores."""
    K, T, P = 12, 3, 128 * 128
    rng = np.random.default_rng(24)
    far = rng.uniform(0.0, 2.0, (1, T, P))
    centre = rng.uniform(0.0, 2.0, (1, T, P))
    f = np.concatenate([far, centre + 1e-6 * rng.standard_normal((K - 1, T, P))])
    f = f.astype(np.float32).astype(np.float64)
    w = np.full(T, 1.0 / T)
    ref = oracle.dissimilarity(f, w, 1.0)
    d = tdse.dissimilarity(torch.from_numpy(f).to("cuda", torch.float32), torch.from_numpy(w),
                           1.0).cpu().numpy()
    off = ~np.eye(K, dtype=bool)
    err = float(np.max(np.abs(d[off] - ref[off]) / ref[off]))
    say("tight cluster far from trajectory 0: max rel", err, "d within", float(ref[1, 2]),
        "d to 0", float(ref[0, 1]))
    assert ref[1, 2] < 1e-4 * ref[0, 1]
    np.testing.assert_array_equal(d, d.T)
    assert err <= 1e-6


def test_dissimilarity_direct_pairs_across_blocks_are_reproducible():
    """A cluster of 40 trajectories far from trajectory 0 straddling the
    edge of two 128-trajectory blocks (its pairs in diagonal and
    off-diagonal blocks go to the direct form), among random ones: every
    entry against the oracle, and two calls bitwise equal (the list of such
    pairs is built in whatever order the reduction appends them)."""
    K, T, P = 300, 4, 2048
    rng = np.random.default_rng(25)
    f = rng.uniform(0.0, 2.0, (K, T, P))
    centre = rng.uniform(0.0, 2.0, (1, T, P)) + 3.0
    f[100:140] = centre + 1e-6 * rng.standard_normal((40, T, P))
    f = f.astype(np.float32).astype(np.float64)
    w = rng.uniform(0.05, 0.2, T)
    ref = oracle.dissimilarity(f, w, 0.5)
    ft = torch.from_numpy(f).to("cuda", torch.float32)
    wt = torch.from_numpy(w)
    d1 = tdse.dissimilarity(ft, wt, 0.5).cpu().numpy()
    d2 = tdse.dissimilarity(ft, wt, 0.5).cpu().numpy()
    np.testing.assert_array_equal(d1, d2)
    np.testing.assert_array_equal(d1, d1.T)
    assert np.all(np.diag(d1) == 0.0)
    off = ~np.eye(K, dtype=bool)
    say("cluster across blocks max rel", float(np.max(np.abs(d1[off] - ref[off]) / ref[off])))
    np.testing.assert_allclose(d1, ref, rtol=1e-6, atol=0)


@pytest.mark.parametrize("K,T,P", [(300, 5, 999), (260, 4, 1024), (129, 2, 33), (1, 3, 7), (2, 1, 1)])
def test_dissimilarity_blocks_and_tails(K, T, P):
    """FP32 frames over several 128-trajectory blocks (off-diagonal and
    ragged ones), pixel counts off the 4-pixel vectors and 32-pixel chunks,
    and the degenerate single trajectory, frame and pixel."""
    rng = np.random.default_rng(K * 1000 + P)
    f = rng.uniform(0.0, 2.0, (K, T, P)).astype(np.float32).astype(np.float64)
    w = rng.uniform(0.05, 0.2, T)
    ref = oracle.dissimilarity(f, w, 0.25)
    d = tdse.dissimilarity(torch.from_numpy(f).to("cuda", torch.float32), torch.from_numpy(w),
                           0.25).cpu().numpy()
    assert np.all(np.diag(d) == 0.0)
    np.testing.assert_array_equal(d, d.T)
    off = ~np.eye(K, dtype=bool)
    if off.any():
        say("blocks", K, T, P, "max rel", float(np.max(np.abs(d[off] - ref[off]) / ref[off])))
    np.testing.assert_allclose(d, ref, rtol=1e-6, atol=0)


def test_dissimilarity_full_size_sampled():
    """The benchmark's size (879 trajectories x 77 frames x 128^2 pixels,
    seeded uniform FP32 frames, the launch the benchmark times): sampled
    trajectories across the 128-trajectory blocks (first, last, both sides
    of block edges) against the oracle run on those trajectories alone."""
    K, T, P = 879, 77, 128 * 128
    g = torch.Generator(device="cuda")
    g.manual_seed(16)
    frames = torch.rand((K, T, P), generator=g, device="cuda", dtype=torch.float32)
    w = np.full(T, 1.0 / T)
    d = tdse.dissimilarity(frames, torch.from_numpy(w), 0.04).cpu().numpy()
    assert np.all(np.diag(d) == 0.0)
    np.testing.assert_array_equal(d, d.T)
    pick = [0, 1, 127, 128, 255, 256, 500, 639, 640, 767, 768, 877, 878]
    sub = frames[pick].double().cpu().numpy()
    del frames
    ref = oracle.dissimilarity(sub, w, 0.04)
    got = d[np.ix_(pick, pick)]
    off = ~np.eye(len(pick), dtype=bool)
    say("full size sampled max rel", float(np.max(np.abs(got[off] - ref[off]) / ref[off])))
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=0)


def test_dissimilarity_of_repeated_and_shifted_trajectories():
    """A trajectory repeated under another index is at distance exactly 0
    (its pairs' d^2 are rounding residues of the expansion, so the pair is
    evaluated from the differences), and a common offset of every frame
    leaves d unchanged."""
    K, T, P = 40, 3, 4096
    rng = np.random.default_rng(23)
    # values on a 2^-20 grid, so that adding 4 below is exact in FP32
    f = (np.floor(rng.uniform(0.0, 1.0, (K, T, P)) * 2.0**20) / 2.0**20).astype(np.float32)
    f[17] = f[5]
    w = np.full(T, 1.0 / T)
    d = tdse.dissimilarity(torch.from_numpy(f).cuda(), torch.from_numpy(w), 1.0).cpu().numpy()
    typical = float(np.median(d[~np.eye(K, dtype=bool)]))
    say("repeated pair", d[5, 17], "typical", typical)
    assert d[5, 17] == 0.0 and d[17, 5] == 0.0 and typical > 0.0
    # the offset is exact in FP32, so the differences are unchanged bit for bit
    g = (f.astype(np.float64) + 4.0).astype(np.float32)
    assert np.array_equal(g.astype(np.float64) - 4.0, f.astype(np.float64))
    d2 = tdse.dissimilarity(torch.from_numpy(g).cuda(), torch.from_numpy(w), 1.0).cpu().numpy()
    off = ~np.eye(K, dtype=bool)
    np.testing.assert_allclose(d2[off], d[off], rtol=1e-12, atol=0)


def test_dissimilarity_of_batch_records():
    """Records of a batch of equal grids (the film physics, different
    molecules), frames inside a time window, against the oracle on the same
    frames."""
    steps, n = 120, 5
    ws = []
    for b in range(n):
        w = workloads.c4_film(b, steps)
        w = w.with_(nx=32, ny=32, nz=64, atoms=workloads.film_atoms(300 + b, 6.4, 6.4, 3.2),
                    r0=(3.2, 3.2, 8.3), sigma=1.5, k_det=35, cap=(8, 8, 50.0), record_every=10,
                    name=f"film-32-{b}")
        ws.append(w)
    bt = tdse.batch_from_workloads(ws, precision="f32", steps=steps)
    bt.prepare()
    bt.run(steps)
    assert all(st == tdse.OK for st in bt.status())
    nrec = steps // 10 + 1
    dts = [m.detect().dt for m in bt.members]
    times = np.arange(nrec) * 10 * dts[0]
    idx, wts = analysis.frame_weights(times, times[2], times[9])
    frames = torch.stack([m.records[:nrec][idx].reshape(len(idx), -1) for m in bt.members])
    dA = ws[0].dx * ws[0].dy
    d = tdse.dissimilarity(frames, torch.from_numpy(wts), dA).cpu().numpy()
    ref = oracle.dissimilarity(frames.double().cpu().numpy(), wts, dA)
    say("batch records d_kj", d[0, 1:])
    np.testing.assert_allclose(d, ref, rtol=1e-6, atol=0)


def test_dissimilarity_rejects_bad_arguments():
    f = torch.ones((3, 2, 10), dtype=torch.float32, device="cuda")
    with pytest.raises(tdse.TdseError):
        tdse.dissimilarity(f, torch.ones(2, dtype=torch.float64), 0.0)
    with pytest.raises(ValueError):
        tdse.dissimilarity(f, torch.ones(3, dtype=torch.float64), 1.0)


# ---- the paper's own set-up (eqs. (10), (11), interpolated cell potential) ---

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_paper_literal_setup_matches_oracle(prec):
    """Interpolated cell potential, 20 appended planes with the one-sided
    eq. (10) CAP, the eq. (11) time step (beyond the Gershgorin bound, inside
    the exact leapfrog limit), records every 20 steps: 300 steps against the
    oracle's own set-up of the same description."""
    w = workloads.paper_cu111(reduced=True)
    say("paper-literal reduced", prec)
    ref = H.oracle_run(w, w.steps)
    for tile in (None, dict(fused=1, two_step=1, two_step_tx=8, two_step_rows=2, two_step_zc=32,
                            two_step_threads=256)):
        gpu = H.gpu_run(w, w.steps, precision=prec, tile=tile)
        assert gpu.dt == pytest.approx(oracle.dt_paper(H.oracle_grid(w)), rel=1e-15)
        tol = (dict(tol_state=1e-11, tol_rec=1e-11, tol_scal=1e-12, tol_flux=1e-12) if prec == "f64"
               else dict(tol_state=1e-4, tol_rec=1e-3, tol_scal=1e-4, tol_flux=1e-5))
        say(" tile", tile, H.compare(gpu, ref, **tol))
