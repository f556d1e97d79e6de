"""Pins of the oracle's unit-cell interpolation (section 2.3: the potential of
one cell repeated in x and y and interpolated onto the mesh; trilinear is the
reading) and of the trajectory dissimilarity of eq. (16).  Each pin comes
from outside the oracle: exact cases of linear interpolation, numpy's and
scipy's own interpolators and distances, metric axioms and closed forms."""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator
from scipy.spatial.distance import cdist

import oracle


def grid(nx, ny, nz, dx, dy, dz):
    return oracle.Grid(nx, ny, nz, dx, dy, dz, hbar=1.0, mass=1.0)


def test_coincident_mesh_copies_the_table():
    rng = np.random.default_rng(1)
    ux, uy, uz = 5, 4, 7
    table = rng.standard_normal((uz, uy, ux))
    g = grid(3 * ux, 2 * uy, uz, 0.3, 0.25, 0.2)
    V = oracle.interp_potential(g, table, (0.3, 0.25, 0.2))
    # i dx / sx lands within rounding of an integer: the neighbour's weight
    # is at most a few ulp
    np.testing.assert_allclose(V, np.tile(table, (1, 2, 3)), rtol=0, atol=1e-14 * np.max(np.abs(table)))


def test_field_linear_in_z_is_reproduced_and_clamped():
    rng = np.random.default_rng(2)
    uz, sz, oz = 9, 0.37, 0.8
    a, b = 1.3, -2.1
    zc = oz + sz * np.arange(uz)
    table = np.broadcast_to((a + b * zc)[:, None, None], (uz, 3, 4)).copy()
    g = grid(5, 6, 30, 0.21, 0.17, 0.13)
    V = oracle.interp_potential(g, table, (0.4, 0.3, sz), origin=(rng.uniform(), rng.uniform(), oz))
    z = np.clip(np.arange(30) * 0.13, zc[0], zc[-1])
    np.testing.assert_allclose(V, np.broadcast_to((a + b * z)[:, None, None], V.shape),
                               rtol=0, atol=1e-13)


def test_separable_table_is_the_product_of_numpy_interps():
    """Trilinear interpolation of a separable table X(a) Y(b) Z(c) is the
    product of 1D linear interpolations (numpy.interp, periodic in x, y)."""
    rng = np.random.default_rng(3)
    ux, uy, uz = 6, 5, 8
    sx, sy, sz = 0.41, 0.33, 0.27
    org = (0.13, -0.52, 0.4)
    X, Y, Z = rng.standard_normal(ux), rng.standard_normal(uy), rng.standard_normal(uz)
    table = Z[:, None, None] * Y[None, :, None] * X[None, None, :]
    g = grid(17, 11, 19, 0.19, 0.23, 0.17)
    V = oracle.interp_potential(g, table, (sx, sy, sz), origin=org)
    x = np.arange(17) * 0.19 - org[0]
    y = np.arange(11) * 0.23 - org[1]
    z = np.arange(19) * 0.17 - org[2]
    fx = np.interp(x, sx * np.arange(ux), X, period=ux * sx)
    fy = np.interp(y, sy * np.arange(uy), Y, period=uy * sy)
    fz = np.interp(z, sz * np.arange(uz), Z)
    ref = fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
    np.testing.assert_allclose(V, ref, rtol=0, atol=1e-13 * np.max(np.abs(ref)))


def test_general_table_matches_scipy_regular_grid_interpolator():
    rng = np.random.default_rng(4)
    ux, uy, uz = 7, 6, 9
    sp = (0.3, 0.35, 0.25)
    org = (0.05, 0.11, -0.3)
    table = rng.standard_normal((uz, uy, ux))
    g = grid(23, 19, 14, 0.17, 0.29, 0.21)
    V = oracle.interp_potential(g, table, sp, origin=org)
    # periodic padding in x and y, coordinates wrapped into one cell, z clipped
    padded = np.concatenate([table, table[:, :1, :]], axis=1)
    padded = np.concatenate([padded, padded[:, :, :1]], axis=2)
    f = RegularGridInterpolator((sp[2] * np.arange(uz), sp[1] * np.arange(uy + 1),
                                 sp[0] * np.arange(ux + 1)), padded, method="linear")
    k, j, i = np.meshgrid(np.arange(14), np.arange(19), np.arange(23), indexing="ij")
    x = np.mod(i * 0.17 - org[0], ux * sp[0])
    y = np.mod(j * 0.29 - org[1], uy * sp[1])
    z = np.clip(k * 0.21 - org[2], 0, (uz - 1) * sp[2])
    ref = f(np.stack([z.ravel(), y.ravel(), x.ravel()], axis=1)).reshape(V.shape)
    np.testing.assert_allclose(V, ref, rtol=0, atol=1e-12)


def test_shift_by_one_cell_changes_nothing():
    rng = np.random.default_rng(5)
    table = rng.standard_normal((4, 5, 6))
    sp = (0.3, 0.2, 0.5)
    g = grid(13, 9, 7, 0.23, 0.31, 0.37)
    a = oracle.interp_potential(g, table, sp, origin=(0.1, 0.2, 0.0))
    b = oracle.interp_potential(g, table, sp, origin=(0.1 + 6 * 0.3, 0.2 - 5 * 0.2, 0.0))
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13)


# ---- eq. (16) ---------------------------------------------------------------

def frames(K, T, P, seed):
    return np.abs(np.random.default_rng(seed).standard_normal((K, T, P)))


def test_dissimilarity_is_a_metric():
    f = frames(7, 5, 40, 6)
    w = np.random.default_rng(7).uniform(0.1, 1.0, 5)
    d = oracle.dissimilarity(f, w, 0.04)
    assert np.all(np.diag(d) == 0.0)
    np.testing.assert_array_equal(d, d.T)
    assert np.all(d[~np.eye(7, dtype=bool)] > 0)
    for a in range(7):
        for b in range(7):
            assert np.all(d[a, b] <= d[a, :] + d[:, b] + 1e-12)


def test_dissimilarity_per_frame_matches_scipy_cdist():
    K, T, P = 6, 4, 33
    f = frames(K, T, P, 8)
    w = np.array([0.1, 0.4, 0.2, 0.3])
    dA = 0.25
    d = oracle.dissimilarity(f, w, dA)
    ref = sum(w[t] * np.sqrt(dA) * cdist(f[:, t, :], f[:, t, :]) for t in range(T))
    np.testing.assert_allclose(d, ref, rtol=1e-13, atol=1e-15)


def test_dissimilarity_of_constant_frames():
    """Frames uniform over P pixels: the plane L2 distance is sqrt(dA P)
    times the difference of the levels."""
    K, T, P = 3, 6, 50
    lev = np.random.default_rng(9).standard_normal((K, T))
    f = np.repeat(lev[:, :, None], P, axis=2)
    w = np.full(T, 1.0 / T)
    d = oracle.dissimilarity(f, w, 0.5)
    for a in range(K):
        for b in range(K):
            ref = np.sum(w * np.sqrt(0.5 * P) * np.abs(lev[a] - lev[b]))
            assert d[a, b] == pytest.approx(ref, rel=1e-13, abs=1e-15)


def test_dissimilarity_scaling_and_common_shift():
    f = frames(5, 3, 20, 10)
    w = np.array([0.2, 0.5, 0.3])
    d = oracle.dissimilarity(f, w, 0.1)
    u = np.random.default_rng(11).standard_normal((1, 3, 20))
    np.testing.assert_allclose(oracle.dissimilarity(f + u, w, 0.1), d, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(oracle.dissimilarity(-2.5 * f, w, 0.1), 2.5 * d, rtol=1e-13)
