"""Pins of the oracle's discrete adjoint (reverse mode through the leapfrog of
arXiv 2401.07416 section 2.1, eqs. (8)-(9) with the CAP, and the records of
eq. (15)) against central finite differences of the forward oracle, which
is itself pinned in test_oracle_pins.py."""
import numpy as np
import pytest

import oracle

RNG = np.random.default_rng


def setup(shape=(3, 4, 10), sp=(0.25, 0.3, 0.2), seed=0, h=3, kdet=4, cap=True):
    nx, ny, nz = shape
    g = oracle.Grid(nx, ny, nz, *sp, hbar=0.6582119569, mass=0.0568563)
    rng = RNG(seed)
    V = -20.0 * np.abs(rng.standard_normal(g.shape))
    W = np.zeros(nz)
    if cap:
        W[:2] = [30.0, 8.0]
        W[-2:] = [8.0, 30.0]
    dt = 0.9 * g.hbar / oracle.emax(g, V)
    R0, I0 = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    return g, V, W, dt, R0, I0, h, kdet


def records(g, V, W, dt, R0, I0, h, kdet, n):
    s = oracle.Sim(g, V, R0, I0, dt, W=W, k_det=kdet, record_every=h, max_records=n // h + 1)
    s.record0()
    s.step(n)
    return s.records()[0]


def loss(rho, T):
    return float(np.sum((rho - T) ** 2))


def gradients(g, V, W, dt, R0, I0, h, kdet, n, T, K):
    s = oracle.Sim(g, V, R0, I0, dt, W=W, k_det=kdet, record_every=h, max_records=n // h + 1)
    s.record0()
    rho = records(g, V, W, dt, R0, I0, h, kdet, n)
    return s.adjoint(n, 2.0 * (rho - T), ckpt_every=K)


def test_adjoint_matches_central_differences_componentwise():
    g, V, W, dt, R0, I0, h, kd = setup()
    n = 30
    T = RNG(1).random((n // h + 1, g.ny, g.nx))
    gV, gR, gI = gradients(g, V, W, dt, R0, I0, h, kd, n, T, K=7)
    eps = 1e-5
    fd_v = np.zeros(g.shape)
    fd_r = np.zeros(g.shape)
    fd_i = np.zeros(g.shape)
    for idx in np.ndindex(g.shape):
        for arr, out, scale in ((V, fd_v, 1.0), (R0, fd_r, 1.0), (I0, fd_i, 1.0)):
            d = eps * scale
            p = arr.copy()
            p[idx] += d
            args = [V, R0, I0]
            which = 0 if arr is V else (1 if arr is R0 else 2)
            args[which] = p
            lp = loss(records(g, args[0], W, dt, args[1], args[2], h, kd, n), T)
            p[idx] -= 2 * d
            lm = loss(records(g, args[0], W, dt, args[1], args[2], h, kd, n), T)
            out[idx] = (lp - lm) / (2 * d)
    for got, fd in ((gV, fd_v), (gR, fd_r), (gI, fd_i)):
        assert np.max(np.abs(got - fd)) <= 1e-6 * np.max(np.abs(fd))


def test_adjoint_directional_derivative_larger_grid():
    g, V, W, dt, R0, I0, h, kd = setup(shape=(8, 6, 16), sp=(0.2, 0.22, 0.19), seed=3, h=5,
                                       kdet=9)
    n = 60
    T = RNG(4).random((n // h + 1, g.ny, g.nx)) * 0.1
    gV, gR, gI = gradients(g, V, W, dt, R0, I0, h, kd, n, T, K=16)
    rng = RNG(5)
    for arr, grad, which in ((V, gV, 0), (R0, gR, 1), (I0, gI, 2)):
        dirn = rng.standard_normal(g.shape)
        eps = 1e-6 * np.linalg.norm(arr) / np.linalg.norm(dirn)
        args = [V, R0, I0]
        args[which] = arr + eps * dirn
        lp = loss(records(g, args[0], W, dt, args[1], args[2], h, kd, n), T)
        args[which] = arr - eps * dirn
        lm = loss(records(g, args[0], W, dt, args[1], args[2], h, kd, n), T)
        fd = (lp - lm) / (2 * eps)
        assert float(np.sum(grad * dirn)) == pytest.approx(fd, rel=1e-7)


def test_adjoint_independent_of_checkpoint_interval():
    g, V, W, dt, R0, I0, h, kd = setup(seed=7)
    n = 31
    T = RNG(8).random((n // h + 1, g.ny, g.nx))
    base = gradients(g, V, W, dt, R0, I0, h, kd, n, T, K=n)
    for K in (1, 4, 13):
        other = gradients(g, V, W, dt, R0, I0, h, kd, n, T, K=K)
        for a, b in zip(other, base):
            np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.max(np.abs(b)))


def test_potential_vjp_matches_central_differences():
    g = oracle.Grid(14, 12, 16, 0.21, 0.23, 0.2)
    rng = RNG(9)
    atoms = np.array([[1.13, 1.37, 1.55, 6.0, 1.0], [2.01, 0.52, 1.91, 8.0, 0.8],
                      [0.47, 2.11, 1.22, 14.0, 1.3]])
    w = rng.standard_normal(g.shape)
    kw = dict(soft=0.1, cutoff=1.25)
    dpos, damp = oracle.potential_vjp(g, atoms, w, **kw)
    eps = 1e-6
    for a in range(len(atoms)):
        for c in range(3):
            p = atoms.copy()
            p[a, c] += eps
            lp = np.sum(w * oracle.potential(g, p, **kw))
            p[a, c] -= 2 * eps
            lm = np.sum(w * oracle.potential(g, p, **kw))
            assert dpos[a, c] == pytest.approx((lp - lm) / (2 * eps), rel=1e-6, abs=1e-9)
        p = atoms.copy()
        p[a, 4] += eps
        lp = np.sum(w * oracle.potential(g, p, **kw))
        p[a, 4] -= 2 * eps
        lm = np.sum(w * oracle.potential(g, p, **kw))
        assert damp[a] == pytest.approx((lp - lm) / (2 * eps), rel=1e-7)


def test_end_to_end_gradient_wrt_atom_positions():
    """Loss of the time-integrated detection intensity against a target, as a
    function of the atom positions, through potential, leapfrog and records."""
    g = oracle.Grid(6, 6, 20, 0.25, 0.25, 0.2, hbar=0.6582119569, mass=0.0568563)
    atoms = np.array([[0.61, 0.77, 1.43, 6.0, 1.0], [0.93, 0.29, 1.61, 8.0, 1.0]])
    W = oracle.cap_quadratic(g.nz, 3, 3, 30.0)
    kw = dict(soft=0.1, cutoff=1.3)
    V = oracle.potential(g, atoms, **kw)
    dt = 0.9 * g.hbar / oracle.emax(g, V)
    R0, I0 = oracle.init_gaussian(g, [0.75, 0.75, 2.9], [0, 0, -4.0], 0.6, dt)
    h, kd, n = 4, 12, 40
    T = RNG(11).random((g.ny, g.nx)) * 1e-3

    def L_of(at):
        Vv = oracle.potential(g, at, **kw)
        rho = records(g, Vv, W, dt, R0, I0, h, kd, n)
        P = h * dt * rho.sum(axis=0)
        return float(np.sum((P - T) ** 2)), rho, P

    L0, rho, P = L_of(atoms)
    s = oracle.Sim(g, V, R0, I0, dt, W=W, k_det=kd, record_every=h, max_records=n // h + 1)
    s.record0()
    dL_drho = np.broadcast_to(2 * h * dt * (P - T), rho.shape).copy()
    gV, _, _ = s.adjoint(n, dL_drho, ckpt_every=9)
    dpos, _ = oracle.potential_vjp(g, atoms, gV, **kw)
    eps = 1e-5
    for a in range(2):
        for c in range(3):
            p = atoms.copy()
            p[a, c] += eps
            lp = L_of(p)[0]
            p[a, c] -= 2 * eps
            lm = L_of(p)[0]
            assert dpos[a, c] == pytest.approx((lp - lm) / (2 * eps), rel=2e-5, abs=1e-12)
