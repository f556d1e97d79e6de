"""Pins of the oracle's literal forms of eq. (10) (the one-sided CAP) and
eq. (11) (the recommended time step), from outside their formulas: the
support and end value of the profile, its constant second difference, the
paper's printed 0.38 as against the 0.48 as eq. (11) gives for its own grid
(the discrepancy the readings record), and the 1.2 ratio to the Gershgorin
step on a free cubic grid."""
import numpy as np
import pytest

import oracle

HBAR = oracle.HBAR_EV_FS
ME = HBAR ** 2 / oracle.HBAR2_OVER_ME


def test_cap_paper_profile():
    nz, dz, alpha = 60, 0.2, 3.0
    r_cut = 20 * dz
    W = oracle.cap_paper(nz, dz, alpha, r_cut)
    assert np.all(W[20:] == 0.0) and np.all(W[:20] > 0)
    assert W[0] == pytest.approx(alpha * r_cut ** 2 / dz, rel=1e-15)
    # quadratic in k: constant second difference 2 alpha dz over the support
    d2 = W[2:20] - 2 * W[1:19] + W[:18]
    np.testing.assert_allclose(d2, 2 * alpha * dz, rtol=1e-10)
    assert np.all(np.diff(W[:21]) < 0)
    assert np.all(oracle.cap_paper(nz, dz, alpha, 0.0) == 0.0)   # r_cut = 0: empty, as printed


def test_dt_paper_on_the_papers_grid():
    g = oracle.Grid(240, 240, 420, 40.9 / 240, 40.9 / 240, 70.0 / 420, hbar=HBAR, mass=ME)
    dt = oracle.dt_paper(g)
    assert dt * 1000 == pytest.approx(0.480, abs=5e-4)     # attoseconds; the paper prints 0.38


@pytest.mark.parametrize("d", [0.1, 0.2, 0.37])
def test_dt_paper_is_1_2_gershgorin_steps_on_a_free_cubic_grid(d):
    g = oracle.Grid(16, 16, 16, d, d, d, hbar=HBAR, mass=ME)
    assert oracle.dt_paper(g) / (HBAR / oracle.emax(g, np.zeros(g.shape))) == pytest.approx(1.2,
                                                                                      rel=1e-13)
