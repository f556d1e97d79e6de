"""Host statistics of section 3.2: the time weights of eq. (16) and the
cluster dispersions of eqs. (17)-(18), against hand-computed values."""
import numpy as np
import pytest

from paper_2401_07416_amd import analysis


def test_frame_weights_are_the_trapezoid_rule_over_the_window():
    times = np.arange(10) * 0.25          # 0 .. 2.25
    idx, w = analysis.frame_weights(times, 0.5, 1.5)
    assert list(idx) == [2, 3, 4, 5, 6]
    np.testing.assert_allclose(w, np.array([0.125, 0.25, 0.25, 0.25, 0.125]) / 1.0)
    # the weighted sum of a linear function is its mean over the window
    f = 3.0 + 2.0 * times[idx]
    assert np.sum(w * f) == pytest.approx(3.0 + 2.0 * 1.0)
    with pytest.raises(ValueError):
        analysis.frame_weights(times, 5.0, 6.0)
    idx, w = analysis.frame_weights(times, 0.5, 0.6)
    assert list(idx) == [2] and list(w) == [1.0]


def test_cluster_dispersion_by_hand():
    # cluster 0: (0,0), (2,0) -> centre (1,0); cluster 1: (4,3), (4,5), (4,4) -> centre (4,4)
    xy = np.array([[0, 0], [2, 0], [4, 3], [4, 5], [4, 4]], dtype=float)
    lab = np.array([0, 0, 1, 1, 1])
    r = analysis.cluster_dispersion(xy, lab)
    centre = np.array([14 / 5, 12 / 5])
    dc = [np.hypot(1 - centre[0], 0 - centre[1]), np.hypot(4 - centre[0], 4 - centre[1])]
    assert r["acd"] == pytest.approx(np.mean(dc))
    assert r["mcd"] == pytest.approx(np.median(dc))
    # point distances: 1, 1, 1, 1, 0
    assert r["aicd"] == pytest.approx(4 / 5)
    assert r["micd"] == pytest.approx(1.0)


def test_cluster_dispersion_of_one_cluster_and_labels_order():
    xy = np.array([[1.0, 1.0], [3.0, 1.0], [2.0, 4.0]])
    r = analysis.cluster_dispersion(xy, [7, 7, 7])
    assert r["acd"] == 0.0 and r["mcd"] == 0.0
    a = analysis.cluster_dispersion(np.array([[0, 0], [2, 0], [4, 4]], float), ["b", "b", "a"])
    b = analysis.cluster_dispersion(np.array([[4, 4], [0, 0], [2, 0]], float), ["a", "b", "b"])
    assert a == pytest.approx(b)
