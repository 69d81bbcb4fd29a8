"""Pins for the oracle's direct sum, eq. (1).  CPU only."""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "direct_hand.json")


def test_direct_hand_values(oracle_lib):
    """Three points evaluated by hand (tests/golden/direct_hand.json)."""
    g = json.load(open(GOLDEN))
    x = np.array(g["points"]).T.copy()
    s = np.array(g["sigma"])
    for kern, e in g["expected"].items():
        f = oracle_lib.direct(kern, e["param"], x, x, s)
        np.testing.assert_allclose(f, e["f"], rtol=1e-14, atol=1e-15, err_msg=kern)


def test_direct_two_points(oracle_lib):
    x = np.array([[0.1, 0.7], [0.2, 0.2], [0.3, 0.3]])
    f = oracle_lib.direct("laplace", 0, x, x, np.array([3.0, 5.0]))
    assert f[0] == pytest.approx(5.0 / 0.6, rel=1e-15)
    assert f[1] == pytest.approx(3.0 / 0.6, rel=1e-15)


def test_direct_sqdist_closed_form(oracle_lib):
    """k(z) = |z|^2 has the O(N) form
    f_i = |x_i|^2 S0 - 2 x_i . S1 + S2 with S0 = sum s, S1 = sum s y, S2 = sum s |y|^2."""
    r = np.random.default_rng(11)
    x = r.random((3, 700))
    y = r.random((3, 500))
    s = r.uniform(-1, 1, 500)
    f = oracle_lib.direct("sqdist", 0, x, y, s)
    S0, S1, S2 = s.sum(), y @ s, (y * y).sum(0) @ s
    ref = (x * x).sum(0) * S0 - 2 * (S1 @ x) + S2
    np.testing.assert_allclose(f, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kern,param", [("laplace", 0.0), ("yukawa", 1.0), ("gauss", 0.01)])
def test_direct_reciprocity(oracle_lib, kern, param):
    """For a symmetric kernel the matrix A_ij = K(x_i, x_j) is symmetric, so
    s'^T (A s) = s^T (A s')."""
    r = np.random.default_rng(3)
    x = r.random((3, 800))
    s1, s2 = r.uniform(-1, 1, 800), r.uniform(-1, 1, 800)
    a = s2 @ oracle_lib.direct(kern, param, x, x, s1)
    b = s1 @ oracle_lib.direct(kern, param, x, x, s2)
    assert a == pytest.approx(b, rel=1e-12)


def test_direct_duplicate_points_skipped(oracle_lib):
    """Singular kernels drop every pair at exactly zero distance (self term and
    duplicates); finite kernels keep K(0)."""
    x = np.array([[0.5, 0.5, 0.25], [0.5, 0.5, 0.5], [0.5, 0.5, 0.5]])
    s = np.array([1.0, 2.0, 4.0])
    f = oracle_lib.direct("laplace", 0, x, x, s)
    np.testing.assert_allclose(f, [4.0 / 0.25, 4.0 / 0.25, 3.0 / 0.25], rtol=1e-15)
    g = oracle_lib.direct("gauss", 0.01, x, x, s)
    e = np.exp(-0.0625 / 0.01)
    np.testing.assert_allclose(g, [3.0 + 4 * e, 3.0 + 4 * e, 4.0 + 3 * e], rtol=1e-14)


def test_direct_compensation(oracle_lib):
    """Neumaier summation: terms 1e16, 1, -1e16 at unit distance sum to exactly 1
    (naive left-to-right summation returns 0)."""
    t = np.zeros((3, 1))
    y = np.eye(3)
    s = np.array([1e16, 1.0, -1e16])
    f = oracle_lib.direct("laplace", 0, t, y, s)
    assert f[0] == 1.0
