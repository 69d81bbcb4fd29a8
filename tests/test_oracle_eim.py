"""Pins for the oracle's greedy EIM (Algorithm 1, the Gamma recursion and the
interpolation property of Sec. 2).  CPU only."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def lap2(oracle_lib):
    return oracle_lib.eim("laplace", 0, 2, 1.0, 1e-4)


def _K(oracle_lib, kern, param, A, B):
    """Kernel matrix K(a_i, b_j) through the oracle's point kernel."""
    z = (A[:, None, :] - B[None, :, :]).reshape(-1, 3)
    return oracle_lib.kernel_eval(kern, param, z).reshape(A.shape[0], B.shape[0])


@pytest.mark.parametrize("kern,param,rank", [
    ("sqdist", 0.0, 5),                 # |x|^2 - 2 x.y + |y|^2: span{1, x, |x|^2}
    ("cosdot", [3.0, 1.0, 2.0], 2),     # cos(w.x)cos(w.y) + sin(w.x)sin(w.y)
    ("expdot", [1.0, 0.5, -0.3], 1),    # exp(a.x) exp(-a.y)
])
def test_finite_rank_stops_at_rank(oracle_lib, kern, param, rank):
    """Under (H) the greedy can only add as many points as the rank of K; after
    that the residual vanishes to rounding and the stopping rule ends the loop."""
    e = oracle_lib.eim(kern, param, 2, 1.0, 1e-10)
    assert e["status"] == 0
    assert e["d"] == rank


def test_factors_structure(oracle_lib, lap2):
    e = lap2
    d, B, G = e["d"], e["B"], e["G"]
    assert d > 10
    # B unit lower triangular with |B_lm| = |q_m(y_l)| <= 1 (q_m peaks at y_m)
    np.testing.assert_array_equal(np.diag(B), np.ones(d))
    assert np.all(np.triu(B, 1) == 0)
    assert np.abs(B).max() <= 1.0 + 1e-15
    # Gamma lower triangular (Sec. 2 calls it upper, but its recursion sets
    # Gamma_{m,k+1} = 0 for m <= k); the diagonal holds the greedy pivots, whose
    # magnitudes are the successive training-set errors eps_k
    assert np.all(np.triu(G, 1) == 0)
    np.testing.assert_allclose(np.abs(np.diag(G)), e["eps"][:d], rtol=0, atol=0)


def test_gamma_bt_is_kernel_matrix(oracle_lib, lap2):
    """Delta = B^{-T} Gamma^{-1} is the inverse of M = K(X, Y): M = Gamma B^T."""
    e = lap2
    M = _K(oracle_lib, "laplace", 0, e["X"], e["Y"])
    R = e["G"] @ e["B"].T - M
    assert np.abs(R).max() <= 1e-12 * np.abs(M).max()


def test_delta_times_m_is_identity(oracle_lib, lap2):
    e = lap2
    M = _K(oracle_lib, "laplace", 0, e["X"], e["Y"])
    for j in (0, 7, e["d"] // 2, e["d"] - 1):
        w = oracle_lib.apply_delta(e["B"], e["G"], M[:, j])
        ej = np.zeros(e["d"]); ej[j] = 1
        np.testing.assert_allclose(w, ej, atol=1e-8)
        wt = oracle_lib.apply_delta(e["B"], e["G"], M[j, :], transpose=True)
        np.testing.assert_allclose(wt, ej, atol=1e-8)


def test_interpolation_property(oracle_lib, lap2):
    """Property 2.1: I_d K(x, y_m) = K(x, y_m) for all x and I_d K(x_m, y) = K(x_m, y)
    for all y, with I_d K(x, y) = K(x, Y) Delta K(X, y) (eq. (5))."""
    e = lap2
    tx, ty = oracle_lib.training_sets("laplace", 2)
    lk = 2.0 ** -3
    r = np.random.default_rng(1)
    xs = tx[r.choice(len(tx), 300, replace=False)] * lk
    ys = ty[r.choice(len(ty), 100, replace=False)] * lk
    KxY = _K(oracle_lib, "laplace", 0, xs, e["Y"])
    for m in (0, 5, e["d"] - 1):
        v = oracle_lib.apply_delta(e["B"], e["G"], _K(oracle_lib, "laplace", 0, e["X"], e["Y"][m:m + 1])[:, 0])
        ref = _K(oracle_lib, "laplace", 0, xs, e["Y"][m:m + 1])[:, 0]
        np.testing.assert_allclose(KxY @ v, ref, rtol=1e-9)
        row = _K(oracle_lib, "laplace", 0, e["X"][m:m + 1], e["Y"])[0]
        KXy = _K(oracle_lib, "laplace", 0, e["X"], ys)
        I = np.array([row @ oracle_lib.apply_delta(e["B"], e["G"], KXy[:, j]) for j in range(len(ys))])
        np.testing.assert_allclose(I, _K(oracle_lib, "laplace", 0, e["X"][m:m + 1], ys)[0], rtol=1e-9)


def test_stopping_rule(oracle_lib, lap2):
    """Stop on eps_k (end of Sec. 2): the last accepted pivot exceeds tau*eps_0 and
    the training error after d points does not."""
    e = lap2
    d, eps = e["d"], e["eps"]
    assert eps[d] <= 1e-4 * eps[0] < eps[d - 1]
    assert eps[0] == e["scale"]


def test_dmax_error(oracle_lib):
    e = oracle_lib.eim("laplace", 0, 2, 1.0, 1e-6, dmax=20)
    assert e["status"] == oracle_lib.EEIM and e["d"] == 20


def test_laplace_homogeneous_levels(oracle_lib):
    """1/r is homogeneous (Sec. 5.3): with training sets that scale with l_k, every
    level selects the same number of points at the same scaled positions."""
    es = [oracle_lib.eim("laplace", 0, k, 1.0, 1e-4) for k in (2, 3, 4)]
    assert es[0]["d"] == es[1]["d"] == es[2]["d"]
    for a, b in zip(es, es[1:]):
        np.testing.assert_array_equal(a["ia"], b["ia"])
        np.testing.assert_array_equal(a["ib"], b["ib"])
        np.testing.assert_array_equal(a["X"] / 2, b["X"])
        np.testing.assert_array_equal(a["Y"] / 2, b["Y"])


@pytest.mark.parametrize("kern,param", [("laplace", 0.0), ("yukawa", 1.0)])
def test_heldout_error_bounded(oracle_lib, kern, param):
    """For harmonic / modified-Helmholtz kernels the interpolation error is bounded
    by its maximum on the training surfaces (maximum principle), so random points
    of I_0 x J_0 stay within a small multiple of tau*eps_0."""
    tau = 1e-4
    e = oracle_lib.eim(kern, param, 2, 1.0, tau)
    lk = 2.0 ** -3
    r = np.random.default_rng(7)
    u = r.uniform(-7, 7, (6000, 3))
    u = u[np.abs(u).max(1) >= 3][:2000]
    v = r.uniform(-3, 3, (2000, 3))
    nrm = np.abs(v).max(1)
    near = v / nrm[:, None] * r.uniform(3, 3.5, 2000)[:, None]  # close to the inner shell
    xs = np.concatenate([u, near]) * lk
    ys = r.uniform(-1, 1, (500, 3)) * lk
    Kt = _K(oracle_lib, kern, param, xs, ys)
    KxY = _K(oracle_lib, kern, param, xs, e["Y"])
    KXy = _K(oracle_lib, kern, param, e["X"], ys)
    DK = np.stack([oracle_lib.apply_delta(e["B"], e["G"], KXy[:, j]) for j in range(len(ys))], 1)
    err = np.abs(Kt - KxY @ DK).max() / e["scale"]
    assert err <= 2 * tau


def test_inhomogeneous_rank_falls_with_depth(oracle_lib):
    """Sec. 5.4.1: for an inhomogeneous kernel (exp(-r^2)) the greedy needs fewer
    points on deeper levels."""
    ds = [oracle_lib.eim("gauss", 1.0, k, 1.0, 1e-6)["d"] for k in (2, 3, 4)]
    assert ds[0] > ds[1] > ds[2]


@pytest.mark.parametrize("kern,param,tau", [("gauss", 1.0, 1e-6), ("cosr", 20.0, 1e-4),
                                            ("mq", 1.0, 1e-6)])
def test_heldout_error_bounded_volume(oracle_lib, kern, param, tau):
    """The kernels of Sec. 5.4 obey no maximum principle, so their training sets
    fill the volumes (an 11^3 grid of J_0 and close shells through I_0): at points
    drawn anywhere in I_0 x J_0, away from every training point, the interpolation
    error must stay within 1.25 tau * eps_0, i.e. the training grid resolves the
    residual of the whole domain (trained on the surfaces only, exp(-r^2) and
    sqrt(r^2+1) miss interior maxima of 2.0 and 1.5 tau at level 2)."""
    k = 2
    e = oracle_lib.eim(kern, param, k, 1.0, tau)
    lk = 2.0 ** -(k + 1)
    top = 2 ** (k + 1) - 1
    r = np.random.default_rng(17)
    u = r.uniform(-top, top, (12000, 3))
    xs = u[np.abs(u).max(1) >= 3][:2500] * lk
    ys = r.uniform(-1, 1, (300, 3)) * lk
    Kt = _K(oracle_lib, kern, param, xs, ys)
    KxY = _K(oracle_lib, kern, param, xs, e["Y"])
    KXy = _K(oracle_lib, kern, param, e["X"], ys)
    DK = np.stack([oracle_lib.apply_delta(e["B"], e["G"], KXy[:, j]) for j in range(len(ys))], 1)
    err = np.abs(Kt - KxY @ DK).max() / e["scale"]
    assert err <= 1.25 * tau, err


def test_absolute_rule_scale_is_training_max(oracle_lib):
    """tol_mode 1 (one absolute threshold for all levels): the scale handed to a
    level's greedy is the largest |K| over another level's training grid, which is
    the first pivot of that level's own greedy; a larger scale (a finer level of
    the Gaussian, whose values near the box are larger) can only stop earlier."""
    kern, param, tau = "gauss", 0.1, 1e-4
    e2, e3 = (oracle_lib.eim(kern, param, k, 1.0, tau) for k in (2, 3))
    tx, ty = oracle_lib.training_sets(kern, 3)
    lk = 2.0 ** -4
    assert e3["scale"] == np.abs(_K(oracle_lib, kern, param, tx * lk, ty * lk)).max()
    a = oracle_lib.eim(kern, param, 2, 1.0, tau, abs_scale=e3["scale"])
    assert a["scale"] == e3["scale"] > 1.5 * e2["scale"]
    assert 0 < a["d"] < e2["d"]
    assert np.abs(a["G"][a["d"] - 1, a["d"] - 1]) > tau * e3["scale"] >= a["eps"][a["d"]]
