"""The oracle's second compression stage of Sec. 4.2: every compressed M2L matrix
C^delta = U^T K^delta U (r x r) replaced by a product Ut_o Vt_o of rank s_o, the
rank chosen by the same two singular-value filters as the first stage.  Pins,
none of which reuses the oracle's own formulas:

  * on a matrix built from random orthogonal factors and prescribed singular
    values 2^-j, the filters keep the rank counted by hand, and the error of the
    product in the spectral norm is the first dropped singular value (the
    Eckart-Young theorem), also for ranks given explicitly;
  * a finite-rank kernel (|x - y|^2, rank 5) gives C^delta of rank <= 5, so the
    two-stage pass equals the direct sum to rounding;
  * with nothing truncated the two-stage pass equals the one-stage pass;
  * at eps = 1e-6 the two-stage pass stays within the accuracy target.
"""
import numpy as np
import pytest

from paper_1408_0210_amd import workloads as W


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _orth(n, seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    return q * np.sign(np.diag(r))[None, :]


@pytest.fixture(scope="module")
def spectrum_matrix():
    n = 40
    sv = 2.0 ** -np.arange(n)
    return _orth(n, 5) @ np.diag(sv) @ _orth(n, 6).T, sv


def test_stage2_rank_and_error_by_hand(oracle_lib, spectrum_matrix):
    """sigma_j = 2^-j, eps = 1e-3: sigma_j / sigma_0 > 1e-3 holds for j <= 9 (10
    values); the prefix sums 2 (1 - 2^-m) first reach (1 - 1e-3) of the total at
    m = 10.  So s = 10 and ||C - Ut Vt||_2 = sigma_10 = 2^-10."""
    C, sv = spectrum_matrix
    s, Ut, Vt = oracle_lib.compression_factors(C[None], 1e-3)
    assert s[0] == 10
    assert Ut[0].shape == (40, 10) and Vt[0].shape == (10, 40)
    err = np.linalg.norm(C - Ut[0] @ Vt[0], 2)
    assert err == pytest.approx(2.0 ** -10, rel=1e-10)


@pytest.mark.parametrize("rank", [1, 3, 17, 40])
def test_stage2_given_rank_is_optimal(oracle_lib, spectrum_matrix, rank):
    C, sv = spectrum_matrix
    s, Ut, Vt = oracle_lib.compression_factors(C[None], 1e-3, ranks=[rank])
    assert s[0] == rank
    err = np.linalg.norm(C - Ut[0] @ Vt[0], 2)
    want = sv[rank] if rank < 40 else 0.0
    assert err == pytest.approx(want, rel=1e-9, abs=1e-14)


def test_stage2_finite_rank_exact(oracle_lib):
    """|x - y|^2 = |x|^2 - 2 x.y + |y|^2 has rank 5: both stages are exact."""
    x = W.uniform_points(1500, 21)
    s = W.potentials(1500, 24)
    P = oracle_lib.Plan("sqdist", 0, [0, 0, 0], 1.0, 3, 1e-8, compress_tol=1e-12,
                        compress_tol2=1e-12)
    for lv in P.levels.values():
        assert lv["s2"].max() <= 5
    fd = oracle_lib.direct("sqdist", 0, x, x, s)
    assert _rel(P.evaluate(x, s), fd) < 1e-11


def test_stage2_without_truncation_equals_stage1(oracle_lib):
    """Every s_o = r: Ut_o Vt_o = C^delta to rounding, so the pass is unchanged."""
    x, s = W.uniform_points(1000, 31), W.potentials(1000, 32)
    P1 = oracle_lib.Plan("laplace", 0, [0, 0, 0], 1.0, 2, 1e-4, compress_tol=1e-6)
    r = {k: lv["r"] for k, lv in P1.levels.items()}
    full = {k: np.full(316, r[k]) for k in r}
    P2 = oracle_lib.Plan("laplace", 0, [0, 0, 0], 1.0, 2, 1e-4, compress_tol=1e-6,
                         compress_rank=r, compress_tol2=1e-6, compress_rank2=full)
    assert all((P2.levels[k]["s2"] == r[k]).all() for k in r)
    assert _rel(P2.evaluate(x, s), P1.evaluate(x, s)) < 1e-12


def test_stage2_accuracy(oracle_lib, c1_inputs, c1_direct):
    """eps = 1e-6 in both stages: ranks s_o well below r, rel-L2 within 1e-6."""
    x, s, w = c1_inputs
    P = oracle_lib.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, w["depth"], w["tau"],
                        compress_tol=1e-6, compress_tol2=1e-6)
    for lv in P.levels.values():
        assert lv["s2"].max() <= lv["r"]
        assert lv["s2"].mean() < 0.8 * lv["r"]
    assert _rel(P.evaluate(x, s), c1_direct) < 1e-6
