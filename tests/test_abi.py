"""C ABI on the CPU: the library loads, exports every declared symbol, validates
its configuration, and its host setup reproduces the oracle's EIM exactly."""
import ctypes

import numpy as np
import pytest


@pytest.fixture(scope="module")
def E():
    from paper_1408_0210_amd import eifmm
    eifmm.lib()
    return eifmm


def test_exports_every_declared_symbol(E):
    names = E.declared_symbols()
    assert len(names) >= 11
    L = E.lib()
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(E):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert E.lib().eifmm_status_str(code)


@pytest.mark.parametrize("field,value", [("depth", 9), ("depth", -1), ("eim_tol", 0.0),
                                         ("L", -1.0), ("max_rhs", 0), ("kernel", 7),
                                         ("precision", 3), ("n", -5), ("struct_size", 8),
                                         ("n_targets", -1), ("n_targets", 1 << 30)])
def test_invalid_config(E, field, value):
    c = E.Config()
    c.struct_size = ctypes.sizeof(E.Config)
    c.kernel, c.kernel_param, c.L, c.n, c.depth = 0, 0.0, 1.0, 10, 2
    c.max_rhs, c.eim_tol, c.flags = 1, 1e-3, E.FLAG_HOST_ONLY
    setattr(c, field, value)
    h = ctypes.c_void_p()
    assert E.lib().eifmm_plan_create(ctypes.byref(c), ctypes.byref(h)) == -1
    assert not h.value


def test_gauss_needs_positive_width(E):
    with pytest.raises(E.EifmmError):
        E.Plan("gauss", 0.0, [0, 0, 0], 1.0, 10, 2, 1e-3, host_only=True)


def test_host_only_plan_refuses_device_calls(E):
    P = E.Plan("laplace", 0, [0, 0, 0], 1.0, 10, 2, 1e-2, host_only=True)
    assert E.lib().eifmm_set_points(P._h, None, None) == -3
    assert P.stats()["d"][2] > 0
    P.close()


def test_host_only_plan_with_targets(E):
    """A plan with separate targets accepts only set_points_targets; a host-only
    plan accepts neither."""
    P = E.Plan("laplace", 0, [0, 0, 0], 1.0, 10, 2, 1e-2, host_only=True, n_targets=7)
    L = E.lib()
    assert L.eifmm_set_points(P._h, None, None) == -3
    assert L.eifmm_set_points_targets(P._h, None, None, None) == -3
    assert P.n_out == 7
    P.close()


def test_eim_dmax_error(E):
    with pytest.raises(E.EifmmError) as e:
        E.Plan("laplace", 0, [0, 0, 0], 1.0, 10, 2, 1e-6, dmax=30, host_only=True)
    assert e.value.code == -4


@pytest.mark.parametrize("kernel,param,depth,tau", [("laplace", 0, 3, 1e-6), ("yukawa", 1.0, 3, 1e-5),
                                                    ("gauss", 1.0, 3, 1e-6), ("sqdist", 0, 3, 1e-8),
                                                    ("cosr", 20.0, 2, 1e-4), ("mq", 1.0, 3, 1e-6)])
def test_host_setup_matches_oracle(E, oracle_lib, kernel, param, depth, tau):
    """The library's greedy (complete-pivot cross approximation and a Crout
    factorisation of K(X, Y)) and the oracle's Algorithm 1 with the Gamma
    recursion select the same points and factors on the same training sets."""
    P = E.Plan(kernel, param, [0, 0, 0], 1.0, 10, depth, tau, host_only=True)
    O = oracle_lib.Plan(kernel, param, [0, 0, 0], 1.0, depth, tau)
    for k in range(2, depth + 1):
        a, b = P.level(k), O.levels[k]
        assert a["d"] == b["d"]
        np.testing.assert_array_equal(a["ia"], b["ia"])
        np.testing.assert_array_equal(a["ib"], b["ib"])
        np.testing.assert_array_equal(a["X"], b["X"])
        np.testing.assert_array_equal(a["Y"], b["Y"])
        scale = np.abs(b["G"]).max()
        assert np.abs(a["G"] - b["G"]).max() <= 1e-12 * scale
        assert np.abs(a["B"] - b["B"]).max() <= 1e-12
    P.close()


def test_host_compression_matches_oracle_svd(E, oracle_lib):
    """The library's SVD (Householder QR, then one-sided Jacobi) against numpy's:
    singular values and the projector onto the kept vectors; the kept rank is the
    rank of the two filters of Sec. 4.2, as the oracle counts it on numpy's values."""
    P = E.Plan("laplace", 0, [0, 0, 0], 1.0, 10, 2, 1e-4, host_only=True, compress_tol=1e-4)
    k = 2
    r, sv, U = P.compression(k)
    Y = P.level(k)["Y"]
    Uo, svo, ro = oracle_lib.compression_basis("laplace", 0, Y, k, 1e-4)
    m = svo / svo[0] > 1e-12
    assert np.abs(sv[m] - svo[m]).max() <= 1e-12 * svo[0]
    assert r == ro
    Uf, _, _ = oracle_lib.compression_basis("laplace", 0, Y, k, 1e-4, rank=r)
    assert np.abs(U @ U.T - Uf @ Uf.T).max() < 1e-9
    assert np.abs(U.T @ U - np.eye(r)).max() < 1e-12
    P.close()


@pytest.mark.parametrize("kernel,param,two", [("advdiff", 1.0, False), ("laplace", 0.0, True)])
def test_host_setup_second_eim_matches_oracle(E, oracle_lib, kernel, param, two):
    """The second EIM of Sec. 3.1 (D_x = J_0, D_y = I_0), run for a kernel that is
    not symmetric or on request: the same points and factors as the oracle's."""
    P = E.Plan(kernel, param, [0, 0, 0], 1.0, 10, 3, 1e-5, host_only=True, two_eim=two)
    O = oracle_lib.Plan(kernel, param, [0, 0, 0], 1.0, 3, 1e-5, two_eim=two)
    for k in (2, 3):
        for second, ref in ((False, O.levels[k]), (True, O.levels2[k])):
            a = P.level(k, second=second)
            assert a["d"] == ref["d"]
            np.testing.assert_array_equal(a["ia"], ref["ia"])
            np.testing.assert_array_equal(a["ib"], ref["ib"])
            np.testing.assert_array_equal(a["X"], ref["X"])
            np.testing.assert_array_equal(a["Y"], ref["Y"])
            assert np.abs(a["G"] - ref["G"]).max() <= 1e-12 * np.abs(ref["G"]).max()
            assert np.abs(a["B"] - ref["B"]).max() <= 1e-12
        assert P.stats()["d2"][k] == O.levels2[k]["d"]
    P.close()


def test_two_eim_compression_matches_oracle_svd(E, oracle_lib):
    """Compression with two EIMs (Sec. 4.2 for K^delta that are not symmetric): the
    singular values of K_fat (rows: the second EIM's x points) and the projector on
    U against numpy's; r covers both filtered ranks, of K_fat and of K_thin."""
    P = E.Plan("advdiff", 1.0, [0, 0, 0], 1.0, 10, 2, 1e-4, host_only=True, compress_tol=1e-4)
    k = 2
    r, sv, U = P.compression(k)
    X, Y = P.level(k, second=True)["X"], P.level(k)["Y"]
    Uo, Vo, svo, sv2o, ro = oracle_lib.compression_bases("advdiff", 1.0, X, Y, k, 1e-4)
    m = svo / svo[0] > 1e-12
    assert np.abs(sv[m] - svo[m]).max() <= 1e-12 * svo[0]
    assert r == ro
    Uf, _, _, _, _ = oracle_lib.compression_bases("advdiff", 1.0, X, Y, k, 1e-4, rank=r)
    assert U.shape == (len(X), r)
    assert np.abs(U @ U.T - Uf @ Uf.T).max() < 1e-9
    P.close()


def test_advdiff_rejects_negative_flow(E):
    with pytest.raises(E.EifmmError):
        E.Plan("advdiff", -1.0, [0, 0, 0], 1.0, 10, 2, 1e-4, host_only=True)

def test_scale_level_absolute_rule(E, oracle_lib):
    """tol_mode 1 with scale_level: the depth itself gives the same tables as the
    default; a finer level's scale (larger |K| for the Gaussian) gives the points
    the oracle's greedy selects with that level's training max as the scale."""
    kw = dict(tol_mode=1, host_only=True)
    a = E.Plan("gauss", 0.1, [0, 0, 0], 1.0, 10, 2, 1e-4, **kw)
    b = E.Plan("gauss", 0.1, [0, 0, 0], 1.0, 10, 2, 1e-4, scale_level=2, **kw)
    c = E.Plan("gauss", 0.1, [0, 0, 0], 1.0, 10, 2, 1e-4, scale_level=3, **kw)
    assert a.stats()["scale_level"] == 2 and c.stats()["scale_level"] == 3
    np.testing.assert_array_equal(a.level(2)["ia"], b.level(2)["ia"])
    sc = oracle_lib.eim("gauss", 0.1, 3, 1.0, 1e-4)["scale"]
    o = oracle_lib.eim("gauss", 0.1, 2, 1.0, 1e-4, abs_scale=sc)
    lc = c.level(2)
    assert lc["d"] == o["d"] < a.level(2)["d"]
    np.testing.assert_array_equal(lc["ia"], o["ia"])
    np.testing.assert_array_equal(lc["ib"], o["ib"])
    for P in (a, b, c):
        P.close()
    for bad in (1, EIFMM_MAX_DEPTH_PLUS_1, -1):
        with pytest.raises(E.EifmmError):
            E.Plan("gauss", 0.1, [0, 0, 0], 1.0, 10, 2, 1e-4, scale_level=bad, **kw)
    with pytest.raises(E.EifmmError):  # d_k above 1024 does not fit the device solves
        E.Plan("laplace", 0, [0, 0, 0], 1.0, 10, 2, 1e-4, dmax=2000, host_only=True)


EIFMM_MAX_DEPTH_PLUS_1 = 9


def test_host_ranks_match_oracle(E, oracle_lib):
    """Both compression stages count their ranks with the filters of Sec. 4.2; the
    library's (its own SVDs) equal the oracle's (numpy SVDs) level by level and,
    for the second stage, offset by offset."""
    P = E.Plan("laplace", 0, [0, 0, 0], 1.0, 10, 2, 1e-4, host_only=True, compress_tol=1e-5,
               compress_tol2=1e-5)
    O = oracle_lib.Plan("laplace", 0, [0, 0, 0], 1.0, 2, 1e-4, compress_tol=1e-5,
                        compress_tol2=1e-5)
    assert P.stats()["rank"][2] == O.levels[2]["r"]
    assert P.stats()["rpad"][2] == 16 * ((O.levels[2]["r"] + 15) // 16)
    np.testing.assert_array_equal(P.compression2(2), O.levels[2]["s2"])
    P.close()


def test_inputs_checked(E):
    """Points and densities the library would read through a wrong layout, or from
    host memory, are refused on the host, before any launch."""
    import torch
    f64 = torch.float64
    for bad, exc in ((torch.empty(3, 10, dtype=torch.float32), "float64"),
                     (torch.empty(3, 10, dtype=torch.int64), "float64"),
                     (torch.empty(10, 3, dtype=f64).t(), "contiguous"),
                     (torch.empty(3, 9, dtype=f64), "shape"),
                     (torch.empty(3, 10, dtype=f64), "GPU")):
        with pytest.raises(ValueError, match=exc):
            E.Plan.check_in(bad, (3, 10), "xyz")
    for bad, exc in ((torch.empty(10, dtype=torch.float32), "float64"),
                     (torch.empty(2, 3, 10, dtype=f64), "shape"),
                     (torch.empty(2, 9, dtype=f64), "shape"),
                     (torch.empty(10, 2, dtype=f64).t(), "contiguous"),
                     (torch.empty(2, 10, dtype=f64), "GPU"),
                     ([0.0] * 10, "tensor")):
        with pytest.raises(ValueError, match=exc):
            E.Plan.check_sigma(bad, 10)
    with pytest.raises(ValueError, match="problems"):
        E.Batch._ptrs([torch.empty(3, 4, dtype=f64)], [4, 5], lambda n: (3, n))
    with pytest.raises(ValueError, match="problem 0"):
        E.Batch._ptrs([torch.empty(3, 4, dtype=f64)], [4], lambda n: (3, n))


def test_evaluate_out_checked(E):
    """An output tensor the library would write past or through a wrong layout is
    refused on the host, before any launch."""
    import torch
    cpu = torch.device("cpu")
    good = torch.empty(2, 10, dtype=torch.float64)
    E.Plan.check_out(good, (2, 10), cpu)
    for bad, exc in ((torch.empty(2, 10, dtype=torch.float32), "float64"),
                     (torch.empty(10, 2, dtype=torch.float64).t(), "contiguous"),
                     (torch.empty(2, 9, dtype=torch.float64), "shape"),
                     (torch.empty(20, dtype=torch.float64), "shape")):
        with pytest.raises(ValueError, match=exc):
            E.Plan.check_out(bad, (2, 10), cpu)
    with pytest.raises(ValueError, match="on"):
        E.Plan.check_out(good, (2, 10), torch.device("cuda", 0))
