"""GPU parity of the HIP evaluation pass against the CPU oracle (through the C ABI).

Tolerances:
  * tree, leaf ranges, lists: bit-exact (integer work);
  * FP64 pass vs the oracle's Algorithm 3 on the same EIM points: both evaluate
    the same formula in a different order; cond(M_k) ~ 2e9 at tau = 1e-6 and the
    triangular solves are backward stable, so the expansions may differ by
    about cond * eps ~ 1e-7 relative in What while the potentials, which are
    well conditioned in What, agree to ~1e-12; the bound used is 1e-10;
  * any pass vs the direct sum: the requested accuracy 1e-6 (rel-L2).
"""
import numpy as np
import pytest

from paper_1408_0210_amd import workloads as W
from parity_util import assert_close, kernel_matrix, rel as _rel, solve_residual

pytestmark = pytest.mark.gpu


def _check_stages(plan, O, D, depth, kernel, param, oracle_lib):
    """W, g and l against the oracle's dumps (rel-L2 and max norm); What and lhat
    through the products they solve: M What = W and M^T lhat = l with the GPU's
    own W and l and M = K(X, Y) from the oracle's points (well conditioned,
    unlike the solved values themselves), plus the loose direct comparison."""
    for k in range(2, depth + 1):
        Wg = plan.export_expansion("W", k)
        assert_close(Wg, D["W"][k], 1e-12, f"W level {k}")
        for name in ("g", "l"):
            assert_close(plan.export_expansion(name, k), D[name][k], 1e-10, f"{name} level {k}")
        lv = O.levels[k]
        M = kernel_matrix(oracle_lib, kernel, param, lv["X"], lv["Y"])
        Wh = plan.export_expansion("What", k)
        r2, rb = solve_residual(M, Wh, Wg)
        assert r2 <= 1e-12 and rb <= 1e-11, ("What residual", k, r2, rb)
        assert _rel(Wh, D["What"][k]) < 1e-5
    lv = O.levels[depth]
    M = kernel_matrix(oracle_lib, kernel, param, lv["X"], lv["Y"])
    lh, lg = plan.export_expansion("lhat", depth), plan.export_expansion("l", depth)
    r2, rb = solve_residual(M, lh, lg, transpose=True)
    assert r2 <= 1e-12 and rb <= 1e-11, ("lhat residual", r2, rb)
    assert _rel(lh, D["lhat"]) < 1e-5


def _oracle_ranks_match(plan, O, depth):
    """The library keeps the rank of the two filters of Sec. 4.2 that the oracle
    counts on its own (numpy) singular values, level by level."""
    st = plan.stats()
    for k in range(2, depth + 1):
        assert st["rank"][k] == O.levels[k]["r"], (k, st["rank"][k], O.levels[k]["r"])
        assert st["rpad"][k] == 16 * ((O.levels[k]["r"] + 15) // 16)
        assert 0 < st["rank"][k] < st["d"][k]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def E():
    from paper_1408_0210_amd import eifmm
    eifmm.lib()
    return eifmm


def _gpu_eval(E, torch_dev, kernel, param, x, s, depth, tau, precision="fp64", plan=None,
              max_rhs=1):
    torch, dev = torch_dev
    n = x.shape[1]
    if plan is None:
        plan = E.Plan(kernel, param, [0, 0, 0], 1.0, n, depth, tau, max_rhs=max_rhs,
                      precision=precision)
    plan.set_points(torch.from_numpy(x).to(dev))
    f = plan.evaluate(torch.from_numpy(np.ascontiguousarray(s)).to(dev))
    torch.cuda.synchronize()
    return plan, f.cpu().numpy()


TREE_CASES = {
    "uniform2k_d3": lambda: (W.uniform_points(2000, 1), 3),
    "cluster3k_d4_faces": lambda: (_faces(W.cluster_points(3000, 3, 0.08, 31, 32)), 4),
    "single_point_d2": lambda: (np.array([[0.3], [0.7], [1.0]]), 2),
    "uniform500_d0": lambda: (W.uniform_points(500, 33), 0),
    "uniform500_d1": lambda: (W.uniform_points(500, 34), 1),
    "uniform100k_d5": lambda: (W.uniform_points(100_000, 35), 5),
    "cluster1m_d5": lambda: (W.make_points(W.WORKLOADS["cluster1m_yukawa"]), 5),
}


def _faces(x):
    """Add points exactly on the domain faces, edges, a corner, and duplicates."""
    x = x.copy()
    x[0, :10] = 1.0
    x[1, 10:20] = 0.0
    x[:, 20:25] = 1.0
    x[:, 25:30] = x[:, 30:35]
    return x


@pytest.mark.parametrize("case", sorted(TREE_CASES))
def test_tree_and_lists_bit_exact(case, E, torch_dev, oracle_lib):
    torch, dev = torch_dev
    x, depth = TREE_CASES[case]()
    n = x.shape[1]
    plan = E.Plan("laplace", 0, [0, 0, 0], 1.0, n, depth, 1e-2)
    plan.set_points(torch.from_numpy(x).to(dev))
    perm, ls, keys = plan.export_tree()
    okeys, operm, ols = oracle_lib.tree(x, [0, 0, 0], 1.0, depth)
    np.testing.assert_array_equal(perm, operm)
    np.testing.assert_array_equal(ls, ols)
    np.testing.assert_array_equal(keys, okeys[operm])
    for level in range(0, depth + 1):
        g = plan.export_lists(level)
        o = oracle_lib.lists(ols, depth, level)
        for name in ("active", "near_ptr", "near_src"):
            np.testing.assert_array_equal(g[name], o[name], err_msg=f"{name} level {level}")
        if level >= 2:
            for name in ("il_ptr", "il_src", "il_off"):
                np.testing.assert_array_equal(g[name], o[name], err_msg=f"{name} level {level}")
            st = plan.stats()
            assert st["il_pairs"][level] == len(o["il_src"])
    plan.close()


@pytest.mark.parametrize("depth,dist", [(3, "uniform"), (4, "cluster")])
def test_finite_rank_pass_exact(depth, dist, E, torch_dev, oracle_lib):
    """k(z) = |z|^2 is interpolated exactly (rank 5): the GPU pass must equal the
    direct sum to rounding, which checks every index and translation path."""
    x = W.uniform_points(3000, 41) if dist == "uniform" else W.cluster_points(3000, 3, 0.05, 42, 43)
    s = W.potentials(3000, 44)
    plan, f = _gpu_eval(E, torch_dev, "sqdist", 0, x, s, depth, 1e-8)
    assert all(v == 5 for v in plan.stats()["d"].values())
    fd = oracle_lib.direct("sqdist", 0, x, x, s)
    assert _rel(f, fd) < 1e-12
    plan.close()


def test_near_field_only(E, torch_dev, oracle_lib):
    """depth < 2: no well-separated pairs, the pass is the near field alone."""
    x = W.uniform_points(3000, 45)
    s = W.potentials(3000, 46)
    for depth in (0, 1):
        plan, f = _gpu_eval(E, torch_dev, "laplace", 0, x, s, depth, 1e-6)
        assert _rel(f, oracle_lib.direct("laplace", 0, x, x, s)) < 1e-13
        plan.close()


def test_crowded_leaves_vs_oracle(E, torch_dev, oracle_lib):
    """One tight cluster at depth 2: leaves of thousands of points, split into many
    64-target chunks (ragged last chunk) by the near-field and L2P kernels."""
    x = W.cluster_points(20000, 1, 0.05, 91, 92)
    s = W.potentials(20000, 93)
    plan, f = _gpu_eval(E, torch_dev, "laplace", 0, x, s, 2, 1e-6)
    O = oracle_lib.Plan("laplace", 0, [0, 0, 0], 1.0, 2, 1e-6)
    assert_close(f, O.evaluate(x, s), 1e-10, "vs oracle EIFMM")
    fd = oracle_lib.direct("laplace", 0, x, x, s)
    assert_close(f, fd, 1e-6, "vs direct sum", max_tol=1e-5)
    plan.close()
    plan, f = _gpu_eval(E, torch_dev, "laplace", 0, x, s, 2, 1e-6, precision="mixed")
    assert _rel(f, fd) < 1e-6
    plan.close()


def test_c1_fp64_vs_oracle(E, torch_dev, c1_inputs, c1_plan, c1_direct):
    """2000 uniform points, 1/r, depth 3, tau 1e-6, FP64."""
    x, s, w = c1_inputs
    plan, f = _gpu_eval(E, torch_dev, w["kernel"], w["param"], x, s, w["depth"], w["tau"])
    for k in range(2, w["depth"] + 1):
        a, b = plan.level(k), c1_plan.levels[k]
        assert a["d"] == b["d"]
        np.testing.assert_array_equal(a["ia"], b["ia"])
        np.testing.assert_array_equal(a["ib"], b["ib"])
    fo = c1_plan.evaluate(x, s)
    assert_close(f, fo, 1e-10, "vs oracle EIFMM")
    assert_close(f, c1_direct, 1e-6, "vs direct sum", max_tol=1e-5)
    plan.close()


def test_c1_stages_vs_oracle(E, torch_dev, oracle_lib, c1_inputs, c1_plan):
    """Each expansion of Algorithm 3 (W, What, g, l, lhat) against the oracle."""
    x, s, w = c1_inputs
    plan, f = _gpu_eval(E, torch_dev, w["kernel"], w["param"], x, s, w["depth"], w["tau"])
    _, D = c1_plan.evaluate(x, s, dumps=True)
    _check_stages(plan, c1_plan, D, w["depth"], w["kernel"], w["param"], oracle_lib)
    plan.close()


@pytest.mark.parametrize("precision,depth,nrhs,mode", [("fp64", 3, 1, 1), ("mixed", 3, 1, 2),
                                                      ("mixed", 3, 2, 1), ("fp64", 1, 1, 0)])
def test_near_field_placement(precision, depth, nrhs, mode, E, torch_dev, oracle_lib):
    """Where the pass runs the near field (eifmm_stats.near_mode): on the plan's
    second stream from P2M on in FP64 and with several right-hand sides, from the
    M2L on in mixed precision with one, on the caller's stream below depth 2 (no
    far field); each placement against the direct sum."""
    torch, dev = torch_dev
    n = 12000
    x = W.uniform_points(n, 81)
    S = np.stack([W.potentials(n, 82), W.potentials(n, 83)])[:nrhs]
    plan = E.Plan("laplace", 0, [0, 0, 0], 1.0, n, depth, 1e-6, max_rhs=2, precision=precision)
    plan.set_points(torch.from_numpy(x).to(dev))
    F = plan.evaluate(torch.from_numpy(np.ascontiguousarray(S if nrhs > 1 else S[0])).to(dev))
    F = F.cpu().numpy().reshape(nrhs, n)
    assert plan.stats()["near_mode"] == mode
    for r in range(nrhs):
        err = _rel(F[r], oracle_lib.direct("laplace", 0, x, x, S[r]))
        assert err <= (1e-13 if depth < 2 else 1e-6), (r, err)
    plan.close()


def test_multi_rhs_matches_single(E, torch_dev, oracle_lib):
    """nrhs = 5 (several column tiles with a ragged tail) equals 5 single passes."""
    torch, dev = torch_dev
    x = W.uniform_points(2500, 51)
    S = np.stack([W.potentials(2500, 60 + r) for r in range(5)])
    plan = E.Plan("laplace", 0, [0, 0, 0], 1.0, 2500, 3, 1e-4, max_rhs=8)
    plan.set_points(torch.from_numpy(x).to(dev))
    F = plan.evaluate(torch.from_numpy(S).to(dev)).cpu().numpy()
    for r in range(5):
        f1 = plan.evaluate(torch.from_numpy(S[r].copy()).to(dev)).cpu().numpy()
        assert _rel(F[r], f1) < 1e-14
    fd = oracle_lib.direct("laplace", 0, x, x, S[3])
    assert _rel(F[3], fd) < 1e-4
    plan.close()


@pytest.mark.parametrize("kernel,param,tau", [("yukawa", 1.0, 1e-6), ("gauss", 0.1, 1e-6),
                                              ("cosr", 20.0, 1e-4), ("mq", 1.0, 1e-6)])
def test_other_kernels_vs_oracle(kernel, param, tau, E, torch_dev, oracle_lib):
    x = W.cluster_points(2000, 4, 0.1, 71, 72)
    s = W.potentials(2000, 73)
    plan, f = _gpu_eval(E, torch_dev, kernel, param, x, s, 3, tau)
    O = oracle_lib.Plan(kernel, param, [0, 0, 0], 1.0, 3, tau)
    assert_close(f, O.evaluate(x, s), 1e-10, f"{kernel} vs oracle EIFMM")
    assert _rel(f, oracle_lib.direct(kernel, param, x, x, s)) < max(1e-5, 10 * tau)
    plan.close()


def test_mixed_precision_small(E, torch_dev, c1_inputs, c1_direct):
    x, s, w = c1_inputs
    plan, f = _gpu_eval(E, torch_dev, w["kernel"], w["param"], x, s, w["depth"], w["tau"],
                        precision="mixed")
    assert _rel(f, c1_direct) < 1e-6
    plan.close()


def test_deterministic(E, torch_dev, c1_inputs):
    torch, dev = torch_dev
    x, s, w = c1_inputs
    for prec in ("fp64", "mixed"):
        plan = E.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, w["n"], w["depth"], w["tau"],
                      precision=prec)
        plan.set_points(torch.from_numpy(x).to(dev))
        st = torch.from_numpy(s).to(dev)
        a = plan.evaluate(st).cpu().numpy()
        b = plan.evaluate(st).cpu().numpy()
        np.testing.assert_array_equal(a, b)
        plan.close()


def test_degenerate_inputs(E, torch_dev, oracle_lib):
    """No points; one point; 300 copies of one point.  A singular kernel skips
    every pair at distance 0, so 1/r gives exactly zero for coincident points;
    exp(-r^2) counts them all (f_i = sum of sigma)."""
    torch, dev = torch_dev
    P = E.Plan("laplace", 0, [0, 0, 0], 1.0, 0, 3, 1e-4)
    P.set_points(torch.zeros(3, 0, dtype=torch.float64, device=dev))
    f = P.evaluate(torch.zeros(0, dtype=torch.float64, device=dev))
    torch.cuda.synchronize()
    assert f.numel() == 0
    P.close()
    one = np.array([[0.25], [0.5], [0.75]])
    P, f = _gpu_eval(E, torch_dev, "laplace", 0, one, np.array([2.0]), 3, 1e-4)
    P.close()
    np.testing.assert_array_equal(f, [0.0])
    same = np.repeat(np.array([[0.3], [0.6], [0.9]]), 300, axis=1)
    s = W.potentials(300, 5)
    P, f = _gpu_eval(E, torch_dev, "laplace", 0, same, s, 3, 1e-4)
    P.close()
    np.testing.assert_array_equal(f, np.zeros(300))
    P, f = _gpu_eval(E, torch_dev, "gauss", 1.0, same, s, 3, 1e-6)
    P.close()
    np.testing.assert_allclose(f, np.full(300, s.sum()), rtol=0, atol=1e-12 * np.abs(s).sum())
    np.testing.assert_allclose(oracle_lib.direct("gauss", 1.0, same, same, s), f, rtol=0,
                               atol=1e-12 * np.abs(s).sum())


def test_evaluate_on_another_stream(E, torch_dev, c1_inputs):
    """The pass follows the caller's stream (its near field forks to the plan's
    second stream and joins back): the same bits on a side torch stream."""
    torch, dev = torch_dev
    x, s, w = c1_inputs
    plan = E.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, x.shape[1], w["depth"], w["tau"])
    plan.set_points(torch.from_numpy(x).to(dev))
    sd = torch.from_numpy(s).to(dev)
    f0 = plan.evaluate(sd)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        f1 = plan.evaluate(sd)
        f2 = plan.evaluate(sd)
    side.synchronize()
    np.testing.assert_array_equal(f1.cpu().numpy(), f0.cpu().numpy())
    np.testing.assert_array_equal(f2.cpu().numpy(), f0.cpu().numpy())
    plan.close()


def test_error_paths(E, torch_dev):
    torch, dev = torch_dev
    x = W.uniform_points(100, 81)
    plan = E.Plan("laplace", 0, [0, 0, 0], 1.0, 100, 2, 1e-3, max_rhs=2)
    s = torch.from_numpy(W.potentials(100, 82)).to(dev)
    with pytest.raises(E.EifmmError) as e:
        plan.evaluate(s)
    assert e.value.code == -3  # evaluate before set_points
    bad = x.copy()
    bad[2, 7] = 1.5
    with pytest.raises(E.EifmmError) as e:
        plan.set_points(torch.from_numpy(bad).to(dev))
    assert e.value.code == -2
    bad[2, 7] = np.nan
    with pytest.raises(E.EifmmError) as e:
        plan.set_points(torch.from_numpy(bad).to(dev))
    assert e.value.code == -2
    with pytest.raises(E.EifmmError):
        plan.evaluate(s)  # the failed set_points left no points
    plan.set_points(torch.from_numpy(x).to(dev))
    f = torch.empty(3, 100, dtype=torch.float64, device=dev)
    s3 = torch.zeros(3, 100, dtype=torch.float64, device=dev)
    assert plan.evaluate_raw(s3.data_ptr(), 3, 100, f.data_ptr(), 100) == -1  # nrhs > max_rhs
    assert plan.evaluate_raw(s3.data_ptr(), 1, 50, f.data_ptr(), 100) == -1   # ld < n
    assert plan.evaluate_raw(None, 1, 100, f.data_ptr(), 100) == -1
    plan.evaluate(s)  # still usable
    torch.cuda.synchronize()
    plan.close()


def test_compressed_fp64_vs_oracle(E, torch_dev, oracle_lib, c1_inputs, c1_direct):
    """M2L compression (Sec. 4.2): the GPU pass against the oracle's compressed pass
    with the same kept rank per level."""
    torch, dev = torch_dev
    x, s, w = c1_inputs
    plan = E.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, w["n"], w["depth"], w["tau"],
                  compress_tol=1e-6)
    O = oracle_lib.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, w["depth"], w["tau"],
                        compress_tol=1e-6)
    _oracle_ranks_match(plan, O, w["depth"])
    plan.set_points(torch.from_numpy(x).to(dev))
    f = plan.evaluate(torch.from_numpy(s).to(dev)).cpu().numpy()
    assert_close(f, O.evaluate(x, s), 1e-10, "vs oracle compressed EIFMM")
    assert_close(f, c1_direct, 1e-6, "vs direct sum", max_tol=1e-5)
    plan.close()


@pytest.mark.parametrize("depth", [2, 3])
def test_compressed_stages_vs_oracle(depth, E, torch_dev, oracle_lib, c1_inputs):
    """With compression the pass folds the factor B^{-T} of Delta = B^{-T} Gamma^{-1}
    into the projection (What' = U^T B^{-T} (Gamma^{-1} W)).  The result and every
    expansion, including What, which the export computes on demand on compressed
    levels, against the oracle's compressed pass, which solves for What."""
    torch, dev = torch_dev
    x, s, w = c1_inputs
    plan = E.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, w["n"], depth, w["tau"],
                  compress_tol=1e-6)
    O = oracle_lib.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, depth, w["tau"],
                        compress_tol=1e-6)
    _oracle_ranks_match(plan, O, depth)
    plan.set_points(torch.from_numpy(x).to(dev))
    f = plan.evaluate(torch.from_numpy(s).to(dev)).cpu().numpy()
    fo, D = O.evaluate(x, s, dumps=True)
    assert_close(f, fo, 1e-10, "vs oracle compressed EIFMM")
    _check_stages(plan, O, D, depth, w["kernel"], w["param"], oracle_lib)
    # the on-demand exports leave the pass intact
    f2 = plan.evaluate(torch.from_numpy(s).to(dev)).cpu().numpy()
    np.testing.assert_array_equal(f2, f)
    plan.close()


def test_compressed_mixed_and_multi_rhs(E, torch_dev, oracle_lib, c1_inputs, c1_direct):
    torch, dev = torch_dev
    x, s, w = c1_inputs
    plan = E.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, w["n"], w["depth"], w["tau"],
                  compress_tol=1e-6, precision="mixed", max_rhs=3)
    plan.set_points(torch.from_numpy(x).to(dev))
    S = np.stack([s, W.potentials(w["n"], 90), -s])
    F = plan.evaluate(torch.from_numpy(S).to(dev)).cpu().numpy()
    assert _rel(F[0], c1_direct) < 1e-6
    assert _rel(F[2], -c1_direct) < 1e-6
    plan.close()


def test_compressed_finite_rank_exact(E, torch_dev, oracle_lib):
    torch, dev = torch_dev
    x = W.uniform_points(3000, 41)
    s = W.potentials(3000, 44)
    plan = E.Plan("sqdist", 0, [0, 0, 0], 1.0, 3000, 3, 1e-8, compress_tol=1e-12)
    plan.set_points(torch.from_numpy(x).to(dev))
    f = plan.evaluate(torch.from_numpy(s).to(dev)).cpu().numpy()
    assert _rel(f, oracle_lib.direct("sqdist", 0, x, x, s)) < 1e-11
    plan.close()


def test_compressed_stage2_vs_oracle(E, torch_dev, oracle_lib, c1_inputs, c1_direct):
    """Second compression stage (Sec. 4.2): each C^delta replaced by the product of
    its two factors; the FP64 pass applies the factors (two MFMA products per
    interaction), the FP32 pass their dense product.  Against the oracle's pass
    with the same ranks (its factors from an exact SVD)."""
    torch, dev = torch_dev
    x, s, w = c1_inputs
    plan = E.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, w["n"], w["depth"], w["tau"],
                  compress_tol=1e-6, compress_tol2=1e-6)
    O = oracle_lib.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, w["depth"], w["tau"],
                        compress_tol=1e-6, compress_tol2=1e-6)
    _oracle_ranks_match(plan, O, w["depth"])
    ranks = plan.stats()["rank"]
    s2 = {k: plan.compression2(k) for k in ranks}
    assert all(0 < v.max() < ranks[k] for k, v in s2.items())
    for k in ranks:  # the second stage's ranks, from the oracle's own SVDs of C^delta
        np.testing.assert_array_equal(s2[k], O.levels[k]["s2"], err_msg=f"level {k}")
    plan.set_points(torch.from_numpy(x).to(dev))
    f = plan.evaluate(torch.from_numpy(s).to(dev)).cpu().numpy()
    assert_close(f, O.evaluate(x, s), 1e-10, "vs oracle stage-2 EIFMM")
    assert_close(f, c1_direct, 1e-6, "vs direct sum", max_tol=1e-5)
    plan.close()
    plan = E.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, w["n"], w["depth"], w["tau"],
                  compress_tol=1e-6, compress_tol2=1e-6, precision="mixed", max_rhs=2)
    plan.set_points(torch.from_numpy(x).to(dev))
    S = np.stack([s, -s])
    F = plan.evaluate(torch.from_numpy(S).to(dev)).cpu().numpy()
    assert _rel(F[0], f) < 1e-6
    np.testing.assert_array_equal(F[1], -F[0])
    plan.close()


def test_compressed_stage2_multi_rhs(E, torch_dev, c1_inputs):
    """nrhs = 3 (ragged 64-column tiles) equals three single passes, FP64."""
    torch, dev = torch_dev
    x, s, w = c1_inputs
    plan = E.Plan(w["kernel"], w["param"], [0, 0, 0], 1.0, w["n"], w["depth"], w["tau"],
                  compress_tol=1e-6, compress_tol2=1e-6, max_rhs=3)
    plan.set_points(torch.from_numpy(x).to(dev))
    S = np.stack([s, W.potentials(w["n"], 95), W.potentials(w["n"], 96)])
    F = plan.evaluate(torch.from_numpy(S).to(dev)).cpu().numpy()
    for r in range(3):
        fr = plan.evaluate(torch.from_numpy(S[r]).to(dev)).cpu().numpy()
        assert _rel(F[r], fr) < 1e-13
    plan.close()
