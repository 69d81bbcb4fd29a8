"""Separate targets and sources: f(x_i) = sum_j sigma_j K(x_i, y_j) (eq. (1) with
targets x_i that are not the sources y_j).

The plan sorts sources and targets into one octree by (leaf key, source before
target, input index).  Numbered as one union array (sources first), that is the
oracle's (key, index) order of the union, so the tree is checked bit for bit
against the oracle's.  With zero potentials at the targets, the union's N-body
pass computes the same sums: the far field identically (same boxes, same
sources in the same order), the near field up to the order of additions.  So
the separate-target pass is compared with the oracle's plain EIFMM on the union
(1e-10, as the N-body parity tests) and with the direct sum (the 1e-6 target).
"""
import numpy as np
import pytest

from paper_1408_0210_amd import workloads as W
from parity_util import assert_close

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


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


def _run(E, torch_dev, kernel, param, xs, xt, s, depth, tau, precision="fp64", compress_tol=0.0,
         max_rhs=1):
    torch, dev = torch_dev
    plan = E.Plan(kernel, param, [0, 0, 0], 1.0, xs.shape[1], depth, tau, max_rhs=max_rhs,
                  precision=precision, compress_tol=compress_tol, n_targets=xt.shape[1])
    plan.set_points(torch.from_numpy(np.ascontiguousarray(xs)).to(dev),
                    targets=torch.from_numpy(np.ascontiguousarray(xt)).to(dev))
    f = plan.evaluate(torch.from_numpy(np.ascontiguousarray(s)).to(dev))
    torch.cuda.synchronize()
    return plan, f.cpu().numpy()


def test_tree_matches_oracle_union(E, torch_dev, oracle_lib):
    """perm, leaf_start and keys equal the oracle's tree of the union, bit for bit."""
    xs = W.cluster_points(3000, 2, 0.05, 11, 12)
    xt = W.uniform_points(1500, 13)
    plan, _ = _run(E, torch_dev, "laplace", 0, xs, xt, W.potentials(3000, 14), 4, 1e-4)
    perm, ls, keys = plan.export_tree()
    ko, po, lso = oracle_lib.tree(np.concatenate([xs, xt], axis=1), [0, 0, 0], 1.0, 4)
    np.testing.assert_array_equal(perm, po)
    np.testing.assert_array_equal(ls, lso)
    np.testing.assert_array_equal(keys, ko[po])
    plan.close()


@pytest.mark.parametrize("kernel,param,depth,compress", [("laplace", 0.0, 3, 0.0),
                                                         ("laplace", 0.0, 3, 1e-6),
                                                         ("yukawa", 1.0, 3, 0.0),
                                                         ("gauss", 1.0, 2, 0.0)])
def test_targets_vs_oracle_union(kernel, param, depth, compress, E, torch_dev, oracle_lib):
    """3000 uniform sources, 2000 uniform targets (other seeds)."""
    xs, xt = W.uniform_points(3000, 21), W.uniform_points(2000, 22)
    s = W.potentials(3000, 23)
    plan, f = _run(E, torch_dev, kernel, param, xs, xt, s, depth, 1e-6, compress_tol=compress)
    xu = np.concatenate([xs, xt], axis=1)
    su = np.concatenate([s, np.zeros(2000)])
    O = oracle_lib.Plan(kernel, param, [0, 0, 0], 1.0, depth, 1e-6, compress_tol=compress)
    if compress:
        assert plan.stats()["rank"] == {k: O.levels[k]["r"] for k in range(2, depth + 1)}
    fo = O.evaluate(xu, su)[3000:]
    assert_close(f, fo, 1e-10, "vs oracle EIFMM on the union")
    fd = oracle_lib.direct(kernel, param, xt, xs, s)
    assert_close(f, fd, 1e-6, "vs direct sum", max_tol=1e-5)
    plan.close()


def test_targets_vs_union_plan(E, torch_dev):
    """The same library on the union with zero target potentials (an N-body plan):
    far field identical, near field up to the order of additions."""
    torch, dev = torch_dev
    xs, xt = W.uniform_points(4000, 31), W.uniform_points(3000, 32)
    s = W.potentials(4000, 33)
    plan, f = _run(E, torch_dev, "laplace", 0, xs, xt, s, 3, 1e-6)
    plan.close()
    xu = np.concatenate([xs, xt], axis=1)
    U = E.Plan("laplace", 0, [0, 0, 0], 1.0, 7000, 3, 1e-6)
    U.set_points(torch.from_numpy(xu).to(dev))
    fu = U.evaluate(torch.from_numpy(np.concatenate([s, np.zeros(3000)])).to(dev)).cpu().numpy()
    U.close()
    assert _rel(f, fu[4000:]) < 1e-13


def test_targets_coinciding_with_sources(E, torch_dev, oracle_lib):
    """Targets that are copies of sources skip the r = 0 pair (singular kernel),
    so they equal the N-body result at those sources."""
    torch, dev = torch_dev
    xs = W.uniform_points(2500, 41)
    s = W.potentials(2500, 42)
    pick = np.random.default_rng(43).choice(2500, 600, replace=False)
    xt = np.ascontiguousarray(xs[:, pick])
    plan, f = _run(E, torch_dev, "laplace", 0, xs, xt, s, 3, 1e-6)
    plan.close()
    N = E.Plan("laplace", 0, [0, 0, 0], 1.0, 2500, 3, 1e-6)
    N.set_points(torch.from_numpy(xs).to(dev))
    fn = N.evaluate(torch.from_numpy(s).to(dev)).cpu().numpy()
    N.close()
    assert _rel(f, fn[pick]) < 1e-13
    assert _rel(f, oracle_lib.direct("laplace", 0, xt, xs, s)) < 1e-6


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_targets_apart_from_sources(precision, E, torch_dev, oracle_lib):
    """Sources in one tight cluster, targets spread over the cube: most target
    leaves hold no source and the source leaves hold no target."""
    xs = W.cluster_points(6000, 1, 0.04, 51, 52)
    xt = W.uniform_points(4000, 53)
    s = W.potentials(6000, 54)
    plan, f = _run(E, torch_dev, "yukawa", 1.0, xs, xt, s, 4, 1e-6, precision=precision)
    assert _rel(f, oracle_lib.direct("yukawa", 1.0, xt, xs, s)) < 1e-6
    st = plan.stats()
    assert st["near_point_pairs"] > 0
    plan.close()


@pytest.mark.parametrize("ns,nt,depth", [(1, 1, 2), (1, 500, 3), (500, 1, 3), (800, 300, 1),
                                         (0, 10, 2)])
def test_targets_edge_sizes(ns, nt, depth, E, torch_dev, oracle_lib):
    """A single source or target, near field only (depth 1), no sources at all."""
    xs = W.uniform_points(ns, 61) if ns else np.zeros((3, 0))
    xt = W.uniform_points(nt, 62)
    s = W.potentials(ns, 63)
    plan, f = _run(E, torch_dev, "laplace", 0, xs, xt, s, depth, 1e-6)
    plan.close()
    if ns == 0:
        np.testing.assert_array_equal(f, np.zeros(nt))
        return
    fd = oracle_lib.direct("laplace", 0, xt, xs, s)
    assert _rel(f, fd) < 1e-6


def test_targets_multi_rhs(E, torch_dev):
    """nrhs = 3 equals three single evaluations (FP64)."""
    torch, dev = torch_dev
    xs, xt = W.uniform_points(3000, 71), W.uniform_points(2000, 72)
    S = np.stack([W.potentials(3000, 73 + r) for r in range(3)])
    plan, F = _run(E, torch_dev, "laplace", 0, xs, xt, S, 3, 1e-6, max_rhs=3)
    for r in range(3):
        fr = plan.evaluate(torch.from_numpy(S[r]).to(dev)).cpu().numpy()
        assert _rel(F[r], fr) < 1e-13
    plan.close()


def test_targets_point_errors(E, torch_dev):
    """A target outside the domain is EIFMM_EDOMAIN; set_points without targets is
    EIFMM_EINVAL on such a plan."""
    torch, dev = torch_dev
    xs, xt = W.uniform_points(100, 81), W.uniform_points(50, 82)
    xt[0, 3] = 1.5
    plan = E.Plan("laplace", 0, [0, 0, 0], 1.0, 100, 2, 1e-4, n_targets=50)
    with pytest.raises(E.EifmmError) as e:
        plan.set_points(torch.from_numpy(xs).to(dev), targets=torch.from_numpy(xt).to(dev))
    assert e.value.code == -2
    assert E.lib().eifmm_set_points(plan._h, None, None) == -1
    plan.close()
